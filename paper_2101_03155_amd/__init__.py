"""MI355X-native screened ACE exchange build (C-ABI library libace + ctypes binding).

Steps of the build, each a call of the C ABI in include/ace.h:
  ace_localize  - SCDM localization (Eq. unit)
  ace_pairlist  - pair screening by the overlap integral of |phi_i phi_j|
  ace_build     - pair Poisson solves, W, M, Cholesky(-M), projectors (Appendix A)
  ace_apply     - V_ACE application
"""
from . import ace  # noqa: F401
from .ace import Context, Grid, AceError  # noqa: F401
