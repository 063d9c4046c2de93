"""FP64 CPU oracle for the screened ACE build.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the tests, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import
it.  The GPU library never calls into it and shares no code with it.

Everything here is NumPy/SciPy in float64, written step by step from the paper:

* Eq. (vx) / Eq. (e:vij): exchange operator and pair potentials by FFT;
* Eq. (unit) and the SCDM paragraph of Sec. Theory: localization by selected
  columns of the density matrix;
* the pair-screening criterion of Sec. Theory (integral of |phi_i phi_j| >= rho_cut);
* Appendix A: W = V_X psi, M = psi^T W, -M = L L^T, P = W L^-T, V_ACE = -P P^T;
* screener_oracle: features, MLP forward/backward/Adam and the budget rule of
  the learned pair screener.

Parity status per function is listed in the module docstrings; functions whose
result no pin fixes say "parity unpinned".
"""
from . import screener_oracle  # noqa: F401
from .ace_oracle import (  # noqa: F401
    grid_G2, coulomb_kernel, pair_potential, pair_energy_forward, build_W,
    ace_from_W, ace_build, ace_apply, scdm_localize, qrcp_pivots, pairlist,
    overlap_abs, exchange_energy_pairs, NotPositiveDefinite, apply_vx_direct, build_W_rows,
    ace_apply_energy, exact_exchange, lowdin_columns, column_quality, localize_step, pairlist_step,
)
