"""Plain FP64 reference for every step of the screened ACE build.

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by tests, the
smoke check and the CPU-baseline leg of the benchmark, never by the library.

Conventions (Hartree atomic units):

* orbitals are real, stored ``phi[orb, z, y, x]`` on an Nz x Ny x Nx grid of a
  periodic orthorhombic box; dV = box volume / grid size;
* orthonormality means sum_r phi_i(r) phi_j(r) dV = delta_ij;
* reciprocal vectors G = 2 pi k / L with k in FFT-frequency order over the full
  FFT box (no spherical cutoff);
* FFTs use NumPy's convention (forward unnormalized, inverse divided by the
  grid size), so irfftn(v(G) * rfftn(rho)) is the periodic convolution of rho
  with the kernel whose Fourier coefficients are v(G)/volume, with dV folded in.

Parity pins live in ``tests/test_oracle_*.py``; each function's docstring says
which pin fixes it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla


class NotPositiveDefinite(ArithmeticError):
    """-M is not positive definite; ``column`` is the failing Cholesky column."""

    def __init__(self, column: int):
        super().__init__(f"-M is not positive definite (Cholesky column {column})")
        self.column = column


def _shape3(N) -> Tuple[int, int, int]:
    """(Nz, Ny, Nx) from a scalar or an (Nx, Ny, Nz) triple."""
    if np.isscalar(N):
        return (int(N),) * 3
    nx, ny, nz = (int(v) for v in N)
    return (nz, ny, nx)


def _len3(L) -> Tuple[float, float, float]:
    """(Lz, Ly, Lx) from a scalar or an (Lx, Ly, Lz) triple."""
    if np.isscalar(L):
        return (float(L),) * 3
    lx, ly, lz = (float(v) for v in L)
    return (lz, ly, lx)


def grid_G2(N, L, half: bool = True) -> np.ndarray:
    """|G|^2 on the FFT box, axes (z, y, x); ``half`` keeps x in [0, Nx/2].

    Pinned by P1/P2/P3 (naive DFT, real-space kernel tabulation, analytic
    Gaussian lattice sums)."""
    nz, ny, nx = _shape3(N)
    lz, ly, lx = _len3(L)
    gz = 2.0 * np.pi * np.fft.fftfreq(nz, d=lz / nz)
    gy = 2.0 * np.pi * np.fft.fftfreq(ny, d=ly / ny)
    if half:
        gx = 2.0 * np.pi * np.fft.rfftfreq(nx, d=lx / nx)
    else:
        gx = 2.0 * np.pi * np.fft.fftfreq(nx, d=lx / nx)
    return (gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2)


def coulomb_kernel(N, L, kind: str = "bare", omega: float = 0.106,
                   half: bool = True) -> np.ndarray:
    """Fourier coefficients v(G) of the interaction kernel (Eq. e:vij uses 1/r).

    * ``bare``: v = 4 pi / G^2 with v(0) = 0 (neutralizing background);
    * ``erfc``: kernel erfc(omega r)/r, v = 4 pi / G^2 (1 - exp(-G^2 / 4 omega^2)),
      whose G -> 0 limit pi / omega^2 is kept at G = 0.

    Pinned by P3 (continuum Gaussian energies; the erfc G=0 value is the only
    one that reproduces the real-space image sum)."""
    g2 = grid_G2(N, L, half=half)
    v = np.zeros_like(g2)
    nz = g2 > 0
    if kind == "bare":
        v[nz] = 4.0 * np.pi / g2[nz]
        v[~nz] = 0.0
    elif kind == "erfc":
        v[nz] = -4.0 * np.pi / g2[nz] * np.expm1(-g2[nz] / (4.0 * omega * omega))
        v[~nz] = np.pi / (omega * omega)
    else:
        raise ValueError(f"unknown kernel {kind!r}")
    return v


def pair_potential(phi_i: np.ndarray, phi_j: np.ndarray, v_half: np.ndarray) -> np.ndarray:
    """v_ij(r) of Eq. (e:vij): periodic Poisson solve of rho_ij = phi_i phi_j.

    One forward real FFT, multiplication by v(G), one inverse real FFT.
    Pinned by P1 (naive DFT) and P2 (real-space brute-force convolution)."""
    rho = phi_i * phi_j
    return sfft.irfftn(v_half * sfft.rfftn(rho, workers=1), s=rho.shape, workers=1)


def _half_weights(nx: int) -> np.ndarray:
    """Multiplicity of each kept x-frequency in a real-to-complex half spectrum."""
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    return w


def pair_energy_forward(phi_i, phi_j, v_half, dV: float, diagonal: bool) -> float:
    """e_ij = -(2 - delta_ij) (ij|ij) with (ij|ij) = dV N^-1 sum_G v(G) |rho_hat(G)|^2.

    Needs only the forward transform (Parseval).  Equal to the energy read off
    the full pipeline, dV sum_r rho_ij v_ij (checked by a test)."""
    rho = phi_i * phi_j
    rh = sfft.rfftn(rho, workers=1)
    w = _half_weights(rho.shape[-1])
    s = float(np.sum(v_half * (rh.real ** 2 + rh.imag ** 2) * w[None, None, :]))
    jj = dV * s / rho.size
    return -(1.0 if diagonal else 2.0) * jj


def _as_pairs(pairs) -> np.ndarray:
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return p


def build_W(phi: np.ndarray, pairs, v_half: np.ndarray, dV: float,
            energies: bool = False, workers: int = 1):
    """W_i = V_X^screened phi_i = -sum_{j: (i,j) kept} v_ij phi_j (Eq. vx over kept pairs).

    Each unordered kept pair (i, j), i <= j, contributes -v_ij phi_j to W_i and,
    if i != j, -v_ij phi_i to W_j (v_ij = v_ji for real orbitals).  Optionally
    returns the per-pair energies e_ij = -(2 - delta_ij) dV sum_r rho_ij v_ij.

    ``workers > 1`` runs the pair potentials of a batch of pairs on threads and
    then applies the batch's updates row by row, each row's updates in pair
    order: every row receives the same subtractions in the same order as the
    serial loop, so the result is bitwise the serial one (checked by a test)."""
    W = np.zeros_like(phi)
    p = _as_pairs(pairs)
    e = np.zeros(len(p))
    if workers <= 1:
        for n, (i, j) in enumerate(p):
            v = pair_potential(phi[i], phi[j], v_half)
            W[i] -= v * phi[j]
            if i != j:
                W[j] -= v * phi[i]
            if energies:
                e[n] = -(1.0 if i == j else 2.0) * dV * float(np.sum(phi[i] * phi[j] * v))
        return (W, e) if energies else W

    batch = 4 * workers
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for start in range(0, len(p), batch):
            chunk = p[start:start + batch]

            def potential(n):
                i, j = int(chunk[n, 0]), int(chunk[n, 1])
                v = pair_potential(phi[i], phi[j], v_half)
                en = -(1.0 if i == j else 2.0) * dV * float(np.sum(phi[i] * phi[j] * v)) if energies else 0.0
                return v, en

            got = list(ex.map(potential, range(len(chunk))))
            if energies:
                e[start:start + len(chunk)] = [g[1] for g in got]
            updates = {}
            for n, (i, j) in enumerate(chunk):
                updates.setdefault(int(i), []).append((n, int(j)))
                if i != j:
                    updates.setdefault(int(j), []).append((n, int(i)))

            def apply_row(row):
                for n, other in updates[row]:
                    W[row] -= got[n][0] * phi[other]

            list(ex.map(apply_row, list(updates)))
    return (W, e) if energies else W


def build_W_rows(phi: np.ndarray, pairs, rows: Sequence[int], v_half: np.ndarray,
                 workers: Optional[int] = None) -> np.ndarray:
    """W_i for selected orbitals only (sampled parity at full size).

    W_i = -sum over kept pairs touching i of v_ij phi_j; threads over rows."""
    p = _as_pairs(pairs)
    workers = workers or max(1, len(os.sched_getaffinity(0)))

    def one(i):
        w = np.zeros_like(phi[i])
        for a, b in p[(p[:, 0] == i) | (p[:, 1] == i)]:
            j = b if a == i else a
            w -= pair_potential(phi[i], phi[j], v_half) * phi[j]
        return w

    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return np.stack(list(ex.map(one, rows)))


def exchange_energy_pairs(phi: np.ndarray, pairs, v_half: np.ndarray, dV: float,
                          workers: Optional[int] = None) -> np.ndarray:
    """Per-pair e_ij for a pair list, forward transforms only, threaded."""
    p = _as_pairs(pairs)
    workers = workers or max(1, len(os.sched_getaffinity(0)))

    def one(ij):
        i, j = int(ij[0]), int(ij[1])
        return pair_energy_forward(phi[i], phi[j], v_half, dV, i == j)

    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return np.fromiter(ex.map(one, p), dtype=np.float64, count=len(p))


def ace_from_W(phi: np.ndarray, W: np.ndarray, dV: float):
    """Appendix A: M_kl = <phi_k|W_l>, -M = L L^T, P = W L^-T.

    M is symmetrized, M <- (M + M^T)/2, before the factorization (a screened M
    need not be exactly symmetric).  E_x = tr M.  Returns (M, L, xi, E_x, asym)
    with xi[k] the k-th projector P_k on the grid and asym = max|M - M^T|.
    Pinned by P4 (V_ACE phi = W, <phi_i|V_ACE|phi_j> = M_ij, rotation
    invariance, agreement with direct application of V_X) and P7 (one orbital)."""
    n = phi.shape[0]
    A = phi.reshape(n, -1)
    B = W.reshape(n, -1)
    M = dV * (A @ B.T)
    asym = float(np.max(np.abs(M - M.T))) if n else 0.0
    M = 0.5 * (M + M.T)
    ex = float(np.trace(M))
    Lc = _cholesky_lower(-M)
    xi = sla.solve_triangular(Lc, B, lower=True).reshape(W.shape)
    return M, Lc, xi, ex, asym


def _cholesky_lower(A: np.ndarray) -> np.ndarray:
    """Column-by-column Cholesky A = L L^T; raises NotPositiveDefinite(col)."""
    n = A.shape[0]
    L = np.zeros_like(A)
    for k in range(n):
        d = A[k, k] - L[k, :k] @ L[k, :k]
        if not (d > 0.0) or not np.isfinite(d):
            raise NotPositiveDefinite(k)
        L[k, k] = np.sqrt(d)
        L[k + 1:, k] = (A[k + 1:, k] - L[k + 1:, :k] @ L[k, :k]) / L[k, k]
    return L


def ace_build(phi: np.ndarray, pairs, N, L, kind: str, omega: float, workers: int = 1):
    """Steps (c)-(e) end to end: returns dict(W, M, L, xi, ex, asym, e).

    ``workers`` threads the pair stage (bitwise the serial result)."""
    dV = float(np.prod(_len3(L))) / phi[0].size
    v = coulomb_kernel(N, L, kind, omega)
    W, e = build_W(phi, pairs, v, dV, energies=True, workers=workers)
    M, Lc, xi, ex, asym = ace_from_W(phi, W, dV)
    return dict(W=W, M=M, L=Lc, xi=xi, ex=ex, asym=asym, e=e)


def ace_apply(xi: np.ndarray, X: np.ndarray, dV: float) -> np.ndarray:
    """V_ACE x = -sum_k P_k <P_k|x> (Appendix A; ACE application equation)."""
    n = xi.shape[0]
    P = xi.reshape(n, -1)
    Xm = X.reshape(X.shape[0], -1)
    c = dV * (P @ Xm.T)
    return (-(c.T @ P)).reshape(X.shape)


def ace_apply_energy(xi: np.ndarray, X: np.ndarray, dV: float):
    """V_ACE on a set of functions and their summed exchange energy.

    Returns (Y, E) with Y = V_ACE X (Appendix A, projector form) and
    E = sum_a <x_a|V_ACE|x_a>, the plain inner product of each function with
    its image.  With X the occupied orbitals this is the exchange energy of an
    SCF cycle.  Pinned by P8: with X the orbitals a full-list build was made
    from, E is that build's tr M (V_ACE phi = W); E is never positive; it is
    unchanged by an orthogonal mixing of the functions."""
    Y = ace_apply(xi, X, dV)
    n = X.shape[0]
    return Y, dV * float(np.sum(X.reshape(n, -1) * Y.reshape(n, -1)))


def exact_exchange(psi: np.ndarray, N, L, kind: str, omega: float):
    """Exact exchange on the orbitals themselves, Eq. (vx) over every (i, j).

    W_i = V_X psi_i = -sum_j v_ij psi_j with no screening and no localization,
    M_kl = <psi_k|W_l> symmetrized, E_x = tr M.  Returns (W, M, E_x).  Pinned
    by P9: W equals the pair-symmetric build over the full list, E_x is
    unchanged by an orthogonal rotation of the orbitals, -M is positive
    definite, and one orbital reduces to its self-exchange."""
    dV = float(np.prod(_len3(L))) / psi[0].size
    v = coulomb_kernel(N, L, kind, omega)
    W = apply_vx_direct(psi, psi, v)
    n = psi.shape[0]
    M = dV * (psi.reshape(n, -1) @ W.reshape(n, -1).T)
    M = 0.5 * (M + M.T)
    return W, M, float(np.trace(M))


def apply_vx_direct(phi: np.ndarray, X: np.ndarray, v_half: np.ndarray) -> np.ndarray:
    """Exact exchange on arbitrary functions, Eq. (vx): V_X x = -sum_j v_xj phi_j."""
    out = np.zeros_like(X)
    for a in range(X.shape[0]):
        for j in range(phi.shape[0]):
            out[a] -= pair_potential(X[a], phi[j], v_half) * phi[j]
    return out


# --------------------------------------------------------------------------
# Localization (Eq. unit; SCDM paragraph of Sec. Theory)
# --------------------------------------------------------------------------

def _top_candidates(res: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k largest entries; ties broken by the smaller index."""
    k = min(k, res.size)
    part = np.argpartition(-res, k - 1)[:k]
    thr = res[part].min()
    # include every entry equal to the threshold so index tie-breaks are exact
    cand = np.flatnonzero(res >= thr)
    order = np.lexsort((cand, -res[cand]))
    return cand[order][:k]


def qrcp_pivots(A: np.ndarray, n_pick: Optional[int] = None, n_verify: int = 8):
    """Greedy QR with column pivoting on A (rows = orbitals, columns = grid points).

    Step k picks the column whose residual, after projecting out the span of the
    previously picked columns, has the largest norm.  Residual norms are
    downdated after every pick; the top ``n_verify`` downdated candidates are then
    re-ranked by their residual recomputed by explicit (twice repeated)
    projection, so the pick does not depend on accumulated rounding in the
    downdate.  Ties go to the smallest grid index.  Returns (pivots, Q) with Q's
    columns the orthonormal residual directions.

    Pinned by P5 (agreement with LAPACK's dgeqp3 pivots when the top residual gap
    is not a near tie; invariance under rotations of the occupied space; first
    pivot = argmax of the density)."""
    n, m = A.shape
    kmax = n if n_pick is None else n_pick
    res = np.einsum("ij,ij->j", A, A)
    Q = np.zeros((n, kmax))
    piv = np.empty(kmax, dtype=np.int64)
    for k in range(kmax):
        Qk = Q[:, :k]
        best, best_r2, best_vec = -1, -np.inf, None
        for c in sorted(_top_candidates(res, n_verify)):
            a = A[:, c].copy()
            for _ in range(2):
                a -= Qk @ (Qk.T @ a)
            r2 = float(a @ a)
            if r2 > best_r2:
                best, best_r2, best_vec = int(c), r2, a
        q = best_vec / np.sqrt(best_r2)
        Q[:, k] = q
        ell = q @ A
        res -= ell * ell
        res[best] = -np.inf
        piv[k] = best
    return piv, Q


def scdm_localize(psi: np.ndarray, dV: float):
    """SCDM localization (Sec. Theory, Eq. unit).

    Columns c_1..c_N of the density matrix P(r, r') = sum_i psi_i(r) psi_i(r') are
    selected by QRCP of the matrix A[i, r] = psi_i(r); the selected columns,
    sum_i psi_i(r) psi_i(c_k), are Loewdin-orthonormalized.  This is the unitary
    rotation phi_k = sum_i psi_i U_ik with U = A_C (A_C^T A_C)^-1/2, A_C = A[:, C],
    computed here through a symmetric eigendecomposition.  Output orbital k
    belongs to pivot k.

    Pinned by P5 (Phi invariant under psi -> psi Q, Phi Phi^T = Psi Psi^T,
    disjoint orbitals returned up to order and sign)."""
    n = psi.shape[0]
    piv, _ = qrcp_pivots(psi.reshape(n, -1))
    U, phi = lowdin_columns(psi, piv)
    return piv, U, phi


def lowdin_columns(psi: np.ndarray, piv):
    """The Loewdin step of SCDM (Eq. unit) on given columns C = piv.

    U = A_C (A_C^T A_C)^-1/2 with A_C = A[:, C], A[i, r] = psi_i(r), by a
    symmetric eigendecomposition; phi_k = sum_i psi_i U_ik.  Any columns with
    a nonsingular A_C give an orthogonal U, so the columns picked at one MD
    step can serve the next.  Returns (U, phi).  Pinned by P5 (through
    scdm_localize) and P10 (A_C = U H with H symmetric positive definite,
    U orthogonal, Phi Phi^T = Psi Psi^T, ValueError on repeated or
    out-of-range columns)."""
    n = psi.shape[0]
    A = psi.reshape(n, -1)
    piv = np.asarray(piv, dtype=np.int64)
    if piv.shape != (n,) or piv.min() < 0 or piv.max() >= A.shape[1] or len(set(piv.tolist())) != n:
        raise ValueError("need one distinct in-range grid column per orbital")
    AC = A[:, piv]
    w, V = np.linalg.eigh(AC.T @ AC)
    U = AC @ (V @ np.diag(w ** -0.5) @ V.T)
    phi = (U.T @ A).reshape(psi.shape)
    return U, phi


def column_quality(psi: np.ndarray, piv) -> float:
    """(max_k |R_kk| / min_k |R_kk|)^2 of the QR factorization A[:, piv] = Q R,
    columns in pivot order (A[i, r] = psi_i(r)); inf when A[:, piv] is
    singular.  Greedy pivoting keeps this ratio small; it is a lower bound on
    the condition number of A_C^T A_C.  Pinned by P12 (R_kk are the residual
    norms greedy QRCP picks its columns with; the bound; diagonal cases)."""
    n = psi.shape[0]
    A = psi.reshape(n, -1)[:, np.asarray(piv, dtype=np.int64)]
    d = np.abs(np.diag(np.linalg.qr(A, mode="r")))
    if d.min() == 0.0 or not np.all(np.isfinite(d)):
        return float("inf")
    return float((d.max() / d.min()) ** 2)


def localize_step(psi: np.ndarray, prev_piv, dV: float, cond_max: float):
    """SCDM at the next MD step with the previous step's columns as the warm
    start (the ACE operator is rebuilt at least once per MD step, Sec. Theory):
    the columns are kept, and only the Loewdin step of Eq. (unit) runs, when
    their column_quality on this step's orbitals is at most cond_max;
    otherwise SCDM picks fresh columns.  Returns (piv, U, phi, reused, quality).
    Pinned by P12."""
    q = column_quality(psi, prev_piv)
    if q <= cond_max:
        U, phi = lowdin_columns(psi, prev_piv)
        return np.asarray(prev_piv, dtype=np.int64), U, phi, True, q
    piv, U, phi = scdm_localize(psi, dV)
    return piv, U, phi, False, q


# --------------------------------------------------------------------------
# Pair screening (criterion of Sec. Theory)
# --------------------------------------------------------------------------

def overlap_abs(phi: np.ndarray, dV: float) -> np.ndarray:
    """O_ij = dV sum_r |phi_i(r)| |phi_j(r)| (Riemann sum of the screening integral)."""
    n = phi.shape[0]
    a = np.abs(phi.reshape(n, -1))
    return dV * (a @ a.T)


def pairlist(phi: np.ndarray, dV: float, rho_cut: float):
    """Kept pairs (i <= j) with O_ij >= rho_cut; diagonal pairs always kept.

    Sorted by (i, j).  Returns (pairs[int64, npairs x 2], O_kept).
    Pinned by P6 (rho_cut -> 0 gives every pair, rho_cut > 1 only the diagonal,
    and the energy of dropped pairs is exactly the screened-minus-full E_x)."""
    O = overlap_abs(phi, dV)
    n = O.shape[0]
    iu, ju = np.triu_indices(n)
    keep = (O[iu, ju] >= rho_cut) | (iu == ju)
    pairs = np.stack([iu[keep], ju[keep]], axis=1)
    return pairs, O[iu[keep], ju[keep]]


def pairlist_step(phi: np.ndarray, dV: float, rho_cut: float, prev_pairs):
    """The screening criterion at the next MD step, compared with the previous
    step's list: returns (pairs, O_kept, added, removed) with added the kept
    pairs absent from prev_pairs and removed the previous pairs no longer
    kept.  Pinned by P12 (brute-force set differences)."""
    pairs, O = pairlist(phi, dV, rho_cut)
    new = {(int(i), int(j)) for i, j in pairs}
    old = {(int(i), int(j)) for i, j in np.asarray(prev_pairs).reshape(-1, 2)}
    return pairs, O, len(new - old), len(old - new)
