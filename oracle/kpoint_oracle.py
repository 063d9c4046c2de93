"""Plain FP64 reference of the ACE build for complex Bloch orbitals with k-points.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The screening criterion of Sec. Theory is written for complex orbitals
(the integral of |phi_i phi_j*|), and Eq. (vx) and Appendix A hold for them
with conjugates in the right places.  Here the orbitals are Bloch functions
psi_{n k}(r) = exp(i k.r) u_{n k}(r) on an N_k-point sampling of the
Brillouin zone, stored by their cell-periodic parts u on the real-space grid,
flattened a = q * norb + m over (k-point q, band m).

For the pair (a, b) with k-points k_a, k_b the pair density
conj(psi_a) psi_b = exp(i (k_b - k_a).r) conj(u_a) u_b is Bloch-periodic,
and its convolution with the lattice-summed kernel is

    exp(i (k_b - k_a).r) * P_{k_b - k_a}[conj(u_a) u_b],
    P_d[f] = IFFT( v(|G + d|) FFT(f) )          (NumPy conventions)

so, on the cell-periodic parts, with the Brillouin-zone average 1/N_k,

    w_b = -(1/N_k) sum_a u_a P_{k_b - k_a}[conj(u_a) u_b]      (Eq. vx)

and P_{-d}[conj f] = conj(P_d[f]), so one transform per unordered pair serves
w_b (u_a times P) and w_a (u_b times conj P).  The operator is block-diagonal
in k: per k-point, M = dV U^H W (Hermitian), -M = L L^H, and the projectors
P = W L^-H (Appendix A), stored by rows as xi = conj(L)^-1 W, so that
V_ACE x = -sum_j xi_j <xi_j|x> dV.  E_x = (1/N_k) sum_k tr M_k.

Pins (tests/test_oracle_kpoints.py): the Gamma point with real orbitals is the
real build; a naive DFT of the shifted-kernel convolution; k-point sampling
of a cell equals the Gamma point of the supercell it unfolds to; rotation
invariance under a unitary mixing per k-point; Hermitian negative definite M
and V_ACE psi = W on the occupied space.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import scipy.linalg as sla

from .ace_oracle import NotPositiveDefinite, _len3, _shape3


def shifted_G2(N, L, d) -> np.ndarray:
    """|G + d|^2 over the full FFT box, axes (z, y, x); d = (dx, dy, dz) in bohr^-1."""
    nz, ny, nx = _shape3(N)
    lz, ly, lx = _len3(L)
    gx = 2.0 * np.pi * np.fft.fftfreq(nx, d=lx / nx) + d[0]
    gy = 2.0 * np.pi * np.fft.fftfreq(ny, d=ly / ny) + d[1]
    gz = 2.0 * np.pi * np.fft.fftfreq(nz, d=lz / nz) + d[2]
    return gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2


def shifted_kernel(N, L, kind: str, omega: float, d) -> np.ndarray:
    """v(|G + d|) for the bare (v(0) = 0) or erfc (v(0) = pi/omega^2) kernel."""
    g2 = shifted_G2(N, L, d)
    v = np.zeros_like(g2)
    nz = g2 > 0
    if kind == "bare":
        v[nz] = 4.0 * np.pi / g2[nz]
    elif kind == "erfc":
        v[nz] = -4.0 * np.pi / g2[nz] * np.expm1(-g2[nz] / (4.0 * omega * omega))
        v[~nz] = np.pi / (omega * omega)
    else:
        raise ValueError(f"unknown kernel {kind!r}")
    return v


def pair_potential_k(u_a, u_b, v_full) -> np.ndarray:
    """P_d[conj(u_a) u_b] with v_full = v(|G + d|): one forward and one inverse complex FFT."""
    return np.fft.ifftn(v_full * np.fft.fftn(np.conj(u_a) * u_b))


def _kvecs(kvec, nk):
    k = np.asarray(kvec, dtype=np.float64).reshape(nk, 3)
    return k


def build_W_k(u: np.ndarray, kvec, norb: int, pairs, N, L, kind: str, omega: float):
    """w_a for every Bloch orbital a over the kept unordered pairs (a <= b),
    and the pair energies e_ab = -(2 - d_ab) N_k^-2 dV Re sum_r conj(f) P[f],
    f = conj(u_a) u_b, whose sum is E_x = (1/N_k) sum_k tr M_k.
    u: complex [N_k * norb][Nz][Ny][Nx]."""
    ntot = u.shape[0]
    nk = ntot // norb
    k = _kvecs(kvec, nk)
    dV = float(np.prod(_len3(L))) / u[0].size
    c = 1.0 / nk
    W = np.zeros_like(u)
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    e = np.zeros(len(p))
    cache = {}
    for n, (a, b) in enumerate(p):
        d = tuple(k[b // norb] - k[a // norb])
        if d not in cache:
            cache[d] = shifted_kernel(N, L, kind, omega, d)
        f = np.conj(u[a]) * u[b]
        V = np.fft.ifftn(cache[d] * np.fft.fftn(f))
        W[b] -= c * u[a] * V
        if a != b:
            W[a] -= c * u[b] * np.conj(V)
        e[n] = -(1.0 if a == b else 2.0) * c * c * dV * float(np.real(np.sum(np.conj(f) * V)))
    return W, e


def ace_from_W_k(u: np.ndarray, W: np.ndarray, norb: int, dV: float):
    """Per k-point: M = dV U^H W made Hermitian, -M = L L^H, xi = conj(L)^-1 W.
    Returns (M [N_k][norb][norb], L, xi like W, E_x = (1/N_k) sum tr M, asym)."""
    ntot = u.shape[0]
    nk = ntot // norb
    Ms, Ls, xi, asym, ex = [], [], np.zeros_like(W), 0.0, 0.0
    for q in range(nk):
        sl = slice(q * norb, (q + 1) * norb)
        A = u[sl].reshape(norb, -1)
        B = W[sl].reshape(norb, -1)
        M = dV * (np.conj(A) @ B.T)
        asym = max(asym, float(np.max(np.abs(M - M.conj().T))))
        M = 0.5 * (M + M.conj().T)
        Lc = _cholesky_lower_c(-M)
        xi[sl] = sla.solve_triangular(np.conj(Lc), B, lower=True).reshape(W[sl].shape)
        ex += float(np.real(np.trace(M))) / nk
        Ms.append(M)
        Ls.append(Lc)
    return np.array(Ms), np.array(Ls), xi, ex, asym


def _cholesky_lower_c(A: np.ndarray) -> np.ndarray:
    """Column-by-column Cholesky A = L L^H of a Hermitian matrix; raises
    NotPositiveDefinite(col)."""
    n = A.shape[0]
    L = np.zeros_like(A)
    for j in range(n):
        d = float(np.real(A[j, j] - L[j, :j] @ np.conj(L[j, :j])))
        if not (d > 0.0) or not np.isfinite(d):
            raise NotPositiveDefinite(j)
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ np.conj(L[j, :j])) / L[j, j]
    return L


def ace_build_k(u: np.ndarray, kvec, norb: int, pairs, N, L, kind: str, omega: float):
    """Steps (c)-(e) for Bloch orbitals: dict(W, M, L, xi, ex, asym, e)."""
    dV = float(np.prod(_len3(L))) / u[0].size
    W, e = build_W_k(u, kvec, norb, pairs, N, L, kind, omega)
    M, Lc, xi, ex, asym = ace_from_W_k(u, W, norb, dV)
    return dict(W=W, M=M, L=Lc, xi=xi, ex=ex, asym=asym, e=e)


def ace_apply_k(xi: np.ndarray, X: np.ndarray, dV: float) -> np.ndarray:
    """V_ACE x = -sum_j xi_j <xi_j|x> dV for the functions of one k-point."""
    n = xi.shape[0]
    P = xi.reshape(n, -1)
    Xm = X.reshape(X.shape[0], -1)
    c = dV * (np.conj(P) @ Xm.T)
    return (-(c.T @ P)).reshape(X.shape)


def pairlist_k(u: np.ndarray, dV: float, rho_cut: float):
    """Kept pairs a <= b of the Bloch orbitals: integral of |psi_a psi_b*|
    = dV sum |u_a| |u_b| >= rho_cut (|exp(i k.r)| = 1); diagonal always kept."""
    n = u.shape[0]
    a = np.abs(u.reshape(n, -1))
    O = dV * (a @ a.T)
    iu, ju = np.triu_indices(n)
    keep = (O[iu, ju] >= rho_cut) | (iu == ju)
    return np.stack([iu[keep], ju[keep]], axis=1), O[iu[keep], ju[keep]]


def full_pairs(n: int) -> np.ndarray:
    iu, ju = np.triu_indices(n)
    return np.stack([iu, ju], axis=1)
