"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

P1  naive O(N^6) DFT                    -> FFT, half-spectrum handling, normalization
P2  real-space periodic convolution      -> dV / volume placement of the kernel
P3  analytic Gaussian lattice energies   -> the 4 pi / G^2 and erfc kernels, G = 0 values
P4  ACE algebra (Appendix A)             -> M, Cholesky, projectors, application
P5  SCDM                                 -> QRCP pivots (LAPACK dgeqp3), invariances
P6  screening                            -> pair selection and the dropped-energy identity
P7  one orbital                          -> closed-form projector
P8-P10 application energy, exact exchange, reused columns
P11 sampled helpers (rows of W, Parseval pair energies, threaded build) -> the serial build
P12 the next MD step: kept columns and their quality measure, the re-screen against the previous list
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import erf

import oracle
from synth import SystemSpec, make_orbitals, config_spec, disjoint_gaussians


# ----------------------------------------------------------------- helpers

def _signed_freqs(n):
    k = np.arange(n)
    return np.where(k < (n + 1) // 2, k, k - n)


def _kernel_direct(g2, kind, omega):
    """v(G) written out from the Fourier transforms of 1/r and erfc(omega r)/r."""
    v = np.zeros_like(g2)
    for idx, x in np.ndenumerate(g2):
        if x == 0.0:
            v[idx] = 0.0 if kind == "bare" else np.pi / omega ** 2
        else:
            v[idx] = 4 * np.pi / x * (1.0 if kind == "bare" else (1 - np.exp(-x / (4 * omega ** 2))))
    return v


def _random_smooth(rng, n, L):
    x = np.arange(n) * L / n
    f = np.zeros((n, n, n))
    for _ in range(2):
        c = rng.uniform(0, L, 3)
        s = rng.uniform(0.6, 1.0) * L / 4
        p = [sum(np.exp(-(x - c[d] - m * L) ** 2 / (2 * s * s)) for m in (-1, 0, 1)) for d in range(3)]
        f += rng.normal() * p[2][:, None, None] * p[1][None, :, None] * p[0][None, None, :]
    return f


# ----------------------------------------------------------------- P1

@pytest.mark.parametrize("n", [6, 8, 10, 12])
@pytest.mark.parametrize("kind", ["bare", "erfc"])
def test_p1_pair_potential_matches_naive_dft(n, kind):
    rng = np.random.default_rng(100 + n)
    L = 5.0 + 0.1 * n
    a = rng.normal(size=(n, n, n))
    b = rng.normal(size=(n, n, n))
    k = _signed_freqs(n)
    g = 2 * np.pi * k / L
    g2 = g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2
    v = _kernel_direct(g2, kind, 0.7)
    # explicit DFT matrix, exp(-2 pi i k x / n)
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    rho = a * b
    rh = np.einsum("az,by,cx,zyx->abc", F, F, F, rho)
    back = np.einsum("az,by,cx,abc->zyx", F.conj(), F.conj(), F.conj(), v * rh) / n ** 3
    got = oracle.pair_potential(a, b, oracle.coulomb_kernel(n, L, kind, 0.7))
    assert np.max(np.abs(back.imag)) < 1e-12 * np.max(np.abs(back.real))
    np.testing.assert_allclose(got, back.real, rtol=0, atol=1e-13 * np.max(np.abs(back.real)))


def test_p1_noncubic_grid_and_box():
    rng = np.random.default_rng(5)
    nx, ny, nz = 8, 6, 10
    Lx, Ly, Lz = 4.0, 5.0, 6.5
    a = rng.normal(size=(nz, ny, nx))
    b = rng.normal(size=(nz, ny, nx))
    gz = 2 * np.pi * _signed_freqs(nz) / Lz
    gy = 2 * np.pi * _signed_freqs(ny) / Ly
    gx = 2 * np.pi * _signed_freqs(nx) / Lx
    g2 = gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2
    v = _kernel_direct(g2, "erfc", 0.4)
    Fz = np.exp(-2j * np.pi * np.outer(np.arange(nz), np.arange(nz)) / nz)
    Fy = np.exp(-2j * np.pi * np.outer(np.arange(ny), np.arange(ny)) / ny)
    Fx = np.exp(-2j * np.pi * np.outer(np.arange(nx), np.arange(nx)) / nx)
    rh = np.einsum("az,by,cx,zyx->abc", Fz, Fy, Fx, a * b)
    back = np.einsum("az,by,cx,abc->zyx", Fz.conj(), Fy.conj(), Fx.conj(), v * rh).real / (nx * ny * nz)
    got = oracle.pair_potential(a, b, oracle.coulomb_kernel((nx, ny, nz), (Lx, Ly, Lz), "erfc", 0.4))
    np.testing.assert_allclose(got, back, atol=1e-13 * np.abs(back).max())


# ----------------------------------------------------------------- P2

@pytest.mark.parametrize("kind", ["bare", "erfc"])
def test_p2_real_space_periodic_convolution(kind):
    n, L = 8, 6.0
    rng = np.random.default_rng(11)
    rho = rng.normal(size=(n, n, n))
    vol, dV = L ** 3, (L / n) ** 3
    k = _signed_freqs(n)
    g = 2 * np.pi * k / L
    g2 = g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2
    v = _kernel_direct(g2, kind, 0.5)
    # tabulate K(r) = (1/vol) sum_G v(G) exp(i G.r) on grid displacements
    x = np.arange(n) * L / n
    ph = np.exp(1j * np.outer(g, x))  # [k, x]
    K = np.einsum("abc,az,by,cx->zyx", v, ph, ph, ph).real / vol
    out = np.zeros_like(rho)
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                sh = K[(iz - np.arange(n)) % n][:, (iy - np.arange(n)) % n][:, :, (ix - np.arange(n)) % n]
                out[iz, iy, ix] = dV * np.sum(sh * rho)
    got = oracle.pair_potential(rho, np.ones_like(rho), oracle.coulomb_kernel(n, L, kind, 0.5))
    np.testing.assert_allclose(got, out, atol=1e-12 * np.abs(out).max())


# ----------------------------------------------------------------- P3

def _periodic_gaussian_density(n, L, c, s):
    x = np.arange(n) * L / n
    p = []
    for d in range(3):
        diff = x[None, :] - c[d] - L * np.arange(-2, 3)[:, None]
        p.append(np.exp(-diff ** 2 / (2 * s * s)).sum(0))
    rho = p[2][:, None, None] * p[1][None, :, None] * p[0][None, None, :]
    return rho * (2 * np.pi * s * s) ** -1.5


def _erfc_image_sum(L, st2, omega, nmax):
    """sum over images of a Gaussian pair distribution (variance st2) with erfc(omega r)/r."""
    tot = np.sqrt(2 / np.pi) * (1 / np.sqrt(st2) - 1 / np.sqrt(st2 + 1 / (2 * omega ** 2)))
    r = np.arange(-nmax, nmax + 1)
    R = L * np.sqrt(r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2)
    R = R[R > 0]
    tot += np.sum((erf(R / np.sqrt(2 * st2)) - erf(R / np.sqrt(2 * st2 + 1 / omega ** 2))) / R)
    return tot


@pytest.mark.parametrize("omega", [0.106, 0.5, 1.3])
def test_p3_erfc_gaussian_self_energy(omega):
    n, L, s = 24, 8.0, 0.75
    rho = _periodic_gaussian_density(n, L, np.array([1.3, 4.4, 6.9]), s)
    dV = (L / n) ** 3
    assert abs(rho.sum() * dV - 1) < 1e-13
    vr = oracle.pair_potential(rho, np.ones_like(rho), oracle.coulomb_kernel(n, L, "erfc", omega))
    e_grid = dV * np.sum(rho * vr)
    e_exact = _erfc_image_sum(L, 2 * s * s, omega, nmax=int(np.ceil(8 / (omega * L))) + 2)
    assert abs(e_grid - e_exact) < 1e-13 * abs(e_exact), (e_grid, e_exact)


def test_p3_erfc_G0_reading_is_the_only_consistent_one():
    """Setting v(0) = 0 for the erfc kernel shifts the energy by pi/(omega^2 vol)."""
    n, L, s, omega = 24, 8.0, 0.75, 0.106
    rho = _periodic_gaussian_density(n, L, np.array([2.0, 2.0, 2.0]), s)
    dV = (L / n) ** 3
    v = oracle.coulomb_kernel(n, L, "erfc", omega)
    v0 = v.copy()
    v0[0, 0, 0] = 0.0
    e_exact = _erfc_image_sum(L, 2 * s * s, omega, nmax=12)
    e_bad = dV * np.sum(rho * oracle.pair_potential(rho, np.ones_like(rho), v0))
    assert abs(e_bad - (e_exact - np.pi / (omega ** 2 * L ** 3))) < 1e-12
    assert abs(e_bad - e_exact) > 1e-3


def test_p3_bare_coulomb_ewald():
    """Bare kernel with v(0)=0 equals an Ewald split evaluated independently."""
    n, L, s, a = 24, 8.0, 0.75, 1.0
    rho = _periodic_gaussian_density(n, L, np.array([3.1, 0.4, 5.5]), s)
    dV, vol = (L / n) ** 3, L ** 3
    vr = oracle.pair_potential(rho, np.ones_like(rho), oracle.coulomb_kernel(n, L, "bare"))
    e_grid = dV * np.sum(rho * vr)
    st2 = 2 * s * s
    real_part = _erfc_image_sum(L, st2, a, nmax=3)
    k = np.arange(-14, 15)
    g = 2 * np.pi * k / L
    g2 = (g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2).ravel()
    g2 = g2[g2 > 0]
    recip = np.sum(4 * np.pi / g2 * np.exp(-g2 / (4 * a * a)) * np.exp(-st2 * g2 / 2)) / vol
    e_exact = real_part - np.pi / (a * a * vol) + recip
    assert abs(e_grid - e_exact) < 1e-13 * abs(e_exact), (e_grid, e_exact)


def test_p3_two_gaussian_interaction():
    """Cross energy of two unit Gaussian densities: erf(R/sqrt(2 st2))/R - erfc part."""
    n, L, s, omega = 24, 8.0, 0.8, 0.9
    c1, c2 = np.array([2.0, 3.0, 4.0]), np.array([3.5, 2.2, 5.1])
    r1 = _periodic_gaussian_density(n, L, c1, s)
    r2 = _periodic_gaussian_density(n, L, c2, s)
    dV = (L / n) ** 3
    v = oracle.coulomb_kernel(n, L, "erfc", omega)
    e_grid = dV * np.sum(r1 * oracle.pair_potential(r2, np.ones_like(r2), v))
    st2 = 2 * s * s
    d = c1 - c2
    rr = np.arange(-4, 5)
    tot = 0.0
    for i in rr:
        for j in rr:
            for k in rr:
                R = np.linalg.norm(d + L * np.array([i, j, k]))
                tot += (erf(R / np.sqrt(2 * st2)) - erf(R / np.sqrt(2 * st2 + 1 / omega ** 2))) / R
    assert abs(e_grid - tot) < 1e-13 * abs(tot)


# ----------------------------------------------------------------- P4

@pytest.fixture(scope="module")
def small_system():
    spec = SystemSpec(n_mol=2, L=8.0, N=16, sigma=0.9, offset=0.8, placement="uniform",
                      seed=77, kernel="erfc", omega=0.3)
    return make_orbitals(spec)


def _full_pairs(n):
    return np.array([(i, j) for i in range(n) for j in range(i, n)])


def test_p4_ace_algebra(small_system):
    o = small_system
    s = o.spec
    phi = o.psi
    r = oracle.ace_build(phi, _full_pairs(s.norb), s.N, s.L, "erfc", s.omega)
    M, xi, W = r["M"], r["xi"], r["W"]
    assert r["asym"] < 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).max() < 0
    # V_ACE phi_i = W_i on the occupied space
    np.testing.assert_allclose(oracle.ace_apply(xi, phi, s.dV), W, atol=1e-12 * np.abs(W).max())
    # <phi_i|V_ACE|phi_j> = M_ij, and tr M = sum_ij e_ij = -||Phi^T xi dV||_F^2
    Vij = s.dV * phi.reshape(s.norb, -1) @ oracle.ace_apply(xi, phi, s.dV).reshape(s.norb, -1).T
    np.testing.assert_allclose(Vij, M, atol=1e-13 * np.abs(M).max())
    proj = s.dV * phi.reshape(s.norb, -1) @ xi.reshape(s.norb, -1).T
    assert abs(r["ex"] - (-np.sum(proj ** 2))) < 1e-12 * abs(r["ex"])
    assert abs(r["ex"] - r["e"].sum()) < 1e-12 * abs(r["ex"])
    # L is lower triangular with -M = L L^T
    np.testing.assert_allclose(r["L"] @ r["L"].T, -M, atol=1e-13 * np.abs(M).max())


def test_p4_matches_direct_exchange_on_occupied_span(small_system):
    o = small_system
    s = o.spec
    phi = o.psi
    v = oracle.coulomb_kernel(s.N, s.L, "erfc", s.omega)
    r = oracle.ace_build(phi, _full_pairs(s.norb), s.N, s.L, "erfc", s.omega)
    rng = np.random.default_rng(3)
    c = rng.normal(size=(2, s.norb))
    X = np.einsum("ak,kzyx->azyx", c, phi)
    direct = oracle.apply_vx_direct(phi, X, v)
    ace = oracle.ace_apply(r["xi"], X, s.dV)
    np.testing.assert_allclose(ace, direct, atol=1e-12 * np.abs(direct).max())


def test_p4_rotation_invariance_and_scdm_equivalence(small_system):
    o = small_system
    s = o.spec
    pairs = _full_pairs(s.norb)
    r0 = oracle.ace_build(o.psi, pairs, s.N, s.L, "erfc", s.omega)
    q, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(s.norb, s.norb)))
    rot = np.einsum("ik,izyx->kzyx", q, o.psi)
    r1 = oracle.ace_build(rot, pairs, s.N, s.L, "erfc", s.omega)
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    r2 = oracle.ace_build(phi, pairs, s.N, s.L, "erfc", s.omega)
    assert abs(r1["ex"] - r0["ex"]) < 1e-12 * abs(r0["ex"])
    assert abs(r2["ex"] - r0["ex"]) < 1e-12 * abs(r0["ex"])
    X = np.random.default_rng(4).normal(size=(3,) + o.psi.shape[1:])
    y0 = oracle.ace_apply(r0["xi"], X, s.dV)
    for r in (r1, r2):
        np.testing.assert_allclose(oracle.ace_apply(r["xi"], X, s.dV), y0, atol=1e-12 * np.abs(y0).max())


def test_p4_energy_routes_agree(small_system):
    o = small_system
    s = o.spec
    v = oracle.coulomb_kernel(s.N, s.L, "erfc", s.omega)
    for i, j in [(0, 0), (0, 3), (2, 7)]:
        vij = oracle.pair_potential(o.psi[i], o.psi[j], v)
        e_real = -(1 if i == j else 2) * s.dV * np.sum(o.psi[i] * o.psi[j] * vij)
        e_fwd = oracle.pair_energy_forward(o.psi[i], o.psi[j], v, s.dV, i == j)
        assert abs(e_real - e_fwd) < 1e-13 * abs(e_real)


def test_p4_not_pd_raises(small_system):
    o = small_system
    s = o.spec
    v = oracle.coulomb_kernel(s.N, s.L, "erfc", s.omega)
    W = oracle.build_W(o.psi, _full_pairs(s.norb), v, s.dV)
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.ace_from_W(o.psi, -W, s.dV)


# ----------------------------------------------------------------- P5

def test_p5_pivots_match_lapack_dgeqp3():
    o = make_orbitals(config_spec("c1"))
    A = o.psi.reshape(o.spec.norb, -1)
    piv, _ = oracle.qrcp_pivots(A)
    _, ref = sla.qr(A, pivoting=True, mode="r")
    np.testing.assert_array_equal(piv, ref[: len(piv)])
    assert piv[0] == np.argmax((A * A).sum(0))


def _same_density_matrix(P, A, probes=6):
    """P^T P = A^T A (the density matrix of Eq. unit is unchanged by the
    rotation), checked on seeded random probe vectors instead of forming the
    N_G x N_G matrices."""
    R = np.random.default_rng(5).normal(size=(A.shape[1], probes))
    lhs, rhs = P.T @ (P @ R), A.T @ (A @ R)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(rhs).max())


def test_p5_scdm_invariances():
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    n = s.norb
    piv, U, phi = oracle.scdm_localize(o.psi, s.dV)
    A = o.psi.reshape(n, -1)
    P = phi.reshape(n, -1)
    np.testing.assert_allclose(P @ P.T * s.dV, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-12)
    _same_density_matrix(P, A)
    q, _ = np.linalg.qr(np.random.default_rng(21).normal(size=(n, n)))
    piv2, _, phi2 = oracle.scdm_localize(np.einsum("ik,izyx->kzyx", q, o.psi), s.dV)
    np.testing.assert_array_equal(piv, piv2)
    np.testing.assert_allclose(phi2, phi, atol=1e-10 * np.abs(phi).max())


def test_p5_disjoint_orbitals_come_back():
    spec = SystemSpec(n_mol=1, L=16.0, N=32, sigma=0.7, seed=1)
    cen = [(2, 2, 2), (10, 2, 2), (2, 10, 2), (2, 2, 10), (10, 10, 10)]
    g = disjoint_gaussians(spec, cen)
    S = np.einsum("azyx,bzyx->ab", g, g) * spec.dV
    w, V = np.linalg.eigh(S)
    g = np.einsum("ab,bzyx->azyx", V @ np.diag(w ** -0.5) @ V.T, g)
    q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(5, 5)))
    psi = np.einsum("ik,izyx->kzyx", q, g)
    _, _, phi = oracle.scdm_localize(psi, spec.dV)
    ov = np.abs(np.einsum("azyx,bzyx->ab", phi, g) * spec.dV)
    # each SCDM orbital is one of the inputs, up to order and sign
    np.testing.assert_allclose(np.sort(ov.max(1)), np.ones(5), atol=1e-9)
    assert np.all(np.sort(ov, axis=1)[:, -2] < 1e-6)


def test_p5_localization_reduces_overlap_mass():
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    before = oracle.overlap_abs(o.psi, s.dV)
    after = oracle.overlap_abs(phi, s.dV)
    off = ~np.eye(s.norb, dtype=bool)
    assert after[off].mean() < 0.8 * before[off].mean()


# ----------------------------------------------------------------- P6

def test_p6_screening_identities():
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    full, _ = oracle.pairlist(phi, s.dV, 0.0)
    assert len(full) == s.norb * (s.norb + 1) // 2
    diag, _ = oracle.pairlist(phi, s.dV, 1.5)
    np.testing.assert_array_equal(diag, np.stack([np.arange(s.norb)] * 2, 1))
    kept, Ok = oracle.pairlist(phi, s.dV, 0.2)
    assert 0 < len(kept) - s.norb < len(full) - s.norb
    # brute-force per-pair integrals
    for (i, j), oij in zip(kept, Ok):
        assert abs(oij - s.dV * np.sum(np.abs(phi[i] * phi[j]))) < 1e-13
    rf = oracle.ace_build(phi, full, s.N, s.L, "bare", 0.1)
    rs = oracle.ace_build(phi, kept, s.N, s.L, "bare", 0.1)
    kset = {tuple(p) for p in kept}
    dropped = sum(e for p, e in zip(full, rf["e"]) if tuple(p) not in kset)
    assert abs((rs["ex"] - rf["ex"]) - (-dropped)) < 1e-13 * abs(rf["ex"])


# ----------------------------------------------------------------- P7

def test_p7_single_orbital_closed_form():
    spec = SystemSpec(n_mol=1, L=7.0, N=16, sigma=0.8, seed=5)
    g = disjoint_gaussians(spec, [(3.0, 3.5, 2.0)])
    r = oracle.ace_build(g, [(0, 0)], spec.N, spec.L, "erfc", 0.4)
    m = r["M"][0, 0]
    assert m < 0
    np.testing.assert_allclose(r["xi"][0], r["W"][0] / np.sqrt(-m), rtol=1e-13, atol=1e-300)
    v = oracle.coulomb_kernel(spec.N, spec.L, "erfc", 0.4)
    jj = spec.dV * np.sum(g[0] ** 2 * oracle.pair_potential(g[0], g[0], v))
    assert abs(r["ex"] + jj) < 1e-13 * jj


# ----------------------------------------------------------------- P8

def test_p8_apply_energy_is_trace_of_M(small_system):
    """With the build's own orbitals and the full list, sum_i <phi_i|V_ACE|phi_i> = tr M
    (V_ACE phi = W once M = Phi^T W dV is symmetric), for canonical and SCDM orbitals."""
    o = small_system
    s = o.spec
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    for orbs in (o.psi, phi):
        r = oracle.ace_build(orbs, _full_pairs(s.norb), s.N, s.L, "erfc", s.omega)
        Y, e = oracle.ace_apply_energy(r["xi"], orbs, s.dV)
        np.testing.assert_allclose(Y, r["W"], atol=1e-12 * np.abs(r["W"]).max())
        assert abs(e - r["ex"]) < 1e-12 * abs(r["ex"])
        assert abs(e - np.trace(r["M"])) < 1e-12 * abs(r["ex"])


def test_p8_apply_energy_sign_and_mixing_invariance(small_system):
    o = small_system
    s = o.spec
    r = oracle.ace_build(o.psi, _full_pairs(s.norb), s.N, s.L, "erfc", s.omega)
    rng = np.random.default_rng(12)
    X = rng.normal(size=(4,) + o.psi.shape[1:])
    _, e = oracle.ace_apply_energy(r["xi"], X, s.dV)
    assert e < 0
    q, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    _, eq = oracle.ace_apply_energy(r["xi"], np.einsum("ab,bzyx->azyx", q, X), s.dV)
    assert abs(eq - e) < 1e-12 * abs(e)
    # each function's energy is its own quadratic form: scaling one by t scales its share by t^2
    _, e0 = oracle.ace_apply_energy(r["xi"], X[:1], s.dV)
    _, e0s = oracle.ace_apply_energy(r["xi"], 3.0 * X[:1], s.dV)
    assert abs(e0s - 9.0 * e0) < 1e-12 * abs(e0s)


# ----------------------------------------------------------------- P9

def test_p9_exact_exchange_matches_pair_symmetric_build(small_system):
    o = small_system
    s = o.spec
    W, M, ex = oracle.exact_exchange(o.psi, s.N, s.L, "erfc", s.omega)
    r = oracle.ace_build(o.psi, _full_pairs(s.norb), s.N, s.L, "erfc", s.omega)
    np.testing.assert_allclose(W, r["W"], atol=1e-12 * np.abs(W).max())
    np.testing.assert_allclose(M, r["M"], atol=1e-13 * np.abs(M).max())
    assert abs(ex - r["ex"]) < 1e-12 * abs(ex)
    assert np.linalg.eigvalsh(M).max() < 0
    np.testing.assert_allclose(M, M.T, atol=0)


def test_p9_exact_exchange_rotation_invariance(small_system):
    o = small_system
    s = o.spec
    _, M0, ex0 = oracle.exact_exchange(o.psi, s.N, s.L, "bare", 0.0)
    q, _ = np.linalg.qr(np.random.default_rng(21).normal(size=(s.norb, s.norb)))
    rot = np.einsum("ik,izyx->kzyx", q, o.psi)
    W1, M1, ex1 = oracle.exact_exchange(rot, s.N, s.L, "bare", 0.0)
    assert abs(ex1 - ex0) < 1e-12 * abs(ex0)
    # M transforms as Q^T M Q
    np.testing.assert_allclose(M1, q.T @ M0 @ q, atol=1e-12 * np.abs(M0).max())


def test_p9_exact_exchange_single_orbital():
    """One normalized Gaussian: W = -v_gg g and E_x = -dV sum g^2 v_gg, where
    v_gg is pinned against the analytic erfc self-energy (P3)."""
    spec = SystemSpec(n_mol=1, L=7.0, N=16, sigma=0.8, seed=5)
    g = disjoint_gaussians(spec, [(3.0, 3.5, 2.0)])
    W, M, ex = oracle.exact_exchange(g, spec.N, spec.L, "erfc", 0.4)
    v = oracle.coulomb_kernel(spec.N, spec.L, "erfc", 0.4)
    vgg = oracle.pair_potential(g[0], g[0], v)
    np.testing.assert_allclose(W[0], -vgg * g[0], rtol=0, atol=1e-14 * np.abs(W).max())
    jj = spec.dV * np.sum(g[0] ** 2 * vgg)
    assert M.shape == (1, 1) and abs(ex + jj) < 1e-13 * jj


# ----------------------------------------------------------------- P10

def test_p10_lowdin_on_reused_columns():
    """Pivots of MD step 0 reused at step 1: U is the orthogonal polar factor of
    A_C (A_C = U H, H symmetric positive definite), Phi is orthonormal and
    spans the occupied space of step 1, and fresh pivots reproduce SCDM."""
    s0 = config_spec("c1")
    psi0 = make_orbitals(s0).psi
    psi1 = make_orbitals(s0.replace(md_step=1)).psi
    n = s0.norb
    piv0, _ = oracle.qrcp_pivots(psi0.reshape(n, -1))
    U, phi = oracle.lowdin_columns(psi1, piv0)
    A1 = psi1.reshape(n, -1)
    AC = A1[:, piv0]
    H = U.T @ AC
    np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(H, H.T, atol=1e-13 * np.abs(H).max())
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0
    P = phi.reshape(n, -1)
    np.testing.assert_allclose(P @ P.T * s0.dV, np.eye(n), atol=1e-12)
    _same_density_matrix(P, A1)
    # with the step's own pivots it is SCDM itself
    piv1, U1, phi1 = oracle.scdm_localize(psi1, s0.dV)
    U1b, phi1b = oracle.lowdin_columns(psi1, piv1)
    np.testing.assert_array_equal(U1b, U1)
    # the reused columns still localize: each orbital peaks at its own pivot
    assert np.all(np.abs(P[np.arange(n), piv0]) >= np.abs(P[:, piv0]).max(axis=0) * (1 - 1e-12))


def test_p10_lowdin_rejects_bad_columns():
    s0 = config_spec("c1")
    psi = make_orbitals(s0).psi
    n = s0.norb
    good = np.arange(n) * 37
    with pytest.raises(ValueError):
        oracle.lowdin_columns(psi, np.r_[good[:-1], good[0]])
    with pytest.raises(ValueError):
        oracle.lowdin_columns(psi, np.r_[good[:-1], s0.N ** 3])
    with pytest.raises(ValueError):
        oracle.lowdin_columns(psi, good[:-1])


# ----------------------------------------------------------------- P11
# The sampled helpers that serve as references at sizes where the whole
# build is too slow for the oracle: each is pinned to the pinned serial build.

def _ragged_list(n, seed):
    rng = np.random.default_rng(seed)
    full = _full_pairs(n)
    keep = (full[:, 0] == full[:, 1]) | (rng.random(len(full)) < 0.45)
    return full[keep]


@pytest.mark.parametrize("which", ["full", "ragged"])
def test_p11_build_W_rows_equals_rows_of_build_W(which):
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    pairs = _full_pairs(s.norb) if which == "full" else _ragged_list(s.norb, 11)
    v = oracle.coulomb_kernel(s.N, s.L, "erfc", 0.3)
    W = oracle.build_W(phi, pairs, v, s.dV)
    # every row, in a shuffled order, with a repeat: rows are independent of each other
    rows = [5, 0, 7, 3, 3, 1, 6, 2, 4]
    Wr = oracle.build_W_rows(phi, pairs, rows, v, workers=3)
    assert Wr.shape == (len(rows),) + phi.shape[1:]
    np.testing.assert_allclose(Wr, W[rows], rtol=0, atol=1e-14 * np.abs(W).max())
    # an orbital whose only kept pair is its diagonal
    lone = np.array([(0, 0), (1, 1), (1, 2), (2, 2)])
    Wl = oracle.build_W_rows(phi, lone, [0, 1, 2], v, workers=2)
    np.testing.assert_allclose(Wl[0], -oracle.pair_potential(phi[0], phi[0], v) * phi[0], rtol=0, atol=1e-300)
    np.testing.assert_allclose(Wl, oracle.build_W(phi, lone, v, s.dV)[:3], rtol=0,
                               atol=1e-14 * np.abs(Wl).max())


@pytest.mark.parametrize("which", ["full", "ragged"])
@pytest.mark.parametrize("kind", ["bare", "erfc"])
def test_p11_exchange_energy_pairs_equals_build_energies_and_trace(which, kind):
    """The Parseval route (forward transform only) against the real-space route
    dV sum rho v of the full build, and their sum against tr M."""
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    pairs = _full_pairs(s.norb) if which == "full" else _ragged_list(s.norb, 12)
    v = oracle.coulomb_kernel(s.N, s.L, kind, 0.3)
    e = oracle.exchange_energy_pairs(phi, pairs, v, s.dV, workers=3)
    W, e_real = oracle.build_W(phi, pairs, v, s.dV, energies=True)
    np.testing.assert_allclose(e, e_real, rtol=1e-13, atol=1e-15)
    assert np.all(e < 0)
    # tr M counts an off-diagonal pair once in row i and once in row j: this fixes
    # the weights 1 (diagonal) and 2 (off-diagonal) of the pair energies
    tr = float(np.trace(s.dV * phi.reshape(s.norb, -1) @ W.reshape(s.norb, -1).T))
    assert abs(e.sum() - tr) < 1e-13 * abs(tr)
    if which == "full":
        r = oracle.ace_build(phi, pairs, s.N, s.L, kind, 0.3)
        assert abs(e.sum() - r["ex"]) < 1e-13 * abs(r["ex"])


def test_p11_threaded_build_W_is_bitwise_serial():
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    pairs = _ragged_list(s.norb, 13)
    v = oracle.coulomb_kernel(s.N, s.L, "bare", 0.0)
    W1, e1 = oracle.build_W(o.psi, pairs, v, s.dV, energies=True)
    for workers in (2, 3, 5):
        Wt, et = oracle.build_W(o.psi, pairs, v, s.dV, energies=True, workers=workers)
        assert np.array_equal(Wt, W1) and np.array_equal(et, e1)
    r1 = oracle.ace_build(o.psi, _full_pairs(s.norb), s.N, s.L, "erfc", 0.2)
    r4 = oracle.ace_build(o.psi, _full_pairs(s.norb), s.N, s.L, "erfc", 0.2, workers=4)
    assert np.array_equal(r1["xi"], r4["xi"]) and r1["ex"] == r4["ex"]


# ----------------------------------------------------------------- P12
# The next MD step: the previous columns as the warm start, the re-screen
# against the previous list.

def test_p12_column_quality_is_the_qrcp_residual_ratio():
    """On fresh SCDM columns the R diagonal of A_C = Q R holds the residual
    norms greedy QRCP picked its columns with (q_k . a_{p_k})."""
    o = make_orbitals(config_spec("c1"))
    n = o.spec.norb
    A = o.psi.reshape(n, -1)
    piv, Q = oracle.qrcp_pivots(A)
    r = np.abs(np.einsum("ik,ik->k", Q, A[:, piv]))
    assert abs(oracle.column_quality(o.psi, piv) - (r.max() / r.min()) ** 2) < 1e-12 * (r.max() / r.min()) ** 2
    # greedy pivoting: the picked residual norms never increase
    assert np.all(np.diff(r) <= 1e-12 * r[0])


def test_p12_column_quality_bounds_and_diagonal_case():
    s0 = config_spec("c1")
    psi = make_orbitals(s0.replace(md_step=2)).psi
    n = s0.norb
    piv0, _ = oracle.qrcp_pivots(make_orbitals(s0).psi.reshape(n, -1))
    q = oracle.column_quality(psi, piv0)
    AC = psi.reshape(n, -1)[:, piv0]
    w = np.linalg.eigvalsh(AC.T @ AC)
    assert 1.0 <= q <= w.max() / w.min() * (1 + 1e-12)
    # disjoint Gaussians sampled at their own centres: A_C is diagonal up to
    # the tiny tails, and the ratio is that of the squared peak values
    spec = SystemSpec(n_mol=1, L=12.0, N=24, sigma=0.6, seed=9)
    cen = [(2.0, 2.0, 2.0), (8.0, 2.0, 2.0), (2.0, 8.0, 8.0), (8.0, 8.0, 5.0)]
    g = disjoint_gaussians(spec, cen)
    g[1] *= 0.5
    h = spec.L / spec.N
    idx = [int(round(z / h)) * spec.N ** 2 + int(round(y / h)) * spec.N + int(round(x / h)) for x, y, z in cen]
    peaks = np.array([g[k].reshape(-1)[idx[k]] for k in range(4)])
    assert abs(oracle.column_quality(g, idx) - (peaks.max() / peaks.min()) ** 2) < 1e-8 * (peaks.max() / peaks.min()) ** 2
    assert oracle.column_quality(g, [idx[0], idx[0] + 1, idx[0] + 2, idx[0] + 3]) > 1e3


def test_p12_localize_step_keeps_or_refreshes_columns():
    s0 = config_spec("c1")
    psi0 = make_orbitals(s0).psi
    psi1 = make_orbitals(s0.replace(md_step=1)).psi
    n = s0.norb
    piv0, _, _ = oracle.scdm_localize(psi0, s0.dV)
    piv, U, phi, reused, q = oracle.localize_step(psi1, piv0, s0.dV, 2.0)
    assert reused and np.array_equal(piv, piv0) and 1.0 < q < 2.0
    U_ref, phi_ref = oracle.lowdin_columns(psi1, piv0)
    assert np.array_equal(U, U_ref) and np.array_equal(phi, phi_ref)
    # a ratio no real column set reaches: fresh SCDM, exactly
    piv, U, phi, reused, _ = oracle.localize_step(psi1, piv0, s0.dV, 1.0)
    pf, Uf, phif = oracle.scdm_localize(psi1, s0.dV)
    assert not reused and np.array_equal(piv, pf) and np.array_equal(phi, phif)


def test_p12_pairlist_step_counts_crossings():
    s0 = config_spec("c1")
    n = s0.norb
    piv0, _, phi0 = oracle.scdm_localize(make_orbitals(s0).psi, s0.dV)
    prev, _ = oracle.pairlist(phi0, s0.dV, 0.05)
    for t in (1, 2, 3):
        psi = make_orbitals(s0.replace(md_step=t)).psi
        _, _, phi, _, _ = oracle.localize_step(psi, piv0, s0.dV, 2.0)
        pairs, O, added, removed = oracle.pairlist_step(phi, s0.dV, 0.05, prev)
        np.testing.assert_array_equal(pairs, oracle.pairlist(phi, s0.dV, 0.05)[0])
        # brute force over every pair of orbitals
        Ofull = np.array([[s0.dV * np.sum(np.abs(phi[i] * phi[j])) for j in range(n)] for i in range(n)])
        was = {tuple(p) for p in prev.tolist()}
        a = sum(1 for i in range(n) for j in range(i, n) if (i == j or Ofull[i, j] >= 0.05) and (i, j) not in was)
        r = sum(1 for (i, j) in was if not (i == j or Ofull[i, j] >= 0.05))
        assert (added, removed) == (a, r)
        assert len(pairs) == len(prev) + added - removed
        prev = pairs
    assert oracle.pairlist_step(phi, s0.dV, 0.05, prev)[2:] == (0, 0)


def test_p12_full_list_energy_is_the_same_for_kept_and_fresh_columns():
    """With every pair the exchange energy does not depend on which columns
    localized the orbitals (rotation invariance), at each MD step."""
    s0 = config_spec("c1")
    n = s0.norb
    piv0, _, _ = oracle.scdm_localize(make_orbitals(s0).psi, s0.dV)
    full = _full_pairs(n)
    for t in (1, 2, 3):
        psi = make_orbitals(s0.replace(md_step=t)).psi
        _, _, phi_r, reused, _ = oracle.localize_step(psi, piv0, s0.dV, 2.0)
        _, _, phi_f, fresh, _ = oracle.localize_step(psi, piv0, s0.dV, 1.0)
        assert reused and not fresh
        er = oracle.ace_build(phi_r, full, s0.N, s0.L, "bare", 0.1)["ex"]
        ef = oracle.ace_build(phi_f, full, s0.N, s0.L, "bare", 0.1)["ex"]
        assert abs(er - ef) < 1e-12 * abs(ef)
