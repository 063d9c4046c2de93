"""Pins of the k-point (complex Bloch orbital) oracle against facts that do
not come from it: the real build at the Gamma point, a naive DFT of the
shifted-kernel convolution, the supercell that a k-point sampling unfolds to,
unitary invariance, and the ACE algebra of Appendix A with conjugates."""
import numpy as np
import pytest

import oracle
from oracle import kpoint_oracle as ko
from synth import SystemSpec, config_spec, make_bloch_orbitals, make_orbitals


def _spec(**kw):
    base = dict(n_mol=1, L=7.0, N=14, sigma=0.8, offset=0.7, placement="uniform", seed=21, kernel="erfc",
                omega=0.4)
    base.update(kw)
    return SystemSpec(**base)


def test_k1_gamma_real_orbitals_are_the_real_build():
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    pairs = ko.full_pairs(s.norb)
    for kind in ("bare", "erfc"):
        r = oracle.ace_build(phi, pairs, s.N, s.L, kind, 0.3)
        rk = ko.ace_build_k(phi.astype(np.complex128), [(0, 0, 0)], s.norb, pairs, s.N, s.L, kind, 0.3)
        assert abs(rk["ex"] - r["ex"]) < 1e-13 * abs(r["ex"])
        np.testing.assert_allclose(rk["W"].real, r["W"], rtol=0, atol=1e-13 * np.abs(r["W"]).max())
        assert np.abs(rk["W"].imag).max() < 1e-13 * np.abs(r["W"]).max()
        np.testing.assert_allclose(rk["M"][0].real, r["M"], rtol=0, atol=1e-13 * np.abs(r["M"]).max())
        np.testing.assert_allclose(rk["xi"].real, r["xi"], rtol=0, atol=1e-12 * np.abs(r["xi"]).max())
        np.testing.assert_allclose(rk["e"], r["e"], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("kind", ["bare", "erfc"])
def test_k2_shifted_convolution_matches_naive_dft(kind):
    n, L = 6, 5.0
    rng = np.random.default_rng(8)
    ua = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    ub = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    d = np.array([0.3, -0.2, 0.55])
    f = np.conj(ua) * ub
    # direct sums over the grid: P[f](r) = N^-1 sum_G v(|G + d|) sum_r' f(r') e^{-i G.r'} e^{i G.r}
    m = np.where(np.arange(n) < (n + 1) // 2, np.arange(n), np.arange(n) - n)
    g = 2 * np.pi * m / L
    x = np.arange(n) * L / n
    out = np.zeros((n, n, n), dtype=complex)
    pos = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1)  # (z, y, x) -> coordinates (z, y, x)
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                G = np.array([g[ix], g[iy], g[iz]])
                q2 = float(np.sum((G + d) ** 2))
                v = 4 * np.pi / q2 if kind == "bare" else 4 * np.pi / q2 * (1 - np.exp(-q2 / (4 * 0.7 ** 2)))
                ph = np.exp(-1j * (G[0] * pos[..., 2] + G[1] * pos[..., 1] + G[2] * pos[..., 0]))
                coef = v * np.sum(f * ph)
                out += coef * np.conj(ph)
    out /= n ** 3
    got = ko.pair_potential_k(ua, ub, ko.shifted_kernel(n, L, kind, 0.7, d))
    np.testing.assert_allclose(got, out, rtol=0, atol=1e-12 * np.abs(out).max())


@pytest.mark.parametrize("kind", ["bare", "erfc"])
def test_k3_kpoint_sampling_equals_its_supercell(kind):
    """Two k-points {0, 1/2} along x on a cell of length L are the Gamma point
    of the supercell 2L x L x L: the unfolded orbitals exp(i k.r) u(r)/sqrt 2
    give the supercell E_x = 2 E_x(cell), and W unfolds the same way."""
    spec = _spec(N=12, L=6.0, seed=5)
    u, kv = make_bloch_orbitals(spec, [(0, 0, 0), (0.5, 0, 0)])
    n, N, L = spec.norb, spec.N, spec.L
    pairs = ko.full_pairs(2 * n)
    rk = ko.ace_build_k(u, kv, n, pairs, N, L, kind, 0.6)
    # unfold onto the (2N) x N x N supercell grid, axes (z, y, x)
    xs = np.arange(2 * N) * (L / N)
    sc = np.empty((2 * n, N, N, 2 * N), dtype=complex)
    Wsc_ref = np.empty_like(sc)
    for q in range(2):
        ph = np.exp(1j * kv[q, 0] * xs)[None, None, :] / np.sqrt(2.0)
        for m in range(n):
            a = q * n + m
            sc[a] = np.concatenate([u[a], u[a]], axis=-1) * ph
            Wsc_ref[a] = np.concatenate([rk["W"][a], rk["W"][a]], axis=-1) * ph
    rs = ko.ace_build_k(sc, [(0, 0, 0)], 2 * n, pairs, (2 * N, N, N), (2 * L, L, L), kind, 0.6)
    assert abs(rs["ex"] - 2.0 * rk["ex"]) < 1e-12 * abs(rs["ex"])
    np.testing.assert_allclose(rs["W"], Wsc_ref, rtol=0, atol=1e-12 * np.abs(Wsc_ref).max())


def test_k4_unitary_invariance_and_ace_algebra():
    spec = _spec(n_mol=2, N=12, L=7.0, seed=31)
    u, kv = make_bloch_orbitals(spec, [(0, 0, 0), (0.5, 0, 0), (0, 0.5, 0.5)])
    n = spec.norb
    pairs = ko.full_pairs(3 * n)
    r = ko.ace_build_k(u, kv, n, pairs, spec.N, spec.L, "erfc", 0.5)
    rng = np.random.default_rng(2)
    u2 = u.copy()
    Us = []
    for q in range(3):
        z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        U, _ = np.linalg.qr(z)
        Us.append(U)
        blk = u[q * n:(q + 1) * n].reshape(n, -1)
        u2[q * n:(q + 1) * n] = (U.T @ blk).reshape(u[q * n:(q + 1) * n].shape)
    r2 = ko.ace_build_k(u2, kv, n, pairs, spec.N, spec.L, "erfc", 0.5)
    assert abs(r2["ex"] - r["ex"]) < 1e-12 * abs(r["ex"])
    for q in range(3):
        M, M2, U = r["M"][q], r2["M"][q], Us[q]
        np.testing.assert_allclose(M2, U.conj().T @ M @ U, rtol=0, atol=1e-12 * np.abs(M).max())
        assert np.abs(M - M.conj().T).max() < 1e-13 * np.abs(M).max()
        assert np.linalg.eigvalsh(M).max() < 0
        # V_ACE psi = W on each k-point's occupied space, and <psi|V_ACE|psi> = M
        sl = slice(q * n, (q + 1) * n)
        y = ko.ace_apply_k(r["xi"][sl], u[sl], spec.dV)
        np.testing.assert_allclose(y, r["W"][sl], rtol=0, atol=1e-12 * np.abs(r["W"]).max())
    assert r["asym"] < 1e-12 * np.abs(r["M"]).max()
    # the pair energies sum to E_x = (1/N_k) sum_k tr M_k
    assert abs(r["e"].sum() - r["ex"]) < 1e-13 * abs(r["ex"])
    assert abs(np.mean([np.trace(M).real for M in r["M"]]) - r["ex"]) < 1e-13 * abs(r["ex"])


def test_k5_screening_identity_and_limits():
    spec = _spec(n_mol=2, N=12, L=9.0, seed=44)
    u, kv = make_bloch_orbitals(spec, [(0, 0, 0), (0.5, 0.5, 0)])
    ntot = u.shape[0]
    full, _ = ko.pairlist_k(u, spec.dV, 0.0)
    assert len(full) == ntot * (ntot + 1) // 2
    diag, _ = ko.pairlist_k(u, spec.dV, 2.0)
    np.testing.assert_array_equal(diag, np.stack([np.arange(ntot)] * 2, 1))
    kept, Ok = ko.pairlist_k(u, spec.dV, 0.05)
    for (a, b), o in zip(kept, Ok):
        assert abs(o - spec.dV * np.sum(np.abs(u[a] * np.conj(u[b])))) < 1e-13
    rf = ko.ace_build_k(u, kv, spec.norb, full, spec.N, spec.L, "erfc", 0.5)
    rs = ko.ace_build_k(u, kv, spec.norb, kept, spec.N, spec.L, "erfc", 0.5)
    ks = {tuple(p) for p in kept.tolist()}
    dropped = sum(e for p, e in zip(full.tolist(), rf["e"]) if tuple(p) not in ks)
    assert abs((rs["ex"] - rf["ex"]) + dropped) < 1e-13 * abs(rf["ex"])
