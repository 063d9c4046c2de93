"""GPU parity of the k-point build (complex Bloch orbitals) against the FP64
k-point oracle on the same seeded inputs: pair lists exactly, W, M and xi
element by element, E_x to 1e-10 relative.  The oracle is pinned by
tests/test_oracle_kpoints.py (Gamma point = real build, naive DFT, supercell
folding, unitary invariance)."""
import numpy as np
import pytest

import oracle
from oracle import kpoint_oracle as ko
from synth import SystemSpec, config_spec, make_bloch_orbitals, make_orbitals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context()


def _grid(n, L):
    from paper_2101_03155_amd import Grid
    return Grid.cubic(n, L)


def _close(a, ref, tol, what):
    err = float(np.abs(np.asarray(a) - np.asarray(ref)).max() / np.abs(np.asarray(ref)).max())
    print(f"  {what}: max elementwise err {err:.3e} (tol {tol:.0e})", flush=True)
    assert err <= tol, what


def test_gamma_real_orbitals_match_real_build(ctx):
    _say("k-points: Gamma point with real orbitals vs the real build")
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    _, _, phi = oracle.scdm_localize(o.psi, s.dV)
    pairs = ko.full_pairs(s.norb).astype(np.int32)
    g = _grid(s.N, s.L)
    dp = torch.as_tensor(pairs, device="cuda")
    rr = ctx.build(torch.as_tensor(phi, device="cuda"), dp, g, kernel="bare", want_W=True)
    rk = ctx.build_kpoints(torch.as_tensor(phi.astype(np.complex128), device="cuda"), [(0.0, 0.0, 0.0)], s.norb, dp, g,
                           kernel="bare", want_W=True)
    assert abs(rk["ex"].item() - rr["ex"].item()) <= 1e-12 * abs(rr["ex"].item())
    _close(rk["W"].cpu().numpy().real, rr["W"].cpu().numpy(), 1e-12, "W")
    _close(rk["xi"].cpu().numpy().real, rr["xi"].cpu().numpy(), 1e-11, "xi")
    assert np.abs(rk["xi"].cpu().numpy().imag).max() <= 1e-12 * np.abs(rr["xi"].cpu().numpy()).max()


KCASES = [
    # (grid, molecules, k-points (fractional), kernel, rho_cut); screened cases use
    # unmixed (localized) Bloch sums, which the criterion can tell apart
    (12, 1, [(0, 0, 0), (0.5, 0, 0)], "bare", 0.0),
    (16, 2, [(0, 0, 0), (0.5, 0, 0), (0, 0.5, 0.5)], "erfc", 0.0),
    (24, 2, [(0, 0, 0), (0.5, 0.5, 0.5)], "erfc", 0.02),
    (32, 3, [(0, 0, 0), (0.25, 0, 0), (0.5, 0, 0), (0.75, 0, 0)], "bare", 0.02),
    (48, 4, [(0, 0, 0), (0.5, 0, 0), (0, 0.5, 0), (0.5, 0.5, 0)], "erfc", 5e-3),
    (64, 6, [(0, 0, 0), (0.5, 0.5, 0.5)], "erfc", 1e-3),
]


@pytest.mark.parametrize("n,nmol,kf,kind,rho_cut", KCASES)
def test_kpoint_build_matches_oracle(ctx, n, nmol, kf, kind, rho_cut):
    _say(f"k-points N={n} molecules={nmol} nk={len(kf)} {kind} rho_cut={rho_cut}")
    spec = SystemSpec(n_mol=nmol, L=0.45 * n, N=n, sigma=0.8, offset=0.7, placement="uniform", seed=600 + n,
                      kernel=kind, omega=0.5)
    u, kv = make_bloch_orbitals(spec, kf, mix=rho_cut == 0.0)
    norb = spec.norb
    g = _grid(n, spec.L)
    ud = torch.as_tensor(u, device="cuda")
    pairs_ref, ov_ref = ko.pairlist_k(u, spec.dV, rho_cut)
    pg, og = ctx.pairlist_kpoints(ud, g, rho_cut)
    np.testing.assert_array_equal(pg.cpu().numpy(), pairs_ref)
    np.testing.assert_allclose(og.cpu().numpy(), ov_ref, rtol=1e-12, atol=1e-15)
    ref = ko.ace_build_k(u, kv, norb, pairs_ref, n, spec.L, kind, 0.5)
    r = ctx.build_kpoints(ud, [tuple(k) for k in kv], norb, pg, g, kernel=kind, omega=0.5, want_W=True)
    ex = r["ex"].item()
    print(f"  {len(pairs_ref)} of {u.shape[0] * (u.shape[0] + 1) // 2} pairs of {u.shape[0]} Bloch orbitals; "
          f"E_x {ex:.12f} oracle {ref['ex']:.12f}", flush=True)
    if rho_cut > 0.0:
        assert len(pairs_ref) < u.shape[0] * (u.shape[0] + 1) // 2  # the criterion drops pairs here
    assert abs(ex - ref["ex"]) <= 1e-10 * abs(ref["ex"])
    _close(r["W"].cpu().numpy(), ref["W"], 1e-12, "W")
    _close(r["M"].cpu().numpy(), ref["M"], 1e-12, "M")
    _close(r["xi"].cpu().numpy(), ref["xi"], 1e-10, "xi")
    # V_ACE psi = W for the full list, per k-point (through the returned projectors)
    if rho_cut == 0.0:
        xi = r["xi"].cpu().numpy()
        for q in range(len(kf)):
            sl = slice(q * norb, (q + 1) * norb)
            y = ko.ace_apply_k(xi[sl], u[sl], spec.dV)
            _close(y, ref["W"][sl], 1e-11, f"V_ACE psi = W at k-point {q}")


def test_kpoint_errors(ctx):
    from paper_2101_03155_amd import AceError
    spec = SystemSpec(n_mol=1, L=6.0, N=12, sigma=0.8, offset=0.7, placement="uniform", seed=5)
    u, kv = make_bloch_orbitals(spec, [(0, 0, 0), (0.5, 0, 0)])
    ud = torch.as_tensor(u, device="cuda")
    g = _grid(12, spec.L)
    # one off-diagonal pair leaves the other orbitals with W = 0: -M singular
    with pytest.raises(AceError) as ei:
        ctx.build_kpoints(ud, [tuple(k) for k in kv], spec.norb, torch.tensor([[0, 5]], dtype=torch.int32,
                                                                              device="cuda"), g)
    assert ei.value.status == "ACE_E_NOT_PD"
    for bad in ([[0, 0], [0, 0]], [[3, 1]], [[0, 8]]):
        with pytest.raises(AceError) as ei:
            ctx.build_kpoints(ud, [tuple(k) for k in kv], spec.norb, torch.tensor(bad, dtype=torch.int32,
                                                                                  device="cuda"), g)
        assert ei.value.status == "ACE_E_ARG"
