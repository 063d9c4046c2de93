"""GPU parity: every C-ABI entry point against the FP64 oracle on the same
seeded inputs.  Tolerances: |dE_x|/|E_x| <= 1e-10 (FP64) and <= 1e-6 (FP32);
ACE matrix elements <= 1e-5 Ha; integer outputs (pivots, pair lists) exact."""
import numpy as np
import pytest

import oracle
from synth import SystemSpec, config_spec, make_orbitals, smooth_test_vectors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _full_pairs(n):
    return np.array([(i, j) for i in range(n) for j in range(i, n)], dtype=np.int32)


def _grid(spec):
    from paper_2101_03155_amd import Grid
    return Grid.cubic(spec.N, spec.L)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _elem_err(a, ref):
    """max |a - ref| over every element, relative to max |ref|."""
    a, ref = np.asarray(a), np.asarray(ref)
    return float(np.abs(a - ref).max() / np.abs(ref).max())


def _close(a, ref, tol, what=""):
    err = _elem_err(a, ref)
    print(f"  {what}: max elementwise err {err:.3e} (tol {tol:.0e})", flush=True)
    assert err <= tol, f"{what}: {err:.3e} > {tol:.0e}"


# ------------------------------------------------------------------ GEMMs via apply

@pytest.mark.parametrize("norb,nvec,n", [(5, 3, 8), (70, 66, 12), (130, 1, 16)])
def test_apply_matches_oracle_ragged(ctx, norb, nvec, n):
    _say(f"apply norb={norb} nvec={nvec} N={n}")
    from paper_2101_03155_amd import Grid
    rng = np.random.default_rng(norb * 1000 + nvec)
    xi = rng.normal(size=(norb, n, n, n))
    x = rng.normal(size=(nvec, n, n, n))
    g = Grid.cubic(n, 6.0)
    y = ctx.apply(_dev(xi), _dev(x), g).cpu().numpy()
    ref = oracle.ace_apply(xi, x, g.dV)
    _close(y, ref, 1e-13, "V_ACE x")


# ------------------------------------------------------------------ c1 end to end

@pytest.fixture(scope="module")
def c1():
    o = make_orbitals(config_spec("c1"))
    s = o.spec
    piv, U, phi = oracle.scdm_localize(o.psi, s.dV)
    return o, piv, U, phi


def test_localize_c1(ctx, c1):
    _say("localize c1")
    o, piv, U, phi = c1
    s = o.spec
    gphi, gpiv, gU = ctx.localize(_dev(o.psi), _grid(s))
    np.testing.assert_array_equal(gpiv.cpu().numpy(), piv)
    np.testing.assert_allclose(gU.cpu().numpy(), U, atol=1e-12)
    np.testing.assert_allclose(gphi.cpu().numpy(), phi, atol=1e-12 * np.abs(phi).max())


@pytest.mark.parametrize("rho_cut", [0.0, 0.05, 0.2, 2.0])
def test_pairlist_c1(ctx, c1, rho_cut):
    _say(f"pairlist c1 rho_cut={rho_cut}")
    o, _, _, phi = c1
    s = o.spec
    ref, ov = oracle.pairlist(phi, s.dV, rho_cut)
    gp, gov = ctx.pairlist(_dev(phi), _grid(s), rho_cut)
    np.testing.assert_array_equal(gp.cpu().numpy(), ref)
    np.testing.assert_allclose(gov.cpu().numpy(), ov, atol=1e-14)


def test_pairlist_capacity_error(ctx, c1):
    from paper_2101_03155_amd import AceError
    o, _, _, phi = c1
    with pytest.raises(AceError) as ei:
        ctx.pairlist(_dev(phi), _grid(o.spec), 0.0, capacity=10)
    assert ei.value.status == "ACE_E_CAPACITY" and "required 36" in str(ei.value)


@pytest.mark.parametrize("which", ["psi", "phi"])
def test_build_c1_full_fp64(ctx, c1, which):
    _say(f"build c1 full fp64 from {which}")
    o, _, _, phi = c1
    s = o.spec
    orbs = o.psi if which == "psi" else phi
    pairs = _full_pairs(s.norb)
    ref = oracle.ace_build(orbs, pairs, s.N, s.L, "bare", 0.1)
    r = ctx.build(_dev(orbs), _dev(pairs), _grid(s), kernel="bare", precision="fp64", want_W=True,
                  want_energies=True)
    ex = float(r["ex"].item())
    assert abs(ex - ref["ex"]) <= 1e-12 * abs(ref["ex"])
    _close(r["W"].cpu().numpy(), ref["W"], 1e-12, "W")
    np.testing.assert_allclose(r["M"].cpu().numpy(), ref["M"], atol=1e-12 * np.abs(ref["M"]).max())
    _close(r["xi"].cpu().numpy(), ref["xi"], 1e-11, "xi")
    np.testing.assert_allclose(r["e"].cpu().numpy(), ref["e"], atol=1e-13 * np.abs(ref["e"]).max())


def test_ace_matrix_elements_c1(ctx, c1):
    _say("ACE matrix elements c1")
    o, _, _, phi = c1
    s = o.spec
    pairs = _full_pairs(s.norb)
    ref = oracle.ace_build(phi, pairs, s.N, s.L, "bare", 0.1)
    r = ctx.build(_dev(phi), _dev(pairs), _grid(s), kernel="bare", precision="fp64")
    vecs = np.concatenate([phi, smooth_test_vectors(s, 16)])
    y = ctx.apply(r["xi"], _dev(vecs), _grid(s)).cpu().numpy()
    yref = oracle.ace_apply(ref["xi"], vecs, s.dV)
    A = vecs.reshape(len(vecs), -1)
    mel = s.dV * A @ y.reshape(len(vecs), -1).T
    mref = s.dV * A @ yref.reshape(len(vecs), -1).T
    assert np.abs(mel - mref).max() <= 1e-10
    # V_ACE phi = W on the occupied space
    _close(y[: s.norb], ref["W"], 1e-11, "V_ACE phi vs W")


def test_split_path_matches_fused(ctx, c1):
    _say("split vs fused path c1")
    o, _, _, phi = c1
    s = o.spec
    pairs = _dev(_full_pairs(s.norb))
    a = ctx.build(_dev(phi), pairs, _grid(s), kernel="bare", want_W=True)
    ctx.set_pair_shape("fp64", s.N, False, 5)
    try:
        b = ctx.build(_dev(phi), pairs, _grid(s), kernel="bare", want_W=True)
    finally:
        ctx.set_pair_shape("fp64", s.N, True, 64)
    _close(b["W"].cpu().numpy(), a["W"].cpu().numpy(), 1e-13, "split vs fused W")
    assert abs(b["ex"].item() - a["ex"].item()) < 1e-13 * abs(a["ex"].item())


def test_release_workspace_then_rebuild(ctx, c1):
    _say("release workspaces, rebuild c1")
    o, _, _, phi = c1
    s = o.spec
    pairs = _dev(_full_pairs(s.norb))
    a = ctx.build(_dev(phi), pairs, _grid(s), kernel="bare")
    ctx.release_workspace()
    b = ctx.build(_dev(phi), pairs, _grid(s), kernel="bare")
    assert torch.equal(a["ex"], b["ex"]) and torch.equal(a["xi"], b["xi"])


def test_fp32_c1(ctx, c1):
    _say("build c1 fp32")
    o, _, _, phi = c1
    s = o.spec
    pairs = _full_pairs(s.norb)
    ref = oracle.ace_build(phi, pairs, s.N, s.L, "bare", 0.1)
    r = ctx.build(_dev(phi), _dev(pairs), _grid(s), kernel="bare", precision="fp32", want_W=True)
    assert abs(r["ex"].item() - ref["ex"]) <= 1e-6 * abs(ref["ex"])
    _close(r["W"].cpu().numpy(), ref["W"], 2e-5, "fp32 W")
    np.testing.assert_allclose(r["M"].cpu().numpy(), ref["M"], atol=1e-5)
    _close(r["xi"].cpu().numpy(), ref["xi"], 1e-4, "fp32 xi")


def test_not_positive_definite_reported(ctx, c1):
    _say("NOT_PD path")
    from paper_2101_03155_amd import AceError
    o, _, _, phi = c1
    s = o.spec
    # a single off-diagonal pair leaves W_k = 0 for every other orbital: -M is singular
    pairs = np.array([(0, 1)], dtype=np.int32)
    with pytest.raises(oracle.NotPositiveDefinite):
        oracle.ace_build(phi, pairs, s.N, s.L, "bare", 0.1)
    with pytest.raises(AceError) as ei:
        ctx.build(_dev(phi), _dev(pairs), _grid(s), kernel="bare")
    assert ei.value.status == "ACE_E_NOT_PD"


def test_bad_pairs_rejected(ctx, c1):
    from paper_2101_03155_amd import AceError
    o, _, _, phi = c1
    s = o.spec
    for bad in ([(0, 0), (0, 0)], [(3, 1)], [(0, s.norb)]):
        with pytest.raises(AceError) as ei:
            ctx.build(_dev(phi), _dev(np.array(bad, dtype=np.int32)), _grid(s))
        assert ei.value.status == "ACE_E_ARG"


# ------------------------------------------------------------------ other grid sizes, ragged lists

SIZE_CASES = [(8, "erfc", "fp64"), (12, "bare", "fp64"), (16, "erfc", "fp64"), (32, "erfc", "fp64"),
              (48, "bare", "fp64"), (16, "erfc", "fp32"), (48, "erfc", "fp32"),
              # the grids of the batched workload, the screener's training sets and the
              # 64- and 128-water systems
              (64, "erfc", "fp64"), (64, "bare", "fp32"), (80, "erfc", "fp64"), (80, "erfc", "fp32"),
              (100, "erfc", "fp64"), (100, "erfc", "fp32"), (108, "erfc", "fp64"), (108, "erfc", "fp32"),
              (120, "erfc", "fp64"), (120, "erfc", "fp32"), (160, "erfc", "fp64"), (160, "erfc", "fp32")]

_SIZE_REF = {}


def _size_case(n, kind):
    """Inputs and oracle build of one size case (shared by paths and precisions)."""
    if (n, kind) not in _SIZE_REF:
        L = n * 0.3 if n <= 48 else 14.4 + 0.05 * n
        spec = SystemSpec(n_mol=3 if n <= 48 else 2, L=L, N=n, sigma=0.7, offset=0.6, placement="uniform",
                          seed=40 + n, kernel=kind, omega=0.4)
        o = make_orbitals(spec)
        rng = np.random.default_rng(n)
        full = _full_pairs(spec.norb)
        keep = (full[:, 0] == full[:, 1]) | (rng.random(len(full)) < 0.55)
        pairs = full[keep]
        if len(pairs) % 2 == 0:
            pairs = pairs[:-1] if pairs[-1, 0] != pairs[-1, 1] else pairs
        v = oracle.coulomb_kernel(n, L, kind, 0.4)
        ref_W, ref_e = oracle.build_W(o.psi, pairs, v, spec.dV, energies=True, workers=8)
        try:
            ref_M, _, ref_xi, ref_ex, _ = oracle.ace_from_W(o.psi, ref_W, spec.dV)
        except oracle.NotPositiveDefinite:
            ref_M = ref_xi = ref_ex = None
        _SIZE_REF.clear()  # keep one case resident (160^3 arrays are large)
        _SIZE_REF[(n, kind)] = dict(spec=spec, psi=o.psi, pairs=pairs, W=ref_W, e=ref_e, M=ref_M, xi=ref_xi,
                                    ex=ref_ex)
    return _SIZE_REF[(n, kind)]


@pytest.mark.parametrize("path", ["fused", "r2c", "split", "owner"])
@pytest.mark.parametrize("n,kind,prec", SIZE_CASES)
def test_sizes_and_screened_lists(ctx, n, kind, prec, path):
    _say(f"sizes N={n} {kind} {prec} path={path}")
    c = _size_case(n, kind)
    spec, pairs = c["spec"], c["pairs"]
    from paper_2101_03155_amd import AceError
    saved = ctx.get_pair_shape(prec, n)
    ctx.set_pair_shape(prec, n, path, 3)
    ran = ctx.get_pair_shape(prec, n)[0]
    try:
        if ran != path:
            # the library runs the split passes where this path's plane does not fit in LDS
            assert ran == "split"
            pytest.skip(f"{path} does not fit at N={n} {prec}; the split path runs (tested on its own)")
        if c["ex"] is None:
            with pytest.raises(AceError) as ei:
                ctx.build(_dev(c["psi"]), _dev(pairs), _grid(spec), kernel=kind, omega=0.4, precision=prec)
            assert ei.value.status == "ACE_E_NOT_PD"
            return
        r = ctx.build(_dev(c["psi"]), _dev(pairs), _grid(spec), kernel=kind, omega=0.4, precision=prec,
                      want_W=True, want_energies=True)
    finally:
        ctx.set_pair_shape(prec, n, *saved)
    f64 = prec == "fp64"
    _close(r["W"].cpu().numpy(), c["W"], 1e-12 if f64 else 2e-5, "W")
    _close(r["e"].cpu().numpy(), c["e"], 1e-12 if f64 else 2e-5, "pair energies")
    np.testing.assert_allclose(r["M"].cpu().numpy(), c["M"], rtol=0,
                               atol=(1e-12 if f64 else 1e-6) * np.abs(c["M"]).max())
    assert abs(r["ex"].item() - c["ex"]) <= (1e-10 if f64 else 1e-6) * abs(c["ex"])
    _close(r["xi"].cpu().numpy(), c["xi"], 1e-10 if f64 else 1e-4, "xi")


# ------------------------------------------------------------------ c2 (128 orbitals, 96^3)

@pytest.fixture(scope="module")
def c2(ctx):
    o = make_orbitals(config_spec("c2"))
    s = o.spec
    piv, U, phi = oracle.scdm_localize(o.psi, s.dV)
    pairs, ov = oracle.pairlist(phi, s.dV, 1e-3)
    return dict(o=o, s=s, piv=piv, phi=phi, pairs=pairs, ov=ov,
                v=oracle.coulomb_kernel(s.N, s.L, "erfc", s.omega))


def test_c2_localize_and_pairlist(ctx, c2):
    _say("c2 localize + pairlist")
    s = c2["s"]
    gphi, gpiv, _ = ctx.localize(_dev(c2["o"].psi), _grid(s))
    np.testing.assert_array_equal(gpiv.cpu().numpy(), c2["piv"])
    phi = gphi.cpu().numpy()
    assert np.abs(phi - c2["phi"]).max() < 1e-10 * np.abs(c2["phi"]).max()
    gp, gov = ctx.pairlist(_dev(c2["phi"]), _grid(s), 1e-3)
    np.testing.assert_array_equal(gp.cpu().numpy(), c2["pairs"])
    np.testing.assert_allclose(gov.cpu().numpy(), c2["ov"], rtol=1e-12)


def _workers():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _c2_screened_ref(c2):
    """The oracle's whole screened build (every row of W, M, L, xi, e)."""
    if "ref" not in c2:
        s = c2["s"]
        _say(f"c2 oracle screened build, {len(c2['pairs'])} pairs on {_workers()} threads")
        c2["ref"] = oracle.ace_build(c2["phi"], c2["pairs"], s.N, s.L, "erfc", s.omega, workers=_workers())
    return c2["ref"]


@pytest.mark.parametrize("path", ["split", "fused", "r2c", "owner"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c2_screened_build(ctx, c2, prec, path):
    _say(f"c2 screened build {prec} path={path}")
    s, phi, pairs = c2["s"], c2["phi"], c2["pairs"]
    saved = ctx.get_pair_shape(prec, s.N)
    ctx.set_pair_shape(prec, s.N, path, 16)
    assert ctx.get_pair_shape(prec, s.N)[0] == path
    try:
        r = ctx.build(_dev(phi), _dev(pairs.astype(np.int32)), _grid(s), kernel="erfc", omega=s.omega,
                      precision=prec, want_W=True, want_energies=True)
    finally:
        ctx.set_pair_shape(prec, s.N, *saved)
    ref = _c2_screened_ref(c2)
    f64 = prec == "fp64"
    assert abs(r["ex"].item() - ref["ex"]) <= (1e-10 if f64 else 1e-6) * abs(ref["ex"])
    # pair energies: FP64 to 1e-12 Ha; FP32 to the FP32 path's 1e-6 relative bound, per pair
    # against the largest pair energy
    np.testing.assert_allclose(r["e"].cpu().numpy(), ref["e"], rtol=0,
                               atol=1e-12 if f64 else 1e-6 * np.abs(ref["e"]).max())
    # every element of W, M and xi against the oracle's build
    _close(r["W"].cpu().numpy(), ref["W"], 1e-12 if f64 else 2e-5, "W (all rows)")
    dM = np.abs(r["M"].cpu().numpy() - ref["M"]).max()
    print(f"  M: max |dM| {dM:.3e} Ha", flush=True)
    assert dM <= (1e-11 if f64 else 1e-5)
    _close(r["xi"].cpu().numpy(), ref["xi"], 1e-10 if f64 else 1e-4, "xi (all rows)")
    # ACE matrix elements <a|V_ACE|b> over {phi_i} and 16 smooth test vectors
    if "vecs" not in c2:
        c2["vecs"] = np.concatenate([phi, smooth_test_vectors(s, 16)])
        A = c2["vecs"].reshape(len(c2["vecs"]), -1)
        c2["mel_ref"] = s.dV * A @ oracle.ace_apply(ref["xi"], c2["vecs"], s.dV).reshape(len(A), -1).T
    vecs = c2["vecs"]
    y = ctx.apply(r["xi"], _dev(vecs), _grid(s)).cpu().numpy()
    mel = s.dV * vecs.reshape(len(vecs), -1) @ y.reshape(len(vecs), -1).T
    dmel = np.abs(mel - c2["mel_ref"]).max()
    print(f"  ACE matrix elements: max |d<a|V|b>| {dmel:.3e} Ha", flush=True)
    assert dmel <= (1e-10 if f64 else 1e-5)


def test_c2_full_pair_energy(ctx, c2):
    _say("c2 full pair list fp64")
    s, phi = c2["s"], c2["phi"]
    pairs = _full_pairs(s.norb)
    r = ctx.build(_dev(phi), _dev(pairs), _grid(s), kernel="erfc", omega=s.omega, want_energies=True)
    e_ref = oracle.exchange_energy_pairs(phi, pairs, c2["v"], s.dV)
    assert abs(r["ex"].item() - e_ref.sum()) <= 1e-10 * abs(e_ref.sum())
    np.testing.assert_allclose(r["e"].cpu().numpy(), e_ref, atol=1e-12)
    # screening identity on the GPU: E_x(screened) - E_x(full) = -sum of dropped e_ij
    kept = {tuple(p) for p in c2["pairs"]}
    dropped = sum(e for p, e in zip(map(tuple, pairs), e_ref) if p not in kept)
    rs = ctx.build(_dev(phi), _dev(c2["pairs"].astype(np.int32)), _grid(s), kernel="erfc", omega=s.omega)
    assert abs((rs["ex"].item() - r["ex"].item()) + dropped) < 1e-9 * abs(e_ref.sum())
    # ACE matrix elements <phi_k|V_ACE|phi_l> for a sampled l against the oracle's
    # <phi_k|V_X|phi_l> = dV <phi_k|W_l> (full list: V_ACE = V_X on the occupied space)
    rows = [0, 31, 127]
    Wref = oracle.build_W_rows(phi, pairs, rows, c2["v"], workers=_workers())
    mref = s.dV * phi.reshape(s.norb, -1) @ Wref.reshape(len(rows), -1).T
    y = ctx.apply(r["xi"], _dev(phi[rows]), _grid(s)).cpu().numpy()
    mel = s.dV * phi.reshape(s.norb, -1) @ y.reshape(len(rows), -1).T
    assert np.abs(mel - mref).max() <= 1e-10


# ------------------------------------------------------------------ failure paths, device-count screening

def test_failure_paths_nonfinite_input_and_workspace_cap(lib, c1):
    """A NaN in the orbitals reaches M and the factorization reports
    ACE_E_NONFINITE; a workspace cap below the build's needs gives
    ACE_E_NOMEM before any allocation; a context without the cap still builds."""
    _say("failure paths: NaN input, workspace cap")
    import os
    from paper_2101_03155_amd import AceError
    o, _, _, phi = c1
    s = o.spec
    pairs = _dev(_full_pairs(s.norb))
    ctx = lib.Context()
    bad = phi.copy()
    bad[3, 5, 5, 5] = np.nan
    with pytest.raises(AceError) as ei:
        ctx.build(_dev(bad), pairs, _grid(s), kernel="bare")
    assert ei.value.status == "ACE_E_NONFINITE"
    old = os.environ.get("ACE_WORKSPACE_MAX")
    os.environ["ACE_WORKSPACE_MAX"] = "4096"
    try:
        capped = lib.Context()
    finally:
        if old is None:
            del os.environ["ACE_WORKSPACE_MAX"]
        else:
            os.environ["ACE_WORKSPACE_MAX"] = old
    with pytest.raises(AceError) as ei:
        capped.build(_dev(phi), pairs, _grid(s), kernel="bare")
    assert ei.value.status == "ACE_E_NOMEM" and "ACE_WORKSPACE_MAX" in str(ei.value)
    r = ctx.build(_dev(phi), pairs, _grid(s), kernel="bare")
    assert np.isfinite(r["ex"].item())


@pytest.mark.parametrize("rho_cut", [0.0, 0.05, 2.0])
def test_pairlist_device_count(ctx, c1, rho_cut):
    _say(f"pairlist with the count on the device, rho_cut={rho_cut}")
    o, _, _, phi = c1
    s = o.spec
    ref, ov = oracle.pairlist(phi, s.dV, rho_cut)
    pairs, gov, n = ctx.pairlist_device(_dev(phi), _grid(s), rho_cut)
    k = int(n.item())
    assert k == len(ref)
    np.testing.assert_array_equal(pairs[:k].cpu().numpy(), ref)
    np.testing.assert_allclose(gov[:k].cpu().numpy(), ov, atol=1e-14)
    # a short capacity: the count is still the full one, only the first rows are written
    pairs, _, n = ctx.pairlist_device(_dev(phi), _grid(s), rho_cut, capacity=5)
    assert int(n.item()) == len(ref)
    np.testing.assert_array_equal(pairs[: min(5, len(ref))].cpu().numpy(), ref[:5])


def test_owner_order_switch_gives_identical_build(lib):
    """The owners' dispatch order (reverse Cuthill-McKee by default, index
    order with ACE_OWNER_ORDER=0 at context creation) changes only which
    workgroups run together: each owner still sums its entries in the same
    order, so W, M, xi and E_x are bitwise equal."""
    _say("owner order: default vs ACE_OWNER_ORDER=0 on the 32^3 size case")
    import os
    c = _size_case(32, "erfc")
    spec, pairs = c["spec"], c["pairs"]
    old = os.environ.get("ACE_OWNER_ORDER")
    os.environ["ACE_OWNER_ORDER"] = "0"
    try:
        plain = lib.Context()
    finally:
        if old is None:
            del os.environ["ACE_OWNER_ORDER"]
        else:
            os.environ["ACE_OWNER_ORDER"] = old
    ordered = lib.Context()
    out = []
    for cx in (ordered, plain):
        cx.set_pair_shape("fp64", 32, "owner", 3)
        assert cx.get_pair_shape("fp64", 32)[0] == "owner"
        out.append(cx.build(_dev(c["psi"]), _dev(pairs), _grid(spec), kernel="erfc", omega=0.4, want_W=True))
    for key in ("W", "M", "xi", "ex"):
        assert torch.equal(out[0][key], out[1][key]), key
    _close(out[0]["W"].cpu().numpy(), c["W"], 1e-12, "W")
