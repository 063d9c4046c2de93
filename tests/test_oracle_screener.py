"""Pins of the screener oracle: gradients by finite differences, Adam's first
step in closed form, features of Gaussians in closed form, the budget rule."""
import numpy as np

from oracle import screener_oracle as so
from synth import SystemSpec, disjoint_gaussians


def _rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(scale=scale, size=so.NPARAM)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _rand_params(2)
    xs = rng.normal(size=(17, so.NIN))
    ts = rng.normal(size=17)
    loss, g = so.loss_and_grad(p, xs, ts)
    idx = rng.choice(so.NPARAM, size=60, replace=False)
    idx = np.concatenate([idx, [so.NPARAM - 1, 0, so.NH * so.NIN + 3]])  # include b3, W1, b1 entries
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (so.loss_and_grad(pp, xs, ts)[0] - so.loss_and_grad(pm, xs, ts)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_forward_special_cases():
    p = np.zeros(so.NPARAM)
    p[-1] = 0.75  # b3 only: constant output
    out, _ = so.forward(p, np.random.default_rng(0).normal(size=(4, so.NIN)))
    np.testing.assert_array_equal(out, 0.75)
    # a single path through the network: out = w3_0 tanh(W2_00 tanh(W1_00 x0))
    W1, b1, W2, b2, w3, b3 = (np.zeros((so.NH, so.NIN)), np.zeros(so.NH), np.zeros((so.NH, so.NH)),
                              np.zeros(so.NH), np.zeros(so.NH), 0.0)
    W1[0, 0], W2[0, 0], w3[0] = 0.7, -1.3, 2.0
    x = np.array([[0.4, 9, 9, 9, 9]])
    out, _ = so.forward(so.pack(W1, b1, W2, b2, w3, b3), x)
    assert abs(out[0] - 2.0 * np.tanh(-1.3 * np.tanh(0.7 * 0.4))) < 1e-15


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -1e-3, 0.5])
    p1, m, v = so.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p1, -0.01 * np.sign(g), rtol=1e-8)


def test_features_of_gaussians_closed_form():
    spec = SystemSpec(n_mol=1, L=14.0, N=48, sigma=0.8, seed=0)
    a, b = np.array([3.0, 5.5, 12.9]), np.array([4.1, 4.0, 1.2])  # b is across the boundary in z
    g = disjoint_gaussians(spec, [a, b])
    cen, spr = so.centroids_spreads(g, spec.L)
    np.testing.assert_allclose(cen[0], a, atol=1e-10)
    np.testing.assert_allclose(cen[1], b, atol=1e-10)
    # |phi|^2 has variance sigma^2/2 per axis
    np.testing.assert_allclose(spr, np.sqrt(1.5) * spec.sigma, rtol=1e-9)
    d = a - b
    d -= spec.L * np.round(d / spec.L)
    dist = np.linalg.norm(d)
    s = spec.sigma
    # the overlap integrals in closed form, on the full grid and on the grid
    # subsampled by 2 per axis.  At stride 2 (spacing 0.58 bohr) the Riemann
    # sum of |phi_i||phi_j| (width sigma) is still exact to ~1e-8 in log10; the
    # one of phi_i^2 phi_j^2 (width sigma / 2 = 0.4 bohr) aliases at ~2e-4.  A
    # wrong weight or stride would be off by O(1).
    for stride, tol_o, tol_p in ((1, 1e-9, 1e-9), (2, 1e-7, 5e-4)):
        f = so.pair_features(g, spec.L, [(0, 1)], stride=stride)[0]
        assert abs(f[0] - dist) < 1e-10
        assert abs(f[3] - np.log10(np.exp(-dist ** 2 / (4 * s * s)))) < tol_o
        assert abs(f[4] - np.log10((2 * np.pi * s * s) ** -1.5 * np.exp(-dist ** 2 / (2 * s * s)))) < tol_p


def test_budget_rule():
    rng = np.random.default_rng(3)
    e = 10 ** rng.uniform(-9, -2, size=200)
    for budget in (1e-8, 1e-5, 1e-3, 1.0):
        keep = so.budget_selection(e, budget)
        dropped = e[~keep]
        assert dropped.sum() <= budget
        if keep.any():
            assert dropped.sum() + e[keep].min() > budget
            assert (dropped.max() if len(dropped) else 0) <= e[keep].min()
