"""FP64 reference for the learned pair screener.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The screener replaces the fixed overlap threshold of the screening criterion
(Sec. Theory) by a prediction of each pair's exchange contribution
e_ij = -(2 - d_ij)(ij|ij).  Its features, model and loss are defined here
plainly:

features of a pair (i, j):
  0  minimum-image distance between the periodic centroids of |phi_i|^2, |phi_j|^2
  1  smaller of the two spreads  (s^2 = dV sum_r |phi|^2 |r - c|^2, minimum image)
  2  larger of the two spreads
  3  log10 of O_ij = dV sum_r |phi_i||phi_j|      (the screening integral)
  4  log10 of P_ij = dV sum_r phi_i^2 phi_j^2     (pair-density L2 overlap)
  (logs of max(., 1e-30); O and P optionally on the grid subsampled by a
  stride s per axis, weight dV s^3)

model: x -> standardize -> tanh(W1 x + b1) -> tanh(W2 h + b2) -> w3 . h + b3,
       prediction = tmean + tstd * output, target = log10 |e_ij|;
loss:  mean over the batch of (output - (t - tmean)/tstd)^2.

Parameter layout (flat FP32 vector in the library): W1[64][5], b1[64],
W2[64][64], b2[64], w3[64], b3.  Pinned by central finite differences of the
loss (tests/test_oracle_screener.py).
"""
from __future__ import annotations

import numpy as np

NIN, NH = 5, 64
NPARAM = NH * NIN + NH + NH * NH + NH + NH + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + NH * NIN].reshape(NH, NIN); o += NH * NIN
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    w3 = p[o:o + NH]; o += NH
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]])


def standardize(x, xmean, xstd):
    return (np.asarray(x, dtype=np.float64) - xmean) / xstd


def forward(p, xs):
    """Network output on standardized inputs xs [n][5]; returns (out, cache)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    a1 = xs @ W1.T + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2.T + b2
    h2 = np.tanh(a2)
    out = h2 @ w3 + b3
    return out, (xs, h1, h2)


def loss_and_grad(p, xs, ts):
    """Mean squared error on standardized targets ts and its gradient in p."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    out, (x, h1, h2) = forward(p, xs)
    n = len(ts)
    r = out - ts
    loss = float(np.mean(r * r))
    dout = 2.0 * r / n
    gw3 = h2.T @ dout
    gb3 = dout.sum()
    dh2 = np.outer(dout, w3) * (1.0 - h2 * h2)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ W2) * (1.0 - h1 * h1)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ features

def centroids_spreads(phi, L):
    """Periodic centroid (per axis: argument of sum |phi|^2 exp(2 pi i x / L)) and
    spread^2 = dV sum |phi|^2 |r - c|^2 with minimum-image displacements."""
    n = phi.shape[0]
    N = phi.shape[1]
    L = float(L)
    dV = (L / N) ** 3
    x = np.arange(N) * L / N
    cen = np.zeros((n, 3))
    spr = np.zeros(n)
    for k in range(n):
        rho = phi[k] ** 2
        # marginal densities along z, y, x (axes 0, 1, 2)
        mz, my, mx = rho.sum((1, 2)), rho.sum((0, 2)), rho.sum((0, 1))
        for ax, m in ((2, mz), (1, my), (0, mx)):
            ang = np.angle(np.sum(m * np.exp(2j * np.pi * x / L)))
            cen[k, ax] = np.mod(ang * L / (2 * np.pi), L)
        s2 = 0.0
        for ax, m in ((2, mz), (1, my), (0, mx)):
            d = x - cen[k, ax]
            d = d - L * np.round(d / L)
            s2 += np.sum(m * d * d)
        spr[k] = np.sqrt(s2 * dV)
    return cen, spr


def pair_features(phi, L, pairs, stride=1):
    """The five features of every listed pair (float64).  With stride s > 1
    the two overlap integrals O and P are Riemann sums over the grid points
    whose three indices are multiples of s (weight dV s^3); centroids and
    spreads always use the full grid."""
    n = phi.shape[0]
    N = phi.shape[1]
    dV = (float(L) / N) ** 3
    cen, spr = centroids_spreads(phi, L)
    A = phi[:, ::stride, ::stride, ::stride].reshape(n, -1)
    dVs = dV * stride ** 3
    O = dVs * np.abs(A) @ np.abs(A).T
    P = dVs * (A * A) @ (A * A).T
    pairs = np.asarray(pairs)
    i, j = pairs[:, 0], pairs[:, 1]
    d = cen[i] - cen[j]
    d = d - L * np.round(d / L)
    out = np.empty((len(pairs), NIN))
    out[:, 0] = np.sqrt((d * d).sum(1))
    out[:, 1] = np.minimum(spr[i], spr[j])
    out[:, 2] = np.maximum(spr[i], spr[j])
    out[:, 3] = np.log10(np.maximum(O[i, j], 1e-30))
    out[:, 4] = np.log10(np.maximum(P[i, j], 1e-30))
    return out


def budget_selection(pred_abs_e, budget):
    """Drop pairs in ascending order of predicted |e| while the dropped sum
    stays within the budget; returns the boolean keep mask."""
    order = np.argsort(pred_abs_e, kind="stable")
    cum = np.cumsum(pred_abs_e[order])
    ndrop = int(np.searchsorted(cum, budget, side="right"))
    keep = np.ones(len(pred_abs_e), bool)
    keep[order[:ndrop]] = False
    return keep
