"""Learned pair screener: training data, training, calibration, selection.

The screening criterion of Sec. Theory keeps a pair (i, j) when the overlap
integral of |phi_i phi_j| exceeds a fixed threshold.  The learned screener
predicts each pair's exchange contribution |e_ij| instead and drops the pairs
whose predicted contributions sum to less than an E_x error budget
(1e-5 Ha per molecule by default); the overlap rule is the fallback.

Everything numerical runs in libace (features, exact pair energies for the
training targets, MLP forward/backward/Adam, the budgeted selection); this
module only sequences the calls and keeps the bookkeeping:

* training set: for seeded synthetic systems of 32-64 molecules, every
  off-diagonal pair with overlap >= rho_near plus a seeded fraction of the
  farther pairs, with targets log10 |e_ij| from the method's own pair solves;
* training: Adam on minibatches, several epochs;
* calibration: on held-out systems, the ratio of the true to the predicted
  dropped energy at the budget gives a safety margin m, and selection then
  uses budget / (1 + m);
* checkpoint: weights, standardization, margin and provenance in one .npz.
"""
from __future__ import annotations

import json
import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

from . import ace

BUDGET_PER_MOLECULE = 1e-5  # Hartree


@dataclass
class TrainingSet:
    x: object  # torch float32 [n][5] on the GPU
    t: object  # torch float32 [n]: log10 |e_ij|
    n_configs: int
    seconds: float
    per_config: List[dict] = field(default_factory=list)
    stride: int = 1  # feature stride of x


def _system(ctx, spec, device="cuda"):
    import torch

    from synth import make_orbitals

    o = make_orbitals(spec, device=device)
    grid = ace.Grid.cubic(spec.N, spec.L)
    phi, _, _ = ctx.localize(o.psi, grid)
    del o
    torch.cuda.empty_cache()
    return phi, grid


FEATURE_STRIDE = 2  # the overlap features of new screeners use every second grid point per axis


def training_set(ctx, specs: Sequence, rho_near: float = 1e-5, far_fraction: float = 0.1, seed: int = 0,
                 precision: str = "fp32", stride: int = FEATURE_STRIDE, log=None) -> TrainingSet:
    """Features and exact pair energies of the seeded training systems."""
    import torch

    rng = np.random.default_rng(seed)
    xs, ts, info = [], [], []
    t0 = time.perf_counter()
    for k, spec in enumerate(specs):
        phi, grid = _system(ctx, spec)
        f = ctx.pair_features(phi, grid, stride=stride)  # every pair i <= j
        n = spec.norb
        iu, ju = np.triu_indices(n)
        logo = f[:, 3].cpu().numpy()
        off = iu != ju
        sel = off & ((logo >= np.log10(rho_near)) | (rng.random(len(iu)) < far_fraction))
        idx = np.flatnonzero(sel)
        pairs = torch.as_tensor(np.stack([iu[idx], ju[idx]], 1).astype(np.int32), device="cuda")
        e = ctx.pair_energies(phi, pairs, grid, kernel=spec.kernel, omega=spec.omega, precision=precision)
        # targets log10 |e_ij| (host bookkeeping of the library's pair energies)
        t = torch.as_tensor(np.log10(np.maximum(np.abs(e.cpu().numpy()), 1e-16)).astype(np.float32), device="cuda")
        xs.append(f[torch.as_tensor(idx, device="cuda")])
        ts.append(t)
        info.append({"seed": spec.seed, "n_mol": spec.n_mol, "N": spec.N, "pairs": int(len(idx))})
        if log:
            log(f"training config {k + 1}/{len(specs)}: {spec.n_mol} molecules, {spec.N}^3, {len(idx)} pairs")
        del phi, f, e
    x = torch.cat(xs).contiguous()
    t = torch.cat(ts).contiguous()
    return TrainingSet(x=x, t=t, n_configs=len(specs), seconds=time.perf_counter() - t0, per_config=info,
                       stride=stride)


class LearnedScreener:
    def __init__(self, model, margin: float = 0.0, meta: Optional[dict] = None):
        self.model = model  # torch float32 [ACE_MLP_NMODEL] on the GPU
        self.margin = float(margin)
        self.meta = dict(meta or {})

    # ---------------------------------------------------------------- training
    @classmethod
    def train(cls, ctx, data: TrainingSet, epochs: int = 30, batch: int = 4096, lr: float = 2e-3,
              seed: int = 0) -> "LearnedScreener":
        import torch

        model = ctx.mlp_init(seed)
        ctx.mlp_fit_norm(model, data.x, data.t)
        m = torch.zeros(ace.MLP_NPARAM, dtype=torch.float32, device="cuda")
        v = torch.zeros_like(m)
        nb = (data.x.shape[0] + batch - 1) // batch
        t0 = time.perf_counter()
        curve = []
        step = 0
        # two phases: lr, then lr/10
        for ep, rate in ((int(epochs * 0.7), lr), (epochs - int(epochs * 0.7), lr * 0.1)):
            if ep <= 0:
                continue
            c = ctx.mlp_train(model, m, v, data.x, data.t, lr=rate, batch=batch, epochs=ep, seed=seed + step,
                              step0=step)
            curve += (c.cpu().numpy() / nb).tolist()
            step += ep * nb
        torch.cuda.synchronize()
        meta = {"epochs": epochs, "batch": batch, "lr": lr, "train_samples": int(data.x.shape[0]),
                "train_configs": data.n_configs, "train_seconds": time.perf_counter() - t0,
                "data_seconds": data.seconds, "feature_stride": data.stride, "loss_curve": curve}
        return cls(model, 0.0, meta)

    @property
    def stride(self) -> int:
        return int(self.meta.get("feature_stride", 1))

    def predict(self, ctx, x):
        return ctx.mlp_forward(self.model, x)

    # ---------------------------------------------------------------- selection
    def select(self, ctx, phi, grid, n_mol: int, budget_per_molecule: float = BUDGET_PER_MOLECULE,
               rho_cut_fallback: float = 1e-3, ood_tol: float = 0.05):
        """Pair list under the budget (margin applied); returns (pairs, used_fallback)."""
        budget = budget_per_molecule * n_mol / (1.0 + self.margin)
        return ctx.screen_learned(phi, grid, self.model, budget, rho_cut_fallback, ood_tol, stride=self.stride)

    def calibrate(self, ctx, specs: Sequence, budget_per_molecule: float = BUDGET_PER_MOLECULE,
                  safety: float = 0.25, precision: str = "fp64", log=None) -> dict:
        """Margin from held-out systems: true vs predicted dropped |e| at the budget."""
        import torch

        ratios = []
        for spec in specs:
            phi, grid = _system(ctx, spec)
            n = spec.norb
            budget = budget_per_molecule * spec.n_mol
            pairs, fb = ctx.screen_learned(phi, grid, self.model, budget, 1e-3, 1e9, stride=self.stride)
            kept = {tuple(p) for p in pairs.cpu().numpy().tolist()}
            iu, ju = np.triu_indices(n)
            drop = np.array([(i, j) for i, j in zip(iu, ju) if i != j and (i, j) not in kept], dtype=np.int32)
            if len(drop) == 0:
                continue
            dpairs = torch.as_tensor(drop, device="cuda")
            e = ctx.pair_energies(phi, dpairs, grid, kernel=spec.kernel, omega=spec.omega, precision=precision)
            f = ctx.pair_features(phi, grid, dpairs, stride=self.stride)
            pred = float(np.sum(10.0 ** ctx.mlp_forward(self.model, f, clamp=True).cpu().numpy().astype(np.float64)))
            true = float(np.sum(np.abs(e.cpu().numpy())))
            ratios.append(true / max(pred, 1e-300))
            if log:
                log(f"calibration {spec.n_mol} molecules: dropped true {true:.3e} Ha, predicted {pred:.3e} Ha")
            del phi
        m = max(0.0, max(ratios) - 1.0) * (1.0 + safety) if ratios else 0.0
        self.margin = m
        self.meta["calibration_ratios"] = ratios
        self.meta["margin"] = m
        return {"ratios": ratios, "margin": m}

    # ---------------------------------------------------------------- checkpoint
    def save(self, path: str):
        np.savez(path, model=self.model.cpu().numpy(), margin=np.float64(self.margin),
                 meta=np.array(json.dumps(self.meta)))

    @classmethod
    def load(cls, path: str) -> "LearnedScreener":
        import torch

        z = np.load(path, allow_pickle=False)
        model = torch.as_tensor(z["model"], device="cuda")
        return cls(model, float(z["margin"]), json.loads(str(z["meta"])))


def main(argv=None):
    """Train, calibrate and save a screener: python -m paper_2101_03155_amd.screener OUT.npz"""
    import argparse

    from synth import batched_like_specs, training_specs

    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--configs", type=int, default=200)
    ap.add_argument("--validation", type=int, default=8)
    ap.add_argument("--validation-batched", type=int, default=8,
                    help="held-out systems drawn like the batched workload (8-64 molecules, coarser grids)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--kernel", default="erfc", choices=["erfc", "bare"])
    args = ap.parse_args(argv)
    ctx = ace.Context()
    log = lambda m: print(m, flush=True)  # noqa: E731
    data = training_set(ctx, training_specs(args.configs, kernel=args.kernel), log=log)
    scr = LearnedScreener.train(ctx, data, epochs=args.epochs)
    held = (training_specs(args.validation, first_seed=7000, kernel=args.kernel)
            + batched_like_specs(args.validation_batched, first_seed=7100, kernel=args.kernel))
    scr.calibrate(ctx, held, log=log)
    scr.meta["kernel"] = args.kernel
    scr.meta["calibration_systems"] = [{"seed": s.seed, "n_mol": s.n_mol, "N": s.N} for s in held]
    scr.save(args.out)
    log(json.dumps({k: v for k, v in scr.meta.items() if k != "loss_curve"}))


if __name__ == "__main__":
    main()
