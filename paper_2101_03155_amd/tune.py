"""Autotuner for the pair-stage launch shape.

For one (precision, grid size) it times the pair stage of real builds with the
library's own HIP events for every candidate shape (fused in-plane path or
split x/y passes; packs per launch) and keeps the fastest in the context.
Results can be cached in a JSON file keyed by device name, precision, grid
size and orbital count.
"""
from __future__ import annotations

import json
import os
from typing import Iterable, Optional, Sequence, Tuple

from . import ace

DEFAULT_PACKS = (16, 32, 64, 128)


def candidates(precision: str, n: int, packs: Sequence[int] = DEFAULT_PACKS) -> Iterable[Tuple[str, int]]:
    for path in ("owner", "r2c", "fused", "split"):
        for mp in packs:
            yield path, mp


def _key(precision, n, norb):
    import torch

    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{dev}|{precision}|{n}|{norb}"


def autotune(ctx: "ace.Context", phi, pairs, grid: "ace.Grid", kernel: str, omega: float, precision: str,
             packs: Sequence[int] = DEFAULT_PACKS, reps: int = 2, cache: Optional[str] = None):
    """Pick the fastest pair-stage shape; returns dict(fused=path name, max_packs, ms, table)."""
    import torch

    n = int(grid.n[0])
    norb = int(phi.shape[0])
    cache = cache or os.environ.get("ACE_TUNE_CACHE")
    key = _key(precision, n, norb)
    if cache and os.path.exists(cache):
        try:
            hit = json.load(open(cache)).get(key)
        except (OSError, ValueError):
            hit = None
        if hit:
            ctx.set_pair_shape(precision, n, hit["fused"], hit["max_packs"])
            return dict(hit, cached=True)
    table = []
    seen = set()
    for fused, mp in candidates(precision, n, packs):
        try:
            ctx.set_pair_shape(precision, n, fused, mp)
        except ace.AceError:
            continue
        f_eff, mp_eff = ctx.get_pair_shape(precision, n)
        if (f_eff, mp_eff) in seen:
            continue
        seen.add((f_eff, mp_eff))
        ctx.build(phi, pairs, grid, kernel=kernel, omega=omega, precision=precision, want_M=False)
        ctx.profile(True)
        ctx.profile_read(ace.ST_PAIRS, reset=True)
        for _ in range(reps):
            ctx.build(phi, pairs, grid, kernel=kernel, omega=omega, precision=precision, want_M=False)
        torch.cuda.synchronize()
        _, ms, _ = ctx.profile_read(ace.ST_PAIRS, reset=True)
        ctx.profile(False)
        table.append({"fused": f_eff, "max_packs": mp_eff, "ms": ms / reps})
    best = min(table, key=lambda r: r["ms"])
    ctx.set_pair_shape(precision, n, best["fused"], best["max_packs"])
    out = dict(best, table=table, cached=False)
    if cache:
        try:
            data = json.load(open(cache)) if os.path.exists(cache) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = {"fused": best["fused"], "max_packs": best["max_packs"], "ms": best["ms"]}
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return out


def autotune_batched(ctx: "ace.Context", systems, precision: str = "fp32", reps: int = 2,
                     modes=("graph", "persistent"), layouts=("owner", "r2c", "split"), txvs=(8, 16), plans=(0, 1),
                     bpcs=(2, 4, 8)):
    """Pick the batched launch form and shape (mode, layout, x-tile, radix
    order, workgroups per CU) by timing whole batched builds; returns
    dict(best, table)."""
    import time

    import torch

    table = []
    for mode in modes:
        for layout in layouts:
            for txv in txvs:
                if layout != "split" and txv != txvs[-1]:
                    continue  # the x-tile only shapes the split layout
                if layout == "owner" and mode == "persistent":
                    continue  # the persistent launch keeps the rounds
                for plan in plans:
                    for bpc in bpcs:
                        if mode == "graph" and bpc != bpcs[-1]:
                            continue  # the per-phase launches size their own grids
                        row = {"mode": mode, "layout": layout, "txv": txv, "plan": plan, "bpc": bpc}
                        ctx.set_batched_shape(txv, plan, bpc, layout)
                        try:
                            ctx.build_batched(systems, precision=precision, mode=mode, want_M=False)
                        except ace.AceError as e:
                            table.append(dict(row, error=str(e)))
                            continue
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        for _ in range(reps):
                            ctx.build_batched(systems, precision=precision, mode=mode, want_M=False)
                        torch.cuda.synchronize()
                        table.append(dict(row, ms=(time.perf_counter() - t0) * 1000.0 / reps))
    ok = [r for r in table if "ms" in r]
    best = min(ok, key=lambda r: r["ms"])
    ctx.set_batched_shape(best["txv"], best["plan"], best["bpc"], best["layout"])
    return {"best": best, "table": table}

