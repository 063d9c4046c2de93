#!/usr/bin/env python3
"""Benchmark of the screened ACE build on one MI355X.

Workload (32-water scale): 128 orbitals on a 96^3 grid, L = 18.6 bohr,
erfc-screened kernel (omega = 0.106), seeded synthetic orbitals.  One step is
the whole hot path from canonical orbitals: SCDM localization, pair screening
at rho_cut = 1e-3, pair Poisson solves + W, M = Phi^T W, Cholesky(-M) and the
projectors xi = L^-1 W.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  value = ACE builds/s (whole step).  Extra fields carry
the pair Poisson solves/s of the pair stage, the E_x errors, the other forms
(full pair list, FP32) and the roofline of the dominant kernel measured with
HIP events inside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = "ACE builds/s and pair Poisson solves/s (128 orb, 96^3), E_x rel. err vs FP64"

CLASS_NAMES = {0: "pair_fwd_xy", 1: "pair_conv_z", 2: "pair_inv_xy_accumulate", 3: "pair_fwd_x",
               4: "pair_fwd_y", 5: "pair_inv_y", 6: "pair_inv_x_accumulate", 7: "gemm_nt_splitk",
               8: "gemm_left_small", 9: "qrcp_update"}
CLASS_KERNEL = {0: "k_fwd_xy", 1: "k_conv_z", 2: "k_inv_xy", 3: "k_fwd_x", 4: "k_line_y", 5: "k_line_y",
                6: "k_inv_x", 7: "k_gemm_nt", 8: "k_gemm_ls", 9: "k_qrcp_update"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--rho-cut", type=float, default=1e-3)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--screener", default=os.path.join(ROOT, "paper_2101_03155_amd", "models",
                                                       "screener_water_erfc.npz"))
    ap.add_argument("--screener-bare", default=os.path.join(ROOT, "paper_2101_03155_amd", "models",
                                                             "screener_water_bare.npz"),
                    help="screener trained on bare-Coulomb pair energies (the batched form mixes kernels)")
    ap.add_argument("--skip-forms", default="", help="comma list of precision,batched,kpoints,learned,learned_batched")
    ap.add_argument("--shape", default="owner", choices=["auto", "default", "fused", "split", "r2c", "owner"],
                    help="pair-stage launch shape: autotuned, library default, or forced (default: owner, the "
                         "fastest measured for this workload, fixed so that profiles and the bench line agree)")
    ap.add_argument("--max-packs", type=int, default=32, help="packs per pair-stage launch for a forced shape")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB three times (calibrates FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


# Files whose code defines the pair-stage kernels; counters are voided when they change.
PAIR_SOURCES = ("paper_2101_03155_amd/csrc/pair.hip", "paper_2101_03155_amd/csrc/pair_phases.h",
                "paper_2101_03155_amd/csrc/fft.h")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_pair_stage.md")


def pair_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_row(kernel, N, prec):
    """The committed counter summary's row for a kernel at this size and
    precision: HBM bytes (read bytes from the per-size read-request counters,
    WRITE_SIZE for the writes, both checked on a plain 1 GiB copy) per
    algorithmic byte.  (None, why) when no row matches or the pair-stage
    sources changed since."""
    import re

    if not os.path.exists(COUNTERS_FILE):
        return None, "no counter summary"
    m = re.search(r"```json\n(.*?)\n```", open(COUNTERS_FILE).read(), re.S)
    if not m:
        return None, "no counter summary"
    for r in json.loads(m.group(1)):
        if r["kernel"] == kernel and r["N"] == N and r["precision"] == prec:
            if r["source_hash"] != pair_source_hash():
                return None, "pair-stage sources changed since the counters were taken"
            return r, ("reads 128 n128 + 64 n64 + 32 n32 from the request-size counters, writes WRITE_SIZE; "
                       "counters of the %s workload" % r.get("workload", "?"))
    return None, "no counter row for this kernel"


def measured_traffic(kernel, N, prec, units_per_launch):
    """HBM bytes per launch from the counter summary, applied to this launch size."""
    r, note = counter_row(kernel, N, prec)
    if r is None:
        return None, note
    return r["traffic_per_algorithmic_byte"] * units_per_launch, note


def copy_probe():
    import torch

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel() * 8, "copies": 3, "source_hash": pair_source_hash()}), flush=True)


def host_workers():
    """Host threads the oracle may use: the cores this process may run on,
    capped by OMP_NUM_THREADS when the environment sets it."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(o, kind, omega, rho_cut):
    """The FP64 oracle on the host cores, the whole step of the bench: SCDM,
    pair screening, every kept pair solve, M, Cholesky and the projectors.
    Returns the baseline record and the oracle's results (for parity)."""
    from threadpoolctl import threadpool_limits

    import oracle

    s = o.spec
    workers = host_workers()
    with threadpool_limits(limits=workers):
        t0 = time.perf_counter()
        piv, _, phi = oracle.scdm_localize(o.psi, s.dV)
        t1 = time.perf_counter()
        pairs, _ = oracle.pairlist(phi, s.dV, rho_cut)
        t2 = time.perf_counter()
        v = oracle.coulomb_kernel(s.N, s.L, kind, omega)
        W, e = oracle.build_W(phi, pairs, v, s.dV, energies=True, workers=workers)
        t3 = time.perf_counter()
        M, _, xi, ex, _ = oracle.ace_from_W(phi, W, s.dV)
        t4 = time.perf_counter()
    rec = {
        "value": 1.0 / (t4 - t0), "unit": "builds/s", "cores": workers, "kind": "oracle",
        "sample": (f"one whole step (not a sample): SCDM of {s.norb} orbitals on {s.N}^3, screening at "
                   f"rho_cut={rho_cut}, all {len(pairs)} kept pair solves on {workers} threads, M, Cholesky and xi"),
        "seconds": round(t4 - t0, 2),
        "stage_s": {"localize": round(t1 - t0, 3), "pairlist": round(t2 - t1, 3), "pair_stage": round(t3 - t2, 3),
                    "tail": round(t4 - t3, 3)},
        "pair_solves_per_s": round(len(pairs) / (t3 - t2), 2),
    }
    return rec, dict(piv=piv, phi=phi, pairs=pairs, W=W, e=e, M=M, xi=xi, ex=ex)


def parity_vs_oracle(ctx, grid, kind, omega, prec, gpu_piv, gpu_pairs, ref):
    """The bench step's outputs against the oracle's whole step: pivots and
    pair list exactly, then a build on the oracle's orbitals element by element."""
    import numpy as np
    import torch

    out = {"pivots_equal": bool(np.array_equal(gpu_piv, ref["piv"])),
           "pairs_equal": bool(np.array_equal(gpu_pairs, ref["pairs"]))}
    phi = torch.as_tensor(ref["phi"], device="cuda")
    pairs = torch.as_tensor(ref["pairs"].astype(np.int32), device="cuda")
    r = ctx.build(phi, pairs, grid, kernel=kind, omega=omega, precision=prec, want_M=True, want_W=True)
    W = r["W"].cpu().numpy()
    out["ex_rel_err"] = abs(float(r["ex"].item()) - ref["ex"]) / abs(ref["ex"])
    out["W_max_elem_err_rel"] = float(np.abs(W - ref["W"]).max() / np.abs(ref["W"]).max())
    out["M_max_abs_err_ha"] = float(np.abs(r["M"].cpu().numpy() - ref["M"]).max())
    xi = r["xi"].cpu().numpy()
    out["xi_max_elem_err_rel"] = float(np.abs(xi - ref["xi"]).max() / np.abs(ref["xi"]).max())
    return out


def _timed(fn, reps=3, warm=True):
    import torch

    if warm:
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / reps, out


def form_apply_energy(ctx, xi, x, grid, reps=10):
    """Per-SCF-cycle application: V_ACE on every orbital fused with the energy.

    Two FP64 products over the grid (c = dV xi x^T, y = -c^T xi): 4 norb nvec
    N_G flops, (2 norb + 2 nvec) N_G 8 bytes of HBM traffic at the least."""
    import torch

    ctx.apply_energy(xi, x, grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y, e = ctx.apply_energy(xi, x, grid)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / reps
    norb, nvec, ng = xi.shape[0], x.shape[0], grid.size
    tf = 4.0 * norb * nvec * ng / (ms / 1000.0) / 1e12
    gbs = (2 * norb + 2 * nvec) * ng * 8 / (ms / 1000.0) / 1e9
    return {"workload": f"V_ACE and E on all {nvec} orbitals, {norb} projectors, {round(ng ** (1 / 3))}^3",
            "ms": round(ms, 3), "tflops": round(tf, 2), "bound": "mfma",
            "frac_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 4), "min_traffic_gbs": round(gbs, 1),
            "e_hartree": float(e.item())}


def form_exact_exchange(ctx, psi, grid, kind, omega, reps=3):
    """Exact exchange on the canonical orbitals over every pair (W, M, E_x)."""
    import torch

    out = {"workload": f"canonical orbitals, all pairs, {psi.shape[0]} orbitals, {round(grid.size ** (1 / 3))}^3",
           "pairs": psi.shape[0] * (psi.shape[0] + 1) // 2}
    for p in ("fp64", "fp32"):
        r = ctx.exact_exchange(psi, grid, kernel=kind, omega=omega, precision=p, want_M=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ctx.exact_exchange(psi, grid, kernel=kind, omega=omega, precision=p, want_M=False,
                                   out={"W": r["W"]})
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / reps
        out[p] = {"ms": round(ms, 3), "pair_solves_per_s": round(out["pairs"] / (ms / 1000.0), 1),
                  "ex": float(r["ex"].item())}
        del r
        torch.cuda.empty_cache()
    out["ex_rel_err_fp32_vs_fp64"] = abs(out["fp32"]["ex"] - out["fp64"]["ex"]) / abs(out["fp64"]["ex"])
    return out


def form_incremental(ctx, psi0, spec, grid, kind, omega, rho_cut, cond_max=2.0, reps=5):
    """MD steps 1-3 (every centre moved 0.05 bohr per step): the previous
    step's columns kept while their quality ratio stays below cond_max
    (Loewdin only) and the re-screen against the previous list, against a
    fresh SCDM and screening at the same step; then the builds."""
    import dataclasses

    import torch

    from synth import make_orbitals

    phi, piv, _ = ctx.localize(psi0, grid)
    pairs, _ = ctx.pairlist(phi, grid, rho_cut)
    out = {"workload": f"MD steps 1-3 of {spec.norb} orbitals, {spec.N}^3, centres moved {spec.md_disp} bohr "
                       f"per step, columns kept while (max R_kk / min R_kk)^2 <= {cond_max}", "steps": []}
    for t in (1, 2, 3):
        psi = make_orbitals(dataclasses.replace(spec, md_step=t), device="cuda").psi
        ms_f, (phi_f, _, _) = _timed(lambda: ctx.localize(psi, grid), reps)
        ms_fp, (pairs_f, _) = _timed(lambda: ctx.pairlist(phi_f, grid, rho_cut), reps)
        ms_k, (phi_k, piv_k, _, info) = _timed(lambda: ctx.localize_step(psi, piv, grid, cond_max), reps)
        ms_kp, (pairs_k, _, pinfo) = _timed(lambda: ctx.pairlist_step(phi_k, grid, rho_cut, pairs), reps)
        rf = ctx.build(phi_f, pairs_f, grid, kernel=kind, omega=omega, want_M=False)
        rk = ctx.build(phi_k, pairs_k, grid, kernel=kind, omega=omega, want_M=False)
        ef, ek = float(rf["ex"].item()), float(rk["ex"].item())
        out["steps"].append({"step": t, "reused_columns": info["reused_columns"], "quality": round(info["gram_cond"], 4),
                             "pairs": int(pairs_k.shape[0]), "pairs_added": pinfo["pairs_added"],
                             "pairs_removed": pinfo["pairs_removed"], "pairs_fresh": int(pairs_f.shape[0]),
                             "localize_ms_kept": round(ms_k, 3), "localize_ms_fresh": round(ms_f, 3),
                             "pairlist_ms_step": round(ms_kp, 3), "pairlist_ms_fresh": round(ms_fp, 3),
                             "ex_rel_diff_kept_vs_fresh": abs(ek - ef) / abs(ef)})
        piv, pairs = piv_k, pairs_k
        del psi, phi_f, phi_k, rf, rk
    st = out["steps"]
    out["localize_speedup"] = round(sum(s["localize_ms_fresh"] for s in st) / sum(s["localize_ms_kept"] for s in st), 2)
    torch.cuda.empty_cache()
    return out


def form_precision(ctx, log, with_oracle=True):
    """64 waters (256 orbitals, 120^3): FP32 pair stage vs the plain FP64 path,
    and both against the FP64 oracle's build of the screened list: E_x, every
    element of W and M, and the ACE matrix elements over the orbitals and 16
    smooth test vectors."""
    import numpy as np
    import torch

    from paper_2101_03155_amd import Grid
    from synth import config_spec, make_orbitals, smooth_test_vectors

    spec = config_spec("c3")
    o = make_orbitals(spec, device="cuda")
    g = Grid.cubic(spec.N, spec.L)
    phi, _, _ = ctx.localize(o.psi, g)
    del o
    torch.cuda.empty_cache()
    pairs, _ = ctx.pairlist(phi, g, 1e-3)
    n = spec.norb
    full = torch.tensor([(i, j) for i in range(n) for j in range(i, n)], dtype=torch.int32, device="cuda")
    out = {"workload": "64 waters: 256 orbitals, 120^3, L=23.4, erfc omega=0.106", "pairs_screened": int(pairs.shape[0]),
           "pairs_full": int(full.shape[0])}
    for name, pl in (("screened", pairs), ("full", full)):
        reps = 3 if name == "screened" else 1
        ms64, r64 = _timed(lambda: ctx.build(phi, pl, g, kernel="erfc", omega=spec.omega, precision="fp64",
                                             want_M=False), reps)
        ms32, r32 = _timed(lambda: ctx.build(phi, pl, g, kernel="erfc", omega=spec.omega, precision="fp32",
                                             want_M=False), reps)
        e64, e32 = r64["ex"].item(), r32["ex"].item()
        out[name] = {"fp64_ms": round(ms64, 2), "fp32_ms": round(ms32, 2), "speedup_fp32": round(ms64 / ms32, 3),
                     "fp64_pair_solves_per_s": round(pl.shape[0] / ms64 * 1000, 1),
                     "fp32_pair_solves_per_s": round(pl.shape[0] / ms32 * 1000, 1),
                     "ex_fp64": e64, "ex_rel_err_fp32_vs_fp64": abs(e32 - e64) / abs(e64)}
        log(f"precision form {name}: {out[name]}")
        del r64, r32
    del full
    torch.cuda.empty_cache()
    if with_oracle:
        import oracle

        t0 = time.perf_counter()
        phi_np = phi.cpu().numpy()
        pairs_np = pairs.cpu().numpy().astype(np.int64)
        ref = oracle.ace_build(phi_np, pairs_np, spec.N, spec.L, "erfc", spec.omega, workers=host_workers())
        vecs = np.concatenate([phi_np, smooth_test_vectors(spec, 16)])
        A = vecs.reshape(len(vecs), -1)
        mel_ref = spec.dV * A @ oracle.ace_apply(ref["xi"], vecs, spec.dV).reshape(len(A), -1).T
        vd = torch.as_tensor(vecs, device="cuda")
        err = {"reference": (f"FP64 oracle build of the screened list ({len(pairs_np)} pairs) on the same orbitals, "
                             f"{host_workers()} host threads, {time.perf_counter() - t0:.1f} s"),
               "ace_matrix_elements": "<a|V_ACE|b> over the 256 orbitals and 16 smooth test vectors"}
        for p in ("fp64", "fp32"):
            r = ctx.build(phi, pairs, g, kernel="erfc", omega=spec.omega, precision=p, want_M=True, want_W=True)
            W = r["W"].cpu().numpy()
            w_err = float(np.abs(W - ref["W"]).max() / np.abs(ref["W"]).max())
            w_fro = float(np.linalg.norm(W - ref["W"]) / np.linalg.norm(ref["W"]))
            del W
            y = ctx.apply(r["xi"], vd, g)
            mel = (vd.reshape(len(A), -1) @ y.reshape(len(A), -1).T).cpu().numpy() * spec.dV
            err[p] = {"ex_rel_err": abs(r["ex"].item() - ref["ex"]) / abs(ref["ex"]),
                      "M_max_abs_err_ha": float(np.abs(r["M"].cpu().numpy() - ref["M"]).max()),
                      "ace_matrix_elements_max_abs_err_ha": float(np.abs(mel - mel_ref).max()),
                      "W_max_elem_err_rel": w_err, "W_frobenius_rel_err": w_fro}
            del r, y
            torch.cuda.empty_cache()
        out["vs_oracle_fp64"] = err
        log(f"precision form vs oracle: {err}")
    return out


def form_batched(ctx, log):
    """16 uneven systems (8-64 molecules, 48^3-96^3), FP32 pair stage, one batched call."""
    import torch

    from paper_2101_03155_amd import Grid
    from paper_2101_03155_amd.tune import autotune_batched
    from synth import batched_specs, make_orbitals

    specs = batched_specs()
    systems = []
    for sp in specs:
        o = make_orbitals(sp, device="cuda")
        g = Grid.cubic(sp.N, sp.L)
        phi, _, _ = ctx.localize(o.psi, g)
        del o
        pairs, _ = ctx.pairlist(phi, g, 1e-3)
        n = phi.shape[0]
        systems.append(dict(phi=phi, pairs=pairs, grid=g, kernel=sp.kernel, omega=sp.omega,
                            xi=torch.empty_like(phi), M=torch.empty(n, n, dtype=torch.float64, device="cuda"),
                            ex=torch.empty(1, dtype=torch.float64, device="cuda")))
    torch.cuda.empty_cache()
    tuned = autotune_batched(ctx, systems, precision="fp32")
    best = tuned["best"]
    ms_b, res = _timed(lambda: ctx.build_batched(systems, precision="fp32", mode=best["mode"]), 3)
    ms_seq32, _ = _timed(lambda: [ctx.build(sy["phi"], sy["pairs"], sy["grid"], kernel=sy["kernel"],
                                            omega=sy["omega"], precision="fp32", want_M=False) for sy in systems], 1)
    ms_seq64, r64 = _timed(lambda: [ctx.build(sy["phi"], sy["pairs"], sy["grid"], kernel=sy["kernel"],
                                              omega=sy["omega"], precision="fp64", want_M=False) for sy in systems], 1)
    errs = [abs(res[q]["ex"].item() - r64[q]["ex"].item()) / abs(r64[q]["ex"].item()) for q in range(len(systems))]
    npairs = sum(int(sy["pairs"].shape[0]) for sy in systems)
    out = {"workload": "16 systems, 8-64 molecules, 48^3-96^3, mixed bare/erfc, rho_cut=1e-3, FP32 pair stage",
           "systems": [{"n_mol": sp.n_mol, "N": sp.N, "kernel": sp.kernel, "pairs": int(sy["pairs"].shape[0])}
                       for sp, sy in zip(specs, systems)],
           "pairs_total": npairs, "tuned": best, "tune_table": tuned["table"],
           "batched_ms": round(ms_b, 2), "builds_per_s": round(len(systems) / ms_b * 1000, 2),
           "pair_solves_per_s": round(npairs / ms_b * 1000, 1),
           "sequential_fp32_ms": round(ms_seq32, 2), "sequential_fp64_ms": round(ms_seq64, 2),
           "max_ex_rel_err_vs_fp64": max(errs)}
    log(f"batched form: {out['batched_ms']} ms for 16 builds (sequential fp32 {out['sequential_fp32_ms']} ms)")
    return out


def form_kpoints(ctx, log, with_oracle=True):
    """Complex Bloch orbitals on a 2x2x2 k-point mesh: 8 waters per cell (the
    32-water cell's density and grid spacing, L = 9.3 bohr on 48^3), 32 bands
    per k-point, localized Bloch sums screened at rho_cut = 1e-3, erfc kernel.
    Times the screening and the FP64 build; the split complex passes move
    16 N^3 16 bytes per pair.  With with_oracle, W rows 0 and n-1 against the
    k-point oracle over the kept pairs that touch them, and the pair list
    against the oracle's."""
    import numpy as np
    import torch

    from paper_2101_03155_amd import Grid
    from synth import SystemSpec, make_bloch_orbitals

    spec = SystemSpec(n_mol=8, L=9.3, N=48, sigma=1.0, offset=0.8, placement="lattice", jitter=0.5, seed=7001,
                      kernel="erfc", omega=0.106)
    kf = [(a, b, c) for a in (0.0, 0.5) for b in (0.0, 0.5) for c in (0.0, 0.5)]
    u, kv = make_bloch_orbitals(spec, kf, mix=False)
    g = Grid.cubic(spec.N, spec.L)
    ud = torch.as_tensor(u, device="cuda")
    rho_cut = 1e-3
    ms_pl, (pairs, _) = _timed(lambda: ctx.pairlist_kpoints(ud, g, rho_cut), 3)
    ms_b, r = _timed(lambda: ctx.build_kpoints(ud, kv, spec.norb, pairs, g, kernel=spec.kernel, omega=spec.omega,
                                               want_W=True), 3)
    npairs = int(pairs.shape[0])
    ntot = u.shape[0]
    per_pair = 16 * spec.N ** 3 * 16
    tbs = per_pair * npairs / (ms_b / 1000.0) / 1e9
    out = {"workload": f"8 waters per cell, 2x2x2 k-points, {spec.norb} bands per k-point ({ntot} in all), "
                       f"{spec.N}^3, L={spec.L}, erfc omega={spec.omega}, rho_cut={rho_cut}",
           "pairs": npairs, "pairs_full": ntot * (ntot + 1) // 2, "pairlist_ms": round(ms_pl, 3),
           "build_ms": round(ms_b, 3), "pair_solves_per_s": round(npairs / ms_b * 1000, 1),
           "bytes_per_pair_16N3x16": per_pair, "achieved_gbs": round(tbs, 1),
           "frac_hbm_peak": round(tbs / HBM_PEAK_GBS, 4), "ex": float(r["ex"].item())}
    if with_oracle:
        from oracle import kpoint_oracle as ko

        pl = pairs.cpu().numpy()
        ref_pairs, _ = ko.pairlist_k(u, spec.dV, rho_cut)
        out["pairs_equal_oracle"] = bool(np.array_equal(pl, ref_pairs))
        rows = [0, ntot - 1]
        touch = pl[np.isin(pl[:, 0], rows) | np.isin(pl[:, 1], rows)]
        t0 = time.perf_counter()
        Wref, _ = ko.build_W_k(u, kv, spec.norb, touch, spec.N, spec.L, spec.kernel, spec.omega)
        Wg = r["W"].cpu().numpy()
        errs = [float(np.abs(Wg[q] - Wref[q]).max() / np.abs(Wref[q]).max()) for q in rows]
        out["vs_oracle"] = {"rows": rows, "pairs_touching": int(touch.shape[0]),
                            "W_max_elem_err_rel": max(errs), "oracle_s": round(time.perf_counter() - t0, 2)}
    log(f"k-point form: {npairs} pairs, {out['build_ms']} ms, {out['achieved_gbs']} GB/s")
    return out


def form_learned_batched(ctx, log, model_paths, mode="graph"):
    """The learned-screened FP32 batched build against the plain FP64
    full-pair builds of the same 16 systems (8-64 molecules, 48^3-96^3):
    builds/s of each and the E_x error of every learned build against its
    full-pair FP64 build, within the budget of 1e-5 Ha per molecule."""
    import torch

    from paper_2101_03155_amd import Grid
    from paper_2101_03155_amd.screener import LearnedScreener
    from synth import batched_specs, make_orbitals

    for k, p in model_paths.items():
        if not os.path.exists(p):
            return {"skipped": f"no {k} screener checkpoint at {p}"}
    scrs = {k: LearnedScreener.load(p) for k, p in model_paths.items()}
    specs = batched_specs()
    systems, fulls, loc_ms, sel_ms, fallbacks = [], [], 0.0, 0.0, 0
    for sp in specs:
        o = make_orbitals(sp, device="cuda")
        g = Grid.cubic(sp.N, sp.L)
        ms, (phi, _, _) = _timed(lambda: ctx.localize(o.psi, g), 1)
        loc_ms += ms
        del o
        # each system is screened by the screener trained on its own kernel
        ms, (pl, fb) = _timed(lambda: scrs[sp.kernel].select(ctx, phi, g, sp.n_mol), 1)
        sel_ms += ms
        fallbacks += int(fb)
        n = phi.shape[0]
        systems.append(dict(phi=phi, pairs=pl, grid=g, kernel=sp.kernel, omega=sp.omega,
                            xi=torch.empty_like(phi), M=torch.empty(n, n, dtype=torch.float64, device="cuda"),
                            ex=torch.empty(1, dtype=torch.float64, device="cuda")))
        fulls.append(torch.tensor([(i, j) for i in range(n) for j in range(i, n)], dtype=torch.int32, device="cuda"))
    torch.cuda.empty_cache()
    ms_b, res = _timed(lambda: ctx.build_batched(systems, precision="fp32", mode=mode), 3)
    ex_l = [float(r["ex"].item()) for r in res]

    def full_builds():
        out = []
        for sy, fp in zip(systems, fulls):
            r = ctx.build(sy["phi"], fp, sy["grid"], kernel=sy["kernel"], omega=sy["omega"], precision="fp64",
                          want_M=False)
            out.append(float(r["ex"].item()))
            del r
        return out

    ms_full, ex_f = _timed(full_builds, 1)
    errs = [abs(a - b) for a, b in zip(ex_l, ex_f)]
    # the screening part of the error: FP64 builds of the learned lists
    ex_l64 = []
    for sy in systems:
        r = ctx.build(sy["phi"], sy["pairs"], sy["grid"], kernel=sy["kernel"], omega=sy["omega"], precision="fp64",
                      want_M=False)
        ex_l64.append(float(r["ex"].item()))
        del r
    scr_errs = [abs(a - b) for a, b in zip(ex_l64, ex_f)]
    budgets = [1e-5 * sp.n_mol for sp in specs]
    npairs = sum(int(sy["pairs"].shape[0]) for sy in systems)
    nfull = sum(int(f.shape[0]) for f in fulls)
    out = {"workload": "16 systems, 8-64 molecules, 48^3-96^3, mixed bare/erfc; learned screeners (one per "
                       f"kernel), FP32 batched build ({mode} mode) vs FP64 full-pair single builds",
           "margins": {k: s.margin for k, s in scrs.items()},
           "pairs_learned": npairs, "pairs_full": nfull, "used_fallback": fallbacks,
           "learned_fp32_batched": {"ms": round(ms_b, 2), "builds_per_s": round(16 / ms_b * 1000, 2),
                                    "builds_per_s_with_localize_and_selection":
                                        round(16 / (ms_b + loc_ms + sel_ms) * 1000, 2),
                                    "localize_ms": round(loc_ms, 2), "selection_ms": round(sel_ms, 2)},
           "full_fp64": {"ms": round(ms_full, 2), "builds_per_s": round(16 / ms_full * 1000, 3),
                         "builds_per_s_with_localize": round(16 / (ms_full + loc_ms) * 1000, 3)},
           "max_abs_err_vs_full_fp64_ha": max(errs),
           "max_screening_err_ha": max(scr_errs),
           "screening_within_budget": all(e <= b for e, b in zip(scr_errs, budgets)),
           "note": ("abs_err_ha: the FP32 learned batched build against the FP64 full-pair build (screening plus "
                    "FP32 rounding); screening_err_ha: the FP64 build of the learned list against the same "
                    "(the part the budget of 1e-5 Ha per molecule bounds)"),
           "per_system": [{"n_mol": sp.n_mol, "N": sp.N, "kernel": sp.kernel, "pairs": int(sy["pairs"].shape[0]),
                           "pairs_full": int(f.shape[0]), "abs_err_ha": e, "screening_err_ha": se, "budget_ha": b}
                          for sp, sy, f, e, se, b in zip(specs, systems, fulls, errs, scr_errs, budgets)]}
    out["speedup_vs_full_fp64"] = round(ms_full / ms_b, 2)
    log(f"learned batched: {ms_b:.1f} ms vs full fp64 {ms_full:.1f} ms, max |dE| {max(errs):.2e}")
    del systems, fulls, res
    torch.cuda.empty_cache()
    return out


def form_learned(ctx, log, model_path):
    """128 waters (512 orbitals, 160^3): learned vs threshold vs full-pair builds."""
    import torch

    from paper_2101_03155_amd import Grid
    from paper_2101_03155_amd.screener import LearnedScreener
    from synth import config_spec, make_orbitals

    if not os.path.exists(model_path):
        return {"skipped": f"no screener checkpoint at {model_path}"}
    scr = LearnedScreener.load(model_path)
    spec = config_spec("c5")
    o = make_orbitals(spec, device="cuda")
    g = Grid.cubic(spec.N, spec.L)
    ctx.localize(o.psi, g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, _, _ = ctx.localize(o.psi, g)
    torch.cuda.synchronize()
    ms_loc = (time.perf_counter() - t0) * 1000
    del o
    torch.cuda.empty_cache()
    budget = 1e-5 * spec.n_mol
    ms_sel, (pl, fb) = _timed(lambda: scr.select(ctx, phi, g, spec.n_mol), 2)
    ms_thr_sel, (pt, _) = _timed(lambda: ctx.pairlist(phi, g, 1e-3), 2)
    n = spec.norb
    full = torch.tensor([(i, j) for i in range(n) for j in range(i, n)], dtype=torch.int32, device="cuda")
    ms_full, rf = _timed(lambda: ctx.build(phi, full, g, kernel="erfc", omega=spec.omega, precision="fp64",
                                           want_M=False), 1, warm=False)
    ex_full = rf["ex"].item()
    del rf
    out = {"workload": "128 waters: 512 orbitals, 160^3, L=29.6, erfc omega=0.106", "budget_ha": budget,
           "margin": scr.margin, "used_fallback": fb, "localize_ms": round(ms_loc, 1),
           "full_fp64": {"pairs": int(full.shape[0]), "build_ms": round(ms_full, 1),
                         "builds_per_s": round(1000 / ms_full, 4), "ex": ex_full},
           "screener_train": {k: v for k, v in scr.meta.items() if k != "loss_curve"}}
    out["full_fp64"]["builds_per_s_with_localize"] = round(1000 / (ms_full + ms_loc), 4)
    for name, pl_, sel_ms in (("learned_fp32", pl, ms_sel), ("threshold_fp32", pt, ms_thr_sel)):
        ms_b, r = _timed(lambda: ctx.build(phi, pl_, g, kernel="erfc", omega=spec.omega, precision="fp32",
                                           want_M=False), 2)
        err = abs(r["ex"].item() - ex_full)
        out[name] = {"pairs": int(pl_.shape[0]), "select_ms": round(sel_ms, 2), "build_ms": round(ms_b, 1),
                     "builds_per_s": round(1000 / (ms_loc + sel_ms + ms_b), 3),
                     "builds_per_s_without_localize": round(1000 / (ms_b + sel_ms), 3), "ex": r["ex"].item(),
                     "abs_err_vs_full_fp64": err, "within_budget": err <= budget}
        log(f"learned form {name}: {out[name]}")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the pair-sharded multi-GPU "
              "form is a design only and is not built", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    import numpy as np
    import torch

    from paper_2101_03155_amd import Context, Grid, ace
    from synth import config_spec, make_orbitals

    spec = config_spec(args.config)
    kind, omega = spec.kernel, spec.omega
    # the oracle baseline needs the orbitals on the host; otherwise they are
    # assembled on the device (the large systems)
    o = make_orbitals(spec, device=None if not args.no_cpu_baseline else "cuda")
    psi = o.psi if args.no_cpu_baseline else torch.as_tensor(o.psi, device="cuda")
    grid = Grid.cubic(spec.N, spec.L)
    ctx = Context()
    prec = args.precision

    def step():
        phi, piv, _ = ctx.localize(psi, grid)
        pairs, _ = ctx.pairlist(phi, grid, args.rho_cut)
        r = ctx.build(phi, pairs, grid, kernel=kind, omega=omega, precision=prec, want_M=False)
        return phi, piv, pairs, r

    tuned = None
    if args.shape == "auto":
        from paper_2101_03155_amd.tune import autotune

        phi0, _, _ = ctx.localize(psi, grid)
        pairs0, _ = ctx.pairlist(phi0, grid, args.rho_cut)
        tuned = autotune(ctx, phi0, pairs0, grid, kind, omega, prec)
        del phi0, pairs0
    elif args.shape in ("fused", "split", "r2c", "owner"):
        ctx.set_pair_shape(prec, spec.N, args.shape, args.max_packs)
    shape = ctx.get_pair_shape(prec, spec.N)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # Timed region: HIP events bracket the stages and the pair-stage kernels
    # only (the dominant kernel is timed live); the many small launches of
    # the pivot search and the GEMMs are left unbracketed, so the events add
    # no measurable time to the steps.
    ctx.profile(True)
    ctx.profile_classes([0, 1, 2, 3, 4, 5, 6, 10, 11, 12, 13, 14])
    for c in range(15):
        ctx.profile_read(c, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        phi, piv, pairs, r = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {c: ctx.profile_read(c, reset=True) for c in range(15)}
    # the other classes' rates from two more, fully bracketed steps
    ctx.profile_classes(None)
    for _ in range(2):
        step()
    for c in (7, 8, 9):
        prof[c] = ctx.profile_read(c, reset=True)
    ctx.profile(False)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    npairs = int(pairs.shape[0])
    ex = float(r["ex"].item())

    stage_ms = {name: prof[c][1] / args.steps for c, name in
                ((10, "localize"), (11, "pairlist"), (12, "pair_stage"), (13, "tail"), (14, "build"))}
    pair_solves = npairs / (stage_ms["pair_stage"] / 1000.0)

    # dominant kernel class (per step: classes 7-9 come from the two extra steps)
    dom = max(range(10), key=lambda c: prof[c][1] / (2 if c in (7, 8, 9) else args.steps))
    n_l, ms_l, units = prof[dom]
    if dom in (7, 8):
        peak = FP64_PEAK_TFLOPS
        achieved = units / (ms_l / 1000.0) / 1e12
        roof = {"bound": "mfma", "unit": "TFLOP/s"}
    else:
        peak = HBM_PEAK_GBS
        achieved = units / (ms_l / 1000.0) / 1e9
        roof = {"bound": "hbm", "unit": "GB/s"}
    kname = CLASS_KERNEL[dom]
    if shape[0] in ("r2c", "owner") and dom in (0, 1, 2):
        kname = "k_inv_owner_r" if (shape[0] == "owner" and dom == 2) else kname + "_r"
    roof.update({"kernel": kname, "class": CLASS_NAMES[dom], "launches_per_step": n_l / args.steps,
                 "avg_launch_us": 1000.0 * ms_l / max(n_l, 1),
                 "algorithmic_per_launch": units / max(n_l, 1),
                 "achieved": round(achieved, 2), "peak": peak, "frac": round(achieved / peak, 4)})
    traffic, note = (measured_traffic(kname, spec.N, prec, units / max(n_l, 1)) if dom < 7
                     else (None, "not an HBM-bound class"))
    roof["traffic"] = round(traffic) if traffic is not None else None
    roof["traffic_note"] = note
    if traffic is not None:
        roof["frac_counter"] = round(traffic / (ms_l / max(n_l, 1) / 1000.0) / 1e9 / peak, 4)
    # the whole pair stage: the 12 N^3 s bytes per pair of the read-modify-write
    # design (two FFT round trips, phi read twice, W read and written), and the
    # counter bytes of its kernels, both over the stage's event time
    s_bytes = 8 if prec == "fp64" else 4
    st_ms = stage_ms["pair_stage"]
    per_pair = 12 * spec.N ** 3 * s_bytes
    stage = {"bytes_per_pair_12N3s": per_pair, "ms": round(st_ms, 3),
             "achieved_12N3s": round(per_pair * npairs / (st_ms / 1000.0) / 1e9, 1)}
    stage["frac_12N3s"] = round(stage["achieved_12N3s"] / HBM_PEAK_GBS, 4)
    pair_classes = [c for c in range(7) if prof[c][0]]
    t_bytes, missing = 0.0, []
    for c in pair_classes:
        kn = CLASS_KERNEL[c] + ("_r" if shape[0] in ("r2c", "owner") and c < 3 else "")
        if shape[0] == "owner" and c == 2:
            kn = "k_inv_owner_r"
        row, why = counter_row(kn, spec.N, prec)
        if row is None:
            missing.append(f"{kn}: {why}")
        else:
            t_bytes += row["traffic_per_algorithmic_byte"] * prof[c][2] / args.steps
    if not missing and pair_classes:
        stage["counter_bytes_per_step"] = round(t_bytes)
        stage["frac_counter"] = round(t_bytes / (st_ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)
    else:
        stage["counter_bytes_per_step"] = None
        stage["counter_note"] = "; ".join(missing)
    roof["stage"] = stage
    kernels = {CLASS_NAMES[c]: {"steps": 2 if c in (7, 8, 9) else args.steps, "launches": prof[c][0],
                                "ms": round(prof[c][1], 3),
                                "rate": (round(prof[c][2] / (prof[c][1] / 1000.0) / (1e12 if c in (7, 8) else 1e9), 2)
                                         if prof[c][1] > 0 else None)}
               for c in range(10) if prof[c][0]}

    out = {
        "metric": METRIC, "value": round(1000.0 / ms_per_step, 4), "unit": "builds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"screened ACE build from canonical orbitals, {spec.norb} orbitals, {spec.N}^3 grid, "
                               f"L={spec.L} bohr, {kind} kernel omega={omega}, rho_cut={args.rho_cut}",
                   "norb": spec.norb, "grid": spec.N, "npairs_kept": npairs, "precision": prec},
        "pair_solves_per_s": round(pair_solves, 1),
        "stage_ms": {k: round(v, 3) for k, v in stage_ms.items()},
        "ex_hartree": ex,
        "pair_shape": {"path": shape[0], "max_packs": shape[1],
                       "tune_table": tuned["table"] if tuned else None},
        "roofline": roof,
        "kernels": kernels,
    }

    pairs_np = pairs.cpu().numpy().astype(np.int64)
    piv_np = piv.cpu().numpy()
    oracle_ref = None
    if not args.no_cpu_baseline:
        # the oracle's whole step on the host cores (rank 0, one GPU): the CPU
        # baseline, and the reference of the step's parity figures
        out["cpu_baseline"], oracle_ref = cpu_baseline(o, kind, omega, args.rho_cut)
        out["parity_vs_oracle"] = parity_vs_oracle(ctx, grid, kind, omega, prec, piv_np, pairs_np, oracle_ref)
        out["ex_rel_err_vs_oracle_fp64"] = abs(ex - oracle_ref["ex"]) / abs(oracle_ref["ex"])
        del oracle_ref
    elif not args.no_oracle_check:
        import oracle

        phi_np = phi.cpu().numpy()
        v = oracle.coulomb_kernel(spec.N, spec.L, kind, omega)
        e_ref = oracle.exchange_energy_pairs(phi_np, pairs_np, v, spec.dV, workers=host_workers())
        out["ex_rel_err_vs_oracle_fp64"] = abs(ex - e_ref.sum()) / abs(e_ref.sum())

    if not args.no_forms:
        log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
        forms = {}
        n = spec.norb
        full = torch.tensor([(i, j) for i in range(n) for j in range(i, n)], dtype=torch.int32, device="cuda")
        for p in ("fp64", "fp32"):
            ctx.build(phi, full, grid, kernel=kind, omega=omega, precision=p, want_M=False)
            ctx.profile(True)
            ctx.profile_read(12, reset=True)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(3):
                rf = ctx.build(phi, full, grid, kernel=kind, omega=omega, precision=p, want_M=False)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            _, pms, _ = ctx.profile_read(12, reset=True)
            ctx.profile(False)
            forms[f"c2_full_{p}_build_ms"] = round((tb - ta) * 1000 / 3, 3)
            forms[f"c2_full_{p}_pair_solves_per_s"] = round(full.shape[0] / (pms / 3 / 1000.0), 1)
            forms[f"c2_full_{p}_ex"] = float(rf["ex"].item())
        r32 = ctx.build(phi, pairs, grid, kernel=kind, omega=omega, precision="fp32", want_M=False)
        forms["c2_screened_ex_rel_err_fp32_vs_fp64"] = abs(float(r32["ex"].item()) - ex) / abs(ex)
        del full, rf, r32
        torch.cuda.empty_cache()
        forms["apply_energy"] = form_apply_energy(ctx, r["xi"], phi, grid)
        forms["exact_exchange"] = form_exact_exchange(ctx, psi, grid, kind, omega)
        forms["incremental"] = form_incremental(ctx, psi, spec, grid, kind, omega, args.rho_cut)
        torch.cuda.empty_cache()
        for name, fn in (("precision", lambda: form_precision(ctx, log)), ("batched", lambda: form_batched(ctx, log)),
                         ("kpoints", lambda: form_kpoints(ctx, log)),
                         ("learned", lambda: form_learned(ctx, log, args.screener)),
                         ("learned_batched", lambda: form_learned_batched(
                             ctx, log, {"erfc": args.screener, "bare": args.screener_bare},
                             forms.get("batched", {}).get("tuned", {}).get("mode", "graph")))):
            if name in args.skip_forms.split(","):
                continue
            ctx.release_workspace()  # each form starts from an empty device workspace
            torch.cuda.empty_cache()
            try:
                forms[name] = fn()
            except Exception as e:  # a failing form is reported, not hidden
                forms[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
        out["forms"] = forms

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
