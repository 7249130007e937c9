"""Throughput benchmark: cell-stage updates/s of the CTENOZ hot path on one MI355X.

Workload: isentropic vortex (strength 5, centred at (5,5)) on the periodic
[0,10]^2 box, 2000 x 2000 squares split into 8,000,000 jittered triangles
(seed 5), cubic CTENOZ (lambda1' = 1e4), SSP-RK3 at CFL 0.3.  The mixed
path (FP32 reconstruction / weights / HLLC, FP64 state and update) gives
`value`; the all-FP64 path is reported beside it, with the error of each
against the exact solution and against each other, and the TENO-cutoff
flip count.  Inputs are resident in HBM before the timed region.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell and stage of the dominant kernel (reconstruction):
# pseudo-inverses (162 central + 24 directional entries), 18 slot indices,
# 1 flag byte, the cell's FP64 state (4 x 8) and its 24 face-point values
RECON_BYTES = {"mixed": 162 * 4 + 24 * 4 + 18 * 4 + 1 + 32 + 24 * 4,
               "fp64": 162 * 8 + 24 * 8 + 18 * 4 + 1 + 32 + 24 * 8}
# flux + residual + RK kernel: own face values, neighbour codes, face
# geometry, area, U^n / stage input / output
FLUX_BYTES = {"mixed": 24 * 4 + 12 + 9 * 4 + 8 + 3 * 32,
              "fp64": 24 * 8 + 12 + 9 * 8 + 8 + 3 * 32}


# HBM bytes per cell and launch of the mixed reconstruction kernel measured
# with the FETCH_SIZE / WRITE_SIZE counters (scaled by the copy-kernel
# calibration), valid only for the kernel source they were taken on
MEASURED_TRAFFIC = {"kernels_sha256_prefix": "19d0de76df99ab6e", "recon_mixed_bytes_per_cell": 966.6}


KERNEL_SOURCES = ("kernels_common.h", "k_recon.inl", "k_recon_ho.inl", "k_recon_f32.hip", "k_recon_f64.hip",
                  "k_recon_ho_f32.hip", "k_recon_ho_f64.hip", "k_precompute.hip", "k_flux.hip")


def kernels_hash():
    """sha256 prefix of the device sources, in a fixed order"""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_17042_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(T, ctx, mesh, sol, u0, prec, steps, warmup):
    import torch
    sol.set(u0, 0.0)
    # warm-up: also captures the step graph
    sol.solve(max_steps=warmup, cfl=0.3, precision=prec, use_graph=True)
    ctx.set_timing(True)
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = sol.solve(max_steps=steps, cfl=0.3, precision=prec, use_graph=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kr = ctx.kernel_stats(T.KERNEL_RECONSTRUCT)
    kf = ctx.kernel_stats(T.KERNEL_FLUX)
    ctx.set_timing(False)
    assert n == steps, (n, steps)
    u, t = sol.download()
    # the same steps replayed as a captured graph (no per-kernel events)
    sol.set(u0, 0.0)
    sol.solve(max_steps=warmup, cfl=0.3, precision=prec, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ng = sol.solve(max_steps=steps, cfl=0.3, precision=prec, use_graph=True)
    torch.cuda.synchronize()
    elg = time.perf_counter() - t0
    assert ng == steps, (ng, steps)
    return dict(elapsed=el, recon=kr, flux=kf, u=u, t=t, graph_elapsed=elg)


def ho_recon_bytes(r, prec):
    """Algorithmic bytes per cell and launch of the reconstruction at degree
    r >= 4: the useful pseudo-inverse entries (K x M central, K_d x M_d per
    directional stencil), M slot indices, the flag byte, the cell's FP64
    state and its 3 N_q x 4 face-point values."""
    K = (r + 1) * (r + 2) // 2 - 1
    rd = (r + 1) // 2
    Kd = (rd + 1) * (rd + 2) // 2 - 1
    Md, M, Nq = 2 * Kd, 2 * K, (r + 2) // 2
    es = 4 if prec == "mixed" else 8
    return (K * M + 3 * Kd * Md) * es + M * 4 + 1 + 32 + 3 * Nq * 4 * es


def orders_bench(T, W, ctx, n=1000, steps=5, warmup=1):
    """Orders 5 to 7 (r = 4, 5, 6) on the isentropic vortex, n x n squares,
    CTENOZ lambda1' = 1e4: mixed-precision throughput and the reconstruction's
    algorithmic bandwidth."""
    import torch
    mesh, u0 = W.vortex_case(n, seed=5, quad=3)
    N = mesh.n_cells
    out = {"workload": f"isentropic vortex, {n}x{n} split/jittered periodic [0,10]^2 ({N} cells), CTENOZ "
                       f"lambda1'=1e4, SSP-RK3 CFL 0.3, mixed precision", "cells": N}
    for r in (4, 5, 6):
        t0 = time.perf_counter()
        m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=T.CTENOZ, degree=r, lambda1_prime=1e4,
                                 precision=T.MIXED)
        t_up = time.perf_counter() - t0
        sol = T.Solution(m, u0)
        res = run_precision(T, ctx, m, sol, u0, T.MIXED, steps, warmup)
        nrec, msrec = res["recon"]
        nfl, msfl = res["flux"]
        avg = msrec / max(1, nrec)
        b = ho_recon_bytes(r, "mixed")
        gbs = b * N / (avg * 1e-3) / 1e9
        out[f"r{r}"] = {"order": r + 1, "value": N * 3 * steps / res["elapsed"], "unit": "cell-stage updates/s",
                        "ms_per_step": 1e3 * res["elapsed"] / steps, "reconstruct_ms": avg,
                        "flux_rk_ms": msfl / max(1, nfl), "recon_bytes_per_cell": b, "recon_GBs": gbs,
                        "recon_frac_of_8TBs": gbs / HBM_PEAK_GBS, "upload_precompute_s": t_up,
                        "device_bytes": int(m.info.device_bytes)}
        log(f"order {r + 1}: {out[f'r{r}']['value']:.3e} cell-stage/s, recon {avg:.3f} ms ({gbs:.0f} GB/s), "
            f"flux {msfl / max(1, nfl):.3f} ms, upload {t_up:.1f}s")
        sol.close()
        m.close()
        torch.cuda.synchronize()
    return out


# normalised computational times the paper prints (with respect to CWENO of
# 5th order) for the single-material triple point problem (Table tab2)
PAPER_SCHEME_TIMES = {"5th": {"CWENO": 1.000, "TENO": 1.024, "CTENO": 1.043, "CTENOZ": 1.081},
                      "7th": {"CWENO": 1.538, "TENO": 1.557, "CTENO": 1.571, "CTENOZ": 1.643}}


def schemes_bench(T, W, ctx, steps=10, warmup=2):
    """CWENO, TENO, CTENO and CTENOZ at orders 5 and 7 on Table tab2's own
    workload, the triple point on 215,000 cells (lambda1' = 1e4, from t = 0):
    time per step from graph replay, FP64 and mixed, normalised to CWENO5
    beside the paper's ratios."""
    mesh, u0 = W.triple_point_case()
    N = mesh.n_cells
    names = [("CWENO", T.CWENO), ("TENO", T.TENO), ("CTENO", T.CTENO), ("CTENOZ", T.CTENOZ)]
    ms = {"fp64": {}, "mixed": {}}
    for order, r in (("5th", 4), ("7th", 6)):
        for p in ms:
            ms[p][order] = {}
        for name, sch in names:
            m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=sch, degree=r, lambda1_prime=1e4,
                                     precision=T.BOTH)
            sol = T.Solution(m, u0)
            for p, prec in (("fp64", T.FP64), ("mixed", T.MIXED)):
                res = run_precision(T, ctx, m, sol, u0, prec, steps, warmup)
                ms[p][order][name] = 1e3 * res["graph_elapsed"] / steps
            sol.close()
            m.close()
    norm = {p: {o: {k: v / d["5th"]["CWENO"] for k, v in row.items()} for o, row in d.items()}
            for p, d in ms.items()}
    for p in norm:
        log(f"schemes {p} (triple point, normalised to CWENO5): " + "; ".join(
            f"{o}: " + ", ".join(f"{k} {v:.3f}" for k, v in row.items()) for o, row in norm[p].items()))
    return {"workload": f"triple point on [0,7]x[0,3], 500x215 split/jittered ({N} cells), walls, "
                        f"lambda1'=1e4, from t = 0, graph replay",
            "ms_per_step": ms, "normalised_time": norm, "paper_table_tab2": PAPER_SCHEME_TIMES}


# the paper's double Mach reflection timings (sec. 3.4): Table tab1's times
# normalised to CWENO5 on 369,604 triangles, and the wall-clock time of one
# CTENO5 iteration on 714,138 triangles with 64 MPI processes (AMD EPYC 7542;
# CTENO7 about 1.5 times that)
PAPER_DMR_TIMES = {"369604": {"CWENO": 1.000, "TENO": 1.036, "CTENO": 1.033, "CTENOZ": 1.000},
                   "714138": {"CWENO": 2.798, "TENO": 2.870, "CTENO": 2.795, "CTENOZ": 2.811}}
PAPER_DMR_CTENO5_S_PER_ITERATION = 1.7


def dmr_bench(T, W, ctx, steps=20, warmup=2):
    """The paper's timing workload: the double Mach reflection on meshes of
    the paper's two sizes, CWENO / TENO / CTENO / CTENOZ of 5th order
    (lambda1' = 1e15, conserved variables) from t = 0, FP64 and mixed, time
    per SSP-RK3 iteration from graph replay; CTENO7 on the larger mesh."""
    names = [("CWENO", T.CWENO), ("TENO", T.TENO), ("CTENO", T.CTENO), ("CTENOZ", T.CTENOZ)]
    out = {"workload": "double Mach reflection on [0,4]x[0,1], split/jittered squares, lambda1'=1e15, "
                       "conserved variables, SSP-RK3 CFL 0.3 from t = 0, graph replay",
           "ms_per_iteration": {}, "paper_table_tab1": PAPER_DMR_TIMES,
           "paper_cteno5_s_per_iteration_64_cpu_processes": PAPER_DMR_CTENO5_S_PER_ITERATION}
    for nx, ny, label in ((860, 215, "369604"), (1196, 299, "714138")):
        mesh, u0 = W.dmr_case(nx, ny)
        row = {"cells": mesh.n_cells}
        runs = [(name, sch, 4) for name, sch in names] + ([("CTENO7", T.CTENO, 6)] if label == "714138" else [])
        for name, sch, r in runs:
            m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=sch, degree=r, lambda1_prime=1e15,
                                     precision=T.BOTH)
            sol = T.Solution(m, u0)
            row[name] = {}
            for pname, prec in (("fp64", T.FP64), ("mixed", T.MIXED)):
                res = run_precision(T, ctx, m, sol, u0, prec, steps, warmup)
                row[name][pname] = 1e3 * res["graph_elapsed"] / steps
            sol.close()
            m.close()
        out["ms_per_iteration"][label] = row
        log(f"dmr {label} ({mesh.n_cells} cells): " + ", ".join(
            f"{k} {v['fp64']:.3f}/{v['mixed']:.3f} ms" for k, v in row.items() if k != "cells"))
    ref = out["ms_per_iteration"]["369604"]["CWENO"]["fp64"]
    out["normalised_fp64"] = {lab: {k: v["fp64"] / ref for k, v in row.items() if k != "cells"}
                              for lab, row in out["ms_per_iteration"].items()}
    big = out["ms_per_iteration"]["714138"]["CTENO"]
    out["cteno5_714k_s_per_iteration"] = {"fp64": big["fp64"] / 1e3, "mixed": big["mixed"] / 1e3}
    return out


def variables_bench(T, W, ctx, n=1000, steps=5, warmup=1):
    """Reconstruction in characteristic variables (per face, three
    projections and selections per cell) against conserved variables:
    mixed-precision step time and reconstruction time at r = 3 and 4."""
    mesh, u0 = W.vortex_case(n, seed=5, quad=3)
    out = {"workload": f"isentropic vortex, {n}x{n} ({mesh.n_cells} cells), CTENOZ lambda1'=1e4, mixed precision"}
    for r in (3, 4):
        row = {}
        for name, var in (("conserved", T.CONSERVED), ("characteristic", T.CHARACTERISTIC)):
            m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=T.CTENOZ, degree=r, lambda1_prime=1e4,
                                     precision=T.MIXED, variables=var)
            sol = T.Solution(m, u0)
            res = run_precision(T, ctx, m, sol, u0, T.MIXED, steps, warmup)
            nrec, msrec = res["recon"]
            row[name] = {"ms_per_step": 1e3 * res["elapsed"] / steps, "reconstruct_ms": msrec / max(1, nrec)}
            sol.close()
            m.close()
        row["step_ratio"] = row["characteristic"]["ms_per_step"] / row["conserved"]["ms_per_step"]
        out[f"r{r}"] = row
        log(f"variables r={r}: conserved {row['conserved']['ms_per_step']:.3f} ms/step, characteristic "
            f"{row['characteristic']['ms_per_step']:.3f} ms/step (x{row['step_ratio']:.3f})")
    return out


def cpu_baseline(W, target_s=12.0, max_steps=40):
    """The FP64 oracle on a bounded sample of the same workload family: SSP-RK3
    steps on a 320k-cell mesh until about target_s seconds of work."""
    import oracle as O
    n = 400
    mesh, u0 = W.vortex_case(n, seed=5)
    o = O.Oracle.from_mesh(mesh, physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)
    o.prepare()                      # stencils + least-squares factors: excluded, as on the GPU
    dt = 0.3 * o.dt_bound(u0)
    steps = 0
    t0 = time.perf_counter()
    U = u0
    while steps < max_steps and time.perf_counter() - t0 < target_s:
        U = o.rk3_step(U, dt)
        steps += 1
    el = time.perf_counter() - t0
    return {"value": mesh.n_cells * 3 * steps / el, "unit": "cell-stage updates/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"isentropic vortex on {n}x{n} split/jittered periodic [0,10]^2 ({mesh.n_cells} cells, same "
                      f"per-cell work as the 8M-cell case), cubic CTENOZ FP64, {steps} SSP-RK3 steps, "
                      f"{el:.2f} s wall, precompute excluded"}


def serving_bench(T, W, ctx, n_requests=256, budget_gb=4.0, max_slots=128, steps=100):
    """Poisson stream of independent Euler solves through the continuous-batching server."""
    import statistics
    t0 = time.perf_counter()
    reqs = W.serving_requests(n_requests, rate_hz=1.0, seed=4)
    items = [W.build_request(r) for r in reqs]
    cells = [m.n_cells for m, _ in items]
    log(f"serving: {n_requests} requests generated ({sum(cells)} cells, {time.perf_counter() - t0:.1f}s)")
    scheme = T.make_scheme(physics=T.EULER, scheme=T.CTENOZ, degree=3, lambda1_prime=1e4, precision=T.MIXED)

    def run(arrivals):
        srv = T.Server(ctx, scheme, budget_bytes=int(budget_gb * (1 << 30)), max_slots=max_slots)
        tickets = []
        start = time.perf_counter()
        for (mesh, u0), at in zip(items, arrivals):
            now = time.perf_counter() - start
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(mesh, u0, steps))
        srv.drain()
        wall = time.perf_counter() - start
        lat, failed = [], 0
        for t in tickets:
            try:
                st, _, _, l = srv.poll(t)
                lat.append(l)
                srv.poll(t, take=True)
            except T.CtenoError:
                failed += 1
        stats = srv.stats()
        srv.close()
        return wall, lat, failed, stats

    wall, lat, failed, st = run([0.0] * n_requests)
    sat = n_requests / wall
    log(f"serving: closed loop {wall:.2f}s -> {sat:.1f} req/s, peak {st['peak_active']} resident")
    rate = 0.7 * sat
    arrivals = [r.arrival_s / rate for r in reqs]
    wall, lat, failed, st = run(arrivals)
    lat_sorted = sorted(lat)

    def pct(p):
        if not lat_sorted:
            return None
        k = min(len(lat_sorted) - 1, max(0, int(math.ceil(p / 100.0 * len(lat_sorted))) - 1))
        return lat_sorted[k]
    out = {"requests": n_requests, "steps_per_request": steps, "scheme": "CTENOZ r=3, FP32-mixed",
           "cells_total": int(sum(cells)), "budget_bytes": int(budget_gb * (1 << 30)), "max_slots": max_slots,
           "saturation_req_per_s": sat, "rate_hz": rate, "wall_s": wall,
           "throughput_req_per_s": n_requests / wall,
           "cell_stages_per_s": st["cell_stages"] / wall,
           "p50_s": pct(50), "p99_s": pct(99),
           "mean_s": statistics.fmean(lat) if lat else None,
           "peak_active": st["peak_active"], "peak_bytes": st["peak_bytes"], "failed": failed,
           "latency": "submission to result on the host (mesh/stencil build, FP64 precompute, queueing, 100 steps)"}
    log(f"serving: Poisson {rate:.1f}/s -> p50 {out['p50_s']:.3f}s p99 {out['p99_s']:.3f}s, {failed} failed")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2000, help="squares per side (2000 -> 8M cells)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--no-orders", action="store_true", help="skip the orders 5-7 measurement")
    ap.add_argument("--no-schemes", action="store_true", help="skip the CWENO/TENO/CTENO/CTENOZ cost comparison")
    ap.add_argument("--no-variables", action="store_true", help="skip the characteristic-variable cost comparison")
    ap.add_argument("--no-dmr", action="store_true", help="skip the double Mach reflection timings")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding is a design "
              f"note, not part of this library", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2312_17042_amd import cteno as T
    from paper_2312_17042_amd import workloads as W

    t0 = time.perf_counter()
    mesh, u0 = W.vortex_case(args.n, seed=5, quad=3)
    log(f"mesh {mesh.n_cells} cells, initial data {time.perf_counter() - t0:.1f}s")

    ctx = T.Context(0)
    t0 = time.perf_counter()
    m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=T.CTENOZ, degree=3, lambda1_prime=1e4,
                             precision=T.BOTH)
    log(f"upload + FP64 precompute {time.perf_counter() - t0:.1f}s, device bytes {m.info.device_bytes / 1e9:.2f} GB")
    sol = T.Solution(m, u0)
    N = mesh.n_cells

    res = {}
    precs = [("mixed", T.MIXED)] + ([] if args.no_fp64 else [("fp64", T.FP64)])
    for name, prec in precs:
        log(f"timing {name}: {args.warmup} warm-up + {args.steps} steps")
        r = run_precision(T, ctx, m, sol, u0, prec, args.steps, args.warmup)
        r["value"] = N * 3 * args.steps / r["elapsed"]
        res[name] = r
        log(f"{name}: {r['value']:.3e} cell-stage/s, {1e3 * r['elapsed'] / args.steps:.3f} ms/step, "
            f"recon {r['recon'][1] / max(1, r['recon'][0]):.3f} ms/launch, flux {r['flux'][1] / max(1, r['flux'][0]):.3f} ms/launch")

    # accuracy at the end of the timed run, on a sample of cells
    mx = res["mixed"]
    sample = np.arange(0, N, 97)
    T_end = mx["t"]
    sub = W.Mesh(mesh.xy, mesh.tri[sample], mesh.box, mesh.bc, mesh.nx, mesh.ny, mesh.seed)
    ue = W.cell_average(sub, W.isentropic_vortex(T_end), n=4)
    err = {"t_end": T_end, "mixed_vs_exact_rho_linf": float(np.abs(mx["u"][0, sample] - ue[0]).max())}
    if "fp64" in res:
        f = res["fp64"]
        err["fp64_vs_exact_rho_linf"] = float(np.abs(f["u"][0, sample] - ue[0]).max())
        err["mixed_vs_fp64_rel_linf"] = float(np.abs(mx["u"] - f["u"]).max() / np.abs(f["u"]).max())
        sol.set(mx["u"], T_end)
        err["teno_flips_fp32_vs_fp64"] = int(sol.count_flips())
        err["flip_unit"] = "cells x variables, final mixed state"

    nrec, msrec = mx["recon"]
    avg_ms = msrec / max(1, nrec)
    achieved = RECON_BYTES["mixed"] * N / (avg_ms * 1e-3) / 1e9
    nfl, msfl = mx["flux"]
    avg_fl = msfl / max(1, nfl)
    traffic = None
    if kernels_hash() == MEASURED_TRAFFIC["kernels_sha256_prefix"]:
        traffic = MEASURED_TRAFFIC["recon_mixed_bytes_per_cell"] * N
    out = {
        "metric": "cell-stage updates/s (mixed FP32 vs FP64) at stated error; serving p50/p99",
        "value": mx["value"],
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mx["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64 mixed",
        "data": "synthetic",
        "config": {"workload": f"isentropic vortex, {args.n}x{args.n} split/jittered periodic [0,10]^2 "
                               f"({N} cells), cubic CTENOZ lambda1'=1e4, SSP-RK3 CFL 0.3",
                   "cells": N, "scheme": "CTENOZ", "degree": 3, "precision": "mixed"},
        "error": err,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_reconstruct (FP32)", "bytes_per_cell": RECON_BYTES["mixed"],
                     "avg_launch_ms": avg_ms},
        "kernels": {"reconstruct_ms": avg_ms, "flux_rk_ms": avg_fl,
                    "flux_rk_GBs": FLUX_BYTES["mixed"] * N / (avg_fl * 1e-3) / 1e9,
                    # the stage's two kernels together, algorithmic bytes over their summed time
                    "recon_plus_flux_GBs": (RECON_BYTES["mixed"] + FLUX_BYTES["mixed"]) * N
                    / ((avg_ms + avg_fl) * 1e-3) / 1e9,
                    "recon_plus_flux_frac": (RECON_BYTES["mixed"] + FLUX_BYTES["mixed"]) * N
                    / ((avg_ms + avg_fl) * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "graph_replay": {"value": N * 3 * args.steps / mx["graph_elapsed"],
                         "ms_per_step": 1e3 * mx["graph_elapsed"] / args.steps,
                         "note": "same steps replayed from a captured HIP graph, no per-kernel events"},
    }
    if "fp64" in res:
        f = res["fp64"]
        n64, ms64 = f["recon"]
        a64 = ms64 / max(1, n64)
        nf64, msf64 = f["flux"]
        out["fp64"] = {"value": f["value"], "ms_per_step": 1e3 * f["elapsed"] / args.steps,
                       "graph_replay_value": N * 3 * args.steps / f["graph_elapsed"],
                       "reconstruct_ms": a64, "flux_rk_ms": msf64 / max(1, nf64),
                       "reconstruct_GBs": RECON_BYTES["fp64"] * N / (a64 * 1e-3) / 1e9}
        out["mixed_over_fp64"] = mx["value"] / f["value"]
    # plain device copy of a known size: practical HBM ceiling, and the
    # calibration kernel for the hardware byte counters
    nbytes = 4 << 30
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    ctx.copy(dst, src, nbytes)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.copy(dst, src, nbytes)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    out["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes, "GBs": 2 * nbytes / el / 1e9,
                               "kernel": "k_copy16"}
    del src, dst
    if not args.no_orders:
        out["orders_5_to_7"] = orders_bench(T, W, ctx)
    if not args.no_schemes:
        out["schemes"] = schemes_bench(T, W, ctx)
    if not args.no_variables:
        out["variables"] = variables_bench(T, W, ctx)
    if not args.no_dmr:
        out["dmr"] = dmr_bench(T, W, ctx)
    if not args.no_serving:
        out["serving"] = serving_bench(T, W, ctx, n_requests=args.serving_requests)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
