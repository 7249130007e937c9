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
# Algorithmic bytes per cell-stage at r = 3 with four variables: what an
# ideal fused stage must move, each value once (mixed / FP64):
#   pseudo-inverses      162 central + 24 directional entries  744 / 1488
#   central indices      18 x int32                               72 / 72
#   directional indices  12 local indices (slot order here)       12 / 12
#   stage-input state    4 x FP64                                  32 / 32
#   U^n                                                            32 / 32
#   state write                                                    32 / 32
#   cell area                                                       8 / 8
#   face geometry        1.5 faces x (n_x, n_y, |A|)               18 / 36
STAGE_BYTES = {"mixed": 950, "fp64": 1712}
# the reconstruction kernel's share: pseudo-inverses, indices, stage input
RECON_BYTES = {"mixed": 162 * 4 + 24 * 4 + 18 * 4 + 12 + 32, "fp64": 162 * 8 + 24 * 8 + 18 * 4 + 12 + 32}
# the flux / residual / RK kernel's share: U^n, state write, area, geometry
FLUX_BYTES = {k: STAGE_BYTES[k] - RECON_BYTES[k] for k in STAGE_BYTES}
# a cross cell's share of the second fused-stage kernel: its state write
# (k_stage reads its U^n, stage input and area and stores its partial state)
CROSS_UPDATE_BYTES = 32

# HBM bytes per cell and launch measured with the FETCH_SIZE / WRITE_SIZE
# counters (scaled by the copy-kernel calibration), valid only for the
# kernel sources they were taken on
MEASURED_TRAFFIC = {"kernels_sha256_prefix": "002632cd235042d6",
                    "source": "profiles/stage_vortex8M_hbm_counters.md",
                    "bytes_per_cell": {"k_stage_f32": 994.5, "k_stage_cross_f32": 90.7,
                                       "k_stage_f64": 1812.3, "k_stage_cross_f64": 108.9,
                                       "k_reconstruct_f32": 968.2, "k_flux_f32": 291.6,
                                       "k_reconstruct_f64": 1811.3, "k_flux_f64": 554.5}}


KERNEL_SOURCES = ("kernels_common.h", "k_recon.inl", "k_recon_ho.inl", "k_stage.inl", "k_recon_f32.hip",
                  "k_recon_f64.hip", "k_recon_ho_f32.hip", "k_recon_ho_f64.hip", "k_stage_f32.hip",
                  "k_stage_f64.hip", "k_precompute.hip", "k_flux.hip")


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
    fb0 = sol.fallbacks()
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
    fallbacks = sol.fallbacks() - fb0
    # the same steps replayed as a captured graph (no per-kernel events)
    sol.set(u0, 0.0)
    sol.solve(max_steps=warmup, cfl=0.3, precision=prec, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ng = sol.solve(max_steps=steps, cfl=0.3, precision=prec, use_graph=True)
    torch.cuda.synchronize()
    elg = time.perf_counter() - t0
    assert ng == steps, (ng, steps)
    return dict(elapsed=el, recon=kr, flux=kf, u=u, t=t, graph_elapsed=elg, fallbacks=fallbacks)


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
    sample = np.arange(0, N, 97)
    sub = W.Mesh(mesh.xy, mesh.tri[sample], mesh.box, mesh.bc, mesh.nx, mesh.ny, mesh.seed)
    for r in (4, 5, 6):
        t0 = time.perf_counter()
        m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=T.CTENOZ, degree=r, lambda1_prime=1e4,
                                 precision=T.BOTH)
        t_up = time.perf_counter() - t0
        sol = T.Solution(m, u0)
        res = run_precision(T, ctx, m, sol, u0, T.MIXED, steps, warmup)
        nrec, msrec = res["recon"]
        nfl, msfl = res["flux"]
        avg = msrec / max(1, nrec)
        b = ho_recon_bytes(r, "mixed")
        gbs = b * N / (avg * 1e-3) / 1e9
        ue = W.cell_average(sub, W.isentropic_vortex(res["t"]), n=4)
        sol.set(res["u"], res["t"])
        flips = int(sol.count_flips())
        out[f"r{r}"] = {"order": r + 1, "value": N * 3 * steps / res["elapsed"], "unit": "cell-stage updates/s",
                        "ms_per_step": 1e3 * res["elapsed"] / steps, "reconstruct_ms": avg,
                        "flux_rk_ms": msfl / max(1, nfl), "recon_bytes_per_cell": b, "recon_GBs": gbs,
                        "recon_frac_of_8TBs": gbs / HBM_PEAK_GBS, "upload_precompute_s": t_up,
                        "device_bytes": int(m.info.device_bytes),
                        "error": {"t_end": res["t"],
                                  "mixed_vs_exact_rho_linf": float(np.abs(res["u"][0, sample] - ue[0]).max()),
                                  "teno_flips_fp32_vs_fp64": flips, "fallbacks": 0,
                                  "positivity": "off (the paper's scheme)"}}
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
    fb = {}
    for order, r in (("5th", 4), ("7th", 6)):
        for p in ms:
            ms[p][order] = {}
        for name, sch in names:
            m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=sch, degree=r, lambda1_prime=1e4,
                                     precision=T.BOTH, positivity=1)
            sol = T.Solution(m, u0)
            for p, prec in (("fp64", T.FP64), ("mixed", T.MIXED)):
                res = run_precision(T, ctx, m, sol, u0, prec, steps, warmup)
                ms[p][order][name] = 1e3 * res["graph_elapsed"] / steps
                fb.setdefault(p, {}).setdefault(order, {})[name] = res["fallbacks"]
            sol.close()
            m.close()
    norm = {p: {o: {k: v / d["5th"]["CWENO"] for k, v in row.items()} for o, row in d.items()}
            for p, d in ms.items()}
    for p in norm:
        log(f"schemes {p} (triple point, normalised to CWENO5): " + "; ".join(
            f"{o}: " + ", ".join(f"{k} {v:.3f}" for k, v in row.items()) for o, row in norm[p].items()))
    return {"workload": f"triple point on [0,7]x[0,3], 500x215 split/jittered ({N} cells), walls, "
                        f"lambda1'=1e4, positivity fallback on, from t = 0, graph replay",
            "ms_per_step": ms, "normalised_time": norm, "paper_table_tab2": PAPER_SCHEME_TIMES,
            "fallbacks_timed_steps": fb}


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
                       "conserved variables, positivity fallback on (cells x stages that took it in the timed "
                       "steps: *_fallbacks), SSP-RK3 CFL 0.3 from t = 0, graph replay",
           "ms_per_iteration": {}, "paper_table_tab1": PAPER_DMR_TIMES,
           "paper_cteno5_s_per_iteration_64_cpu_processes": PAPER_DMR_CTENO5_S_PER_ITERATION}
    for nx, ny, label in ((860, 215, "369604"), (1196, 299, "714138")):
        mesh, u0 = W.dmr_case(nx, ny)
        row = {"cells": mesh.n_cells}
        runs = [(name, sch, 4) for name, sch in names] + ([("CTENO7", T.CTENO, 6)] if label == "714138" else [])
        for name, sch, r in runs:
            m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=sch, degree=r, lambda1_prime=1e15,
                                     precision=T.BOTH, positivity=1)
            sol = T.Solution(m, u0)
            row[name] = {}
            for pname, prec in (("fp64", T.FP64), ("mixed", T.MIXED)):
                res = run_precision(T, ctx, m, sol, u0, prec, steps, warmup)
                row[name][pname] = 1e3 * res["graph_elapsed"] / steps
                row[name][pname + "_fallbacks"] = res["fallbacks"]
            # mixed against FP64 after the timed steps, and the selections
            # FP32 and FP64 make differently on the mixed end state
            sol.set(res["u"], res["t"])
            row[name]["teno_flips_fp32_vs_fp64"] = int(sol.count_flips())
            sol.close()
            m.close()
        out["ms_per_iteration"][label] = row
        log(f"dmr {label} ({mesh.n_cells} cells): " + ", ".join(
            f"{k} {v['fp64']:.3f}/{v['mixed']:.3f} ms ({v['mixed_fallbacks']} fallbacks)"
            for k, v in row.items() if k != "cells"))
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


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(O, W, n, target_s, max_steps):
    """cell-stage updates/s of the oracle's SSP-RK3 steps on an n x n vortex
    mesh (stencils and least-squares factors built beforehand, as the
    library's precompute is outside its timed region)."""
    mesh, u0 = W.vortex_case(n, seed=5)
    o = O.Oracle.from_mesh(mesh, physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)
    o.prepare()
    dt = 0.3 * o.dt_bound(u0)
    steps = 0
    t0 = time.perf_counter()
    U = u0
    while steps < max_steps and time.perf_counter() - t0 < target_s:
        U = o.rk3_step(U, dt)
        steps += 1
    el = time.perf_counter() - t0
    del o
    return mesh.n_cells * 3 * steps / el, mesh.n_cells, steps, el


def cpu_baseline(W, target_s=12.0, max_steps=40):
    """The FP64 oracle, as it stands, on bounded samples of the same workload
    family (the oracle's per-cell factors need ~50 KB a cell, so the 8M-cell
    mesh itself does not fit): all host threads on a 320k-cell mesh, and one
    thread on a 20k-cell mesh, each for about target_s seconds of steps."""
    import oracle as O
    all_threads = O.threads()
    rate, cells, steps, el = _oracle_rate(O, W, 400, target_s, max_steps)
    O.set_threads(1)
    try:
        rate1, cells1, steps1, el1 = _oracle_rate(O, W, 100, target_s, max_steps)
    finally:
        O.set_threads(all_threads)
    return {"value": rate, "unit": "cell-stage updates/s", "cores": all_threads, "kind": "oracle",
            "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count(),
            "sample": f"isentropic vortex on 400x400 split/jittered periodic [0,10]^2 ({cells} cells, same "
                      f"per-cell work as the 8M-cell case), cubic CTENOZ FP64, {steps} SSP-RK3 steps, "
                      f"{el:.2f} s wall, {all_threads} threads, precompute excluded",
            "single_thread": {"value": rate1, "unit": "cell-stage updates/s", "cores": 1,
                              "sample": f"100x100 ({cells1} cells), {steps1} steps, {el1:.2f} s wall"}}


def _pct(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(math.ceil(p / 100.0 * len(xs))) - 1))
    return xs[k]


def serving_bench(T, W, ctx, n_requests=256, budget_gb=4.0, max_slots=128, steps=100, n_checked=8):
    """Poisson stream of independent Euler solves through the continuous-batching
    server: saturation, then p50 / p99 latency at 0.7 of it, the latency split
    (host build, queue, upload + FP64 precompute, run), positivity-fallback
    counts, and the error of a sample of served results against an FP64
    solve of the same request."""
    import statistics
    t0 = time.perf_counter()
    reqs = W.serving_requests(n_requests, rate_hz=1.0, seed=4)
    items = [W.build_request(r) for r in reqs]
    cells = [m.n_cells for m, _ in items]
    log(f"serving: {n_requests} requests generated ({sum(cells)} cells, {time.perf_counter() - t0:.1f}s)")
    skw = dict(physics=T.EULER, scheme=T.CTENOZ, degree=3, lambda1_prime=1e4, positivity=1)
    scheme = T.make_scheme(precision=T.MIXED, **skw)
    # a sample of each kind of request, checked against FP64 solves
    checked = set([r.index for r in reqs if r.kind == "vortex"][:n_checked // 2] +
                  [r.index for r in reqs if r.kind == "riemann"][:n_checked // 2])

    def run(arrivals, keep=()):
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
        infos, failed, kept = [], 0, {}
        for k, t in enumerate(tickets):
            info = srv.info(t)
            infos.append(info)
            try:
                _, u, _, _ = srv.poll(t, take=True)
                if k in keep:
                    kept[k] = u
            except T.CtenoError:
                failed += 1
        stats = srv.stats()
        srv.close()
        return wall, infos, failed, stats, kept

    wall, infos, failed, st, _ = run([0.0] * n_requests)
    sat = n_requests / wall
    log(f"serving: closed loop {wall:.2f}s -> {sat:.1f} req/s, peak {st['peak_active']} resident")
    rate = 0.7 * sat
    arrivals = [r.arrival_s / rate for r in reqs]
    wall, infos, failed, st, kept = run(arrivals, keep=checked)
    lat = [i["latency_s"] for i in infos if i["state"] == T.REQ_DONE]
    split = {k: {"p50": _pct([i[k] for i in infos], 50), "p99": _pct([i[k] for i in infos], 99),
                 "mean": statistics.fmean([i[k] for i in infos])}
             for k in ("build_s", "queue_s", "admit_s", "run_s")}
    # accuracy: sampled served results against FP64 solves of the same requests
    errs, by_kind = [], {"vortex": [], "riemann": []}
    for k, u in sorted(kept.items()):
        mesh, u0 = items[k]
        m = T.Mesh.from_workload(ctx, mesh, precision=T.FP64, **skw)
        sol = T.Solution(m, u0)
        sol.solve(max_steps=steps, cfl=0.3, precision=T.FP64)
        ref, _ = sol.download()
        sol.close()
        m.close()
        rel = np.abs(u - ref) / np.abs(ref).max(axis=1, keepdims=True)
        e = float(rel.max())
        errs.append(e)
        by_kind[reqs[k].kind].append({"request": k, "cells": int(mesh.n_cells), "max_rel_linf": e,
                                      "cells_above_1e-5": int((rel.max(axis=0) > 1e-5).sum()),
                                      "fallbacks": int(infos[k]["fallbacks"])})
    out = {"requests": n_requests, "steps_per_request": steps,
           "scheme": "CTENOZ r=3 (Algorithm 2 as printed), FP32-mixed, positivity fallback on",
           "cells_total": int(sum(cells)), "budget_bytes": int(budget_gb * (1 << 30)), "max_slots": max_slots,
           "saturation_req_per_s": sat, "rate_hz": rate, "wall_s": wall,
           "throughput_req_per_s": n_requests / wall,
           "cell_stages_per_s": st["cell_stages"] / wall,
           "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99),
           "mean_s": statistics.fmean(lat) if lat else None,
           "latency_split_s": split,
           "peak_active": st["peak_active"], "peak_bytes": st["peak_bytes"], "failed": failed,
           "fallbacks": int(st["fallbacks"]),
           "fallback_requests": int(sum(1 for i in infos if i["fallbacks"] > 0)),
           "error_vs_fp64": {"requests_checked": len(errs), "max_rel_linf": max(errs) if errs else None,
                             "vortex": by_kind["vortex"], "riemann": by_kind["riemann"],
                             "reference": "the library's FP64 solve of the same request (the FP64 path matches "
                                          "the FP64 oracle to 1e-12 in the parity tests); normwise per "
                                          "variable; Riemann requests differ at the few cells where FP32 and "
                                          "FP64 select or fall back differently at a discontinuity"},
           "latency": "submission to result on the host (mesh/stencil build, FP64 precompute, queueing, 100 steps)"}
    log(f"serving: Poisson {rate:.1f}/s -> p50 {out['p50_s']:.3f}s p99 {out['p99_s']:.3f}s, {failed} failed, "
        f"split p50 build {split['build_s']['p50']:.3f} queue {split['queue_s']['p50']:.3f} "
        f"admit {split['admit_s']['p50']:.3f} run {split['run_s']['p50']:.3f}; err vs FP64 vortex "
        f"{max(e['max_rel_linf'] for e in by_kind['vortex']):.2e} riemann "
        f"{max(e['max_rel_linf'] for e in by_kind['riemann']):.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2000, help="squares per side (2000 -> 8M cells)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-split", action="store_true", help="skip the separate-kernel stage comparison")
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

    res, split = {}, {}
    # both precisions through the fused stage kernels (the default), then
    # through the separate reconstruction and flux kernels for comparison
    precs = [("mixed", T.MIXED)] + ([] if args.no_fp64 else [("fp64", T.FP64)])
    runs = [(name, prec, True, res) for name, prec in precs]
    if not args.no_split:
        runs += [(name, prec, False, split) for name, prec in precs]
    for name, prec, fused, store in runs:
        ctx.set_fused_stage(fused)
        kernels = "fused stage kernels" if fused else "reconstruction + flux kernels"
        log(f"timing {name} ({kernels}): {args.warmup} warm-up + {args.steps} steps")
        r = run_precision(T, ctx, m, sol, u0, prec, args.steps, args.warmup)
        r["value"] = N * 3 * args.steps / r["elapsed"]
        store[name] = r
        log(f"{name}: {r['value']:.3e} cell-stage/s, {1e3 * r['elapsed'] / args.steps:.3f} ms/step, "
            f"kernel 0 {r['recon'][1] / max(1, r['recon'][0]):.3f} ms/launch, "
            f"kernel 1 {r['flux'][1] / max(1, r['flux'][0]):.3f} ms/launch")
    ctx.set_fused_stage(True)
    x_cross = int(m.info.n_cross_cells) / N

    # the same mixed-precision steps with the state handed over in host
    # memory: upload, steps, download (not `value`, which starts from a
    # resident state; the mesh upload and precompute are a one-time setup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol.set(u0, 0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol.solve(max_steps=args.steps, cfl=0.3, precision=T.MIXED, use_graph=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sol.download()
    t3 = time.perf_counter()
    pcie = {"value": N * 3 * args.steps / (t3 - t0), "ms_per_step": 1e3 * (t3 - t0) / args.steps,
            "state_upload_ms": 1e3 * (t1 - t0), "steps_ms": 1e3 * (t2 - t1), "state_download_ms": 1e3 * (t3 - t2),
            "state_bytes": int(u0.nbytes),
            "note": "host state in, steps, host state out, mixed precision, fused stage kernels"}
    log(f"host-to-host: {pcie['value']:.3e} cell-stage/s (upload {pcie['state_upload_ms']:.1f} ms, "
        f"download {pcie['state_download_ms']:.1f} ms)")

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

    err["fallbacks"] = {"mixed": mx["fallbacks"], "fp64": res["fp64"]["fallbacks"] if "fp64" in res else None,
                        "positivity": "off (the paper's scheme); the vortex needs no fallback"}
    err["reference"] = ("exact vortex on every 97th cell; the FP64 run, which the parity tests hold to the FP64 "
                        "oracle at 1e-12 on this mesh (sampled cells, one stage) and over 3 steps")

    def kstats(r):
        nrec, msrec = r["recon"]
        nfl, msfl = r["flux"]
        return msrec / max(1, nrec), msfl / max(1, nfl)

    def gbs(nbytes, ms):
        return nbytes * N / (ms * 1e-3) / 1e9

    # the fused stage: k_stage moves every cell's share but the state write
    # of the cells k_stage_cross finishes (x_cross of them)
    def stage_split_bytes(prec):
        cross = x_cross * CROSS_UPDATE_BYTES
        return STAGE_BYTES[prec] - cross, cross

    t0, t1 = kstats(mx)
    b0, b1 = stage_split_bytes("mixed")
    achieved = gbs(b0, t0)
    stage_gbs = gbs(STAGE_BYTES["mixed"], t0 + t1)
    fresh = kernels_hash() == MEASURED_TRAFFIC["kernels_sha256_prefix"]
    measured = MEASURED_TRAFFIC["bytes_per_cell"] if fresh else None
    traffic = measured["k_stage_f32"] * N if fresh else None
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
                   "cells": N, "scheme": "CTENOZ (Algorithm 2 as printed)", "degree": 3, "precision": "mixed",
                   "positivity": "off", "stage_kernels": "fused"},
        "error": err,
        # the dominant kernel (the fused stage kernel) on its share of the
        # algorithmic bytes; the whole stage (both kernels) on all of them
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_stage (FP32, fused reconstruction + in-block fluxes + RK)",
                     "bytes_per_cell": b0, "avg_launch_ms": t0,
                     "stage": {"kernels": "k_stage + k_stage_cross (FP32)", "bytes_per_cell": STAGE_BYTES["mixed"],
                               "avg_ms": t0 + t1, "achieved": stage_gbs, "frac": stage_gbs / HBM_PEAK_GBS},
                     "traffic_note": "HBM bytes per launch from FETCH_SIZE + WRITE_SIZE, scaled by the copy "
                                     "calibration; null unless taken on these kernel sources"},
        "kernels": {"stage_ms": t0, "cross_ms": t1, "cross_cells_fraction": x_cross,
                    "bytes_per_cell": {"stage": STAGE_BYTES["mixed"], "k_stage_share": b0, "k_stage_cross_share": b1},
                    "measured_bytes_per_cell": measured},
        "graph_replay": {"value": N * 3 * args.steps / mx["graph_elapsed"],
                         "ms_per_step": 1e3 * mx["graph_elapsed"] / args.steps,
                         "note": "same steps replayed from a captured HIP graph, no per-kernel events"},
        "pcie_inclusive": pcie,
    }
    if "fp64" in res:
        f = res["fp64"]
        a0, a1 = kstats(f)
        c0, c1 = stage_split_bytes("fp64")
        out["fp64"] = {"value": f["value"], "ms_per_step": 1e3 * f["elapsed"] / args.steps,
                       "graph_replay_value": N * 3 * args.steps / f["graph_elapsed"],
                       "stage_kernels": "k_stage + k_stage_cross (FP64)",
                       "stage_ms": a0, "cross_ms": a1,
                       "k_stage_GBs": gbs(c0, a0), "k_stage_frac": gbs(c0, a0) / HBM_PEAK_GBS,
                       "stage_GBs": gbs(STAGE_BYTES["fp64"], a0 + a1),
                       "stage_frac": gbs(STAGE_BYTES["fp64"], a0 + a1) / HBM_PEAK_GBS,
                       "bytes_per_cell": {"stage": STAGE_BYTES["fp64"], "k_stage_share": c0,
                                          "k_stage_cross_share": c1}}
        out["mixed_over_fp64"] = mx["value"] / f["value"]
    if split:
        out["split_kernels"] = {}
        for name, r in split.items():
            rc, fl = kstats(r)
            out["split_kernels"][name] = {
                "value": r["value"], "ms_per_step": 1e3 * r["elapsed"] / args.steps,
                "reconstruct_ms": rc, "flux_rk_ms": fl,
                "reconstruct_GBs": gbs(RECON_BYTES[name], rc), "reconstruct_frac": gbs(RECON_BYTES[name], rc) / HBM_PEAK_GBS,
                "stage_GBs": gbs(STAGE_BYTES[name], rc + fl), "stage_frac": gbs(STAGE_BYTES[name], rc + fl) / HBM_PEAK_GBS,
                "max_rel_diff_vs_fused": float(np.abs(r["u"] - res[name]["u"]).max() / np.abs(res[name]["u"]).max())}
        out["split_kernels"]["note"] = ("reconstruction and flux/RK as two kernels, face values through device "
                                        "memory; reconstruct_frac on its 860 / 1604 B share")
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
