#!/usr/bin/env python3
"""Benchmark of the delayed-assembly multigrid hot path on one MI355X.

Workload (headline): 3D unit cube, 512^3 trilinear Q1 cells (133,432,831
interior DoF, 27-point stencils), eps = 1 with 512 seeded random boxes of eps
log-uniform in [1e-4, 1e4] (painter's order), load of u = prod sin(pi x_m).
One step = one complete solve to a 1e-8 relative residual of the mixed form
with lazy assembly: V-cycles start on the centre-sample operator while the
ladder s = 2, 4, 8, 16 runs on a second stream (bf16 hi+lo MFMA integration),
the surplus store picks FP8 / FP16 / FP32 per 64-vertex tile by the size of
the deviation from the centre-sample stencil (tolerance 1e-6 of the local
stencil magnitude), FP32 BoxMG V(2,2), FP64 outer conjugate gradients.  The
same material is solved beside it with the mixed form assembled up front,
with the lazy schedule that waits for the final operator instead of cycling
on provisional ones, and with the plain FP64 form assembled up front.  Inputs
(load vector, material data) are resident in HBM before timing.

Components: the same comparison on the 2D 1024^2 balls workload and on the
3D 256^3 Gaussian-field workload, cell integrations per second by s, the
serving replay (2048 requests), the roofline of the mixed finest-level
sweep at 512^3, the additive adaFAC-PI / adaFAC-Jac cycles against V(2,2)
on a 3D 256^3 sine material, and the paper's own ladder and byte format
(memory-footprint table) on a 2D 243^2 grid.

Prints one JSON line.  `value` is the mixed-lazy form's fine-grid V-cycle
throughput over the whole solve: (n-1)^3 DoF x V-cycles / time-to-solution.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell integrations/s, V-cycle DoF/s, time-to-1e-8 residual: mixed vs FP64"
HBM_PEAK_GBS = 8000.0
WORKLOAD = ("3D 512^3 Q1 cells (27-point stencils), eps=1 + 512 seeded boxes (sides 1/64-1/8) of eps "
            "log-uniform in [1e-4,1e4], load of u=prod sin(pi x) for eps=1 (not the solution here), lazy ladder s=2..16 (C=1%), "
            "FP8/FP16/FP32 surplus tiers (tau 1e-6 of the local stencil), BoxMG V(2,2) omega=0.6 + FP64 "
            "outer CG to 1e-8; mixed-lazy vs FP64-up-front")
TIERS_C5 = dict(min_tier=1, max_tier=3, tau_abs=0.0, tau_rel=1e-6)
TIERS_FP16 = dict(min_tier=2, max_tier=2, tau_abs=0.0, tau_rel=1e-7)
FORMS = ("mixed_lazy", "mixed_lazy_guarded", "mixed_lazy_parked", "mixed_upfront", "fp64_upfront")
# the roofline kernel: one damped-Jacobi sweep of the 3D mixed finest level
# as the solve runs it (four vertices per thread; items whose coupling
# sources are all tier-0 tiles re-evaluate their couplings from the centre
# samples, the others read the store's FP32 decode); its traffic record
# (counter runs of `bench.py --kernels-only`) is valid only for the source it
# was taken on
SWEEP_KERNEL = "k_sweep3x4h<0>"
KERNEL_SOURCES = ("paper_2005_03606_amd/csrc/cycle.hip", "paper_2005_03606_amd/csrc/common.h")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "sweep3x4h_boxes512_traffic.md")
# half-stencil offsets of a 27-point stencil (the 13 upper neighbours)
HALF3 = [((i % 3) - 1, (i // 3) % 3 - 1, i // 9 - 1) for i in range(14, 27)]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="cells per axis of the headline workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=20, help="grid of the oracle's sample of the same material")
    ap.add_argument("--sweeps", type=int, default=40, help="timed launches of the roofline kernel")
    ap.add_argument("--serve-requests", type=int, default=2048,
                    help="requests in the serving replay (0 skips it)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--n2d", type=int, default=1024, help="2D balls component (0 skips)")
    ap.add_argument("--n3d", type=int, default=256, help="3D Gaussian-field component (0 skips)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the roofline sweep and a calibration copy (for counter runs)")
    ap.add_argument("--solve-only", action="store_true",
                    help="only one mixed up-front solve of the headline workload and a calibration copy "
                         "(for counter runs over a whole cycle)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ solves
def solve_forms(P, W, d, n, fld, tiers, steps, warmup, s_max=16, main=None):
    """Time-to-1e-8 at n^d cells of
    - mixed_lazy: the paper's schedule, cycling on the provisional operator
      while the ladder runs on the assembly stream (the iterate carried over
      at the publish);
    - mixed_lazy_guarded: the same schedule with the growth guard 2 (cycles
      on a provisional operator stop once they have doubled the residual);
    - mixed_lazy_parked: the same lazy assembly with the provisional target
      1 (no cycles on a provisional operator: the assembly has the GPU);
    - mixed_upfront and fp64_upfront: every cell's ladder first.
    One context (device-resident solve state) at a time; `main` gets
    `steps` timed solves after `warmup`, the others 1 + 2."""
    import torch
    eps = P.Eps(fld)
    f_host = W.load_sine(d, n)
    f = torch.from_numpy(f_host).cuda()
    base = dict(transfer=P.BOXMG, outer=P.PCG, s_max=s_max, tol=1e-8, max_cycles=600)
    kws = {"mixed_lazy": dict(base, precision=P.MIXED, schedule=P.LAZY, **tiers),
           "mixed_lazy_guarded": dict(base, precision=P.MIXED, schedule=P.LAZY, prov_growth=2.0, **tiers),
           "mixed_lazy_parked": dict(base, precision=P.MIXED, schedule=P.LAZY, prov_tol=1.0, **tiers),
           "mixed_upfront": dict(base, precision=P.MIXED, schedule=P.UPFRONT, **tiers),
           "fp64_upfront": dict(base, precision=P.FP64, schedule=P.UPFRONT)}
    out = {"ms": {}, "rep": {}, "all_ms": {}}
    sol = {}
    for k in FORMS:
        ctx = P.Context(0)
        w, s = (warmup, steps) if k == main else (1, 2)
        for _ in range(w):
            P.solve(ctx, d, n, eps, f, torch.zeros_like(f), **kws[k])
        torch.cuda.synchronize()
        reps, times = [], []
        t0 = time.perf_counter()
        for _ in range(s):
            t1 = time.perf_counter()
            u, r = P.solve(ctx, d, n, eps, f, torch.zeros_like(f), **kws[k])
            times.append((time.perf_counter() - t1) * 1e3)
            reps.append(r)
        torch.cuda.synchronize()
        out["ms"][k] = (time.perf_counter() - t0) / s * 1e3
        out["all_ms"][k] = times
        assert all(r["status"] == 0 for r in reps), (k, [r["status"] for r in reps])
        out["rep"][k] = reps[-1]
        sol[k] = u
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
        log(f"{d}D {n}: {k} {out['ms'][k]:.1f} ms, {reps[-1]['cycles']} cycles")
    uf = sol["fp64_upfront"]
    out["err"] = {k: float(torch.linalg.norm(sol[k] - uf) / torch.linalg.norm(uf)) for k in FORMS[:-1]}
    out["f_host"] = f_host
    return out


def forms_summary(b, n, d):
    """Times, cycles and speedups over FP64 up front of every form."""
    ms, rep = b["ms"], b["rep"]
    o = {}
    for k in FORMS:
        o[f"time_to_1e8_{k}_ms"] = round(ms[k], 3)
        o[f"cycles_{k}"] = rep[k]["cycles"]
        o[f"true_final_residual_{k}"] = rep[k]["r_final"] / rep[k]["r0"]
    for k in FORMS[:-1]:
        o[f"speedup_{k}_vs_fp64_upfront"] = round(ms["fp64_upfront"] / ms[k], 3)
        o[f"solution_rel_err_vs_fp64_{k}"] = b["err"][k]
    for k in ("mixed_lazy", "mixed_upfront", "fp64_upfront"):
        o[f"t_first_cycle_ms_{k}"] = round(rep[k]["t_first_cycle_ms"], 3)
    o["vcycle_dof_per_s_fp64_upfront"] = (n - 1) ** d * rep["fp64_upfront"]["cycles"] / (ms["fp64_upfront"] / 1e3)
    m = rep["mixed_upfront"]
    o["cells_at_s_1_2_4_8_16"] = m["cells_at_s"]
    o["store_tier_tiles_0_fp8_fp16_fp32"] = m["tier_tiles"]
    o["store_bytes_per_stencil_mixed"] = m["store_bytes"] / (n + 1) ** d
    o["store_bytes_per_stencil_fp64"] = rep["fp64_upfront"]["store_bytes"] / (n + 1) ** d
    return o


# --------------------------------------------------------------- roofline
def ladder_operator(P, ctx, d, n, eps, s_max=16, C_thr=0.01):
    """The final element matrices of the adaptive ladder as the solver's
    mixed form computes them (same kernels, same criterion), cell lists
    compacted on the device between rungs."""
    import torch
    K, _, _ = P.assemble_cells(ctx, d, n, 1, eps, P.MIXED)
    cells = None
    s = 2
    while s <= s_max:
        Kold = K if cells is None else K[cells]
        Kn, _, done = P.assemble_cells(ctx, d, n, s, eps, P.MIXED, cells=cells, K_old=Kold, C_thr=C_thr)
        if cells is None:
            K = Kn
            cells = torch.nonzero(done == 0).flatten()
        else:
            K[cells] = Kn
            cells = cells[done == 0]
        if cells.numel() == 0:
            break
        s *= 2
    return K


def source_sha16():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(n):
    """HBM bytes per launch of the roofline kernel from the committed counter
    record, if it was taken on this source and size; else None."""
    try:
        text = open(TRAFFIC_RECORD).read()
    except OSError:
        return None
    m = re.search(r"traffic-record: n=(\d+) bytes_per_launch=(\d+) source_sha16=([0-9a-f]{16})", text)
    if not m or int(m.group(1)) != n or m.group(3) != source_sha16():
        return None
    return int(m.group(2))


def tier0_items(tier, n):
    """Items of four finest-level vertices (x0 = 1 + 4c on interior rows)
    whose coupling sources all lie in tier-0 tiles (own couplings: the tiles
    of v and v + 3; mirrored ones: those of v - o and v - o + 3 for every half
    slot o), i.e. the items whose couplings the default 3D sweep re-evaluates
    from the centre samples.  Counted on the device from the exported tile
    tiers, 32 planes at a time."""
    import torch
    nv, T = n + 1, n // 4
    t0 = tier == 0
    dev = tier.device
    c = torch.arange(T, device=dev, dtype=torch.int64)
    y = torch.arange(1, n, device=dev, dtype=torch.int64)
    row = (1 + 4 * c)[None, :] + nv * y[:, None]
    count = 0
    for z0 in range(1, n, 32):
        z = torch.arange(z0, min(z0 + 32, n), device=dev, dtype=torch.int64)
        v = row[None] + nv * nv * z[:, None, None]
        ok = t0[v >> 6] & t0[(v + 3) >> 6]
        for ox, oy, oz in HALF3:
            w = v - (ox + oy * nv + oz * nv * nv)
            ok &= t0[w >> 6] & t0[(w + 3) >> 6]
        count += int(ok.sum())
    return count


def sweep_roofline(P, W, n, sweeps):
    """One damped-Jacobi sweep of the mixed finest level of the headline
    workload (3D 512^3 boxes, the final operator of the adaptive ladder), the
    kernel that moves most of the mixed cycle's bytes, with the solve's
    operator source and launch shape: four vertices per thread; an item whose
    coupling sources all lie in tier-0 tiles re-evaluates its couplings from
    its 5 x 2 x 2 cells' centre samples, every other item reads the store's
    FP32 decode.  Timed with HIP events on the stream the kernels run on.

    Algorithmic bytes per launch: FP32 u in, f in, u out (12 B per vertex),
    the 13 FP32 couplings of the half stencil and their mirrored ones for
    every vertex of a decode-reading item (208 B per item: each slot read as
    its own vertex's and as its neighbour's), each tier-0 item's cells once
    (16 B: four cells per item), and the item flags (1 B per item).
    `decode_form_frac` prices the same time at the 64 B per vertex of a sweep
    that reads the decode everywhere (the work this pass replaces);
    `store_form_frac` at the compressed store's own bytes (payload + tier byte
    and offset per 64-vertex tile + FP32 centre sample per cell), the least
    any sweep of this operator must read."""
    import torch
    d = 3
    ctx = P.Context(0)
    eps = P.Eps(W.config_field(4))
    K = ladder_operator(P, ctx, d, n, eps)
    S32 = P.gather_stencils(ctx, d, n, K, P.MIXED, P.MIXED)
    del K
    eps_c = P.centre_samples(ctx, d, n, eps)
    h = P.Hierarchy(ctx, d, n, precision=P.MIXED, transfer=P.BOXMG)
    h.compress(S32, eps_c, **TIERS_C5)
    del S32
    torch.cuda.empty_cache()
    ntile, payload, tier_tiles = h.store_info()
    tier = h.store_export()[0]
    NV = (n + 1) ** d
    items, items_inner = (n // 4) * (n + 1) ** 2, (n // 4) * (n - 1) ** 2
    t0 = tier0_items(tier, n)
    del tier
    t0_lib = h.tier0_items()[1]  # the library's own count (equal by construction)
    pass_bytes = 12 * NV + 208 * (items_inner - t0) + 16 * t0 + items
    decode_pass_bytes = 64 * NV
    store_pass_bytes = payload + 5 * ntile + 4 * n ** d + 12 * NV
    inner = torch.from_numpy(W.interior_mask(d, n)).cuda()
    f32 = inner.to(torch.float32)
    u32 = torch.zeros_like(f32)
    st = torch.cuda.current_stream()
    h.smooth(0, u32, f32, sweeps=2)
    torch.cuda.synchronize()
    calls = max(sweeps // 2, 1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(st)
    for _ in range(calls):
        h.smooth(0, u32, f32, sweeps=2)  # two launches, ping-pong through the level's spare vector
    ev[1].record(st)
    torch.cuda.synchronize()
    avg_ms = ev[0].elapsed_time(ev[1]) / (2 * calls)
    h.close()
    ctx.close()
    torch.cuda.empty_cache()
    achieved = pass_bytes / (avg_ms / 1e3) / 1e9
    frac = lambda b: round(b / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(n),
            "kernel": SWEEP_KERNEL, "bytes_per_launch": int(pass_bytes),
            "bytes_per_dof": round(pass_bytes / NV, 2), "tier0_items": t0, "tier0_items_library": t0_lib,
            "items": items_inner,
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches_timed": 2 * calls,
            "decode_form_bytes_per_launch": int(decode_pass_bytes), "decode_form_frac": frac(decode_pass_bytes),
            "store_form_bytes_per_launch": int(store_pass_bytes), "store_form_frac": frac(store_pass_bytes),
            "store_tiers_0_fp8_fp16_fp32": tier_tiles,
            "workload": f"finest level of the headline workload ({n}^3 cells), final ladder operator"}


def integration_rates(P, W, ctx, n3=512, ncells=1 << 20):
    """Cell integrations per second by s on the headline material: the first
    `ncells` cells of the 512^3 grid (a slab through the boxes), every s of
    the ladder, bf16 hi+lo MFMA and FP64."""
    import torch
    eps = P.Eps(W.config_field(4))
    cells = torch.arange(ncells, dtype=torch.int64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {}
    for mode, name in ((P.MIXED, "mixed_bf16_mfma"), (P.FP64, "fp64")):
        rates = {}
        for s in (2, 4, 8, 16):
            P.assemble_cells(ctx, 3, n3, s, eps, mode, cells=cells)
            ev[0].record()
            reps = 2
            for _ in range(reps):
                P.assemble_cells(ctx, 3, n3, s, eps, mode, cells=cells)
            ev[1].record()
            torch.cuda.synchronize()
            rates[f"s{s}"] = round(ncells * reps / (ev[0].elapsed_time(ev[1]) / 1e3), 1)
        out[name] = rates
    out["sample"] = f"first {ncells} cells of the {n3}^3 boxes grid, every cell at that s"
    return out


def kernels_only(args):
    """Counter runs: the roofline sweep at the workload size, a plain device
    copy of known size (calibration of the traffic counters), then one bf16
    hi+lo MFMA integration launch per s = 4, 8, 16 over the first 2^20 cells
    of the headline grid (matrix-core counters)."""
    import torch
    import paper_2005_03606_amd as P
    import workload as W
    r = sweep_roofline(P, W, args.n, args.sweeps)
    nbytes = 2 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    ctx = P.Context(0)
    eps = P.Eps(W.config_field(4))
    ncells = 1 << 20
    cells = torch.arange(ncells, dtype=torch.int64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    mfma = {}
    for s in (4, 8, 16):
        ev[0].record()
        P.assemble_cells(ctx, 3, args.n, s, eps, P.MIXED, cells=cells)
        ev[1].record()
        torch.cuda.synchronize()
        mfma[f"s{s}_ms"] = round(ev[0].elapsed_time(ev[1]), 3)
    ctx.close()
    print(json.dumps({"sweep": r, "copy_bytes_each_way": nbytes, "copies": 4, "mfma_launches": mfma,
                      "mfma_cells": ncells, "source_sha16": source_sha16()}), flush=True)


def solve_only(args):
    """Counter runs over whole cycles: one mixed up-front solve of the
    headline workload (the solve's own kernels, every level), then four
    2 GiB device copies for the calibration of the traffic counters."""
    import torch
    import paper_2005_03606_amd as P
    import workload as W
    d, n = 3, args.n
    ctx = P.Context(0)
    f = torch.from_numpy(W.load_sine(d, n)).cuda()
    u, r = P.solve(ctx, d, n, P.Eps(W.config_field(4)), f, torch.zeros_like(f), transfer=P.BOXMG, outer=P.PCG,
                   s_max=16, tol=1e-8, max_cycles=600, precision=P.MIXED, schedule=P.UPFRONT, **TIERS_C5)
    ctx.close()
    del u, f
    torch.cuda.empty_cache()
    nbytes = 2 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"solve_status": r["status"], "cycles": r["cycles"], "copy_bytes_each_way": nbytes, "copies": 4,
                      "source_sha16": source_sha16()}), flush=True)


# --------------------------------------------------------------- adaFAC
def adafac_component(P, W, ctx, n=256, tol=1e-8):
    """The additive adaFAC-PI / adaFAC-Jac corrections against the
    multiplicative V(2,2) one, each inside the stationary FP64 outer
    iteration, 3D n^3 sine material (eps = 1 + 0.9 sin 2 pi x sin 2 pi y
    sin 2 pi z), BoxMG transfers, s = 4 up front: time to tol and cycles, in
    the FP64 and the mixed form (FP16 surplus store)."""
    import torch
    d = 3
    eps = P.Eps(W.sine_field(d, 0.9))
    f = torch.from_numpy(W.load_sine(d, n)).cuda()
    out = {"workload": f"3D {n}^3 sine material, s = 4 up front, BoxMG, stationary outer iteration to {tol}"}
    for prec, pname in ((P.FP64, "fp64"), (P.MIXED, "mixed")):
        for cyc, cname in ((P.CYCLE_V, "vcycle"), (P.CYCLE_ADAFAC_PI, "adafac_pi"), (P.CYCLE_ADAFAC_JAC, "adafac_jac")):
            kw = dict(precision=prec, transfer=P.BOXMG, outer=P.STATIONARY, s_fixed=4, tol=tol, max_cycles=400,
                      cycle=cyc, **TIERS_FP16)
            P.solve(ctx, d, n, eps, f, torch.zeros_like(f), **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, rep = P.solve(ctx, d, n, eps, f, torch.zeros_like(f), **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            out[f"{pname}_{cname}"] = {"ms": round(ms, 2), "cycles": rep["cycles"], "status": rep["status"],
                                       "ms_per_cycle": round(rep["t_cycles_ms"] / max(rep["cycles"], 1), 3)}
    return out


# ------------------------------------------------------------ paper mode
def paper_mode_table(P, W, ctx, n=243, cycles=10, C_thr=0.01, tau=1e-8):
    """Table memory-footprint (Sec. 6.3) in the paper's own mode on the GPU:
    the n -> n + 1 ladder keeping the older matrix, p3-byte surplus format,
    theta = 1 / 16 / 64 on a 2D grid of h = 1/n; per cycle (max n, mean n,
    compression) and the time of the whole table (ladder steps + encoding)."""
    import numpy as np
    import torch
    d = 2
    out = {"grid": f"2D {n}^2 cells (h = 1/{n}), C = {C_thr}, tau = {tau}, {cycles} cycles"}
    nn = (1 << d) ** 2
    for theta in (1.0, 16.0, 64.0):
        eps = P.Eps(W.theta_field(d, theta))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K1, _, _ = P.assemble_cells(ctx, d, n, 1, eps, P.FP64)
        K = K1.clone()
        ncell = n ** d
        nfin = torch.ones(ncell, dtype=torch.int64, device="cuda")
        cells = torch.arange(ncell, dtype=torch.int64, device="cuda")
        rows = []
        for k in range(1, cycles + 1):
            if k >= 2 and cells.numel():
                _, done = P.ladder_step_keep(ctx, d, n, k, eps, K, cells=cells, C_thr=C_thr)
                cells = cells[done == 0]
                nfin[cells] = k
            p3, _ = P.p3_encode(ctx, d, K, K1, tau)
            nb = int((1 + nn * p3.to(torch.int64)).sum())
            rows.append([int(nfin.max()), round(float(nfin.double().mean()), 4), round(ncell * nn * 8.0 / nb, 2)])
        torch.cuda.synchronize()
        out[f"theta_{int(theta)}"] = {"rows_max_n_mean_n_compression": rows,
                                      "ms": round((time.perf_counter() - t0) * 1e3, 2)}
    return out


# ---------------------------------------------------------------- serving
def serving_bench(P, W, count, slots):
    """Serving replay: mixed 2D/3D requests with Gaussian-field materials,
    Poisson arrivals at 0.8x the measured single-stream capacity."""
    import numpy as np
    import torch
    from paper_2005_03606_amd import serving

    opts = dict(precision=P.MIXED, schedule=P.LAZY, transfer=P.BOXMG, outer=P.PCG, s_max=16, tol=1e-8,
                max_cycles=400, **TIERS_FP16)
    ctx = P.Context(0)
    loads = {}
    reqs = []
    for i in range(count):
        d, n, fld = W.serving_request(i)
        if (d, n) not in loads:
            loads[(d, n)] = torch.from_numpy(W.load_sine(d, n)).cuda()
        reqs.append((d, n, P.Eps(fld), loads[(d, n)]))
    srv = P.Server(ctx, max_slots=slots, budget_bytes=96e9)
    try:
        warm = {}
        for r in reqs:
            warm.setdefault((r[0], r[1]), r)
        serving.replay(ctx, list(warm.values()), None, server=srv, **opts)
        calib = reqs[:min(len(reqs), 24)]
        t_alone = []
        for d, n, eps, f in calib:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = serving.replay(ctx, [(d, n, eps, f)], None, server=srv, **opts)
            t_alone.append(time.perf_counter() - t0)
            assert res["status"][0] == P.OK
        mean_service = float(np.mean(t_alone))
        rate = 0.8 / mean_service
        arr = W.poisson_arrivals(len(reqs), rate, 4242)
        res = serving.replay(ctx, reqs, arr, server=srv, **opts)
    finally:
        srv.close()
        ctx.close()
    ok = res["status"] == P.OK
    lat = res["latency_ms"][ok]
    dof_cyc = sum((n - 1) ** d * c for (d, n, _, _), c in zip(reqs, res["cycles"]))
    failed = [[i, reqs[i][0], reqs[i][1], int(res["status"][i])] for i in range(len(reqs)) if not ok[i]]
    out = {"requests": len(reqs), "ok": int(ok.sum()), "failed_i_dim_n_status": failed, "slots": slots,
           "single_stream_service_ms": round(mean_service * 1e3, 3),
           "arrival_rate_per_s": round(rate, 2),
           "throughput_req_per_s": round(len(reqs) / res["wall_s"], 2),
           "throughput_dof_cycles_per_s": dof_cyc / res["wall_s"],
           "queue_ms_mean": round(float(np.mean(res["queue_ms"])), 3)}
    out.update({k: round(v, 3) for k, v in serving.percentiles(lat).items()})
    for dim in (2, 3):
        sel = np.array([r[0] == dim for r in reqs]) & ok
        if sel.any():
            out[f"{dim}d"] = {"requests": int(sel.sum()),
                              **{k: round(v, 3) for k, v in serving.percentiles(res["latency_ms"][sel]).items()}}
    return out


# -------------------------------------------------------------- CPU leg
def cpu_baseline(W, n, gpu_rate):
    """The oracle, untouched, on one host core: a complete solve of the same
    material (same boxes, same law, same load, same ladder, transfers, outer
    CG and tolerance) on an n^3 grid, timed end to end."""
    import oracle as O
    d = 3
    fld = W.config_field(4)
    f = W.load_sine(d, n)
    t0 = time.perf_counter()
    u, rep = O.solve(fld, d, n, f, s_max=16, tol=1e-8, transfer=O.BOXMG, outer=O.PCG, max_cycles=400)
    t = time.perf_counter() - t0
    dof = (n - 1) ** d
    value = dof * rep["cycles"] / t
    return {"value": value, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"plain-C FP64 oracle, single thread: complete solve of the headline material on {n}^3 "
                       f"cells ({dof} DoF, ladder to s = 16, BoxMG, CG, 1e-8): {rep['cycles']} cycles in "
                       f"{t:.1f} s (status {rep['status']})"),
            "gpu_over_cpu": round(gpu_rate / value, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU decomposition "
              "is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if args.kernels_only:
        return kernels_only(args)
    if args.solve_only:
        return solve_only(args)
    import torch

    import paper_2005_03606_amd as P
    import workload as W

    d, n = 3, args.n
    main_run = solve_forms(P, W, d, n, W.config_field(4), TIERS_C5, args.steps, args.warmup, main="mixed_lazy")
    ms_main = main_run["ms"]["mixed_lazy"]
    rep_m = main_run["rep"]["mixed_lazy"]
    dof = (n - 1) ** d
    value = dof * rep_m["cycles"] / (ms_main / 1e3)
    comps = {**forms_summary(main_run, n, d),
             "publishes_mixed_lazy": rep_m["publishes"],
             "cell_integrations_per_solve": rep_m["integrations"],
             "step_times_ms_mixed_lazy": [round(t, 1) for t in main_run["all_ms"]["mixed_lazy"]]}
    del main_run
    torch.cuda.empty_cache()
    log("roofline sweep")
    roofline = sweep_roofline(P, W, n, args.sweeps)
    ctx = P.Context(0)
    log("integration rates")
    comps["cell_integrations_per_s"] = integration_rates(P, W, ctx)
    log("paper mode")
    comps["paper_mode_memory_footprint"] = paper_mode_table(P, W, ctx)
    log("adafac")
    comps["adafac"] = adafac_component(P, W, ctx)
    ctx.close()
    if args.n2d > 0:
        m = args.n2d
        b = solve_forms(P, W, 2, m, W.config_field(1), TIERS_FP16, 2, 1)
        comps["time_to_solution_2d_balls"] = {
            "workload": (f"2D {m}^2 Q1 cells, eps=1 + 200 seeded balls (r 0.005-0.05) of eps=1e3, ladder "
                         "s = 2..16, FP16 surplus store, sine load (the eps = 1 load of prod sin(pi x))"), **forms_summary(b, m, 2)}
        del b
    if args.n3d > 0:
        m = args.n3d
        b = solve_forms(P, W, 3, m, W.config_field(2, n=m), TIERS_FP16, 2, 1, s_max=8)
        comps["time_to_solution_3d_gaussian"] = {
            "workload": (f"3D {m}^3 Q1 cells (27-point stencils), eps = exp(g), g a seeded Gaussian field "
                         "(correlation length 1/32, sigma 1), ladder s = 2..8, FP16 surplus store, "
                         "sine load (the eps = 1 load of prod sin(pi x))"), **forms_summary(b, m, 3)}
        del b
    torch.cuda.empty_cache()
    if args.serve_requests > 0:
        log("serving replay")
        comps["serving"] = serving_bench(P, W, args.serve_requests, args.serve_slots)

    out = {"metric": METRIC, "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_main, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16x2-mfma/fp8-fp16-fp32-store/f32-cycle/f64-outer",
           "data": "synthetic",
           "config": {"workload": WORKLOAD, "cells": n ** d, "dof": dof, "levels": rep_m["nlev"]},
           "components": comps, "roofline": roofline}
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_n, value)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
