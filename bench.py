#!/usr/bin/env python3
"""Benchmark of the delayed-assembly multigrid hot path on one MI355X.

Workload: 2D unit square, 1024 x 1024 Q1 cells, eps = 1 with 200 seeded balls
(radius 0.005-0.05) of eps = 1e3, load of u = sin(pi x) sin(pi y).  Lazily,
V-cycles start on the centre-sample operator while the ladder s = 2, 4, 8,
16 runs on a second stream.  One step = one complete solve to a 1e-8
relative residual of the mixed form (bf16 hi+lo MFMA integration, FP16
surplus store, FP32 BoxMG V(2,2), FP64 outer conjugate gradients) with lazy
assembly; the same lazy assembly without cycles on provisional operators,
the mixed form with up-front assembly and the plain FP64 form with up-front
assembly are timed beside it.  Inputs (load vector, material data) are
resident in HBM before timing.  The same comparison is repeated at 4096^2
cells, where the operators no longer fit in the 256 MB Infinity Cache, on
the 3D Gaussian-field workload at 256^3 cells (27-point stencils, ladder to
s = 8), and as a mean over seeded instances of the 1024^2 balls material.

Prints one JSON line.  `value` is the mixed-lazy form's fine-grid V-cycle
throughput over the whole solve: (n-1)^2 DoF x V-cycles / time-to-solution.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell integrations/s, V-cycle DoF/s, time-to-1e-8 residual: mixed vs FP64"
HBM_PEAK_GBS = 8000.0
WORKLOAD = ("2D 1024^2 Q1 cells, eps=1 + 200 seeded balls (r 0.005-0.05) of eps=1e3, "
            "manufactured u=sin(pi x)sin(pi y), lazy ladder s=2..16 (C=1%), BoxMG V(2,2) omega=0.6 "
            "+ FP64 outer CG to 1e-8; mixed-lazy vs FP64-up-front")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweeps", type=int, default=200, help="timed launches of the roofline kernel")
    ap.add_argument("--serve-requests", type=int, default=96,
                    help="requests in the serving replay (0 skips it)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--big-n", type=int, default=4096,
                    help="also time the sweep at this size, beyond the Infinity Cache (0 skips)")
    ap.add_argument("--n3d", type=int, default=256,
                    help="also time both forms on the 3D Gaussian-field workload at this size (0 skips)")
    ap.add_argument("--seeds", type=int, default=8,
                    help="seeded instances of the 1024^2 balls material for the mean times (0: none)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the roofline sweep and a calibration copy (for counter runs)")
    return ap.parse_args()


def cpu_baseline(fld, d, n, f, cycles):
    """The oracle, untouched, on host cores: setup (full ladder + hierarchy)
    and two outer cycles, extrapolated to the GPU's cycle count."""
    import oracle as O
    kw = dict(s_max=16, tol=1e-8, transfer=O.BOXMG, outer=O.PCG)
    t0 = time.perf_counter()
    O.solve(fld, d, n, f, max_cycles=0, **kw)
    t1 = time.perf_counter()
    O.solve(fld, d, n, f, max_cycles=2, **kw)
    t2 = time.perf_counter()
    t_setup = t1 - t0
    t_cycle = max((t2 - t1) - t_setup, 0.0) / 2.0
    t_tts = t_setup + cycles * t_cycle
    dof = (n - 1) ** d
    return {"value": dof * cycles / t_tts, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"plain-C FP64 oracle, single thread, same 1024^2 problem: up-front ladder + BoxMG "
                       f"hierarchy ({t_setup:.2f} s) and 2 PCG cycles ({t_cycle:.3f} s/cycle), "
                       f"extrapolated to {cycles} cycles = {t_tts:.1f} s time-to-solution")}


# pre half (2 sweeps + residual) of the mixed form's finest level, by the
# source of its operator: the compressed store, or the store's FP32 decode
SWEEP_KERNEL = {"decode": "k_lev2<float, 16, 0, true, true, false, false>",
                "copy": "k_lev2<float, 16, 0, false, true, false, false>"}
# the library's automatic choice: decode the store from this many finest
# vertices on (levels streamed from HBM), read the FP32 decode below
STORE_MIN_NV = 1 << 22
PASSES_PER_LAUNCH = 3  # stencil passes one launch performs: two Jacobi sweeps and the residual
# Memory traffic per launch of the timed kernel at n (bytes), from FETCH_SIZE
# and WRITE_SIZE counter runs of `bench.py --kernels-only` scaled by a 256 MiB
# copy; valid only for the kernel version they were taken on.
SWEEP_TRAFFIC = {1024: 30443057, 4096: 298793616}


def sweep_roofline(ctx, P, d, n, eps, tiers, sweeps):
    """Pre-smoothing half of the finest level of the mixed V-cycle: two
    damped-Jacobi sweeps from zero and the residual in one pass over the
    finest operator, the kernel the mixed cycle moves most of its bytes in,
    with the operator source the solve uses at this size (the compressed
    store from STORE_MIN_NV vertices on, its FP32 decode below).  Timed with
    HIP events on the stream it runs on, same kernel and launch shape as in
    the solve.

    Algorithmic bytes, per DoF and stencil pass (a Jacobi sweep or the
    residual): the stencil (store: payload + tier byte and offset per tile +
    FP32 centre sample per cell; FP32 decode: 4 couplings of 4 bytes) + FP32
    u in, f in, u (or r) out.  One launch performs PASSES_PER_LAUNCH such
    passes; fused, it moves the bytes of about one (stencil, f in, u out, r
    out), reported as the single-pass figure."""
    import torch
    NV = (n + 1) ** d
    path = "decode" if NV >= STORE_MIN_NV else "copy"
    h = P.Hierarchy(ctx, d, n, precision=P.MIXED, transfer=P.BOXMG,
                    store_path=P.STORE_DECODE if path == "decode" else P.STORE_COPY)
    K16, _, _ = P.assemble_cells(ctx, d, n, 16, eps, P.MIXED)
    S32 = P.gather_stencils(ctx, d, n, K16, P.MIXED, P.MIXED)
    eps_c = P.centre_samples(ctx, d, n, eps)
    h.compress(S32, eps_c, **tiers)
    h.coarsen()
    del K16, S32
    ntile, payload, tier_tiles = h.store_info()
    stencil_bytes = payload + 5 * ntile + 4 * n ** d if path == "decode" else 16 * NV
    pass_bytes = stencil_bytes + 12 * NV
    alg_bytes = PASSES_PER_LAUNCH * pass_bytes
    f32 = torch.ones(NV, dtype=torch.float32, device="cuda")
    u32 = torch.zeros_like(f32)
    r32 = torch.zeros_like(f32)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    st = torch.cuda.current_stream()
    h.presmooth(0, None, f32, u32, r32)
    torch.cuda.synchronize()
    calls = max(sweeps, 1)
    ev[0].record(st)
    for _ in range(calls):
        h.presmooth(0, None, f32, u32, r32)
    ev[1].record(st)
    torch.cuda.synchronize()
    avg_ms = ev[0].elapsed_time(ev[1]) / calls
    h.close()
    achieved = alg_bytes / (avg_ms / 1e3) / 1e9
    single = pass_bytes / (avg_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": SWEEP_TRAFFIC.get(n),
            "kernel": SWEEP_KERNEL[path], "operator": "compressed store" if path == "decode" else "FP32 decode",
            "bytes_per_launch": int(alg_bytes),
            "stencil_passes_per_launch": PASSES_PER_LAUNCH, "single_pass_bytes": int(pass_bytes),
            "single_pass_frac": round(single / HBM_PEAK_GBS, 4),
            "avg_launch_us": round(avg_ms * 1e3, 3), "store_tiers": tier_tiles}


FORMS = ("mixed_lazy", "mixed_lazy_parked", "mixed_upfront", "fp64_upfront")


def solve_forms(P, W, n, steps, warmup, tiers, d=2, fld=None, s_max=16):
    """Time-to-1e-8 at n^d cells (default: the 2D balls workload) of
    - mixed_lazy: the paper's schedule, cycling on the provisional operator
      while the ladder runs on the assembly stream;
    - mixed_lazy_parked: the same lazy assembly with the provisional target
      1 (no cycles on a provisional operator: the assembly has the GPU);
    - mixed_upfront and fp64_upfront: every cell's ladder first.
    Each form keeps its device-resident solve state in its own context, so
    no timed loop re-creates another's workspace."""
    import torch
    eps = P.Eps(fld if fld is not None else W.config_field(1))
    f_host = W.load_sine(d, n)
    f = torch.from_numpy(f_host).cuda()
    base = dict(transfer=P.BOXMG, outer=P.PCG, s_max=s_max, tol=1e-8, max_cycles=600)
    kws = {"mixed_lazy": dict(base, precision=P.MIXED, schedule=P.LAZY, **tiers),
           "mixed_lazy_parked": dict(base, precision=P.MIXED, schedule=P.LAZY, prov_tol=1.0, **tiers),
           "mixed_upfront": dict(base, precision=P.MIXED, schedule=P.UPFRONT, **tiers),
           "fp64_upfront": dict(base, precision=P.FP64, schedule=P.UPFRONT)}
    ctxs = {k: P.Context(0) for k in FORMS}
    out = {"eps": eps, "f_host": f_host, "ms": {}, "rep": {}}
    sol = {}
    for k in FORMS:
        for _ in range(warmup):
            P.solve(ctxs[k], d, n, eps, f, torch.zeros_like(f), **kws[k])
        torch.cuda.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(steps):
            u, r = P.solve(ctxs[k], d, n, eps, f, torch.zeros_like(f), **kws[k])
            reps.append(r)
        torch.cuda.synchronize()
        out["ms"][k] = (time.perf_counter() - t0) / steps * 1e3
        assert all(r["status"] == 0 for r in reps), (k, [r["status"] for r in reps])
        out["rep"][k] = reps[-1]
        sol[k] = u
    uf = sol["fp64_upfront"]
    out["err"] = float(torch.linalg.norm(sol["mixed_lazy"] - uf) / torch.linalg.norm(uf))
    for c in ctxs.values():
        c.close()
    return out


def forms_summary(b):
    """Times, cycles and speedups over FP64 up front of every form."""
    ms, rep = b["ms"], b["rep"]
    o = {}
    for k in FORMS:
        o[f"time_to_1e8_{k}_ms"] = round(ms[k], 3)
        o[f"cycles_{k}"] = rep[k]["cycles"]
    for k in FORMS[:-1]:
        o[f"speedup_{k}_vs_fp64_upfront"] = round(ms["fp64_upfront"] / ms[k], 3)
    for k in ("mixed_lazy", "mixed_upfront", "fp64_upfront"):
        o[f"t_first_cycle_ms_{k}"] = round(rep[k]["t_first_cycle_ms"], 3)
    o["mixed_vs_fp64_solution_rel_err"] = b["err"]
    return o


def seed_instances(P, W, n, tiers, seeds):
    """Mean time-to-1e-8 of each form over seeded instances of the balls
    material (200 balls, radii 0.005-0.05, eps 1e3): the cycle count near
    the 1e-8 target varies by a few cycles from instance to instance."""
    import numpy as np
    acc = {k: [] for k in FORMS}
    cyc = {k: [] for k in FORMS}
    for sd in range(seeds):
        b = solve_forms(P, W, n, 1, 1, tiers, fld=W.balls_field(2, 200, 20260 + sd))
        for k in FORMS:
            acc[k].append(b["ms"][k])
            cyc[k].append(b["rep"][k]["cycles"])
    o = {"instances": seeds, "material": "200 balls (r 0.005-0.05, eps 1e3), seeds 20260.."}
    for k in FORMS:
        o[f"mean_time_{k}_ms"] = round(float(np.mean(acc[k])), 3)
        o[f"mean_cycles_{k}"] = round(float(np.mean(cyc[k])), 2)
    for k in FORMS[:-1]:
        o[f"mean_speedup_{k}_vs_fp64_upfront"] = round(float(np.mean(acc["fp64_upfront"]) / np.mean(acc[k])), 3)
    return o


def kernels_only(args):
    """Counter runs: the roofline sweep at the workload size, then a plain
    device copy of known size (calibration of the traffic counters)."""
    import torch
    import paper_2005_03606_amd as P
    import workload as W
    ctx = P.Context(0)
    tiers = dict(min_tier=2, max_tier=2, tau_abs=0.0, tau_rel=1e-7)
    r = sweep_roofline(ctx, P, 2, args.n, P.Eps(W.config_field(1)), tiers, args.sweeps)
    nbytes = 256 << 20
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"sweep": r, "copy_bytes_each_way": nbytes, "copies": 4}), flush=True)


def serving_bench(ctx, P, W, count, slots):
    """Serving replay: mixed 2D/3D requests with Gaussian-field materials,
    Poisson arrivals at 0.8x the measured single-stream capacity."""
    import numpy as np
    import torch
    from paper_2005_03606_amd import serving

    opts = dict(precision=P.MIXED, schedule=P.LAZY, transfer=P.BOXMG, outer=P.PCG, s_max=16, tol=1e-8,
                max_cycles=400, min_tier=2, max_tier=2, tau_rel=1e-7)
    loads = {}
    reqs = []
    for i in range(count):
        d, n, fld = W.serving_request(i)
        if (d, n) not in loads:
            loads[(d, n)] = torch.from_numpy(W.load_sine(d, n)).cuda()
        reqs.append((d, n, P.Eps(fld), loads[(d, n)]))
    srv = P.Server(ctx, max_slots=slots, budget_bytes=96e9)
    try:
        # resident state for every shape, then single-stream service times
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
    return out


def main():
    args = parse()
    if args.kernels_only:
        return kernels_only(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU decomposition "
              "is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2005_03606_amd as P
    import workload as W

    d, n = 2, args.n
    tiers = dict(min_tier=2, max_tier=2, tau_abs=0.0, tau_rel=1e-7)
    fld = W.config_field(1)
    main_run = solve_forms(P, W, n, args.steps, args.warmup, tiers)
    ms_mixed, ms_fp64 = main_run["ms"]["mixed_lazy"], main_run["ms"]["fp64_upfront"]
    rep_m, rep_f = main_run["rep"]["mixed_lazy"], main_run["rep"]["fp64_upfront"]
    eps, f_host, err = main_run["eps"], main_run["f_host"], main_run["err"]
    dof = (n - 1) ** d
    cyc_m = rep_m["cycles"]
    value = dof * cyc_m / (ms_mixed / 1e3)
    ctx = P.Context(0)

    # cell integrations per second (all cells, s = 16), both precisions
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    integ = {}
    for mode, name in ((P.MIXED, "mixed_bf16x2_mfma"), (P.FP64, "fp64")):
        P.assemble_cells(ctx, d, n, 16, eps, mode)
        ev[0].record()
        reps = 3
        for _ in range(reps):
            P.assemble_cells(ctx, d, n, 16, eps, mode)
        ev[1].record()
        torch.cuda.synchronize()
        integ[name] = n ** d * reps / (ev[0].elapsed_time(ev[1]) / 1e3)

    roofline = sweep_roofline(ctx, P, d, n, eps, tiers, args.sweeps)
    big = big_tts = None
    if args.big_n > 0:
        big_eps = P.Eps(W.config_field(1))
        big = sweep_roofline(ctx, P, d, args.big_n, big_eps, tiers, args.sweeps)
        big = {k: big[k] for k in ("achieved", "frac", "single_pass_frac", "bytes_per_launch", "single_pass_bytes",
                                   "traffic", "avg_launch_us", "kernel", "operator", "store_tiers")}
        big["workload"] = f"same material, {args.big_n}^2 cells (store and vectors beyond the 256 MB Infinity Cache)"
        b = solve_forms(P, W, args.big_n, 2, 1, tiers)
        big_tts = {"workload": f"same material and load at {args.big_n}^2 cells (beyond the Infinity Cache)",
                   **forms_summary(b)}
    NV = (n + 1) ** d

    out = {"metric": METRIC, "value": value, "unit": "DoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_mixed, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16x2-mfma/f16-store/f32-cycle/f64-outer",
           "data": "synthetic",
           "config": {"workload": WORKLOAD, "cells": n ** d, "dof": dof, "levels": rep_m["nlev"]},
           "components": {
               **forms_summary(main_run),
               "publishes_mixed_lazy": rep_m["publishes"],
               "vcycle_dof_per_s_fp64_upfront": dof * rep_f["cycles"] / (ms_fp64 / 1e3),
               "cell_integrations_per_s_s16": {k: round(v, 1) for k, v in integ.items()},
               "cell_integrations_per_solve": rep_m["integrations"],
               "cells_at_s_1_2_4_8_16": rep_m["cells_at_s"],
               "store_bytes_per_stencil_mixed": rep_m["store_bytes"] / NV,
               "store_bytes_per_stencil_fp64": rep_f["store_bytes"] / NV,
           },
           "roofline": roofline}
    if big is not None:
        out["components"]["sweep_roofline_beyond_cache"] = big
        out["components"]["time_to_solution_beyond_cache"] = big_tts
    if args.n3d > 0:
        m = args.n3d
        b = solve_forms(P, W, m, 2, 1, tiers, d=3, fld=W.config_field(2, n=m), s_max=8)
        out["components"]["time_to_solution_3d"] = {
            "workload": (f"3D {m}^3 Q1 cells (27-point stencils), eps = exp(g), g a seeded Gaussian field "
                         "(correlation length 1/32, sigma 1), ladder s = 2..8, manufactured sine load"),
            **forms_summary(b),
            "store_bytes_per_stencil_mixed": b["rep"]["mixed_lazy"]["store_bytes"] / (m + 1) ** 3,
            "store_bytes_per_stencil_fp64": b["rep"]["fp64_upfront"]["store_bytes"] / (m + 1) ** 3}
        del b
        torch.cuda.empty_cache()
    if args.seeds > 0:
        out["components"]["instances_1024"] = seed_instances(P, W, n, tiers, args.seeds)
    if args.serve_requests > 0:
        out["components"]["serving"] = serving_bench(ctx, P, W, args.serve_requests, args.serve_slots)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(fld, d, n, f_host, rep_f["cycles"])
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
