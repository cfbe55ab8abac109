"""Replay of an arrival trace against the continuous-batching solve server.

Each request is submitted at its arrival time (host clock); between arrivals
the loop polls the server, which advances every active solve by one step and
admits waiting requests as slots and device memory free up.  Latency is the
time from arrival to the moment the server saw the solve finish.
"""
import time

import numpy as np
import torch

from . import binding as B


def replay(ctx, requests, arrivals, max_slots=8, budget_bytes=64e9, keep=False, server=None, **opts):
    """requests: list of (dim, n, Eps, f) with f a device float64 load vector;
    arrivals: ascending arrival times in seconds from the start (None: all at
    once).  Keyword options go to every solve.  Returns a dict with the
    per-request latency (ms), status, cycles, and the wall time; with
    keep=True also the solutions.  An existing `server` (and its resident
    state pool) may be passed in; it is left open."""
    m = len(requests)
    arrivals = np.zeros(m) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    srv = server or B.Server(ctx, max_slots=max_slots, budget_bytes=budget_bytes)
    lat = np.full(m, np.nan)
    status = np.zeros(m, dtype=np.int64)
    cycles = np.zeros(m, dtype=np.int64)
    sols = [None] * m
    tickets = {}
    py_lag = np.zeros(m)
    srv_t = np.zeros((m, 3))
    nxt = 0
    done = 0
    t_start = time.perf_counter()
    try:
        while done < m:
            now = time.perf_counter() - t_start
            while nxt < m and arrivals[nxt] <= now:
                dim, n, eps, f = requests[nxt]
                u = torch.zeros_like(f)
                tickets[srv.submit(dim, n, eps, f, u, **opts)] = nxt
                py_lag[nxt] = (time.perf_counter() - t_start) - arrivals[nxt]
                nxt += 1
            fin, act, wait = srv.poll()
            if fin == 0 and act == 0 and wait == 0 and nxt < m:
                time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t_start), 1e-3)))
                continue
            for t in list(tickets):
                res = srv.result(t)
                if res is None:
                    continue
                i = tickets.pop(t)
                st, rep, times, held = res
                status[i] = st
                cycles[i] = rep["cycles"]
                srv_t[i] = times
                lat[i] = (times[2] - times[0]) + py_lag[i] * 1e3
                if keep:
                    sols[i] = held[2]
                done += 1
        wall = time.perf_counter() - t_start
    finally:
        torch.cuda.synchronize()
        if server is None:
            srv.close()
    out = dict(latency_ms=lat, status=status, cycles=cycles, wall_s=wall,
               queue_ms=srv_t[:, 1] - srv_t[:, 0])
    if keep:
        out["solutions"] = sols
    return out


def percentiles(lat_ms):
    a = np.asarray(lat_ms, dtype=np.float64)
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max())}
