"""Serving measurement: concurrent matvec requests over resident geometries.

Drives the library's continuous-batching server (mlfma_server_*) with a
seeded Poisson stream of requests and reports throughput and p50/p99
latency next to one-at-a-time complex128 products served in arrival order
under the same arrivals.
"""
import math
import threading
import time

import numpy as np
import torch

from . import binding as mf


def _percentiles(lat):
    a = np.sort(np.asarray(lat))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def make_requests(geoms, n_requests, seed, dtype, max_rhs=16):
    """Geometry uniform, nrhs ~ U{1..max_rhs}, coefficients N(0,1) + jN(0,1)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_requests):
        gi = int(rng.integers(len(geoms)))
        nr = int(rng.integers(1, max_rhs + 1))
        n2 = 2 * geoms[gi].n_rwg
        x = (rng.standard_normal((nr, n2)) + 1j * rng.standard_normal((nr, n2))).astype(dtype)
        reqs.append((gi, torch.from_numpy(x).cuda()))
    return reqs


def run_stream(server, geoms, reqs, arrivals, op="C"):
    """Submit reqs at the given arrival offsets (seconds; None = all at once)
    from one thread, wait from another; returns (latencies, wall seconds, batch sizes)."""
    ys = [torch.empty_like(x) for _, x in reqs]
    tickets = [None] * len(reqs)
    ready = [threading.Event() for _ in reqs]
    lat = [0.0] * len(reqs)
    bsz = [0] * len(reqs)

    errors = []

    def waiter():
        for i in range(len(reqs)):
            ready[i].wait()
            try:
                lat[i], bsz[i] = server.wait(tickets[i])
            except Exception as e:          # reported to the caller below
                errors.append(e)

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for i, (gi, x) in enumerate(reqs):
        if arrivals is not None:
            dt = t0 + arrivals[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        tickets[i] = server.submit(geoms[gi], x, ys[i], op=op)
        ready[i].set()
    th.join()
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    return lat, wall, bsz, ys


def one_at_a_time(geoms, reqs, arrivals, op="C"):
    """Loaded one-at-a-time baseline: the same requests, arriving at the same
    offsets, served in arrival order by plain complex128 products from one
    host thread, each product finished before the next starts.  Returns
    (latencies from arrival to completion, summed service seconds)."""
    xs = [x.to(torch.complex128).t() for _, x in reqs]
    torch.cuda.synchronize()
    lat, busy = [], 0.0
    t0 = time.perf_counter()
    for (gi, _), x128, a in zip(reqs, xs, arrivals):
        dt = t0 + a - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        s0 = time.perf_counter()
        geoms[gi].matvec(x128, op=op)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        busy += t1 - s0
        lat.append(t1 - (t0 + a))
    return lat, busy


def geometry_batch(geoms, nrhs=4, seed=9, reps=10, op="C", dtype=torch.complex64):
    """One product of every resident geometry (nrhs right-hand sides each),
    three ways: one after another on one stream, mlfma_matvec_batch (each
    geometry on its own stream) and mlfma_matvec_batch_fused (the same, with
    the translations of all geometries in shared launches).  Milliseconds per
    round (mean of reps after one warm-up) and the largest relative
    difference of the fused products from the single ones."""
    rng = np.random.default_rng(seed)
    xs = []
    for g in geoms:
        n2 = 2 * g.n_rwg
        x = rng.standard_normal((n2, nrhs)) + 1j * rng.standard_normal((n2, nrhs))
        xs.append(torch.from_numpy(x).to(dtype).cuda())
    items = [(g, x, op) for g, x in zip(geoms, xs)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    single = lambda: [g.matvec(x, op=op) for g, x in zip(geoms, xs)]
    ms_seq = timed(single)
    ms_fork = timed(lambda: mf.matvec_batch(items))
    ms_fused = timed(lambda: mf.matvec_batch(items, fused=True))
    ys = mf.matvec_batch(items, fused=True)
    ref = single()
    torch.cuda.synchronize()
    diff = max(float(torch.linalg.norm(y - r) / torch.linalg.norm(r)) for y, r in zip(ys, ref))
    unknowns = sum(2 * g.n_rwg * nrhs for g in geoms)
    return {"geometries": len(geoms), "nrhs": nrhs, "dtype": str(dtype).replace("torch.", ""),
            "sequential_ms": ms_seq, "forked_streams_ms": ms_fork, "fused_ms": ms_fused,
            "fused_unknowns_rhs_per_s": unknowns / (ms_fused * 1e-3),
            "max_rel_diff_fused_vs_single": diff}


def run(geom_list, n_requests=512, seed=5, streams=4, max_batch_rhs=16, load=0.7, op="C",
        dtype=np.complex64, log=print, use_graphs=True):
    geoms = []
    for name, v, t in geom_list:
        g = mf.Geometry(v, t, max_rhs=max_batch_rhs).precompute()
        geoms.append(g)
        log("[serve] geometry %s: N=%d levels=%d" % (name, g.n_rwg, g.levels))
    reqs = make_requests(geoms, n_requests, seed, dtype, max_rhs=16)
    unknowns = sum(2 * geoms[gi].n_rwg * x.shape[0] for gi, x in reqs)
    # arena footprint with every slot holding the largest geometry, and a
    # budget below it so that admission by memory is exercised
    from .binding import lib  # noqa: F401
    probe = mf.Server(streams=streams, max_batch_rhs=max_batch_rhs, use_graphs=use_graphs)
    lat, wall, bsz, _ = run_stream(probe, geoms, reqs[:64], None, op)
    full = probe.stats()["arena_bytes"]
    probe.close()
    budget = int(0.75 * full) if full else 0
    server = mf.Server(streams=streams, max_batch_rhs=max_batch_rhs, hbm_budget_bytes=budget, use_graphs=use_graphs)
    # capacity: everything submitted at once (closed loop)
    lat_c, wall_c, bsz_c, ys = run_stream(server, geoms, reqs, None, op)
    capacity = len(reqs) / wall_c
    log("[serve] capacity %.1f requests/s (batched, all queued at once)" % capacity)
    # open loop: Poisson arrivals at `load` x capacity
    rng = np.random.default_rng(seed + 1)
    rate = load * capacity
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
    lat_p, wall_p, bsz_p, ys_p = run_stream(server, geoms, reqs, arrivals, op)
    p50, p99 = _percentiles(lat_p)
    stats = server.stats()
    # each result the same alone and in the mix (alone: a single product of
    # the library with the request's own right-hand sides)
    worst = 0.0
    for i in range(0, len(reqs), max(1, len(reqs) // 32)):
        gi, x = reqs[i]
        alone = geoms[gi].matvec(x.t(), op=op).t()
        d = float(torch.linalg.norm(alone - ys_p[i]) / torch.linalg.norm(alone))
        worst = max(worst, d)
    server.close()
    # one-at-a-time complex128 products in arrival order, measured under the
    # same arrivals
    lat_b, busy = one_at_a_time(geoms, reqs, arrivals, op)
    b50, b99 = _percentiles(lat_b)
    batch = geometry_batch(geoms, op=op)
    log("[serve] one product of each geometry (4 RHS): sequential %.2f ms, forked %.2f ms, fused %.2f ms"
        % (batch["sequential_ms"], batch["forked_streams_ms"], batch["fused_ms"]))
    res = {
        "requests": len(reqs), "geometries": [g.n_rwg for g in geoms], "streams": streams,
        "max_batch_rhs": max_batch_rhs, "dtype": np.dtype(dtype).name, "budget_bytes": budget,
        "arena_bytes_all_slots_largest": full,
        "capacity_requests_per_s": capacity,
        "throughput_unknowns_rhs_per_s": unknowns / wall_c,
        "poisson_rate_requests_per_s": rate,
        "p50_ms": 1e3 * p50, "p99_ms": 1e3 * p99,
        "mean_batch_rhs": float(np.mean(bsz_p)),
        "launches": stats["launches"],
        "graphs": bool(use_graphs), "graph_captures": stats["graph_captures"],
        "max_rel_diff_alone_vs_mix": worst,
        "one_at_a_time_c128": {"kind": "measured: same arrivals, served in order by plain complex128 "
                                       "products from one host thread",
                               "throughput_unknowns_rhs_per_s": unknowns / busy,
                               "p50_ms": 1e3 * b50, "p99_ms": 1e3 * b99},
        "geometry_batch": batch,
    }
    for g in geoms:
        g.release()
    return res
