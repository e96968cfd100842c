#!/usr/bin/env python3
"""Benchmark of the MLFMA boundary-integral matvec on one MI355X.

One step = one whole product y = C x (the BI block of the hybrid solver's
matrix-vector subroutine: near-field blocks plus the MLFMA far field) over
one batch of right-hand sides, inputs resident in HBM.  Default workload:
sphere of radius 3 wavelengths meshed at lambda/10 (25 920 triangles,
38 880 RWG, 77 760 unknowns), 6-level octree with 0.25-wavelength leaves,
one seeded N(0,1) complex right-hand side.

Prints one JSON line: throughput in unknowns*RHS/s for the complex64
(single-precision) path, the complex128 path beside it, stage timings from
HIP events recorded on the launch stream, the roofline of the dominant
kernel, and the CPU oracle timed on a bounded sample of rows with the
error of both GPU paths on those rows.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFS = 157.3          # MI355X FP32, vector and dense MFMA alike
FP64_PEAK_TFS = 78.6           # MI355X vector FP64


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="sphere_r3")
    p.add_argument("--nrhs", type=int, default=None, help="override the workload's RHS count")
    p.add_argument("--cpu-rows", type=int, default=320, help="rows of the oracle sample (0 = skip)")
    p.add_argument("--op", default="C", choices=["C", "EM"])
    p.add_argument("--leaf-extra", type=int, default=2, help="extra multipoles at the leaf level")
    p.add_argument("--interp-order", type=int, default=8, help="Lagrange points per angle")
    p.add_argument("--digits", type=int, default=3, help="MLFMA accuracy parameter d0")
    p.add_argument("--serve-requests", type=int, default=512,
                   help="requests of the serving measurement (0 = skip it)")
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="after the bench, run a plain elementwise copy (torch.neg) over this many MiB of float32 "
                        "three times: the reference kernel that calibrates HBM byte counters")
    return p.parse_args()


def stage_bytes(g, levels_info, n, nrhs, esz, op):
    """Algorithmic HBM bytes of each stage for one product (every operand
    read once, every result written once)."""
    ni = g.near_info()
    leaf = levels_info[max(levels_info)] if levels_info else None
    vec = 2 * n * nrhs * esz
    b = {}
    b["permute_in"] = 2 * vec
    b["permute_out"] = 2 * vec
    ident = ni["identity"] * (4 + esz) if op == "C" else 0
    b["near"] = ni["slots"] * 2 * esz + 2 * vec + ident
    if leaf is None:
        return b, ni
    pat = n * leaf["K"] * 2 * esz
    box = {l: d["boxes"] * d["K"] * 2 * esz * nrhs for l, d in levels_info.items()}
    lmax = max(levels_info)
    b["radiate"] = pat + vec + box[lmax]
    b["aggregate"] = sum(box[l + 1] + box[l] for l in levels_info if l < lmax)
    b["translate"] = sum(2 * box[l] + 316 * levels_info[l]["K"] * esz for l in levels_info)
    b["disaggregate"] = sum(box[l - 1] + 2 * box[l] for l in levels_info if l > min(levels_info))
    b["receive"] = pat + box[lmax] + 2 * vec
    return b, ni


def kernel_sources_sha1():
    """sha1 over the library's kernel and launch sources under csrc/ (file
    name, then bytes); the ABI header's documentation does not change them."""
    import glob
    import hashlib
    h = hashlib.sha1()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2210_04892_amd", "csrc", "*")))
    for f in files:
        if f.endswith((".hip", ".cpp", ".hpp", ".h")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, stage):
    """Calibrated HBM bytes per product of one stage from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (profiles/traffic.json), or None
    when they were taken on other kernel sources than the ones built now."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha1") != kernel_sources_sha1():
        return None
    st = t.get("workloads", {}).get(workload, {}).get("stages", {}).get(stage)
    return None if st is None else st["bytes"]


def stage_flops(g, levels_info, n, nrhs, op, taps):
    """Algorithmic real flops of each stage for one product (complex
    multiply-add = 8, real-times-complex multiply-add = 4)."""
    ni = g.near_info()
    f = {"permute_in": 0, "permute_out": 0}
    f["near"] = 32 * ni["slots"] * nrhs + (12 * ni["identity"] * nrhs if op == "C" else 0)
    if not levels_info:
        return f
    lmax = max(levels_info)
    K = levels_info[lmax]["K"]
    f["radiate"] = 32 * n * K * nrhs
    f["receive"] = 32 * n * K * nrhs
    agg = 0
    for l in levels_info:
        if l == lmax:
            continue
        P, C = levels_info[l], levels_info[l + 1]
        mid = (P["L"] + 1) * (2 * C["L"] + 2)
        agg += C["boxes"] * (2 * mid * taps * 4 + 2 * P["K"] * taps * 4 + 2 * P["K"] * 8) * nrhs
    f["aggregate"] = agg
    f["disaggregate"] = agg
    f["translate"] = sum(16 * d["translations"] * d["K"] * nrhs for d in levels_info.values())
    return f


MFMA_STAGES = ("near", "radiate", "receive")   # on the matrix cores for complex64 and 16+ RHS


def roofline(stage, secs, nbytes, nflops, dtype_bits, nrhs=1):
    """Roofline of one stage: bound by HBM bytes or by flops (vector ALU, or
    the matrix cores for the stages that run on them), whichever takes longer
    at the published peaks."""
    fpeak = FP32_PEAK_TFS if dtype_bits == 32 else FP64_PEAK_TFS
    mfma = dtype_bits == 32 and nrhs >= 16 and stage in MFMA_STAGES
    t_mem = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = nflops / (fpeak * 1e12)
    if t_alu > t_mem:
        ach = nflops / secs / 1e12
        return {"bound": "mfma" if mfma else "alu", "achieved": round(ach, 2), "peak": fpeak, "unit": "TFLOP/s",
                "frac": round(ach / fpeak, 4), "traffic": None, "kernel": stage,
                "algorithmic_flops": int(nflops), "algorithmic_bytes": int(nbytes)}
    ach = nbytes / secs / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": stage,
            "algorithmic_bytes": int(nbytes), "algorithmic_flops": int(nflops)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the matvec shards by right-hand sides or geometries, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_2210_04892_amd as mf

    v, t, spec = synth.workload(a.workload)
    nrhs = a.nrhs or spec["nrhs"]
    k = 2 * math.pi
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = mf.Geometry(v, t, k=k, leaf=spec["leaf"], max_rhs=nrhs, digits=a.digits, interp_order=a.interp_order,
                    leaf_extra_L=a.leaf_extra)
    t1 = time.perf_counter()
    g.precompute()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    N = g.n_rwg
    levels_info = {l: g.level_info(l) for l in range(2, g.levels)} if g.levels >= 3 else {}
    stream = torch.cuda.current_stream()
    if spec.get("rhs") == "plane_waves":
        # incident plane waves projected on the RWG functions by the library (eqs. 49-50)
        khat, pol = synth.plane_waves(nrhs, spec["seed"])
        x = g.plane_wave_rhs(khat, pol).cpu().numpy()
    else:
        x = synth.gaussian_coeffs(2 * N, nrhs, spec["seed"])
    results = {}
    ys = {}
    for name, dt, code in (("c64", np.complex64, mf.C64), ("c128", np.complex128, mf.C128)):
        xt = torch.from_numpy(np.ascontiguousarray(x.T.astype(dt))).cuda()    # column-major 2N x nrhs
        yt = torch.empty_like(xt)
        run = lambda: g.matvec_raw(a.op, code, nrhs, xt.data_ptr(), 2 * N, yt.data_ptr(), 2 * N, stream.cuda_stream)
        for _ in range(a.warmup):
            run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(a.steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        ms = e0.elapsed_time(e1) / a.steps
        # stage split in separate, profiled steps (events between the stages
        # add small gaps, so these steps are not the timed ones)
        g.profile(True)
        for _ in range(max(1, min(a.steps, 10))):
            run()
        torch.cuda.synchronize()
        stages, calls = g.profile_read()
        g.profile(False)
        esz = np.dtype(dt).itemsize
        sb, ni = stage_bytes(g, levels_info, N, nrhs, esz, a.op)
        sf = stage_flops(g, levels_info, N, nrhs, a.op, a.interp_order)
        per = {s: stages[s] / max(calls, 1) for s in stages}
        dom = max(per, key=per.get)
        rl = roofline(dom, per[dom] * 1e-3, sb[dom], sf.get(dom, 0), 32 if name == "c64" else 64, nrhs)
        results[name] = {
            "ms_per_step": ms, "wall_ms_per_step": (w1 - w0) * 1e3 / a.steps,
            "value": 2 * N * nrhs / (ms * 1e-3),
            "stage_ms": {s: round(per[s], 5) for s in per},
            "dominant": dom,
            "roofline": rl,
            "stage_roofline": {st_: roofline(st_, per[st_] * 1e-3, sb[st_], sf.get(st_, 0),
                                             32 if name == "c64" else 64, nrhs)["frac"]
                               for st_ in per if per[st_] > 0 and st_ in sb},
            "near_roofline_GBs": round(sb["near"] / (per["near"] * 1e-3) / 1e9, 1),
        }
        ys[name] = yt.t().cpu().numpy().astype(np.complex128)
    hbm_bytes = g.hbm_bytes
    tuning = g.tuning()
    # outer solver on the same geometry: GMRES(30) on the BI block for the
    # workload's first plane wave (or seeded right-hand side), tol 1e-3
    gm = {}
    b0 = torch.from_numpy(np.ascontiguousarray(x[:, :1])).cuda()
    for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        xs, its, rel = g.gmres(b0.to(dt), op=a.op, restart=30, max_iters=300, tol=1e-3)
        torch.cuda.synchronize()
        gm[name] = {"steps": its, "seconds": round(time.perf_counter() - t_0, 4), "true_rel_residual": float(rel[0])}
        # radar cross section cut of the solution's currents: theta = 0..180 deg, phi = 0
        th = np.radians(np.arange(181.0))
        cut = np.stack([np.sin(th), 0 * th, np.cos(th)], axis=1)
        t_0 = time.perf_counter()
        F = g.far_field(xs, cut)
        torch.cuda.synchronize()
        gm[name]["rcs_cut_181_seconds"] = round(time.perf_counter() - t_0, 4)
        sig = 4 * np.pi * (F.abs() ** 2).sum(dim=1)[:, 0].double().cpu().numpy()
        gm[name]["rcs_dBsm_theta_0_90_180"] = [round(float(10 * np.log10(max(sig[i], 1e-300))), 2) for i in (0, 90, 180)]
    # the same solves right-preconditioned with the SAI of the near field
    # (16 nearest RWGs per pattern), built once on the device
    g.sai_build(a.op, 16)
    sinfo = g.sai_info(a.op)
    gm["sai_k16"] = {"build_ms": round(sinfo["build_ms"], 2), "rwg_pair_entries": sinfo["nnz"],
                     "bytes": sinfo["bytes"]}
    for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        xs, its, rel = g.gmres(b0.to(dt), op=a.op, restart=30, max_iters=300, tol=1e-3, precond="sai")
        torch.cuda.synchronize()
        gm["sai_k16"][name] = {"steps": its, "seconds": round(time.perf_counter() - t_0, 4),
                               "true_rel_residual": float(rel[0])}
    # consistency of the two precisions (same tables, same tree)
    d = np.linalg.norm(ys["c64"] - ys["c128"]) / np.linalg.norm(ys["c128"])
    cpu = None
    errs = {}
    if a.cpu_rows > 0:
        import oracle
        nr = min(a.cpu_rows, N)
        rows = np.sort(np.random.default_rng(spec["seed"] + 1000).choice(N, nr, replace=False))
        c0 = time.perf_counter()
        xo = x
        if spec.get("rhs") == "plane_waves":
            xo = oracle.plane_wave_rhs(v, t, k, khat, pol)      # the oracle's own right-hand sides
        ref = oracle.matvec(v, t, k, xo, op=oracle.OP_C if a.op == "C" else oracle.OP_EM, rows=rows)
        c1 = time.perf_counter()
        secs = c1 - c0
        # a full product evaluates N rows (each giving a J and an M unknown)
        cpu = {"value": 2 * nr * nrhs / secs, "unit": "unknowns*RHS/s", "cores": oracle.threads(),
               "kind": "oracle", "seconds": round(secs, 2),
               "sample": "%d of %d RWG rows (both halves), %d RHS, dense Galerkin product with converged "
                         "touching-pair quadrature; full-matvec time extrapolated as seconds * N / rows" % (nr, N, nrhs)}
        for name in ys:
            got = np.concatenate([ys[name][rows], ys[name][N + rows]])
            errs[name] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    serving = None
    if a.serve_requests > 0:
        from paper_2210_04892_amd import serving as srv
        g.release()
        serving = srv.run(synth.serving_set(5), n_requests=a.serve_requests, seed=5,
                          log=lambda m: print(m, file=sys.stderr, flush=True))
    head = results["c64"]
    head["roofline"]["traffic"] = measured_traffic(spec["name"], head["roofline"]["kernel"])
    out = {
        "metric": "MLFMA L/K matvec unknowns*RHS/s at <=1e-3 rel err vs FP64; p50/p99 latency",
        "value": round(head["value"], 1),
        "unit": "unknowns*RHS/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": "%s: %s" % (spec["name"], {kk: vv for kk, vv in spec.items() if kk != "name"}),
                   "op": a.op, "n_rwg": N, "unknowns": 2 * N, "nrhs": nrhs, "levels": g.levels,
                   "digits": a.digits, "interp_order": a.interp_order, "leaf_extra_L": a.leaf_extra,
                   "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "err_vs_oracle_sampled_rows": errs,
        "c64_vs_c128_rel_diff": float(d),
        "c128": {"value": round(results["c128"]["value"], 1), "ms_per_step": round(results["c128"]["ms_per_step"], 5),
                 "roofline": results["c128"]["roofline"]},
        "stage_ms": {"c64": head["stage_ms"], "c128": results["c128"]["stage_ms"]},
        "stage_roofline_frac": {"c64": head["stage_roofline"], "c128": results["c128"]["stage_roofline"]},
        "near_GBs": {"c64": head["near_roofline_GBs"], "c128": results["c128"]["near_roofline_GBs"]},
        "setup_s": {"tree_tables_patterns": round(t1 - t0, 3), "near_field": round(t2 - t1, 3)},
        "hbm_bytes": hbm_bytes,
        "translation_tile_shape": tuning,
        "serving": serving,
        "gmres_tol_1e-3_and_rcs": gm,
    }
    print(json.dumps(out), flush=True)
    if a.copy_probe_mib > 0:
        n = a.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
