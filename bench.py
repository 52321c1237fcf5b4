#!/usr/bin/env python3
"""Benchmark of the BAMG-preconditioned FGMRES solve on one MI355X.

Workload (default): 256 x 256 periodic lattice, quenched U(1) links from 500
Metropolis sweeps at beta = 10 (seed 3), mass calibrated so that
min |eig(D)| ~ 1e-4, one complex Gaussian right-hand side (seed 103); 4-level
hierarchy (4x4 then 2x2 aggregates, 8 test vectors), V(4,4) cycle, FGMRES(32)
to a relative residual of 1e-10 on the reduced system.  Setup is done once
and timed separately; every timed step is one full solve (reduction, FGMRES,
reconstruction) with the right-hand side already in HBM.

Prints one JSON line (rank 0).  Besides solves/s it reports the Dhat
("D_oe") bandwidth at three sizes, the roofline of the dominant kernel and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s to rel-res 1e-10 @256² (mixed vs FP64); D_oe HBM GB/s; p99 ms"
PRECISIONS = {"fp64": 0, "mixed_fp16": 1, "mixed_bf16": 2, "mixed_fp32": 3}
DTYPES = {"fp64": "f64", "mixed_fp16": "f64 outer / f32 cycle / f16 coarse storage",
          "mixed_bf16": "f64 outer / f32 cycle / bf16 coarse storage",
          "mixed_fp32": "f64 outer / f32 cycle"}
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3_256_b10")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dhat", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--batch", default="8,32", help="right-hand sides per batched solve (comma list, '' for none)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--precisions", default="mixed_fp16+graphs,mixed_fp16,fp64,fp64+graphs,mixed_bf16,mixed_fp32",
                    help="single-RHS precisions to time; the first one is the headline value")
    ap.add_argument("--serve", type=int, default=48, help="requests of the serving run (0: skip it)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate of the serving run (1/s)")
    ap.add_argument("--c4", type=int, default=1, help="time the 512^2 x 64 RHS batched solve (0: skip)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="set up the headline hierarchy, time only the roofline kernel and a plain copy of "
                         "COPY_MIB MiB (the scale of the HBM byte counters), print them and exit")
    return ap.parse_args()


COPY_MIB = 256


def copy_calibration(torch):
    """One plain copy kernel of known size (reads and writes COPY_MIB MiB):
    its FETCH_SIZE / WRITE_SIZE counters give the scale of those counters."""
    src = torch.ones(COPY_MIB * 2 ** 20 // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    torch.mul(src, 1.0, out=dst)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    del src, dst
    return {"kernel": "torch mul(src, 1.0) (vectorized elementwise)", "bytes_read": COPY_MIB * 2 ** 20,
            "bytes_written": COPY_MIB * 2 ** 20, "us": t * 1e6, "GB/s": 2 * COPY_MIB * 2 ** 20 / t / 1e9}


T0 = time.time()


def progress(msg):
    """One line per finished stage on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg} ({time.time() - T0:.1f} s)", file=sys.stderr, flush=True)


def time_launches(fn, reps, launches_per_call, torch):
    """Average duration per kernel launch of fn() (events on the library's stream)."""
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / (reps * launches_per_call)


SERVE_FIELDS = ["s1_64_b3", "c2_128_b6", "c3_256_b10", "c4_512_b10"]


def serving(bamg, inputs, torch, np, n_req, rate, tol):
    """Poisson arrivals of solve requests over four gauge fields (64^2 beta=3,
    128^2 beta=6, 256^2 beta=10, 512^2 beta=10), 1-32 right-hand sides each,
    on a threaded server with memory admission and continuous batching (mixed
    FP16 hierarchies, 32 slots per field).  The hierarchies are made resident
    by one warm-up request per field; then every request's right-hand sides
    are placed in HBM and the requests are submitted at their arrival times.
    Latency is submit -> completion as the server measures it."""
    rng = np.random.default_rng(4242)
    sp = bamg.bamg_server_default_params(threaded=1, slots_per_field=32)
    srv = bamg.bamg_server_create(sp)
    fids, Ns = [], []
    t0 = time.time()
    for name in SERVE_FIELDS:
        w = inputs.workload(name)
        U = torch.from_numpy(inputs.load_gauge(w)).to("cuda:0")
        p = bamg.bamg_default_params(N=w["N"], n_levels=w["n_levels"], seed=w["tv_seed"],
                                     precision=PRECISIONS["mixed_fp16"])
        fids.append(bamg.bamg_server_add_field(srv, U, w["m"], p))
        Ns.append(w["N"])
        del U
    t_gauge = time.time() - t0
    t0 = time.time()
    keep = []
    for f, N in zip(fids, Ns):  # warm-up: setup + one solve per field
        B = torch.from_numpy(inputs.gaussian((1, 2 * N * N), 7000 + N)).to("cuda:0")
        X = torch.zeros_like(B)
        rid = bamg.bamg_server_submit(srv, f, B, X, 1, tol)
        keep.append((rid, B, X))
    for rid, B, X in keep:
        bamg.bamg_server_wait(srv, rid, 1)
    t_warm = time.time() - t0
    warm = bamg.bamg_server_get_stats(srv)
    bamg.bamg_server_reset_stats(srv)
    # the request stream
    which = rng.integers(0, len(fids), n_req)
    nrhs = rng.integers(1, 33, n_req)
    gaps = rng.exponential(1.0 / rate, n_req)
    reqs = []
    for i in range(n_req):
        N = Ns[which[i]]
        B = torch.from_numpy(inputs.gaussian((int(nrhs[i]), 2 * N * N), 8000 + i)).to("cuda:0")
        reqs.append((fids[which[i]], int(nrhs[i]), B, torch.zeros_like(B)))
    torch.cuda.synchronize()
    ids = []
    t_start = time.perf_counter()
    t_next = t_start
    for i, (f, k, B, X) in enumerate(reqs):
        t_next += gaps[i]
        dt = t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        ids.append(bamg.bamg_server_submit(srv, f, B, X, k, tol))
    iters, conv = [], True
    per_field = {name: 0 for name in SERVE_FIELDS}
    for (f, k, B, X), rid in zip(reqs, ids):
        st, infos = bamg.bamg_server_wait(srv, rid, k)
        conv = conv and st == 0 and all(v["relres_reduced"] <= tol for v in infos)
        iters.append(max(v["iters"] for v in infos))
        per_field[SERVE_FIELDS[fids.index(f)]] += k
    t_end = time.perf_counter()
    st = bamg.bamg_server_get_stats(srv)
    bamg.bamg_server_free(srv)
    n_timed, rhs_timed = st["completed"], st["rhs_completed"]
    return {
        "fields": {n: {"N": N_} for n, N_ in zip(SERVE_FIELDS, Ns)}, "precision": "mixed_fp16",
        "slots_per_field": sp.slots_per_field, "requests": n_timed, "rhs": rhs_timed, "rhs_per_field": per_field,
        "arrival_rate_per_s": rate, "offered_s": float(np.sum(gaps)),
        "solves_per_s": rhs_timed / (t_end - t_start), "wall_s": t_end - t_start,
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"], "max_ms": st["max_ms"],
        "latency": "submit to completion per request (server clock), nearest-rank percentiles",
        "max_iters": int(max(iters)), "converged": conv, "setups": st["setups"], "evictions": st["evictions"],
        "bytes_in_use": st["bytes_in_use"], "budget_bytes": st["budget_bytes"], "rounds": st["rounds"],
        "setup_warmup_s": t_warm, "warmup_setups": warm["setups"], "gauge_gen_s": t_gauge,
    }


def c4_batched(bamg, inputs, torch, tol, reps=2):
    """512^2, beta=10, 64 right-hand sides on one gauge field: the multi-RHS
    solve (mixed FP16 hierarchy, MFMA coarse smoother, batched kernels)."""
    w = inputs.workload("c4_512_b10")
    N = w["N"]
    U = torch.from_numpy(inputs.load_gauge(w)).to("cuda:0")
    out = {"workload": w["name"], "N": N, "nrhs": w["nrhs"], "m": w["m"], "precision": "mixed_fp16"}
    p = bamg.bamg_default_params(N=N, n_levels=w["n_levels"], seed=w["tv_seed"], precision=PRECISIONS["mixed_fp16"])
    torch.cuda.synchronize()
    t0 = time.time()
    h = bamg.bamg_setup(U, w["m"], p)
    torch.cuda.synchronize()
    out["setup_s"] = time.time() - t0
    out["levels"] = bamg.bamg_n_levels(h)
    R = w["nrhs"]
    B = torch.from_numpy(inputs.gaussian((R, 2 * N * N), w["rhs_seed"])).to("cuda:0")
    X = torch.zeros_like(B)
    bamg.bamg_solve_batch(h, B, X, R, tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st, infos = bamg.bamg_solve_batch(h, B, X, R, tol)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    out.update({"solves_per_s": R / t, "ms_per_batch": 1e3 * t, "max_iters": max(i["iters"] for i in infos),
                "converged": all(i["relres_reduced"] <= tol for i in infos)})
    bamg.bamg_free(h)
    del U, B, X
    torch.cuda.empty_cache()
    return out


def dhat_bandwidth(bamg, inputs, torch, N, nrhs, reps):
    """GB/s of the Dhat kernel: 64 N^2 bytes per right-hand side per apply
    (x and y 16 N^2 each, links 32 N^2), algorithmic; operator-only handle."""
    U = torch.from_numpy(inputs.gauge_random(N, 77)).to("cuda:0")
    p = bamg.bamg_default_params(N=N, n_levels=1)
    h = bamg.bamg_setup(U, -0.05, p)
    x = torch.from_numpy(inputs.gaussian((nrhs, N * N), 78)).to("cuda:0")
    y = torch.empty_like(x)
    t = time_launches(lambda: bamg.bamg_apply_dhat(h, x, y, nrhs), reps, 1, torch)
    bytes_ = 64.0 * N * N * nrhs
    bamg.bamg_free(h)
    del x, y, U
    torch.cuda.empty_cache()
    return {"N": N, "nrhs": nrhs, "us": t * 1e6, "GB/s": bytes_ / t / 1e9}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (a multi-GPU run would shard "
              "right-hand sides, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import inputs
    import paper_1308_5992_amd as bamg

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    w = inputs.workload(args.workload)
    N = w["N"]
    t0 = time.time()
    U_np = inputs.load_gauge(w)
    t_gauge = time.time() - t0
    U = torch.from_numpy(U_np).to("cuda:0")
    b = torch.from_numpy(inputs.gaussian(2 * N * N, w["rhs_seed"])).to("cuda:0")
    precs = [v.strip() for v in args.precisions.split(",") if v.strip()]
    head = precs[0]
    if args.roofline_only:
        hp = head.partition("+")[0]
        p = bamg.bamg_default_params(N=N, n_levels=w["n_levels"], seed=w["tv_seed"], precision=PRECISIONS[hp])
        h = bamg.bamg_setup(U, w["m"], p)
        out = {"workload": w["name"], "precision": hp, "roofline": roofline(bamg, torch, h, hp),
               "copy_calibration": copy_calibration(torch)}
        bamg.bamg_free(h)
        print(json.dumps(out), flush=True)
        return
    results, hier, xs = {}, {}, {}
    for prec in precs:
        base, _, opt = prec.partition("+")  # "<precision>+graphs": iterations replayed as hipGraphs
        p = bamg.bamg_default_params(N=N, n_levels=w["n_levels"], seed=w["tv_seed"], precision=PRECISIONS[base],
                                     graphs=1 if opt == "graphs" else 0)
        torch.cuda.synchronize()
        t0 = time.time()
        h = bamg.bamg_setup(U, w["m"], p)
        torch.cuda.synchronize()
        t_setup = time.time() - t0
        x = torch.zeros_like(b)
        for _ in range(args.warmup):
            bamg.bamg_solve(h, b, x, args.tol)
        torch.cuda.synchronize()
        times, infos = [], []
        t_all0 = time.perf_counter()
        for _ in range(args.steps):
            t1 = time.perf_counter()
            st, info = bamg.bamg_solve(h, b, x, args.tol)
            times.append(time.perf_counter() - t1)
            infos.append(info)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t_all0
        ms = [1e3 * t for t in times]
        results[prec] = {
            "solves_per_s": args.steps / t_all, "ms_per_solve": 1e3 * t_all / args.steps,
            "p50_ms": statistics.median(ms), "p99_ms": float(np.percentile(ms, 99)),
            "iters": infos[-1]["iters"], "relres_reduced": infos[-1]["relres_reduced"],
            "converged": all(i["relres_reduced"] <= args.tol for i in infos), "setup_s": t_setup,
        }
        hier[prec] = h
        xs[prec] = x.cpu().numpy()
        progress(f"{prec}: {results[prec]['solves_per_s']:.1f} solves/s")
    if "fp64" in xs:
        for prec in precs:
            if prec != "fp64":
                results[prec]["rel_err_vs_fp64"] = float(np.linalg.norm(xs[prec] - xs["fp64"]) /
                                                         np.linalg.norm(xs["fp64"]))
    h = hier[head]
    n_levels = bamg.bamg_n_levels(h)
    r0 = results[head]
    out = {
        "metric": METRIC,
        "value": r0["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r0["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[head.partition("+")[0]],
        "data": "synthetic",
        "config": {
            "workload": w["name"], "N": N, "beta": w["beta"], "metropolis_sweeps": w["sweeps"],
            "m": w["m"], "min_abs_eig_D": w["min_abs_eig_D"], "levels": n_levels,
            "aggregates": "4x4 half-x, then 2x2", "test_vectors": 8, "cycle": "V(4,4)",
            "krylov": "FGMRES(32)", "tol": args.tol, "nrhs": 1, "precision": head,
        },
        "p50_ms": r0["p50_ms"],
        "p99_ms": r0["p99_ms"],
        "iters": r0["iters"],
        "relres_reduced": r0["relres_reduced"],
        "converged": r0["converged"],
        "gauge_gen_s": t_gauge,
        "precisions": results,
    }

    # ---- batched solves: R right-hand sides per call, lockstep FGMRES
    batched = []
    for R in [int(v) for v in args.batch.split(",") if v.strip()]:
        B = torch.from_numpy(inputs.gaussian((R, 2 * N * N), w["rhs_seed"] + 1000)).to("cuda:0")
        X = torch.zeros_like(B)
        bamg.bamg_solve_batch(h, B, X, R, args.tol)
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        for _ in range(args.batch_steps):
            st, infs = bamg.bamg_solve_batch(h, B, X, R, args.tol)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - tb0) / args.batch_steps
        batched.append({"nrhs": R, "precision": head, "solves_per_s": R / tb, "ms_per_batch": 1e3 * tb,
                        "max_iters": max(i["iters"] for i in infs),
                        "converged": all(i["relres_reduced"] <= args.tol for i in infs)})
        del B, X
        progress(f"batched R={R}: {batched[-1]['solves_per_s']:.1f} solves/s")
    if batched:
        out["batched"] = batched

    # ---- 512^2 x 64 right-hand sides on one field (multi-RHS form)
    if args.c4:
        out["c4_512x64"] = c4_batched(bamg, inputs, torch, args.tol)
        progress(f"512^2 x 64: {out['c4_512x64']['solves_per_s']:.1f} solves/s")

    # ---- serving: Poisson arrivals over four fields, continuous batching
    if args.serve > 0:
        out["serving"] = serving(bamg, inputs, torch, np, args.serve, args.serve_rate, args.tol)
        out["serving_p99_ms"] = out["serving"]["p99_ms"]
        progress(f"serving: p50 {out['serving']['p50_ms']:.1f} ms p99 {out['serving']['p99_ms']:.1f} ms")

    # ---- Dhat ("D_oe") bandwidth: cache-resident, batched, cache-busting
    if not args.no_dhat:
        pts = []
        for (n_, r_, reps) in ((256, 1, 200), (512, 64, 20), (4096, 1, 20)):
            pts.append(dhat_bandwidth(bamg, inputs, torch, n_, r_, reps))
        out["dhat_bandwidth"] = pts
        progress("dhat bandwidth")

    # ---- roofline of the dominant kernel of the solve
    if not args.no_roofline:
        out["roofline"] = roofline(bamg, torch, h, head.partition("+")[0])
        progress("roofline")

    # ---- CPU oracle on a bounded sample of the same workload
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, U_np, args.tol)
        progress("cpu baseline")

    for hh in hier.values():
        bamg.bamg_free(hh)
    print(json.dumps(out), flush=True)


# Algorithmic bytes one coarse site moves in its colour pass of the Kaczmarz
# smoother: the 7 blocks of 16x16 complex of its rows (storage type), the 16x16
# smoother matrix Kinv (cycle type), its 16 right-hand-side entries, and the
# 7 x 16 unknowns of its row support read and written (the supports of one
# colour are disjoint, so nothing is counted twice within a launch).
def _site_bytes(s_op, s_vec):
    return 7 * 256 * s_op + 256 * s_vec + 16 * s_vec + 2 * 7 * 16 * s_vec


SITE_SWEEP_BYTES = {"fp64": _site_bytes(16, 16), "mixed_fp32": _site_bytes(8, 8),
                    "mixed_fp16": _site_bytes(4, 8), "mixed_bf16": _site_bytes(4, 8)}

# HBM byte counters of the same launches (rocprofv3 --pmc FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, median over the roofline sweeps), each divided
# by what the counter reads per KiB moved by a plain 256 MiB copy kernel in the
# same run.  Valid only for the kernel source they were taken on (sha256 of
# coarse.hip); any change to it makes the reported traffic null.
PMC_TRAFFIC = {
    "mixed_fp16": {"coarse_hip_sha256": "676578ea4fbb84cbfe95f0270878300590c3ed8b8a3c4a9fb0a712aea4efed1e",
                   "fetch_kib": 1313.0, "write_kib": 224.0, "fetch_per_kib": 131090.6 / 262144.0,
                   "write_per_kib": 262144.0 / 262144.0,
                   "profile": "profiles/kaczmarz_coarse_level1_c3_256_mixed_fp16_pmc.md"},
}


def pmc_traffic(prec):
    import hashlib
    e = PMC_TRAFFIC.get(prec)
    if e is None:
        return None
    with open(os.path.join(ROOT, "paper_1308_5992_amd", "csrc", "coarse.hip"), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != e["coarse_hip_sha256"]:
            return None
    return 1024.0 * (e["fetch_kib"] / e["fetch_per_kib"] + e["write_kib"] / e["write_per_kib"])


def roofline(bamg, torch, h, prec):
    """Coarse Kaczmarz colour pass on level 1 of the headline hierarchy (with
    the fine pass, the kernels that take the solve's time; see the kernel
    trace).  One launch is one colour: 1/ncol of the level's sites, each moving
    SITE_SWEEP_BYTES[prec] algorithmic bytes.  Timed with HIP events over 50
    sweeps on the library's stream (torch's current stream); a mixed hierarchy
    is driven through the complex64 hook, which launches exactly the ncol
    colour passes of one sweep and nothing else."""
    inf = bamg.bamg_level_info(h, 1)
    ns = inf["ex"] * inf["ey"]
    ncol = inf["colours"]
    n = inf["n"]
    if prec == "fp64":
        dt, op = torch.complex128, bamg.OP_SWEEP
        kname = "k_kaczmarz_coarse<double,cx<double>>"
    else:
        dt, op = torch.complex64, bamg.OP_SWEEP_F32
        kname = {"mixed_fp16": "k_kaczmarz_coarse<float,hcx>", "mixed_bf16": "k_kaczmarz_coarse<float,bcx>",
                 "mixed_fp32": "k_kaczmarz_coarse<float,cx<float>>"}[prec]
    xb = torch.zeros(n, dtype=dt, device="cuda:0")
    bb = torch.ones(n, dtype=dt, device="cuda:0")
    t = time_launches(lambda: bamg.bamg_level_op(h, 1, op, bb, xb, 1), 50, ncol, torch)
    bytes_launch = ns * SITE_SWEEP_BYTES[prec] / ncol
    achieved = bytes_launch / t / 1e9
    return {"kernel": kname + f" (level 1, {ns // ncol} sites per launch)", "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": pmc_traffic(prec), "traffic_unit": "bytes per launch",
            "avg_launch_us": t * 1e6, "bytes_per_launch": bytes_launch}


def cpu_baseline(w, U_np, tol):
    """The oracle (single-threaded C++ FP64) solving the same system: its setup
    runs untimed, the sample is one full solve."""
    import numpy as np
    import inputs
    import oracle
    N = w["N"]
    b = inputs.gaussian(2 * N * N, w["rhs_seed"])
    o = oracle.Hierarchy(U_np, w["m"], n_levels=w["n_levels"], seed=w["tv_seed"])
    t0 = time.perf_counter()
    st, xo, info = o.solve(b, tol=tol)
    t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of the same workload ({info['iters']} FGMRES iterations, "
                      f"{t:.2f} s); oracle setup untimed", "iters": info["iters"]}


if __name__ == "__main__":
    main()
