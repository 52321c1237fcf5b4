#!/usr/bin/env python3
"""Benchmark of the BAMG-preconditioned FGMRES solve on one MI355X.

Workload (default): 256 x 256 periodic lattice, quenched U(1) links from 500
Metropolis sweeps at beta = 10 (seed 3), mass calibrated so that
min |eig(D)| ~ 1e-4, one complex Gaussian right-hand side (seed 103); the
hierarchy has 3 levels (4x4 then 2x2 aggregates, 8 test vectors, coarsest
level of dimension 8192 solved with its dense FP64 inverse), FGMRES(32) to a
relative residual of 1e-10 on the reduced system.  The headline variant is
mixed FP16 with a V(2,2) cycle and hipGraph replay; the other variants (FP64,
V(4,4), BF16 and FP32 storage, the FP32 copy of the coarsest inverse) are timed
beside it.  Setup is done once and
timed separately; every timed step is one full solve (reduction, FGMRES,
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
    ap.add_argument("--no-dhat", action="store_true", help="skip the Dhat and fine-sweep bandwidth points")
    ap.add_argument("--bandwidth-only", action="store_true",
                    help="time only the Dhat and fine-sweep bandwidth points (and the copy of COPY_MIB MiB), print "
                         "them and exit")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--batch", default="8,32", help="right-hand sides per batched solve (comma list, '' for none)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--precisions",
                    default="mixed_fp16+graphs+v22+bootV,mixed_fp16+graphs+v22+bootV+c32,fp64+graphs+v22+bootV,"
                            "mixed_fp16+graphs+v22,"
                            "fp64+graphs+v22,mixed_fp16+graphs+v22+bootW,mixed_fp16+graphs,fp64+graphs,mixed_fp16,"
                            "mixed_bf16+graphs+v22,mixed_fp32+graphs+v22,mixed_fp16+graphs+v22+bootV+W,"
                            "mixed_fp16+graphs+v22+bootV+K,fp64+graphs+v22+bootV+K",
                    help="single-RHS variants to time, <precision>[+graphs][+v22][+bootW|+bootV][+c32][+W|+K] "
                         "(graphs: iterations replayed as hipGraphs; v22: V(2,2) cycle instead of V(4,4) (W(2,2), "
                         "K(2,2) with +W, +K); bootW / bootV: bootstrap setup with the multigrid eigensolver, W or "
                         "super-V cycles; c32: the mixed cycle's coarsest solve reads an FP32 copy of the FP64 "
                         "inverse; W / K: W-cycle or K-cycle); the first one is the headline value; the batched "
                         "solves also run on the first +c32 variant")
    ap.add_argument("--serve", type=int, default=1000, help="requests per load point of the serving run (0: skip it)")
    ap.add_argument("--serve-loads", default="0.5,0.8,1.0",
                    help="offered loads of the serving run, as fractions of the measured capacity")
    ap.add_argument("--serve256", type=int, default=200,
                    help="requests of the 256^2-only served run at saturation (0: skip it)")
    ap.add_argument("--c4", type=int, default=1, help="time the 512^2 x 64 RHS batched solve (0: skip)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="set up the headline hierarchy, time only the roofline kernel and a plain copy of "
                         "COPY_MIB MiB (the scale of the HBM byte counters), print them and exit")
    return ap.parse_args()


COPY_MIB = 256


def variant(spec):
    """Solver parameters of a bench variant '<precision>[+graphs][+v22][+bootW|+bootV][+c32][+W|+K]'
    (bootW / bootV: bootstrap setup with the multigrid eigensolver, W or super-V
    setup cycles; c32: FP32 copy of the coarsest inverse in the mixed cycle;
    W / K: W-cycle or K-cycle instead of V)."""
    base, *opts = spec.split("+")
    kw = {"precision": PRECISIONS[base], "graphs": 1 if "graphs" in opts else 0}
    if "v22" in opts:
        kw.update(pre=2, post=2)
    if "bootW" in opts:
        kw.update(setup_mode=1)
    if "bootV" in opts:
        kw.update(setup_mode=2)
    if "c32" in opts:
        kw.update(coarsest_fp32=1)
    if "W" in opts:
        kw.update(cycle=1)
    if "K" in opts:
        kw.update(cycle=2)
    unknown = set(opts) - {"graphs", "v22", "bootW", "bootV", "c32", "W", "K"}
    if unknown:
        raise SystemExit(f"bench.py: unknown variant option(s) {sorted(unknown)} in {spec!r}")
    return base, kw


def copy_calibration(torch):
    """One plain copy kernel of known size (reads and writes COPY_MIB MiB):
    its FETCH_SIZE / WRITE_SIZE counters give the scale of those counters."""
    src = torch.ones(COPY_MIB * 2 ** 20 // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.mul(src[:1024], 1.0, out=dst[:1024])  # load the kernel before the timed call
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


def _server_with_fields(bamg, inputs, torch, names, tol, kw, slots=32):
    """A threaded server with the given fields registered and made resident by
    one warm-up request each (setup + one solve)."""
    sp = bamg.bamg_server_default_params(threaded=1, slots_per_field=slots)
    srv = bamg.bamg_server_create(sp)
    fids, Ns = [], []
    for name in names:
        w = inputs.workload(name)
        U = torch.from_numpy(inputs.load_gauge(w)).to("cuda:0")
        # the 512^2 field has 4 levels: K-cycle there (see c4_batched)
        kwf = dict(kw, cycle=2) if w["N"] >= 512 else kw
        p = bamg.bamg_default_params(N=w["N"], n_levels=w["n_levels"], seed=w["tv_seed"], **kwf)
        fids.append(bamg.bamg_server_add_field(srv, U, w["m"], p))
        Ns.append(w["N"])
        del U
    t0 = time.time()
    keep = []
    for f, N in zip(fids, Ns):
        B = torch.from_numpy(inputs.gaussian((1, 2 * N * N), 7000 + N)).to("cuda:0")
        X = torch.zeros_like(B)
        keep.append((bamg.bamg_server_submit(srv, f, B, X, 1, tol), B, X))
    for rid, B, X in keep:
        bamg.bamg_server_wait(srv, rid, 1)
    return srv, fids, Ns, time.time() - t0


def _request_stream(bamg, torch, np, srv, fids, Ns, which, nrhs, gaps, tol, pools):
    """Submit requests at their arrival times (gaps in s; 0: all at once), wait
    for all; the right-hand sides come from a per-field pool of 32 Gaussian
    vectors (request i takes the first nrhs of its field's pool), the outputs
    are allocated before the stream starts.  Returns the server's statistics
    with the wall time, convergence and the largest full-system residual."""
    outs = [torch.zeros(int(k), 2 * Ns[f] ** 2, dtype=torch.complex128, device="cuda:0")
            for f, k in zip(which, nrhs)]
    torch.cuda.synchronize()
    bamg.bamg_server_reset_stats(srv)
    ids = []
    t_start = time.perf_counter()
    t_next = t_start
    for i in range(len(which)):
        t_next += gaps[i]
        dt = t_next - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        ids.append(bamg.bamg_server_submit(srv, fids[which[i]], pools[which[i]], outs[i], int(nrhs[i]), tol))
    conv, worst_full, iters = True, 0.0, []
    for i, rid in enumerate(ids):
        st, infos = bamg.bamg_server_wait(srv, rid, int(nrhs[i]))
        conv = conv and st == 0 and all(v["relres_reduced"] <= tol for v in infos)
        worst_full = max([worst_full] + [v["relres_full"] for v in infos])
        iters.append(max(v["iters"] for v in infos))
    wall = time.perf_counter() - t_start
    stt = bamg.bamg_server_get_stats(srv)
    del outs
    return {"requests": stt["completed"], "rhs": stt["rhs_completed"], "wall_s": wall,
            "solves_per_s": stt["rhs_completed"] / wall, "requests_per_s": stt["completed"] / wall,
            "p50_ms": stt["p50_ms"], "p99_ms": stt["p99_ms"], "mean_ms": stt["mean_ms"], "max_ms": stt["max_ms"],
            "converged": conv, "max_relres_full": worst_full, "max_iters": int(max(iters)),
            "evictions": stt["evictions"], "setups": stt["setups"], "rounds": stt["rounds"]}


def serving(bamg, inputs, torch, np, n_req, loads, tol, kw, n_cal=200):
    """Solve requests over four gauge fields (64^2 beta=3, 128^2 beta=6, 256^2
    beta=10, 512^2 beta=10), each for one field chosen uniformly with 1-32
    right-hand sides (uniform), on a threaded server with memory admission and
    continuous batching (the headline solver parameters, 32 slots per field).
    Capacity is measured first: n_cal requests submitted at once, completed
    requests per second of the burst.  Then for each load factor f a Poisson
    stream of n_req requests arrives at f x capacity.  Latency is submit to
    completion per request, as the server measures it (nearest-rank
    percentiles)."""
    rng = np.random.default_rng(4242)
    t0 = time.time()
    srv, fids, Ns, t_warm = _server_with_fields(bamg, inputs, torch, SERVE_FIELDS, tol, kw)
    pools = [torch.from_numpy(inputs.gaussian((32, 2 * N * N), 9000 + N)).to("cuda:0") for N in Ns]
    which = rng.integers(0, len(fids), n_cal)
    nrhs = rng.integers(1, 33, n_cal)
    cal = _request_stream(bamg, torch, np, srv, fids, Ns, which, nrhs, np.zeros(n_cal), tol, pools)
    cap = cal["requests_per_s"]
    progress(f"serving capacity {cap:.1f} requests/s ({cal['solves_per_s']:.0f} solves/s)")
    points = []
    for f in loads:
        which = rng.integers(0, len(fids), n_req)
        nrhs = rng.integers(1, 33, n_req)
        gaps = rng.exponential(1.0 / (f * cap), n_req)
        r = _request_stream(bamg, torch, np, srv, fids, Ns, which, nrhs, gaps, tol, pools)
        r.update({"load": f, "offered_requests_per_s": f * cap, "offered_s": float(np.sum(gaps))})
        points.append(r)
        progress(f"serving load {f}: p50 {r['p50_ms']:.1f} ms p99 {r['p99_ms']:.1f} ms, {r['solves_per_s']:.0f} solves/s")
    bamg.bamg_server_free(srv)
    del pools
    torch.cuda.empty_cache()
    return {"fields": {n: {"N": N_} for n, N_ in zip(SERVE_FIELDS, Ns)}, "solver": kw,
            "solver_note": "K-cycle on the 512^2 field (4 levels), V elsewhere", "slots_per_field": 32,
            "requests_per_load": n_req, "capacity": cal, "loads": points, "setup_warmup_s": t_warm,
            "wall_s": time.time() - t0,
            "latency": "submit to completion per request (server clock), nearest-rank percentiles"}


def serving_256(bamg, inputs, torch, np, n_req, tol, kw):
    """The 256^2 field alone (beta = 10, min |eig D| ~ 1e-4), mixed FP16 with
    continuous batching: n_req requests of 1-32 right-hand sides submitted at
    once (the served throughput at saturation), every right-hand side to the
    same reduced residual 1e-10 as the single-RHS lines."""
    rng = np.random.default_rng(4343)
    srv, fids, Ns, t_warm = _server_with_fields(bamg, inputs, torch, ["c3_256_b10"], tol, kw)
    pools = [torch.from_numpy(inputs.gaussian((32, 2 * Ns[0] ** 2), 9500)).to("cuda:0")]
    which = np.zeros(n_req, dtype=int)
    nrhs = rng.integers(1, 33, n_req)
    r = _request_stream(bamg, torch, np, srv, fids, Ns, which, nrhs, np.zeros(n_req), tol, pools)
    bamg.bamg_server_free(srv)
    del pools
    torch.cuda.empty_cache()
    r.update({"field": "c3_256_b10", "solver": kw, "slots_per_field": 32, "setup_warmup_s": t_warm})
    return r


def c4_batched(bamg, inputs, torch, tol, kw, reps=2):
    """512^2, beta=10, 64 right-hand sides on one gauge field: the multi-RHS
    solve (MFMA coarse smoother, batched kernels) with the given solver
    parameters."""
    w = inputs.workload("c4_512_b10")
    N = w["N"]
    U = torch.from_numpy(inputs.load_gauge(w)).to("cuda:0")
    p = bamg.bamg_default_params(N=N, n_levels=w["n_levels"], seed=w["tv_seed"], **kw)
    out = {"workload": w["name"], "N": N, "nrhs": w["nrhs"], "m": w["m"], "precision": p.precision,
           "cycle": f"{'VWK'[p.cycle]}({p.pre},{p.post})", "graphs": bool(p.graphs)}
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
    """GB/s of the FP64 Dhat kernel from its compulsory bytes per apply: x read
    and y written for every right-hand side (16 N^2 each) and the links read
    once (32 N^2), (32 R + 32) N^2 in all; operator-only handle."""
    U = torch.from_numpy(inputs.gauge_random(N, 77)).to("cuda:0")
    p = bamg.bamg_default_params(N=N, n_levels=1)
    h = bamg.bamg_setup(U, -0.05, p)
    x = torch.from_numpy(inputs.gaussian((nrhs, N * N), 78)).to("cuda:0")
    y = torch.empty_like(x)
    t = time_launches(lambda: bamg.bamg_apply_dhat(h, x, y, nrhs), reps, 1, torch)
    bytes_ = (32.0 * nrhs + 32.0) * N * N
    bamg.bamg_free(h)
    del x, y, U
    torch.cuda.empty_cache()
    return {"N": N, "nrhs": nrhs, "us": t * 1e6, "GB/s": bytes_ / t / 1e9, "frac": bytes_ / t / 1e9 / HBM_PEAK_GBS}


def sweep_bandwidth(bamg, inputs, torch, N, nrhs, reps):
    """GB/s of one FP64 fine multicolour Kaczmarz sweep in the library's form for
    the size, from the method's algorithmic bytes per sweep: the links (32 N^2)
    and squared row norms (8 N^2) once and, per right-hand side, x read and
    written and b read (48 N^2): (40 + 48 R) N^2, 88 N^2 for one right-hand
    side.  design_GB/s counts this design's bytes instead: the stored slot
    blocks (36 complex per even site, 288 N^2) and x read and written per
    right-hand side, (288 + 32 R) N^2.  Operator-only handle."""
    U = torch.from_numpy(inputs.gauge_random(N, 77)).to("cuda:0")
    p = bamg.bamg_default_params(N=N, n_levels=1)
    h = bamg.bamg_setup(U, -0.05, p)
    x = torch.from_numpy(inputs.gaussian((nrhs, N * N), 79)).to("cuda:0")
    b = torch.zeros_like(x)
    t = time_launches(lambda: bamg.bamg_level_op(h, 0, bamg.OP_SWEEP, b, x, nrhs), reps, 1, torch)
    alg = (40.0 + 48.0 * nrhs) * N * N
    design = (288.0 + 32.0 * nrhs) * N * N
    bamg.bamg_free(h)
    del x, b, U
    torch.cuda.empty_cache()
    return {"N": N, "nrhs": nrhs, "us_per_sweep": t * 1e6, "GB/s": alg / t / 1e9, "frac": alg / t / 1e9 / HBM_PEAK_GBS,
            "design_GB/s": design / t / 1e9, "design_frac": design / t / 1e9 / HBM_PEAK_GBS}


BANDWIDTH_POINTS = ((256, 1, 200), (512, 64, 20), (4096, 1, 20))


def bandwidth_points(bamg, inputs, torch):
    return ([dhat_bandwidth(bamg, inputs, torch, n_, r_, reps) for (n_, r_, reps) in BANDWIDTH_POINTS],
            [sweep_bandwidth(bamg, inputs, torch, n_, r_, max(3, reps // 10)) for (n_, r_, reps) in BANDWIDTH_POINTS])


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU; --gpus must be 1 (a multi-GPU run would shard the "
              "right-hand sides over GPUs, one hierarchy per GPU)", file=sys.stderr)
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
    head_base, head_kw = variant(head)
    if args.bandwidth_only:
        d_, s_ = bandwidth_points(bamg, inputs, torch)
        print(json.dumps({"dhat_bandwidth": d_, "fine_sweep_bandwidth": s_, "copy_calibration": copy_calibration(torch)}),
              flush=True)
        return
    if args.roofline_only:
        p = bamg.bamg_default_params(N=N, n_levels=w["n_levels"], seed=w["tv_seed"], **head_kw)
        h = bamg.bamg_setup(U, w["m"], p)
        dom, others = roofline(bamg, torch, h, head_base, head_kw.get("coarsest_fp32", 0), p.pre + p.post)
        out = {"workload": w["name"], "precision": head_base, "roofline": dom, "roofline_others": others,
               "copy_calibration": copy_calibration(torch)}
        bamg.bamg_free(h)
        print(json.dumps(out), flush=True)
        return
    results, hier, xs = {}, {}, {}
    for prec in precs:
        _, kw = variant(prec)
        p = bamg.bamg_default_params(N=N, n_levels=w["n_levels"], seed=w["tv_seed"], **kw)
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
        cyc = "VWK"[p.cycle]
        results[prec] = {
            "solves_per_s": args.steps / t_all, "ms_per_solve": 1e3 * t_all / args.steps,
            "p10_ms": float(np.percentile(ms, 10)), "p50_ms": statistics.median(ms),
            "p90_ms": float(np.percentile(ms, 90)), "p99_ms": float(np.percentile(ms, 99)),
            "iters": infos[-1]["iters"], "relres_reduced": infos[-1]["relres_reduced"],
            "converged": all(i["relres_reduced"] <= args.tol for i in infos), "setup_s": t_setup,
            "relres_full": infos[-1]["relres_full"],
            "levels": bamg.bamg_n_levels(h), "cycle": f"{cyc}({p.pre},{p.post})", "graphs": bool(p.graphs),
            "setup": {0: "relax-fit passes", 1: "bootstrap W cycles", 2: "bootstrap super-V"}[p.setup_mode],
        }
        hier[prec] = h
        xs[prec] = x.cpu().numpy()
        progress(f"{prec}: {results[prec]['solves_per_s']:.1f} solves/s")
    # error of every variant against the FP64 solve with the same cycle
    for prec in precs:
        base, kw = variant(prec)
        key = lambda kw_: (kw_.get("pre"), kw_.get("post"), kw_.get("setup_mode"), kw_.get("cycle", 0))
        refs = [q for q in precs if variant(q)[0] == "fp64" and key(variant(q)[1]) == key(kw)]
        if base != "fp64" and refs:
            results[prec]["rel_err_vs_fp64"] = float(np.linalg.norm(xs[prec] - xs[refs[0]]) /
                                                     np.linalg.norm(xs[refs[0]]))
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
        "dtype": DTYPES[head_base],
        "data": "synthetic",
        "config": {
            "workload": w["name"], "N": N, "beta": w["beta"], "metropolis_sweeps": w["sweeps"],
            "m": w["m"], "min_abs_eig_D": w["min_abs_eig_D"], "levels": n_levels,
            "aggregates": "4x4 half-x, then 2x2", "test_vectors": 8, "cycle": r0["cycle"],
            "coarsest": "dense inverse, FP64" if not head_kw.get("coarsest_fp32") else "dense inverse, FP64 built, FP32 applied",
            "hipgraph": r0["graphs"], "setup": r0["setup"],
            "krylov": "FGMRES(32)", "tol": args.tol, "nrhs": 1, "precision": head_base, "variant": head,
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
    bvars = [head] + [q for q in precs if "c32" in q.split("+")[1:] and q != head][:1]
    for bv in bvars:
        hb = hier[bv]
        for R in [int(v) for v in args.batch.split(",") if v.strip()]:
            B = torch.from_numpy(inputs.gaussian((R, 2 * N * N), w["rhs_seed"] + 1000)).to("cuda:0")
            X = torch.zeros_like(B)
            bamg.bamg_solve_batch(hb, B, X, R, args.tol)
            torch.cuda.synchronize()
            tb0 = time.perf_counter()
            for _ in range(args.batch_steps):
                st, infs = bamg.bamg_solve_batch(hb, B, X, R, args.tol)
            torch.cuda.synchronize()
            tb = (time.perf_counter() - tb0) / args.batch_steps
            batched.append({"nrhs": R, "precision": bv, "solves_per_s": R / tb, "ms_per_batch": 1e3 * tb,
                            "max_iters": max(i["iters"] for i in infs),
                            "converged": all(i["relres_reduced"] <= args.tol for i in infs)})
            del B, X
            progress(f"batched {bv} R={R}: {batched[-1]['solves_per_s']:.1f} solves/s")
    if batched:
        out["batched"] = batched

    # ---- 512^2 x 64 right-hand sides on one field (multi-RHS form)
    if args.c4:
        # the 512^2 batch and the serving mix use the headline parameters with the
        # relax-fit setup (at 512^2 it gives fewer iterations than the bootstrap
        # cycles, and the serving warm-up builds four hierarchies)
        # 4 levels: the K-cycle (two GCR steps on level 2 per visit) keeps the
        # iteration count of the 3-level hierarchies, where one V visit of level 2
        # is a poor coarse solve; the V-cycle line is kept beside it
        multi_kw = {k: v for k, v in head_kw.items() if k != "setup_mode"}
        out["c4_512x64"] = c4_batched(bamg, inputs, torch, args.tol, dict(multi_kw, cycle=2))
        out["c4_512x64"]["v_cycle"] = c4_batched(bamg, inputs, torch, args.tol, multi_kw)
        progress(f"512^2 x 64: {out['c4_512x64']['solves_per_s']:.1f} solves/s "
                 f"(V-cycle {out['c4_512x64']['v_cycle']['solves_per_s']:.1f})")

    # ---- serving: Poisson arrivals over four fields at 0.5 / 0.8 / 1.0 x capacity
    multi_kw = {k: v for k, v in head_kw.items() if k != "setup_mode"}
    if args.serve > 0:
        loads = [float(v) for v in args.serve_loads.split(",") if v.strip()]
        out["serving"] = serving(bamg, inputs, torch, np, args.serve, loads, args.tol, multi_kw)
        out["serving_p99_ms"] = {str(pt["load"]): pt["p99_ms"] for pt in out["serving"]["loads"]}
    # ---- the served form at 256^2 against the FP64 single-RHS solve at the same tolerance
    if args.serve256 > 0:
        s256 = serving_256(bamg, inputs, torch, np, args.serve256, args.tol, multi_kw)
        ref = next((q for q in precs if q.split("+")[0] == "fp64" and "v22" in q.split("+")
                    and not any(o_ in q.split("+") for o_ in ("bootV", "bootW", "W", "K"))), None)
        if ref is not None:
            s256["fp64_single_rhs_line"] = ref
            s256["fp64_single_rhs_solves_per_s"] = results[ref]["solves_per_s"]
            s256["served_over_fp64_single"] = s256["solves_per_s"] / results[ref]["solves_per_s"]
        out["serving_256"] = s256
        progress(f"serving 256^2: {s256['solves_per_s']:.0f} solves/s")

    # ---- Dhat ("D_oe") bandwidth: cache-resident, batched, cache-busting
    if not args.no_dhat:
        out["dhat_bandwidth"], out["fine_sweep_bandwidth"] = bandwidth_points(bamg, inputs, torch)
        progress("dhat and fine-sweep bandwidth")

    # ---- roofline of the dominant kernel of the solve
    if not args.no_roofline:
        ph = bamg.bamg_default_params(**head_kw)
        out["roofline"], out["roofline_others"] = roofline(bamg, torch, h, head_base, head_kw.get("coarsest_fp32", 0),
                                                           ph.pre + ph.post)
        if head_base != "fp64":
            hm = next((hier[q] for q in precs if "c32" in q.split("+")[1:]), h)
            out["mfma"] = mfma_utilisation(bamg, torch, hm)
        progress("roofline")

    # ---- the stand-alone convergence rate of Sec. 4 of the timed hierarchies
    out["rho_standalone"] = {q: convergence_rate(bamg, inputs, torch, hier[q], N) for q in precs
                             if q == head or variant(q)[1].get("cycle")}
    progress("stand-alone rates")

    # ---- CPU oracle on a bounded sample of the same workload
    if not args.no_cpu_baseline:
        ph = bamg.bamg_default_params(**head_kw)
        Ps = [bamg.bamg_export_level(h, l, P=True, D=False)[0] for l in range(n_levels - 1)]
        out["cpu_baseline"] = cpu_baseline(w, U_np, args.tol, Ps, ph.pre, ph.post)
        progress("cpu baseline")

    for hh in hier.values():
        bamg.bamg_free(hh)
    print(json.dumps(out), flush=True)


# Bytes of the three kernels that take the solve's time, per launch.  The
# roofline fraction uses the algorithmic (compulsory) bytes of the method:
#  - fine sweep: 88 N^2 B per 16-colour sweep in FP64 (x read and written,
#    b, the links, the squared row norms), 44 N^2 B in FP32; a colour pass is
#    1/16 of it;
#  - coarse colour pass: the operator rows of the colour's sites, 7 blocks of
#    16 x 16 entries per site in the operator's storage type (28 KiB FP64,
#    7 KiB FP16);
#  - coarsest product: the entries of the inverse the product must read (its
#    64 x 64 blocks on and above the diagonal: the inverse is gamma5-Hermitian,
#    so they fix the rest) and the two vectors.
# This design's own bytes are reported beside them (design_bytes_per_launch):
#  - fine colour pass: per even site of the colour its 9 x 4 stored couplings,
#    2 right-hand-side entries and the 9 x 2 unknowns of its support read and
#    written; the blocked sweep: 36 stored couplings, b, x read and written once
#    per even site;
#  - coarse colour pass: the operator rows, the 16 x 16 smoother matrix Kinv,
#    16 right-hand-side entries and the 7 x 16 unknowns of the support read
#    and written.
def fine_sweep_alg_bytes(N, s_vec):
    """88 N^2 B (FP64) per sweep: x read + written 32 N^2, b 16 N^2, links 32 N^2,
    row norms 8 N^2; halved for FP32 (s_vec = 8)."""
    return 88.0 * N * N * s_vec / 16.0


def fine_sweep_site_bytes(s_vec):
    return 36 * s_vec + 2 * s_vec + 2 * 2 * s_vec


def fine_sweep_blocked(N, nrhs, s_vec):
    """Whether the library runs a level-0 sweep as one launch blocked in LDS
    (fine.hip: tiles need N >= 64 and N/2 a multiple of 8, and x of at most
    1 MiB)."""
    return N >= 64 and N % 16 == 0 and N * N * nrhs * s_vec <= 1 << 20


def fine_site_bytes(s_vec):
    return 36 * s_vec + 2 * s_vec + 2 * 9 * 2 * s_vec


def coarse_site_alg_bytes(s_op):
    return 7 * 256 * s_op


def coarse_site_bytes(s_op, s_vec):
    return 7 * 256 * s_op + 256 * s_vec + 16 * s_vec + 2 * 7 * 16 * s_vec


def coarse_pair_wg_bytes(s_op, s_vec):
    """Bytes one work-group of the fused colour pair reads and writes: the
    rows, Kinv and b of its three projected sites (t1, t2, s), x on the 15
    sites of their supports, and 8 sites written."""
    return 3 * (7 * 256 * s_op + 256 * s_vec + 16 * s_vec) + 15 * 16 * s_vec + 8 * 16 * s_vec


def coarse_pairs_used(inf):
    """Whether the library runs a level's single-RHS sweep as fused colour
    pairs (coarse.hip: the 8-colouring on extents that are multiples of 8)."""
    return inf["colours"] == 8 and inf["ex"] % 8 == 0 and inf["ey"] % 8 == 0


VEC_BYTES = {"fp64": 16, "mixed_fp32": 8, "mixed_fp16": 8, "mixed_bf16": 8}
OP_BYTES = {"fp64": 16, "mixed_fp32": 8, "mixed_fp16": 4, "mixed_bf16": 4}

# HBM byte counters of the same launches (rocprofv3 --pmc FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, median over the roofline launches), each
# divided by what the counter reads per KiB moved by a plain 256 MiB copy
# kernel in the same run.  Valid only for the kernel source they were taken on
# (sha256 of the kernel's file); any change to it makes the traffic null.
COPY_SCALE = {"fetch_per_kib": 131090.8 / 262144.0, "write_per_kib": 262144.0 / 262144.0}
PMC_PROFILE = "profiles/roofline_kernels_c3_256_mixed_fp16_pmc.md"
PMC_TRAFFIC = {
    ("fine_sweep", "mixed_fp16"): {"src": "fine.hip",
                                   "sha256": "607b1a3a175d23870f457411a1aba9f6b8c81191c9bbe5eb94820270b6cc3a23",
                                   "fetch_kib": 10143.5, "write_kib": 640.0, **COPY_SCALE},
    ("coarse_pair", "mixed_fp16"): {"src": "coarse.hip",
                                    "sha256": "2b1b26e11d8d45d10fb43512862560425d957eaf5981e90d62072440ad9955a4",
                                    "fetch_kib": 2679.0, "write_kib": 256.0, **COPY_SCALE},
    # the packed products and their reductions, per call (the sum of the two kernels' counters):
    # the FP64 blocks (headline) and their FP32 copy (+c32)
    ("dense_g5", "mixed_fp16"): {"src": "dense.hip",
                                 "sha256": "fcad5180b394c3da8894dd3f729d70e9d06cb378996fb119a42d132b8d768ba2",
                                 "fetch_kib": 265259.5 + 8208.0, "write_kib": 16389.1 + 128.0, **COPY_SCALE},
    ("dense32_g5", "mixed_fp16"): {"src": "dense.hip",
                                   "sha256": "fcad5180b394c3da8894dd3f729d70e9d06cb378996fb119a42d132b8d768ba2",
                                   "fetch_kib": 132908.5 + 8208.0, "write_kib": 16384.0 + 64.0, **COPY_SCALE},
}


def pmc_traffic(kind, prec):
    import hashlib
    e = PMC_TRAFFIC.get((kind, prec))
    if e is None:
        return None
    with open(os.path.join(ROOT, "paper_1308_5992_amd", "csrc", e["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != e["sha256"]:
            return None
    return 1024.0 * (e["fetch_kib"] / e["fetch_per_kib"] + e["write_kib"] / e["write_per_kib"])


def _roof(kname, kind, prec, alg_bytes, design_bytes, t, basis):
    achieved = alg_bytes / t / 1e9
    traffic = pmc_traffic(kind, prec)
    return {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "bytes per launch",
            "avg_launch_us": t * 1e6, "bytes_per_launch": alg_bytes, "bytes_basis": basis,
            "design_bytes_per_launch": design_bytes, "design_over_algorithmic": design_bytes / alg_bytes,
            "traffic_over_algorithmic": None if traffic is None else traffic / alg_bytes}


def roofline(bamg, torch, h, prec, c32=0, sweeps=8):
    """The kernels that take the solve's time, each timed with HIP events on
    the library's stream (torch's current stream) over back-to-back calls of
    the level hooks: the fine smoother on level 0, the coarse colour pass on
    level 1 (ncol launches per sweep) and the coarsest dense product (one
    call per cycle: with the FP64 inverse the packed product and the reduction
    of its partial products).  A mixed hierarchy is driven through the
    complex64 hooks.
    The fine smoother is either 16 colour passes per sweep or, where the
    library blocks the sweep in LDS, one launch per sweep; the hook then also
    copies x once (it keeps x in place, the kernel writes a second copy), so
    the time per call is an upper bound of the kernel's.  The coarsest product
    is the FP64 inverse's (op 4) or, with c32, its FP32 copy's (op 12).
    `sweeps` is the smoothing sweeps per cycle (pre + post); the dominant
    kernel is the one with the largest time per cycle.  Returns (dominant,
    [others])."""
    mixed = prec != "fp64"
    dt = torch.complex64 if mixed else torch.complex128
    sweep = bamg.OP_SWEEP_F32 if mixed else bamg.OP_SWEEP
    tname = "float" if mixed else "double"
    sname = {"fp64": "cx<double>", "mixed_fp32": "cx<float>", "mixed_fp16": "hcx", "mixed_bf16": "bcx"}[prec]
    out = []  # (entry, time per cycle)
    # fine smoother, level 0
    inf = bamg.bamg_level_info(h, 0)
    N = int(round(inf["n"] ** 0.5))  # level 0: N^2 / 2 even sites, 2 unknowns each
    sv = VEC_BYTES[prec]
    xb = torch.zeros(inf["n"], dtype=dt, device="cuda:0")
    bb = torch.ones(inf["n"], dtype=dt, device="cuda:0")
    fbasis = f"{88 * sv // 16} N^2 B per sweep (x read and written, b, links, row norms)"
    if fine_sweep_blocked(N, 1, sv):
        t = time_launches(lambda: bamg.bamg_level_op(h, 0, sweep, bb, xb, 1), 50, 1, torch)
        e = _roof(f"k_kaczmarz_fine_sweep<{tname}> (level 0, one 16-colour sweep of {inf['n'] // 2} sites per launch; "
                  f"timed per sweep call, which also copies x)", "fine_sweep", prec,
                  fine_sweep_alg_bytes(N, sv), inf["n"] // 2 * fine_sweep_site_bytes(sv), t, fbasis)
        out.append((e, t * sweeps))
    else:
        nsite = inf["n"] // 2 // 16  # even sites per colour
        t = time_launches(lambda: bamg.bamg_level_op(h, 0, sweep, bb, xb, 1), 50, 16, torch)
        e = _roof(f"k_kaczmarz_fine<{tname}, 1> (level 0, {nsite} sites per launch)", "fine", prec,
                  fine_sweep_alg_bytes(N, sv) / 16, nsite * fine_site_bytes(sv), t, fbasis + ", 1/16 per colour pass")
        out.append((e, t * 16 * sweeps))
    L = bamg.bamg_n_levels(h)
    if L > 2:  # coarse smoother, level 1
        inf = bamg.bamg_level_info(h, 1)
        ns, ncol = inf["ex"] * inf["ey"], inf["colours"]
        xb = torch.zeros(inf["n"], dtype=dt, device="cuda:0")
        bb = torch.ones(inf["n"], dtype=dt, device="cuda:0")
        so = OP_BYTES[prec]
        if coarse_pairs_used(inf):
            # two colours per launch: ncol / 2 launches per sweep
            per = ns // ncol
            t = time_launches(lambda: bamg.bamg_level_op(h, 1, sweep, bb, xb, 1), 50, ncol // 2, torch)
            e = _roof(f"k_kaczmarz_coarse_pair<{tname},{sname}> (level 1, colours c and c + 1, 2 x {per} sites "
                      f"per launch)", "coarse_pair", prec, 2 * per * coarse_site_alg_bytes(so),
                      per * coarse_pair_wg_bytes(so, sv), t,
                      f"the operator rows of the two colours' sites: 7 x 256 entries of {so} B per site")
            out.append((e, t * (ncol // 2) * sweeps))
        else:
            t = time_launches(lambda: bamg.bamg_level_op(h, 1, sweep, bb, xb, 1), 50, ncol, torch)
            e = _roof(f"k_kaczmarz_coarse<{tname},{sname}> (level 1, {ns // ncol} sites per launch)", "coarse",
                      prec, ns // ncol * coarse_site_alg_bytes(so), ns // ncol * coarse_site_bytes(so, sv), t,
                      f"the operator rows of the colour's sites: 7 x 256 entries of {so} B per site")
            out.append((e, t * ncol * sweeps))
    if L > 1:  # coarsest product
        inf = bamg.bamg_level_info(h, L - 1)
        n = inf["n"]
        cdt = torch.complex64 if c32 else torch.complex128
        xb = torch.zeros(n, dtype=cdt, device="cuda:0")
        bb = torch.ones(n, dtype=cdt, device="cuda:0")
        op = bamg.OP_COARSEST_F32 if c32 else bamg.OP_COARSEST
        t = time_launches(lambda: bamg.bamg_level_op(h, L - 1, op, bb, xb, 1), 20, 1, torch)
        half = "the 64 x 64 blocks of the gamma5-Hermitian inverse on and above the diagonal, and x, y"
        if c32 and n % 64 == 0:
            # the FP32 copy of the packed blocks (complex64 entries), x and y complex64
            b_ = 8.0 * (n * n / 2 + 32 * n) + 16.0 * n
            e = _roof(f"k_dense_mv_g5<cx<float>> + k_dense_mv_g5_reduce (coarsest inverse, FP32 copy of the packed "
                      f"gamma5 half, n = {n}; timed per call)", "dense32_g5", prec, b_, b_, t, half + " (FP32)")
        elif c32:
            b_ = 8.0 * n * n + 16.0 * n
            e = _roof(f"k_dense_mv32 (coarsest inverse, n = {n})", "dense32", prec, b_, b_, t, "the FP32 inverse, x, y")
        elif n % 64 == 0:
            # the call is the block product and the reduction of its partial products
            b_ = 16.0 * (n * n / 2 + 32 * n) + 32.0 * n
            e = _roof(f"k_dense_mv_g5 + k_dense_mv_g5_reduce (coarsest inverse, packed gamma5 half, n = {n}; "
                      f"timed per call)", "dense_g5", prec, b_, b_, t, half)
        else:
            b_ = 16.0 * n * n + 32.0 * n
            e = _roof(f"k_dense_mv (coarsest inverse, n = {n})", "dense", prec, b_, b_, t, "the inverse, x, y")
        out.append((e, t))
    for e, tc in out:
        e["us_per_cycle"] = tc * 1e6
    out.sort(key=lambda et: -et[1])
    return out[0][0], [e for e, _ in out[1:]]


MFMA_F32_PEAK_TFLOPS = 157.3  # dense FP32 matrix peak of the MI355X
MFMA_F64_PEAK_TFLOPS = 78.6   # dense FP64 matrix peak of the MI355X


def mfma_utilisation(bamg, torch, h, R=32):
    """Achieved FP32 matrix-core rate of the MFMA kernels of the batched solve
    at R right-hand sides, timed with HIP events like the roofline kernels:
    - the coarse block-stencil smoother k_kaczmarz_coarse_mfma4 on level 1
      (per site and 16 right-hand sides 240 v_mfma_f32_16x16x4f32 of 2048 flops:
      residual 112, Kinv step 16 (counted once although the four waves each
      form it), update 112), one launch per colour;
    - the split-K product with the FP64 coarsest inverse, k_dense_mm64 (op 4;
      8 n^2 R flops, FP64 matrix peak; the call's small reduction launch is
      included in its time);
    - with an FP32 copy of the coarsest inverse (op 12), the split-K product
      k_dense_mm32 (likewise)."""
    out = []
    L = bamg.bamg_n_levels(h)
    if L > 2:
        inf = bamg.bamg_level_info(h, 1)
        ns, ncol, n = inf["ex"] * inf["ey"], inf["colours"], inf["n"]
        xb = torch.zeros(R, n, dtype=torch.complex64, device="cuda:0")
        bb = torch.ones(R, n, dtype=torch.complex64, device="cuda:0")
        t = time_launches(lambda: bamg.bamg_level_op(h, 1, bamg.OP_SWEEP_F32, bb, xb, R), 20, ncol, torch)
        fl = (ns // ncol) * ((R + 15) // 16) * 240 * 2048.0
        out.append({"kernel": f"k_kaczmarz_coarse_mfma4 (level 1, {ns // ncol} sites x {R} RHS per launch)",
                    "flops_per_launch": fl, "avg_launch_us": 1e6 * t, "achieved_tflops": fl / t / 1e12,
                    "peak_tflops": MFMA_F32_PEAK_TFLOPS, "frac": fl / t / 1e12 / MFMA_F32_PEAK_TFLOPS})
    p = bamg.bamg_level_info(h, L - 1) if L > 1 else None
    if p is not None:
        n = p["n"]
        xb = torch.zeros(R, n, dtype=torch.complex128, device="cuda:0")
        bb = torch.ones(R, n, dtype=torch.complex128, device="cuda:0")
        t = time_launches(lambda: bamg.bamg_level_op(h, L - 1, bamg.OP_COARSEST, bb, xb, R), 10, 1, torch)
        fl = 8.0 * n * n * R
        out.append({"kernel": f"k_dense_mm64 (coarsest inverse, FP64, n = {n}, {R} RHS)", "flops_per_launch": fl,
                    "avg_launch_us": 1e6 * t, "achieved_tflops": fl / t / 1e12, "peak_tflops": MFMA_F64_PEAK_TFLOPS,
                    "frac": fl / t / 1e12 / MFMA_F64_PEAK_TFLOPS})
        del xb, bb
        xb = torch.zeros(R, n, dtype=torch.complex64, device="cuda:0")
        bb = torch.ones(R, n, dtype=torch.complex64, device="cuda:0")
        try:
            t = time_launches(lambda: bamg.bamg_level_op(h, L - 1, bamg.OP_COARSEST_F32, bb, xb, R), 10, 1, torch)
        except bamg.BamgError:  # no FP32 copy of the coarsest inverse on this hierarchy
            return out
        fl = 8.0 * n * n * R
        out.append({"kernel": f"k_dense_mm32 (coarsest inverse, n = {n}, {R} RHS)", "flops_per_launch": fl,
                    "avg_launch_us": 1e6 * t, "achieved_tflops": fl / t / 1e12, "peak_tflops": MFMA_F32_PEAK_TFLOPS,
                    "frac": fl / t / 1e12 / MFMA_F32_PEAK_TFLOPS})
    return out


def cpu_baseline(w, U_np, tol, Ps, pre, post, reps=3):
    """The oracle (plain C++ FP64; test infrastructure, loaded only here) solving
    the same 256^2 system with the hierarchy of the GPU's FP64 line
    'fp64+graphs+v22+bootV': the interpolation operators of the headline setup
    (bootstrap super-V), the oracle's own Galerkin products, smoothers and
    V(pre,post) cycle, the 8192-dim coarsest level factored by LAPACK (setup,
    untimed).  Timed: full solves (reduction, FGMRES(32), reconstruction) to tol.
      single thread: `reps` solves of the benchmark's right-hand side one after
        another, median;
      all host cores: as many threads as cores, each solving its own
        right-hand side at the same time (the oracle's solve is sequential
        code; right-hand sides are independent), solves / wall time, median of
        `reps` rounds."""
    import inputs
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    N = w["N"]
    t0 = time.perf_counter()
    o = oracle.Hierarchy.from_interpolation(U_np, w["m"], Ps, pre=pre, post=post)
    t_setup = time.perf_counter() - t0
    b = inputs.gaussian(2 * N * N, w["rhs_seed"])
    single, iters = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        st, xo, info = o.solve(b, tol=tol)
        single.append(time.perf_counter() - t0)
        iters = info["iters"]
    cores = len(os.sched_getaffinity(0))
    B = [inputs.gaussian(2 * N * N, w["rhs_seed"] + 2000 + i) for i in range(cores)]
    rates, conv = [], True
    with ThreadPoolExecutor(max_workers=cores) as ex:
        for _ in range(reps):
            t0 = time.perf_counter()
            res = list(ex.map(lambda bb: o.solve(bb, tol=tol), B))
            rates.append(cores / (time.perf_counter() - t0))
            conv = conv and all(r_[0] == 0 for r_ in res)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    t1 = statistics.median(single)
    return {"value": statistics.median(rates), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} rounds of {cores} concurrent full solves (one per core, independent right-hand "
                      f"sides) of the same 256^2 system, median; oracle FP64 with the headline setup's P, "
                      f"3 levels, V({pre},{post}), FGMRES(32) to {tol:g}",
            "config": {"workload": w["name"], "levels": len(Ps) + 1, "cycle": f"V({pre},{post})",
                       "setup": "the GPU's bootstrap super-V interpolation", "precision": "fp64",
                       "coarsest": "LAPACK LU of the oracle's Galerkin operator (setup)",
                       "gpu_line": "precisions['fp64+graphs+v22+bootV']"},
            "single_thread": {"value": 1.0 / t1, "unit": "solves/s", "median_s": t1, "runs_s": single,
                              "iters": iters},
            "all_core_rounds_solves_per_s": rates, "converged": conv, "twin_setup_s": t_setup,
            "host_cores_available": cores, "host_cpu": model}


def convergence_rate(bamg, inputs, torch, h, N, iters=12):
    """The stand-alone rate of Sec. 4, rho = ||e^nu|| / ||e^{nu-1}||: the solver's
    preconditioner used on its own, x <- x + M(0 - Dhat x) from a Gaussian start
    (the iterate is the error)."""
    import numpy as np
    x = torch.from_numpy(inputs.gaussian(N * N, 4321)).to("cuda:0")
    norms = bamg.bamg_stationary(h, x, iters)
    r = norms[1:] / norms[:-1]
    return {"rho_last": float(r[-1]), "rho_geomean_last5": float(np.exp(np.mean(np.log(r[-5:])))),
            "iters": iters, "rates": [float(v) for v in r]}


if __name__ == "__main__":
    main()
