"""Serving with continuous batching (bamg_server_*): requests for several
gauge fields join and leave the running batch; every right-hand side's result
must be bitwise the one it gets alone (the slot engine treats right-hand sides
independently with fixed reduction orders), and correct against the Wilson
operator.  Memory admission and eviction, and per-request failures, are
checked through the statistics and statuses; the footprint estimate that
admission uses is checked against what a setup allocates on the device."""
import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-10


@pytest.fixture(scope="module")
def bamg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_5992_amd as b
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda:0")


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def fields():
    """Two fields of different size and precision: the 32^2 beta=3 workload
    (FP64, 2 levels) and a 64^2 beta=3 field (mixed FP16, 3 levels)."""
    w = inputs.workload("c1_32_b3")
    UA = inputs.load_gauge(w)
    UB = inputs.gauge_metropolis(64, 3.0, 40, 5)
    return [
        dict(U=UA, m=w["m"], N=32, kw=dict(n_levels=w["n_levels"], seed=w["tv_seed"], precision=0)),
        dict(U=UB, m=-0.05, N=64, kw=dict(n_levels=3, max_coarse=512, seed=11, precision=1)),
    ]


def add_fields(bamg, srv, fields):
    ids = []
    for f in fields:
        p = bamg.bamg_default_params(N=f["N"], **f["kw"])
        ids.append(bamg.bamg_server_add_field(srv, dev(f["U"]), f["m"], p))
    return ids


def rhs(N, nrhs, seed):
    return inputs.gaussian((nrhs, 2 * N * N), seed)


def drive(bamg, srv, pending):
    """Run rounds until every request in `pending` (id -> nrhs) is finished."""
    out = {}
    for _ in range(100000):
        bamg.bamg_server_progress(srv)
        for rid in list(pending):
            st, infos = bamg.bamg_server_wait(srv, rid, pending[rid], 0.0)
            if st != bamg.BAMG_PENDING:
                out[rid] = (st, infos)
                del pending[rid]
        if not pending:
            return out
    raise AssertionError("requests did not finish")


def full_relres(f, B, X):
    return max(np.linalg.norm(B[r] - oracle.wilson_apply(f["U"], f["m"], X[r])) / np.linalg.norm(B[r])
               for r in range(B.shape[0]))


def test_results_are_the_same_alone_and_in_the_mix(bamg, fields):
    srv = bamg.bamg_server_create(bamg.bamg_server_default_params(threaded=0, slots_per_field=8))
    fa, fb = add_fields(bamg, srv, fields)
    NA, NB = fields[0]["N"], fields[1]["N"]
    BA, BB = rhs(NA, 3, 901), rhs(NB, 2, 902)
    # alone
    XA = torch.zeros(3, 2 * NA * NA, dtype=torch.complex128, device="cuda:0")
    dA = dev(BA)  # B must stay alive until the request finishes
    ra = bamg.bamg_server_submit(srv, fa, dA, XA, 3, TOL)
    res = drive(bamg, srv, {ra: 3})
    assert res[ra][0] == 0
    XB = torch.zeros(2, 2 * NB * NB, dtype=torch.complex128, device="cuda:0")
    dB = dev(BB)
    rb = bamg.bamg_server_submit(srv, fb, dB, XB, 2, TOL)
    res = drive(bamg, srv, {rb: 2})
    assert res[rb][0] == 0
    XA_alone, XB_alone = XA.cpu().numpy(), XB.cpu().numpy()
    it_alone = [i["iters"] for i in res[rb][1]]
    # the mix: other requests of both fields before, during and after, more
    # right-hand sides than slots (8 per field), arrivals between rounds
    keep, pend = [], {}

    def submit(f, N, nrhs, seed, B=None):
        B = rhs(N, nrhs, seed) if B is None else B
        dBm = dev(B)
        X = torch.zeros(nrhs, 2 * N * N, dtype=torch.complex128, device="cuda:0")
        rid = bamg.bamg_server_submit(srv, f, dBm, X, nrhs, TOL)
        keep.append((rid, B, dBm, X))
        pend[rid] = nrhs
        return rid

    submit(fa, NA, 5, 911)
    submit(fb, NB, 3, 912)
    for _ in range(3):
        bamg.bamg_server_progress(srv)
    ra2 = submit(fa, NA, 3, 0, BA)
    submit(fb, NB, 6, 913)
    for _ in range(2):
        bamg.bamg_server_progress(srv)
    rb2 = submit(fb, NB, 2, 0, BB)
    submit(fa, NA, 2, 914)
    res = drive(bamg, srv, pend)
    for rid, B, _, X in keep:
        st, infos = res[rid]
        assert st == 0, (rid, st)
        assert all(i["relres_reduced"] <= TOL for i in infos)
    XA_mix = [k[3] for k in keep if k[0] == ra2][0].cpu().numpy()
    XB_mix = [k[3] for k in keep if k[0] == rb2][0].cpu().numpy()
    assert np.array_equal(XA_mix, XA_alone)
    assert np.array_equal(XB_mix, XB_alone)
    assert [i["iters"] for i in res[rb2][1]] == it_alone
    # correct against the full Wilson operator (FP64 outer residual 1e-10)
    assert full_relres(fields[0], BA, XA_alone) < 2e-10
    assert full_relres(fields[1], BB, XB_alone) < 2e-10
    st = bamg.bamg_server_get_stats(srv)
    log(f"serving mix: {st}")
    assert st["completed"] == 8 and st["rhs_completed"] == 26 and st["setups"] == 2 and st["evictions"] == 0
    # the same as bamg_solve_batch on a hierarchy with the same parameters
    f0 = fields[0]
    h = bamg.bamg_setup(dev(f0["U"]), f0["m"], bamg.bamg_default_params(N=NA, **f0["kw"]))
    Xs = torch.zeros(3, 2 * NA * NA, dtype=torch.complex128, device="cuda:0")
    stb, _ = bamg.bamg_solve_batch(h, dev(BA), Xs, 3, TOL)
    assert stb == 0
    d = np.linalg.norm(Xs.cpu().numpy() - XA_alone) / np.linalg.norm(XA_alone)
    log(f"server vs bamg_solve_batch: rel diff {d:.2e} (bitwise {np.array_equal(Xs.cpu().numpy(), XA_alone)})")
    assert d < 1e-12
    bamg.bamg_server_free(srv)


def test_threaded_server_concurrent_requests(bamg, fields):
    srv = bamg.bamg_server_create(bamg.bamg_server_default_params(threaded=1, slots_per_field=16))
    fa, fb = add_fields(bamg, srv, fields)
    NA, NB = fields[0]["N"], fields[1]["N"]
    reqs = [(fa, NA, 4, 921), (fb, NB, 3, 922), (fa, NA, 1, 923), (fb, NB, 5, 924), (fa, NA, 7, 925)]
    alone = []
    for f, N, k, seed in reqs:  # one at a time
        B = rhs(N, k, seed)
        X = torch.zeros(k, 2 * N * N, dtype=torch.complex128, device="cuda:0")
        dBm = dev(B)
        rid = bamg.bamg_server_submit(srv, f, dBm, X, k, TOL)
        st, infos = bamg.bamg_server_wait(srv, rid, k, 60000.0)
        assert st == 0
        alone.append(X.cpu().numpy())
    live = []
    for f, N, k, seed in reqs:  # all at once
        B = rhs(N, k, seed)
        X = torch.zeros(k, 2 * N * N, dtype=torch.complex128, device="cuda:0")
        dBm = dev(B)
        live.append((bamg.bamg_server_submit(srv, f, dBm, X, k, TOL), k, dBm, X))
    for (rid, k, _, X), Xa in zip(live, alone):
        st, infos = bamg.bamg_server_wait(srv, rid, k, 60000.0)
        assert st == 0 and all(i["relres_reduced"] <= TOL for i in infos)
        assert np.array_equal(X.cpu().numpy(), Xa)
    st = bamg.bamg_server_get_stats(srv)
    log(f"threaded: {st}")
    assert st["completed"] == 10 and st["p99_ms"] >= st["p50_ms"] > 0
    bamg.bamg_server_free(srv)


def test_memory_admission_and_eviction(bamg, fields):
    probe = bamg.bamg_server_create(bamg.bamg_server_default_params(threaded=0, slots_per_field=4))
    ids = add_fields(bamg, probe, fields)
    sizes = [bamg.bamg_server_field_bytes(probe, i) for i in ids]
    bamg.bamg_server_free(probe)
    # room for the larger field alone: the two must take turns
    srv = bamg.bamg_server_create(bamg.bamg_server_default_params(threaded=0, slots_per_field=4,
                                                                  hbm_budget=max(sizes) + 1024))
    fa, fb = add_fields(bamg, srv, fields)
    out = []
    for f, fi in ((fa, 0), (fb, 1), (fa, 0)):
        N = fields[fi]["N"]
        B = rhs(N, 2, 931 + fi)
        X = torch.zeros(2, 2 * N * N, dtype=torch.complex128, device="cuda:0")
        dBm = dev(B)
        rid = bamg.bamg_server_submit(srv, f, dBm, X, 2, TOL)
        res = drive(bamg, srv, {rid: 2})
        assert res[rid][0] == 0
        out.append(X.cpu().numpy())
        st = bamg.bamg_server_get_stats(srv)
        assert st["resident_fields"] == 1 and st["bytes_in_use"] <= st["budget_bytes"]
    st = bamg.bamg_server_get_stats(srv)
    log(f"admission: sizes {sizes}, {st}")
    assert st["setups"] == 3 and st["evictions"] == 2
    # the re-built hierarchy gives the same solution (the setup is deterministic)
    d = np.linalg.norm(out[2] - out[0]) / np.linalg.norm(out[0])
    assert d < 1e-12
    bamg.bamg_server_free(srv)
    # a field larger than the whole budget fails its requests, the server goes on
    small = bamg.bamg_server_create(bamg.bamg_server_default_params(threaded=0, slots_per_field=4,
                                                                    hbm_budget=min(sizes) + 1024))
    fa, fb = add_fields(bamg, small, fields)
    big = fb if sizes[1] > sizes[0] else fa
    ok = fa if big == fb else fb
    Nb, No = fields[big]["N"], fields[ok]["N"]
    Xb = torch.zeros(1, 2 * Nb * Nb, dtype=torch.complex128, device="cuda:0")
    Xo = torch.zeros(1, 2 * No * No, dtype=torch.complex128, device="cuda:0")
    dBb, dBo = dev(rhs(Nb, 1, 941)), dev(rhs(No, 1, 942))
    r1 = bamg.bamg_server_submit(small, big, dBb, Xb, 1, TOL)
    r2 = bamg.bamg_server_submit(small, ok, dBo, Xo, 1, TOL)
    res = drive(bamg, small, {r1: 1, r2: 1})
    assert res[r1][0] == bamg.BAMG_ENOMEM and res[r2][0] == 0
    bamg.bamg_server_free(small)


def test_non_finite_request_fails_alone(bamg, fields):
    srv = bamg.bamg_server_create(bamg.bamg_server_default_params(threaded=0, slots_per_field=4))
    fa, _ = add_fields(bamg, srv, fields)
    N = fields[0]["N"]
    Bbad = rhs(N, 2, 951)
    Bbad[1, 7] = np.nan
    Bgood = rhs(N, 1, 952)
    Xbad = torch.zeros(2, 2 * N * N, dtype=torch.complex128, device="cuda:0")
    Xgood = torch.zeros(1, 2 * N * N, dtype=torch.complex128, device="cuda:0")
    dbad, dgood = dev(Bbad), dev(Bgood)
    r1 = bamg.bamg_server_submit(srv, fa, dbad, Xbad, 2, TOL)
    r2 = bamg.bamg_server_submit(srv, fa, dgood, Xgood, 1, TOL)
    res = drive(bamg, srv, {r1: 2, r2: 1})
    assert res[r1][0] == bamg.BAMG_EINVAL
    assert res[r2][0] == 0 and res[r2][1][0]["relres_reduced"] <= TOL
    bamg.bamg_server_free(srv)


@pytest.mark.parametrize("kw", [dict(precision=0), dict(precision=1), dict(precision=1, setup_mode=2, n_ev=8)],
                         ids=["fp64", "mixed_fp16", "mixed_fp16_bootV"])
def test_footprint_matches_device_allocation(bamg, kw):
    """bamg_footprint_bytes against the device memory a 256^2 setup and one
    solve (3 levels, coarsest n = 8192: 1 GiB FP64 inverse, 0.5 GiB FP32 copy)
    take, and bamg_free gives all of it back."""
    warm = bamg.bamg_setup(dev(inputs.gauge_random(32, 40)), -0.05,
                           bamg.bamg_default_params(N=32, setup_sweeps=1, setup_adapt=0, **kw))
    bamg.bamg_free(warm)  # code objects and runtime state are loaded before the measurement
    N = 256
    U = dev(inputs.gauge_random(N, 41))
    b = dev(inputs.gaussian(2 * N * N, 42))
    x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    p = bamg.bamg_default_params(N=N, setup_sweeps=1, setup_adapt=0, **kw)
    h = bamg.bamg_setup(U, -0.05, p)
    st, _ = bamg.bamg_solve(h, b, x, 1e-8)
    assert st == 0
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    fp = bamg.bamg_footprint_bytes(p)
    bamg.bamg_free(h)
    torch.cuda.synchronize()
    left = free0 - torch.cuda.mem_get_info()[0]
    log(f"footprint {fp / 2**20:.1f} MiB, allocated {used / 2**20:.1f} MiB, after free {left / 2**20:.1f} MiB")
    assert abs(used - fp) <= 0.01 * fp + 8 * 2**20
    assert abs(left) <= 8 * 2**20
