"""GPU against the oracle at the configuration of the headline solve: the
256 x 256 lattice at beta = 10 (min |eig D| ~ 1e-4), 3 levels with a directly
solved coarsest level of dimension 8192, bootstrap super-V setup (Sec. 4.2),
V(2,2), mixed FP16 storage, FGMRES(32) to 1e-10.

The oracle's hierarchy is built from the GPU setup's interpolation operators
P_0 and P_1 (its own Galerkin products, colour orders and cycle); the
coarsest operator is factored by LAPACK's LU (scipy) because the oracle's
plain elimination takes minutes at n = 8192.  Compared:
* the coarse operators D_1, D_2 (FP64);
* the coarsest direct solve at n = 8192 (the packed gamma5 half of the
  inverse for 1-2 right-hand sides, the whole inverse's MFMA product for 3),
  gated at 10 kappa eps with kappa LAPACK's 1-norm estimate;
* one FP64 cycle and one mixed cycle from level 0;
* the headline mixed solve and an FP64 GPU solve with the same operators
  against the oracle's FP64 solve.
"""
import time

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import blocks_to_csr, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
EPS = 2.2e-16


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def log(msg):
    print(msg, flush=True)


HEAD = dict(precision=1, graphs=1, pre=2, post=2, setup_mode=2)


@pytest.fixture(scope="module")
def head():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_5992_amd as bamg
    w = inputs.workload("c3_256_b10")
    N = w["N"]
    U = inputs.load_gauge(w)
    t0 = time.time()
    p = bamg.bamg_default_params(N=N, n_levels=w["n_levels"], seed=w["tv_seed"], **HEAD)
    h = bamg.bamg_setup(dev(U), w["m"], p)
    L = bamg.bamg_n_levels(h)
    assert L == 3 and bamg.bamg_level_info(h, 2)["n"] == 8192
    Ps = [bamg.bamg_export_level(h, l, P=True, D=False)[0] for l in range(L - 1)]
    t1 = time.time()
    o = oracle.Hierarchy.from_interpolation(U, w["m"], Ps, pre=2, post=2)
    log(f"headline: GPU setup {t1 - t0:.1f} s, oracle twin (Galerkin, LAPACK LU of 8192) {time.time() - t1:.1f} s, "
        f"coarsest kappa_1 {o.kappa1:.2e}")
    return bamg, w, U, h, o, Ps


def test_headline_coarse_operators(head):
    bamg, w, U, h, o, Ps = head
    for l in (1, 2):
        inf = bamg.bamg_level_info(h, l)
        _, D, _ = bamg.bamg_export_level(h, l, P=False, D=True)
        A = blocks_to_csr(D, inf["ex"], inf["ey"])
        Ao = o.operator(l)
        d = abs(A - Ao).max() / abs(Ao).max()
        log(f"headline D_{l} (n = {inf['n']}): {d:.2e}")
        assert d < 1e-12


@pytest.mark.parametrize("nrhs", [1, 2, 3])
def test_headline_coarsest_solve(head, nrhs):
    bamg, w, U, h, o, Ps = head
    n = 8192
    b = inputs.gaussian((nrhs, n), 700 + nrhs)
    x = torch.zeros(nrhs, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 2, bamg.OP_COARSEST, dev(b), x, nrhs)
    ref = o.coarsest_solve(b, nrhs=nrhs).reshape(nrhs, n)
    d = rel(host(x), ref)
    log(f"headline coarsest solve, {nrhs} rhs: {d:.2e} (gate 10 kappa eps = {10 * o.kappa1 * EPS:.1e})")
    assert d < max(1e-12, 10 * o.kappa1 * EPS)


def test_headline_cycles(head):
    bamg, w, U, h, o, Ps = head
    N = w["N"]
    b = inputs.gaussian(N * N, 710)
    ref = o.cycle(b)
    x = torch.zeros(N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 0, bamg.OP_CYCLE, dev(b), x, 1)
    d64 = rel(host(x), ref)
    xm = torch.zeros(N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 0, bamg.OP_CYCLE_MIXED, dev(b), xm, 1)
    dm = rel(host(xm), ref)
    log(f"headline V(2,2) cycle: FP64 {d64:.2e}, mixed FP16 storage {dm:.2e}")
    assert d64 < max(1e-11, 10 * o.kappa1 * EPS)
    # FP32 cycle with FP16-stored coarse operators (unit roundoff 4.9e-4)
    assert dm < 2e-2


def _reduced(x, N):
    return np.array([x.reshape(N, N, 2)[y, 2 * xh + (y % 2)] for y in range(N) for xh in range(N // 2)]).reshape(-1)


def test_headline_solves_match_oracle(head):
    """The headline mixed solve (graphs, FP16 storage, FP64 coarsest inverse)
    and an FP64 GPU solve on the same P against the oracle's FP64 solve."""
    bamg, w, U, h, o, Ps = head
    N = w["N"]
    b = inputs.gaussian(2 * N * N, w["rhs_seed"])
    t0 = time.time()
    sto, xo, io = o.solve(b, tol=1e-10)
    t_o = time.time() - t0
    bh = oracle.eo_reduce(U, w["m"], b)
    x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, info = bamg.bamg_solve(h, dev(b), x, 1e-10)
    xg = host(x)
    rr = np.linalg.norm(bh - oracle.dhat_apply(U, w["m"], _reduced(xg, N))) / np.linalg.norm(bh)
    dx = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    log(f"headline mixed solve: iters {info['iters']} (oracle FP64 {io['iters']}, {t_o:.1f} s), reduced relres "
        f"{rr:.2e}, full {info['relres_full']:.2e}, |x - x_oracle|/|x| {dx:.2e}")
    assert st == 0 and sto == 0 and rr <= 1.05e-10
    # both reduced residuals <= 1e-10: the solutions differ by at most about
    # tol * cond(Dhat) (cond ~ 1e4 at min |eig D| ~ 1e-4)
    assert dx < 1e-8
    # the FP64 path on the same P: the oracle's iterations and solution
    p64 = bamg.bamg_default_params(N=N, n_levels=3, graphs=1, pre=2, post=2, setup_sweeps=1, setup_adapt=0)
    h64 = bamg.bamg_setup(dev(U), w["m"], p64)
    for l, P in enumerate(Ps):
        bamg.bamg_import_level(h64, l, P)
    x64 = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st64, i64 = bamg.bamg_solve(h64, dev(b), x64, 1e-10)
    d64 = np.linalg.norm(host(x64) - xo) / np.linalg.norm(xo)
    log(f"headline FP64 solve on the same P: iters {i64['iters']} (oracle {io['iters']}), "
        f"|x - x_oracle|/|x| {d64:.2e}")
    assert st64 == 0 and i64["iters"] == io["iters"] and d64 < 1e-10
    bamg.bamg_free(h64)
