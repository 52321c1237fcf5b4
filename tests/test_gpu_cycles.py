"""GPU parity of the cycle variants, the stand-alone iteration and the
residual of the unreduced system, through the C ABI.

* W (two coarse visits, the solve cycle of Sec. 4) and K (two flexible GCR
  steps on every coarse system that is not the coarsest, each preconditioned
  by one cycle from that level) against the oracle's cycle, on imported
  random interpolation (both sides build every operator from the same P),
  3 and 4 levels, 1 to 6 right-hand sides;
* full solves with W and K cycles against the oracle: equal iteration counts
  and solutions within 1e-10;
* the mixed-precision K-cycle solve reaches the FP64 accuracy; batched K
  solves are bitwise independent of the batch;
* the stand-alone iteration x <- x + M(0 - Dhat x) (the convergence rate of
  Sec. 4) against the oracle's;
* ||b - D x|| / ||b|| of the unreduced system: in every solve's info and
  from the hierarchy-free entry point, against the oracle's operator;
* replacing D_l through the import hook;
* the free field at m = 0 (D singular at zero momentum, Sec. 2): setup or
  solve fails with a status, never with a non-finite result.
"""
import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import blocks_to_csr, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CYC = {"V": 0, "W": 1, "K": 2}


@pytest.fixture(scope="module")
def bamg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_5992_amd as b
    return b


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def log(msg):
    print(msg, flush=True)


def make_h(bamg, U, m, **kw):
    N = U.shape[-1]
    init_tv = kw.pop("init_tv", None)
    p = bamg.bamg_default_params(N=N, **kw)
    return bamg.bamg_setup(dev(U), m, p, init_tv=init_tv)


def _imported(bamg, N, L, cycle, pre=2, post=2, seed=5):
    """GPU and oracle hierarchies with the same seeded random interpolation."""
    U = inputs.gauge_metropolis(N, 3.0, 40, seed)
    m = -0.05
    kw = dict(n_levels=L, setup_sweeps=2, setup_adapt=0, pre=pre, post=post, cycle=CYC[cycle])
    h = make_h(bamg, U, m, **kw)
    o = oracle.Hierarchy(U, m, **kw)
    assert bamg.bamg_n_levels(h) == o.n_levels == L
    for l in range(L - 1):
        P = inputs.gaussian(o.P_blocks(l).shape, 100 + l)
        bamg.bamg_import_level(h, l, P)
        o.import_P(l, P)
    kappa = np.linalg.cond(o.operator(L - 1).toarray())
    return U, m, h, o, kappa


@pytest.mark.parametrize("N,L", [(64, 3), (128, 4)])
@pytest.mark.parametrize("cycle", ["W", "K"])
@pytest.mark.parametrize("nrhs", [1, 2, 6])
def test_cycle_matches_oracle(bamg, N, L, cycle, nrhs):
    log(f"cycle {cycle} N={N} L={L} nrhs={nrhs}")
    U, m, h, o, kappa = _imported(bamg, N, L, cycle)
    n = N * N
    b = inputs.gaussian((nrhs, n), 90)
    x = torch.zeros(nrhs, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 0, bamg.OP_CYCLE, dev(b), x, nrhs)
    ref = o.cycle(b, nrhs=nrhs).reshape(nrhs, n)
    d = rel(host(x), ref)
    log(f"  diff {d:.2e} (coarsest kappa {kappa:.1e})")
    assert d < max(1e-11, 10 * kappa * 2.2e-16)


@pytest.mark.parametrize("cycle", ["V", "W", "K"])
def test_stationary_iteration_matches_oracle(bamg, cycle):
    """rho of Sec. 4: ||e^nu|| / ||e^{nu-1}|| of the solver used on its own."""
    N = 64
    U, m, h, o, kappa = _imported(bamg, N, 3, cycle)
    x0 = inputs.gaussian(N * N, 33)
    x = dev(x0)
    norms = bamg.bamg_stationary(h, x, 5)
    xo, no = o.stationary(x0, 5)
    log(f"stationary {cycle}: rates {np.round(norms[1:] / norms[:-1], 4)}; x diff {rel(host(x), xo):.2e}")
    assert np.allclose(norms, no, rtol=1e-10, atol=0)
    assert rel(host(x), xo) < max(1e-11, 10 * kappa * 2.2e-16)
    assert norms[-1] < norms[0]


@pytest.mark.parametrize("name", ["c1_32_b3", "c2_128_b6"])
@pytest.mark.parametrize("cycle", ["W", "K"])
def test_full_solve_cycles(bamg, name, cycle):
    log(f"solve {name} {cycle}")
    w = inputs.workload(name)
    U = inputs.load_gauge(w)
    N = w["N"]
    tv = oracle.gaussian_tv(N, 8, w["tv_seed"])
    kw = dict(n_levels=w["n_levels"], cycle=CYC[cycle])
    h = make_h(bamg, U, w["m"], init_tv=tv, **kw)
    b = inputs.gaussian(2 * N * N, w["rhs_seed"])
    x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, info = bamg.bamg_solve(h, dev(b), x, 1e-10)
    xg = host(x)
    o = oracle.Hierarchy(U, w["m"], init_tv=tv, **kw)
    sto, xo, io = o.solve(b, tol=1e-10)
    full = np.linalg.norm(b - oracle.wilson_apply(U, w["m"], xg)) / np.linalg.norm(b)
    dx = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    log(f"  gpu iters {info['iters']} oracle iters {io['iters']} full relres {full:.2e} "
        f"(reported {info['relres_full']:.2e}, oracle {io['relres_full']:.2e}) dx {dx:.2e}")
    assert st == 0 and sto == 0
    assert info["iters"] == io["iters"]
    assert dx < 1e-10
    assert abs(info["relres_full"] - full) <= 1e-6 * full + 1e-15


def test_mixed_kcycle_solve_and_batch_invariance(bamg):
    """Mixed FP16 with the K-cycle (FP32 vectors, FP64 sums and coefficients)
    reaches the FP64 solution; a right-hand side's batched result does not
    depend on the batch (per right-hand side reductions of fixed order)."""
    w = inputs.workload("c2_128_b6")
    U = inputs.load_gauge(w)
    N = w["N"]
    tv = oracle.gaussian_tv(N, 8, w["tv_seed"])
    kw = dict(n_levels=3, cycle=CYC["K"], pre=2, post=2)
    h64 = make_h(bamg, U, w["m"], init_tv=tv, **kw)
    h16 = make_h(bamg, U, w["m"], init_tv=tv, precision=1, **kw)
    B = inputs.gaussian((3, 2 * N * N), 555)
    x64 = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, i64 = bamg.bamg_solve(h64, dev(B[0]), x64, 1e-10)
    x16 = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st16, i16 = bamg.bamg_solve(h16, dev(B[0]), x16, 1e-10)
    e = rel(host(x16), host(x64))
    full = np.linalg.norm(B[0] - oracle.wilson_apply(U, w["m"], host(x16))) / np.linalg.norm(B[0])
    log(f"K mixed: iters fp64 {i64['iters']} fp16 {i16['iters']}; error against FP64 {e:.2e}; full relres {full:.2e}")
    assert st == 0 and st16 == 0 and full < 2e-10 and e < 1e-7
    X3 = torch.zeros(3, 2 * N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_solve_batch(h16, dev(B), X3, 3, 1e-10)
    X1 = torch.zeros(1, 2 * N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_solve_batch(h16, dev(B[1:2]), X1, 1, 1e-10)
    assert np.array_equal(host(X3)[1], host(X1)[0])


def test_full_residual_entry_point(bamg):
    """||b - D x|| / ||b|| per right-hand side, hierarchy-free, against the
    oracle's Wilson operator (eq. wilson); a zero b gives ||D x||."""
    for N, nrhs in [(16, 1), (64, 3), (256, 2)]:
        U = inputs.gauge_random(N, 7 + N)
        m = -0.03
        B = inputs.gaussian((nrhs, 2 * N * N), 1 + N)
        X = inputs.gaussian((nrhs, 2 * N * N), 2 + N)
        if nrhs == 3:
            B[2] = 0
        out = torch.zeros(nrhs, dtype=torch.float64, device="cuda:0")
        bamg.bamg_full_residual(N, dev(U), m, dev(B), dev(X), nrhs, out)
        got = out.cpu().numpy()
        for r in range(nrhs):
            res = np.linalg.norm(B[r] - oracle.wilson_apply(U, m, X[r]))
            ref = res / np.linalg.norm(B[r]) if B[r].any() else res
            assert abs(got[r] - ref) <= 1e-13 * ref, (N, r, got[r], ref)


def test_import_coarse_operator(bamg):
    """D_l from the host replaces level l (its smoother data, or the coarsest
    inverse, follow), and a following P import rebuilds level l+1 from it."""
    N = 64
    U, m, h, o, kappa = _imported(bamg, N, 3, "V")
    P1, D1, _ = bamg.bamg_export_level(h, 1)
    _, D2, _ = bamg.bamg_export_level(h, 2)
    n1 = bamg.bamg_level_info(h, 1)["n"]
    x = inputs.gaussian(n1, 3)
    y0 = torch.zeros(n1, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 1, bamg.OP_APPLY, dev(x), y0, 1)
    bamg.bamg_import_level(h, 1, D=2.0 * D1)
    y1 = torch.zeros(n1, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 1, bamg.OP_APPLY, dev(x), y1, 1)
    assert rel(host(y1), 2.0 * host(y0)) < 1e-15
    # a sweep on (2 D) x = 2 b from x0 equals the sweep on D x = b (scale-invariant projections)
    inf1 = bamg.bamg_level_info(h, 1)
    b = inputs.gaussian(n1, 4)
    xs = dev(inputs.gaussian(n1, 5))
    bamg.bamg_level_op(h, 1, bamg.OP_SWEEP, dev(2.0 * b), xs, 1)
    ref = o.sweep(1, inputs.gaussian(n1, 5), b)
    assert rel(host(xs), ref) < 1e-11
    bamg.bamg_import_level(h, 1, P=P1)  # level 2 = P^H (2 D_1) P
    _, D2b, _ = bamg.bamg_export_level(h, 2)
    assert rel(D2b, 2.0 * D2) < 1e-13
    n2 = bamg.bamg_level_info(h, 2)["n"]
    bb = inputs.gaussian(n2, 6)
    xc = torch.zeros(n2, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 2, bamg.OP_COARSEST, dev(bb), xc, 1)
    A2 = blocks_to_csr(2.0 * D2, inf1["ex"] // 2, inf1["ey"] // 2).toarray()
    assert rel(host(xc), np.linalg.solve(A2, bb)) < max(1e-12, 10 * kappa * 2.2e-16)
    # both at once: D_1 back to the original, level 2 rebuilt from it
    bamg.bamg_import_level(h, 1, P=P1, D=D1)
    _, D2c, _ = bamg.bamg_export_level(h, 2)
    assert rel(D2c, D2) < 1e-13


def test_free_field_massless_fails_cleanly(bamg):
    """U = 1, m = 0: D has a zero mode at p = 0 (Sec. 2, free-field spectrum),
    so Dhat is singular.  The setup reports a singular coarsest operator, or
    the solve stops without convergence; no call returns non-finite values.
    The oracle behaves alike."""
    N = 16
    U = inputs.gauge_free(N)
    b = inputs.gaussian(2 * N * N, 3)
    p = bamg.bamg_default_params(N=N, max_iter=40)
    try:
        h = bamg.bamg_setup(dev(U), 0.0, p)
    except bamg.BamgError as err:
        log(f"free field m = 0: setup status {err.status} ({bamg.bamg_last_error()})")
        assert err.status == bamg.BAMG_ESINGULAR
        h = None
    if h is not None:
        x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
        st, info = bamg.bamg_solve(h, dev(b), x, 1e-10)
        xg = host(x)
        log(f"free field m = 0: solve status {st} iters {info['iters']} relres {info['relres_reduced']:.2e}")
        assert st == bamg.BAMG_NOT_CONVERGED
        assert np.isfinite(xg).all() and np.isfinite(info["relres_reduced"]) and np.isfinite(info["relres_full"])
    o = oracle.Hierarchy(U, 0.0)
    singular = o.level_info(o.n_levels - 1)["singular"]
    if not singular:
        sto, xo, io = o.solve(b, tol=1e-10, max_iter=40)
        assert sto == 1 and np.isfinite(xo).all()
