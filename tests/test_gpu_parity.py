"""GPU parity: every kernel of the HIP path against the CPU FP64 oracle on the
same seeded inputs, through the C ABI (bamg.h).

Tolerances (FP64): element-wise results of a fixed sequence of operations
agree to a few ulps times the number of accumulated terms, so kernels are
gated at 1e-12 relative to the largest entry.  Results that pass through a
least-squares basis or the coarsest inverse are gated by their conditioning
(stated at each test).
"""
import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import blocks_to_csr, projector_diff, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


# ---------------------------------------------------------------- fine level
@pytest.mark.parametrize("N,nrhs", [(16, 1), (40, 2), (128, 3), (256, 1), (512, 1), (512, 5), (1024, 1), (1024, 4)])
def test_dhat_apply(bamg, N, nrhs):
    """The three kernels of the operator, chosen by the amount of work:
    N <= 256 (few right-hand sides): tiles of 64 x 4 sites; 512^2 x 1, 512^2 x 5
    and 1024^2 x 1: 32 x 16 tiles; 1024^2 x 4: strips of 62 columns streamed
    down segments of 16 rows."""
    log(f"dhat N={N} nrhs={nrhs}")
    U = inputs.gauge_random(N, 10 + N)
    m = -0.07
    h = make_h(bamg, U, m, setup_sweeps=1, setup_adapt=0)
    x = inputs.gaussian((nrhs, N * N), 20 + N)
    y = torch.zeros(nrhs, N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_apply_dhat(h, dev(x), y, nrhs)
    ref = oracle.dhat_apply(U, m, x).reshape(nrhs, N * N)
    assert rel(host(y), ref) < 1e-13


def test_binding_imported_before_torch():
    """A process that imports the binding before torch: the library must bind
    to the HIP runtime torch uses (the binding loads torch first), else it
    sees no device.  Runs in a fresh process, as the import order is per
    process."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import paper_1308_5992_amd as bamg\n"
        "import numpy as np, torch, inputs, oracle\n"
        "N = 16; U = inputs.gauge_random(N, 26); m = -0.07\n"
        "d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to('cuda:0')\n"
        "h = bamg.bamg_setup(d(U), m,"
        " bamg.bamg_default_params(N=N, setup_sweeps=1, setup_adapt=0))\n"
        "x = inputs.gaussian((1, N * N), 36)\n"
        "y = torch.zeros(1, N * N, dtype=torch.complex128, device='cuda:0')\n"
        "bamg.bamg_apply_dhat(h, d(x), y, 1)\n"
        "ref = oracle.dhat_apply(U, m, x).reshape(1, N * N)\n"
        "print(float(np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()))\n"
    )
    log("binding imported before torch (subprocess)")
    env = dict(os.environ, PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    assert float(r.stdout.strip().splitlines()[-1]) < 1e-13


@pytest.mark.parametrize("N,nrhs", [(128, 2), (512, 3), (1024, 2)])
def test_dhat_apply_fp32(bamg, N, nrhs):
    """The FP32 operator of the mixed cycle (level op 10 on level 0, FP32 links
    rounded from FP64) against the FP64 oracle: within a few FP32 roundings of
    the 9-term sums (|Dhat| |x| scale)."""
    U = inputs.gauge_random(N, 30 + N)
    m = -0.07
    h = make_h(bamg, U, m, n_levels=1, precision=3)
    x = inputs.gaussian((nrhs, N * N), 31 + N).astype(np.complex64)
    y = torch.zeros(nrhs, N * N, dtype=torch.complex64, device="cuda:0")
    bamg.bamg_level_op(h, 0, bamg.OP_APPLY_F32, torch.from_numpy(x).to("cuda:0"), y, nrhs)
    ref = oracle.dhat_apply(U, m, x.astype(np.complex128)).reshape(nrhs, N * N)
    e = rel(host(y).astype(np.complex128), ref)
    log(f"dhat fp32 N={N} nrhs={nrhs}: {e:.2e}")
    assert e < 2e-6


@pytest.mark.parametrize("N,R,prec", [(256, 64, 0), (512, 64, 0), (2048, 4, 3)])
def test_dhat_kernels_give_the_same_bits(bamg, N, R, prec):
    """The operator's kernels are chosen by the amount of work, so a batch and
    its right-hand sides applied one at a time take different kernels (256^2:
    strips against 64 x 4 tiles; 512^2: strips against 32 x 16 tiles; FP32
    2048^2: 64-row strips against 32 x 16 tiles).  Each product is rounded
    the same way in all of them, so the batch result is bitwise the single
    one, which the batched solver's independence of its batch relies on."""
    U = inputs.gauge_random(N, 50 + N)
    m = -0.07
    h = make_h(bamg, U, m, n_levels=1, precision=prec)
    dt = torch.complex64 if prec else torch.complex128
    X = torch.from_numpy(inputs.gaussian((R, N * N), 51 + N)).to("cuda:0").to(dt)
    Y = torch.zeros_like(X)

    def apply(x, y, k):
        if prec:
            bamg.bamg_level_op(h, 0, bamg.OP_APPLY_F32, x, y, k)
        else:
            bamg.bamg_apply_dhat(h, x, y, k)

    apply(X, Y, R)
    for r in sorted({0, R // 2, R - 1}):
        y1 = torch.zeros_like(X[r:r + 1])
        apply(X[r:r + 1].contiguous(), y1, 1)
        assert torch.equal(y1[0], Y[r]), r


@pytest.mark.parametrize("N,nrhs", [(16, 2), (40, 1)])
def test_eo_reduce_reconstruct(bamg, N, nrhs):
    log(f"eo N={N}")
    U = inputs.gauge_random(N, 3)
    m = 0.11
    h = make_h(bamg, U, m, setup_sweeps=1, setup_adapt=0)
    b = inputs.gaussian((nrhs, 2 * N * N), 4)
    bh = torch.zeros(nrhs, N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_eo_reduce(h, dev(b), bh, nrhs)
    assert rel(host(bh), oracle.eo_reduce(U, m, b).reshape(nrhs, -1)) < 1e-13
    xe = inputs.gaussian((nrhs, N * N), 5)
    x = torch.zeros(nrhs, 2 * N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_eo_reconstruct(h, dev(b), dev(xe), x, nrhs)
    assert rel(host(x), oracle.eo_reconstruct(U, m, b, xe).reshape(nrhs, -1)) < 1e-13


@pytest.mark.parametrize("N,nrhs", [(16, 1), (40, 2), (64, 1), (40, 5), (40, 16), (64, 17), (64, 40), (40, 70),
                                    (80, 3), (96, 2), (128, 1), (512, 1), (256, 5), (1024, 1), (1040, 2)])
def test_fine_kaczmarz_sweep(bamg, N, nrhs):
    """From 32 right-hand sides the sweeps run on right-hand-side-interleaved
    copies (16, 32 or 64 lanes per site; 70 takes two chunks of 64), from 16
    where no sweep blocked in LDS applies (40 x 16).  Otherwise, from N = 64
    on, one launch per sweep blocked in LDS (64 x 17: the streaming form; 80: 8-wide
    tiles in v, 96: tiles of 32 in u; 512 x 1: the streaming form; 256 x 5
    and 1024: the pipelined march along v); 16, 40 and 1040 x 2 take the
    colour passes (1040: 33800 sites per colour, a count of work-groups that
    is not a multiple of 8, and N/2 no multiple of 32)."""
    log(f"kaczmarz fine N={N}")
    U = inputs.gauge_random(N, 7)
    m = 0.02
    # operator-only handles for the large lattices (1040 has no 8192-dim coarsest level)
    h = make_h(bamg, U, m, setup_sweeps=1, setup_adapt=0, **({"n_levels": 1} if N >= 1024 else {}))
    x0 = inputs.gaussian((nrhs, N * N), 8)
    b = inputs.gaussian((nrhs, N * N), 9)
    x = dev(x0)
    for _ in range(2):
        bamg.bamg_level_op(h, 0, bamg.OP_SWEEP, dev(b), x, nrhs)
    ref = oracle.kaczmarz_fine(U, m, x0, b, sweeps=2).reshape(nrhs, -1)
    assert rel(host(x), ref) < 1e-12


@pytest.mark.parametrize("N", [40, 64, 96, 256, 512, 1024])
@pytest.mark.parametrize("prec", [0, 3])
def test_fine_sweep_batch_gives_the_same_bits(bamg, prec, N):
    """32 right-hand sides take the interleaved sweep; 16 of them take it too
    except where the streaming form applies (FP32 256^2 x 16); one or three of
    them alone take the colour passes (N = 40) or a sweep blocked in LDS (from
    N = 64; the streaming form for 256^2 x 3, 512^2 x 1 and FP32 512^2 x 3 and
    1024^2 x 1, the pipelined march for FP64 512^2 x 3 and 1024^2, FP32
    1024^2 x 3): the same bits (each lane adds the slot terms in
    the butterfly's order; the blocked sweeps project every site a tile depends
    on with the values the colour passes give it)."""
    R = 32
    log(f"sweep bits N={N} prec={prec}")
    U = inputs.gauge_random(N, 27)
    h = make_h(bamg, U, 0.02, n_levels=1, precision=prec)
    dt = torch.complex64 if prec else torch.complex128
    op = bamg.OP_SWEEP_F32 if prec else bamg.OP_SWEEP
    X = torch.from_numpy(inputs.gaussian((R, N * N), 28)).to("cuda:0").to(dt)
    B = torch.from_numpy(inputs.gaussian((R, N * N), 29)).to("cuda:0").to(dt)
    X1 = X.clone()
    for _ in range(2):
        bamg.bamg_level_op(h, 0, op, B, X, R)
    for r0, r1 in ((0, 1), (7, 10), (0, 16), (31, 32)):
        x1 = X1[r0:r1].clone()  # (a copy: the subsets overlap, and a contiguous slice is a view)
        for _ in range(2):
            bamg.bamg_level_op(h, 0, op, B[r0:r1].contiguous(), x1, r1 - r0)
        assert torch.equal(x1, X[r0:r1]), (r0, r1)


@pytest.mark.parametrize("N,prec", [(128, 0), (256, 3), (512, 0), (1024, 0), (1024, 3), (4096, 0)])
def test_fine_sweep_forms_give_the_colour_pass_bits(bamg, N, prec):
    """One sweep in the library's form for the size (128^2, FP32 256^2: blocked
    in LDS; 512^2: streaming; 1024^2 and 4096^2: pipelined) against op 13 / 14,
    the 16 colour passes: the same bits."""
    log(f"sweep forms vs colour passes N={N} prec={prec}")
    U = inputs.gauge_random(N, 31)
    h = make_h(bamg, U, 0.02, n_levels=1, precision=prec)
    dt = torch.complex64 if prec else torch.complex128
    op, opc = (bamg.OP_SWEEP_F32, bamg.OP_SWEEP_COLOURS_F32) if prec else (bamg.OP_SWEEP, bamg.OP_SWEEP_COLOURS)
    x1 = torch.from_numpy(inputs.gaussian(N * N, 32)).to("cuda:0").to(dt)
    b = torch.from_numpy(inputs.gaussian(N * N, 33)).to("cuda:0").to(dt)
    x2 = x1.clone()
    bamg.bamg_level_op(h, 0, op, b, x1, 1)
    bamg.bamg_level_op(h, 0, opc, b, x2, 1)
    assert torch.equal(x1, x2)
    bamg.bamg_free(h)
    del x1, x2, b
    torch.cuda.empty_cache()


def test_philox_test_vectors(bamg):
    N, k, seed = 32, 8, 0x1234_5678_9ABC
    out = torch.zeros(k, N * N, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_gaussian_tv(N, k, seed, out)
    ref = oracle.gaussian_tv(N, k, seed)
    # same counters and bits; log/cos/sin of the two math libraries may differ in the last ulp
    assert rel(host(out), ref) < 1e-14


# ---------------------------------------------------------------- imported hierarchy
def _random_P(shape, seed):
    return inputs.gaussian(shape, seed)


@pytest.fixture(scope="module")
def imported(bamg):
    """GPU and oracle hierarchies whose interpolation operators are the same
    seeded random spin-block matrices (so every coarse operator, smoother and
    the coarsest inverse are built by each side from identical inputs)."""
    N = 64
    U = inputs.gauge_metropolis(N, 3.0, 40, 5)
    m = -0.05
    kw = dict(n_levels=3, max_coarse=512, setup_sweeps=2, setup_adapt=0)
    h = make_h(bamg, U, m, **kw)
    o = oracle.Hierarchy(U, m, **kw)
    assert bamg.bamg_n_levels(h) == o.n_levels == 3
    for l in range(2):
        P = _random_P(o.P_blocks(l).shape, 100 + l)
        bamg.bamg_import_level(h, l, P)
        o.import_P(l, P)
    return N, U, m, h, o


def test_galerkin_operators(bamg, imported):
    N, U, m, h, o = imported
    for l in (1, 2):
        inf = bamg.bamg_level_info(h, l)
        _, D, _ = bamg.bamg_export_level(h, l)
        A = blocks_to_csr(D, inf["ex"], inf["ey"]).toarray()
        Ao = o.operator(l).toarray()
        log(f"galerkin level {l}: {rel(A, Ao):.2e}")
        assert rel(A, Ao) < 1e-12


@pytest.mark.parametrize("l", [0, 1])
def test_transfers(bamg, imported, l):
    N, U, m, h, o = imported
    n = bamg.bamg_level_info(h, l)["n"]
    nc = bamg.bamg_level_info(h, l + 1)["n"]
    r = inputs.gaussian((2, n), 30 + l)
    rc = torch.zeros(2, nc, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, l, bamg.OP_RESTRICT, dev(r), rc, 2)
    assert rel(host(rc), o.restrict(l, r, nrhs=2).reshape(2, nc)) < 1e-13
    xc = inputs.gaussian((2, nc), 40 + l)
    y0 = inputs.gaussian((2, n), 50 + l)
    y = dev(y0)
    bamg.bamg_level_op(h, l, bamg.OP_PROLONG, dev(xc), y, 2)
    assert rel(host(y), o.prolong_add(l, xc, y0, nrhs=2).reshape(2, n)) < 1e-13


@pytest.mark.parametrize("l", [0, 1, 2])
def test_level_apply(bamg, imported, l):
    N, U, m, h, o = imported
    n = bamg.bamg_level_info(h, l)["n"]
    x = inputs.gaussian((2, n), 60 + l)
    y = torch.zeros(2, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, l, bamg.OP_APPLY, dev(x), y, 2)
    assert rel(host(y), o.apply(l, x, nrhs=2).reshape(2, n)) < 1e-12


@pytest.mark.parametrize("nrhs", [2, 5, 19])
def test_coarse_kaczmarz_sweep(bamg, imported, nrhs):
    """nrhs >= 4 runs the multi-RHS kernel (block row staged once per 16 RHS)."""
    N, U, m, h, o = imported
    l = 1
    n = bamg.bamg_level_info(h, l)["n"]
    x0 = inputs.gaussian((nrhs, n), 70)
    b = inputs.gaussian((nrhs, n), 71)
    x = dev(x0)
    bamg.bamg_level_op(h, l, bamg.OP_SWEEP, dev(b), x, nrhs)
    ref = o.sweep(l, x0, b, nrhs=nrhs).reshape(nrhs, n)
    # block form tril(G)^-1 of the 16 sequential projections: rounding
    # differences scale with cond(tril(G)); random P keeps it moderate
    assert rel(host(x), ref) < 1e-11


@pytest.mark.parametrize("nrhs", [1, 3])
def test_coarse_fused_pairs_give_the_colour_pass_bits(bamg, imported, nrhs):
    """Level 1 (8 x 16 sites, 8 colours): op 1 runs two colours per launch
    (the fused pairs, out of place between x and a second copy), op 13 one
    launch per colour: the same bits, over two sweeps."""
    N, U, m, h, o = imported
    n = bamg.bamg_level_info(h, 1)["n"]
    x0 = inputs.gaussian((nrhs, n), 74)
    b = dev(inputs.gaussian((nrhs, n), 75))
    x1, x2 = dev(x0), dev(x0)
    for _ in range(2):
        bamg.bamg_level_op(h, 1, bamg.OP_SWEEP, b, x1, nrhs)
        bamg.bamg_level_op(h, 1, bamg.OP_SWEEP_COLOURS, b, x2, nrhs)
    assert torch.equal(x1, x2)
    assert not torch.equal(x1, dev(x0))


@pytest.mark.parametrize("nrhs", [1, 2, 3, 9, 17, 37, 70])
def test_coarsest_solve(bamg, imported, nrhs):
    """nrhs <= 2: the product with the packed gamma5-Hermitian half of the
    inverse (64 x 64 blocks on and above the diagonal); else the split-K FP64
    MFMA product with the whole inverse (8, 16, 32 and 64 right-hand sides per
    work-group; 70 spans two groups), whose columns do not depend on the other
    columns."""
    N, U, m, h, o = imported
    L = 2
    n = bamg.bamg_level_info(h, L)["n"]
    b = inputs.gaussian((nrhs, n), 80)
    x = torch.zeros(nrhs, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, L, bamg.OP_COARSEST, dev(b), x, nrhs)
    A = o.operator(L).toarray()
    kappa = np.linalg.cond(A)
    ref = o.coarsest_solve(b, nrhs=nrhs).reshape(nrhs, n)
    log(f"coarsest cond {kappa:.2e} diff {rel(host(x), ref):.2e}")
    assert rel(host(x), ref) < max(1e-12, 10 * kappa * 2.2e-16)
    if nrhs > 8:
        x9 = torch.zeros(9, n, dtype=torch.complex128, device="cuda:0")
        bamg.bamg_level_op(h, L, bamg.OP_COARSEST, dev(b[:9]), x9, 9)
        assert np.array_equal(host(x9), host(x)[:9])


def test_coarsest_packed_half_matches_whole_inverse(bamg, imported):
    """The single-RHS coarsest product reads only the blocks on and above the
    diagonal of the inverse and mirrors the rest through gamma5-Hermiticity
    (A[j][i] = g_i g_j conj(A[i][j]), Sec. 3.5); the off-diagonal blocks are
    averaged with their mirrors.  Its result against the whole inverse's
    (split-K product, 3 right-hand sides), within the inverse's rounding
    (10 kappa eps), and the relation itself on the oracle's inverse."""
    N, U, m, h, o = imported
    L = 2
    n = bamg.bamg_level_info(h, L)["n"]
    A = o.operator(L).toarray()
    kappa = np.linalg.cond(A)
    Ainv = np.linalg.inv(A)
    g = np.where((np.arange(n) % 16) >= 8, -1.0, 1.0)
    assert rel(Ainv.conj().T, g[:, None] * Ainv * g[None, :]) < 10 * kappa * 2.2e-16
    b = inputs.gaussian((3, n), 81)
    X3 = torch.zeros(3, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, L, bamg.OP_COARSEST, dev(b), X3, 3)
    for r in range(3):
        x1 = torch.zeros(1, n, dtype=torch.complex128, device="cuda:0")
        bamg.bamg_level_op(h, L, bamg.OP_COARSEST, dev(b[r:r + 1]), x1, 1)
        e = rel(host(x1)[0], host(X3)[r])
        log(f"packed half against whole inverse, rhs {r}: {e:.2e} (kappa {kappa:.1e})")
        assert e < max(1e-12, 10 * kappa * 2.2e-16)


@pytest.mark.parametrize("nrhs", [2, 6])
def test_cycle(bamg, imported, nrhs):
    N, U, m, h, o = imported
    n = N * N
    b = inputs.gaussian((nrhs, n), 90)
    x = torch.zeros(nrhs, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, 0, bamg.OP_CYCLE, dev(b), x, nrhs)
    ref = o.cycle(b, nrhs=nrhs).reshape(nrhs, n)
    kappa = np.linalg.cond(o.operator(2).toarray())
    log(f"cycle diff {rel(host(x), ref):.2e}")
    assert rel(host(x), ref) < max(1e-11, 10 * kappa * 2.2e-16)


# ---------------------------------------------------------------- setup and solve
@pytest.fixture(scope="module")
def c1(bamg):
    w = inputs.workload("c1_32_b3")
    U = inputs.load_gauge(w)
    tv = oracle.gaussian_tv(w["N"], 8, w["tv_seed"])
    h = make_h(bamg, U, w["m"], n_levels=w["n_levels"], init_tv=tv)
    o = oracle.Hierarchy(U, w["m"], n_levels=w["n_levels"], init_tv=tv)
    return w, U, h, o


def test_setup_matches_oracle(bamg, c1):
    w, U, h, o = c1
    P, _, T = bamg.bamg_export_level(h, 0, D=False, tv=True)
    d_tv = rel(T, o.test_vectors())
    d_p = projector_diff(P, o.P_blocks(0))
    inf = bamg.bamg_level_info(h, 1)
    _, D, _ = bamg.bamg_export_level(h, 1)
    d_d = rel(blocks_to_csr(D, inf["ex"], inf["ey"]).toarray(), o.operator(1).toarray())
    log(f"setup: tv {d_tv:.2e} projector {d_p:.2e} coarse op {d_d:.2e}")
    assert d_tv < 1e-11 and d_p < 1e-11 and d_d < 1e-11


def _check_solution(w, U, b, x, tol):
    r = b - oracle.wilson_apply(U, w["m"], x)
    bh = oracle.eo_reduce(U, w["m"], b)
    return np.linalg.norm(r) / np.linalg.norm(b), bh


@pytest.mark.parametrize("name", ["c1_32_b3", "c2_128_b6"])
def test_full_solve(bamg, name):
    log(f"solve {name}")
    w = inputs.workload(name)
    U = inputs.load_gauge(w)
    N = w["N"]
    tv = oracle.gaussian_tv(N, 8, w["tv_seed"])
    h = make_h(bamg, U, w["m"], n_levels=w["n_levels"], init_tv=tv)
    b = inputs.gaussian(2 * N * N, w["rhs_seed"])
    x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, info = bamg.bamg_solve(h, dev(b), x, 1e-10)
    xg = host(x)
    o = oracle.Hierarchy(U, w["m"], n_levels=w["n_levels"], init_tv=tv)
    sto, xo, io = o.solve(b, tol=1e-10)
    # reduced residual of the GPU solution, measured with the oracle's operator
    xe = np.array([xg.reshape(N, N, 2)[y, 2 * xh + (y % 2)] for y in range(N) for xh in range(N // 2)]).reshape(-1)
    bh = oracle.eo_reduce(U, w["m"], b)
    rr = np.linalg.norm(bh - oracle.dhat_apply(U, w["m"], xe)) / np.linalg.norm(bh)
    full = np.linalg.norm(b - oracle.wilson_apply(U, w["m"], xg)) / np.linalg.norm(b)
    dx = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    log(f"{name}: gpu iters {info['iters']} oracle iters {io['iters']} reduced relres {rr:.2e} "
        f"full relres {full:.2e} |x_gpu - x_oracle|/|x| {dx:.2e}")
    assert st == 0 and sto == 0
    assert rr <= 1.05e-10
    assert info["iters"] == io["iters"]
    assert dx < 1e-10
    assert abs(info["relres_full"] - full) <= 1e-6 * full + 1e-15


def test_failure_handling(bamg, c1):
    w, U, h, o = c1
    N = w["N"]
    b = inputs.gaussian(2 * N * N, 1)
    x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    bn = b.copy()
    bn[7] = np.nan
    with pytest.raises(bamg.BamgError) as e:
        bamg.bamg_solve(h, dev(bn), x, 1e-10)
    assert e.value.status == bamg.BAMG_EINVAL
    z = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, info = bamg.bamg_solve(h, z, x, 1e-10)
    assert st == 0 and info["iters"] == 0 and not host(x).any()
    p = bamg.bamg_default_params(N=36)
    with pytest.raises(bamg.BamgError) as e:
        bamg.bamg_setup(dev(U), w["m"], p)
    assert e.value.status == bamg.BAMG_EINVAL


def test_not_converged_status(bamg):
    N = 32
    U = inputs.gauge_random(N, 2)
    h = make_h(bamg, U, 0.05, max_iter=1, setup_sweeps=3)
    b = inputs.gaussian(2 * N * N, 3)
    x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, info = bamg.bamg_solve(h, dev(b), x, 1e-14)
    assert st == bamg.BAMG_NOT_CONVERGED and info["iters"] == 1
    assert np.isfinite(host(x)).all()


def test_batch_results_do_not_depend_on_the_batch(bamg, c1):
    """Each right-hand side of a batched solve gives bitwise the result of a
    batched solve of that right-hand side alone (the batched path uses the
    same kernels for every batch size and treats right-hand sides
    independently with fixed reduction orders), and the result of the
    single-RHS solver up to rounding."""
    w, U, h, o = c1
    N = w["N"]
    R = 5
    B = inputs.gaussian((R, 2 * N * N), 555)
    B[1] *= 1e-3  # different scales converge at different iterations
    B[3] = inputs.gaussian(2 * N * N, 556) + 1e2 * B[3]
    X = torch.zeros(R, 2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, infos = bamg.bamg_solve_batch(h, dev(B), X, R, 1e-10)
    assert st == 0
    Xb = host(X)
    for r in range(R):
        x1 = torch.zeros(1, 2 * N * N, dtype=torch.complex128, device="cuda:0")
        st1, inf1 = bamg.bamg_solve_batch(h, dev(B[r:r + 1]), x1, 1, 1e-10)
        assert st1 == 0 and inf1[0]["iters"] == infos[r]["iters"]
        assert np.array_equal(host(x1)[0], Xb[r])
        x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
        st2, info = bamg.bamg_solve(h, dev(B[r]), x, 1e-10)
        assert st2 == 0 and abs(info["iters"] - infos[r]["iters"]) <= 1
        assert rel(host(x), Xb[r]) < 1e-9


# ---------------------------------------------------------------- mixed precision
# FP32 arithmetic with operators stored in FP32 / FP16 / BF16: errors against
# the FP64 oracle scale with the unit roundoff of the storage type
# (FP32 6e-8, FP16 4.9e-4, BF16 3.9e-3) times a small growth factor.
MIXED = {"fp32": (3, 2e-5), "fp16": (1, 2e-2), "bf16": (2, 1e-1)}


@pytest.fixture(scope="module", params=list(MIXED))
def imported_mixed(bamg, request):
    prec, tol = MIXED[request.param]
    N = 64
    U = inputs.gauge_metropolis(N, 3.0, 40, 5)
    m = -0.05
    kw = dict(n_levels=3, max_coarse=512, setup_sweeps=2, setup_adapt=0)
    h = make_h(bamg, U, m, precision=prec, coarsest_fp32=1, **kw)
    o = oracle.Hierarchy(U, m, **kw)
    for l in range(2):
        P = _random_P(o.P_blocks(l).shape, 100 + l)
        bamg.bamg_import_level(h, l, P)
        o.import_P(l, P)
    return request.param, tol, N, U, m, h, o


@pytest.mark.parametrize("l,nrhs", [(0, 2), (1, 2), (1, 5), (1, 21)])
def test_mixed_apply_and_sweep(bamg, imported_mixed, l, nrhs):
    """On coarse levels nrhs >= 4 runs the MFMA smoother (16 RHS per wave)."""
    name, tol, N, U, m, h, o = imported_mixed
    n = bamg.bamg_level_info(h, l)["n"]
    x = inputs.gaussian((nrhs, n), 160 + l)
    y = torch.zeros(nrhs, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, l, bamg.OP_APPLY_MIXED, dev(x), y, nrhs)
    ea = rel(host(y), o.apply(l, x, nrhs=nrhs).reshape(nrhs, n))
    b = inputs.gaussian((nrhs, n), 170 + l)
    xs = dev(x)
    bamg.bamg_level_op(h, l, bamg.OP_SWEEP_MIXED, dev(b), xs, nrhs)
    es = rel(host(xs), o.sweep(l, x, b, nrhs=nrhs).reshape(nrhs, n))
    # level 0 is FP32 links in every mixed mode
    t = 2e-5 if l == 0 else tol
    log(f"mixed {name} level {l} nrhs {nrhs}: apply err {ea:.2e} sweep err {es:.2e}")
    assert ea < t and es < t


@pytest.mark.parametrize("l,nrhs", [(0, 1), (1, 1), (1, 6)])
def test_f32_operand_ops_match_mixed_ops(bamg, imported_mixed, l, nrhs):
    """Ops 10/11 run the same kernels as ops 7/8 on complex64 operands in
    place: for inputs exactly representable in FP32 the results agree bitwise."""
    name, tol, N, U, m, h, o = imported_mixed
    n = bamg.bamg_level_info(h, l)["n"]
    x = inputs.gaussian((nrhs, n), 180 + l).astype(np.complex64)
    b = inputs.gaussian((nrhs, n), 190 + l).astype(np.complex64)
    y64 = torch.zeros(nrhs, n, dtype=torch.complex128, device="cuda:0")
    bamg.bamg_level_op(h, l, bamg.OP_APPLY_MIXED, dev(x.astype(np.complex128)), y64, nrhs)
    y32 = torch.zeros(nrhs, n, dtype=torch.complex64, device="cuda:0")
    bamg.bamg_level_op(h, l, bamg.OP_APPLY_F32, torch.from_numpy(x).to("cuda:0"), y32, nrhs)
    assert np.array_equal(host(y64).astype(np.complex64), y32.cpu().numpy())
    xs64 = dev(x.astype(np.complex128))
    bamg.bamg_level_op(h, l, bamg.OP_SWEEP_MIXED, dev(b.astype(np.complex128)), xs64, nrhs)
    xs32 = torch.from_numpy(x).to("cuda:0")
    bamg.bamg_level_op(h, l, bamg.OP_SWEEP_F32, torch.from_numpy(b).to("cuda:0"), xs32, nrhs)
    assert np.array_equal(host(xs64).astype(np.complex64), xs32.cpu().numpy())


@pytest.mark.parametrize("nrhs", [1, 3])
def test_mixed_coarse_fused_pairs_give_the_colour_pass_bits(bamg, imported_mixed, nrhs):
    """FP32 sweeps on level 1 with the operator in the storage type: fused
    pairs (op 11) against one launch per colour (op 14)."""
    name, tol, N, U, m, h, o = imported_mixed
    n = bamg.bamg_level_info(h, 1)["n"]
    x1 = torch.from_numpy(inputs.gaussian((nrhs, n), 76).astype(np.complex64)).to("cuda:0")
    b = torch.from_numpy(inputs.gaussian((nrhs, n), 77).astype(np.complex64)).to("cuda:0")
    x2 = x1.clone()
    for _ in range(2):
        bamg.bamg_level_op(h, 1, bamg.OP_SWEEP_F32, b, x1, nrhs)
        bamg.bamg_level_op(h, 1, bamg.OP_SWEEP_COLOURS_F32, b, x2, nrhs)
    assert torch.equal(x1, x2)


def test_mixed_coarse_apply_matrix_cores_against_vector_units(bamg, imported_mixed):
    """From 4 right-hand sides the FP32 coarse apply runs on the matrix cores
    (16 right-hand sides per work-group); 2 at a time it runs on the vector
    units.  Both sum the same 112 FP32 products per entry in different orders:
    they agree to FP32 rounding."""
    name, tol, N, U, m, h, o = imported_mixed
    n = bamg.bamg_level_info(h, 1)["n"]
    R = 20
    x = torch.from_numpy(inputs.gaussian((R, n), 78).astype(np.complex64)).to("cuda:0")
    y = torch.zeros_like(x)
    bamg.bamg_level_op(h, 1, bamg.OP_APPLY_F32, x, y, R)
    y2 = torch.zeros_like(x)
    for r in range(0, R, 2):
        yr = torch.zeros(2, n, dtype=torch.complex64, device="cuda:0")
        bamg.bamg_level_op(h, 1, bamg.OP_APPLY_F32, x[r:r + 2].contiguous(), yr, 2)
        y2[r:r + 2] = yr
    d = rel(y.cpu().numpy().astype(np.complex128), y2.cpu().numpy().astype(np.complex128))
    log(f"coarse apply MFMA vs VALU ({name}): {d:.2e}")
    assert d < 1e-5


U32 = 2.0 ** -24  # unit roundoff of FP32


@pytest.mark.parametrize("nrhs", [1, 2, 3, 9, 17, 40, 70])
def test_mixed_coarsest_solve_fp32_inverse(bamg, imported_mixed, nrhs):
    """Op 12: the mixed cycle's coarsest solve with the FP32 copy of the
    inverse (coarsest_fp32 = 1), complex64 in and out.  nrhs <= 2: the FP32
    copy of the packed gamma5-Hermitian half (64 x 64 blocks on and above the
    diagonal, rounded from the averaged FP64 blocks) with FP64 sums; else the
    split-K MFMA product with the whole FP32 copy (8, 16, 32 and 64 right-hand sides per
    work-group; 70 spans two groups).  Componentwise bounds: rounding the
    inverse to FP32 costs u |A^-1| |b| (u = 2^-24); FP32 sums over the 2n real
    products of a row add at most 2n u |A^-1| |b|."""
    name, tol, N, U, m, h, o = imported_mixed
    L = 2
    n = bamg.bamg_level_info(h, L)["n"]
    b = inputs.gaussian((nrhs, n), 190 + nrhs).astype(np.complex64)
    x = torch.zeros(nrhs, n, dtype=torch.complex64, device="cuda:0")
    bamg.bamg_level_op(h, L, bamg.OP_COARSEST_F32, torch.from_numpy(b).to("cuda:0"), x, nrhs)
    xg = host(x).astype(np.complex128)
    b64 = b.astype(np.complex128)
    ref = o.coarsest_solve(b64, nrhs=nrhs).reshape(nrhs, n)
    Ainv_abs = np.abs(np.linalg.inv(o.operator(L).toarray()))
    scale = np.abs(b64) @ Ainv_abs.T  # (|A^-1| |b_r|)_i per right-hand side
    k = 4 if nrhs <= 2 else 2 * n + 8
    worst = (np.abs(xg - ref) / scale).max()
    log(f"mixed {name} coarsest FP32 nrhs {nrhs}: normwise {rel(xg, ref):.2e}, "
        f"componentwise {worst:.2e} (bound {k * U32:.1e})")
    assert worst <= k * U32
    assert rel(xg, ref) < 1e-4
    if nrhs > 8:  # a column's result does not depend on the other columns of the product
        x9 = torch.zeros(9, n, dtype=torch.complex64, device="cuda:0")
        bamg.bamg_level_op(h, L, bamg.OP_COARSEST_F32, torch.from_numpy(b[:9].copy()).to("cuda:0"), x9, 9)
        assert np.array_equal(host(x9), host(x)[:9])


def test_fp32_coarsest_needs_the_copy(bamg):
    U = inputs.gauge_random(32, 17)
    h = make_h(bamg, U, -0.05, n_levels=2, setup_sweeps=1, setup_adapt=0, precision=1)
    n = bamg.bamg_level_info(h, 1)["n"]
    x = torch.zeros(n, dtype=torch.complex64, device="cuda:0")
    with pytest.raises(bamg.BamgError) as e:
        bamg.bamg_level_op(h, 1, bamg.OP_COARSEST_F32, torch.ones_like(x), x, 1)
    assert e.value.status == bamg.BAMG_EINVAL
    with pytest.raises(bamg.BamgError):
        make_h(bamg, U, -0.05, n_levels=2, coarsest_fp32=1)  # FP64 hierarchy


@pytest.mark.parametrize("prec,c32", [("fp32", 0), ("fp16", 0), ("bf16", 0), ("fp16", 1), ("bf16", 1)])
def test_mixed_solve_reaches_fp64_accuracy(bamg, prec, c32):
    """The FP64 outer FGMRES drives the true residual to 1e-10 whatever the
    precision of the preconditioner (c32: the cycle's coarsest solve reads the
    FP32 copy of the inverse); the solution agrees with the FP64 oracle's to
    the conditioning of the problem."""
    w = inputs.workload("c2_128_b6")
    U = inputs.load_gauge(w)
    N = w["N"]
    tv = oracle.gaussian_tv(N, 8, w["tv_seed"])
    h = make_h(bamg, U, w["m"], n_levels=w["n_levels"], init_tv=tv, precision=MIXED[prec][0], coarsest_fp32=c32)
    b = inputs.gaussian(2 * N * N, w["rhs_seed"])
    x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, info = bamg.bamg_solve(h, dev(b), x, 1e-10)
    xg = host(x)
    o = oracle.Hierarchy(U, w["m"], n_levels=w["n_levels"], init_tv=tv)
    sto, xo, io = o.solve(b, tol=1e-10)
    full = np.linalg.norm(b - oracle.wilson_apply(U, w["m"], xg)) / np.linalg.norm(b)
    dx = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    log(f"mixed {prec} (coarsest fp32 {c32}) solve: iters {info['iters']} (fp64 oracle {io['iters']}), "
        f"full relres {full:.2e}, "
        f"|x - x_fp64|/|x| {dx:.2e}")
    assert st == 0 and info["relres_reduced"] <= 1e-10
    # both solutions have reduced residuals <= 1e-10; their difference is bounded
    # by about tol * cond(Dhat) (~1e-7 here) and measured near 1e-12
    assert full < 2e-10 and dx < 1e-9


def test_work_carried_by_the_fine_sweeps_gives_the_same_bits(bamg):
    """One right-hand side takes the fine sweep blocked in LDS, which carries
    the mixed preconditioner's input conversion and zero start, the
    prolongation into the first post-smoothing sweep and the FP64 output of
    the last (FP32 at 320^2; the FP64 cycle at 256^2 carries the
    prolongation), and every coarse level that is not the coarsest forms its
    residual and the restriction in one launch; two right-hand sides take
    the streaming sweep, the separate conversion, prolongation and conversion
    launches and the separate coarse residual and restriction.  Every other
    kernel of the cycle is the same for both (fused colour pairs on level 1,
    colour passes below, the packed coarsest product), and right-hand sides
    are independent, so the preconditioner (op 9) and the FP64 cycle (op 5)
    give each right-hand side the same bits either way."""
    for prec, op, N, L in ((1, bamg.OP_CYCLE_MIXED, 320, 4), (0, bamg.OP_CYCLE, 256, 3)):
        fp32 = prec != 0
        assert bamg.bamg_fine_sweep_plan(N, 1, fp32=fp32)[0] == 1 and bamg.bamg_fine_sweep_plan(N, 2, fp32=fp32)[0] == 2
        U = inputs.gauge_metropolis(N, 3.0, 20, 11)
        B = dev(inputs.gaussian((2, N * N), 98))
        h = make_h(bamg, U, -0.05, n_levels=L, setup_sweeps=1, setup_adapt=0, precision=prec)
        assert bamg.bamg_n_levels(h) == L
        X2 = torch.zeros_like(B)
        bamg.bamg_level_op(h, 0, op, B, X2, 2)
        for r in range(2):
            x1 = torch.zeros(1, N * N, dtype=torch.complex128, device="cuda:0")
            bamg.bamg_level_op(h, 0, op, B[r:r + 1].contiguous(), x1, 1)
            assert torch.equal(x1[0], X2[r]), (prec, r)
        assert bool(torch.isfinite(X2).all()) and float(X2.abs().max()) > 0
        bamg.bamg_free(h)


@pytest.mark.parametrize("prec,c32", [("fp16", 0), ("bf16", 0), ("fp16", 1)])
def test_mixed_batch_results_do_not_depend_on_the_batch(bamg, prec, c32):
    w = inputs.workload("c1_32_b3")
    U = inputs.load_gauge(w)
    N = w["N"]
    h = make_h(bamg, U, w["m"], n_levels=w["n_levels"], precision=MIXED[prec][0], seed=w["tv_seed"],
               coarsest_fp32=c32)
    R = 19
    B = inputs.gaussian((R, 2 * N * N), 777)
    B[2] *= 1e4
    X = torch.zeros(R, 2 * N * N, dtype=torch.complex128, device="cuda:0")
    st, infos = bamg.bamg_solve_batch(h, dev(B), X, R, 1e-10)
    assert st == 0
    Xb = host(X)
    for r in (0, 2, 17, 18):
        x1 = torch.zeros(1, 2 * N * N, dtype=torch.complex128, device="cuda:0")
        st1, inf1 = bamg.bamg_solve_batch(h, dev(B[r:r + 1]), x1, 1, 1e-10)
        assert st1 == 0 and inf1[0]["iters"] == infos[r]["iters"]
        assert np.array_equal(host(x1)[0], Xb[r])
        full = np.linalg.norm(B[r] - oracle.wilson_apply(U, w["m"], Xb[r])) / np.linalg.norm(B[r])
        assert full < 2e-10


# ---------------------------------------------------------------- hipGraph replay
@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_equals_eager(bamg, prec):
    """graphs = 1 replays each FGMRES iteration as a captured graph (one per
    iteration index, and one per batch size in the batched engine).  Every
    replay, with eager work and synchronisations in between, gives bitwise the
    eager result, single and batched."""
    w = inputs.workload("c1_32_b3")
    U = inputs.load_gauge(w)
    N = w["N"]
    kw = dict(n_levels=w["n_levels"], seed=w["tv_seed"], precision=prec)
    he = make_h(bamg, U, w["m"], **kw)
    hg = make_h(bamg, U, w["m"], graphs=1, **kw)
    B = inputs.gaussian((6, 2 * N * N), 61)
    for rep in range(3):
        for r in range(2):
            b = dev(B[r + rep])
            xe = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
            xg = torch.zeros_like(xe)
            ste, ie = bamg.bamg_solve(he, b, xe, 1e-10)
            junk = torch.randn(1000, device="cuda:0").sum()  # eager work between replays
            stg, ig = bamg.bamg_solve(hg, b, xg, 1e-10)
            torch.cuda.synchronize()
            assert ste == 0 and stg == 0 and ie["iters"] == ig["iters"]
            assert np.array_equal(host(xe), host(xg)), (rep, r)
        for R in (3, 2):
            Xe = torch.zeros(R, 2 * N * N, dtype=torch.complex128, device="cuda:0")
            Xg = torch.zeros_like(Xe)
            bamg.bamg_solve_batch(he, dev(B[:R]), Xe, R, 1e-10)
            float(junk)
            bamg.bamg_solve_batch(hg, dev(B[:R]), Xg, R, 1e-10)
            assert np.array_equal(host(Xe), host(Xg)), (rep, R)


SOLVE_INFO_KEYS = ("iters", "restarts", "relres_reduced", "relres_full", "rho_est")


@pytest.mark.parametrize("prec", [0, 1])
def test_lookahead_gives_the_same_bits(bamg, prec):
    """Look-ahead of the single-RHS FGMRES: iteration j + 1 is queued before
    the host reads iteration j's norms (its results in the second set of host
    slots).  Off (0), while the estimated residual exceeds 1000 tol (1, the
    default) and at every iteration (2, which also leaves a queued iteration
    unused at the end of every pass) give bitwise the same x, status and
    counts, eager and as graphs: at 1e-10, at a loose tolerance, with a
    restart every 3 iterations, and stopped by the iteration cap."""
    w = inputs.workload("c1_32_b3")
    U = inputs.load_gauge(w)
    N = w["N"]
    B = inputs.gaussian((2, 2 * N * N), 71)
    for graphs in (0, 1):
        for restart, max_iter, tols in ((32, 1000, (1e-10, 1e-3)), (3, 1000, (1e-10,)), (32, 4, (1e-14,))):
            log(f"lookahead prec={prec} graphs={graphs} restart={restart} max_iter={max_iter}")
            kw = dict(n_levels=w["n_levels"], seed=w["tv_seed"], precision=prec, graphs=graphs,
                      restart=restart, max_iter=max_iter)
            hs = [make_h(bamg, U, w["m"], lookahead=la, **kw) for la in (0, 1, 2)]
            for tol in tols:
                for r in range(2):
                    b = dev(B[r])
                    res = []
                    for h in hs:
                        x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
                        st, info = bamg.bamg_solve(h, b, x, tol)
                        res.append((st, tuple(info[k] for k in SOLVE_INFO_KEYS), host(x)))
                    st0, info0, x0 = res[0]
                    assert st0 == (1 if max_iter == 4 else 0), (st0, info0)
                    assert info0[0] == min(max_iter, info0[0]) and info0[0] >= 1
                    if restart == 3:
                        assert info0[1] >= 1
                    for la, (st, info, x) in zip((1, 2), res[1:]):
                        assert st == st0 and info == info0, (la, tol, r, info, info0)
                        assert np.array_equal(x, x0), (la, tol, r)
            for h in hs:
                bamg.bamg_free(h)


def test_lookahead_headline_shape(bamg):
    """The single-RHS solve in the shape of the headline (256^2, 3 levels,
    mixed FP16, V(2,2), graphs), with and without look-ahead, twice each: the
    same bits."""
    N = 256
    U = inputs.gauge_metropolis(N, 3.0, 20, 11)
    B = inputs.gaussian((1, 2 * N * N), 72)
    kw = dict(n_levels=3, setup_sweeps=4, setup_adapt=0, precision=1, pre=2, post=2, graphs=1)
    hs = [make_h(bamg, U, -0.05, lookahead=la, **kw) for la in (0, 1)]
    b = dev(B[0])
    res = []
    for h in hs:
        for rep in range(2):
            x = torch.zeros(2 * N * N, dtype=torch.complex128, device="cuda:0")
            st, info = bamg.bamg_solve(h, b, x, 1e-10)
            res.append((st, tuple(info[k] for k in SOLVE_INFO_KEYS), host(x)))
    st0, info0, x0 = res[0]
    assert st0 == 0 and info0[0] >= 3, info0
    for i, (st, info, x) in enumerate(res[1:]):
        assert st == st0 and info == info0, (i, info, info0)
        assert np.array_equal(x, x0), i
    for h in hs:
        bamg.bamg_free(h)
