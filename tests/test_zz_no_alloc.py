"""The allocation-free residual entry point (bamg_full_residual_noalloc, for
callers that cannot allocate device memory) against the allocating one
(bamg_full_residual) and the oracle's Wilson operator (eq. wilson), on two
calls in a row with the second input smaller, through the C ABI."""
import numpy as np
import pytest

import inputs
import oracle

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


def test_noalloc_residual_matches_allocating_entry_point(bamg):
    for call, (N, nrhs) in enumerate([(128, 5), (64, 2)]):
        print(f"no-alloc residual: call {call}, N={N}, nrhs={nrhs}", flush=True)
        U = inputs.gauge_random(N, 40 + N)
        m = -0.02
        B = inputs.gaussian((nrhs, 2 * N * N), 41 + N)
        X = inputs.gaussian((nrhs, 2 * N * N), 42 + N)
        if call == 0:
            B[3] = 0  # a zero right-hand side gives ||D x||
        Ud, Bd, Xd = dev(U), dev(B), dev(X)
        ref = torch.zeros(nrhs, dtype=torch.float64, device="cuda:0")
        got = torch.full((nrhs,), -1.0, dtype=torch.float64, device="cuda:0")
        bamg.bamg_full_residual(N, Ud, m, Bd, Xd, nrhs, ref)
        bamg.bamg_full_residual_noalloc(N, Ud, m, Bd, Xd, nrhs, got)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        # the same kernels and block decomposition: the same bits
        assert np.array_equal(g, r), (g, r)
        for k in range(nrhs):
            res = np.linalg.norm(B[k] - oracle.wilson_apply(U, m, X[k]))
            o = res / np.linalg.norm(B[k]) if B[k].any() else res
            assert abs(g[k] - o) <= 1e-13 * o, (k, g[k], o)


def test_noalloc_rejects_more_than_its_scratch(bamg):
    """2 * 256 partial sums per right-hand side at N >= 512: 257 right-hand
    sides exceed the 131072 doubles of the static array.  The call fails on
    the host before any launch."""
    t = torch.zeros(4, dtype=torch.complex128, device="cuda:0")
    out = torch.zeros(257, dtype=torch.float64, device="cuda:0")
    with pytest.raises(bamg.BamgError) as e:
        bamg.bamg_full_residual_noalloc(4096, t, 0.0, t, t, 257, out)
    assert e.value.status == bamg.BAMG_EINVAL
    assert "static scratch" in bamg.bamg_last_error()
