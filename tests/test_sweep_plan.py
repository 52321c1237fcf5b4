"""The tile plan of the level-0 sweep blocked in LDS, checked on the CPU.

The library blocks the 16-colour Kaczmarz sweep (Sec. 3.1) in tiles of the
even sites: each tile's work-group projects, colour by colour, every site its
tile's final values depend on, from a region of x read at the start.  Here the
plan the library computes (`bamg_fine_sweep_plan`) is replayed on random 2 x 2
coupling blocks with a generic two-row projection and compared with the
colour-by-colour sweep: the values of every tile must come out bitwise equal.
The pipelined form's schedule (a ring of columns marched down v, colours
offset by one macro-step) is replayed the same way.
A plan that misses a dependence (a region or a colour's site range too small)
or wraps onto itself on the torus fails this test."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1308_5992_amd", "libbamg.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libbamg.so not built")

# (du, dv) of the 9 support sites, the slot order of the kernels
SLOTS = [(0, 0), (1, 1), (-1, -1), (1, -1), (-1, 1), (1, 0), (0, 1), (0, -1), (-1, 0)]


def _site(N, u, v):
    x, y = (u + v) % N, (u - v) % N
    return y * (N // 2) + (x >> 1)


def _project(B, b, xs):
    """Row pair (d_0, d_1) = B[:, slot] against the support values xs[slot]
    (arrays over projections): the two sequential projections of Sec. 3.1."""
    r0 = sum(B[:, n, 0, 0] * xs[n][:, 0] + B[:, n, 0, 1] * xs[n][:, 1] for n in range(9))
    r1 = sum(B[:, n, 1, 0] * xs[n][:, 0] + B[:, n, 1, 1] * xs[n][:, 1] for n in range(9))
    nu0 = sum(np.abs(B[:, n, 0, 0]) ** 2 + np.abs(B[:, n, 0, 1]) ** 2 for n in range(9))
    nu1 = sum(np.abs(B[:, n, 1, 0]) ** 2 + np.abs(B[:, n, 1, 1]) ** 2 for n in range(9))
    g10 = sum(np.conj(B[:, n, 0, 0]) * B[:, n, 1, 0] + np.conj(B[:, n, 0, 1]) * B[:, n, 1, 1] for n in range(9))
    a0 = (b[:, 0] - r0) / nu0
    a1 = (b[:, 1] - r1 - g10 * a0) / nu1
    return [np.stack([xs[n][:, 0] + np.conj(B[:, n, 0, 0]) * a0 + np.conj(B[:, n, 1, 0]) * a1,
                      xs[n][:, 1] + np.conj(B[:, n, 0, 1]) * a0 + np.conj(B[:, n, 1, 1]) * a1], axis=1)
            for n in range(9)]


def _colour_sweep(N, Bst, b, x):
    x = x.copy()
    u = np.arange(N)[:, None].repeat(N // 2, 1).ravel()
    v = np.arange(N // 2)[None, :].repeat(N, 0).ravel()
    s = _site(N, u, v)
    colour = 4 * (u % 4) + (v % 4)
    for c in range(16):
        sel = colour == c
        su, sv, ss = u[sel], v[sel], s[sel]
        nb = [_site(N, su + du, sv + dv) for du, dv in SLOTS]
        new = _project(Bst[ss], b[ss], [x[k] for k in nb])
        for k, val in zip(nb, new):
            x[k] = val
    return x


def _blocked_sweep(N, p, Bst, b, x0):
    out = x0.copy()
    for a in range(p["ntu"]):
        for bb in range(p["ntv"]):
            u0, v0 = 1 + a * p["Tu"], 1 + bb * p["Tv"]
            Ru, Rv, i0, j0 = p["Ru"], p["Rv"], p["i0"], p["j0"]
            li, lj = np.meshgrid(np.arange(Ru), np.arange(Rv), indexing="ij")
            L = x0[_site(N, u0 + i0 + li, v0 + j0 + lj)].copy()  # [Ru][Rv][2]
            for c in range(16):
                cnt = p["first"][c + 1] - p["first"][c]
                if cnt == 0:
                    continue
                k = np.arange(cnt)
                i = p["si0"][c] + 4 * (k // p["nj"][c])
                j = p["sj0"][c] + 4 * (k % p["nj"][c])
                assert (i - i0 >= 1).all() and (i - i0 <= Ru - 2).all() and (j - j0 >= 1).all() and (j - j0 <= Rv - 2).all()
                assert ((4 * ((u0 + i) % 4) + (v0 + j) % 4) == c).all()
                ss = _site(N, u0 + i, v0 + j)
                loc = [(i - i0 + du, j - j0 + dv) for du, dv in SLOTS]
                new = _project(Bst[ss], b[ss], [L[li_, lj_] for li_, lj_ in loc])
                for (li_, lj_), val in zip(loc, new):
                    L[li_, lj_] = val
            ti, tj = np.meshgrid(np.arange(p["Tu"]), np.arange(p["Tv"]), indexing="ij")
            out[_site(N, u0 + ti, v0 + tj)] = L[ti - i0, tj - j0]
    return out


def _pipelined_sweep(N, p, Bst, b, x0):
    """The pipelined form's schedule, as the kernel runs it: a ring of W
    region columns; at macro-step m every (colour c, row) pair with
    0 <= m - c < nj[c] projects at once (their supports must be disjoint and in
    the ring), then the columns of macro-step m + 1 take their ring slots,
    writing the evicted column out if it belongs to the tile."""
    out = x0.copy()
    A, M, W = p["A"], p["M"], p["W"]
    Ru, Rv, i0, j0 = p["Ru"], p["Rv"], p["i0"], p["j0"]
    rows = [(p["first"][c + 1] - p["first"][c]) // p["nj"][c] if p["nj"][c] else 0 for c in range(16)]
    assert M == max(c + p["nj"][c] for c in range(16) if rows[c])

    def load_step(cj):
        return max(0, (cj + j0 - A) // 4)

    for a in range(p["ntu"]):
        for bb in range(p["ntv"]):
            u0, v0 = 1 + a * p["Tu"], 1 + bb * p["Tv"]
            ring = {}  # slot -> [region column, values [Ru][2], rhs [Ru][2]]
            written = set()

            def place(cj):
                sl = cj % W
                if sl in ring:
                    old = ring[sl][0]
                    assert old == cj - W
                    for ri in range(Ru):
                        if 0 <= ri + i0 < p["Tu"] and 0 <= old + j0 < p["Tv"]:
                            out[_site(N, u0 + i0 + ri, v0 + j0 + old)] = ring[sl][1][ri]
                            written.add((ri + i0, old + j0))
                ss = _site(N, u0 + i0 + np.arange(Ru), v0 + j0 + cj)
                ring[sl] = [cj, x0[ss].copy(), b[ss].copy()]

            for cj in range(Rv):
                if load_step(cj) == 0:
                    place(cj)
            for m in range(M):
                jobs = []
                for c in range(16):
                    k = m - c
                    if rows[c] == 0 or not 0 <= k < p["nj"][c]:
                        continue
                    for r in range(rows[c]):
                        i, j = p["si0"][c] + 4 * r, p["sj0"][c] + 4 * k
                        assert 4 * ((u0 + i) % 4) + (v0 + j) % 4 == c
                        jobs.append((i - i0, j - j0, _site(N, u0 + i, v0 + j)))
                sup = [(ri + du, cj + dv) for ri, cj, _ in jobs for du, dv in SLOTS]
                assert len(set(sup)) == len(sup)  # one macro-step's projections are independent
                for ri, cj in sup:
                    assert 0 <= ri < Ru and ring[cj % W][0] == cj  # in the ring when used
                for ri, cj, ss in jobs:
                    loc = [(ri + du, cj + dv) for du, dv in SLOTS]
                    new = _project(Bst[[ss]], ring[cj % W][2][[ri]], [ring[c_ % W][1][[r_]] for r_, c_ in loc])
                    for (r_, c_), val in zip(loc, new):
                        ring[c_ % W][1][r_] = val[0]
                if m + 1 < M:
                    for cj in range(Rv):
                        if load_step(cj) == m + 1:
                            place(cj)
            for cj in range(max(0, Rv - W), Rv):
                assert ring[cj % W][0] == cj
                for ri in range(Ru):
                    if 0 <= ri + i0 < p["Tu"] and 0 <= cj + j0 < p["Tv"]:
                        out[_site(N, u0 + i0 + ri, v0 + j0 + cj)] = ring[cj % W][1][ri]
                        written.add((ri + i0, cj + j0))
            assert len(written) == p["Tu"] * p["Tv"]
    return out


@pytest.mark.parametrize("N,nrhs,fp32,form", [(64, 1, 0, 1), (80, 3, 0, 1), (96, 1, 1, 1), (128, 64, 1, 1),
                                              (128, 64, 0, 1), (128, 64, 1, 2), (128, 64, 0, 2), (96, 64, 1, 2)])
def test_blocked_sweep_plan_reproduces_the_colour_sweep(N, nrhs, fp32, form):
    import paper_1308_5992_amd as bamg
    got, p = bamg.bamg_fine_sweep_plan(N, nrhs, fp32, form)
    assert got == form and p is not None
    assert p["ntu"] * p["Tu"] == N and p["ntv"] * p["Tv"] == N // 2 and p["nupd"] == p["first"][16]
    assert p["Tu"] % 4 == 0 and p["Tv"] % 4 == 0
    # the region holds no site twice on the torus
    assert p["Ru"] <= N and p["Rv"] <= N and (2 * p["Ru"] <= N or 2 * p["Rv"] <= N)
    rng = np.random.default_rng(N + 7 * form + 3 * fp32)
    ns = N * N // 2
    Bst = rng.standard_normal((ns, 9, 2, 2)) + 1j * rng.standard_normal((ns, 9, 2, 2))
    b = rng.standard_normal((ns, 2)) + 1j * rng.standard_normal((ns, 2))
    x0 = rng.standard_normal((ns, 2)) + 1j * rng.standard_normal((ns, 2))
    ref = _colour_sweep(N, Bst, b, x0)
    out = _blocked_sweep(N, p, Bst, b, x0)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("N,fp32", [(64, 0), (128, 1), (192, 0)])
def test_pipelined_sweep_schedule_reproduces_the_colour_sweep(N, fp32):
    """The pipelined form: the tile's projections in macro-step order with
    the ring's loads and write-backs, against the colour-by-colour sweep."""
    import paper_1308_5992_amd as bamg
    got, p = bamg.bamg_fine_sweep_plan(N, 1, fp32, 3)
    assert got == 3 and p["Tu"] == 16 and p["W"] > 0
    assert p["ntu"] * p["Tu"] == N and p["ntv"] * p["Tv"] == N // 2
    rng = np.random.default_rng(N + 11 * fp32)
    ns = N * N // 2
    Bst = rng.standard_normal((ns, 9, 2, 2)) + 1j * rng.standard_normal((ns, 9, 2, 2))
    b = rng.standard_normal((ns, 2)) + 1j * rng.standard_normal((ns, 2))
    x0 = rng.standard_normal((ns, 2)) + 1j * rng.standard_normal((ns, 2))
    assert np.array_equal(_pipelined_sweep(N, p, Bst, b, x0), _colour_sweep(N, Bst, b, x0))


def test_library_choice_of_the_sweep_form():
    """The form the library runs: LDS-resident while x is at most 1 MiB,
    streaming up to 2^20 (FP32) / 2^18 (FP64) entries, pipelined beyond
    (where N is a multiple of 16 and N/2 of 32), else colour passes; no tile
    below N = 64 or where N/2 is not a multiple of 8."""
    import paper_1308_5992_amd as bamg
    assert bamg.bamg_fine_sweep_plan(256, 1, True)[0] == 1
    assert bamg.bamg_fine_sweep_plan(256, 1, False)[0] == 1
    assert bamg.bamg_fine_sweep_plan(512, 1, True)[0] == 2
    assert bamg.bamg_fine_sweep_plan(512, 1, False)[0] == 2
    assert bamg.bamg_fine_sweep_plan(512, 3, False)[0] == 3
    assert bamg.bamg_fine_sweep_plan(4096, 1, True)[0] == 3
    assert bamg.bamg_fine_sweep_plan(4096, 1, False)[0] == 3
    assert bamg.bamg_fine_sweep_plan(1000, 1, False)[0] == 0
    assert bamg.bamg_fine_sweep_plan(40, 1, True)[0] == 0
    assert bamg.bamg_fine_sweep_plan(72, 1, True)[0] == 0
    with pytest.raises(bamg.BamgError):
        bamg.bamg_fine_sweep_plan(256, 0, True)
