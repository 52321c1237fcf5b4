"""Pins of the oracle's multicolour Kaczmarz smoother (Sec. 3.1).

* the colour classes have disjoint column support (the property that makes a
  colour pass parallel), checked by brute force on the operator's pattern;
* one sweep equals a brute-force dense row-projection loop (written here from
  the definition x += (r_i / ||d_i||^2) d_i^H, in colour order);
* the properties of a sequence of orthogonal projections: the error of a
  consistent system never grows, and the residual of a row vanishes right
  after the row is projected.
"""
import numpy as np
import pytest

import inputs
import oracle


def _fine_colour_rule(x, y):
    u = (x + y) // 2
    v = (x - y) // 2
    return 4 * (u % 4) + (v % 4)


def _even_sites(N):
    return [(2 * xh + (y % 2), y) for y in range(N) for xh in range(N // 2)]


@pytest.mark.parametrize("N", [8, 16, 32])
def test_fine_colours_have_disjoint_support(N):
    Dh = oracle.dhat_dense(inputs.gauge_random(N, 1), 0.1)
    pat = np.abs(Dh) > 0
    sites = _even_sites(N)
    cols = np.array([oracle.fine_colour(x, y) for (x, y) in sites])
    assert set(cols.tolist()) == set(range(16))
    for (x, y), c in zip(sites, cols):
        assert c == _fine_colour_rule(x, y)
    for c in range(16):
        idx = np.nonzero(cols == c)[0]
        rows = np.stack([2 * idx, 2 * idx + 1], axis=1).reshape(-1)
        # every column is touched by at most one site of the colour
        touched = pat[rows].reshape(len(idx), 2, -1).any(axis=1).sum(axis=0)
        assert touched.max() <= 1


@pytest.mark.parametrize("ex,ey", [(8, 8), (8, 16), (16, 32), (4, 8), (4, 4), (32, 64)])
def test_coarse_colours_have_disjoint_support(ex, ey):
    offs = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]
    ncol = oracle.coarse_ncolours(ex, ey)
    colour = {(ax, ay): oracle.coarse_colour(ax, ay, ex, ey) for ay in range(ey) for ax in range(ex)}
    assert set(colour.values()) == set(range(ncol))
    for c in range(ncol):
        seen = set()
        for (ax, ay), cc in colour.items():
            if cc != c:
                continue
            sup = {((ax + dx) % ex, (ay + dy) % ey) for dx, dy in offs}
            assert not (sup & seen)
            seen |= sup
    if ex % 8 == 0 and ey % 8 == 0:
        assert ncol == 8


def _brute_sweep(Dh, order, x, b):
    x = x.copy()
    for r in order:
        d = Dh[r]
        alpha = (b[r] - d @ x) / np.vdot(d, d).real
        x = x + alpha * d.conj()
    return x


def test_sweep_equals_dense_row_projection_loop():
    N = 16
    U = inputs.gauge_random(N, 2)
    m = 0.05
    Dh = oracle.dhat_dense(U, m)
    x0 = inputs.gaussian(N * N, 3)
    b = inputs.gaussian(N * N, 4)
    sites = _even_sites(N)
    order = []
    for c in range(16):
        for e, (x, y) in enumerate(sites):
            if _fine_colour_rule(x, y) == c:
                order += [2 * e, 2 * e + 1]
    ref = _brute_sweep(Dh, order, x0, b)
    got = oracle.kaczmarz_fine(U, m, x0, b, sweeps=1)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-13


def test_projection_properties():
    N = 8
    U = inputs.gauge_random(N, 5)
    m = 0.1
    Dh = oracle.dhat_dense(U, m)
    xs = inputs.gaussian(N * N, 6)
    b = Dh @ xs
    x = np.zeros(N * N, complex)
    err = [np.linalg.norm(x - xs)]
    for _ in range(6):
        x = oracle.kaczmarz_fine(U, m, x, b, sweeps=1)
        err.append(np.linalg.norm(x - xs))
    assert all(err[i + 1] <= err[i] * (1 + 1e-14) for i in range(len(err) - 1))
    # residual of a row vanishes right after that row is projected
    d = Dh[5]
    x1 = x + ((b[5] - d @ x) / np.vdot(d, d).real) * d.conj()
    assert abs(b[5] - d @ x1) < 1e-14 * np.linalg.norm(b)


def test_homogeneous_sweeps_damp_large_singular_components():
    """Kaczmarz on Dhat v = 0 reduces ||Dhat v|| / ||v|| (smoothing, Sec. 3.1/3.4)."""
    N = 16
    U = inputs.gauge_random(N, 8)
    m = 0.05
    v = inputs.gaussian(N * N, 9)
    r0 = np.linalg.norm(oracle.dhat_apply(U, m, v)) / np.linalg.norm(v)
    v = oracle.kaczmarz_fine(U, m, v, None, sweeps=10)
    r1 = np.linalg.norm(oracle.dhat_apply(U, m, v)) / np.linalg.norm(v)
    assert r1 < 0.6 * r0
