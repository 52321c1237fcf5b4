"""The fused colour pairs of the coarse smoother, checked on the CPU.

The library runs colours c and c + 1 (c even) of the 8-colouring
(ax - 3 ay) mod 8 of a coarse level in one launch (Sec. 3.1 fixes only that
sites of one colour have disjoint supports): a work-group per site s of colour
c + 1 projects the two sites t1 = s + (-1, 0) and t2 = s + (2, 1) of colour c,
then s, from the values of x on the 15 sites of their supports, and writes the
support of s and the site s + (-1, 1).  Here that schedule is replayed on
random block rows with a generic projection and compared bitwise with the
colour-by-colour sweep, on tori from 8 x 8 sites: a colour-c site missing
from a work-group's list, or a site written twice or never, fails."""
import numpy as np
import pytest

# the 7 offsets of the coarse stencil, in the kernels' order
OFF = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]


def _colour(ax, ay):
    return (ax - 3 * ay) % 8


def _project(A, b, xs):
    """One site's block of rows A (d x 7d) against its support values xs (7 x d):
    the d sequential row projections."""
    x = np.concatenate(xs).copy()
    for i in range(A.shape[0]):
        a = A[i]
        x += np.conj(a) * (b[i] - a @ x) / np.vdot(a, a).real
    d = len(xs[0])
    return [x[k * d:(k + 1) * d] for k in range(7)]


def _site(ex, ey, ax, ay):
    return (ay % ey) * ex + (ax % ex)


def _colour_sweep(ex, ey, A, b, x):
    x = x.copy()
    for c in range(8):
        for ay in range(ey):
            for ax in range(ex):
                if _colour(ax, ay) != c:
                    continue
                s = _site(ex, ey, ax, ay)
                sup = [_site(ex, ey, ax + dx, ay + dy) for dx, dy in OFF]
                for k, v in zip(sup, _project(A[s], b[s], [x[j] for j in sup])):
                    x[k] = v
    return x


def _pair_sweep(ex, ey, A, b, x):
    for c in range(0, 8, 2):
        xin, xout = x, np.full_like(x, np.nan)
        written = np.zeros(ex * ey, dtype=int)
        for ay in range(ey):
            for ax in range(ex):
                if _colour(ax, ay) != c + 1:
                    continue
                loc = {}  # this work-group's copy of x on the supports it projects

                def get(px, py):
                    j = _site(ex, ey, px, py)
                    if j not in loc:
                        loc[j] = xin[j].copy()
                    return j

                for tx, ty in ((ax - 1, ay), (ax + 2, ay + 1)):
                    assert _colour(tx % ex, ty % ey) == c
                    t = _site(ex, ey, tx, ty)
                    sup = [get(tx + dx, ty + dy) for dx, dy in OFF]
                    for k, v in zip(sup, _project(A[t], b[t], [loc[j] for j in sup])):
                        loc[k] = v
                s = _site(ex, ey, ax, ay)
                sup = [get(ax + dx, ay + dy) for dx, dy in OFF]
                for k, v in zip(sup, _project(A[s], b[s], [loc[j] for j in sup])):
                    loc[k] = v
                for j in sup + [get(ax - 1, ay + 1)]:
                    xout[j] = loc[j]
                    written[j] += 1
        assert (written == 1).all()
        x = xout
    return x


@pytest.mark.parametrize("ex,ey", [(8, 8), (16, 8), (8, 16), (24, 16)])
def test_fused_pairs_reproduce_the_colour_sweep(ex, ey):
    rng = np.random.default_rng(ex * 100 + ey)
    d = 3  # unknowns per site (16 in the library; the schedule does not depend on it)
    ns = ex * ey
    A = rng.standard_normal((ns, d, 7 * d)) + 1j * rng.standard_normal((ns, d, 7 * d))
    b = rng.standard_normal((ns, d)) + 1j * rng.standard_normal((ns, d))
    x0 = rng.standard_normal((ns, d)) + 1j * rng.standard_normal((ns, d))
    assert np.array_equal(_pair_sweep(ex, ey, A, b, x0), _colour_sweep(ex, ey, A, b, x0))


def test_a_missing_dependence_is_caught():
    """Without t2 the replay differs from the colour sweep (the test above
    would catch a schedule that misses a dependence)."""
    ex, ey, d = 8, 8, 2
    rng = np.random.default_rng(3)
    ns = ex * ey
    A = rng.standard_normal((ns, d, 7 * d)) + 1j * rng.standard_normal((ns, d, 7 * d))
    b = rng.standard_normal((ns, d)) + 1j * rng.standard_normal((ns, d))
    x0 = rng.standard_normal((ns, d)) + 1j * rng.standard_normal((ns, d))
    ref = _colour_sweep(ex, ey, A, b, x0)
    # the pair schedule with t2 left out
    x = x0
    for c in range(0, 8, 2):
        xin, xout = x, x.copy()
        for ay in range(ey):
            for ax in range(ex):
                if _colour(ax, ay) != c + 1:
                    continue
                loc = {}

                def get(px, py):
                    j = _site(ex, ey, px, py)
                    if j not in loc:
                        loc[j] = xin[j].copy()
                    return j

                t = _site(ex, ey, ax - 1, ay)
                sup = [get(ax - 1 + dx, ay + dy) for dx, dy in OFF]
                for k, v in zip(sup, _project(A[t], b[t], [loc[j] for j in sup])):
                    loc[k] = v
                s = _site(ex, ey, ax, ay)
                sup = [get(ax + dx, ay + dy) for dx, dy in OFF]
                for k, v in zip(sup, _project(A[s], b[s], [loc[j] for j in sup])):
                    loc[k] = v
                for j in sup + [get(ax - 1, ay + 1)]:
                    xout[j] = loc[j]
        x = xout
    assert not np.allclose(x, ref)
