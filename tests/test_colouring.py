"""The GPU smoother kernels enumerate the sites of a colour arithmetically
(no site tables).  These CPU tests restate those enumerations and check that,
for every colour, they produce exactly the oracle's colour class: each site
once per sweep, in the colour the oracle assigns (Sec. 3.1 multicolouring)."""
import pytest

import oracle


def fine_colour_site(c, t, N):
    # rows y = a - b (mod 4), x = 2a - y (mod 8) for colour c = 4a + b
    a, b, per = c >> 2, c & 3, N >> 3
    r, k = divmod(t, per)
    y = 4 * r + ((a - b) & 3)
    x = 8 * k + ((2 * a - y) & 7)
    return x, y


def coarse_colour_site(c, mode, t, ex):
    if mode == 8:
        per = ex >> 3
        ay = t // per
        return ay * ex + 8 * (t - ay * per) + ((c + 3 * ay) & 7)
    if mode == 16:
        per = ex >> 2
        r = t // per
        return (4 * r + (c >> 2)) * ex + 4 * (t - r * per) + (c & 3)
    return c


@pytest.mark.parametrize("N", [16, 24, 32, 40, 64, 256])
def test_fine_enumeration_is_the_oracle_colouring(N):
    seen = set()
    for c in range(16):
        for t in range(N * N // 32):
            x, y = fine_colour_site(c, t, N)
            assert 0 <= x < N and 0 <= y < N and (x + y) % 2 == 0
            assert oracle.fine_colour(x, y) == c
            seen.add((x, y))
    assert len(seen) == N * N // 2


@pytest.mark.parametrize("ex,ey", [(8, 16), (16, 32), (32, 64), (4, 8), (12, 12), (4, 4), (3, 6)])
def test_coarse_enumeration_is_the_oracle_colouring(ex, ey):
    nc = oracle.coarse_ncolours(ex, ey)
    mode = 8 if nc == 8 else (16 if nc == 16 else 1)
    per = ex * ey // (mode if mode != 1 else ex * ey)
    seen = set()
    for c in range(nc):
        for t in range(per):
            s = coarse_colour_site(c, mode, t, ex)
            assert 0 <= s < ex * ey
            assert oracle.coarse_colour(s % ex, s // ex, ex, ey) == c
            seen.add(s)
    assert len(seen) == ex * ey
