"""Pins of the oracle's bootstrap multigrid eigensolver (Sec. 3.4, Theorem 1 of
Sec. 3.5) against what linear algebra fixes independently of it:

* the Jacobi eigen-decomposition against LAPACK (numpy.linalg.eigh);
* Theorem 1 (iii): the smallest |eigenvalues| of Z_L = Gamma_5 D_L are the
  smallest singular values of D_L (numpy SVD of the dense coarsest operator),
  which also pins the Gamma_5 convention of the coarse levels;
* the Ritz value of eq. eqevZ (T = I) against v^H Z v / v^H v in dense form;
* the shifted Kaczmarz sweep on (D - lambda Gamma_5) v = 0 against a dense
  row-projection loop in colour order, and an exact eigenpair of Z as its
  fixed point (Theorem 1 (ii));
* the rank-8 least squares fit against the dominant singular subspace of each
  aggregate block (numpy SVD) and, for 8 vectors, against the exact fit;
* the whole bootstrap setup: its Ritz values approach the smallest |eigenvalues|
  of Z_1 = Gamma_e Dhat, and the solver it builds converges.
"""
import numpy as np
import pytest

import inputs
import oracle


def _g5(n, dps):
    if dps == 2:
        return np.tile([1.0, -1.0], n // 2)
    return np.tile(np.repeat([1.0, -1.0], 8), n // 16)


@pytest.mark.parametrize("n,seed", [(5, 1), (16, 2), (33, 3)])
def test_jacobi_matches_lapack(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    H = A + A.conj().T
    w, V = oracle.jacobi_eig(H)
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(H), atol=1e-12 * np.abs(w).max())
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-13
    assert np.abs(V @ np.diag(w) @ V.conj().T - H).max() < 1e-12 * np.abs(H).max()


@pytest.fixture(scope="module")
def h16():
    U = inputs.gauge_metropolis(16, 3.0, 30, 4)
    return oracle.Hierarchy(U, -0.05, n_levels=2, setup_sweeps=8, setup_adapt=0, seed=9), U


def test_coarsest_eigs_are_singular_values(h16):
    """Theorem 1 (i), (iii): sigma = |lambda| with Z_L = Gamma_5 D_L."""
    h, _ = h16
    L = h.n_levels - 1
    D = h.operator(L).toarray()
    n = D.shape[0]
    g = _g5(n, 16)
    Z = g[:, None] * D
    assert np.abs(Z - Z.conj().T).max() < 1e-13 * np.abs(Z).max()
    vals, vecs = h.coarsest_eigs(8)
    sv = np.sort(np.linalg.svd(D, compute_uv=False))[:8]
    assert np.allclose(np.abs(vals), sv, rtol=1e-10, atol=1e-13)
    for lam, v in zip(vals, vecs):
        assert abs(np.linalg.norm(v) - 1) < 1e-12
        assert np.linalg.norm(Z @ v - lam * v) < 1e-10 * np.abs(Z).max()


@pytest.mark.parametrize("l", [0, 1])
def test_ritz_value(h16, l):
    h, _ = h16
    A = h.operator(l).toarray()
    n = A.shape[0]
    g = _g5(n, 2 if l == 0 else 16)
    X = inputs.gaussian((3, n), 40 + l)
    lam = h.ritz(l, X, nrhs=3)
    for j in range(3):
        v = X[j]
        ref = (np.vdot(v, g * (A @ v)) / np.vdot(v, v)).real
        assert abs(lam[j] - ref) < 1e-13 * (1 + abs(ref))


def _order(h, l):
    """The level's Kaczmarz row order: colours in increasing order, sites in
    index order within a colour, the site's dofs in order."""
    inf = h.level_info(l)
    ex, ey, dps = inf["ex"], inf["ey"], inf["dps"]
    order = []
    if l == 0:
        N = ey
        for c in range(16):
            for y in range(N):
                for xh in range(N // 2):
                    x = 2 * xh + (y % 2)
                    if oracle.fine_colour(x, y) == c:
                        order += [2 * (y * (N // 2) + xh), 2 * (y * (N // 2) + xh) + 1]
    else:
        for c in range(oracle.coarse_ncolours(ex, ey)):
            for ay in range(ey):
                for ax in range(ex):
                    if oracle.coarse_colour(ax, ay, ex, ey) == c:
                        order += [(ay * ex + ax) * dps + d for d in range(dps)]
    return order


@pytest.mark.parametrize("l", [0, 1])
def test_shifted_sweep_equals_dense_projections(h16, l):
    h, _ = h16
    A = h.operator(l).toarray()
    n = A.shape[0]
    g = _g5(n, 2 if l == 0 else 16)
    lam = 0.37
    As = A - lam * np.diag(g)
    x = inputs.gaussian(n, 50 + l)
    ref = x.copy()
    for r in _order(h, l):
        d = As[r]
        ref = ref + ((0 - d @ ref) / np.vdot(d, d).real) * d.conj()
    got = h.sweep_shifted(l, x, [lam])
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("l", [0, 1])
def test_exact_eigenpair_is_a_fixed_point(h16, l):
    """Theorem 1 (ii): Kaczmarz on (D - lambda Gamma_5) v = 0 is Kaczmarz on
    (Z - lambda) v = 0, which an exact eigenpair of Z satisfies."""
    h, _ = h16
    A = h.operator(l).toarray()
    n = A.shape[0]
    g = _g5(n, 2 if l == 0 else 16)
    w, V = np.linalg.eigh(g[:, None] * A)
    k = int(np.argmin(np.abs(w)))
    v = V[:, k]
    got = h.sweep_shifted(l, v, [w[k]])
    assert np.linalg.norm(got - v) < 1e-11
    assert np.linalg.norm(h.sweep_shifted(l, v, [w[k] + 0.3]) - v) > 1e-3


def test_ls_fit_spans_dominant_singular_subspace():
    U = inputs.gauge_metropolis(16, 3.0, 30, 4)
    h = oracle.Hierarchy(U, -0.05, n_levels=2, setup_sweeps=4, setup_adapt=0, seed=9)
    n = 16 * 16
    V = inputs.gaussian((16, n), 60)
    h.fit_ls(0, V)
    P = h.P_blocks(0)  # [agg][s][row][8]
    na = P.shape[0]
    # aggregate a = (y // 4) * (NH / 4) + xh // 4, row = 4 (y % 4) + xh % 4; dof = 2 site + s
    NH = 8
    blocks = np.zeros((na, 2, 16, 16), dtype=complex)
    for y in range(16):
        for xh in range(NH):
            a, row = (y // 4) * (NH // 4) + xh // 4, 4 * (y % 4) + xh % 4
            for s in range(2):
                blocks[a, s, row, :] = V[:, 2 * (y * NH + xh) + s]
    for a in range(na):
        for s in range(2):
            B = blocks[a, s]
            Q = P[a, s]
            assert np.abs(Q.conj().T @ Q - np.eye(8)).max() < 1e-12
            Uu, S, _ = np.linalg.svd(B)
            Pi = Uu[:, :8] @ Uu[:, :8].conj().T
            assert np.abs(Q @ Q.conj().T - Pi).max() < 1e-10
            # basis: Gram-Schmidt of the projected first 8 vectors (R_jj > 0)
            W = Pi @ B[:, :8]
            q, r = np.linalg.qr(W)
            ph = np.sign(np.diag(r).real)
            assert np.abs(Q - q * ph).max() < 1e-9
    # with 8 vectors the fit is the exact one of the relax-fit setup
    h.fit_ls(0, V[:8])
    P8 = h.P_blocks(0)
    h2 = oracle.Hierarchy(U, -0.05, n_levels=2, setup_sweeps=0, setup_adapt=0, init_tv=V[:8])
    assert np.abs(P8 - h2.P_blocks(0)).max() < 1e-13


@pytest.mark.parametrize("boot", [1, 2])
def test_bootstrap_setup_finds_small_eigenvalues_and_converges(boot):
    """W (boot = 1) and super-V (boot = 2) schedules on a 32^2 lattice with 3
    levels (coarsest 128 unknowns)."""
    N = 32
    U = inputs.gauge_metropolis(N, 3.0, 60, 11)
    m = -0.12
    h = oracle.Hierarchy(U, m, n_levels=3, boot=boot, k_e=8, nu1=10, nu2=5, seed=12)
    lam, ve = h.boot_vectors()
    assert lam.shape == (8,)
    Dh = oracle.dhat_dense(U, m)
    g = np.tile([1.0, -1.0], N * N // 2)
    ev = np.linalg.eigvalsh(g[:, None] * Dh)
    smallest = np.sort(np.abs(ev))[:8]
    # the eigenvector approximations are Ritz vectors of Z_1 with small Ritz values
    assert np.abs(lam).min() < 1.5 * smallest[0]
    assert np.median(np.abs(lam)) < 10 * smallest[7]
    for j in range(8):
        assert abs(h.ritz(0, ve[j]) - lam[j]) < 1e-12 * (1 + abs(lam[j]))
    b = inputs.gaussian(2 * N * N, 13)
    st, x, info = h.solve(b, tol=1e-10)
    assert st == 0 and info["relres"] <= 1e-10
    full = np.linalg.norm(b - oracle.wilson_apply(U, m, x)) / np.linalg.norm(b)
    assert full < 2e-10
