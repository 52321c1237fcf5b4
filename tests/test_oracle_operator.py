"""Pins of the oracle's Wilson operator, odd-even reduction and gamma5 structure.

Each test checks the oracle against something the paper or mathematics fixes
independently of the oracle's own code: the spin-block form eq. (bst), the
gamma5 symmetry (Sec. 2.2, eq. eqevZ2), the free-field closed-form spectrum
(Sec. 2, remark after eq. bst), the Schur complement identity (Sec. 3.2) and
dense LAPACK solves.
"""
import numpy as np
import pytest

import inputs
import oracle


def _eo_index(N):
    """half-x even and odd site lists -> full-lattice site index."""
    ev, od = [], []
    for y in range(N):
        for xh in range(N // 2):
            ev.append(y * N + 2 * xh + (y % 2))
            od.append(y * N + 2 * xh + 1 - (y % 2))
    return np.array(ev), np.array(od)


def _dofs(sites):
    return np.stack([2 * sites, 2 * sites + 1], axis=1).reshape(-1)


def _paper_bst_dense(U, m):
    """D from eq. (bst): 1/2 [[A, B], [-B^H, A]] in spin-major order, built
    with the links conjugated (the convention of eq. wilson), then permuted to
    site-major order (site, spin)."""
    V = np.conj(U)
    N = U.shape[-1]
    n = N * N
    A = np.zeros((n, n), complex)
    B = np.zeros((n, n), complex)
    idx = lambda x, y: (y % N) * N + (x % N)
    for y in range(N):
        for x in range(N):
            z = idx(x, y)
            A[z, z] += 4 + 2 * m
            A[z, idx(x - 1, y)] -= V[0, y, (x - 1) % N]
            A[z, idx(x, y - 1)] -= V[1, (y - 1) % N, x]
            A[z, idx(x + 1, y)] -= np.conj(V[0, y, x])
            A[z, idx(x, y + 1)] -= np.conj(V[1, y, x])
            B[z, idx(x + 1, y)] += np.conj(V[0, y, x])
            B[z, idx(x - 1, y)] -= V[0, y, (x - 1) % N]
            B[z, idx(x, y + 1)] += 1j * np.conj(V[1, y, x])
            B[z, idx(x, y - 1)] -= 1j * V[1, (y - 1) % N, x]
    D = 0.5 * np.block([[A, B], [-B.conj().T, A]])
    perm = np.empty(2 * n, int)
    perm[0::2] = np.arange(n)          # site z, spin 0 <- spin-major row z
    perm[1::2] = n + np.arange(n)      # site z, spin 1 <- row n + z
    return D[np.ix_(perm, perm)]


@pytest.mark.parametrize("N,seed", [(4, 1), (8, 2)])
def test_wilson_equals_block_spin_form(N, seed):
    """eq. (wilson) equals eq. (bst) with the link convention of eq. (wilson)."""
    U = inputs.gauge_random(N, seed)
    m = -0.3
    D = oracle.wilson_dense(U, m)
    assert np.abs(D - _paper_bst_dense(U, m)).max() < 1e-14


@pytest.mark.parametrize("N", [4, 8])
def test_gamma5_hermiticity(N):
    """Gamma5 D Gamma5 = D^H and Gamma_e Dhat Gamma_e = Dhat^H (Sec. 2.2, 3.2)."""
    U = inputs.gauge_random(N, 7)
    m = 0.05
    D = oracle.wilson_dense(U, m)
    G5 = np.kron(np.eye(N * N), np.diag([1.0, -1.0]))
    assert np.abs(G5 @ D @ G5 - D.conj().T).max() < 1e-13
    Dh = oracle.dhat_dense(U, m)
    Ge = np.kron(np.eye(N * N // 2), np.diag([1.0, -1.0]))
    assert np.abs(Ge @ Dh @ Ge - Dh.conj().T).max() < 1e-13


@pytest.mark.parametrize("N", [4, 8])
def test_schur_complement_matches_dense_blocks(N):
    """Dhat = (D_ee - D_eo D_oo^-1 D_oe)/c from the dense full operator (Sec. 3.2)."""
    U = inputs.gauge_random(N, 3)
    m = 0.2
    c = m + 2.0
    D = oracle.wilson_dense(U, m)
    ev, od = _eo_index(N)
    e, o = _dofs(ev), _dofs(od)
    Dee, Deo, Doe, Doo = D[np.ix_(e, e)], D[np.ix_(e, o)], D[np.ix_(o, e)], D[np.ix_(o, o)]
    assert np.abs(Dee - c * np.eye(len(e))).max() == 0.0
    assert np.abs(Doo - c * np.eye(len(o))).max() == 0.0
    S = (Dee - Deo @ np.linalg.solve(Doo, Doe)) / c
    assert np.abs(S - oracle.dhat_dense(U, m)).max() < 1e-13


@pytest.mark.parametrize("N", [4, 8])
def test_two_step_solve_equals_full_solve(N):
    """Solve Dhat x_e = bhat, reconstruct x_o: equals the dense solve of D (Sec. 3.2)."""
    U = inputs.gauge_random(N, 4)
    m = 0.1
    D = oracle.wilson_dense(U, m)
    b = inputs.gaussian(2 * N * N, 5)
    x_ref = np.linalg.solve(D, b)
    bh = oracle.eo_reduce(U, m, b)
    xe = np.linalg.solve(oracle.dhat_dense(U, m), bh)
    x = oracle.eo_reconstruct(U, m, b, xe)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-12


def test_apply_matches_dense():
    N = 8
    U = inputs.gauge_random(N, 9)
    m = -0.1
    x = inputs.gaussian(2 * N * N, 1)
    assert np.abs(oracle.wilson_apply(U, m, x) - oracle.wilson_dense(U, m) @ x).max() < 1e-13
    xe = inputs.gaussian(N * N, 2)
    assert np.abs(oracle.dhat_apply(U, m, xe) - oracle.dhat_dense(U, m) @ xe).max() < 1e-13


def _multiset_close(a, b, tol):
    a = np.sort_complex(np.round(a, 9))
    b = np.sort_complex(np.round(b, 9))
    return np.abs(a - b).max() < tol


def test_free_field_spectrum_closed_form():
    """U = 1: lambda_+-(p) = m + 2 - cos px - cos py +- i sqrt(sin^2 px + sin^2 py)."""
    N, m = 8, 0.3
    c = m + 2
    U = inputs.gauge_free(N)
    p = 2 * np.pi * np.arange(N) / N
    px, py = np.meshgrid(p, p, indexing="ij")
    re = (c - np.cos(px) - np.cos(py)).ravel()
    im = np.sqrt(np.sin(px) ** 2 + np.sin(py) ** 2).ravel()
    lam = np.concatenate([re + 1j * im, re - 1j * im])
    ev = np.linalg.eigvals(oracle.wilson_dense(U, m))
    assert _multiset_close(ev, lam, 1e-8)
    # Dhat = I - H_eo H_oe / c^2: eigenvalues 1 - mu^2/c^2 over eigenvalues mu of H,
    # each value once per +-mu pair
    mu = c - lam
    dh = np.linalg.eigvals(oracle.dhat_dense(U, m))
    assert _multiset_close(np.concatenate([dh, dh]), 1 - mu ** 2 / c ** 2, 1e-8)


def test_free_field_dhat_structure():
    """Diagonal block exactly I2, 17 nonzeros per row, ||row||^2 = 1 + 5/c^4."""
    N, m = 16, 0.4
    c = m + 2
    Dh = oracle.dhat_dense(inputs.gauge_free(N), m)
    n = Dh.shape[0]
    for e in range(0, n, 2):
        assert np.array_equal(Dh[e:e + 2, e:e + 2], np.eye(2))
    nnz = (np.abs(Dh) > 1e-14).sum(axis=1)
    assert (nnz == 17).all()
    assert np.abs((np.abs(Dh) ** 2).sum(axis=1) - (1 + 5 / c ** 4)).max() < 1e-14


def test_dhat_diagonal_block_identity_any_gauge():
    N = 8
    Dh = oracle.dhat_dense(inputs.gauge_random(N, 11), -0.2)
    for e in range(0, Dh.shape[0], 2):
        assert np.abs(Dh[e:e + 2, e:e + 2] - np.eye(2)).max() < 1e-15


def test_gauge_generator_plaquette_matches_exact_2d():
    """2D U(1): <cos theta_p> = I1(beta)/I0(beta) in infinite volume (checks the
    sign of the gauge action and the Metropolis fixture)."""
    from scipy.special import i0, i1
    for beta in (3.0, 6.0):
        U = inputs.gauge_metropolis(48, beta, 300, 5)
        pl = inputs.plaquette_cos(U)
        # average over the last configuration; statistical error ~ std/sqrt(N^2)
        err = pl.std() / np.sqrt(pl.size)
        assert abs(pl.mean() - i1(beta) / i0(beta)) < 5 * err + 2e-3
