"""Pins of the oracle's cycles and setup schedules against dense replays.

Each replay below is written here from the definitions, on dense matrices:
the fine operator Dhat (pinned by the operator tests), the oracle's
interpolation P_l expanded to a dense matrix, the Galerkin products
P^H A P formed with numpy, row projections over dense rows in the colour
order of the readings, numpy's LU solve on the coarsest level.  Nothing
here calls the oracle's cycle, sweep, fit or Galerkin code; the oracle is
then compared element by element.

* the cycle of Sec. 1 (two-grid scheme, applied recursively) with smoothing,
  as V (one coarse visit), W (two visits, the solve cycle of Sec. 4) and K
  (two steps of flexible GCR on each coarse system that is not the coarsest,
  each preconditioned by one cycle from that level), on 2, 3 and 4 levels
  with 1, 2 and 4 sweeps;
* the stand-alone iteration x <- x + M(0 - Dhat x) whose error reduction is
  the convergence rate rho of Sec. 4;
* the relax-fit setup with its adaptive pass (two cycles per test vector on
  Dhat v = 0, then the pass again);
* the bootstrap setup cycles of Sec. 3.4 / 4.1 / 4.2 (W and super-V) in the
  node order of the setup-cycle figure: arrive (relax V^r, relax V^e with
  Ritz updates, fit, coarsen, restrict), coarsest eigenpairs of Z_L,
  interpolation of V^e coming back up, a second arrival between two W
  visits, relaxation of V^e after the last visit; the adaptive step between
  the two setup cycles.
A plausible slip in any of these (a dropped post-smoothing, a sweep against
the wrong right-hand side, a missing second W visit, a GCR coefficient
conjugated the wrong way, a node out of order) changes the result far beyond
the rounding tolerance.
"""
import numpy as np
import pytest

import inputs
import oracle
from tests.test_oracle_hierarchy import _P_csr

OFFS7 = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]


# ------------------------------------------------------------- dense pieces
def _fine_order(N):
    """Row order of the fine sweep: colours 4 (u mod 4) + (v mod 4) of the even
    site (u = (x+y)/2, v = (x-y)/2), sites of a colour in (y, xh) order, spin 0
    then 1."""
    half = N // 2
    order = []
    for c in range(16):
        for y in range(N):
            for xh in range(half):
                x = 2 * xh + (y % 2)
                if 4 * (((x + y) // 2) % 4) + (((x - y) // 2) % 4) == c:
                    e = y * half + xh
                    order += [2 * e, 2 * e + 1]
    return order


def _coarse_order(ex, ey):
    """Row order of a coarse sweep: colour (ax - 3 ay) mod 8 when both extents
    are multiples of 8, else 4 (ay mod 4) + (ax mod 4) when multiples of 4,
    else every site alone in (ay, ax) order; rows of a site 0..15."""
    def colour(ax, ay):
        if ex % 8 == 0 and ey % 8 == 0:
            return (ax - 3 * ay) % 8
        if ex % 4 == 0 and ey % 4 == 0:
            return 4 * (ay % 4) + (ax % 4)
        return ay * ex + ax
    ncol = 8 if (ex % 8 == 0 and ey % 8 == 0) else (16 if (ex % 4 == 0 and ey % 4 == 0) else ex * ey)
    order = []
    for c in range(ncol):
        for ay in range(ey):
            for ax in range(ex):
                if colour(ax, ay) == c:
                    order += [16 * (ay * ex + ax) + d for d in range(16)]
    return order


def _sweep(A, order, x, b):
    """One sweep of row projections x += (b_r - d_r x)/||d_r||^2 d_r^H."""
    x = x.copy()
    for r in order:
        d = A[r]
        nu = np.vdot(d, d).real
        if nu == 0.0:
            continue
        res = (0.0 if b is None else b[r]) - d @ x
        x += (res / nu) * d.conj()
    return x


def _g5(n, fine):
    """Gamma_5 on a level: +1 on spin 0, -1 on spin 1."""
    if fine:
        return np.tile([1.0, -1.0], n // 2)
    return np.tile(np.r_[np.ones(8), -np.ones(8)], n // 16)


class Dense:
    """Dense copy of a hierarchy's levels, built from Dhat and the oracle's P."""

    def __init__(self, U, m, h):
        self.N = U.shape[-1]
        self.U, self.m = U, m
        self.L = h.n_levels
        self.info = [h.level_info(l) for l in range(self.L)]
        self.A = [oracle.dhat_dense(U, m)]
        self.P = []
        self.order = [_fine_order(self.N)]
        for l in range(self.L - 1):
            self.set_P(l, _P_csr(h, l, h.P_blocks(l)).toarray())

    def set_P(self, l, P):
        if len(self.P) <= l:
            self.P.append(None)
            self.A.append(None)
            self.order.append(None)
        self.P[l] = P
        self.A[l + 1] = P.conj().T @ self.A[l] @ P
        inf = self.info[l + 1]
        self.order[l + 1] = _coarse_order(inf["ex"], inf["ey"])

    # -------------------------------------------------------------- cycle
    def cycle(self, l, b, x, kind, pre, post):
        A = self.A[l]
        last = self.L - 1
        if l == last:
            return np.linalg.solve(A, b)
        for _ in range(pre):
            x = _sweep(A, self.order[l], x, b)
        r = b - A @ x
        P = self.P[l]
        bc = P.conj().T @ r
        if kind == "K" and l + 1 < last:
            xc = self.kvisit(l + 1, bc, pre, post)
        else:
            xc = np.zeros_like(bc)
            for _ in range(2 if kind == "W" else 1):
                xc = self.cycle(l + 1, bc, xc, kind, pre, post)
                if l + 1 == last:
                    break
        x = x + P @ xc
        for _ in range(post):
            x = _sweep(A, self.order[l], x, b)
        return x

    def kvisit(self, c, r0, pre, post):
        """Two flexible GCR steps on A_c x = r0 from x = 0, preconditioned by a
        K-cycle from level c: the step directions z are made A-orthogonal
        (w = A z orthogonal), each coefficient minimises the residual norm."""
        A = self.A[c]
        z1 = self.cycle(c, r0, np.zeros_like(r0), "K", pre, post)
        w1 = A @ z1
        rho1 = np.vdot(w1, w1).real
        a1 = np.vdot(w1, r0) / rho1
        x = a1 * z1
        r1 = r0 - a1 * w1
        z2 = self.cycle(c, r1, np.zeros_like(r0), "K", pre, post)
        w2 = A @ z2
        beta = np.vdot(w1, w2) / rho1
        w2 = w2 - beta * w1
        z2 = z2 - beta * z1
        a2 = np.vdot(w2, r1) / np.vdot(w2, w2).real
        return x + a2 * z2

    # -------------------------------------------------------------- setup
    def relax(self, l, V, sweeps):
        out = []
        for v in V:
            for _ in range(sweeps):
                v = _sweep(self.A[l], self.order[l], v, None)
            out.append(v / np.linalg.norm(v))
        return np.array(out)

    def fit_exact(self, l, V, P_template):
        """P_{a,s}: orthonormal basis of the k <= 8 test vectors on the block in
        test-vector order with positive R_jj (the exact least-squares fit)."""
        return self._fit(l, V, P_template, rank8=False)

    def fit_rank8(self, l, V, P_template):
        """k > 8: the span of the 8 dominant left singular vectors of the block
        (the best rank-8 fit with unit weights), with the basis of the
        projections of the first 8 test vectors (positive R_jj)."""
        return self._fit(l, V, P_template, rank8=True)

    def _fit(self, l, V, Pt, rank8):
        # the sparsity of P: which fine dofs belong to which (aggregate, spin) column block
        P = np.zeros_like(Pt)
        nc = Pt.shape[1]
        for cb in range(0, nc, 8):
            rows = np.nonzero(np.abs(Pt[:, cb:cb + 8]).sum(axis=1) > 0)[0]
            B = V[:, rows].T  # rows x k
            if rank8:
                Usv, _, _ = np.linalg.svd(B)
                U8 = Usv[:, :8]
                B = U8 @ (U8.conj().T @ B[:, :8])
            Q, R = np.linalg.qr(B[:, :8])
            ph = np.diag(R) / np.abs(np.diag(R))
            P[np.ix_(rows, np.arange(cb, cb + 8))] = Q * ph[None, :]
        return P


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _hier(N, L, pre, post, cycle, seed=7):
    U = inputs.gauge_metropolis(N, 3.0, 30, seed)
    m = -0.05
    h = oracle.Hierarchy(U, m, n_levels=L, pre=pre, post=post, cycle=cycle, seed=seed,
                         setup_sweeps=4, setup_adapt=0)
    assert h.n_levels == L
    return U, m, h


KINDS = {"V": 0, "W": 1, "K": 2}


# ------------------------------------------------------------- cycles
@pytest.mark.parametrize("N,L", [(16, 2), (32, 2), (32, 3)])
@pytest.mark.parametrize("nu", [1, 2, 4])
@pytest.mark.parametrize("kind", ["V", "W", "K"])
def test_cycle_equals_dense_replay(N, L, nu, kind):
    U, m, h = _hier(N, L, nu, nu, KINDS[kind])
    D = Dense(U, m, h)
    b = inputs.gaussian(N * N, 40 + nu)
    got = h.cycle(b)
    ref = D.cycle(0, b, np.zeros_like(b), kind, nu, nu)
    assert _rel(got, ref) < 1e-12


def test_cycle_kinds_differ_from_three_levels_on():
    """On 3 levels the W and K visits of level 1 change the result (so the
    pins above tell the kinds apart); on 2 levels all three are the same."""
    outs = {}
    for kind in KINDS:
        U, m, h = _hier(32, 3, 2, 2, KINDS[kind])
        outs[kind] = h.cycle(inputs.gaussian(32 * 32, 5))
    assert _rel(outs["W"], outs["V"]) > 1e-4
    assert _rel(outs["K"], outs["V"]) > 1e-4
    assert _rel(outs["K"], outs["W"]) > 1e-4
    outs2 = {}
    for kind in KINDS:
        U, m, h = _hier(32, 2, 2, 2, KINDS[kind])
        outs2[kind] = h.cycle(inputs.gaussian(32 * 32, 5))
    assert _rel(outs2["W"], outs2["V"]) < 1e-15 and _rel(outs2["K"], outs2["V"]) < 1e-15


def test_kcycle_four_levels_equals_dense_replay():
    """K visits nest: the level-1 GCR steps are preconditioned by cycles that
    themselves take GCR steps on level 2."""
    U, m, h = _hier(64, 4, 2, 2, KINDS["K"])
    D = Dense(U, m, h)
    b = inputs.gaussian(64 * 64, 8)
    assert _rel(h.cycle(b), D.cycle(0, b, np.zeros_like(b), "K", 2, 2)) < 1e-12


def test_kcycle_visit_minimises_the_coarse_residual():
    """Two GCR steps give the minimiser of ||r0 - A_c x|| over the span of the
    two (A-orthogonalised) preconditioned directions: the final residual is
    orthogonal to A z1 and A z2."""
    U, m, h = _hier(32, 3, 2, 2, KINDS["K"])
    D = Dense(U, m, h)
    r0 = inputs.gaussian(D.A[1].shape[0], 3)
    x = D.kvisit(1, r0, 2, 2)
    A = D.A[1]
    z1 = D.cycle(1, r0, np.zeros_like(r0), "K", 2, 2)
    res = r0 - A @ x
    assert abs(np.vdot(A @ z1, res)) < 1e-12 * np.linalg.norm(A @ z1) * np.linalg.norm(r0)
    assert np.linalg.norm(res) < np.linalg.norm(r0 - (np.vdot(A @ z1, r0) / np.vdot(A @ z1, A @ z1)) * (A @ z1))


@pytest.mark.parametrize("kind", ["V", "W", "K"])
def test_stationary_iteration_and_rho(kind):
    """rho of Sec. 4: ||e^nu|| / ||e^{nu-1}|| of x <- x + M(0 - Dhat x)."""
    U, m, h = _hier(32, 3, 2, 2, KINDS[kind])
    D = Dense(U, m, h)
    x0 = inputs.gaussian(32 * 32, 21)
    xo, norms = h.stationary(x0, 4)
    x = x0.copy()
    ref = [np.linalg.norm(x)]
    for _ in range(4):
        x = x + D.cycle(0, -(D.A[0] @ x), np.zeros_like(x), kind, 2, 2)
        ref.append(np.linalg.norm(x))
    assert _rel(xo, x) < 1e-11
    assert np.allclose(norms, ref, rtol=1e-11, atol=0)
    assert norms[-1] < norms[0]  # a convergent iteration


# ------------------------------------------------------------- relax-fit setup
@pytest.mark.parametrize("L,adapt", [(2, 0), (3, 0), (3, 1)])
def test_relax_fit_setup_equals_dense_replay(L, adapt):
    N, sweeps = 32, 3
    U = inputs.gauge_metropolis(N, 3.0, 30, 11)
    m = -0.05
    tv = oracle.gaussian_tv(N, 8, 13)
    h = oracle.Hierarchy(U, m, n_levels=L, pre=2, post=2, init_tv=tv, setup_sweeps=sweeps, setup_adapt=adapt)
    D = Dense(U, m, h)  # shapes and a template of P's sparsity
    templ = [D.P[l].copy() for l in range(L - 1)]

    def setup_pass(V):
        saved = None
        for l in range(L - 1):
            V = D.relax(l, V, sweeps)
            if l == 0:
                saved = V.copy()
            D.set_P(l, D.fit_exact(l, V, templ[l]))
            V = (D.P[l].conj().T @ V.T).T
        return saved

    tv0 = setup_pass(tv)
    for _ in range(adapt):
        W = []
        for v in tv0:
            for _ in range(2):
                v = D.cycle(0, np.zeros_like(v), v, "V", 2, 2)
            W.append(v / np.linalg.norm(v))
        tv0 = setup_pass(np.array(W))
    for l in range(L - 1):
        Po = _P_csr(h, l, h.P_blocks(l)).toarray()
        assert _rel(Po, D.P[l]) < 1e-10, l
    assert _rel(h.test_vectors(), tv0) < 1e-10


# ------------------------------------------------------------- bootstrap setup
class BootReplay:
    """The bootstrap setup cycles in the node order of the setup-cycle figure
    (reading of Sec. 3.4 / 4.1 / 4.2 in the Hermitian form of Theorem 1:
    Z_l = Gamma_5 A_l, Kaczmarz on (A_l - lambda Gamma_5) v = 0 with the
    Ritz value <Z v, v>/<v, v> refreshed after every sweep)."""

    def __init__(self, D, templ, ke, gamma, nu_of):
        self.D, self.templ, self.ke, self.gamma, self.nu_of = D, templ, ke, gamma, nu_of
        self.Vr = [None] * D.L
        self.Ve = [None] * D.L
        self.lam = None

    def g5(self, l):
        return _g5(self.D.A[l].shape[0], l == 0)

    def ritz(self, l, v):
        return (np.vdot(v, self.g5(l) * (self.D.A[l] @ v)) / np.vdot(v, v)).real

    def relax_r(self, l, nu):
        self.Vr[l] = self.D.relax(l, self.Vr[l], nu)

    def relax_e(self, l, nu):
        if self.lam is None:
            return
        out = []
        for j, v in enumerate(self.Ve[l]):
            for _ in range(nu):
                As = self.D.A[l] - self.lam[j] * np.diag(self.g5(l))
                v = _sweep(As, self.D.order[l], v, None)
                self.lam[j] = self.ritz(l, v)
            out.append(v / np.linalg.norm(v))
        self.Ve[l] = np.array(out)

    def fit(self, l):
        V = self.Vr[l] if self.lam is None else np.vstack([self.Vr[l], self.Ve[l]])
        P = self.D.fit_rank8(l, V, self.templ[l]) if V.shape[0] > 8 else self.D.fit_exact(l, V, self.templ[l])
        self.D.set_P(l, P)
        self.Vr[l + 1] = (P.conj().T @ self.Vr[l].T).T
        if self.lam is not None:
            self.Ve[l + 1] = (P.conj().T @ self.Ve[l].T).T

    def coarsest(self):
        Lc = self.D.L - 1
        Z = self.g5(Lc)[:, None] * self.D.A[Lc]
        w, E = np.linalg.eigh(0.5 * (Z + Z.conj().T))
        idx = np.argsort(np.abs(w), kind="stable")[: self.ke]
        self.lam = list(w[idx])
        self.Ve[Lc] = E[:, idx].T.copy()

    def interp_e(self, l):
        self.Ve[l] = (self.D.P[l] @ self.Ve[l + 1].T).T

    def arrive(self, l, nu, first):
        self.relax_r(l, nu)
        if not first:
            self.relax_e(l, nu)
        self.fit(l)

    def visit(self, l, nu, first):
        Lc = self.D.L - 1
        self.arrive(l, nu[l], first)
        for g in range(self.gamma):
            if l + 1 == Lc:
                self.coarsest()
            else:
                self.visit(l + 1, nu, first and g == 0)
            self.interp_e(l)
            if g < self.gamma - 1:
                self.arrive(l, nu[l], False)
            else:
                self.relax_e(l, nu[l])

    def setup_cycle(self, mu, first):
        nu = [self.nu_of(mu, l) for l in range(self.D.L)]
        self.arrive(0, nu[0], first)
        if self.D.L == 2:
            self.coarsest()
        else:
            self.visit(1, nu, first)
        self.interp_e(0)
        self.relax_e(0, nu[0])


@pytest.mark.parametrize("mode", [1, 2])
def test_bootstrap_setup_equals_dense_replay(mode):
    """mode 1: W setup cycles (gamma = 2, mu sweeps per node); mode 2: super-V
    (gamma = 1, mu 2^l sweeps on level l); mu = nu1, adaptive step, mu = nu2."""
    N, L, ke, nu1, nu2 = 32, 3, 8, 3, 2
    U = inputs.gauge_metropolis(N, 3.0, 30, 17)
    m = -0.05
    tv = oracle.gaussian_tv(N, 8, 19)
    h = oracle.Hierarchy(U, m, n_levels=L, pre=2, post=2, boot=mode, k_e=ke, nu1=nu1, nu2=nu2, init_tv=tv)
    D = Dense(U, m, h)
    templ = [D.P[l].copy() for l in range(L - 1)]
    nu_of = (lambda mu, l: mu) if mode == 1 else (lambda mu, l: mu * 2 ** l)
    R = BootReplay(D, templ, ke, 2 if mode == 1 else 1, nu_of)
    R.Vr[0] = tv.copy()
    R.setup_cycle(nu1, True)
    # adaptive step: two solve cycles on Dhat v = 0 for the V^e of smallest |Ritz value|
    k = int(np.argmin(np.abs(R.lam)))
    v = R.Ve[0][k]
    for _ in range(2):
        v = D.cycle(0, np.zeros_like(v), v, "V", 2, 2)
    v = v / np.linalg.norm(v)
    R.Ve[0][k] = v
    R.lam[k] = R.ritz(0, v)
    R.setup_cycle(nu2, False)

    lam_o, ve_o = h.boot_vectors()
    assert np.allclose(lam_o, R.lam, rtol=1e-9, atol=1e-12)
    # eigenvector approximations up to their arbitrary phases (set on the coarsest level)
    for j in range(ke):
        assert abs(abs(np.vdot(ve_o[j], R.Ve[0][j])) - 1.0) < 1e-9
    for l in range(L - 1):
        Po = _P_csr(h, l, h.P_blocks(l)).toarray()
        assert _rel(Po, D.P[l]) < 1e-9, l
    assert _rel(h.test_vectors(), R.Vr[0]) < 1e-9
