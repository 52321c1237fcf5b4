"""ctypes binding of the CPU FP64 oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: the oracle is loaded by the test-suite, by the smoke
check and by the CPU-baseline leg of the benchmark.  The GPU library never
imports or links it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (FP64, no fast-math, OpenMP for the LU)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, I, D, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
        sig = {
            "oracle_philox4x32_10": (None, [P, P, P]),
            "oracle_gaussian_tv": (None, [I, I, U64, P]),
            "oracle_wilson_apply": (None, [I, P, D, P, P]),
            "oracle_wilson_dense": (None, [I, P, D, P]),
            "oracle_wilson_csr_nnz": (I, [I, P]),
            "oracle_wilson_csr": (None, [I, P, D, P, P, P]),
            "oracle_dhat_dense": (None, [I, P, D, P]),
            "oracle_dhat_apply": (None, [I, P, D, P, P, I]),
            "oracle_eo_reduce": (None, [I, P, D, P, P, I]),
            "oracle_eo_reconstruct": (None, [I, P, D, P, P, P, I]),
            "oracle_kaczmarz_fine": (None, [I, P, D, P, P, I, I]),
            "oracle_fine_colour": (I, [I, I]),
            "oracle_coarse_colour": (I, [I, I, I, I]),
            "oracle_coarse_ncolours": (I, [I, I]),
            "oracle_setup": (P, [I, P, D, I, I, I, I, I, I, I, I, U64, P]),
            "oracle_free": (None, [P]),
            "oracle_n_levels": (I, [P]),
            "oracle_level_info": (None, [P, I, P]),
            "oracle_export_op": (None, [P, I, P, P, P]),
            "oracle_export_P": (None, [P, I, P]),
            "oracle_export_tv": (None, [P, P]),
            "oracle_import_P": (None, [P, I, P, I]),
            "oracle_set_coarsest_lu": (None, [P, P, P]),
            "oracle_stationary": (None, [P, P, I, P]),
            "oracle_level_op": (I, [P, I, I, P, P, I]),
            "oracle_solve_reduced": (I, [P, P, P, D, I, I, P]),
            "oracle_solve": (I, [P, P, P, D, I, I, P]),
            "oracle_setup_boot": (P, [I, P, D, I, I, I, I, I, U64, P, I, I, I, I, I]),
            "oracle_jacobi_eig": (None, [I, P, P, P]),
            "oracle_ritz": (None, [P, I, P, P, I]),
            "oracle_sweep_shifted": (None, [P, I, P, P, I]),
            "oracle_coarsest_eigs": (None, [P, I, P, P]),
            "oracle_fit_ls": (None, [P, I, P, I]),
            "oracle_export_boot": (I, [P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _c(a: np.ndarray, dtype=np.complex128) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def gaussian_tv(N, k, seed):
    out = np.zeros((k, N * N), dtype=np.complex128)
    lib().oracle_gaussian_tv(N, k, seed, _p(out))
    return out


def wilson_apply(U, m, psi):
    U = _c(U); N = U.shape[-1]
    x = _c(psi).reshape(-1)
    y = np.zeros_like(x)
    lib().oracle_wilson_apply(N, _p(U), m, _p(x), _p(y))
    return y


def wilson_dense(U, m):
    U = _c(U); N = U.shape[-1]
    n = 2 * N * N
    out = np.zeros((n, n), dtype=np.complex128)
    lib().oracle_wilson_dense(N, _p(U), m, _p(out))
    return out


def wilson_csr(U, m):
    """(indptr, indices, data) of the full Wilson matrix D."""
    U = _c(U); N = U.shape[-1]
    n = 2 * N * N
    nnz = lib().oracle_wilson_csr_nnz(N, _p(U))
    ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.complex128)
    lib().oracle_wilson_csr(N, _p(U), m, _p(ptr), _p(col), _p(val))
    return ptr, col, val


def dhat_dense(U, m):
    U = _c(U); N = U.shape[-1]
    n = N * N
    out = np.zeros((n, n), dtype=np.complex128)
    lib().oracle_dhat_dense(N, _p(U), m, _p(out))
    return out


def dhat_apply(U, m, x):
    U = _c(U); N = U.shape[-1]
    x = _c(x); nrhs = x.size // (N * N)
    y = np.zeros_like(x)
    lib().oracle_dhat_apply(N, _p(U), m, _p(x), _p(y), nrhs)
    return y


def eo_reduce(U, m, b):
    U = _c(U); N = U.shape[-1]
    b = _c(b); nrhs = b.size // (2 * N * N)
    out = np.zeros(nrhs * N * N, dtype=np.complex128)
    lib().oracle_eo_reduce(N, _p(U), m, _p(b), _p(out), nrhs)
    return out.reshape((nrhs, N * N)) if nrhs > 1 else out


def eo_reconstruct(U, m, b, xe):
    U = _c(U); N = U.shape[-1]
    b = _c(b); xe = _c(xe); nrhs = b.size // (2 * N * N)
    out = np.zeros(nrhs * 2 * N * N, dtype=np.complex128)
    lib().oracle_eo_reconstruct(N, _p(U), m, _p(b), _p(xe), _p(out), nrhs)
    return out.reshape((nrhs, 2 * N * N)) if nrhs > 1 else out


def kaczmarz_fine(U, m, x, b=None, sweeps=1):
    U = _c(U); N = U.shape[-1]
    x = _c(x).copy(); nrhs = x.size // (N * N)
    bb = None if b is None else _c(b)
    lib().oracle_kaczmarz_fine(N, _p(U), m, _p(x), None if bb is None else _p(bb), sweeps, nrhs)
    return x


def fine_colour(x, y):
    return lib().oracle_fine_colour(x, y)


def coarse_colour(ax, ay, ex, ey):
    return lib().oracle_coarse_colour(ax, ay, ex, ey)


def coarse_ncolours(ex, ey):
    return lib().oracle_coarse_ncolours(ex, ey)


# ---------------------------------------------------------------- hierarchy
def jacobi_eig(H):
    """Eigenvalues (unsorted) and eigenvectors (columns) of a Hermitian matrix by cyclic Jacobi."""
    H = _c(H)
    n = H.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n), dtype=np.complex128)
    lib().oracle_jacobi_eig(n, _p(H), _p(w), _p(V))
    return w, V


class Hierarchy:
    """Oracle bootstrap-AMG hierarchy (setup, cycle, FGMRES).

    boot = 0: relax-fit setup passes (setup_sweeps, setup_adapt); boot = 1: the
    bootstrap W setup cycle schedule with the multigrid eigensolver (k_e
    eigenvector approximations, W(nu1,nu1), adaptive step, W(nu2,nu2));
    boot = 2: the super-V schedule (mu 2^l sweeps on level l, mu = nu1 then nu2)."""

    def __init__(self, U, m, *, n_levels=0, max_coarse=8192, n_tv=8, setup_sweeps=20,
                 setup_adapt=1, pre=4, post=4, cycle=0, seed=0, init_tv=None,
                 boot=0, k_e=8, nu1=10, nu2=5, adapt_cycles=2):
        U = _c(U)
        self.N = U.shape[-1]
        self.U, self.m = U, float(m)
        self._tv = None if init_tv is None else _c(init_tv)
        tvp = None if self._tv is None else _p(self._tv)
        if boot:
            h = lib().oracle_setup_boot(self.N, _p(U), self.m, n_levels, max_coarse, pre, post, cycle, seed,
                                        tvp, boot, k_e, nu1, nu2, adapt_cycles)
        else:
            h = lib().oracle_setup(self.N, _p(U), self.m, n_levels, max_coarse, n_tv, setup_sweeps,
                                   setup_adapt, pre, post, cycle, seed, tvp)
        if not h:
            raise ValueError("oracle_setup rejected the parameters")
        self.h = h
        self.n_tv = n_tv

    @classmethod
    def from_interpolation(cls, U, m, Ps, *, pre=4, post=4, cycle=0, lapack_lu=True):
        """The oracle's hierarchy on len(Ps) + 1 levels from given interpolation
        operators P_0 .. P_{L-2} (aggregate blocks [agg][s][row][8]): every
        coarse operator is the oracle's Galerkin product, the smoothers its
        colour orders.  The coarsest operator is factored by LAPACK's LU with
        partial pivoting (scipy) when lapack_lu, else by the oracle's own LU;
        its 1-norm condition number (LAPACK's estimate from the factors) is
        kept as .kappa1."""
        h = cls(U, m, n_levels=len(Ps) + 1, setup_adapt=-1, pre=pre, post=post, cycle=cycle)
        if h.n_levels != len(Ps) + 1:
            raise ValueError("lattice does not give len(Ps) + 1 levels")
        for l, P in enumerate(Ps):
            h.import_P(l, P, factor=not (lapack_lu and l == len(Ps) - 1))
        A = h.operator(h.n_levels - 1).toarray()
        import scipy.linalg as sl
        lu, piv = sl.lu_factor(A, check_finite=False)
        if lapack_lu:
            h.set_coarsest_lu(lu, piv.astype(np.int32))
        anorm = np.abs(A).sum(axis=0).max()
        rcond, _ = sl.lapack.zgecon(lu, anorm, norm="1")
        h.kappa1 = 1.0 / rcond if rcond > 0 else np.inf
        return h

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().oracle_free(h)
            self.h = None

    @property
    def n_levels(self):
        return lib().oracle_n_levels(self.h)

    def level_info(self, l):
        info = np.zeros(6, dtype=np.int32)
        lib().oracle_level_info(self.h, l, _p(info))
        return dict(ex=int(info[0]), ey=int(info[1]), dps=int(info[2]), n=int(info[3]),
                    nnz=int(info[4]), singular=bool(info[5]))

    def operator(self, l):
        """Level operator as a scipy CSR matrix."""
        import scipy.sparse as sp
        inf = self.level_info(l)
        ptr = np.zeros(inf["n"] + 1, dtype=np.int32)
        col = np.zeros(inf["nnz"], dtype=np.int32)
        val = np.zeros(inf["nnz"], dtype=np.complex128)
        lib().oracle_export_op(self.h, l, _p(ptr), _p(col), _p(val))
        return sp.csr_matrix((val, col, ptr), shape=(inf["n"], inf["n"]))

    def P_blocks(self, l):
        inf, cinf = self.level_info(l), self.level_info(l + 1)
        rows = 16 if l == 0 else 32
        out = np.zeros((cinf["ex"] * cinf["ey"], 2, rows, 8), dtype=np.complex128)
        lib().oracle_export_P(self.h, l, _p(out))
        return out

    def import_P(self, l, P, factor=True):
        """Replace P_l and rebuild level l+1 by the Galerkin product.  With
        factor=False a new coarsest level is not factored: the caller then
        supplies its LU factors through set_coarsest_lu."""
        P = _c(P)
        lib().oracle_import_P(self.h, l, _p(P), 1 if factor else 0)

    def set_coarsest_lu(self, lu, piv):
        """Factors P A = L U of the coarsest operator (LAPACK getrf convention:
        unit L below the diagonal, U on and above it, piv[k] the row swapped
        with row k at step k, 0-based); the coarsest solve substitutes with them."""
        n = self.level_info(self.n_levels - 1)["n"]
        lu = np.ascontiguousarray(lu, dtype=np.complex128)
        piv = np.ascontiguousarray(piv, dtype=np.int32)
        assert lu.shape == (n, n) and piv.shape == (n,)
        lib().oracle_set_coarsest_lu(self.h, _p(lu), _p(piv))

    def stationary(self, x0, iters):
        """Stand-alone iteration x <- x + M(0 - Dhat x) (Sec. 4) from x0:
        (final x, norms of x after 0..iters iterations)."""
        x = _c(x0).copy()
        norms = np.zeros(iters + 1)
        lib().oracle_stationary(self.h, _p(x), iters, _p(norms))
        return x, norms

    def test_vectors(self):
        out = np.zeros((self.n_tv, self.N * self.N), dtype=np.complex128)
        lib().oracle_export_tv(self.h, _p(out))
        return out

    def level_op(self, l, op, x, out=None, nrhs=1):
        x = _c(x)
        n = self.level_info(l)["n"]
        if op == 2:
            nout = self.level_info(l + 1)["n"]
        elif op == 3:
            nout = n
        else:
            nout = n
        if out is None:
            out = np.zeros(nrhs * nout, dtype=np.complex128)
        else:
            out = _c(out).copy()
        st = lib().oracle_level_op(self.h, l, op, _p(x), _p(out), nrhs)
        if st != 0:
            raise RuntimeError(f"oracle_level_op status {st}")
        return out

    def apply(self, l, x, nrhs=1):
        return self.level_op(l, 0, x, nrhs=nrhs)

    def sweep(self, l, x, b, nrhs=1):
        return self.level_op(l, 1, b, out=x, nrhs=nrhs)

    def restrict(self, l, x, nrhs=1):
        return self.level_op(l, 2, x, nrhs=nrhs)

    def prolong_add(self, l, xc, y, nrhs=1):
        return self.level_op(l, 3, xc, out=y, nrhs=nrhs)

    def coarsest_solve(self, x, nrhs=1):
        return self.level_op(self.n_levels - 1, 4, x, nrhs=nrhs)

    def cycle(self, b, l=0, nrhs=1):
        return self.level_op(l, 5, b, nrhs=nrhs)

    # ---- bootstrap eigensolver pieces (Sec. 3.4, Theorem 1)
    def ritz(self, l, X, nrhs=1):
        X = _c(X)
        lam = np.zeros(nrhs)
        lib().oracle_ritz(self.h, l, _p(X), _p(lam), nrhs)
        return lam

    def sweep_shifted(self, l, X, lam, nrhs=1):
        X = _c(X).copy()
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        lib().oracle_sweep_shifted(self.h, l, _p(X), _p(lam), nrhs)
        return X

    def coarsest_eigs(self, ke):
        n = self.level_info(self.n_levels - 1)["n"]
        vals = np.zeros(ke)
        vecs = np.zeros((ke, n), dtype=np.complex128)
        lib().oracle_coarsest_eigs(self.h, ke, _p(vals), _p(vecs))
        return vals, vecs

    def fit_ls(self, l, V):
        V = _c(V)
        lib().oracle_fit_ls(self.h, l, _p(V), V.shape[0])

    def boot_vectors(self):
        """(Ritz values, level-1 eigenvector approximations) after a bootstrap setup."""
        ke = lib().oracle_export_boot(self.h, None, None)
        lam = np.zeros(ke)
        ve = np.zeros((ke, self.N * self.N), dtype=np.complex128)
        lib().oracle_export_boot(self.h, _p(lam), _p(ve))
        return lam, ve

    def solve_reduced(self, bh, tol=1e-10, restart=32, max_iter=1000):
        bh = _c(bh)
        x = np.zeros_like(bh)
        info = np.zeros(5)
        st = lib().oracle_solve_reduced(self.h, _p(bh), _p(x), tol, restart, max_iter, _p(info))
        return st, x, dict(iters=int(info[0]), restarts=int(info[1]), relres=float(info[2]),
                           rho=float(info[4]))

    def solve(self, b, tol=1e-10, restart=32, max_iter=1000):
        b = _c(b)
        x = np.zeros_like(b)
        info = np.zeros(5)
        st = lib().oracle_solve(self.h, _p(b), _p(x), tol, restart, max_iter, _p(info))
        return st, x, dict(iters=int(info[0]), restarts=int(info[1]), relres=float(info[2]),
                           relres_full=float(info[3]), rho=float(info[4]))
