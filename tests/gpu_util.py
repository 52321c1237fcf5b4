"""Helpers shared by the GPU parity tests (test code only)."""
import numpy as np
import scipy.sparse as sp

OFFS = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1)]


def blocks_to_csr(D, ex, ey):
    """Expand [site][7][16][16] blocks (periodic ex x ey grid) to a sparse matrix,
    summing blocks whose offsets alias on small grids."""
    rows, cols, vals = [], [], []
    ns = ex * ey
    ii, jj = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    for a in range(ns):
        ax, ay = a % ex, a // ex
        for o, (dx, dy) in enumerate(OFFS):
            b = ((ay + dy) % ey) * ex + (ax + dx) % ex
            rows.append((16 * a + ii).ravel())
            cols.append((16 * b + jj).ravel())
            vals.append(D[a, o].ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(16 * ns, 16 * ns))
    return A.tocsr()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.abs(a - b).max()
    s = np.abs(b).max()
    return d / s if s > 0 else d


def projector_diff(Pa, Pb):
    """max over aggregate blocks of || Pa Pa^H - Pb Pb^H ||_max (basis-independent)."""
    worst = 0.0
    for a in range(Pa.shape[0]):
        for s in range(2):
            A = Pa[a, s] @ Pa[a, s].conj().T
            B = Pb[a, s] @ Pb[a, s].conj().T
            worst = max(worst, np.abs(A - B).max())
    return worst
