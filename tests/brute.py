"""Brute-force checkers for the oracle (tests only; NumPy/SciPy, tiny grids).

Written independently of oracle/: partitions come from numpy.array_split,
matrices are assembled globally with vectorised NumPy and solved with SciPy's
sparse direct solver.  Point index P = x + n0*(y + n1*z).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# diagonal order P, W, E, S, N, B, F: axis a, side -1 -> 1+2a, side +1 -> 2+2a
def kidx(a, s):
    return 1 + 2 * a + (1 if s > 0 else 0)


def coords(dim, n):
    N = int(np.prod(n))
    P = np.arange(N)
    c = []
    stride = 1
    for a in range(dim):
        c.append((P // stride) % n[a])
        stride *= n[a]
    return c


def owners(n_a, p_a):
    parts = np.array_split(np.arange(n_a), p_a)
    own = np.empty(n_a, np.int64)
    for r, part in enumerate(parts):
        own[part] = r
    return own


def cell_dirs(dim, n, p, dirs):
    """Direction sign per point and axis, shape (dim, N)."""
    c = coords(dim, n)
    sid = np.zeros(c[0].size, np.int64)
    mult = 1
    for a in range(dim):
        sid += owners(n[a], p[a])[c[a]] * mult
        mult *= p[a]
    return np.stack([np.asarray(dirs)[sid, a].astype(np.int64) for a in range(dim)])


def neighbour(dim, n, a, s):
    """(mask, index) of the neighbour of every point on axis a, side s."""
    c = coords(dim, n)
    q = c[a] + s
    mask = (q >= 0) & (q < n[a])
    stride = int(np.prod(n[:a])) if a > 0 else 1
    idx = np.arange(c[0].size) + s * stride
    return mask, idx


def dense_A(dim, n, diags):
    N = int(np.prod(n))
    A = np.diag(np.asarray(diags[0], float))
    for a in range(dim):
        for s in (-1, 1):
            m, q = neighbour(dim, n, a, s)
            A[np.arange(N)[m], q[m]] -= np.asarray(diags[kidx(a, s)])[m]
    return A


def upstream_matrix(dim, n, p, dirs, diags):
    """Sparse N with N[P, Q] = a_{P->Q} when Q is upstream of P (the side P's sweep starts from)."""
    N = int(np.prod(n))
    cd = cell_dirs(dim, n, p, dirs)
    rows, cols, vals = [], [], []
    for a in range(dim):
        for s in (-1, 1):
            m, q = neighbour(dim, n, a, s)
            up = m & (s == -cd[a])
            P = np.arange(N)[up]
            rows.append(P); cols.append(q[up]); vals.append(np.asarray(diags[kidx(a, s)])[up])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def k1_sweep(dim, n, p, dirs, diags, f, uold=None, piv=None, omega_corner=None):
    """One decomposed sweep as the solution of one global sparse system.

    x_P - (w/D) sum_{Q up} a x_Q = (1-w) uold_P + (w/D)(f_P + sum_{Q down} a uold_Q)
    """
    N = int(np.prod(n))
    cd = cell_dirs(dim, n, p, dirs)
    D = np.asarray(diags[0], float) if piv is None else np.asarray(piv, float)
    if omega_corner is None:
        w = np.ones(N)
    else:
        corner = np.zeros(N, np.int64)
        for a in range(dim):
            corner += (cd[a] < 0).astype(np.int64) << a
        w = np.asarray(omega_corner, float)[corner]
    uo = np.zeros(N) if uold is None else np.asarray(uold, float)
    acc = np.asarray(f, float).copy()
    rows, cols, vals = [np.arange(N)], [np.arange(N)], [np.ones(N)]
    for a in range(dim):
        for s in (-1, 1):
            m, q = neighbour(dim, n, a, s)
            coef = np.asarray(diags[kidx(a, s)], float)
            up = m & (s == -cd[a])
            down = m & ~(s == -cd[a])
            P = np.arange(N)[up]
            rows.append(P); cols.append(q[up]); vals.append(-(w / D)[up] * coef[up])
            acc[down] += coef[down] * uo[q[down]]
    M = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    b = (1 - w) * uo + (w / D) * acc
    return spla.spsolve(M, b)
