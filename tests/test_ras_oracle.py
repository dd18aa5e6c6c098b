"""The restricted-overlap sweep of the oracle (the reading under which the paper's parallel table rows are
reproduced) pinned to things other than itself.

* One subdomain: the sweep is lexicographic SOR in the subdomain's direction, whatever the overlap.
* An overlap that covers the grid: every subdomain sweeps the whole grid from the old iterate, so its
  points equal a lexicographic sweep of the whole grid in its direction.
* No overlap: every subdomain is an independent SOR sweep of its own box with old values outside,
  checked against lexicographic SOR on the box as a problem of its own (outside values folded into f).
* The paper's PGS / PSOR counts (Sec. 8, Tables 2d:1, 2d:3, 3d:1) within 2 % with one point of overlap,
  on the model problem and stopping rule that reproduce its sequential rows exactly.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_parallel_tables.json")


def _case(dim, n, seed):
    pr = synth.random_small(seed, dim, n)
    return pr, O.assemble(dim, n, pr["alphas"])


@pytest.mark.parametrize("dim,n", [(1, (17,)), (2, (11, 9)), (3, (6, 5, 4))])
def test_one_subdomain_is_lexicographic_sor(dim, n):
    pr, diags = _case(dim, n, 3)
    p = (1,) * dim
    for k in range(1 << dim):
        dirs = O.schedule(dim, p, k)
        for ov in (0, 2, 5):
            got = O.ras_sweep(dim, n, p, dirs, diags, pr["f"], pr["u"], 1.3, ov)
            ref = O.sor_lex(dim, n, diags, 1.3, dirs[0, :dim], pr["f"], pr["u"])
            assert np.array_equal(got, ref), (k, ov)


@pytest.mark.parametrize("dim,n,p", [(2, (13, 11), (3, 2)), (3, (7, 6, 5), (2, 2, 2)), (1, (20,), (4,))])
def test_overlap_covering_the_grid_is_a_whole_grid_sweep(dim, n, p):
    pr, diags = _case(dim, n, 5)
    om = [1.1, 1.4, 0.9, 1.6, 1.2, 0.8, 1.5, 1.0][: 1 << dim]
    dirs = O.schedule(dim, p, 1)
    got = O.ras_sweep(dim, n, p, dirs, diags, pr["f"], pr["u"], om, max(n))
    owner = _owner(dim, n, p)
    for s in range(dirs.shape[0]):
        d = dirs[s, :dim]
        ref = O.sor_lex(dim, n, diags, om[O.corner(dim, d)], d, pr["f"], pr["u"])
        mask = owner == s
        assert np.array_equal(got[mask], ref[mask]), s


def _owner(dim, n, p):
    """subdomain id of every point (x fastest), from the oracle's partition"""
    coords = np.indices(tuple(reversed(n))).reshape(dim, -1)[::-1]  # coords[a] of flat point index
    sid = np.zeros(coords.shape[1], np.int64)
    mult = 1
    for a in range(dim):
        lo, hi = O.partition(n[a], p[a])
        r = np.searchsorted(hi, coords[a])
        sid += r * mult
        mult *= p[a]
    return sid


def test_no_overlap_is_independent_subdomain_sor():
    dim, n, p = 2, (12, 10), (3, 2)
    pr, diags = _case(dim, n, 7)
    om = [1.3, 1.1, 1.5, 0.9]
    dirs = O.schedule(dim, p, 2)
    got = O.ras_sweep(dim, n, p, dirs, diags, pr["f"], pr["u"], om, 0)
    lo0, hi0 = O.partition(n[0], p[0])
    lo1, hi1 = O.partition(n[1], p[1])
    U = pr["u"].reshape(n[1], n[0])
    F = pr["f"].reshape(n[1], n[0])
    D = [d.reshape(n[1], n[0]) for d in diags]
    G = got.reshape(n[1], n[0])
    for s1 in range(p[1]):
        for s0 in range(p[0]):
            s = s0 + p[0] * s1
            ys, xs = slice(lo1[s1], hi1[s1] + 1), slice(lo0[s0], hi0[s0] + 1)
            fb = F[ys, xs].copy()
            # couplings that leave the box take the old values outside: fold them into f
            if lo0[s0] > 0:
                fb[:, 0] += D[1][ys, lo0[s0]] * U[ys, lo0[s0] - 1]
            if hi0[s0] < n[0] - 1:
                fb[:, -1] += D[2][ys, hi0[s0]] * U[ys, hi0[s0] + 1]
            if lo1[s1] > 0:
                fb[0, :] += D[3][lo1[s1], xs] * U[lo1[s1] - 1, xs]
            if hi1[s1] < n[1] - 1:
                fb[-1, :] += D[4][hi1[s1], xs] * U[hi1[s1] + 1, xs]
            nb = (hi0[s0] - lo0[s0] + 1, hi1[s1] - lo1[s1] + 1)
            db = [d[ys, xs].reshape(-1).copy() for d in D]
            d = dirs[s, :2]
            ref = O.sor_lex(2, nb, db, om[O.corner(2, d)], d, fb.reshape(-1), U[ys, xs].reshape(-1))
            assert np.allclose(G[ys, xs].reshape(-1), ref, rtol=0, atol=1e-14 * np.abs(ref).max()), s


def _model_run(dim, N, p, omega, tol, overlap=1, maxit=20000):
    n, diags, f, ue = O.model_problem(dim, N)
    u = np.zeros_like(f)
    for k in range(maxit):
        u = O.ras_sweep(dim, (n,) * dim, p, O.schedule(dim, p, k, 0), diags, f, u, omega, overlap)
        if O.l1_error(dim, N, u, ue) < tol:
            return k + 1
    return maxit


@pytest.mark.parametrize("row", json.load(open(GOLD))["rows"], ids=lambda r: f"{r['table']}-{r['p']}-w{r['omega']}")
def test_paper_parallel_rows_within_two_percent(row):
    it = _model_run(row["dim"], row["N"], tuple(row["p"]), row["omega"], row["tol"])
    assert abs(it - row["iters"]) <= 0.02 * row["iters"], (it, row)
