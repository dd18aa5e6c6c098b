"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test would fail under a plausible mistake in the oracle: a dropped
coupling term, a wrong upstream side or sign, a transposed coefficient, a
wrong pivot recurrence or schedule.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import brute
import synth
from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def _rows():
    rows = json.load(open(GOLD))["rows"]
    return [pytest.param(r, id=f"{r['table']}-{r['method']}-{r['N']}") for r in rows]


# ---------------------------------------------------------------- paper tables (Sec. 8)
@pytest.mark.parametrize("row", _rows())
def test_paper_sequential_rows(row):
    if row["dim"] == 2 and row["N"] > 101:
        pytest.skip("covered by the 51^2 and 101^2 rows; kept in the fixture for reference")
    it, l1 = O.model_run(row["dim"], row["N"], row["dirs"], row["omegas"], row["tol"])
    assert it == row["iters"]
    if row["kind"] == "exact":
        assert abs(l1 - row["l1"]) <= row["rtol_l1"] * row["l1"]


# ---------------------------------------------------------------- textbook SOR facts
def _poisson(dim, n):
    N = n ** dim
    return [np.full(N, 2.0 * dim)] + [np.ones(N) for _ in range(2 * dim)]


def _rate(dim, n, omega, d, sweeps=600, tail=100):
    """Asymptotic error reduction per sweep of lexicographic SOR with f = 0."""
    diags = _poisson(dim, n)
    g = synth.rng(7)
    u = g.uniform(0.5, 1.0, n ** dim)
    f = np.zeros_like(u)
    for _ in range(sweeps - tail):
        u = O.sor_lex(dim, [n] * dim, diags, omega, d, f, u)
        u /= np.linalg.norm(u)
    n0 = np.linalg.norm(u)
    for _ in range(tail):
        u = O.sor_lex(dim, [n] * dim, diags, omega, d, f, u)
    return (np.linalg.norm(u) / n0) ** (1.0 / tail)


@pytest.mark.parametrize("dim,n", [(2, 15), (3, 9)])
def test_gauss_seidel_spectral_radius(dim, n):
    h = 1.0 / (n + 1)
    rho = np.cos(np.pi * h) ** 2
    for d in ([1] * dim, [-1] * dim):
        assert abs(_rate(dim, n, 1.0, d) - rho) < 2e-4


def test_sor_young_formula_and_optimum():
    """Young: for w < w_opt, rho = ((w mu + sqrt(w^2 mu^2 - 4(w-1)))/2)^2, mu = cos(pi h);
    for w >= w_opt every eigenvalue has modulus w - 1; w_opt = 2/(1 + sin(pi h))."""
    n = 15
    h = 1.0 / (n + 1)
    mu = np.cos(np.pi * h)
    w = 1.5
    rho = ((w * mu + np.sqrt(w * w * mu * mu - 4 * (w - 1))) / 2) ** 2
    assert abs(_rate(2, n, w, [1, 1], sweeps=1200, tail=200) - rho) < 5e-4
    wopt = 2.0 / (1.0 + np.sin(np.pi * h))
    w2 = wopt + 0.08
    assert abs(_rate(2, n, w2, [1, -1], sweeps=1500, tail=600) - (w2 - 1)) < 5e-3
    r_lo = _rate(2, n, wopt - 0.1, [1, 1], sweeps=1500, tail=300)
    r_hi = _rate(2, n, wopt + 0.1, [1, 1], sweeps=1500, tail=300)
    r_opt = _rate(2, n, wopt, [1, 1], sweeps=3000, tail=600)
    assert r_opt < r_lo and r_opt < r_hi


def test_sor_fixed_point_is_dense_solution():
    pr = synth.random_small(11, 2, (7, 5))
    diags = O.assemble(2, pr["n"], pr["alphas"])
    A = brute.dense_A(2, pr["n"], diags)
    x = np.linalg.solve(A, pr["f"])
    u = np.zeros_like(x)
    for k in range(400):
        u = O.sor_lex(2, pr["n"], diags, 1.3, [1, -1] if k % 2 else [-1, 1], pr["f"], u)
    assert np.allclose(u, x, rtol=1e-12, atol=1e-12)


def test_assemble_harmonic_means():
    """eq. d2d: a^E_P is the harmonic mean of the two node coefficients; a^P the sum of the four."""
    n = (3, 2)
    ax = np.arange(1.0, 21.0)
    ay = np.arange(2.0, 22.0) ** 1.5
    d = O.assemble(2, n, [ax, ay], beta=0.25)
    # interior point (1,0) -> node (2,1); node index i + 5*j
    node = 2 + 5 * 1
    hm = lambda a, b: 2 * a * b / (a + b)
    P = 1
    assert d[2][P] == pytest.approx(hm(ax[node], ax[node + 1]), rel=1e-15)
    assert d[1][P] == pytest.approx(hm(ax[node], ax[node - 1]), rel=1e-15)
    assert d[4][P] == pytest.approx(hm(ay[node], ay[node + 5]), rel=1e-15)
    assert d[3][P] == pytest.approx(hm(ay[node], ay[node - 5]), rel=1e-15)
    assert d[0][P] == pytest.approx(d[1][P] + d[2][P] + d[3][P] + d[4][P] + 0.25, rel=1e-15)


# ---------------------------------------------------------------- schedule (Sec. 3 Sweeping directions, Sec. 4)
def test_schedule_paper_2x2_example():
    """Fig. split2d text: sub-domains 1..4 (SW, SE, NW, NE boxes) start at NE, NW, SE, SW; then reversed."""
    d0 = O.schedule(2, (2, 2), 0)[:, :2].tolist()
    assert d0 == [[-1, -1], [1, -1], [-1, 1], [1, 1]]
    d1 = O.schedule(2, (2, 2), 1)[:, :2].tolist()
    assert d1 == [[1, 1], [-1, 1], [1, -1], [-1, -1]]


@pytest.mark.parametrize("dim,p", [(1, (5,)), (2, (4, 3)), (3, (3, 2, 2))])
def test_schedule_rules(dim, p):
    per = 1 << dim
    for k in range(2 * per):
        d = O.schedule(dim, p, k)[:, :dim].reshape(tuple(reversed(p)) + (dim,))
        for a in range(dim):
            ax = dim - 1 - a
            # neighbours along each axis sweep in opposite directions along that axis
            assert np.all(np.diff(d[..., a], axis=ax) != 0)
        nxt = O.schedule(dim, p, k + 1)[:, :dim]
        if k % 2 == 0:
            assert np.array_equal(O.schedule(dim, p, k)[:, :dim], -nxt)
    # each pair uses a new diagonal in 2D and 3D: the 2^d/2 pairs cover distinct diagonals
    if dim > 1:
        diagonals = {tuple(sorted([tuple(O.schedule(dim, p, 2 * i)[0, :dim]), tuple(-O.schedule(dim, p, 2 * i)[0, :dim])]))
                     for i in range(per // 2)}
        assert len(diagonals) == per // 2


def test_partition_almost_equal():
    lo, hi = O.partition(10, 4)
    assert lo.tolist() == [0, 3, 6, 8] and hi.tolist() == [2, 5, 7, 9]


# ---------------------------------------------------------------- one decomposed sweep vs brute force
CASES = [
    (1, (17,), (4,)), (1, (9,), (9,)),
    (2, (13, 11), (3, 2)), (2, (12, 12), (4, 4)), (2, (9, 7), (2, 3)), (2, (6, 6), (6, 3)),
    (3, (7, 6, 5), (2, 2, 2)), (3, (6, 5, 7), (3, 1, 2)), (3, (4, 4, 4), (4, 2, 1)),
]


@pytest.mark.parametrize("dim,n,p", CASES)
def test_dsweep_equals_global_solve(dim, n, p):
    pr = synth.random_small(100 + sum(n), dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    g = synth.rng(5)
    om = g.uniform(0.6, 1.9, 1 << dim)
    for phase in (0, 1):
        for k in range(1 << dim):
            dirs = O.schedule(dim, p, k, phase)
            x = O.dsweep(dim, n, p, dirs, diags, pr["f"], uold=pr["u"], omega=om)
            ref = brute.k1_sweep(dim, n, p, dirs, diags, pr["f"], uold=pr["u"], omega_corner=om)
            assert np.max(np.abs(x - ref)) <= 1e-12 * np.max(np.abs(ref))
    # pivot form, no old iterate: (Piv - N) x = f
    piv = diags[0] * g.uniform(0.8, 1.5, diags[0].size)
    dirs = O.schedule(dim, p, 0)
    x = O.dsweep(dim, n, p, dirs, diags, pr["f"], piv=piv)
    Nm = brute.upstream_matrix(dim, n, p, dirs, diags)
    res = piv * x - Nm @ x - pr["f"]
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(pr["f"]))


@pytest.mark.parametrize("dim,n", [(1, (15,)), (2, (9, 8)), (3, (5, 4, 6))])
def test_single_subdomain_is_lexicographic_sor(dim, n):
    pr = synth.random_small(3, dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    for k in range(1 << dim):
        dirs = O.schedule(dim, [1] * dim, k)
        x = O.dsweep(dim, n, [1] * dim, dirs, diags, pr["f"], uold=pr["u"], omega=1.37)
        y = O.sor_lex(dim, n, diags, 1.37, dirs[0, :dim], pr["f"], pr["u"])
        assert np.array_equal(x, y)


def test_closed_form_2x2_eq_1d_sorc():
    """Two 1D sub-domains at the iteration where both start at the interface (eq. 1d:sorc)."""
    n = 10
    pr = synth.random_small(21, 1, (n,))
    d = O.assemble(1, (n,), pr["alphas"])
    b, a, c = d[0], d[2], d[1]  # b_i, a_i (east), c_i (west)
    wL, wR = 1.3, 1.7
    dirs = O.schedule(1, (2,), 1)  # sub 0 sweeps right-to-left, sub 1 left-to-right
    assert dirs[:, 0].tolist() == [-1, 1]
    x = O.dsweep(1, (n,), (2,), dirs, d, pr["f"], uold=pr["u"], omega=[wL, wR])
    m = 4  # last point of sub 0 (0-based); m+1 first point of sub 1
    u, f = pr["u"], pr["f"]
    M = np.array([[1.0, -a[m] * wR / b[m]], [-c[m + 1] * wL / b[m + 1], 1.0]])
    r = np.array([(1 - wR) * u[m] + wR / b[m] * (c[m] * u[m - 1] + f[m]),
                  (1 - wL) * u[m + 1] + wL / b[m + 1] * (a[m + 1] * u[m + 2] + f[m + 1])])
    sol = np.linalg.solve(M, r)
    assert np.allclose(x[m:m + 2], sol, rtol=1e-13, atol=0)


def test_closed_form_4x4_and_2x2_eq_2d():
    """Cross point of a 2x2 decomposition (eq. 2d:sor4b4 with row 2 divided by a^P_{i+1,j}) and the
    next interface pair (eq. 2d:sor2b2 with the f terms written in)."""
    n = (8, 8)
    pr = synth.random_small(31, 2, n)
    D = O.assemble(2, n, pr["alphas"])
    aP, aW, aE, aS, aN = D
    u, f = pr["u"], pr["f"]
    wSW, wSE, wNW, wNE = 1.1, 1.2, 1.3, 1.4  # corner bits: x high = 1, y high = 2
    om = [wSW, wSE, wNW, wNE]
    dirs = O.schedule(2, (2, 2), 0)
    x = O.dsweep(2, n, (2, 2), dirs, D, f, uold=u, omega=om)
    I = lambda i, j: i + 8 * j
    i, j = 3, 3  # node 1 of sub-domain 1 (its NE corner)
    p1, p2, p3, p4 = I(i, j), I(i + 1, j), I(i, j + 1), I(i + 1, j + 1)
    M = np.array([
        [1, -wNE * aE[p1] / aP[p1], -wNE * aN[p1] / aP[p1], 0],
        [-wNW * aW[p2] / aP[p2], 1, 0, -wNW * aN[p2] / aP[p2]],
        [-wSE * aS[p3] / aP[p3], 0, 1, -wSE * aE[p3] / aP[p3]],
        [0, -wSW * aS[p4] / aP[p4], -wSW * aW[p4] / aP[p4], 1]])
    r = np.array([
        (1 - wNE) * u[p1] + wNE * (aS[p1] * u[I(i, j - 1)] + aW[p1] * u[I(i - 1, j)] + f[p1]) / aP[p1],
        (1 - wNW) * u[p2] + wNW * (aS[p2] * u[I(i + 1, j - 1)] + aE[p2] * u[I(i + 2, j)] + f[p2]) / aP[p2],
        (1 - wSE) * u[p3] + wSE * (aW[p3] * u[I(i - 1, j + 1)] + aN[p3] * u[I(i, j + 2)] + f[p3]) / aP[p3],
        (1 - wSW) * u[p4] + wSW * (aE[p4] * u[I(i + 2, j + 1)] + aN[p4] * u[I(i + 1, j + 2)] + f[p4]) / aP[p4]])
    sol = np.linalg.solve(M, r)
    assert np.allclose(x[[p1, p2, p3, p4]], sol, rtol=1e-13, atol=0)
    # next pair: (i-1, j) in sub-domain 1 (sweeping NE) and (i-1, j+1) in sub-domain 3 (sweeping SE)
    q1, q2 = I(i - 1, j), I(i - 1, j + 1)
    M2 = np.array([[1, -wNE * aN[q1] / aP[q1]], [-wSE * aS[q2] / aP[q2], 1]])
    r2 = np.array([
        (1 - wNE) * u[q1] + wNE * (aS[q1] * u[I(i - 1, j - 1)] + aW[q1] * u[I(i - 2, j)] + aE[q1] * x[p1] + f[q1]) / aP[q1],
        (1 - wSE) * u[q2] + wSE * (aW[q2] * u[I(i - 2, j + 1)] + aE[q2] * x[p3] + aN[q2] * u[I(i - 1, j + 2)] + f[q2]) / aP[q2]])
    sol2 = np.linalg.solve(M2, r2)
    assert np.allclose(x[[q1, q2]], sol2, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- preconditioners (Sec. 5)
PCASES = [(1, (16,), (4,)), (2, (12, 10), (3, 2)), (2, (16, 16), (4, 4)), (3, (6, 7, 5), (2, 2, 2))]


@pytest.mark.parametrize("dim,n,p", PCASES)
def test_ilu_pattern_property(dim, n, p):
    """(D~ - N1) D~^-1 (D~ - N2) equals A on A's sparsity pattern."""
    pr = synth.random_small(41, dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    pc = O.Precond("ilu0", dim, n, p, diags)
    N1 = brute.upstream_matrix(dim, n, p, pc.dirs_f, diags).toarray()
    N2 = brute.upstream_matrix(dim, n, p, pc.dirs_b, diags).toarray()
    Dt = np.diag(pc.piv)
    M = (Dt - N1) @ np.diag(1 / pc.piv) @ (Dt - N2)
    A = brute.dense_A(dim, n, diags)
    mask = A != 0
    assert np.max(np.abs((M - A)[mask])) <= 1e-13 * np.max(np.abs(A))
    # and the operator applied by the oracle is M^-1
    r = pr["f"]
    assert np.allclose(M @ pc.apply(r), r, rtol=0, atol=1e-12 * np.abs(r).max())


def test_tridiagonal_ilu_is_lu():
    n = (25,)
    pr = synth.random_small(51, 1, n)
    diags = O.assemble(1, n, pr["alphas"])
    pc = O.Precond("ilu0", 1, n, (1,), diags)
    A = brute.dense_A(1, n, diags)
    z = pc.apply(pr["f"])
    assert np.allclose(z, np.linalg.solve(A, pr["f"]), rtol=1e-12, atol=1e-14)
    _, it, rel = O.cg(lambda v: O.spmv(1, n, diags, v), pc.apply, pr["f"], rtol=1e-10)
    assert it == 1 and rel < 1e-10


@pytest.mark.parametrize("dim,n,p", PCASES)
def test_ssor_factored_equals_two_sweeps(dim, n, p):
    pr = synth.random_small(61, dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    w = 1.3
    pc = O.Precond("ssor", dim, n, p, diags, omega=w)
    z = pc.apply(pr["f"])
    u1 = O.dsweep(dim, n, p, pc.dirs_f, diags, pr["f"], uold=np.zeros_like(pr["f"]), omega=w)
    u2 = O.dsweep(dim, n, p, pc.dirs_b, diags, pr["f"], uold=u1, omega=w)
    assert np.allclose(z, u2, rtol=1e-12, atol=1e-13 * np.abs(u2).max())


@pytest.mark.parametrize("dim,n", [(2, (9, 7)), (3, (5, 4, 3))])
def test_single_subdomain_matches_textbook(dim, n):
    """p = 1, d = (+...+) after reversal: Saad's SSOR M = (D - wE)D^-1(D - wF)/(w(2-w)) and ILU(0)."""
    pr = synth.random_small(71, dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    A = brute.dense_A(dim, n, diags)
    r = pr["f"]
    pc = O.Precond("ssor", dim, n, [1] * dim, diags, omega=1.4, phase=1)  # phase 1: forward (+,...,+)
    assert np.all(pc.dirs_f[0, :dim] == 1)
    Dm = np.diag(np.diag(A))
    L = np.tril(A, -1)
    U = np.triu(A, 1)
    w = 1.4
    M = (Dm + w * L) @ np.linalg.inv(Dm) @ (Dm + w * U) / (w * (2 - w))
    assert np.allclose(pc.apply(r), np.linalg.solve(M, r), rtol=1e-11, atol=1e-13)
    # textbook ILU(0): Gaussian elimination keeping only A's pattern
    Nn = A.shape[0]
    W = A.copy()
    pat = A != 0
    for i in range(1, Nn):
        for k in range(i):
            if pat[i, k]:
                W[i, k] /= W[k, k]
                for j in range(k + 1, Nn):
                    if pat[i, j]:
                        W[i, j] -= W[i, k] * W[k, j]
    Lf = np.tril(W, -1) + np.eye(Nn)
    Uf = np.triu(W)
    pci = O.Precond("ilu0", dim, n, [1] * dim, diags, phase=1)
    assert np.allclose(pci.piv, np.diag(Uf), rtol=1e-13)
    assert np.allclose(pci.apply(r), np.linalg.solve(Lf @ Uf, r), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
@pytest.mark.parametrize("dim,n,p", PCASES)
def test_transposed_is_adjoint(kind, dim, n, p):
    """<M^-1 x, y> = <x, M^-T y>; the symmetric form is symmetric."""
    pr = synth.random_small(81, dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    pc = O.Precond(kind, dim, n, p, diags, omega=1.2)
    g = synth.rng(9)
    x = g.standard_normal(pr["f"].size)
    y = g.standard_normal(pr["f"].size)
    lhs = pc.apply(x) @ y
    rhs = x @ pc.apply_t(y)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    assert abs(pc.apply_sym(x) @ y - x @ pc.apply_sym(y)) <= 1e-12 * (abs(lhs) + 1)


# ---------------------------------------------------------------- solvers
def test_cg_and_fgmres_reach_direct_solution():
    n = (20, 18)
    pr = synth.random_small(91, 2, n)
    diags = O.assemble(2, n, pr["alphas"])
    A = sp.csc_matrix(brute.dense_A(2, n, diags))
    xs = spla.spsolve(A, pr["f"])
    Aop = lambda v: O.spmv(2, n, diags, v)
    kappa = np.linalg.cond(A.toarray())
    for kind in ("ssor", "ilu0"):
        pc = O.Precond(kind, 2, n, (4, 3), diags, omega=1.0)
        x, it, rel = O.cg(Aop, pc.apply_sym, pr["f"], rtol=1e-10)
        assert rel < 1e-9 and np.linalg.norm(x - xs) <= kappa * 1e-9 * np.linalg.norm(xs)
        x, it, rel = O.fgmres(Aop, pc.apply, pr["f"], rtol=1e-10, restart=30)
        assert rel < 1e-9 and np.linalg.norm(x - xs) <= kappa * 1e-9 * np.linalg.norm(xs)


def test_stationary_decomposed_converges_to_exact_model_solution():
    """Model problem of Sec. 8: the parallel sweep converges to the d-linear exact solution."""
    n, diags, f, ue = O.model_problem(2, 21)
    u, it, rel = O.stationary_solve(2, (n, n), (3, 2), diags, 1.5, f, rtol=1e-12)
    assert rel <= 1e-12 and np.max(np.abs(u - ue)) < 1e-10
