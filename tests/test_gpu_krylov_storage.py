"""Krylov solves on operators given as user diagonals, symmetric and not.

The library checks at set-up whether the lower couplings equal the neighbours' upper ones bit for
bit; the CG / FGMRES loops then read only the upper couplings.  Here:
* a symmetric operator (the oracle's assembly) given through psw_set_diagonals: CG and FGMRES
  counts within 1 of the oracle's and the CG solution within 1e-6;
* the same operator with one coupling changed in its last bit (no longer symmetric): the general
  SpMV runs, and CG reaches the oracle's solution (1e-6) with its count within 1;
* a non-symmetric operator (W and E couplings scaled differently, a^P raised to keep diagonal
  dominance): FGMRES with the preconditioner pair against the oracle's FGMRES;
* a 3D operator one bit off with FP32 sweeps: CG against the oracle's FP64 CG.
"""
import numpy as np
import pytest

import synth
from gpu_util import dev, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu

CASES = [(2, (41, 30), (3, 2)), (3, (12, 10, 9), (2, 2, 3))]


def _problem(dim, n, diags):
    import paper_1008_3699_amd as P
    g = P.Problem(dim, n)
    g.set_diagonals([np.ascontiguousarray(d) for d in diags], prec="f64")
    g.set_relaxation([1.0])
    return g


@pytest.mark.parametrize("dim,n,p", CASES)
def test_symmetric_user_diagonals_and_one_bit_off(dim, n, p):
    import torch
    pr = synth.random_small(700 + sum(n), dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    f = pr["f"]
    Aop = lambda v: O.spmv(dim, n, diags, v)
    pc = O.Precond("ilu0", dim, n, p, diags, omega=1.0)
    xr, it_cg, _ = O.cg(Aop, pc.apply_sym, f, rtol=1e-8)
    _, it_gm, _ = O.fgmres(Aop, pc.apply, f, rtol=1e-8, restart=30)
    N = int(np.prod(n))
    g = _problem(dim, n, diags)
    g.set_decomposition(p, overlap=2)
    u = torch.zeros(N, dtype=torch.float64, device=dev())
    info = g.solve("cg", "ilu0", to_dev(f), u, rtol=1e-8)
    assert info["converged"] and abs(info["iters"] - it_cg) <= 1, (info, it_cg)
    x_sym = to_np(u)
    assert np.linalg.norm(x_sym - xr) <= 1e-6 * np.linalg.norm(xr)
    u.zero_()
    info = g.solve("fgmres", "ilu0", to_dev(f), u, rtol=1e-8, restart=30)
    assert info["converged"] and abs(info["iters"] - it_gm) <= 1, (info, it_gm)
    # one east coupling one unit in the last place larger: not symmetric any more
    d2 = [d.copy() for d in diags]
    k = N // 2
    assert d2[2][k] > 0
    d2[2][k] = np.nextafter(d2[2][k], np.inf)
    h = _problem(dim, n, d2)
    h.set_decomposition(p, overlap=2)
    u.zero_()
    info2 = h.solve("cg", "ilu0", to_dev(f), u, rtol=1e-8)
    assert info2["converged"] and abs(info2["iters"] - it_cg) <= 1, (info2, it_cg)
    assert np.linalg.norm(to_np(u) - xr) <= 1e-6 * np.linalg.norm(xr)


@pytest.mark.parametrize("dim,n,p", CASES)
def test_nonsymmetric_user_diagonals_fgmres(dim, n, p):
    import torch
    pr = synth.random_small(800 + sum(n), dim, n)
    diags = [d.copy() for d in O.assemble(dim, n, pr["alphas"])]
    # upwind-like skew along x: W couplings x1.5, E couplings x0.6; a^P covers the larger sum
    extra = 0.5 * diags[1] - 0.4 * diags[2]
    diags[1] *= 1.5
    diags[2] *= 0.6
    diags[0] = diags[0] + np.maximum(extra, 0.0)
    f = pr["f"]
    Aop = lambda v: O.spmv(dim, n, diags, v)
    pc = O.Precond("ssor", dim, n, p, diags, omega=1.0)
    xr, it_gm, _ = O.fgmres(Aop, pc.apply, f, rtol=1e-8, restart=30)
    g = _problem(dim, n, diags)
    g.set_decomposition(p, overlap=2)
    u = torch.zeros(int(np.prod(n)), dtype=torch.float64, device=dev())
    info = g.solve("fgmres", "ssor", to_dev(f), u, rtol=1e-8, restart=30)
    assert info["converged"] and abs(info["iters"] - it_gm) <= 1, (info, it_gm)
    x = to_np(u)
    assert np.linalg.norm(x - xr) <= 1e-6 * np.linalg.norm(xr)
    rel = np.linalg.norm(f - Aop(x)) / np.linalg.norm(f)
    assert rel <= 1.05e-8


def test_nonsymmetric_storage_fp32_sweeps_3d_cg():
    """3D CG with FP32 sweeps (the LDS-tile passes, whose transposed pair stays a separate FP32 piece of
    z) on an operator given as user diagonals with one coupling one unit in the last place off: the
    general operator product inside the fused CG step, against the oracle's FP64 CG on the same
    perturbed operator (solution within 1e-7, count within 10 %, true residual through the oracle's
    SpMV)."""
    import torch
    dim, n, p = 3, (24, 20, 18), (2, 2, 2)
    pr = synth.random_small(900 + sum(n), dim, n)
    diags = [d.copy() for d in O.assemble(dim, n, pr["alphas"])]
    N = int(np.prod(n))
    k = N // 3
    assert diags[6][k] > 0
    diags[6][k] = np.nextafter(diags[6][k], np.inf)  # one F coupling: no longer symmetric
    f = pr["f"]
    Aop = lambda v: O.spmv(dim, n, diags, v)
    pc = O.Precond("ilu0", dim, n, p, diags, omega=1.0)
    xr, it_or, _ = O.cg(Aop, pc.apply_sym, f, rtol=1e-8)
    import paper_1008_3699_amd as P
    g = P.Problem(dim, n)
    g.set_diagonals([np.ascontiguousarray(d) for d in diags], prec="f32")
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2)
    u = torch.zeros(N, dtype=torch.float64, device=dev())
    info = g.solve("cg", "ilu0", to_dev(f), u, rtol=1e-8, maxit=5000)
    x = to_np(u)
    rel = np.linalg.norm(f - Aop(x)) / np.linalg.norm(f)
    err = np.linalg.norm(x - xr) / np.linalg.norm(xr)
    print(f"iters {info['iters']} (oracle FP64 {it_or}), true relres {rel:.2e}, error {err:.2e}", flush=True)
    assert info["converged"] and rel <= 1.05e-8
    assert abs(info["iters"] - it_or) <= max(2, 0.1 * it_or)
    assert err <= 1e-7
