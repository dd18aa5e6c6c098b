"""1D (tridiagonal) problems on the GPU (Sec. 2): decomposed sweeps with the 2x2 coupled blocks of
eq. 1d:sorc, the preconditioner passes, ILU(0) = LU on one subdomain, Krylov counts, and the
restricted-overlap sweep, all against the CPU FP64 oracle."""
import numpy as np
import pytest

import synth
from gpu_util import dev, make_problem, relmax, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu

CASES = [((40,), (4,)), ((37,), (5,)), ((9,), (1,)), ((64,), (32,)), ((1000,), (7,))]


def _prob(n, seed=1):
    pr = synth.random_small(seed + n[0], 1, n)
    return pr, O.assemble(1, n, pr["alphas"])


@pytest.mark.parametrize("path", ["auto", "generic"])
@pytest.mark.parametrize("n,p", CASES)
def test_1d_stationary_sweep(n, p, path):
    import torch
    pr, diags = _prob(n)
    g = make_problem(1, n, pr["alphas"])
    g.set_path(path)
    om = [1.6, 0.8]
    g.set_relaxation(om)
    u = to_dev(pr["u"]); f = to_dev(pr["f"]); out = torch.empty_like(u)
    for phase in (0, 1):
        g.set_decomposition(p, overlap=2, phase=phase)
        for k in range(2):
            g.sweep(k, u, f, out)
            ref = O.dsweep(1, n, p, O.schedule(1, p, k, phase), diags, pr["f"], uold=pr["u"], omega=om)
            assert relmax(to_np(out), ref) <= 1e-12, (phase, k)


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
@pytest.mark.parametrize("n,p", CASES)
def test_1d_preconditioner_passes(kind, n, p):
    import torch
    pr, diags = _prob(n, seed=5)
    g = make_problem(1, n, pr["alphas"])
    g.set_relaxation([1.3])
    g.set_decomposition(p, overlap=2, phase=0)
    pc = O.Precond(kind, 1, n, p, diags, omega=1.3)
    refs = {0: pc.forward(pr["f"]), 1: pc.backward(pr["u"]),
            2: O.dsolve_t(1, n, p, pc.dirs_b, diags, pc.piv, pr["f"]),
            3: pc.c * O.dsolve_t(1, n, p, pc.dirs_f, diags, pc.piv, pc.piv * pr["u"])}
    inputs = {0: pr["f"], 1: pr["u"], 2: pr["f"], 3: pr["u"]}
    out = torch.empty(n[0], dtype=torch.float64, device=dev())
    for which in range(4):
        g.precond_half(kind, which, to_dev(inputs[which]), out)
        assert relmax(to_np(out), refs[which]) <= 1e-12, which
    g.precond_apply(kind, to_dev(pr["f"]), out, symmetric=True)
    assert relmax(to_np(out), pc.apply_sym(pr["f"])) <= 1e-12


def test_1d_ilu_on_one_subdomain_is_exact_lu():
    """Tridiagonal ILU(0) with one subdomain drops nothing: M = A, so preconditioned CG takes one step and
    the preconditioner applied to A x returns x."""
    import torch
    n = (500,)
    pr, diags = _prob(n, seed=9)
    g = make_problem(1, n, pr["alphas"])
    g.set_relaxation([1.0])
    g.set_decomposition((1,), overlap=2)
    x = to_dev(pr["u"]); ax = torch.empty_like(x); z = torch.empty_like(x)
    g.spmv(x, ax)
    g.precond_apply("ilu0", ax, z, symmetric=False)
    assert relmax(to_np(z), pr["u"]) <= 1e-12
    u = torch.zeros_like(x)
    info = g.solve("cg", "ilu0", to_dev(pr["f"]), u, rtol=1e-10)
    assert info["converged"] and info["iters"] == 1, info


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
def test_1d_krylov_counts_match_oracle(kind):
    """1D Poisson (unit coefficients), 300 points, 6 subdomains: CG and FGMRES counts within 1 of the
    oracle's (random coefficients make a 300-point 1D operator so ill-conditioned that CG's count is a
    matter of rounding)."""
    import torch
    n, p = (300,), (6,)
    al = synth.constant_field(1, n)
    pr = {"alphas": [al], "f": synth.uniform_rhs(synth.rng(21), 300)}
    diags = O.assemble(1, n, pr["alphas"])
    Aop = lambda v: O.spmv(1, n, diags, v)
    pc = O.Precond(kind, 1, n, p, diags, omega=1.0)
    xr, it_cg, _ = O.cg(Aop, pc.apply_sym, pr["f"], rtol=1e-8)
    _, it_gm, _ = O.fgmres(Aop, pc.apply, pr["f"], rtol=1e-8, restart=30)
    g = make_problem(1, n, pr["alphas"])
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2)
    f = to_dev(pr["f"])
    u = torch.zeros_like(f)
    info = g.solve("cg", kind, f, u, rtol=1e-8)
    assert info["converged"] and abs(info["iters"] - it_cg) <= 1, (info, it_cg)
    assert np.linalg.norm(to_np(u) - xr) <= 1e-6 * np.linalg.norm(xr)
    u.zero_()
    info = g.solve("fgmres", kind, f, u, rtol=1e-8, restart=30)
    assert info["converged"] and abs(info["iters"] - it_gm) <= 1, (info, it_gm)


@pytest.mark.parametrize("overlap", [0, 1, 3])
def test_1d_restricted_sweep(overlap):
    import torch
    n, p = (50,), (5,)
    pr, diags = _prob(n, seed=31)
    g = make_problem(1, n, pr["alphas"])
    om = [1.4, 1.1]
    g.set_relaxation(om)
    g.set_decomposition(p, overlap=overlap)
    u = to_dev(pr["u"]); f = to_dev(pr["f"]); out = torch.empty_like(u)
    for k in range(2):
        g.sweep_restricted(k, u, f, out)
        ref = O.ras_sweep(1, n, p, O.schedule(1, p, k), diags, pr["f"], pr["u"], om, overlap)
        assert relmax(to_np(out), ref) <= 1e-12, k
