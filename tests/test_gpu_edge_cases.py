"""The smallest legal decompositions against the CPU FP64 oracle.

Every subdomain is 2 points long on some axis (the minimum the decomposition takes), so the
coupled blocks touch each other or cover the whole subdomain: 2x2 tiles in 2D are all face
pair and cross point, 2x2x2 tiles in 3D all face, edge and corner blocks.  One subdomain on the
whole 2-point grid, ragged splits (5 = 3 + 2) and 1D grids of 2 and 4 points are included.  Each
case: every schedule step of the stationary sweep in both phases with per-corner factors, the
four preconditioner half-sweeps, the pair and the symmetric form, on both kernel paths, at 1e-12;
the 3D cases also with FP32 sweeps on the LDS-tile passes against the FP64 oracle.
"""
import numpy as np
import pytest

import synth
from gpu_util import dev, make_problem, relmax, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu

CASES = [
    (1, (2,), (1,)), (1, (4,), (2,)), (1, (5,), (2,)),
    (2, (2, 2), (1, 1)), (2, (4, 4), (2, 2)), (2, (5, 4), (2, 2)), (2, (4, 2), (2, 1)), (2, (6, 6), (3, 3)),
    (3, (2, 2, 2), (1, 1, 1)), (3, (4, 4, 4), (2, 2, 2)), (3, (5, 4, 4), (2, 2, 2)), (3, (6, 4, 2), (3, 2, 1)),
]


def _prob(dim, n, seed):
    pr = synth.random_small(seed + sum(n), dim, n)
    return pr, O.assemble(dim, n, pr["alphas"])


@pytest.mark.parametrize("path", ["auto", "generic"])
@pytest.mark.parametrize("dim,n,p", CASES)
def test_smallest_decompositions_sweep(dim, n, p, path):
    import torch
    pr, diags = _prob(dim, n, 11)
    g = make_problem(dim, n, pr["alphas"])
    g.set_path(path)
    om = list(synth.rng(5).uniform(0.7, 1.9, 1 << dim))
    g.set_relaxation(om)
    u = to_dev(pr["u"]); f = to_dev(pr["f"]); out = torch.empty_like(u)
    for phase in (0, 1):
        g.set_decomposition(p, overlap=2, phase=phase)
        for k in range(1 << dim):
            g.sweep(k, u, f, out)
            ref = O.dsweep(dim, n, p, O.schedule(dim, p, k, phase), diags, pr["f"], uold=pr["u"], omega=om)
            assert relmax(to_np(out), ref) <= 1e-12, (phase, k)


@pytest.mark.parametrize("path", ["auto", "generic"])
@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
@pytest.mark.parametrize("dim,n,p", CASES)
def test_smallest_decompositions_preconditioner(dim, n, p, kind, path):
    import torch
    pr, diags = _prob(dim, n, 13)
    g = make_problem(dim, n, pr["alphas"])
    g.set_path(path)
    w = 1.2
    g.set_relaxation([w])
    g.set_decomposition(p, overlap=2, phase=0)
    pc = O.Precond(kind, dim, n, p, diags, omega=w)
    refs = {
        0: pc.forward(pr["f"]),
        1: pc.backward(pr["u"]),
        2: O.dsolve_t(dim, n, p, pc.dirs_b, diags, pc.piv, pr["f"]),
        3: pc.c * O.dsolve_t(dim, n, p, pc.dirs_f, diags, pc.piv, pc.piv * pr["u"]),
    }
    inputs = {0: pr["f"], 1: pr["u"], 2: pr["f"], 3: pr["u"]}
    out = torch.empty(int(np.prod(n)), dtype=torch.float64, device=dev())
    for which in range(4):
        g.precond_half(kind, which, to_dev(inputs[which]), out)
        assert relmax(to_np(out), refs[which]) <= 1e-12, which
    r = to_dev(pr["f"])
    g.precond_apply(kind, r, out, symmetric=False)
    assert relmax(to_np(out), pc.apply(pr["f"])) <= 1e-12
    g.precond_apply(kind, r, out, symmetric=True)
    assert relmax(to_np(out), pc.apply_sym(pr["f"])) <= 1e-12


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
@pytest.mark.parametrize("dim,n,p", [c for c in CASES if c[0] == 3])
def test_smallest_3d_tiles_fp32(dim, n, p, kind):
    """FP32 sweeps (the LDS-tile passes where they apply): relative 2-norm error against the FP64
    oracle within 2e-6 for every pass and both forms."""
    import torch
    pr, diags = _prob(dim, n, 17)
    g = make_problem(dim, n, pr["alphas"], prec="f32")
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2, phase=0)
    pc = O.Precond(kind, dim, n, p, diags, omega=1.0)
    refs = {
        0: pc.forward(pr["f"]),
        1: pc.backward(pr["u"]),
        2: O.dsolve_t(dim, n, p, pc.dirs_b, diags, pc.piv, pr["f"]),
        3: pc.c * O.dsolve_t(dim, n, p, pc.dirs_f, diags, pc.piv, pc.piv * pr["u"]),
    }
    inputs = {0: pr["f"], 1: pr["u"], 2: pr["f"], 3: pr["u"]}
    out = torch.empty(int(np.prod(n)), dtype=torch.float64, device=dev())
    for which in range(4):
        g.precond_half(kind, which, to_dev(inputs[which]), out)
        ref = refs[which]
        err = np.linalg.norm(to_np(out) - ref) / np.linalg.norm(ref)
        assert err <= 2e-6, (which, err)
    for sym in (False, True):
        g.precond_apply(kind, to_dev(pr["f"]), out, symmetric=sym)
        ref = pc.apply_sym(pr["f"]) if sym else pc.apply(pr["f"])
        err = np.linalg.norm(to_np(out) - ref) / np.linalg.norm(ref)
        assert err <= 2e-6, (sym, err)
