"""Batched CG (psw_batch_solve): results identical alone and in a batch; counts match the oracle."""
import numpy as np
import pytest

import synth
from gpu_util import dev, make_problem, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _aniso(n, eps, seed):
    g = synth.rng(seed)
    nn = (n, n)
    al = [synth.constant_field(2, nn, 1.0), synth.constant_field(2, nn, eps)]
    return al, synth.uniform_rhs(g, n * n)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
def test_batch_equals_alone(kind, prec):
    import paper_1008_3699_amd as P
    import torch
    specs = [(40, 0.3, (2, 2)), (96, 0.01, (1, 1)), (150, 1.0, (2, 3)), (33, 0.05, (3, 1)), (200, 0.002, (2, 2))]
    probs, fs, alone = [], [], []
    for i, (n, eps, p) in enumerate(specs):
        al, f = _aniso(n, eps, 700 + i)
        g = make_problem(2, (n, n), al, prec=prec)
        g.set_relaxation([1.0])
        g.set_decomposition(p, overlap=2)
        probs.append(g)
        fs.append(to_dev(f))
    hosts = []
    for g, f in zip(probs, fs):
        u = torch.zeros_like(f)
        info = P.batch_solve([g], [f], [u], precond=kind, rtol=1e-8)[0]  # alone: a batch of one
        alone.append((info, to_np(u)))
        v = torch.zeros_like(f)
        g.solve("cg", kind, f, v, rtol=1e-8)  # the host-driven solver, other reduction order
        hosts.append(to_np(v))
    us = [torch.zeros_like(f) for f in fs]
    infos = P.batch_solve(probs, fs, us, precond=kind, rtol=1e-8)
    for (ia, ua), ib, ub, uh in zip(alone, infos, us, hosts):
        assert ib["converged"] and ia["converged"]
        assert ib["iters"] == ia["iters"]
        assert np.array_equal(to_np(ub), ua)  # bitwise: the mix does not change a problem's arithmetic
        assert ib["relres"] <= 1.5e-8
        assert np.linalg.norm(to_np(ub) - uh) <= 1e-5 * np.linalg.norm(uh)


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
def test_batch_iterations_match_oracle(kind):
    import paper_1008_3699_amd as P
    import torch
    specs = [(48, 0.1, (2, 2)), (70, 0.7, (3, 2))]
    probs, fs, refs = [], [], []
    for i, (n, eps, p) in enumerate(specs):
        al, f = _aniso(n, eps, 900 + i)
        diags = O.assemble(2, (n, n), al)
        pc = O.Precond(kind, 2, (n, n), p, diags, omega=1.0)
        _, it, _ = O.cg(lambda v: O.spmv(2, (n, n), diags, v), pc.apply_sym, f, rtol=1e-8)
        refs.append(it)
        g = make_problem(2, (n, n), al)
        g.set_relaxation([1.0])
        g.set_decomposition(p, overlap=2)
        probs.append(g)
        fs.append(to_dev(f))
    us = [torch.zeros_like(f) for f in fs]
    infos = P.batch_solve(probs, fs, us, precond=kind, rtol=1e-8)
    for info, it in zip(infos, refs):
        assert info["converged"] and abs(info["iters"] - it) <= 1, (info, it)
