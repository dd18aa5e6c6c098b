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


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
def test_batch_solution_matches_oracle(kind):
    """Batched FP64 CG against the oracle's FP64 CG: every solution within 1e-6 (relative 2-norm) of the
    oracle's iterate, and a true residual, through the oracle's own product, within the tolerance."""
    import paper_1008_3699_amd as P
    import torch
    specs = [(64, 0.05, (2, 2)), (90, 0.6, (3, 2)), (37, 1.0, (1, 1)), (120, 0.003, (4, 3))]
    probs, fs, refs, ops = [], [], [], []
    for i, (n, eps, p) in enumerate(specs):
        al, f = _aniso(n, eps, 1300 + i)
        diags = O.assemble(2, (n, n), al)
        pc = O.Precond(kind, 2, (n, n), p, diags, omega=1.0)
        x, it, _ = O.cg(lambda v, d=diags, m=n: O.spmv(2, (m, m), d, v), pc.apply_sym, f, rtol=1e-8)
        refs.append((x, it))
        ops.append((diags, f))
        g = make_problem(2, (n, n), al)
        g.set_relaxation([1.0])
        g.set_decomposition(p, overlap=2)
        probs.append(g)
        fs.append(to_dev(f))
    us = [torch.zeros_like(f) for f in fs]
    infos = P.batch_solve(probs, fs, us, precond=kind, rtol=1e-8)
    for (n, _, _), info, u, (x, it), (diags, f) in zip(specs, infos, us, refs, ops):
        got = to_np(u)
        err = np.linalg.norm(got - x) / np.linalg.norm(x)
        rel = np.linalg.norm(f - O.spmv(2, (n, n), diags, got)) / np.linalg.norm(f)
        print(f"n={n}: iters {info['iters']} (oracle {it}), error vs oracle {err:.2e}, true relres {rel:.2e}",
              flush=True)
        assert info["converged"] and abs(info["iters"] - it) <= 1
        assert err <= 1e-6
        assert rel <= 1.05e-8
