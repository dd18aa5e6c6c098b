"""psw_precond_apply_noalloc (the preconditioner call that allocates nothing) against psw_precond_apply.

The variant keeps the pair form's intermediate vector in the library's fixed device array; its result
must equal psw_precond_apply(symmetric = 0) bit for bit (same kernels, same inputs), on consecutive
calls whose second input is smaller, and the handle's device memory must not grow.
"""
import numpy as np
import pytest

import synth
from gpu_util import make_problem, to_dev, to_np

pytestmark = pytest.mark.gpu


def _problem(dim, n, p, prec, kind, seed, setup=True):
    pr = synth.random_small(seed, dim, n)
    g = make_problem(dim, n, pr["alphas"], prec=prec)
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2)
    if setup:
        g.precond_setup(kind)
    return g, pr


def test_noalloc_equals_precond_apply_on_consecutive_calls():
    import torch
    # pipelined 2D FP64 (8 MiB of scratch), then smaller inputs: the 3D LDS-tile path with BF16 storage
    # (FP32 intermediate) and a 2D FP32 problem
    cases = [(2, (1024, 1000), (8, 8), "f64", "ilu0", 1), (3, (40, 36, 33), (2, 2, 2), "bf16", "ssor", 2),
             (2, (100, 90), (3, 2), "f32", "ilu0", 3)]
    for dim, n, p, prec, kind, seed in cases:
        print(f"case dim={dim} n={n} p={p} {prec} {kind}", flush=True)
        g, pr = _problem(dim, n, p, prec, kind, seed)
        r = to_dev(pr["f"])
        ref = torch.empty_like(r)
        g.precond_apply(kind, r, ref, symmetric=False)
        held = g.device_bytes()
        for rep in range(2):
            z = torch.full_like(r, float("nan"))
            g.precond_apply_noalloc(kind, r, z)
            assert np.array_equal(to_np(z), to_np(ref)), (dim, n, prec, kind, rep)
        assert g.device_bytes() == held


def test_noalloc_rejects_what_it_cannot_do():
    import torch
    import paper_1008_3699_amd as P
    # FP64 intermediate of 8,400,000 points: 67.2 MB, beyond the 64 MiB array
    big = P.Problem(2, (3000, 2800))
    r = torch.zeros(big.N, dtype=torch.float64, device="cuda:0")
    z = torch.empty_like(r)
    with pytest.raises(P.PswError) as e:
        big.precond_apply_noalloc("ilu0", r, z)
    assert e.value.status == -1  # PSW_EINVAL
    # a preconditioner that is not set up would need allocation: PSW_ESTATE
    g, pr = _problem(2, (64, 64), (2, 2), "f64", "ssor", 4, setup=False)
    r = to_dev(pr["f"])
    with pytest.raises(P.PswError) as e:
        g.precond_apply_noalloc("ssor", r, torch.empty_like(r))
    assert e.value.status == -9  # PSW_ESTATE
