"""Helpers for the GPU parity tests: seeded inputs to torch, tolerances."""
import numpy as np


def dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(x, ref):
    """max |x - ref| / max |ref| (FP64 parity metric; single-sweep bar 1e-12)."""
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def make_problem(dim, n, alphas, prec="f64"):
    import paper_1008_3699_amd as P
    pr = P.Problem(dim, n)
    pr.assemble([to_dev(a) for a in alphas], 0.0, prec)
    return pr
