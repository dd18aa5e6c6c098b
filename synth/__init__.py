"""Seeded synthetic inputs shaped like the paper's model problems.

This module holds no arithmetic of the method: it draws coefficient fields,
right-hand sides, problem sizes and arrival times from NumPy PCG64 streams.
Both the GPU path and the CPU oracle assemble their own matrices from these
raw fields.

Fields are node arrays on (n+2)^d nodes, boundary ring included, x fastest
(node (i,j,k) at i + (n0+2)*(j + (n1+2)*k)); right-hand sides are interior
arrays, x fastest.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def node_shape(dim, n):
    n = list(n) if np.ndim(n) else [n] * dim
    return tuple(v + 2 for v in reversed(n))


def constant_field(dim, n, value=1.0):
    return np.full(int(np.prod(node_shape(dim, n))), float(value))


def log_uniform_field(g: np.random.Generator, dim, n, lo=1e-2, hi=1e2):
    """Cell coefficients 10**U(log10 lo, log10 hi) i.i.d. on all nodes."""
    size = int(np.prod(node_shape(dim, n)))
    return 10.0 ** g.uniform(np.log10(lo), np.log10(hi), size)


def uniform_rhs(g: np.random.Generator, N, lo=-1.0, hi=1.0):
    return g.uniform(lo, hi, int(N))


# ------------------------------------------------------------ named workloads
def poisson_2d_64(seed=1001):
    """64x64 interior, unit coefficients, rhs U[-1,1]."""
    n = (64, 64)
    f = uniform_rhs(rng(seed), 64 * 64)
    return dict(dim=2, n=n, alphas=[constant_field(2, n)] * 2, beta=0.0, f=f)


def varcoef_2d(n=2048, seed_alpha=2001, seed_f=2002):
    """n x n interior, isotropic cell coefficient log-uniform in [1e-2, 1e2], rhs U[-1,1]."""
    nn = (n, n)
    al = log_uniform_field(rng(seed_alpha), 2, nn)
    f = uniform_rhs(rng(seed_f), n * n)
    return dict(dim=2, n=nn, alphas=[al, al], beta=0.0, f=f)


def poisson_3d(n=256, seed=3001):
    nn = (n, n, n)
    f = uniform_rhs(rng(seed), n ** 3)
    c = constant_field(3, nn)
    return dict(dim=3, n=nn, alphas=[c, c, c], beta=0.0, f=f)


def anisotropic_batch(count=512, nmin=32, nmax=512, seed0=4000):
    """Problems -(u_xx + eps u_yy): n ~ U{nmin..nmax}, eps = 10**U(-3, 0), rhs U[-1,1]."""
    out = []
    for b in range(count):
        g = rng(seed0 + b)
        n = int(g.integers(nmin, nmax + 1))
        eps = 10.0 ** g.uniform(-3.0, 0.0)
        nn = (n, n)
        f = uniform_rhs(g, n * n)
        out.append(dict(dim=2, n=nn, alphas=[constant_field(2, nn, 1.0), constant_field(2, nn, eps)],
                        beta=0.0, f=f, eps=eps))
    return out


def serving_stream(count=2000, rate=200.0, seed=5000, n2=(64, 1024), n3=(32, 128), lo=1e-2, hi=1e2):
    """Poisson arrivals; each request is 2D (prob 1/2) or 3D with log-uniform coefficients.

    Returns a list of dicts with arrival time t (s), dim, n, and a per-request
    seed from which ``request_fields`` draws the coefficient field and rhs.
    """
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    reqs = []
    for i in range(count):
        dim = 2 if g.uniform() < 0.5 else 3
        lo_n, hi_n = n2 if dim == 2 else n3
        n = int(g.integers(lo_n, hi_n + 1))
        reqs.append(dict(t=float(t[i]), dim=dim, n=(n,) * dim, seed=int(g.integers(0, 2 ** 31 - 1))))
    return reqs


def request_fields(req, lo=1e-2, hi=1e2):
    g = rng(req["seed"])
    dim, n = req["dim"], req["n"]
    al = log_uniform_field(g, dim, n, lo, hi)
    f = uniform_rhs(g, int(np.prod(n)))
    return dict(dim=dim, n=n, alphas=[al] * dim, beta=0.0, f=f)


def random_small(seed, dim, n, lo=1e-1, hi=1e1):
    """Small random variable-coefficient problem for parity tests."""
    g = rng(seed)
    al = [log_uniform_field(g, dim, n, lo, hi) for _ in range(dim)]
    N = int(np.prod(n))
    return dict(dim=dim, n=tuple(n), alphas=al, beta=0.0, f=uniform_rhs(g, N), u=uniform_rhs(g, N))
