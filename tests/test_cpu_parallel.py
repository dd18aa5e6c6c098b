"""The multi-core CPU baseline (bench_cpu: OpenMP over subdomains, partner points across coupled start
faces recomputed per subdomain) against the oracle: stationary sweeps with per-corner factors and
start-coupled preconditioner half-sweeps, 1D to 3D, within 1e-12."""
import numpy as np
import pytest

import bench_cpu as C
import synth
from oracle import oracle as O

CASES = [(1, (40,), (4,)), (2, (13, 11), (3, 2)), (2, (37, 29), (5, 3)), (2, (16, 16), (4, 4)),
         (3, (7, 6, 5), (2, 2, 2)), (3, (12, 9, 10), (3, 2, 4)), (2, (20, 8), (1, 1))]


def _rel(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("dim,n,p", CASES)
def test_stationary_sweep_matches_oracle(dim, n, p):
    pr = synth.random_small(7 + sum(n), dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    om = list(synth.rng(9).uniform(0.7, 1.8, 1 << dim))
    for phase in (0, 1):
        for k in range(1 << dim):
            dirs = O.schedule(dim, p, k, phase)
            got = C.dsweep(dim, n, p, dirs, diags, pr["f"], uold=pr["u"], omega=om)
            ref = O.dsweep(dim, n, p, dirs, diags, pr["f"], uold=pr["u"], omega=om)
            assert _rel(got, ref) <= 1e-12, (phase, k)


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
@pytest.mark.parametrize("dim,n,p", CASES)
def test_preconditioner_half_sweeps_match_oracle(kind, dim, n, p):
    pr = synth.random_small(3 + sum(n), dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    pc = O.Precond(kind, dim, n, p, diags, omega=1.2)
    got = C.dsweep(dim, n, p, pc.dirs_f, diags, pr["f"], piv=pc.piv)
    assert _rel(got, pc.forward(pr["f"])) <= 1e-12
    got = C.dsweep(dim, n, p, pc.dirs_b, diags, pc.piv * pr["u"], piv=pc.piv)
    assert _rel(pc.c * got, pc.backward(pr["u"])) <= 1e-12


def test_threads_and_triad():
    assert C.threads() >= 1
    assert C.triad_gbs(n=1 << 20, reps=2) > 0
