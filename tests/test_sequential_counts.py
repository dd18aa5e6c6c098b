"""Decomposed against sequential iteration counts (CPU oracle, stored runs).

The decomposed sweep is a different iteration from lexicographic SOR / ILU(0), so its counts to a
tolerance differ; the stored runs of tests/golden/make_sequential_iterations.py record both.  Here the
64^2 SOR case is recomputed (it takes well under a second) and the stored counts are held to the 10 %
margin of the measured configurations.
"""
import json
import math
import os

import numpy as np

import synth
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sequential_iterations.json")


def _stored():
    return json.load(open(GOLDEN))


def test_sor64_counts_reproduce_and_stay_within_ten_percent():
    rec = _stored()["poisson2d64_sor"]
    w = synth.poisson_2d_64()
    diags = O.assemble(2, w["n"], w["alphas"], w["beta"])
    omega = 2.0 / (1.0 + math.sin(math.pi / 65))
    assert rec["omega"] == omega
    got = {}
    for key, p in (("sweeps_sequential", (1, 1)), ("sweeps_4x4", (4, 4))):
        _, sweeps, rel = O.stationary_solve(2, w["n"], p, diags, omega, w["f"], rtol=1e-8, maxit=20000)
        assert rel <= 1e-8
        got[key] = sweeps
    assert got["sweeps_sequential"] == rec["sweeps_sequential"]
    assert got["sweeps_4x4"] == rec["sweeps_4x4"]
    assert got["sweeps_4x4"] <= 1.10 * got["sweeps_sequential"]


def test_sor64_row_wise_and_symmetric_counts_reproduce():
    """The two other sequential comparators of the 64^2 SOR case: row-wise SOR from the SW corner every
    sweep (RSOR) and symmetric SOR (SSOR).  At the optimal factor the alternating schedule (FSOR, and the
    decomposed sweep that follows it) needs about twice RSOR's sweeps; both comparators are reported."""
    rec = _stored()["poisson2d64_sor"]
    w = synth.poisson_2d_64()
    diags = O.assemble(2, w["n"], w["alphas"], w["beta"])
    omega = rec["omega"]
    nf = np.linalg.norm(w["f"])
    for key, dirs in (("sweeps_rsor", [(1, 1)]), ("sweeps_ssor", [(1, 1), (-1, -1)])):
        u = np.zeros(4096)
        k = 0
        while True:
            u = O.sor_lex(2, w["n"], diags, omega, dirs[k % len(dirs)], w["f"], u)
            k += 1
            if np.linalg.norm(w["f"] - O.spmv(2, w["n"], diags, u)) / nf <= 1e-8:
                break
        assert k == rec[key], (key, k, rec[key])
    assert rec["sweeps_rsor"] < rec["sweeps_sequential"]


def test_stored_3d_sequential_count_is_a_converged_run():
    rec = _stored()["poisson3d256"]
    assert rec["subdomains"] == [1, 1, 1] and rec["rtol"] == 1e-8
    assert rec["relres_true"] <= 1e-8 * 1.05 and 100 < rec["iterations"] < 1000
    assert np.isfinite(rec["cpu_s"])


def test_stored_2048_counts_are_converged_runs_within_ten_percent():
    """The 2048^2 ILU(0) and SSOR(1) CG counts from the oracle: one subdomain (lexicographic ILU(0) /
    SSOR) and 16x16 subdomains (the decomposed preconditioner's symmetric form); every stored run
    converged, and each decomposed count is within 10 % of its sequential one."""
    recs = _stored()
    for kind, ks, kd in (("ilu0", "varcoef2048", "varcoef2048_p16"), ("ssor", "varcoef2048_ssor", "varcoef2048_ssor_p16")):
        seq, dec = recs[ks], recs[kd]
        assert seq["subdomains"] == [1, 1] and dec["subdomains"] == [16, 16]
        for r in (seq, dec):
            assert r["rtol"] == 1e-8 and r["relres_true"] <= 1.05e-8 and r["precond"] == kind
        assert dec["iterations"] <= 1.10 * seq["iterations"], kind
