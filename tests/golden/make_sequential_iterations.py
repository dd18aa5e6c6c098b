"""Iteration counts of the sequential and decomposed preconditioners on the measured workloads.

With one subdomain the decomposed ILU(0) is lexicographic ILU(0), and its symmetric form is M^-1
itself.  The counts are the CG iterations to a relative residual of 1e-8 from x0 = 0, computed by the
FP64 CPU oracle on the same seeded inputs as the GPU measurements, and written to
sequential_iterations.json beside this script.  Run: python tests/golden/make_sequential_iterations.py
[sor64|2d|2d16|2dssor|2dssor16|3d]  (each 2048^2 case takes one to two hours on one core).
"""
import fcntl
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "sequential_iterations.json")


def run(name, w, kind="ilu0", rtol=1e-8, p=None):
    dim, n = w["dim"], w["n"]
    p = (1,) * dim if p is None else tuple(p)
    diags = O.assemble(dim, n, w["alphas"], w["beta"])
    pc = O.Precond(kind, dim, n, p, diags, omega=1.0)
    calls = [0]
    t0 = time.time()

    def apply_m(r):
        calls[0] += 1
        if calls[0] % 200 == 0:
            print(f"{name}: {calls[0]} preconditioner applications, {time.time() - t0:.0f} s", flush=True)
        return pc.apply_sym(r)

    _, iters, rel = O.cg(lambda x: O.spmv(dim, n, diags, x), apply_m, w["f"], rtol=rtol, maxit=100000)
    rec = {"workload": name, "precond": kind, "subdomains": list(p), "rtol": rtol, "iterations": int(iters),
           "relres_true": float(rel), "cpu_s": round(time.time() - t0, 1)}
    print(json.dumps(rec), flush=True)
    return rec


def lex_sweeps(n, diags, omega, f, directions, rtol=1e-8, maxit=20000):
    """Sweeps of lexicographic SOR (one subdomain) cycling through the given directions until
    ||f - A u|| / ||f|| <= rtol, from u = 0."""
    u = np.zeros_like(f)
    nf = np.linalg.norm(f)
    for k in range(maxit):
        u = O.sor_lex(2, n, diags, omega, directions[k % len(directions)], f, u)
        if np.linalg.norm(f - O.spmv(2, n, diags, u)) / nf <= rtol:
            return k + 1
    return maxit


def run_sor64():
    """64^2 Poisson, SOR at omega = 2/(1+sin(pi/65)) to 1e-8: sweeps with one subdomain (the alternating
    schedule, FSOR), with 4x4, and of row-wise SOR always sweeping from the SW corner (RSOR) and of
    symmetric SOR (SW then NE, SSOR)."""
    w = synth.poisson_2d_64()
    n = w["n"]
    diags = O.assemble(2, n, w["alphas"], w["beta"])
    omega = 2.0 / (1.0 + math.sin(math.pi / 65))
    rec = {"workload": "2D Poisson 5-point 64x64, SOR", "omega": omega, "rtol": 1e-8}
    for key, p in (("sweeps_sequential", (1, 1)), ("sweeps_4x4", (4, 4))):
        _, sweeps, _ = O.stationary_solve(2, n, p, diags, omega, w["f"], rtol=1e-8, maxit=20000)
        rec[key] = int(sweeps)
    rec["sweeps_rsor"] = lex_sweeps(n, diags, omega, w["f"], [(1, 1)])
    rec["sweeps_ssor"] = lex_sweeps(n, diags, omega, w["f"], [(1, 1), (-1, -1)])
    print(json.dumps(rec), flush=True)
    return rec


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    O.build(force=False)
    new = {}
    if which in ("sor64", "all"):
        new["poisson2d64_sor"] = run_sor64()
    if which in ("3d", "all"):
        new["poisson3d256"] = run("3D Poisson 7-point 256^3", synth.poisson_3d(n=256))
    name2 = "2D var-coef diffusion 2048x2048"
    if which in ("2d", "all"):
        new["varcoef2048"] = run(name2, synth.varcoef_2d(n=2048))
    if which in ("2d16", "all"):
        new["varcoef2048_p16"] = run(name2, synth.varcoef_2d(n=2048), p=(16, 16))
    if which in ("2dssor", "all"):
        new["varcoef2048_ssor"] = run(name2, synth.varcoef_2d(n=2048), kind="ssor")
    if which in ("2dssor16", "all"):
        new["varcoef2048_ssor_p16"] = run(name2, synth.varcoef_2d(n=2048), kind="ssor", p=(16, 16))
    # several runs may finish at once: merge under an exclusive lock
    with open(OUT + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        recs = json.load(open(OUT)) if os.path.exists(OUT) else {}
        recs.update(new)
        json.dump(recs, open(OUT, "w"), indent=1, sort_keys=True)
