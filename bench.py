"""Benchmark: preconditioned CG on the 2D variable-coefficient diffusion problem.

Workload (one step = one full solve on inputs resident in HBM): 2048x2048
interior grid, 5-point operator -div(alpha grad u) with cell coefficients
log-uniform in [1e-2, 1e2] (seed 2001) and harmonic face means, rhs U[-1,1]
(seed 2002), 16x16 subdomains, overlap 4, CG with the symmetric form of the
parallel ILU(0) preconditioner (SSOR with omega = 1 via --precond ssor) to
relative residual 1e-8, FP64.

Printed: one JSON line.  `value` is sweep Gpoints/s over the whole job:
interior points x half-sweeps executed / wall time of the timed steps.  The
roofline object is the decomposed sweep: the start-coupled forward
half-sweep, the sweep kernel with the largest share of the solve's kernel
time, timed with HIP events on the stream it runs on inside the timed
solves; the other three half-sweeps and the fused CG step are reported
beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SEQ_ITERS_FILE = os.path.join(ROOT, "tests", "golden", "sequential_iterations.json")


def sequential_iterations(key, iters, decomposed_key=None):
    """CG iterations of the sequential preconditioner (one subdomain) on the same input, from the CPU
    oracle's stored run, and the decomposed solve's count relative to it; with decomposed_key also the
    oracle's count for the same decomposition (FP64, same input)."""
    try:
        recs = json.load(open(SEQ_ITERS_FILE))
        rec = recs[key]
    except (OSError, ValueError, KeyError):
        return {"iterations_sequential": None}
    seq = rec["iterations"]
    out = {"iterations_sequential": seq, "iterations_vs_sequential": round(max(iters) / seq, 4),
           "sequential_source": "CPU FP64 oracle, one subdomain, same input (tests/golden/sequential_iterations.json)"}
    if decomposed_key and decomposed_key in recs:
        od = recs[decomposed_key]["iterations"]
        out.update({"iterations_oracle": od, "iterations_vs_oracle": max(iters) - od,
                    "oracle_source": "CPU FP64 oracle, the same decomposition and symmetric preconditioner, "
                                     "same input (tests/golden/sequential_iterations.json)"})
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--overlap", type=int, default=4)
    ap.add_argument("--precond", default="ilu0", choices=["ilu0", "ssor"])
    ap.add_argument("--prec", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=100000)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample-s", type=float, default=15.0)
    ap.add_argument("--workload", default="varcoef2048",
                    choices=["varcoef2048", "batch512", "serve", "poisson3d256", "poisson64", "sor2048"],
                    help="varcoef2048: one 2048^2 solve per step (default); batch512: 512 anisotropic problems "
                         "solved together per step; serve: a stream of Poisson arrivals through the server; "
                         "poisson3d256: the 3D solve; poisson64: the 64^2 stationary SOR solve; sor2048: "
                         "decomposed SOR sweeps on the 2048^2 operator")
    ap.add_argument("--sweeps", type=int, default=200, help="sor2048: sweeps per step")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--n3", type=int, default=256, help="poisson3d256: grid points per axis")
    ap.add_argument("--p3", type=int, default=8, help="poisson3d256: subdomains per axis")
    ap.add_argument("--prec3", default="f32", choices=["f32", "bf16"], help="poisson3d256: sweep precision")
    ap.add_argument("--no-fp64-reference", dest="fp64_reference", action="store_false",
                    help="poisson3d256: skip the plain FP64 GPU solve that the result is compared with")
    ap.add_argument("--plain-sample", type=int, default=24, help="batch512: problems solved one by one in FP64")
    ap.add_argument("--serve-count", type=int, default=400, help="serve: number of requests in the stream")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="serve: mean arrival rate (requests/s)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0, help="serve: admission budget (GiB of HBM)")
    ap.add_argument("--serve-precond", default="ssor", choices=["ilu0", "ssor"], help="serve: preconditioner")
    ap.add_argument("--serve-lanes3d", type=int, default=4, help="serve: 3D requests solved at once")
    ap.add_argument("--serve-plain-s", type=float, default=10.0,
                    help="serve: time spent solving a sample one by one with the plain FP64 solver")
    ap.add_argument("--roofline-only", action="store_true",
                    help="varcoef2048 and poisson3d256: only the timed half-sweeps of the roofline object and a "
                         "plain copy of 512 MiB (the reference for hardware byte counters); no solve")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1008_3699_amd as P
    import synth

    if args.workload == "batch512":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "poisson3d256":
        return bench_poisson3d(args)
    if args.workload == "poisson64":
        return bench_poisson64(args)
    if args.workload == "sor2048":
        return bench_sor2048(args)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    n, p = args.n, args.p
    w = synth.varcoef_2d(n=n)
    N = n * n
    al = torch.from_numpy(w["alphas"][0]).to(dev)
    f = torch.from_numpy(w["f"]).to(dev)
    g = P.Problem(2, (n, n))
    g.assemble([al, al], 0.0, args.prec)
    g.set_relaxation([1.0])
    g.set_decomposition((p, p), overlap=args.overlap, phase=0)
    g.precond_setup(args.precond)
    u = torch.zeros(N, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    if args.roofline_only:
        roofline = measure_roofline(g, N, args, stream)
        # a few CG iterations, so that counter runs also see the fused CG step
        u.zero_()
        g.solve("cg", args.precond, f, u, rtol=args.rtol, maxit=40, check=False)
        torch.cuda.synchronize()
        # reference for byte counters: one plain device copy of 512 MiB
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"roofline": roofline, "copy_bytes_each_way": src.numel() * 8}), flush=True)
        return

    def one_solve():
        u.zero_()
        return g.solve("cg", args.precond, f, u, rtol=args.rtol, maxit=args.maxit)

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    # the four half-sweeps and the fused CG step are timed with HIP events on their stream inside
    # the timed solves (every 8th launch of each)
    for which in range(5):
        g.pass_timing_enable(which, True)
    lat = []
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos.append(one_solve())
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    iters = [i["iters"] for i in infos]
    # half-sweeps per CG iteration with the symmetric preconditioner: 4, plus the initial application
    half_sweeps = sum(4 * (it + 1) for it in iters)
    value = N * half_sweeps / elapsed / 1e9

    live = {}
    for which in range(5):
        live[which] = g.pass_timing(which)
        g.pass_timing_enable(which, False)
    roofline = measure_roofline(g, N, args, stream, k_ms=live[0][0], k_n=live[0][1])
    passes = pass_table(N, args, live)
    roofline_cg = cg_step_roofline(N, args, *live[4])
    cpu = cpu_par = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, n, p, args.precond, args.cpu_sample_s)
        from oracle import oracle as O
        diags = O.assemble(2, (n, n), w["alphas"])
        pc = O.Precond(args.precond, 2, (n, n), (p, p), diags, omega=1.0)
        cpu_par = cpu_parallel(2, (n, n), (p, p), pc.dirs_f, diags, w["f"], args.cpu_sample_s, 40,
                               f"forward half-sweeps of the {args.precond} preconditioner ({p}x{p} subdomains)",
                               piv=pc.piv)

    rec = {
        "metric": "sweep Gpoints/s (whole job, PCG to 1e-8)",
        "value": round(value, 3),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"2D var-coef diffusion {n}x{n}, {p}x{p} subdomains, overlap {args.overlap}, "
                               f"{args.precond.upper()}-PCG (symmetric form) to {args.rtol:g}",
                   "n": n, "subdomains": [p, p], "overlap": args.overlap, "precond": args.precond},
        "solves_per_s": round(args.steps / elapsed, 4),
        "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
        "iterations": iters,
        "relres": [i["relres"] for i in infos],
        **(sequential_iterations({"ilu0": "varcoef2048", "ssor": "varcoef2048_ssor"}[args.precond], iters,
                                 {"ilu0": "varcoef2048_p16", "ssor": "varcoef2048_ssor_p16"}[args.precond])
           if n == 2048 and p == 16 else {}),
        "roofline": roofline,
        "roofline_passes": passes,
        "roofline_cg_step": roofline_cg,
        "cpu_baseline": cpu,
        "cpu_parallel": cpu_par,
    }
    print(json.dumps(rec), flush=True)


def pass_bytes(prec):
    """Algorithmic bytes per point of the four half-sweeps inside CG.  s = stored coefficient size,
    y = intermediate (sweep precision, FP64 or FP32).  Passes 0 and 2 read r (8), 1/Piv and two
    pre-divided couplings (3 s) and write y; passes 1 and 3 read y and two pre-scaled couplings (2 s)
    and write the FP64 piece of z (8)."""
    sz = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    y = 8 if prec == "f64" else 4
    return {0: 8 + 3 * sz + y, 1: y + 2 * sz + 8, 2: 8 + 3 * sz + y, 3: y + 2 * sz + 8}


PASS_NAMES = {0: "forward start-coupled (Piv - N1)^-1", 1: "backward start-coupled c (Piv - N2)^-1 Piv",
              2: "first transposed (Piv - N2)^-T, interior", 3: "second transposed c (Piv - N1)^-T Piv, interior"}


def pass_table(N, args, live):
    """Live duration and fraction of HBM peak of each half-sweep inside the timed solves."""
    bpp = pass_bytes(args.prec)
    out = []
    for which in range(4):
        ms, cnt = live[which]
        gbs = bpp[which] * N / (ms * 1e-3) / 1e9 if ms > 0 else None
        out.append({"pass": which, "what": PASS_NAMES[which], "bytes_per_point": bpp[which],
                    "kernel_ms": round(ms, 4), "timed_launches": cnt,
                    "achieved": round(gbs, 1) if gbs else None,
                    "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None})
    return out


def cg_step_roofline(N, args, c_ms, c_n):
    """The fused 2D CG step (k_cg_pq2d): p = z + beta p with z formed from its two pieces, the
    deferred x update, q = A p and the p.q partials.  Algorithmic bytes per point: z1, z2, old p,
    three diagonals (the operator is stored symmetric: a^P, a^E, a^N) and x read (56), new p, q and
    x written (24)."""
    bpp = 80
    alg = bpp * N
    achieved = alg / (c_ms * 1e-3) / 1e9
    traffic = None
    if args.prec == "f64" and args.n == 2048 and args.p == 16:
        traffic = measured_traffic(CG_TRAFFIC_FILE, CG_KERNEL_SRC)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_cg_pq2d<true,2,true> (fused CG step on symmetric storage: p update, x update, q = A p, p.q partials)",
            "kernel_ms": round(c_ms, 4), "timed_launches": c_n,
            "timing": "HIP events on the launching stream around every 8th fused step inside the timed solves",
            "bytes_per_point": bpp, "algorithmic_bytes": alg}


def bench_poisson64(args):
    """64x64 Poisson, 5-point, 4x4 subdomains, overlap 2, decomposed SOR at w = 2/(1+sin(pi/65)) to a
    relative residual of 1e-8 from u = 0 (residual tested after every sweep).  A launch-bound problem:
    one sweep is a right-hand-side kernel and a pipelined pass over 16 tiles of 16^2 points."""
    import math

    import numpy as np
    import torch

    import paper_1008_3699_amd as P
    import synth

    dev = torch.device("cuda:0")
    w = synth.poisson_2d_64()
    n = w["n"]
    N = n[0] * n[1]
    omega = 2.0 / (1.0 + math.sin(math.pi / 65))
    g = P.Problem(2, n)
    g.assemble([torch.from_numpy(a).to(dev) for a in w["alphas"]], 0.0, "f64")
    g.set_relaxation([omega])
    g.set_decomposition((4, 4), overlap=2, phase=0)
    f = torch.from_numpy(w["f"]).to(dev)
    u = torch.zeros(N, dtype=torch.float64, device=dev)

    def one():
        u.zero_()
        return g.solve("sor", "none", f, u, rtol=args.rtol, maxit=20000)

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    infos, lat = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos.append(one())
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
    elapsed = time.perf_counter() - t0
    sweeps = [i["iters"] for i in infos]
    # one sweep alone, back to back, with events on this stream
    x = torch.randn(N, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for k in range(8):
        g.sweep(k, x, f, y)
    e0.record()
    for k in range(400):
        g.sweep(k, x, f, y)
    e1.record()
    torch.cuda.synchronize()
    sweep_ms = e0.elapsed_time(e1) / 400
    seq = {}
    try:
        seq = json.load(open(SEQ_ITERS_FILE))["poisson2d64_sor"]
    except (OSError, ValueError, KeyError):
        pass
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        diags = O.assemble(2, n, w["alphas"])
        t1 = time.perf_counter()
        _, s_or, _ = O.stationary_solve(2, n, (4, 4), diags, omega, w["f"], rtol=args.rtol, maxit=20000)
        dt = time.perf_counter() - t1
        cpu = {"value": round(N * s_or / dt / 1e9, 5), "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole stationary solve ({s_or} decomposed sweeps, residual after each), "
                         "single-threaded C oracle", "sweeps": s_or, "solve_s": round(dt, 3)}
    bpp = 64
    rec = {
        "metric": "sweep Gpoints/s (whole job, stationary SOR to 1e-8)",
        "value": round(N * sum(sweeps) / elapsed / 1e9, 4), "unit": "Gpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D Poisson 5-point 64x64, 4x4 subdomains, overlap 2, decomposed SOR at "
                               f"w = 2/(1+sin(pi/65)) = {omega:.6f} to {args.rtol:g}", "n": 64, "subdomains": [4, 4],
                   "overlap": 2},
        "sweeps": sweeps,
        "relres": [i["relres"] for i in infos],
        "sweeps_sequential_fsor": seq.get("sweeps_sequential"), "sweeps_sequential_rsor": seq.get("sweeps_rsor"),
        "sweeps_sequential_ssor": seq.get("sweeps_ssor"), "sweeps_oracle_4x4": seq.get("sweeps_4x4"),
        "sequential_source": "CPU FP64 oracle on the same input (tests/golden/sequential_iterations.json): FSOR = "
                             "one subdomain with the alternating schedule, RSOR = row-wise from the SW corner, "
                             "SSOR = SW then NE",
        "roofline": {"bound": "hbm", "achieved": round(N * bpp / (sweep_ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(N * bpp / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 6),
                     "traffic": None, "kernel": "one decomposed sweep (k_sor_rhs2d + k_fast2d start-coupled pass)",
                     "kernel_ms": round(sweep_ms, 5), "timed_launches": 400, "bytes_per_point": bpp,
                     "timing": "events around 400 back-to-back sweeps after the timed solves; 4096 points, so the "
                               "two launches, not HBM, set the time",
                     "algorithmic_bytes": N * bpp},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def bench_sor2048(args):
    """Decomposed SOR sweeps (Gauss-Seidel, w = 1) on the 2048^2 variable-coefficient operator with 16x16
    subdomains: u_out = sweep(u_in) at successive schedule steps, ping-pong buffers, on inputs resident in
    HBM.  Algorithmic bytes per point: u_in, f, five diagonals, u_out = 64."""
    import torch

    import paper_1008_3699_amd as P
    import synth

    cpu_par = None
    dev = torch.device("cuda:0")
    n, p = args.n, args.p
    w = synth.varcoef_2d(n=n)
    N = n * n
    al = torch.from_numpy(w["alphas"][0]).to(dev)
    g = P.Problem(2, (n, n))
    g.assemble([al, al], 0.0, "f64")
    g.set_relaxation([1.0])
    g.set_decomposition((p, p), overlap=args.overlap, phase=0)
    f = torch.from_numpy(w["f"]).to(dev)
    ua = torch.zeros(N, dtype=torch.float64, device=dev)
    ub = torch.empty_like(ua)
    for k in range(8):
        g.sweep(k, ua, f, ub)
        ua, ub = ub, ua
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    it = 0
    for a, b in ev:
        a.record(stream)
        for _ in range(args.sweeps):
            g.sweep(it, ua, f, ub)
            ua, ub = ub, ua
            it += 1
        b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev])) / args.sweeps
    bpp = 64
    achieved = N * bpp / (ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        diags = O.assemble(2, (n, n), w["alphas"])
        u0 = np.zeros(N)
        t1 = time.perf_counter()
        k = 0
        while time.perf_counter() - t1 < args.cpu_sample_s:
            u0 = O.dsweep(2, (n, n), (p, p), O.schedule(2, (p, p), k, 0), diags, w["f"], uold=u0, omega=[1.0] * 4)
            k += 1
        dt = time.perf_counter() - t1
        cpu = {"value": round(N * k / dt / 1e9, 5), "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} decomposed sweeps on the full {n}x{n} grid ({p}x{p} subdomains), single-threaded C oracle"}
        cpu_par = cpu_parallel(2, (n, n), (p, p), O.schedule(2, (p, p), 0, 0), diags, w["f"], args.cpu_sample_s, 64,
                               f"decomposed SOR sweeps ({p}x{p} subdomains)", uold=np.zeros(N), omega=[1.0] * 4)
    rec = {
        "metric": "decomposed SOR sweep Gpoints/s",
        "value": round(N * args.sweeps * args.steps / elapsed / 1e9, 3), "unit": "Gpoints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"2D var-coef diffusion {n}x{n}, {p}x{p} subdomains, overlap {args.overlap}, "
                               f"{args.sweeps} decomposed SOR sweeps (w = 1) per step", "n": n, "subdomains": [p, p]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "one decomposed sweep: k_sor_rhs2d (f + (1/w-1) a^P u_old + N2 u_old, 48 B/pt moved) "
                               "then the start-coupled pipelined pass k_fast2d (40 B/pt)",
                     "kernel_ms": round(ms, 4), "timed_launches": args.sweeps * args.steps,
                     "timing": "HIP events on the launching stream around each step's sweeps",
                     "bytes_per_point": bpp, "algorithmic_bytes": N * bpp},
        "cpu_baseline": cpu,
        "cpu_parallel": cpu_par,
    }
    print(json.dumps(rec), flush=True)


def cg_iteration_bytes(dim, prec):
    """Algorithmic HBM bytes per point of one CG iteration with the symmetric preconditioner: the four
    half-sweeps (pass_bytes; 3D passes read three couplings), the operator product on symmetric
    storage (a^P and one coupling per axis, and p read, q written: dim + 3 FP64 values) and the
    vector work (r update with its norm, r.z, p update: about 13 FP64 values moved)."""
    pb = pass_bytes(prec)
    sz = {"f64": 8, "f32": 4, "bf16": 2}[prec]
    passes = sum(pb.values()) + (2 * sz if dim == 3 else 0)  # one more coupling per pass in 3D
    spmv = 8 * (dim + 3)
    return passes + spmv + 13 * 8


def oracle_solve_rate(items, budget_s, kind="ssor"):
    """The CPU FP64 oracle (single-threaded) solving the given problems in order until budget_s has
    passed: (solves, seconds, points)."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    done, pts = 0, 0
    for dim, n, alphas, f, p in items:
        diags = O.assemble(dim, n, alphas)
        pc = O.Precond(kind, dim, n, p, diags, omega=1.0)
        O.cg(lambda v: O.spmv(dim, n, diags, v), pc.apply_sym, f, rtol=1e-8, maxit=100000)
        done += 1
        pts += int(np.prod(n))
        if time.perf_counter() - t0 > budget_s:
            break
    return done, time.perf_counter() - t0, pts


def bench_batch(args):
    """512 independent anisotropic problems -(u_xx + eps u_yy), n ~ U{32..512}, SSOR(1)-PCG to 1e-8,
    FP64 CG with FP32 sweeps, all problems advanced together by the batched executor."""
    import numpy as np
    import torch

    import paper_1008_3699_amd as P
    import synth

    dev = torch.device("cuda:0")
    specs = synth.anisotropic_batch(count=args.batch_count)
    prec = "f32" if args.prec == "f64" else args.prec
    # autotuned tile side per size bucket (64-point buckets)
    side_of = {}
    for b in sorted({max(32, int(round(s["n"][0] / 64.0)) * 64) for s in specs}):
        pb, _ = P.autotune(2, (b, b), prec, "ssor")
        side_of[b] = max(2, b // pb[0])
    probs, fs, tiles = [], [], 0
    for s in specs:
        n = s["n"][0]
        side = side_of[max(32, int(round(n / 64.0)) * 64)]
        p = max(1, min(n // 2, -(-n // side)))
        g = P.Problem(2, (n, n))
        g.assemble([torch.from_numpy(a).to(dev) for a in s["alphas"]], 0.0, prec)
        g.set_relaxation([1.0])
        g.set_decomposition((p, p), overlap=2)
        g.precond_setup("ssor")
        probs.append(g)
        fs.append(torch.from_numpy(s["f"]).to(dev))
        tiles += p * p
    us = [torch.zeros_like(f) for f in fs]
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        for u in us:
            u.zero_()
        P.batch_solve(probs, fs, us, precond="ssor", rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = None
    for _ in range(args.steps):
        for u in us:
            u.zero_()
        infos = P.batch_solve(probs, fs, us, precond="ssor", rtol=args.rtol, maxit=args.maxit)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iters = np.array([i["iters"] for i in infos])
    Ns = np.array([s["n"][0] ** 2 for s in specs])
    half = float(np.sum(Ns * 4 * (iters + 1)))
    nconv = int(sum(i["converged"] for i in infos))
    # the plain solver: FP64 sweeps, one problem at a time, on a sample
    rng = np.random.default_rng(0)
    sample = rng.choice(len(specs), size=min(args.plain_sample, len(specs)), replace=False)
    t_plain, err = 0.0, []
    for k in sample:
        s = specs[k]
        n = s["n"][0]
        g = probs[k]
        h = P.Problem(2, (n, n))
        h.assemble([torch.from_numpy(a).to(dev) for a in s["alphas"]], 0.0, "f64")
        h.set_relaxation([1.0])
        side = side_of[max(32, int(round(n / 64.0)) * 64)]
        p = max(1, min(n // 2, -(-n // side)))
        h.set_decomposition((p, p), overlap=2)
        h.precond_setup("ssor")
        u = torch.zeros_like(fs[k])
        torch.cuda.synchronize()
        a = time.perf_counter()
        h.solve("cg", "ssor", fs[k], u, rtol=args.rtol, maxit=args.maxit)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - a
        err.append(float(torch.linalg.norm(us[k] - u) / torch.linalg.norm(u)))
    plain_rate = len(sample) / t_plain
    # the whole batched iteration against HBM: algorithmic bytes of every problem's iterations / time
    bit = cg_iteration_bytes(2, prec)
    moved = float(np.sum(Ns * (iters + 1))) * bit * args.steps
    gbs = moved / elapsed / 1e9
    rl = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
          "kernel": "the whole batched CG iteration (four batched passes, end faces, SpMV, dots, updates) "
                    "over all problems",
          "kernel_ms": round(1e3 * elapsed / args.steps, 3), "timed_launches": args.steps,
          "timing": "host clock around the timed batched solves", "bytes_per_point": bit,
          "bytes_per_point_note": f"{bit} B per point and CG iteration (FP32 sweeps, FP64 vectors)",
          "algorithmic_bytes": int(moved / args.steps)}
    cpu = None
    if not args.no_cpu:
        items = []
        for k in sample:
            sp = specs[k]
            n = sp["n"][0]
            side = side_of[max(32, int(round(n / 64.0)) * 64)]
            pp = max(1, min(n // 2, -(-n // side)))
            items.append((2, (n, n), sp["alphas"], sp["f"], (pp, pp)))
        done, dt, pts = oracle_solve_rate(items, args.cpu_sample_s, "ssor")
        cpu = {"value": round(done / dt, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} problems of the batch (the plain-solver sample, {pts} points) solved one by one "
                         "by the single-threaded FP64 oracle (SSOR(1)-CG, same decompositions)"}
    rec = {
        "metric": "batched PCG solves/s to 1e-8 (512 uneven 2D problems)",
        "value": round(args.steps * len(specs) / elapsed, 3),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": f"{len(specs)} anisotropic 2D problems -(u_xx + eps u_yy), n ~ U{{32..512}}, "
                               "eps log-uniform [1e-3,1], SSOR(1)-PCG to 1e-8, FP64 CG / FP32 sweeps, batched",
                   "total_points": int(Ns.sum()), "tiles": tiles, "tile_side_by_bucket": side_of},
        "sweep_gpoints_per_s": round(half / elapsed / 1e9, 3),
        "converged": nconv,
        "iterations_mean": float(iters.mean()), "iterations_max": int(iters.max()),
        "plain_fp64_sequential_solves_per_s": round(plain_rate, 3),
        "speedup_vs_plain": round(args.steps * len(specs) / elapsed / plain_rate, 2),
        "max_rel_diff_vs_plain_fp64": max(err),
        "roofline": rl, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def bench_serve(args):
    """A stream of Poisson arrivals (mixed 2D 64^2..1024^2 and 3D 32^3..128^3 variable-coefficient problems,
    coefficients log-uniform [1e-2,1e2]) served to 1e-8 by the continuously batched server."""
    import numpy as np
    import torch

    import paper_1008_3699_amd as P
    import synth

    dev = torch.device("cuda:0")
    prec = "f32" if args.prec == "f64" else args.prec
    reqs = synth.serving_stream(count=args.serve_count, rate=args.serve_rate)
    fields = [synth.request_fields(r) for r in reqs]
    # tile shapes for every 2D size bucket are tuned before the stream starts
    precond = args.serve_precond
    for b in sorted({max(32, ((r["n"][0] + 32) // 64) * 64) for r in reqs if r["dim"] == 2}):
        P.autotune(2, (b, b), prec, precond)
    torch.cuda.synchronize()
    budget = int(args.serve_budget_gib * (1 << 30))
    srv = P.Server(budget, prec=prec, precond=precond, rtol=args.rtol, maxit=args.maxit, lanes3d=args.serve_lanes3d)
    t0 = time.perf_counter()
    tickets = []
    for r, fl in zip(reqs, fields):
        wait = t0 + r["t"] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tickets.append(srv.submit(fl["dim"], fl["n"], fl["alphas"], fl["f"], fl["beta"]))
    t_sub = time.perf_counter() - t0
    out = []
    for k, t in enumerate(tickets):
        out.append(srv.poll(t, wait=True))
        if (k + 1) % 20 == 0:
            print(f"# {k + 1}/{len(tickets)} requests done", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    srv.close()
    lat = np.array([o[1]["t_total_ms"] for o in out])
    queue = np.array([o[1]["t_queue_ms"] for o in out])
    iters = np.array([o[1]["iters"] for o in out])
    dims = np.array([r["dim"] for r in reqs])
    nconv = int(sum(o[1]["converged"] for o in out))
    # the plain solver (FP64 sweeps, one request at a time, host-driven CG) on a sample, same decompositions
    rng = np.random.default_rng(0)
    order = rng.permutation(len(reqs))
    t_plain, n_plain, err = 0.0, 0, []
    for k in order:
        if t_plain > args.serve_plain_s:
            break
        fl = fields[k]
        dim, n = fl["dim"], fl["n"]
        g = P.Problem(dim, n)
        g.assemble([torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dev) for a in fl["alphas"]], 0.0)
        g.set_relaxation([1.0])
        if dim == 2:
            pp = tuple(max(1, min(v // 2, -(-v // 128))) for v in n)
        else:
            pp = tuple(max(1, min(v // 2, -(-v // 32))) for v in n)
        g.set_decomposition(pp, overlap=2)
        g.precond_setup(precond)
        f = torch.from_numpy(fl["f"]).to(dev)
        u = torch.zeros_like(f)
        torch.cuda.synchronize()
        a = time.perf_counter()
        g.solve("cg", precond, f, u, rtol=args.rtol, maxit=args.maxit)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - a
        n_plain += 1
        us = torch.from_numpy(out[k][0]).to(dev)
        err.append(float(torch.linalg.norm(us - u) / torch.linalg.norm(u)))
        g.close()
    rate = len(reqs) / elapsed
    moved = sum(int(np.prod(r["n"])) * (o[1]["iters"] + 1) * cg_iteration_bytes(r["dim"], prec)
                for r, o in zip(reqs, out))
    gbs = moved / elapsed / 1e9
    rl = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
          "kernel": "all served CG iterations (2D batch and 3D lanes together)",
          "kernel_ms": round(1e3 * elapsed, 1), "timed_launches": 1,
          "timing": "host clock from the first arrival to the last result",
          "bytes_per_point": cg_iteration_bytes(2, prec),
          "bytes_per_point_note": "per point and CG iteration: 2D as given, 3D " + str(cg_iteration_bytes(3, prec)),
          "algorithmic_bytes": int(moved)}
    cpu = None
    if not args.no_cpu:
        items = []
        for k in order:
            fl = fields[k]
            nn = fl["n"]
            pp = tuple(max(1, min(v // 2, -(-v // (128 if fl["dim"] == 2 else 32)))) for v in nn)
            items.append((fl["dim"], nn, fl["alphas"], fl["f"], pp))
        done, dt, pts = oracle_solve_rate(items, args.cpu_sample_s, precond)
        cpu = {"value": round(done / dt, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} requests of the stream ({pts} points) solved one by one by the single-threaded "
                         f"FP64 oracle ({precond.upper()}(1)-CG)"}
    rec = {
        "metric": "served PCG solves/s to 1e-8 with p50/p99 latency (Poisson arrivals)",
        "value": round(rate, 3),
        "unit": "solves/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * elapsed, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": f"{len(reqs)} requests, Poisson arrivals at {args.serve_rate:g}/s, 2D 5-point "
                               "64^2..1024^2 and 3D 7-point 32^3..128^3, coefficients log-uniform [1e-2,1e2], "
                               f"rhs U[-1,1], {precond.upper()}(1)-PCG to {args.rtol:g}, FP64 CG / {prec} sweeps",
                   "budget_gib": args.serve_budget_gib, "lanes3d": args.serve_lanes3d,
                   "requests_2d": int((dims == 2).sum()),
                   "requests_3d": int((dims == 3).sum())},
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "p50_ms_2d": round(float(np.percentile(lat[dims == 2], 50)), 2) if (dims == 2).any() else None,
        "p50_ms_3d": round(float(np.percentile(lat[dims == 3], 50)), 2) if (dims == 3).any() else None,
        "queue_p50_ms": round(float(np.percentile(queue, 50)), 2),
        "queue_p99_ms": round(float(np.percentile(queue, 99)), 2),
        "offered_rate": args.serve_rate, "arrival_window_s": round(t_sub, 3),
        "converged": nconv, "iterations_mean": float(iters.mean()),
        "plain_fp64_sequential_solves_per_s": round(n_plain / t_plain, 3) if t_plain > 0 else None,
        "plain_sample": n_plain,
        "max_rel_diff_vs_plain_fp64": max(err) if err else None,
        "capacity_note": ("queueing-dominated: the offered load exceeds what the GPU serves, so requests wait "
                          "for admission and latency grows with the stream"
                          if float(np.percentile(queue, 99)) > float(np.percentile(lat, 50))
                          else "stable: the 99th percentile of the admission wait stays below the median latency"),
        "roofline": rl, "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_fast2d_fwd_varcoef2048.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1008_3699_amd", "csrc", "psw_fast2d.hip")
CG_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_cg_pq2d_varcoef2048.json")
CG_KERNEL_SRC = os.path.join(ROOT, "paper_1008_3699_amd", "csrc", "psw_kernels.hip")


def measured_traffic(traffic_file=None, kernel_src=None):
    """HBM bytes per launch of the timed kernel from the committed counter runs, or None when the
    kernel source has changed since they were taken."""
    import hashlib
    traffic_file = traffic_file or TRAFFIC_FILE
    kernel_src = kernel_src or KERNEL_SRC
    try:
        rec = json.load(open(traffic_file))
        h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != h:
        return None
    return rec.get("hbm_bytes_per_launch")


def measure_roofline(g, N, args, stream, k_ms=None, k_n=None):
    """The decomposed sweep: the forward start-coupled half-sweep (pass 0), the sweep kernel with the
    largest share of the solve's kernel time.  k_ms: its mean duration from the library's HIP events
    around its launches inside the timed solves.  Without it (the --roofline-only run) the four passes
    run in turn as inside CG and pass 0 is timed the same way."""
    import torch
    how = "HIP events on the launching stream around every 8th pass-0 launch inside the timed solves"
    if k_ms is None:
        r = torch.randn(N, dtype=torch.float64, device=stream.device)
        y = torch.empty_like(r)
        g.pass_timing_enable(0, True)
        for k in range(8 * args.kernel_reps):
            for which in (0, 1, 2, 3):
                g.precond_half(args.precond, which, r, y)
        k_ms, k_n = g.pass_timing()
        g.pass_timing_enable(0, False)
        how = "HIP events around every 8th pass-0 launch, the four passes running in turn"
    else:
        # the same kernel is also timed back to back after the timed solves
        r = torch.randn(N, dtype=torch.float64, device=stream.device)
        y = torch.empty_like(r)
        for _ in range(4):
            g.precond_half(args.precond, 0, r, y)
        g.pass_timing_enable(0, True)
        for k in range(8 * args.kernel_reps):
            g.precond_half(args.precond, 0, r, y)
        a_ms, a_n = g.pass_timing()
        g.pass_timing_enable(0, False)
    bpp = pass_bytes(args.prec)[0]  # r + 1/Piv + 2 upstream couplings + y
    alg_bytes = bpp * N
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic() if (args.prec == "f64" and args.n == 2048 and args.p == 16) else None
    alone = {}
    if how.endswith("inside the timed solves"):
        alone = {"kernel_ms_alone": round(a_ms, 4), "timed_launches_alone": a_n,
                 "frac_alone": round(alg_bytes / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "timing_alone": "the same events around every 8th of back-to-back pass-0 launches after the timed solves"}
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_fast2d<2,double,...,SC=false,CPL=true> (forward start-coupled half-sweep)",
            "kernel_ms": round(k_ms, 4), "timed_launches": k_n, "timing": how, "bytes_per_point": bpp,
            "algorithmic_bytes": alg_bytes, **alone}


TRAFFIC3_FILE = os.path.join(ROOT, "profiles", "traffic_pass0_poisson3d256_f32.json")


def roofline3d(g, f, N, args):
    """The 3D forward start-coupled half-sweep (start-face kernel + LDS-tile interior kernel), timed with
    HIP events on the stream it runs on, standalone applications after the timed solves."""
    import numpy as np
    import torch
    y = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    reps = 20
    for _ in range(3):
        g.precond_half(args.precond, 0, f, y)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        g.precond_half(args.precond, 0, f, y)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    bpp = 8 + 16 + 8  # FP64 input, packed FP32 coefficients (1/Piv and three couplings), FP64 output
    if args.prec3 == "bf16":
        bpp = 8 + 8 + 8
    achieved = N * bpp / (ms * 1e-3) / 1e9
    traffic = None
    if args.prec3 == "f32" and args.n3 == 256 and args.p3 == 8 and args.precond == "ilu0":
        traffic = measured_traffic(TRAFFIC3_FILE, CG_KERNEL_SRC)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "3D forward start-coupled half-sweep: k_start_faces3g (coupled start faces) + k_tile3 (interior)",
            "kernel_ms": round(ms, 4), "timed_launches": reps,
            "timing": "HIP events on the launching stream around standalone pass-0 applications after the timed solves",
            "bytes_per_point": bpp, "algorithmic_bytes": N * bpp}


def bench_poisson3d(args):
    """3D Poisson, 7-point, n^3 grid (256^3), p^3 subdomains (8^3), overlap 2: FP64 CG with ILU(0) (or
    SSOR) sweeps in FP32 (FP32- or BF16-stored coefficients) to 1e-8."""
    import numpy as np
    import torch

    import paper_1008_3699_amd as P
    import synth

    cpu_par = None
    dev = torch.device("cuda:0")
    n, p = args.n3, args.p3
    w = synth.poisson_3d(n=n)
    N = n ** 3
    g = P.Problem(3, (n, n, n))
    g.assemble([torch.from_numpy(a).to(dev) for a in w["alphas"]], 0.0, args.prec3)
    g.set_relaxation([1.0])
    g.set_decomposition((p, p, p), overlap=2, phase=0)
    g.precond_setup(args.precond)
    f = torch.from_numpy(w["f"]).to(dev)
    u = torch.zeros(N, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    if args.roofline_only:
        roofline = roofline3d(g, f, N, args)
        # reference for byte counters: one plain device copy of 512 MiB
        src = torch.ones(64 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"roofline": roofline, "copy_bytes_each_way": src.numel() * 8}), flush=True)
        return

    def one_solve():
        u.zero_()
        return g.solve("cg", args.precond, f, u, rtol=args.rtol, maxit=args.maxit)

    for _ in range(args.warmup):
        one_solve()
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        infos.append(one_solve())
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
    elapsed = time.perf_counter() - t0
    iters = [i["iters"] for i in infos]
    value = N * sum(4 * (it + 1) for it in iters) / elapsed / 1e9

    roofline = roofline3d(g, f, N, args)
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        diags = O.assemble(3, (n, n, n), w["alphas"])
        pc = O.Precond(args.precond, 3, (n, n, n), (p, p, p), diags, omega=1.0)
        t1 = time.perf_counter()
        halves = 0
        while True:
            pc.forward(w["f"])
            halves += 1
            if time.perf_counter() - t1 > args.cpu_sample_s:
                break
        dt = time.perf_counter() - t1
        cpu = {"value": round(N * halves / dt / 1e9, 5), "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
               "sample": f"{halves} forward half-sweeps of the {args.precond} preconditioner on the full {n}^3 grid "
                         f"({p}^3 subdomains), single-threaded C oracle in FP64"}
        cpu_par = cpu_parallel(3, (n, n, n), (p, p, p), pc.dirs_f, diags, w["f"], args.cpu_sample_s, 48,
                               f"FP64 forward half-sweeps of the {args.precond} preconditioner ({p}^3 subdomains)",
                               piv=pc.piv)
    # the result against the plain FP64 GPU solver (FP64 sweeps, same decomposition and preconditioner)
    ref64 = None
    if args.fp64_reference:
        h = P.Problem(3, (n, n, n))
        h.assemble([torch.from_numpy(a).to(dev) for a in w["alphas"]], 0.0, "f64")
        h.set_relaxation([1.0])
        h.set_decomposition((p, p, p), overlap=2, phase=0)
        u64 = torch.zeros_like(u)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        i64 = h.solve("cg", args.precond, f, u64, rtol=args.rtol, maxit=args.maxit)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - a0
        err = float(torch.linalg.norm(u - u64) / torch.linalg.norm(u64))
        ref64 = {"rel_error_vs_fp64_solver": err, "fp64_iterations": i64["iters"], "fp64_relres": i64["relres"],
                 "fp64_solve_s": round(t64, 3),
                 "what": "||u - u64|| / ||u64||, u64 from the plain FP64 GPU solver (FP64 sweeps on the level "
                         "kernels, same decomposition and preconditioner, same tolerance); the FP64 oracle's error "
                         "is stated per result at 64^3 with the same 32^3 tiles in tests/test_gpu_precision.py"}
        h.close()
    rec = {
        "metric": "sweep Gpoints/s (whole job, PCG to 1e-8)",
        "value": round(value, 3),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec3,
        "data": "synthetic",
        "config": {"workload": f"3D Poisson 7-point {n}^3, {p}^3 subdomains, overlap 2, FP64 CG with "
                               f"{args.prec3.upper()} {args.precond.upper()} sweeps (symmetric form) to {args.rtol:g}",
                   "n": n, "subdomains": [p, p, p], "overlap": 2, "precond": args.precond},
        "solves_per_s": round(args.steps / elapsed, 4),
        "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
        "iterations": iters,
        "relres": [i["relres"] for i in infos],
        **(sequential_iterations("poisson3d256", iters) if n == 256 and args.precond == "ilu0" else {}),
        "error_vs_fp64": ref64,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_parallel": cpu_par,
    }
    print(json.dumps(rec), flush=True)


def host_info():
    """CPU model, logical CPUs of the host, and its STREAM triad bandwidth (all threads)."""
    import bench_cpu
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "omp_threads": bench_cpu.threads(),
            "host_triad_gbs": round(bench_cpu.triad_gbs(), 1)}


def cpu_parallel(dim, n, p, dirs, diags, f, budget_s, bytes_per_point, what, uold=None, piv=None, omega=None):
    """The decomposed sweep on all host cores (bench_cpu: OpenMP over subdomains), timed for about
    budget_s seconds on the full grid, with the host's triad bandwidth beside it."""
    import bench_cpu
    N = int(np.prod(n))
    bench_cpu.dsweep(dim, n, p, dirs, diags, f, uold=uold, piv=piv, omega=omega)  # warm-up
    t0 = time.perf_counter()
    k = 0
    while True:
        bench_cpu.dsweep(dim, n, p, dirs, diags, f, uold=uold, piv=piv, omega=omega)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    hi = host_info()
    gbs = N * bytes_per_point * k / dt / 1e9
    return {"value": round(N * k / dt / 1e9, 5), "unit": "Gpoints/s", "cores": hi["omp_threads"],
            "kind": "decomposed sweep on all host cores (OpenMP over subdomains, held to the oracle in tests)",
            "sample": f"{k} {what} on the full grid", "achieved_gbs": round(gbs, 2),
            "frac_of_host_triad": round(gbs / hi["host_triad_gbs"], 3) if hi["host_triad_gbs"] > 0 else None,
            **hi}


def cpu_baseline(w, n, p, kind, budget_s):
    """The CPU oracle timed on this host: preconditioner half-sweeps on the full grid."""
    import numpy as np

    from oracle import oracle as O
    diags = O.assemble(2, (n, n), w["alphas"])
    pc = O.Precond(kind, 2, (n, n), (p, p), diags, omega=1.0)
    r = w["f"]
    t0 = time.perf_counter()
    halves = 0
    while True:
        pc.forward(r)
        halves += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": round(n * n * halves / dt / 1e9, 5), "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"{halves} forward half-sweeps of the {kind} preconditioner on the full {n}x{n} grid "
                      f"({p}x{p} subdomains), single-threaded C oracle"}


if __name__ == "__main__":
    main()
