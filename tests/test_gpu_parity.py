"""GPU parity: every kernel of libpsweep.so against the CPU FP64 oracle.

Bars: one FP64 sweep / half-sweep within 1e-12 (max abs error over max abs
value); ILU pivots and SpMV within 1e-13; iteration counts to tolerance
within 1 of the oracle's; FP32 / BF16 sweeps report their error against the
FP64 oracle and must stay inside the bounds below.
"""
import numpy as np
import pytest

import synth
from gpu_util import dev, make_problem, relmax, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SWEEP_CASES = [
    (2, (13, 11), (3, 2)), (2, (16, 16), (4, 4)), (2, (37, 29), (5, 3)), (2, (64, 40), (2, 5)),
    (2, (10, 9), (1, 1)), (2, (20, 8), (10, 4)),
    (3, (7, 6, 5), (2, 2, 2)), (3, (12, 9, 10), (3, 2, 4)), (3, (9, 9, 9), (1, 1, 1)), (3, (16, 8, 6), (4, 2, 3)),
]


def _prob(dim, n, seed=1):
    pr = synth.random_small(seed + sum(n), dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    return pr, diags


@pytest.mark.parametrize("dim,n", [(2, (33, 17)), (3, (9, 7, 5))])
def test_assemble(dim, n):
    pr, diags = _prob(dim, n)
    g = make_problem(dim, n, pr["alphas"])
    import torch
    out = torch.empty(int(np.prod(n)), dtype=torch.float64, device=dev())
    for k in range(2 * dim + 1):
        g.get_diagonal(k, out)
        assert relmax(to_np(out), diags[k]) <= 1e-14


@pytest.mark.parametrize("path", ["auto", "generic"])
@pytest.mark.parametrize("dim,n,p", SWEEP_CASES)
def test_stationary_sweep(dim, n, p, path):
    """Every schedule step, both phases, per-corner relaxation factors.  'auto' runs 2D sweeps as a
    right-hand-side kernel plus the pipelined start-coupled pass; 'generic' the level kernel."""
    pr, diags = _prob(dim, n)
    g = make_problem(dim, n, pr["alphas"])
    g.set_path(path)
    om = synth.rng(3).uniform(0.7, 1.9, 1 << dim)
    g.set_relaxation(list(om))
    import torch
    u = to_dev(pr["u"]); f = to_dev(pr["f"])
    out = torch.empty_like(u)
    for phase in (0, 1):
        g.set_decomposition(p, overlap=2, phase=phase)
        for k in range(1 << dim):
            g.sweep(k, u, f, out)
            ref = O.dsweep(dim, n, p, O.schedule(dim, p, k, phase), diags, pr["f"], uold=pr["u"], omega=om)
            err = relmax(to_np(out), ref)
            assert err <= 1e-12, (phase, k, err)


PRECOND_CASES = SWEEP_CASES + [(2, (300, 250), (3, 2)), (2, (130, 128), (1, 1)), (2, (256, 190), (4, 3))]


@pytest.mark.parametrize("dim,n,p", [(2, (37, 29), (5, 3)), (3, (12, 9, 10), (3, 2, 4))])
def test_overlap_changes_no_result(dim, n, p):
    """The exact-coupling sweep reads one layer beyond a subdomain (two across a coupled start face)
    whatever the overlap: the overlap, which only the restricted-overlap sweep uses, changes no value."""
    pr, diags = _prob(dim, n)
    g = make_problem(dim, n, pr["alphas"])
    g.set_relaxation([1.4])
    import torch
    u = to_dev(pr["u"]); f = to_dev(pr["f"])
    outs = []
    for o in (0, 1, 2, 5):
        g.set_decomposition(p, overlap=o, phase=0)
        out = torch.empty_like(u)
        g.sweep(1, u, f, out)
        outs.append(to_np(out))
    assert all(np.array_equal(outs[0], x) for x in outs[1:])
    ref = O.dsweep(dim, n, p, O.schedule(dim, p, 1, 0), diags, pr["f"], uold=pr["u"], omega=[1.4] * (1 << dim))
    assert relmax(outs[0], ref) <= 1e-12


@pytest.fixture(params=["auto", "generic"])
def path(request):
    """Kernel path of the preconditioner passes (psw_set_path): 'auto' takes the wavefront-pipelined
    2D passes and the 3D LDS-tile passes where they apply, 'generic' the level kernels."""
    return request.param


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
@pytest.mark.parametrize("dim,n,p", PRECOND_CASES)
def test_precond_half_sweeps_f64(kind, dim, n, p, path):
    pr, diags = _prob(dim, n, seed=5)
    g = make_problem(dim, n, pr["alphas"])
    g.set_path(path)  # FP64 3D passes run the level kernels on either path
    w = 1.3
    g.set_relaxation([w])
    g.set_decomposition(p, overlap=2, phase=0)
    pc = O.Precond(kind, dim, n, p, diags, omega=w)
    import torch
    r = to_dev(pr["f"]); out = torch.empty_like(r)
    y = pc.forward(pr["f"])
    refs = {
        0: y,
        1: pc.backward(pr["u"]),
        2: O.dsolve_t(dim, n, p, pc.dirs_b, diags, pc.piv, pr["f"]),
        3: pc.c * O.dsolve_t(dim, n, p, pc.dirs_f, diags, pc.piv, pc.piv * pr["u"]),
    }
    inputs = {0: pr["f"], 1: pr["u"], 2: pr["f"], 3: pr["u"]}
    for which in range(4):
        g.precond_half(kind, which, to_dev(inputs[which]), out)
        err = relmax(to_np(out), refs[which])
        assert err <= 1e-12, (which, err)
    z = torch.empty_like(r)
    g.precond_apply(kind, r, z, symmetric=False)
    assert relmax(to_np(z), pc.apply(pr["f"])) <= 1e-12
    g.precond_apply(kind, r, z, symmetric=True)
    assert relmax(to_np(z), pc.apply_sym(pr["f"])) <= 1e-12


@pytest.mark.parametrize("dim,n,p", SWEEP_CASES[:6] + SWEEP_CASES[6:8])
def test_ilu_pivots(dim, n, p):
    pr, diags = _prob(dim, n, seed=9)
    g = make_problem(dim, n, pr["alphas"])
    g.set_decomposition(p, overlap=2, phase=0)
    import torch
    out = torch.empty(int(np.prod(n)), dtype=torch.float64, device=dev())
    g.ilu_pivots(out)
    ref = O.ilu_pivots(dim, n, p, O.schedule(dim, p, 0), diags)
    assert relmax(to_np(out), ref) <= 1e-13


@pytest.mark.parametrize("dim,n", [(2, (50, 33)), (3, (11, 8, 13))])
def test_spmv_and_dot(dim, n):
    pr, diags = _prob(dim, n, seed=13)
    g = make_problem(dim, n, pr["alphas"])
    import torch
    x = to_dev(pr["u"]); y = torch.empty_like(x)
    g.spmv(x, y)
    assert relmax(to_np(y), O.spmv(dim, n, diags, pr["u"])) <= 1e-13
    d = g.dot(x, to_dev(pr["f"]))
    assert abs(d - pr["u"] @ pr["f"]) <= 1e-12 * np.abs(pr["u"]).sum()
    # deterministic: identical on repeat
    assert g.dot(x, to_dev(pr["f"])) == d


@pytest.mark.parametrize("prec,bound", [("f32", 1e-5), ("bf16", 3e-2)])
@pytest.mark.parametrize("dim,n,p", [(2, (40, 36), (4, 3)), (2, (260, 200), (2, 2)), (3, (12, 10, 9), (2, 2, 3))])
def test_precond_mixed_precision_error(prec, bound, dim, n, p, path):
    pr, diags = _prob(dim, n, seed=17)
    g = make_problem(dim, n, pr["alphas"], prec=prec)
    g.set_path(path)
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2, phase=0)
    import torch
    r = to_dev(pr["f"]); z = torch.empty_like(r)
    for kind in ("ssor", "ilu0"):
        pc = O.Precond(kind, dim, n, p, diags, omega=1.0)
        for sym in (False, True):
            g.precond_apply(kind, r, z, symmetric=sym)
            ref = pc.apply_sym(pr["f"]) if sym else pc.apply(pr["f"])
            err = np.linalg.norm(to_np(z) - ref) / np.linalg.norm(ref)
            assert err <= bound, (kind, sym, err)


TILE3_CASES = [((12, 10, 9), (2, 2, 3)), ((9, 9, 9), (1, 1, 1)), ((17, 13, 11), (3, 2, 2)), ((16, 8, 6), (4, 2, 3)),
               ((40, 32, 32), (2, 1, 1))]


@pytest.mark.parametrize("prec,bound", [("f32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("n,p", TILE3_CASES)
def test_tile3_half_sweeps(prec, bound, n, p):
    """3D passes with the whole tile in LDS (FP32 arithmetic): every pass against the FP64 oracle, and
    against the generic level kernels in the same precision.  Ragged tiles, a single tile, and tiles of
    20 x 32 x 32 points (the largest cross-section, 1024 pencils, that one workgroup holds)."""
    import torch
    dim = 3
    pr, diags = _prob(dim, n, seed=31)
    outs = {}
    for mode in ("tile", "generic"):
        g = make_problem(dim, n, pr["alphas"], prec=prec)
        g.set_path("auto" if mode == "tile" else "generic")
        g.set_relaxation([1.2])
        g.set_decomposition(p, overlap=2, phase=0)
        for kind in ("ssor", "ilu0"):
            out = torch.empty(int(np.prod(n)), dtype=torch.float64, device=dev())
            inputs = {0: pr["f"], 1: pr["u"], 2: pr["f"], 3: pr["u"]}
            for which in range(4):
                g.precond_half(kind, which, to_dev(inputs[which]), out)
                outs[(mode, kind, which)] = to_np(out)
            z = torch.empty_like(out)
            g.precond_apply(kind, to_dev(pr["f"]), z, symmetric=True)
            outs[(mode, kind, "sym")] = to_np(z)
    for kind in ("ssor", "ilu0"):
        pc = O.Precond(kind, dim, n, p, diags, omega=1.2)
        refs = {
            0: pc.forward(pr["f"]),
            1: pc.backward(pr["u"]),
            2: O.dsolve_t(dim, n, p, pc.dirs_b, diags, pc.piv, pr["f"]),
            3: pc.c * O.dsolve_t(dim, n, p, pc.dirs_f, diags, pc.piv, pc.piv * pr["u"]),
            "sym": pc.apply_sym(pr["f"]),
        }
        for which, ref in refs.items():
            a, b = outs[("tile", kind, which)], outs[("generic", kind, which)]
            err = np.linalg.norm(a - ref) / np.linalg.norm(ref)
            print(f"{kind} {which}: tile {err:.2e} generic {np.linalg.norm(b - ref) / np.linalg.norm(ref):.2e}", flush=True)
            assert err <= bound, (kind, which, err)
            assert np.linalg.norm(a - b) / np.linalg.norm(ref) <= 2 * bound, (kind, which)


def test_tile3_face_images_follow_updates():
    """The 3D face kernels read the coefficient part of their records from per-pass images written when
    the preconditioner is set up.  After a change of relaxation, decomposition or coefficients a reused
    problem must give, bit for bit, what a fresh problem with the new settings gives.  Tiles of 20 x 32 x 32
    and 10 x 32 x 32 points take the face kernels with gathered records (four waves per level)."""
    import torch
    dim, n = 3, (40, 32, 32)
    pa, _ = _prob(dim, n, seed=5)
    pb, _ = _prob(dim, n, seed=6)
    f = to_dev(pa["f"])

    def fresh(alphas, omega, p):
        g = make_problem(dim, n, alphas, prec="f32")
        g.set_relaxation([omega])
        g.set_decomposition(p, overlap=2, phase=0)
        return g

    def apply(g, kind):
        z = torch.empty_like(f)
        g.precond_apply(kind, f, z, symmetric=True)
        return to_np(z)

    g = fresh(pa["alphas"], 1.2, (2, 1, 1))
    for kind in ("ssor", "ilu0"):
        assert np.array_equal(apply(g, kind), apply(fresh(pa["alphas"], 1.2, (2, 1, 1)), kind)), kind
    g.set_relaxation([1.5])
    assert np.array_equal(apply(g, "ssor"), apply(fresh(pa["alphas"], 1.5, (2, 1, 1)), "ssor"))
    g.set_decomposition((4, 1, 1), overlap=2, phase=0)
    for kind in ("ssor", "ilu0"):
        assert np.array_equal(apply(g, kind), apply(fresh(pa["alphas"], 1.5, (4, 1, 1)), kind)), kind
    g.assemble([to_dev(a) for a in pb["alphas"]], 0.0, "f32")
    for kind in ("ssor", "ilu0"):
        assert np.array_equal(apply(g, kind), apply(fresh(pb["alphas"], 1.5, (4, 1, 1)), kind)), kind


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_cg_3d_tile_sweeps_two_pieces(prec):
    """3D CG with FP32 arithmetic sweeps on the LDS-tile passes (16^3 tiles: face levels in four waves),
    the transposed pair on the side stream and z kept in two pieces: converges to 1e-8 in the true
    residual, with the iteration count of the oracle's FP64 CG within 10 %."""
    import torch
    dim, n, p = 3, (32, 32, 32), (2, 2, 2)
    pr, diags = _prob(dim, n, seed=41)
    pc = O.Precond("ilu0", dim, n, p, diags, omega=1.0)
    _, it_ref, _ = O.cg(lambda v: O.spmv(dim, n, diags, v), pc.apply_sym, pr["f"], rtol=1e-8)
    g = make_problem(dim, n, pr["alphas"], prec=prec)
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2, phase=0)
    u = torch.zeros(int(np.prod(n)), dtype=torch.float64, device=dev())
    info = g.solve("cg", "ilu0", to_dev(pr["f"]), u, rtol=1e-8, maxit=2000)
    assert info["converged"] and info["relres"] <= 1.05e-8, info
    assert abs(info["iters"] - it_ref) <= max(2, 0.1 * it_ref), (info, it_ref)


def test_stationary_solve_poisson_64():
    """64x64 Poisson, 4x4 subdomains, omega = 2/(1+sin(pi/65)), relres 1e-8: sweeps within 1 of the oracle
    and within 10 % of sequential SOR."""
    w = synth.poisson_2d_64()
    n = w["n"]
    diags = O.assemble(2, n, w["alphas"])
    omega = 2.0 / (1.0 + np.sin(np.pi / 65))
    _, it_ref, _ = O.stationary_solve(2, n, (4, 4), diags, omega, w["f"], rtol=1e-8, maxit=5000)
    g = make_problem(2, n, w["alphas"])
    g.set_relaxation([omega])
    g.set_decomposition((4, 4), overlap=2)
    import torch
    u = torch.zeros(4096, dtype=torch.float64, device=dev())
    info = g.solve("sor", "none", to_dev(w["f"]), u, rtol=1e-8, maxit=5000)
    assert info["converged"] and abs(info["iters"] - it_ref) <= 1, (info, it_ref)
    # within 10 % of sequential SOR (one subdomain), whose count the oracle's stored run records
    import json
    import os
    seq = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sequential_iterations.json")))
    assert info["iters"] <= 1.10 * seq["poisson2d64_sor"]["sweeps_sequential"], (info, seq)


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
@pytest.mark.parametrize("dim,n,p", [(2, (48, 40), (4, 4)), (3, (12, 12, 10), (2, 3, 2))])
def test_krylov_iterations_match_oracle(kind, dim, n, p):
    pr, diags = _prob(dim, n, seed=21)
    Aop = lambda v: O.spmv(dim, n, diags, v)
    pc = O.Precond(kind, dim, n, p, diags, omega=1.0)
    xr, it_cg, _ = O.cg(Aop, pc.apply_sym, pr["f"], rtol=1e-8)
    _, it_gm, _ = O.fgmres(Aop, pc.apply, pr["f"], rtol=1e-8, restart=30)
    g = make_problem(dim, n, pr["alphas"])
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2)
    import torch
    N = int(np.prod(n))
    f = to_dev(pr["f"])
    u = torch.zeros(N, dtype=torch.float64, device=dev())
    info = g.solve("cg", kind, f, u, rtol=1e-8)
    assert info["converged"] and abs(info["iters"] - it_cg) <= 1, (info, it_cg)
    assert np.linalg.norm(to_np(u) - xr) <= 1e-6 * np.linalg.norm(xr)
    u.zero_()
    info = g.solve("fgmres", kind, f, u, rtol=1e-8, restart=30)
    assert info["converged"] and abs(info["iters"] - it_gm) <= 1, (info, it_gm)


@pytest.mark.parametrize("kind", ["none", "ssor", "ilu0"])
@pytest.mark.parametrize("n,p", [((300, 37), (3, 2)), ((260, 70), (2, 4))])
def test_cg_2d_ragged_strips_match_oracle(kind, n, p):
    """The fused 2D CG step works on strips of 16 rows by 256 columns: grids with a ragged last
    strip in both directions and more than one column band reach the oracle's iterate."""
    pr, diags = _prob(2, n, seed=21)
    Aop = lambda v: O.spmv(2, n, diags, v)
    if kind == "none":
        apply_m = lambda v: v.copy()
    else:
        apply_m = O.Precond(kind, 2, n, p, diags, omega=1.0).apply_sym
    xr, it_ref, _ = O.cg(Aop, apply_m, pr["f"], rtol=1e-8)
    g = make_problem(2, n, pr["alphas"])
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2)
    import torch
    f = to_dev(pr["f"])
    u = torch.zeros(int(np.prod(n)), dtype=torch.float64, device=dev())
    info = g.solve("cg", kind, f, u, rtol=1e-8)
    # unpreconditioned CG runs hundreds of steps; rounding order may move the stop by a few
    slack = 1 if kind != "none" else max(2, it_ref // 100)
    assert info["converged"] and abs(info["iters"] - it_ref) <= slack, (info, it_ref)
    assert info["relres"] <= 1e-8
    assert np.linalg.norm(to_np(u) - xr) <= 1e-6 * np.linalg.norm(xr)


@pytest.mark.parametrize("kind", ["ssor", "ilu0"])
def test_full_size_varcoef_2048_half_sweeps(kind):
    """The benchmark workload at full size: 2048^2, 16x16 subdomains, overlap 4; every output point."""
    w = synth.varcoef_2d(n=2048)
    n, p = (2048, 2048), (16, 16)
    diags = O.assemble(2, n, w["alphas"])
    pc = O.Precond(kind, 2, n, p, diags, omega=1.0)
    g = make_problem(2, n, w["alphas"])
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=4, phase=0)
    import torch
    r = to_dev(w["f"]); out = torch.empty_like(r)
    g.precond_half(kind, 0, r, out)
    y = pc.forward(w["f"])
    assert relmax(to_np(out), y) <= 1e-12
    g.precond_half(kind, 2, r, out)
    yt = O.dsolve_t(2, n, p, pc.dirs_b, diags, pc.piv, w["f"])
    assert relmax(to_np(out), yt) <= 1e-12
    # the two passes that take the intermediate (start-coupled backward, end-coupled second transposed)
    g.precond_half(kind, 1, to_dev(y), out)
    assert relmax(to_np(out), pc.backward(y)) <= 1e-12
    g.precond_half(kind, 3, to_dev(yt), out)
    assert relmax(to_np(out), pc.c * O.dsolve_t(2, n, p, pc.dirs_f, diags, pc.piv, pc.piv * yt)) <= 1e-12
    # the symmetric form the CG measurement applies
    g.precond_apply(kind, r, out, symmetric=True)
    assert relmax(to_np(out), pc.apply_sym(w["f"])) <= 1e-12


def test_full_size_varcoef_2048_stationary_sweeps():
    """The decomposed SOR sweep on the 2048^2 variable-coefficient operator, 16x16 subdomains, per-corner
    factors, all four directions of the cycle: every output point against the oracle.  With coefficients
    spanning 1e4 one coupling can carry almost all of a^P, so a sweep multiplies rounding errors by up to
    w per point along its direction; factors near 1 keep two correct roundings within 1e-12 (the small
    cases above take w up to 1.9 on milder coefficients)."""
    w = synth.varcoef_2d(n=2048)
    n, p = (2048, 2048), (16, 16)
    diags = O.assemble(2, n, w["alphas"])
    om = [1.2, 0.9, 1.1, 1.0]
    g = make_problem(2, n, w["alphas"])
    g.set_relaxation(om)
    g.set_decomposition(p, overlap=4, phase=0)
    import torch
    u0 = synth.rng(77).uniform(-1, 1, 2048 * 2048)
    u = to_dev(u0); f = to_dev(w["f"]); out = torch.empty_like(u)
    for k in range(4):
        g.sweep(k, u, f, out)
        ref = O.dsweep(2, n, p, O.schedule(2, p, k, 0), diags, w["f"], uold=u0, omega=om)
        err = relmax(to_np(out), ref)
        assert err <= 1e-12, (k, err)


def test_pass_timing_records_launches():
    """The measurement aid counts every 8th launch of the selected pass and reports a positive mean."""
    import torch
    n, p = (256, 192), (4, 3)
    pr, diags = _prob(2, n, seed=8)
    g = make_problem(2, n, pr["alphas"])
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2)
    g.precond_setup("ilu0")
    r = to_dev(pr["f"]); y = torch.empty_like(r)
    g.pass_timing_enable(0, True)
    for _ in range(17):
        g.precond_half("ilu0", 0, r, y)
        g.precond_half("ilu0", 1, r, y)
    ms, cnt = g.pass_timing()
    g.pass_timing_enable(0, False)
    assert cnt == 3 and ms > 0.0  # launches 0, 8 and 16 of pass 0
    # pass 1 and the fused CG step keep records of their own, timed in the same solve
    g.pass_timing_enable(1, True)
    g.pass_timing_enable(4, True)
    u = torch.zeros_like(r)
    info = g.solve("cg", "ilu0", r, u, rtol=1e-30, maxit=20, check=False)
    assert info["iters"] == 20
    ms1, n1 = g.pass_timing(1)
    ms4, n4 = g.pass_timing(4)
    g.pass_timing_enable(1, False)
    g.pass_timing_enable(4, False)
    assert n4 == 3 and ms4 > 0.0  # CG steps 0, 8 and 16
    assert n1 == 3 and ms1 > 0.0  # 21 backward passes (the first before the loop): 0, 8, 16
