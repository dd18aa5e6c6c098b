"""Mixed precision (FP32 / BF16-stored sweeps inside FP64 CG) at the shapes the measurements run.

* The stored sweep-precision coefficients are the round-to-nearest-even
  conversions of the FP64 values, bit for bit (FP32 by NumPy's conversion,
  BF16 by an integer rounding of the FP64 bit pattern written here), on
  values chosen to hit ties, carries into the exponent and the inputs where
  rounding through FP32 first would round twice.
* 3D passes with 32^3 tiles (the tile the 256^3 measurement sweeps: 128 KB
  of LDS, 94 levels, full-size face records) against the FP64 oracle, every
  pass and the symmetric form; the forward pass and the symmetric form on the
  full 256^3 grid with 8x8x8 subdomains.
* The CG solution with FP32 / BF16 sweeps against the FP64 oracle's solution,
  ||u - u_oracle|| / ||u_oracle||, stated per result.
"""
import numpy as np
import pytest

import synth
from gpu_util import dev, make_problem, relmax, to_dev, to_np
from rounding import bf16_rne_bits
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def crafted_values(N, seed):
    """Positive values with hand-placed rounding cases at the front, log-uniform values after."""
    t = 2.0 ** -8  # half a BF16 unit in the last place at [1, 2)
    special = [
        1 + t,                 # tie between 1 and 1+2^-7: even is 1
        1 + 3 * t,             # tie between 1+2^-7 and 1+2^-6: even is 1+2^-6
        1 + t + 2.0 ** -30,    # just above a tie: up (rounding to FP32 first lands on the tie, then down)
        1 + 3 * t - 2.0 ** -30,  # just below a tie: down (through FP32 it would go up to even)
        2 - 2.0 ** -9,         # rounds up across the binade: 2.0
        1 + 2 * t - 2.0 ** -20,  # truncation gives 1, nearest gives 1+2^-7
        1.5 + t, 1.75 - 2.0 ** -40, 3 - 2.0 ** -8, 0.75 + 2.0 ** -10,
    ]
    g = synth.rng(seed)
    v = 10.0 ** g.uniform(-2, 2, N)
    v[:len(special)] = special
    v[len(special):2 * len(special)] = np.array(special) * 0.5  # the same cases one binade lower
    return v


@pytest.mark.parametrize("on_device", [0, 1])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_sweep_coefficients_round_to_nearest_even(prec, on_device):
    """psw_set_diagonals (host and device arrays), then the stored pivots and couplings of SSOR (w = 1:
    pivots = a^P exactly) and ILU(0) (pivots from psw_ilu_pivots in FP64) against RNE conversions."""
    import torch
    import paper_1008_3699_amd as P
    n, p = (48, 40), (3, 2)
    N = n[0] * n[1]
    off = [crafted_values(N, 100 + k) for k in range(4)]
    # a^P above the row sums keeps every ILU(0) pivot positive; its crafted values scaled by 16 (exact)
    diag_p = 16.0 * crafted_values(N, 99) + 450.0
    diags = [diag_p] + off
    g = P.Problem(2, n)
    if on_device:
        g.set_diagonals([to_dev(d) for d in diags], prec=prec)
    else:
        g.set_diagonals(diags, prec=prec)
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2)
    # the FP64 copy itself is exact
    out64 = torch.empty(N, dtype=torch.float64, device=dev())
    for k in range(5):
        g.get_diagonal(k, out64)
        assert np.array_equal(to_np(out64), diags[k])
    g.ilu_pivots(out64)
    piv_ilu = to_np(out64)
    ref_piv = O.ilu_pivots(2, n, p, O.schedule(2, p, 0), diags)
    assert relmax(piv_ilu, ref_piv) <= 1e-13
    for kind, piv in (("ssor", diag_p), ("ilu0", piv_ilu)):
        for k in range(5):
            src = piv if k == 0 else diags[k]
            if prec == "f32":
                out = torch.empty(N, dtype=torch.float32, device=dev())
                g.sweep_coefficients(kind, k, out)
                got = to_np(out)
                assert np.array_equal(got.view(np.uint32), src.astype(np.float32).view(np.uint32)), (kind, k)
            else:
                out = torch.empty(N, dtype=torch.int16, device=dev())
                g.sweep_coefficients(kind, k, out)
                got = to_np(out).view(np.uint16)
                ref = bf16_rne_bits(src)
                bad = np.nonzero(got != ref)[0]
                assert bad.size == 0, (kind, k, bad[:5], src[bad[:5]], got[bad[:5]], ref[bad[:5]])


def _poisson3d(n, seed):
    w = synth.poisson_3d(n=n, seed=seed)
    return w, O.assemble(3, w["n"], w["alphas"])


@pytest.mark.parametrize("prec,bound", [("f32", 2e-6), ("bf16", 2e-2)])
def test_tile3_passes_32cubed_tiles(prec, bound):
    """64^3 variable-coefficient grid, 2x2x2 subdomains: the 32^3 tiles of the 256^3 measurement.  All four
    passes and the symmetric form, SSOR and ILU(0), against the FP64 oracle (relative 2-norm)."""
    import torch
    dim, n, p = 3, (64, 64, 64), (2, 2, 2)
    pr = synth.random_small(4242, dim, n)
    diags = O.assemble(dim, n, pr["alphas"])
    g = make_problem(dim, n, pr["alphas"], prec=prec)
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2, phase=0)
    N = int(np.prod(n))
    out = torch.empty(N, dtype=torch.float64, device=dev())
    inputs = {0: pr["f"], 1: pr["u"], 2: pr["f"], 3: pr["u"]}
    for kind in ("ssor", "ilu0"):
        pc = O.Precond(kind, dim, n, p, diags, omega=1.0)
        refs = {
            0: pc.forward(pr["f"]),
            1: pc.backward(pr["u"]),
            2: O.dsolve_t(dim, n, p, pc.dirs_b, diags, pc.piv, pr["f"]),
            3: pc.c * O.dsolve_t(dim, n, p, pc.dirs_f, diags, pc.piv, pc.piv * pr["u"]),
        }
        for which in range(4):
            g.precond_half(kind, which, to_dev(inputs[which]), out)
            got = to_np(out)
            err = np.linalg.norm(got - refs[which]) / np.linalg.norm(refs[which])
            print(f"{prec} {kind} pass {which}: {err:.2e}", flush=True)
            assert err <= bound, (kind, which, err)
        for sym in (False, True):
            g.precond_apply(kind, to_dev(pr["f"]), out, symmetric=sym)
            ref = pc.apply_sym(pr["f"]) if sym else pc.apply(pr["f"])
            err = np.linalg.norm(to_np(out) - ref) / np.linalg.norm(ref)
            print(f"{prec} {kind} apply sym={sym}: {err:.2e}", flush=True)
            assert err <= bound, (kind, sym, err)


@pytest.mark.parametrize("prec,bound", [("f32", 2e-6), ("bf16", 2e-2)])
def test_full_size_poisson_256_forward_and_symmetric(prec, bound):
    """The 256^3 Poisson measurement at full size (8x8x8 subdomains of 32^3): the ILU(0) forward pass and
    the symmetric form against the FP64 oracle over every point."""
    import torch
    w, diags = _poisson3d(256, 3001)
    n, p = w["n"], (8, 8, 8)
    pc = O.Precond("ilu0", 3, n, p, diags, omega=1.0)
    g = make_problem(3, n, w["alphas"], prec=prec)
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2, phase=0)
    r = to_dev(w["f"])
    out = torch.empty_like(r)
    g.precond_half("ilu0", 0, r, out)
    y = pc.forward(w["f"])
    err = np.linalg.norm(to_np(out) - y) / np.linalg.norm(y)
    print(f"{prec} forward 256^3: {err:.2e}", flush=True)
    assert err <= bound
    g.precond_apply("ilu0", r, out, symmetric=True)
    z = pc.apply_sym(w["f"])
    err = np.linalg.norm(to_np(out) - z) / np.linalg.norm(z)
    print(f"{prec} symmetric 256^3: {err:.2e}", flush=True)
    assert err <= bound


@pytest.mark.parametrize("kind", ["ilu0", "ssor"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_cg_error_against_fp64_oracle_32cubed_tiles(prec, kind):
    """FP64 CG with FP32 / BF16-stored sweeps on 64^3 Poisson, 2x2x2 subdomains (32^3 tiles): the solution
    against the oracle's FP64 CG solution (same preconditioner in FP64, tolerance 1e-8).  Both reach a
    relative residual of 1e-8 and take the same number of iterations; the measured differences are 1e-12
    (FP32 ILU(0)) to 5e-9 (BF16 SSOR), and the test holds them to 1e-7."""
    import torch
    w, diags = _poisson3d(64, 3001)
    n, p = w["n"], (2, 2, 2)
    pc = O.Precond(kind, 3, n, p, diags, omega=1.0)
    x_or, it_or, rel_or = O.cg(lambda v: O.spmv(3, n, diags, v), pc.apply_sym, w["f"], rtol=1e-8)
    g = make_problem(3, n, w["alphas"], prec=prec)
    g.set_relaxation([1.0])
    g.set_decomposition(p, overlap=2, phase=0)
    u = torch.zeros(int(np.prod(n)), dtype=torch.float64, device=dev())
    info = g.solve("cg", kind, to_dev(w["f"]), u, rtol=1e-8, maxit=5000)
    x = to_np(u)
    err = np.linalg.norm(x - x_or) / np.linalg.norm(x_or)
    rel = np.linalg.norm(w["f"] - O.spmv(3, n, diags, x)) / np.linalg.norm(w["f"])
    print(f"{prec} {kind}: iters {info['iters']} (oracle FP64 {it_or}), true relres {rel:.2e}, "
          f"error vs FP64 oracle {err:.2e}", flush=True)
    assert info["converged"] and rel <= 1.05e-8
    assert abs(info["iters"] - it_or) <= max(2, 0.1 * it_or)
    assert err <= 1e-7
