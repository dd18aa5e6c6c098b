"""CPU FP64 oracle for the decomposed SOR / SSOR / ILU(0) sweeps (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code with the GPU library:
the arithmetic lives in ``psw_oracle.c`` (plain C, FP64, no contraction) and
in the plain NumPy drivers below.

Readings of the paper that this oracle fixes (R. Tavakoli, "Parallelizing
sequential sweeping on structured grids"):

* One decomposed sweep (Secs. 2-4): every point takes new values from the
  neighbours on the side where its own subdomain's sweep begins and old
  values from the other side; points on a start face whose neighbour subdomain
  also starts there are solved jointly (eqs. 1d:sorc, 2d:sor2b2, 2d:sor4b4,
  and the 3D 2x2 / 4x4 / 8x8 systems of Sec. 4).
* Direction schedule (Sec. 3, Sweeping directions; Sec. 4): base cycle for subdomain (0,0,0) --
  1D: +, -; 2D: (-,-), (+,+), (+,-), (-,+); 3D: the pairs (s,-s) for
  s = (-,-,-), (+,-,-), (-,+,-), (+,+,-); the sign on axis a flips for odd
  subdomain coordinate a.  ``phase`` swaps the two members of every pair.
* Relaxation factors are per start corner (Sec. 3, omega_SW, omega_NE, ...): corner
  index = sum of 2**a over axes a whose sweep starts at the high end.
* Preconditioners (Sec. 5; the paper never writes them out):
  SSOR:  z = (2-w) (D/w - N2)^-1 (D/w) (D/w - N1)^-1 r
  ILU(0): z = (D~ - N2)^-1 D~ (D~ - N1)^-1 r, with D~ from ``ilu_pivots``
  where N1 are the upstream couplings under the direction map d (schedule
  step 0) and N2 those under -d (so N1 + N2 = all off-diagonal couplings).
  The symmetric form used by CG is (M^-1 + M^-T)/2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psw_oracle.c")
_SO = os.path.join(_HERE, "libpsw_oracle.so")
_lib = None

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -6: "non-positive ILU pivot",
          -9: "singular coupled block"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile the C oracle into oracle/libpsw_oracle.so (plain gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        i64p = P(ctypes.c_int64)
        ip = P(ctypes.c_int)
        i8p = P(ctypes.c_int8)
        dpp = P(dp)
        L.or_partition.argtypes = [ctypes.c_int64, ctypes.c_int, i64p, i64p]
        L.or_schedule.argtypes = [ctypes.c_int, ip, ctypes.c_int64, ctypes.c_int, i8p]
        L.or_corner.argtypes = [ctypes.c_int, i8p]
        L.or_spmv.argtypes = [ctypes.c_int, i64p, dpp, dp, dp]
        L.or_assemble.argtypes = [ctypes.c_int, i64p, dpp, ctypes.c_double, dpp]
        L.or_sor_lex.argtypes = [ctypes.c_int, i64p, dpp, ctypes.c_double, i8p, dp, dp]
        L.or_dsweep.argtypes = [ctypes.c_int, i64p, ip, i8p, dpp, dp, dp, dp, dp, dp]
        L.or_dsolve_t.argtypes = [ctypes.c_int, i64p, ip, i8p, dpp, dp, dp, dp]
        L.or_ilu_pivots.argtypes = [ctypes.c_int, i64p, ip, i8p, dpp, dp]
        L.or_ras_sweep.argtypes = [ctypes.c_int, i64p, ip, i8p, dpp, dp, ctypes.c_int, dp, dp, dp]
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers
def _n3(dim, n):
    n = tuple(int(v) for v in (n if np.ndim(n) else [n] * dim))
    assert len(n) == dim
    return (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - dim)))


def _p3(dim, p):
    p = tuple(int(v) for v in (p if np.ndim(p) else [p] * dim))
    assert len(p) == dim
    return (ctypes.c_int * 3)(*(list(p) + [1] * (3 - dim)))


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _diag_pp(diags):
    arr = [np.ascontiguousarray(d, dtype=np.float64) for d in diags]
    pp = (ctypes.POINTER(ctypes.c_double) * len(arr))(*[_dptr(a) for a in arr])
    return pp, arr


def _check(st):
    if st != 0:
        raise OracleError(STATUS.get(st, str(st)))


def _flat(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))


def npoints(dim, n):
    return int(np.prod(n if np.ndim(n) else [n] * dim))


# ---------------------------------------------------------------- basic ops
def partition(n, p):
    lo = np.zeros(p, np.int64)
    hi = np.zeros(p, np.int64)
    _check(lib().or_partition(int(n), int(p), lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              hi.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return lo, hi


def schedule(dim, p, iteration, phase=0):
    """Per-subdomain direction signs, shape (nsub, 3) int8 (unused axes +1)."""
    pp = _p3(dim, p)
    nsub = pp[0] * pp[1] * pp[2]
    dirs = np.zeros((nsub, 3), np.int8)
    _check(lib().or_schedule(dim, pp, int(iteration), int(phase),
                             dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
    return dirs


def corner(dim, d):
    d = np.ascontiguousarray(np.asarray(list(d) + [1] * (3 - len(d)), np.int8))
    return lib().or_corner(dim, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))


def spmv(dim, n, diags, x):
    pp, keep = _diag_pp(diags)
    x = _flat(x)
    y = np.empty_like(x)
    _check(lib().or_spmv(dim, _n3(dim, n), pp, _dptr(x), _dptr(y)))
    return y


def assemble(dim, n, alphas, beta=0.0):
    """Diagonals [P, W, E, S, N, B, F][:2*dim+1] from per-axis node coefficients on (n+2)^dim nodes."""
    N = npoints(dim, n)
    al = [_flat(a) for a in alphas]
    app = (ctypes.POINTER(ctypes.c_double) * dim)(*[_dptr(a) for a in al])
    out = [np.zeros(N) for _ in range(2 * dim + 1)]
    opp = (ctypes.POINTER(ctypes.c_double) * len(out))(*[_dptr(a) for a in out])
    _check(lib().or_assemble(dim, _n3(dim, n), app, float(beta), opp))
    return out


def sor_lex(dim, n, diags, omega, d, f, u):
    """One lexicographic directional SOR sweep; returns the updated copy of u."""
    pp, keep = _diag_pp(diags)
    u = _flat(u).copy()
    f = _flat(f)
    dd = np.ascontiguousarray(np.asarray(list(d) + [1] * (3 - len(d)), np.int8))
    _check(lib().or_sor_lex(dim, _n3(dim, n), pp, float(omega),
                            dd.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), _dptr(f), _dptr(u)))
    return u


def dsweep(dim, n, p, dirs, diags, f, uold=None, piv=None, omega=None):
    """One decomposed sweep; see or_dsweep in psw_oracle.c."""
    pp, keep = _diag_pp(diags)
    f = _flat(f)
    uold = None if uold is None else _flat(uold)
    piv = None if piv is None else _flat(piv)
    om = None
    if omega is not None:
        om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega, np.float64).reshape(-1),
                                                  (1 << dim,)) if np.size(omega) == 1 else
                                  np.asarray(omega, np.float64))
        assert om.size == 1 << dim
    dirs = np.ascontiguousarray(dirs, np.int8)
    x = np.zeros_like(f)
    _check(lib().or_dsweep(dim, _n3(dim, n), _p3(dim, p), dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                           pp, _dptr(piv), _dptr(om), _dptr(uold), _dptr(f), _dptr(x)))
    return x


def _omega_corners(dim, omega):
    om = np.asarray(omega, np.float64).reshape(-1)
    return np.ascontiguousarray(np.broadcast_to(om, (1 << dim,)) if om.size == 1 else om)


def ras_sweep(dim, n, p, dirs, diags, f, uold, omega, overlap):
    """One restricted-overlap sweep (see or_ras_sweep in psw_oracle.c): each subdomain sweeps its box
    widened by `overlap` points, in its own direction, with old values outside; keeps its own points."""
    pp, keep = _diag_pp(diags)
    f = _flat(f)
    uold = _flat(uold)
    om = _omega_corners(dim, omega)
    assert om.size == 1 << dim
    dirs = np.ascontiguousarray(dirs, np.int8)
    x = np.empty_like(f)
    _check(lib().or_ras_sweep(dim, _n3(dim, n), _p3(dim, p), dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                              pp, _dptr(om), int(overlap), _dptr(uold), _dptr(f), _dptr(x)))
    return x


def dsolve_t(dim, n, p, dirs, diags, piv, b):
    """Solve (Piv - N)^T x = b for the upstream couplings N of the direction map dirs."""
    pp, keep = _diag_pp(diags)
    b = _flat(b)
    piv = None if piv is None else _flat(piv)
    dirs = np.ascontiguousarray(dirs, np.int8)
    x = np.zeros_like(b)
    _check(lib().or_dsolve_t(dim, _n3(dim, n), _p3(dim, p), dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                             pp, _dptr(piv), _dptr(b), _dptr(x)))
    return x


def ilu_pivots(dim, n, p, dirs, diags):
    pp, keep = _diag_pp(diags)
    N = npoints(dim, n)
    piv = np.zeros(N)
    dirs = np.ascontiguousarray(dirs, np.int8)
    _check(lib().or_ilu_pivots(dim, _n3(dim, n), _p3(dim, p), dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                               pp, _dptr(piv)))
    return piv


# ---------------------------------------------------------------- preconditioners
class Precond:
    """SSOR_par / ILU0_par of the paper's decomposition (direction map of schedule step 0)."""

    def __init__(self, kind, dim, n, p, diags, omega=1.0, phase=0):
        assert kind in ("ssor", "ilu0")
        self.kind, self.dim, self.n, self.p = kind, dim, n, p
        self.diags = [_flat(d) for d in diags]
        self.dirs_f = schedule(dim, p, 0, phase)
        self.dirs_b = (-self.dirs_f.astype(np.int16)).astype(np.int8)
        if kind == "ssor":
            self.piv = self.diags[0] / omega
            self.c = 2.0 - omega
        else:
            self.piv = ilu_pivots(dim, n, p, self.dirs_f, self.diags)
            self.c = 1.0

    def forward(self, r):
        """y = (Piv - N1)^-1 r (start-coupled, direction d)."""
        return dsweep(self.dim, self.n, self.p, self.dirs_f, self.diags, r, piv=self.piv)

    def backward(self, y):
        """z = c (Piv - N2)^-1 Piv y (start-coupled, direction -d)."""
        return self.c * dsweep(self.dim, self.n, self.p, self.dirs_b, self.diags, self.piv * y, piv=self.piv)

    def apply(self, r):
        return self.backward(self.forward(r))

    def apply_t(self, r):
        """M^-T r = c (Piv - N1)^-T Piv (Piv - N2)^-T r (end-coupled)."""
        y = dsolve_t(self.dim, self.n, self.p, self.dirs_b, self.diags, self.piv, r)
        return self.c * dsolve_t(self.dim, self.n, self.p, self.dirs_f, self.diags, self.piv, self.piv * y)

    def apply_sym(self, r):
        return 0.5 * (self.apply(r) + self.apply_t(r))


# ---------------------------------------------------------------- drivers
def stationary_solve(dim, n, p, diags, omega, f, rtol=1e-8, maxit=100000, phase=0, x0=None):
    """Repeat the decomposed sweep with the schedule; stop when ||f-Au||/||f|| <= rtol.

    Returns (u, sweeps, relres).  The residual is tested after every sweep.
    """
    f = _flat(f)
    u = np.zeros_like(f) if x0 is None else _flat(x0).copy()
    nf = np.linalg.norm(f)
    for k in range(maxit):
        dirs = schedule(dim, p, k, phase)
        u = dsweep(dim, n, p, dirs, diags, f, uold=u, omega=omega)
        rel = np.linalg.norm(f - spmv(dim, n, diags, u)) / nf
        if rel <= rtol:
            return u, k + 1, rel
    return u, maxit, rel


def ras_solve(dim, n, p, diags, omega, f, overlap, rtol=1e-8, maxit=100000, phase=0):
    """Repeat the restricted-overlap sweep with the schedule; stop when ||f-Au||/||f|| <= rtol.
    Returns (u, sweeps, relres)."""
    f = _flat(f)
    u = np.zeros_like(f)
    nf = np.linalg.norm(f)
    rel = 1.0
    for k in range(maxit):
        u = ras_sweep(dim, n, p, schedule(dim, p, k, phase), diags, f, u, omega, overlap)
        rel = np.linalg.norm(f - spmv(dim, n, diags, u)) / nf
        if rel <= rtol:
            return u, k + 1, rel
    return u, maxit, rel


def cg(apply_a, apply_m, f, rtol=1e-8, maxit=10000, flexible=False):
    """Preconditioned CG from x0 = 0; stops on the recurrence residual.  Returns (x, iters, relres_true)."""
    f = _flat(f)
    x = np.zeros_like(f)
    r = f.copy()
    nf = np.linalg.norm(f)
    z = apply_m(r)
    pvec = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = apply_a(pvec)
        pq = pvec @ q
        if not pq > 0:
            raise OracleError("CG breakdown (p.Ap <= 0)")
        alpha = rz / pq
        x += alpha * pvec
        r_old = r
        r = r - alpha * q
        it += 1
        if np.linalg.norm(r) / nf <= rtol:
            break
        z_old = z
        z = apply_m(r)
        rz_new = r @ z
        beta = ((r - r_old) @ z) / rz if flexible else rz_new / rz
        pvec = z + beta * pvec
        rz = rz_new
    true = np.linalg.norm(f - apply_a(x)) / nf
    return x, it, true


def fgmres(apply_a, apply_m, f, rtol=1e-8, maxit=10000, restart=50):
    """Right-preconditioned flexible GMRES(m) from x0 = 0.  Returns (x, iters, relres_true)."""
    f = _flat(f)
    N = f.size
    x = np.zeros(N)
    nf = np.linalg.norm(f)
    it = 0
    while it < maxit:
        r = f - apply_a(x)
        beta = np.linalg.norm(r)
        if beta / nf <= rtol:
            break
        m = restart
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(m):
            Z[k] = apply_m(V[k])
            w = apply_a(Z[k])
            for i in range(k + 1):
                H[i, k] = w @ V[i]
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] > 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):
                t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_used = k + 1
            if abs(g[k + 1]) / nf <= rtol or it >= maxit:
                break
        yk = np.zeros(k_used)
        for i in range(k_used - 1, -1, -1):
            yk[i] = (g[i] - H[i, i + 1:k_used] @ yk[i + 1:k_used]) / H[i, i]
        x = x + yk @ Z[:k_used]
        if abs(g[k_used]) / nf <= rtol:
            break
    true = np.linalg.norm(f - apply_a(x)) / nf
    return x, it, true


# ---------------------------------------------------------------- paper model problem
def model_problem(dim, N):
    """Laplace model problem of Sec. 8: u = prod x_i on the boundary of [0,1]^d.

    N points per axis including both boundary points, h = 1/(N-1); unit-spaced
    coefficients (a^X = 1, a^P = 2d); Dirichlet data folded into f.
    Returns (n, diags, f, u_exact).
    """
    n = N - 2
    h = 1.0 / (N - 1)
    shape = (n,) * dim
    Ni = n ** dim
    diags = [np.full(Ni, 2.0 * dim)] + [np.ones(Ni) for _ in range(2 * dim)]
    xs = np.arange(1, N - 1) * h
    grids = np.meshgrid(*([xs] * dim), indexing="ij")  # grids[a][i0,...] = coordinate a
    u_exact = np.ones(shape)
    for a in range(dim):
        u_exact = u_exact * grids[a]
    # point index x + n*(y + n*z): array axis order (z, y, x) for the flat layout
    u_exact = np.transpose(u_exact).reshape(-1).copy()
    f = np.zeros(Ni)
    idx = np.arange(Ni)
    coords = [(idx // n ** a) % n for a in range(dim)]
    for a in range(dim):
        for side, bval in ((-1, 0.0), (+1, 1.0)):
            edge = coords[a] == (0 if side < 0 else n - 1)
            # boundary neighbour value: product of coordinates with axis a at 0 or 1
            val = np.full(Ni, bval)
            for b in range(dim):
                if b != a:
                    val = val * ((coords[b] + 1) * h)
            f[edge] += val[edge]
    return n, diags, f, u_exact


L1_NORM = {1: lambda N: N, 2: lambda N: 3.0 * N * N, 3: lambda N: float(N) ** 3}


def l1_error(dim, N, u, u_exact):
    """L1 error as tabulated in Sec. 8 (normalisation decoded: N, 3N^2, N^3 in 1D/2D/3D)."""
    return np.abs(u - u_exact).sum() / L1_NORM[dim](N)


def model_run(dim, N, directions, omegas, tol, maxit=200000):
    """Sequential sweeps on the model problem: sweep k uses directions[k % len] with omegas[k % len].

    Returns (iterations, l1_error) at the first sweep whose L1 error is below tol.
    """
    n, diags, f, ue = model_problem(dim, N)
    u = np.zeros_like(f)
    for k in range(maxit):
        j = k % len(directions)
        u = sor_lex(dim, [n] * dim, diags, omegas[j], directions[j], f, u)
        e = l1_error(dim, N, u, ue)
        if e < tol:
            return k + 1, e
    return maxit, e
