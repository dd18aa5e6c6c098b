"""Python binding of libpsweep.so: parallel SOR / SSOR / ILU(0) sweeps on MI355X.

Argument marshalling only: every step runs in the HIP kernels of
``libpsweep.so`` (see ``include/psweep.h`` for the semantics of each call).
Vectors are torch CUDA float64 tensors with N = prod(n) elements, x fastest;
PyTorch provides device memory and the current stream.  There is no CPU
fallback: without the built library, or without a GPU, calls raise.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Problem", "Server", "PswError", "lib", "batch_solve", "autotune", "SSOR", "ILU0", "NONE",
           "STATIONARY", "CG", "FGMRES"]

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libpsweep.so")

SSOR, ILU0, NONE = 0, 1, 2
STATIONARY, CG, FGMRES = 0, 1, 2
_PREC = {"f64": 0, "f32": 1, "bf16": 2}
_KIND = {"ssor": SSOR, "ilu0": ILU0, "none": NONE}
_METHOD = {"sor": STATIONARY, "stationary": STATIONARY, "cg": CG, "fgmres": FGMRES, "sor_restricted": 3}


class PswError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("relres", ctypes.c_double), ("converged", ctypes.c_int),
                ("status", ctypes.c_int), ("t_total_ms", ctypes.c_double), ("t_precond_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libpsweep.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with `python -m paper_1008_3699_amd.build`")
        # torch first: its HIP runtime then satisfies the library's libamdhip64.so.7 dependency by soname.
        # Loaded the other way round, the process maps two HIP runtimes and torch's fails to find the GPU.
        import torch  # noqa: F401
        L = ctypes.CDLL(SO_PATH)
        vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        pp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "psw_problem_create": [ci, ctypes.POINTER(i64), ci, ctypes.POINTER(vp)],
            "psw_problem_destroy": [vp],
            "psw_set_diagonals": [vp, pp, ci, ci, vp],
            "psw_assemble_diffusion": [vp, pp, dbl, ci, vp],
            "psw_get_diagonal": [vp, ci, vp, vp],
            "psw_set_relaxation": [vp, ctypes.POINTER(dbl), ci],
            "psw_set_decomposition": [vp, ctypes.POINTER(ci), ci, ci],
            "psw_sweep": [vp, i64, vp, vp, vp, vp],
            "psw_precond_setup": [vp, ci, vp],
            "psw_precond_apply": [vp, ci, ci, vp, vp, vp],
            "psw_precond_half": [vp, ci, ci, vp, vp, vp],
            "psw_ilu_pivots": [vp, vp, vp],
            "psw_spmv": [vp, vp, vp, vp],
            "psw_dot": [vp, vp, vp, ctypes.POINTER(dbl), vp],
            "psw_solve": [vp, ci, ci, dbl, i64, ci, vp, vp, ctypes.POINTER(Info), vp],
            "psw_batch_solve": [ci, pp, pp, pp, ci, ci, dbl, i64, ctypes.POINTER(Info), vp],
            "psw_pass_timing_enable": [vp, ci, ci],
            "psw_pass_timing": [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
            "psw_pass_timing_of": [vp, ci, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
            "psw_set_path": [vp, ci],
            "psw_get_sweep_coefficients": [vp, ci, ci, vp, vp],
            "psw_problem_device_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
            "psw_precond_apply_noalloc": [vp, ci, vp, vp, vp],
            "psw_sweep_restricted": [vp, i64, vp, vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ci
        L.psw_status_string.argtypes = [ci]
        L.psw_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(st):
    try:
        return lib().psw_status_string(int(st)).decode()
    except Exception:  # library not loadable: report the raw code
        return str(st)


def _check(st, where):
    if st != 0:
        raise PswError(st, where)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, N, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != N:
        raise ValueError(f"{name} must be a contiguous float64 tensor of {N} elements")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """One structured n-diagonal problem on the current HIP device."""

    def __init__(self, dim, n):
        n = tuple(int(v) for v in n)
        assert len(n) == dim
        self.dim, self.n = dim, n
        self.N = 1
        for v in n:
            self.N *= v
        arr = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - dim)))
        h = ctypes.c_void_p()
        _check(lib().psw_problem_create(dim, arr, 2 * dim + 1, ctypes.byref(h)), "psw_problem_create")
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            lib().psw_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ---- set-up
    def set_diagonals(self, diags, prec="f64", stream=None):
        """Diagonals P,W,E,S,N(,B,F): CUDA float64 tensors (device copy) or numpy float64 arrays (host copy)."""
        import numpy as np
        if all(isinstance(d, np.ndarray) for d in diags):
            host = [np.ascontiguousarray(d, dtype=np.float64).reshape(-1) for d in diags]
            if any(h.size != self.N for h in host):
                raise ValueError(f"each diagonal needs {self.N} values")
            ptrs = (ctypes.c_void_p * 7)(*([h.ctypes.data for h in host] + [0] * (7 - len(host))))
            _check(lib().psw_set_diagonals(self._h, ptrs, 0, _PREC[prec], _stream(stream)), "psw_set_diagonals")
            return
        ptrs = (ctypes.c_void_p * 7)(*([_ptr(d, self.N, "diag").value for d in diags] + [0] * (7 - len(diags))))
        _check(lib().psw_set_diagonals(self._h, ptrs, 1, _PREC[prec], _stream(stream)), "psw_set_diagonals")

    def assemble(self, alphas, beta=0.0, prec="f64", stream=None):
        nn = 1
        for v in self.n:
            nn *= v + 2
        ptrs = (ctypes.c_void_p * 3)(*([_ptr(a, nn, "alpha").value for a in alphas] + [0] * (3 - len(alphas))))
        _check(lib().psw_assemble_diffusion(self._h, ptrs, float(beta), _PREC[prec], _stream(stream)),
               "psw_assemble_diffusion")

    def get_diagonal(self, k, out, stream=None):
        _check(lib().psw_get_diagonal(self._h, int(k), _ptr(out, self.N, "out"), _stream(stream)), "psw_get_diagonal")

    def set_relaxation(self, omega):
        om = list(omega) if hasattr(omega, "__len__") else [omega]
        arr = (ctypes.c_double * len(om))(*om)
        _check(lib().psw_set_relaxation(self._h, arr, len(om)), "psw_set_relaxation")

    def set_decomposition(self, p, overlap=2, phase=0):
        arr = (ctypes.c_int * 3)(*(list(p) + [1] * (3 - len(p))))
        _check(lib().psw_set_decomposition(self._h, arr, int(overlap), int(phase)), "psw_set_decomposition")

    def set_path(self, path):
        """'auto' (pipelined 2D / LDS-tile 3D passes where they apply) or 'generic' (level kernels)."""
        _check(lib().psw_set_path(self._h, {"auto": 0, "generic": 1}[path]), "psw_set_path")

    def sweep_coefficients(self, kind, k, out, stream=None):
        """Stored sweep-precision coefficients (k = 0 pivots, 1..2*dim couplings) into the CUDA tensor
        out (N elements of 8, 4 or 2 bytes: float64, float32, or int16 holding BF16 bits)."""
        import torch
        if not isinstance(out, torch.Tensor) or not out.is_cuda or not out.is_contiguous() or out.numel() != self.N:
            raise ValueError(f"out must be a contiguous CUDA tensor of {self.N} elements")
        _check(lib().psw_get_sweep_coefficients(self._h, _KIND[kind], int(k), ctypes.c_void_p(out.data_ptr()),
                                                _stream(stream)), "psw_get_sweep_coefficients")

    def device_bytes(self):
        b = ctypes.c_size_t()
        _check(lib().psw_problem_device_bytes(self._h, ctypes.byref(b)), "psw_problem_device_bytes")
        return b.value

    # ---- operations
    def sweep(self, iteration, u_in, f, u_out, stream=None):
        _check(lib().psw_sweep(self._h, int(iteration), _ptr(u_in, self.N, "u_in"), _ptr(f, self.N, "f"),
                               _ptr(u_out, self.N, "u_out"), _stream(stream)), "psw_sweep")

    def sweep_restricted(self, iteration, u_in, f, u_out, stream=None):
        """One restricted-overlap sweep (widened boxes of the decomposition's overlap)."""
        _check(lib().psw_sweep_restricted(self._h, int(iteration), _ptr(u_in, self.N, "u_in"), _ptr(f, self.N, "f"),
                                          _ptr(u_out, self.N, "u_out"), _stream(stream)), "psw_sweep_restricted")

    def precond_setup(self, kind, stream=None):
        _check(lib().psw_precond_setup(self._h, _KIND[kind], _stream(stream)), "psw_precond_setup")

    def precond_apply(self, kind, r, z, symmetric=False, stream=None):
        _check(lib().psw_precond_apply(self._h, _KIND[kind], int(bool(symmetric)), _ptr(r, self.N, "r"),
                                       _ptr(z, self.N, "z"), _stream(stream)), "psw_precond_apply")

    def precond_apply_noalloc(self, kind, r, z, stream=None):
        """z = M^-1 r (pair form) with the library's fixed scratch array; no device allocation."""
        _check(lib().psw_precond_apply_noalloc(self._h, _KIND[kind], _ptr(r, self.N, "r"), _ptr(z, self.N, "z"),
                                               _stream(stream)), "psw_precond_apply_noalloc")

    def precond_half(self, kind, which, inp, out, stream=None):
        _check(lib().psw_precond_half(self._h, _KIND[kind], int(which), _ptr(inp, self.N, "in"),
                                      _ptr(out, self.N, "out"), _stream(stream)), "psw_precond_half")

    def ilu_pivots(self, out, stream=None):
        _check(lib().psw_ilu_pivots(self._h, _ptr(out, self.N, "piv"), _stream(stream)), "psw_ilu_pivots")

    def spmv(self, x, y, stream=None):
        _check(lib().psw_spmv(self._h, _ptr(x, self.N, "x"), _ptr(y, self.N, "y"), _stream(stream)), "psw_spmv")

    def dot(self, x, y, stream=None):
        out = ctypes.c_double()
        _check(lib().psw_dot(self._h, _ptr(x, self.N, "x"), _ptr(y, self.N, "y"), ctypes.byref(out),
                             _stream(stream)), "psw_dot")
        return out.value

    def pass_timing_enable(self, which, enable=True):
        _check(lib().psw_pass_timing_enable(self._h, int(which), int(bool(enable))), "psw_pass_timing_enable")

    def pass_timing(self, which=None):
        """(mean ms, number of timed launches) of pass `which` (default: the one enabled last);
        which 0..3 are the pipelined 2D passes, 4 the fused 2D CG step."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        if which is None:
            _check(lib().psw_pass_timing(self._h, ctypes.byref(ms), ctypes.byref(n)), "psw_pass_timing")
        else:
            _check(lib().psw_pass_timing_of(self._h, int(which), ctypes.byref(ms), ctypes.byref(n)),
                   "psw_pass_timing_of")
        return ms.value, n.value

    def solve(self, method, precond, f, u, rtol=1e-8, maxit=100000, restart=30, stream=None, check=True):
        info = Info()
        st = lib().psw_solve(self._h, _METHOD[method], _KIND[precond], float(rtol), int(maxit), int(restart),
                             _ptr(f, self.N, "f"), _ptr(u, self.N, "u"), ctypes.byref(info), _stream(stream))
        if check and st not in (0, -4):
            raise PswError(st, "psw_solve")
        d = info.as_dict()
        d["status"] = st
        return d


def batch_solve(problems, fs, us, precond="ssor", rtol=1e-8, maxit=100000, method="cg", stream=None):
    """Solve several problems together (psw_batch_solve); returns a list of info dicts."""
    n = len(problems)
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
    fp = (ctypes.c_void_p * n)(*[_ptr(f, p.N, "f").value for f, p in zip(fs, problems)])
    up = (ctypes.c_void_p * n)(*[_ptr(u, p.N, "u").value for u, p in zip(us, problems)])
    infos = (Info * n)()
    st = lib().psw_batch_solve(n, hp, fp, up, _METHOD[method], _KIND[precond], float(rtol), int(maxit), infos,
                               _stream(stream))
    if st not in (0, -4):
        raise PswError(st, "psw_batch_solve")
    return [i.as_dict() for i in infos]


def autotune(dim, n, prec="f64", precond="ssor", stream=None):
    """Subdomain counts chosen by psw_autotune for a problem size; returns (p, us_per_problem)."""
    L = lib()
    L.psw_autotune.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    L.psw_autotune.restype = ctypes.c_int
    arr = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - len(n))))
    p = (ctypes.c_int * 3)()
    us = ctypes.c_double()
    _check(L.psw_autotune(dim, arr, _PREC[prec], _KIND[precond], p, ctypes.byref(us), _stream(stream)),
           "psw_autotune")
    return tuple(p[:dim]), us.value


class ServerOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("precond", ctypes.c_int), ("rtol", ctypes.c_double),
                ("maxit", ctypes.c_int64), ("epoch_iters", ctypes.c_int), ("max_active", ctypes.c_int),
                ("lanes3d", ctypes.c_int)]


class Server:
    """Continuously batched solver of independent diffusion problems (psw_server_*).

    Requests are host numpy arrays: per-axis node coefficients of (n+2)^dim
    values and a right-hand side of prod(n) values; results come back to the host.
    """

    def __init__(self, budget_bytes, prec="f32", precond="ilu0", rtol=1e-8, maxit=100000, epoch_iters=16,
                 max_active=1024, lanes3d=4):
        L = lib()
        vp = ctypes.c_void_p
        L.psw_server_create.argtypes = [ctypes.c_size_t, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        L.psw_server_submit.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.c_double, vp,
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.psw_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(Info), vp, ctypes.POINTER(ctypes.c_double)]
        L.psw_server_destroy.argtypes = [vp]
        L.psw_server_request_bytes.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_size_t)]
        for fn in (L.psw_server_create, L.psw_server_submit, L.psw_server_poll, L.psw_server_destroy,
                   L.psw_server_request_bytes):
            fn.restype = ctypes.c_int
        opts = ServerOpts(_PREC[prec], _KIND[precond], float(rtol), int(maxit), int(epoch_iters), int(max_active),
                          int(lanes3d))
        h = ctypes.c_void_p()
        _check(L.psw_server_create(int(budget_bytes), ctypes.byref(opts), ctypes.byref(h)), "psw_server_create")
        self._h = h
        self._size = {}

    def submit(self, dim, n, alphas, f, beta=0.0):
        """Queue one request; returns its ticket.  Raises PswError (PSW_EBUSY) if it can never fit."""
        import numpy as np
        n = tuple(int(v) for v in n)
        N = int(np.prod(n))
        nodes = int(np.prod([v + 2 for v in n]))
        al = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in alphas]
        fh = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if len(al) != dim or any(a.size != nodes for a in al) or fh.size != N:
            raise ValueError("alphas need (n+2)^dim values per axis and f prod(n) values")
        arr = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - dim)))
        ptrs = (ctypes.c_void_p * 3)(*([a.ctypes.data for a in al] + [0] * (3 - dim)))
        t = ctypes.c_uint64()
        _check(lib().psw_server_submit(self._h, dim, arr, ptrs, float(beta), ctypes.c_void_p(fh.ctypes.data),
                                       ctypes.byref(t)), "psw_server_submit")
        self._size[t.value] = N
        return t.value

    def request_bytes(self, dim, n):
        """Device bytes that admission reserves for a request of this shape."""
        arr = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - dim)))
        b = ctypes.c_size_t()
        _check(lib().psw_server_request_bytes(self._h, dim, arr, ctypes.byref(b)), "psw_server_request_bytes")
        return b.value

    def poll(self, ticket, wait=False):
        """None while the request runs; else (solution u as numpy, info dict with t_queue_ms)."""
        import numpy as np
        done = ctypes.c_int()
        info = Info()
        u = np.empty(self._size[ticket], dtype=np.float64)
        tq = ctypes.c_double()
        _check(lib().psw_server_poll(self._h, ticket, int(bool(wait)), ctypes.byref(done), ctypes.byref(info),
                                     ctypes.c_void_p(u.ctypes.data), ctypes.byref(tq)), "psw_server_poll")
        if not done.value:
            return None
        del self._size[ticket]
        d = info.as_dict()
        d["t_queue_ms"] = tq.value
        return u, d

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().psw_server_destroy(self._h), "psw_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
