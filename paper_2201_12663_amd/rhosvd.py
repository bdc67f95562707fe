"""ctypes binding of librhosvd.so (include/rhosvd.h).

Argument marshalling only: every step of the reduction runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  The library must be
built (python -m paper_2201_12663_amd.build); nothing here falls back to another
implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librhosvd.so")

FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
PHASES = ["norms", "anorm", "gram", "eig", "trunc_z", "project", "core"]

STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_NONFINITE", -3: "ERR_ALLOC", -4: "ERR_DEVICE",
          -5: "ERR_NOCONV", -6: "ERR_STATE", -7: "ERR_UNSUPPORTED"}

# every symbol include/rhosvd.h declares
EXPORTS = ["rhosvd_create", "rhosvd_destroy", "rhosvd_set_options", "rhosvd_reduce", "rhosvd_get",
           "rhosvd_get_xi", "rhosvd_get_spectrum", "rhosvd_get_v", "rhosvd_phase_ms",
           "rhosvd_last_error", "rhosvd_version"]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_eig_sweeps", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class Report(ctypes.Structure):
    _fields_ = [("xi_norm", ctypes.c_double), ("a_norm", ctypes.c_double), ("tau", ctypes.c_double),
                ("bound", ctypes.c_double), ("tail", ctypes.c_double * 3), ("ranks", ctypes.c_int32 * 3),
                ("m", ctypes.c_int32), ("eig_sweeps", ctypes.c_int32), ("dropped", ctypes.c_int32)]


class RhosvdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load librhosvd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2201_12663_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.rhosvd_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(Options)]
        lib.rhosvd_destroy.argtypes = [vp]
        lib.rhosvd_set_options.argtypes = [vp, ctypes.POINTER(Options)]
        lib.rhosvd_reduce.argtypes = [vp, i64, i64, vp, vp, vp, vp, dbl, ctypes.POINTER(i32)]
        lib.rhosvd_get.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(Report)]
        lib.rhosvd_get_xi.argtypes = [vp, vp]
        lib.rhosvd_get_spectrum.argtypes = [vp, i32, vp]
        lib.rhosvd_get_v.argtypes = [vp, i32, vp]
        lib.rhosvd_phase_ms.argtypes = [vp, i32]
        lib.rhosvd_phase_ms.restype = dbl
        lib.rhosvd_last_error.argtypes = [vp]
        lib.rhosvd_last_error.restype = ctypes.c_char_p
        lib.rhosvd_version.restype = ctypes.c_char_p
        for f in ("rhosvd_create", "rhosvd_destroy", "rhosvd_set_options", "rhosvd_reduce", "rhosvd_get",
                  "rhosvd_get_xi", "rhosvd_get_spectrum", "rhosvd_get_v"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _colmajor(t, name):
    """Pointer of an (n, R) column-major float64 CUDA tensor."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2):
        raise ValueError(f"{name}: expected a 2-D float64 CUDA tensor")
    n = t.shape[0]
    if t.stride(0) != 1 or (t.shape[1] > 1 and t.stride(1) != n):
        raise ValueError(f"{name}: expected column-major layout (strides (1, n))")
    return ctypes.c_void_p(t.data_ptr())


def to_device(U, device="cuda"):
    """numpy (n, R) array -> column-major float64 CUDA tensor."""
    import numpy as np
    import torch
    t = torch.from_numpy(np.asfortranarray(U, dtype=np.float64))
    out = torch.empty((t.shape[1], t.shape[0]), dtype=torch.float64, device=device).t()
    out.copy_(t)
    return out


def colmajor_empty(rows, cols, device="cuda"):
    import torch
    return torch.empty((cols, rows), dtype=torch.float64, device=device).t()


@dataclass
class Result:
    ranks: tuple
    Z: list            # (n, r_l) column-major float64 tensors
    beta: object       # (r1, r2, r3) Fortran-ordered float64 tensor (or None)
    sigma: object      # (r1 + r2 + r3,) float64 tensor
    report: dict


class Reducer:
    """One library handle bound to a stream."""

    def __init__(self, precision="fp64", stream=None, max_eig_sweeps=0, profile=False):
        import torch
        self.lib = load()
        self.opt = Options()
        self.opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.opt.max_eig_sweeps = int(max_eig_sweeps)
        self.opt.profile = 1 if profile else 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.h = ctypes.c_void_p()
        s = self.lib.rhosvd_create(ctypes.byref(self.h), ctypes.c_void_p(stream.cuda_stream),
                                   ctypes.byref(self.opt))
        if s != 0:
            raise RhosvdError(s, self.lib.rhosvd_last_error(None).decode())
        self.n = self.R = 0
        self.ranks = (0, 0, 0)

    def close(self):
        if self.h:
            self.lib.rhosvd_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s):
        if s != 0:
            raise RhosvdError(s, self.lib.rhosvd_last_error(self.h).decode())

    def set_precision(self, precision):
        self.opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._check(self.lib.rhosvd_set_options(self.h, ctypes.byref(self.opt)))

    def reduce(self, U1, U2, U3, xi, eps):
        import torch
        if not (xi.is_cuda and xi.dtype == torch.float64 and xi.is_contiguous()):
            raise ValueError("xi: expected a contiguous float64 CUDA tensor")
        n, R = U1.shape
        for U in (U2, U3):
            if tuple(U.shape) != (n, R):
                raise ValueError("side matrices must share the shape (n, R)")
        ranks = (ctypes.c_int32 * 3)()
        self._check(self.lib.rhosvd_reduce(self.h, n, R, _colmajor(U1, "U1"), _colmajor(U2, "U2"),
                                           _colmajor(U3, "U3"), ctypes.c_void_p(xi.data_ptr()),
                                           float(eps), ranks))
        self.n, self.R = n, R
        self.ranks = tuple(int(r) for r in ranks)
        return self.ranks

    def get(self, beta=True, Z=True, sigma=True, beta_out=None):
        """Core and copy-out for the last reduce (enqueued on the stream)."""
        import torch
        r1, r2, r3 = self.ranks
        dev = "cuda"
        Zs = [colmajor_empty(self.n, r, dev) for r in self.ranks] if Z else [None] * 3
        b = None
        if beta:
            if beta_out is not None:
                if beta_out.numel() < r1 * r2 * r3 or beta_out.dtype != torch.float64:
                    raise ValueError("beta_out too small or not float64")
                flat = beta_out
            else:
                flat = torch.empty(r1 * r2 * r3, dtype=torch.float64, device=dev)
            b = flat[: r1 * r2 * r3]
        sig = torch.empty(r1 + r2 + r3, dtype=torch.float64, device=dev) if sigma else None
        rep = Report()
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p()
        self._check(self.lib.rhosvd_get(self.h, ptr(Zs[0]), ptr(Zs[1]), ptr(Zs[2]), ptr(b), ptr(sig),
                                        ctypes.byref(rep)))
        report = dict(xi_norm=rep.xi_norm, a_norm=rep.a_norm, tau=rep.tau, bound=rep.bound,
                      tail=list(rep.tail), ranks=list(rep.ranks), m=rep.m, eig_sweeps=rep.eig_sweeps,
                      dropped=rep.dropped)
        beta_t = None
        if b is not None:
            beta_t = b.view(r3, r2, r1).permute(2, 1, 0) if b.numel() > 0 else b.view(r1, r2, r3)
        return Result(self.ranks, Zs, beta_t, sig, report)

    def core_only(self, beta_flat):
        """Enqueue only the core contraction into beta_flat (for timing loops)."""
        self._check(self.lib.rhosvd_get(self.h, None, None, None, ctypes.c_void_p(beta_flat.data_ptr()),
                                        None, None))

    def xi_prime(self):
        import torch
        out = torch.empty(self.R, dtype=torch.float64, device="cuda")
        self._check(self.lib.rhosvd_get_xi(self.h, ctypes.c_void_p(out.data_ptr())))
        return out

    def spectrum(self, l):
        import torch
        out = torch.empty(min(self.n, self.R), dtype=torch.float64, device="cuda")
        self._check(self.lib.rhosvd_get_spectrum(self.h, int(l), ctypes.c_void_p(out.data_ptr())))
        return out

    def V(self, l):
        out = colmajor_empty(self.ranks[l], self.R)
        if out.numel():
            self._check(self.lib.rhosvd_get_v(self.h, int(l), ctypes.c_void_p(out.data_ptr())))
        return out

    def phase_ms(self):
        return {name: float(self.lib.rhosvd_phase_ms(self.h, i)) for i, name in enumerate(PHASES)}


def reduce(U1, U2, U3, xi, eps, precision="fp64", **kw):
    """One-shot reduction: returns Result (ranks, Z, beta, sigma, report)."""
    r = Reducer(precision=precision, **kw)
    try:
        r.reduce(U1, U2, U3, xi, eps)
        return r.get()
    finally:
        import torch
        torch.cuda.current_stream().synchronize()
        r.close()
