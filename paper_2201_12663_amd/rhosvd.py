"""ctypes binding of librhosvd.so (include/rhosvd.h).

Argument marshalling only: every step of the reduction runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  The library must be
built (python -m paper_2201_12663_amd.build); nothing here falls back to another
implementation.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librhosvd.so")

FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
PHASES = ["norms", "anorm", "gram", "eig", "trunc_z", "project", "core"]
ANORM = {"auto": 0, "exact": 1, "probe": 2}
REFINE = {"auto": 0, "refine": 1, "deflate": 2, "off": 3}

STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_NONFINITE", -3: "ERR_ALLOC", -4: "ERR_DEVICE",
          -5: "ERR_NOCONV", -6: "ERR_STATE", -7: "ERR_UNSUPPORTED", -8: "ERR_CAPACITY"}

# every symbol include/rhosvd.h declares
EXPORTS = ["rhosvd_create", "rhosvd_create_with_allocator", "rhosvd_destroy", "rhosvd_set_options", "rhosvd_reduce", "rhosvd_get",
           "rhosvd_get_xi", "rhosvd_get_spectrum", "rhosvd_get_v", "rhosvd_reduce_batched",
           "rhosvd_batch_uses_graph", "rhosvd_last_core_tile", "rhosvd_net_num_params", "rhosvd_net_set_params", "rhosvd_net_get_params",
           "rhosvd_net_forward", "rhosvd_net_train_step", "rhosvd_sketch_features", "rhosvd_reduce_learned",
           "rhosvd_phase_ms", "rhosvd_last_error", "rhosvd_version", "rhosvd_t2c", "rhosvd_t2c_get",
           "rhosvd_t2c_noalloc"]

NET_IN, NET_OUT = 67, 2
PATHS = {0: "range finder", 1: "gram (chosen)", 2: "gram (certificate failed)", 3: "gram (R < n)"}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """rhosvd_allocator"""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_eig_sweeps", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("beta_fp32", ctypes.c_int32), ("refine_tails", ctypes.c_int32),
                ("core_tile", ctypes.c_int32), ("certificate", ctypes.c_int32), ("anorm", ctypes.c_int32),
                ("als_sweeps", ctypes.c_int32), ("gram_precision", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("xi_norm", ctypes.c_double), ("a_norm", ctypes.c_double), ("tau", ctypes.c_double),
                ("bound", ctypes.c_double), ("tail", ctypes.c_double * 3), ("ranks", ctypes.c_int32 * 3),
                ("m", ctypes.c_int32), ("eig_sweeps", ctypes.c_int32), ("dropped", ctypes.c_int32),
                ("certificate", ctypes.c_double), ("a_norm_upper", ctypes.c_double),
                ("anorm_method", ctypes.c_int32), ("refine_used", ctypes.c_int32),
                ("core_precision", ctypes.c_int32), ("gram_precision", ctypes.c_int32)]


class Problem(ctypes.Structure):
    """rhosvd_problem: one reduction of a batch (device pointers)."""
    _fields_ = [("n", ctypes.c_int64), ("R", ctypes.c_int64), ("U1", ctypes.c_void_p), ("U2", ctypes.c_void_p),
                ("U3", ctypes.c_void_p), ("xi", ctypes.c_void_p), ("eps", ctypes.c_double),
                ("cap_rank", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("cap_beta", ctypes.c_int64),
                ("Z1", ctypes.c_void_p), ("Z2", ctypes.c_void_p), ("Z3", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("result", ctypes.c_void_p),
                ("V1", ctypes.c_void_p), ("V2", ctypes.c_void_p), ("V3", ctypes.c_void_p)]


class LearnedInfo(ctypes.Structure):
    """rhosvd_learned_info"""
    _fields_ = [("proposal", ctypes.c_int32 * 3), ("width", ctypes.c_int32 * 3), ("fallback", ctypes.c_int32 * 3),
                ("reserved", ctypes.c_int32), ("residual", ctypes.c_double * 3)]


# Handles still open when the interpreter exits are closed by an atexit hook,
# which runs before the C runtime's exit handlers (where the HIP runtime and
# any loaded profiler tear down), so no library call reaches a finalized runtime.
_live = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    for r in list(_live):
        try:
            r.close()
        except Exception:
            pass


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
        lib.rhosvd_create_with_allocator.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(Allocator),
                                                     ctypes.POINTER(Options)]
        lib.rhosvd_destroy.argtypes = [vp]
        lib.rhosvd_set_options.argtypes = [vp, ctypes.POINTER(Options)]
        lib.rhosvd_reduce.argtypes = [vp, i64, i64, vp, vp, vp, vp, dbl, ctypes.POINTER(i32)]
        lib.rhosvd_get.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(Report)]
        lib.rhosvd_get_xi.argtypes = [vp, vp]
        lib.rhosvd_get_spectrum.argtypes = [vp, i32, vp]
        lib.rhosvd_get_v.argtypes = [vp, i32, vp]
        lib.rhosvd_reduce_batched.argtypes = [vp, i32, ctypes.POINTER(Problem)]
        lib.rhosvd_batch_uses_graph.argtypes = [vp]
        lib.rhosvd_batch_uses_graph.restype = i32
        lib.rhosvd_last_core_tile.argtypes = [vp]
        lib.rhosvd_last_core_tile.restype = i32
        fp = ctypes.c_float
        lib.rhosvd_net_num_params.restype = i32
        lib.rhosvd_net_set_params.argtypes = [vp, vp]
        lib.rhosvd_net_get_params.argtypes = [vp, vp]
        lib.rhosvd_net_forward.argtypes = [vp, i32, vp, vp]
        lib.rhosvd_net_train_step.argtypes = [vp, i32, vp, vp, fp, vp, vp]
        lib.rhosvd_sketch_features.argtypes = [vp, i64, i64, vp, vp, vp, vp, dbl, vp, i32, vp]
        lib.rhosvd_reduce_learned.argtypes = [vp, i64, i64, vp, vp, vp, vp, dbl, vp, i32, ctypes.POINTER(i32),
                                              ctypes.POINTER(LearnedInfo)]
        lib.rhosvd_t2c.argtypes = [vp, i32, i32, i32, vp, dbl, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
        lib.rhosvd_t2c_get.argtypes = [vp, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        lib.rhosvd_t2c_noalloc.argtypes = [vp, i32, i32, i32, vp, dbl, i64, vp, vp, vp, vp, vp, vp, vp]
        lib.rhosvd_phase_ms.argtypes = [vp, i32]
        lib.rhosvd_phase_ms.restype = dbl
        lib.rhosvd_last_error.argtypes = [vp]
        lib.rhosvd_last_error.restype = ctypes.c_char_p
        lib.rhosvd_version.restype = ctypes.c_char_p
        for f in ("rhosvd_create", "rhosvd_create_with_allocator", "rhosvd_destroy", "rhosvd_set_options", "rhosvd_reduce", "rhosvd_get",
                  "rhosvd_get_xi", "rhosvd_get_spectrum", "rhosvd_get_v", "rhosvd_reduce_batched",
                  "rhosvd_net_set_params", "rhosvd_net_get_params", "rhosvd_net_forward", "rhosvd_net_train_step",
                  "rhosvd_sketch_features", "rhosvd_reduce_learned", "rhosvd_t2c", "rhosvd_t2c_get", "rhosvd_t2c_noalloc"):
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

    def __init__(self, precision="fp64", stream=None, max_eig_sweeps=0, profile=False, beta_fp32=False,
                 refine_tails="auto", core_tile=0, certificate=False, anorm="auto", als_sweeps=0,
                 gram_precision="fp64", torch_allocator=True):
        """torch_allocator: the handle's device workspace comes from PyTorch's
        caching allocator (rhosvd_create_with_allocator), so it is counted by
        torch.cuda.memory_allocated and shares torch's pool; False: hipMalloc.
        gram_precision: "fp64" (default), "fp32" or "bf16x3" (rhosvd_options.gram_precision)."""
        import torch
        self.lib = load()
        self.opt = Options()
        self.opt.core_tile = int(core_tile)
        self.opt.certificate = 1 if certificate else 0
        self.opt.anorm = ANORM[anorm] if isinstance(anorm, str) else int(anorm)
        self.opt.als_sweeps = int(als_sweeps)
        self.opt.beta_fp32 = 1 if beta_fp32 else 0
        self.opt.refine_tails = REFINE.get(refine_tails, -1) if isinstance(refine_tails, str) else \
            (int(refine_tails) if refine_tails in (0, 1, 2, 3) else -1)
        self.beta_dtype = torch.float32 if beta_fp32 else torch.float64
        self.opt.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.opt.gram_precision = PRECISIONS.get(gram_precision, -1) if isinstance(gram_precision, str) else \
            int(gram_precision)
        self.opt.max_eig_sweeps = int(max_eig_sweeps)
        self.opt.profile = 1 if profile else 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.h = ctypes.c_void_p()
        self._allocator = None
        if torch_allocator:
            dev = torch.cuda.current_device()

            def _alloc(size, ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(int(size), dev, stream)
                except Exception:      # out of memory: the library reports RHOSVD_ERR_ALLOC
                    return None

            def _free(ptr, ctx):
                torch.cuda.caching_allocator_delete(ptr)

            self._allocator = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
            s = self.lib.rhosvd_create_with_allocator(ctypes.byref(self.h), ctypes.c_void_p(stream.cuda_stream),
                                                      ctypes.byref(self._allocator), ctypes.byref(self.opt))
        else:
            s = self.lib.rhosvd_create(ctypes.byref(self.h), ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(self.opt))
        if s != 0:
            raise RhosvdError(s, self.lib.rhosvd_last_error(None).decode())
        self.n = self.R = 0
        self.ranks = (0, 0, 0)
        _live.add(self)

    def close(self):
        """Release the handle (waits for its stream).  Idempotent."""
        if self.h:
            self.lib.rhosvd_destroy(self.h)
            self.h = ctypes.c_void_p()
        _live.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter teardown the HIP runtime may already be gone: the
        # atexit hook has closed every handle by then, so nothing is left to do
        # (module globals may already be None then, hence the bound default)
        if _finalizing() or not self.h:
            return
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
                if beta_out.numel() < r1 * r2 * r3 or beta_out.dtype != self.beta_dtype:
                    raise ValueError(f"beta_out too small or not {self.beta_dtype}")
                flat = beta_out
            else:
                flat = torch.empty(r1 * r2 * r3, dtype=self.beta_dtype, device=dev)
            b = flat[: r1 * r2 * r3]
        sig = torch.empty(r1 + r2 + r3, dtype=torch.float64, device=dev) if sigma else None
        rep = Report()
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p()
        self._check(self.lib.rhosvd_get(self.h, ptr(Zs[0]), ptr(Zs[1]), ptr(Zs[2]), ptr(b), ptr(sig),
                                        ctypes.byref(rep)))
        report = dict(xi_norm=rep.xi_norm, a_norm=rep.a_norm, tau=rep.tau, bound=rep.bound,
                      tail=list(rep.tail), ranks=list(rep.ranks), m=rep.m, eig_sweeps=rep.eig_sweeps,
                      dropped=rep.dropped, certificate=rep.certificate, a_norm_upper=rep.a_norm_upper,
                      anorm_method=rep.anorm_method, refine_used=rep.refine_used,
                      core_precision=rep.core_precision, gram_precision=rep.gram_precision)
        beta_t = None
        if b is not None:
            beta_t = b.view(r3, r2, r1).permute(2, 1, 0) if b.numel() > 0 else b.view(r1, r2, r3)
        return Result(self.ranks, Zs, beta_t, sig, report)

    def core_only(self, beta_flat):
        """Enqueue only the core contraction into beta_flat (for timing loops)."""
        if beta_flat.dtype != self.beta_dtype:
            raise ValueError(f"beta_flat must be {self.beta_dtype}")
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

    # ---- batched reductions
    def batch_descriptors(self, problems, results, outputs=None, cap_rank=None, v_outputs=None):
        """Descriptor array for rhosvd_reduce_batched.

        problems: list of (U1, U2, U3, xi, eps) with column-major CUDA tensors.
        results:  (count, 8) int32 CUDA tensor (ranks, status, dropped).
        outputs:  None (ranks only), or a list of (Z1, Z2, Z3, beta_flat) per problem
                  (Z_l: (n, cap) column-major float64, beta_flat: the handle's beta dtype, or None).
        cap_rank: per-problem rank caps when outputs is None (default min(n, R)).
        v_outputs: None, or per problem (V1, V2, V3) column-major float64 tensors of
                  shape (cap_rank, R) (the mixed Tucker-canonical factors), or None."""
        import torch
        if not (results.is_cuda and results.dtype == torch.int32 and results.is_contiguous()
                and tuple(results.shape) == (len(problems), 8)):
            raise ValueError("results: expected a contiguous (count, 8) int32 CUDA tensor")
        arr = (Problem * len(problems))()
        for i, (U1, U2, U3, xi, eps) in enumerate(problems):
            n, R = U1.shape
            d = arr[i]
            d.n, d.R = n, R
            d.U1, d.U2, d.U3 = (_colmajor(U1, "U1").value, _colmajor(U2, "U2").value, _colmajor(U3, "U3").value)
            if not (xi.is_cuda and xi.dtype == torch.float64 and xi.is_contiguous() and xi.numel() == R):
                raise ValueError("xi: expected a contiguous float64 CUDA tensor of length R")
            d.xi = xi.data_ptr()
            d.eps = float(eps)
            d.result = results[i].data_ptr()
            if outputs is None:
                d.cap_rank = int(cap_rank[i]) if cap_rank is not None else min(n, R)
            else:
                Z1, Z2, Z3, b = outputs[i]
                d.cap_rank = int(Z1.shape[1])
                if Z1.shape[1] > 0:
                    for Z in (Z1, Z2, Z3):
                        if tuple(Z.shape) != (n, d.cap_rank):
                            raise ValueError("Z outputs must be (n, cap_rank)")
                    d.Z1, d.Z2, d.Z3 = (_colmajor(Z1, "Z1").value, _colmajor(Z2, "Z2").value,
                                        _colmajor(Z3, "Z3").value)
                if d.cap_rank < 1:
                    d.cap_rank = 1
                if b is not None and b.numel() > 0:
                    if b.dtype != self.beta_dtype:
                        raise ValueError(f"beta outputs must be {self.beta_dtype}")
                    d.beta = b.data_ptr()
                    d.cap_beta = int(b.numel())
            if v_outputs is not None and v_outputs[i] is not None:
                Vs = v_outputs[i]
                for V in Vs:
                    if tuple(V.shape) != (d.cap_rank, R):
                        raise ValueError("V outputs must be (cap_rank, R)")
                d.V1, d.V2, d.V3 = (_colmajor(Vs[0], "V1").value, _colmajor(Vs[1], "V2").value,
                                    _colmajor(Vs[2], "V3").value)
        return arr

    def reduce_batched_raw(self, descriptors):
        """Enqueue one batched pass (see include/rhosvd.h)."""
        self._check(self.lib.rhosvd_reduce_batched(self.h, len(descriptors), descriptors))

    # ---- rank-proposal network and the learned path
    @staticmethod
    def _f32(t, name, numel=None):
        import torch
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor")
        if numel is not None and t.numel() < numel:
            raise ValueError(f"{name}: expected at least {numel} elements")
        return ctypes.c_void_p(t.data_ptr())

    def net_set(self, params):
        self._check(self.lib.rhosvd_net_set_params(self.h, self._f32(params, "params", self.lib.rhosvd_net_num_params())))

    def net_get(self):
        import torch
        out = torch.empty(self.lib.rhosvd_net_num_params(), dtype=torch.float32, device="cuda")
        self._check(self.lib.rhosvd_net_get_params(self.h, ctypes.c_void_p(out.data_ptr())))
        return out

    def net_forward(self, x):
        import torch
        y = torch.empty((x.shape[0], NET_OUT), dtype=torch.float32, device="cuda")
        self._check(self.lib.rhosvd_net_forward(self.h, x.shape[0], self._f32(x, "x"), ctypes.c_void_p(y.data_ptr())))
        return y

    def net_train_step(self, x, target, lr, want_grad=False):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        grad = torch.empty(self.lib.rhosvd_net_num_params(), dtype=torch.float32, device="cuda") if want_grad else None
        self._check(self.lib.rhosvd_net_train_step(self.h, x.shape[0], self._f32(x, "x"), self._f32(target, "target"),
                                                   float(lr), ctypes.c_void_p(loss.data_ptr()),
                                                   ctypes.c_void_p(grad.data_ptr()) if grad is not None else None))
        return loss, grad

    def sketch_features(self, U1, U2, U3, xi, eps, omega):
        import torch
        n, R = U1.shape
        if not (omega.is_cuda and omega.dtype == torch.float64 and omega.dim() == 2 and omega.shape[0] == R):
            raise ValueError("omega: expected an (R, w) float64 CUDA tensor")
        feat = torch.empty((3, NET_IN), dtype=torch.float32, device="cuda")
        self._check(self.lib.rhosvd_sketch_features(self.h, n, R, _colmajor(U1, "U1"), _colmajor(U2, "U2"),
                                                    _colmajor(U3, "U3"), ctypes.c_void_p(xi.data_ptr()), float(eps),
                                                    _colmajor(omega, "omega"), omega.shape[1],
                                                    ctypes.c_void_p(feat.data_ptr())))
        return feat

    def reduce_learned(self, U1, U2, U3, xi, eps, omega):
        import torch
        n, R = U1.shape
        if not (omega.is_cuda and omega.dtype == torch.float64 and omega.dim() == 2 and omega.shape[0] == R):
            raise ValueError("omega: expected an (R, w) float64 CUDA tensor")
        ranks = (ctypes.c_int32 * 3)()
        info = LearnedInfo()
        self._check(self.lib.rhosvd_reduce_learned(self.h, n, R, _colmajor(U1, "U1"), _colmajor(U2, "U2"),
                                                   _colmajor(U3, "U3"), ctypes.c_void_p(xi.data_ptr()), float(eps),
                                                   _colmajor(omega, "omega"), omega.shape[1], ranks,
                                                   ctypes.byref(info)))
        self.n, self.R = n, R
        self.ranks = tuple(int(r) for r in ranks)
        return self.ranks, dict(proposal=list(info.proposal), width=list(info.width),
                                path=list(info.fallback), residual=list(info.residual))

    # ---- Tucker-to-canonical transform (Remark 2.6)
    def t2c(self, beta, eps, Z=None):
        """Canonical form of a core: beta (r1, r2, r3) float64 CUDA tensor in
        Fortran order (as Result.beta), eps the absolute accuracy.  Returns a dict:
        weights (R,), F1 (r1, R), F2 (r2, R) column-major, slice (R,) int32, sigma
        (r3, min(r1, r2)), bound, and with Z = [Z1, Z2, Z3] the lifted factors
        C1, C2, C3 (n, R)."""
        import torch
        if not (beta.is_cuda and beta.dtype == torch.float64 and beta.dim() == 3):
            raise ValueError("beta: expected a 3-D float64 CUDA tensor")
        r1, r2, r3 = beta.shape
        if beta.numel() and beta.stride() != (1, r1, r1 * r2):
            raise ValueError("beta: expected Fortran order (strides (1, r1, r1 r2))")
        R = ctypes.c_int64()
        bound = ctypes.c_double()
        self._check(self.lib.rhosvd_t2c(self.h, r1, r2, r3, ctypes.c_void_p(beta.data_ptr()), float(eps),
                                        ctypes.byref(R), ctypes.byref(bound)))
        R = int(R.value)
        w = torch.empty(R, dtype=torch.float64, device="cuda")
        F1, F2 = colmajor_empty(r1, R), colmajor_empty(r2, R)
        sl = torch.empty(R, dtype=torch.int32, device="cuda")
        sig = torch.empty((r3, min(r1, r2)), dtype=torch.float64, device="cuda")
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p()
        out = dict(R=R, bound=bound.value, weights=w, F1=F1, F2=F2, slice=sl, sigma=sig)
        n = 0
        Zp = [ctypes.c_void_p()] * 3
        Cp = [ctypes.c_void_p()] * 3
        if Z is not None:
            n = Z[0].shape[0]
            Cs = [colmajor_empty(n, R) for _ in range(3)]
            Zp = [_colmajor(z, f"Z{l + 1}") for l, z in enumerate(Z)]
            Cp = [ptr(c) for c in Cs]
            out.update(C1=Cs[0], C2=Cs[1], C3=Cs[2])
            if R == 0:
                n = 0
                Zp = [ctypes.c_void_p()] * 3
                Cp = [ctypes.c_void_p()] * 3
        self._check(self.lib.rhosvd_t2c_get(self.h, ptr(w), ptr(F1), ptr(F2), ptr(sl), ptr(sig), n,
                                            Zp[0], Zp[1], Zp[2], Cp[0], Cp[1], Cp[2]))
        return out

    def batch_uses_graph(self):
        return bool(self.lib.rhosvd_batch_uses_graph(self.h))

    def last_core_tile(self):
        """Rows per workgroup tile of the last core launch (64 or 128; 0 before any)."""
        return int(self.lib.rhosvd_last_core_tile(self.h))

    def reduce_batched(self, problems, beta=True):
        """Batched reductions with outputs sized exactly: a ranks-only pass, then
        the full pass into freshly allocated Z (and beta).  Returns a list of
        dicts (ranks, status, dropped, Z, beta) and the descriptor array of the
        full pass (replaying it reuses the recorded graph)."""
        import torch
        count = len(problems)
        res = torch.zeros((count, 8), dtype=torch.int32, device="cuda")
        self.reduce_batched_raw(self.batch_descriptors(problems, res))
        self.stream.synchronize()   # the pass runs on the handle's stream, the copy on the current one
        ranks = res.cpu().numpy()
        outs = []
        for i, (U1, _, _, _, _) in enumerate(problems):
            n = U1.shape[0]
            r = [int(x) for x in ranks[i, :3]]
            cap = max(1, max(r))
            Zs = [colmajor_empty(n, cap) for _ in range(3)]
            b = torch.empty(max(1, r[0] * r[1] * r[2]), dtype=self.beta_dtype, device="cuda") if beta else None
            outs.append((Zs[0], Zs[1], Zs[2], b))
        res2 = torch.zeros((count, 8), dtype=torch.int32, device="cuda")
        desc = self.batch_descriptors(problems, res2, outputs=outs)
        self.reduce_batched_raw(desc)
        self.stream.synchronize()
        rr = res2.cpu().numpy()
        out = []
        for i in range(count):
            r = tuple(int(x) for x in rr[i, :3])
            Z1, Z2, Z3, b = outs[i]
            bt = None
            if b is not None and all(x > 0 for x in r):
                bt = b[: r[0] * r[1] * r[2]].view(r[2], r[1], r[0]).permute(2, 1, 0)
            out.append(dict(ranks=r, status=int(rr[i, 3]), dropped=int(rr[i, 4]), core_precision=int(rr[i, 5]),
                            Z=[Z1[:, :r[0]], Z2[:, :r[1]], Z3[:, :r[2]]], beta=bt))
        return out, desc, res2, outs


def t2c_noalloc(beta, eps, cap, weights, F1, F2, slice_, R, bound, status, stream=None):
    """rhosvd_t2c_noalloc (include/rhosvd.h): enqueue the transform of beta into
    caller-allocated device tensors (no allocation by the library, no wait).
    beta: (r1, r2, r3) float64 CUDA tensor in Fortran order; weights (cap,) float64;
    F1 (r1, cap), F2 (r2, cap) column-major float64; slice_ (cap,) int32; R (1,)
    int64; bound (1,) float64 or None; status (1,) int32.  Returns the host status."""
    import torch
    lib = load()
    if not (beta.is_cuda and beta.dtype == torch.float64 and beta.dim() == 3):
        raise ValueError("beta: expected a 3-D float64 CUDA tensor")
    r1, r2, r3 = beta.shape
    if beta.stride() != (1, r1, r1 * r2):
        raise ValueError("beta: expected Fortran order")
    if stream is None:
        stream = torch.cuda.current_stream()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p()
    return int(lib.rhosvd_t2c_noalloc(ctypes.c_void_p(stream.cuda_stream), r1, r2, r3, ptr(beta), float(eps),
                                      int(cap), ptr(weights), ptr(F1), ptr(F2), ptr(slice_), ptr(R), ptr(bound),
                                      ptr(status)))


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
