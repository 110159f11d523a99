"""Thin ctypes binding of liblp_unwrap.so (the C ABI in include/lp_unwrap.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Tensors are torch CUDA (HIP) tensors; their device pointers and the current
stream are handed to the library.  Importing this module fails loudly when the
library has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblp_unwrap.so")

# status codes
OK = 0
NOT_CONVERGED = 1
ERR_INVALID_ARG = -1
ERR_OOM = -2
ERR_HIP = -3
ERR_NONFINITE = -4
ERR_BREAKDOWN = -5

PRECONDITIONERS = {"none": 0, "jacobi": 1, "ilu0": 2, "ic0": 3, "ssor": 4, "dct": 5,
                   "ilu0_rb": 6, "ic0_rb": 7, "ssor_rb": 8}
STOP_RULES = {"relres": 0, "paper": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}
DCT_MODES = {"fp32": 0, "split_bf16": 1, "fp16_scaled": 2}


class LpuOptions(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int), ("outer_tol", ctypes.c_double),
                ("l_max", ctypes.c_longlong), ("stop_rule", ctypes.c_int),
                ("eps_cg", ctypes.c_double), ("residual_period", ctypes.c_int),
                ("ssor_omega", ctypes.c_double), ("precision", ctypes.c_int),
                ("dct_mode", ctypes.c_int), ("use_phi0", ctypes.c_int),
                ("refine_eta", ctypes.c_double), ("max_refine", ctypes.c_int)]


class LpuStats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters_total", ctypes.c_longlong),
                ("refinements", ctypes.c_int), ("final_relres", ctypes.c_double),
                ("outer_err", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("converged", ctypes.c_int),
                ("status", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LpuMap(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int), ("cols", ctypes.c_int), ("psi", ctypes.c_void_p),
                ("mask", ctypes.c_void_p), ("phi", ctypes.c_void_p)]


class LpuTuning(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int), ("grid", ctypes.c_int), ("dct_grid", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("max_batch_iters", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTED = ["lpu_default_options", "lp_unwrap_create", "lp_unwrap_destroy", "lp_unwrap_solve",
            "lp_unwrap_batch", "lp_unwrap_status_string", "lp_unwrap_last_error",
            "lpu_wrapped_differences", "lpu_weights", "lpu_apply_A", "lpu_rhs",
            "lpu_precond_apply", "lpu_ilu_pivots", "lpu_kernel_timing", "lpu_kernel_timing_get",
            "lpu_default_tuning", "lp_unwrap_set_tuning", "lp_unwrap_get_tuning",
            "lp_unwrap_autotune", "lpu_debug_force_breakdown", "lpu_precond_apply_noalloc"]

# kernel classes of the instrumentation (lpu_kernel_class)
KERNEL_CLASSES = {"spmv": 0, "update": 1, "confirm": 2, "init": 3, "dct": 4, "sweep": 5,
                  "setup": 6, "twocolor": 7}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(
            "liblp_unwrap.so is not built (%s); run __graft_entry__.build() or "
            "python -m paper_2203_13675_amd.build_lib" % path)
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.lpu_default_options.argtypes = [ctypes.POINTER(LpuOptions)]
    lib.lpu_default_options.restype = None
    lib.lp_unwrap_create.argtypes = [ctypes.POINTER(vp), ip, vp, ip, ip]
    lib.lp_unwrap_create.restype = ip
    lib.lp_unwrap_destroy.argtypes = [vp]
    lib.lp_unwrap_destroy.restype = None
    lib.lp_unwrap_solve.argtypes = [vp, ip, ip, vp, vp, dp, dp, ip, dp,
                                    ctypes.POINTER(LpuOptions), vp, ctypes.POINTER(LpuStats)]
    lib.lp_unwrap_solve.restype = ip
    lib.lp_unwrap_batch.argtypes = [vp, ip, ctypes.POINTER(LpuMap), dp, dp, ip, dp,
                                    ctypes.POINTER(LpuOptions), ctypes.POINTER(LpuStats)]
    lib.lp_unwrap_batch.restype = ip
    lib.lp_unwrap_status_string.argtypes = [ip]
    lib.lp_unwrap_status_string.restype = ctypes.c_char_p
    lib.lp_unwrap_last_error.argtypes = [vp]
    lib.lp_unwrap_last_error.restype = ctypes.c_char_p
    lib.lpu_wrapped_differences.argtypes = [vp, ip, ip, vp, vp, vp]
    lib.lpu_wrapped_differences.restype = ip
    lib.lpu_weights.argtypes = [vp, ip, ip, ip, vp, vp, vp, vp, dp, dp, vp, vp]
    lib.lpu_weights.restype = ip
    lib.lpu_apply_A.argtypes = [vp, ip, ip, ip, vp, vp, vp, vp]
    lib.lpu_apply_A.restype = ip
    lib.lpu_rhs.argtypes = [vp, ip, ip, ip, vp, vp, vp, vp, vp]
    lib.lpu_rhs.restype = ip
    lib.lpu_precond_apply.argtypes = [vp, ip, ip, ip, ip, ip, dp, vp, vp, vp, vp]
    lib.lpu_precond_apply.restype = ip
    lib.lpu_ilu_pivots.argtypes = [vp, ip, ip, ip, vp, vp, vp]
    lib.lpu_ilu_pivots.restype = ip
    lib.lpu_kernel_timing.argtypes = [vp, ctypes.c_uint]
    lib.lpu_kernel_timing.restype = ip
    lib.lpu_kernel_timing_get.argtypes = [vp, ip, ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_longlong),
                                          ctypes.POINTER(dp), ctypes.POINTER(dp)]
    lib.lpu_kernel_timing_get.restype = ip
    lib.lpu_default_tuning.argtypes = [ctypes.POINTER(LpuTuning)]
    lib.lpu_default_tuning.restype = None
    lib.lp_unwrap_set_tuning.argtypes = [vp, ctypes.POINTER(LpuTuning)]
    lib.lp_unwrap_set_tuning.restype = ip
    lib.lp_unwrap_get_tuning.argtypes = [vp, ctypes.POINTER(LpuTuning)]
    lib.lp_unwrap_get_tuning.restype = ip
    lib.lp_unwrap_autotune.argtypes = [vp, ip, ctypes.POINTER(LpuMap), dp, dp, ip, dp,
                                       ctypes.POINTER(LpuOptions), ip, ctypes.c_char_p,
                                       ctypes.POINTER(LpuTuning), ctypes.POINTER(dp)]
    lib.lp_unwrap_autotune.restype = ip
    lib.lpu_precond_apply_noalloc.argtypes = [vp, ip, ip, ip, ip, dp, vp, vp, vp, vp]
    lib.lpu_precond_apply_noalloc.restype = ip
    lib.lpu_debug_force_breakdown.argtypes = [vp, ctypes.c_longlong]
    lib.lpu_debug_force_breakdown.restype = ip
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def status_string(code: int) -> str:
    return lib().lp_unwrap_status_string(code).decode()


class LpuError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (status_string(code), code, msg))
        self.code = code


def default_options(**kw) -> LpuOptions:
    o = LpuOptions()
    lib().lpu_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "stop_rule" and isinstance(v, str):
            v = STOP_RULES[v]
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "dct_mode" and isinstance(v, str):
            v = DCT_MODES[v]
        setattr(o, k, v)
    return o


def paper_options(**kw) -> LpuOptions:
    """Algorithm 1 with the stopping criteria of the paper's experiments (Section 3):
    the inner test on the preconditioned residual with eps = 0.005, k_max = 500, outer
    tolerance 1e-6 on the relative change, l_max = 2MN, FP64, starting from the phi the
    caller passes (a seeded random field stands for the paper's random start).  Keyword
    arguments override single fields."""
    base = dict(stop_rule="paper", eps_cg=0.005, k_max=500, outer_tol=1e-6, l_max=0,
                precision="fp64", use_phi0=1)
    base.update(kw)
    return default_options(**base)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_dev(t, dtype, n, name):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be contiguous with %d elements" % (name, n))


@dataclass
class SolveResult:
    phi: torch.Tensor
    status: int
    stats: dict


class Context:
    """An lp_unwrap context bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None, max_rows: int = 0, max_cols: int = 0):
        self._lib = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = ctypes.c_void_p()
        rc = self._lib.lp_unwrap_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream),
                                        max_rows, max_cols)
        if rc != OK:
            raise LpuError(rc, "lp_unwrap_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lp_unwrap_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return self._lib.lp_unwrap_last_error(self._h).decode()

    def _raise(self, rc):
        if rc < 0:
            raise LpuError(rc, self.last_error())
        return rc

    # -- whole solves -------------------------------------------------------
    def solve(self, psi, mask=None, *, p=0.0, eps=0.01, preconditioner="dct", tol=1e-6,
              options: LpuOptions | None = None, phi=None, check=True, **opt_kw) -> SolveResult:
        M, N = psi.shape
        n = M * N
        _check_dev(psi, torch.float64, n, "psi")
        _check_dev(mask, torch.float32, n, "mask")
        if options is None:
            options = default_options(**opt_kw)
        if phi is None:
            phi = torch.zeros((M, N), dtype=torch.float64, device=psi.device)
            options.use_phi0 = 0 if "use_phi0" not in opt_kw else options.use_phi0
        _check_dev(phi, torch.float64, n, "phi")
        st = LpuStats()
        pc = PRECONDITIONERS[preconditioner] if isinstance(preconditioner, str) else preconditioner
        rc = self._lib.lp_unwrap_solve(self._h, M, N, _ptr(psi), _ptr(mask), float(p), float(eps),
                                       pc, float(tol), ctypes.byref(options), _ptr(phi),
                                       ctypes.byref(st))
        if check:
            self._raise(rc)
        return SolveResult(phi, rc, st.as_dict())

    @staticmethod
    def _maps(psis, masks, phis):
        k = len(psis)
        if masks is None:
            masks = [None] * k
        if phis is None:
            phis = [torch.zeros(t.shape, dtype=torch.float64, device=t.device) for t in psis]
        arr = (LpuMap * k)()
        for i, (ps, mk, ph) in enumerate(zip(psis, masks, phis)):
            M, N = ps.shape
            _check_dev(ps, torch.float64, M * N, "psi")
            _check_dev(mk, torch.float32, M * N, "mask")
            _check_dev(ph, torch.float64, M * N, "phi")
            arr[i] = LpuMap(M, N, ps.data_ptr(), mk.data_ptr() if mk is not None else None,
                            ph.data_ptr())
        return arr, phis

    def batch(self, psis, masks=None, *, p=0.0, eps=0.01, preconditioner="dct", tol=1e-6,
              options: LpuOptions | None = None, phis=None, check=True, **opt_kw):
        k = len(psis)
        if options is None:
            options = default_options(**opt_kw)
        arr, phis = self._maps(psis, masks, phis)
        stats = (LpuStats * k)()
        pc = PRECONDITIONERS[preconditioner] if isinstance(preconditioner, str) else preconditioner
        rc = self._lib.lp_unwrap_batch(self._h, k, arr, float(p), float(eps), pc, float(tol),
                                       ctypes.byref(options), stats)
        if check:
            self._raise(rc)
        return phis, rc, [s.as_dict() for s in stats]

    # -- launch tuning ------------------------------------------------------
    def tuning(self) -> dict:
        t = LpuTuning()
        self._raise(self._lib.lp_unwrap_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw) -> dict:
        """Change fields of the context's tuning (tile_rows, grid, dct_grid, use_graph,
        max_batch_iters); "default" restores lpu_default_tuning."""
        t = LpuTuning()
        if kw.pop("default", False):
            self._lib.lpu_default_tuning(ctypes.byref(t))
        else:
            self._raise(self._lib.lp_unwrap_get_tuning(self._h, ctypes.byref(t)))
        for k, v in kw.items():
            if k not in t.as_dict():
                raise KeyError(k)
            setattr(t, k, int(v))
        self._raise(self._lib.lp_unwrap_set_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def autotune(self, psis, masks=None, *, p=0.0, eps=0.01, preconditioner="dct", tol=1e-6,
                 options: LpuOptions | None = None, probe_iters=20, cache_path=None, phis=None,
                 **opt_kw):
        """Run lp_unwrap_autotune on a batch; returns (tuning dict, tuning wall ms)."""
        if options is None:
            options = default_options(**opt_kw)
        arr, phis = self._maps(psis, masks, phis)
        best, ms = LpuTuning(), ctypes.c_double()
        pc = PRECONDITIONERS[preconditioner] if isinstance(preconditioner, str) else preconditioner
        path = None if cache_path is None else str(cache_path).encode()
        rc = self._lib.lp_unwrap_autotune(self._h, len(psis), arr, float(p), float(eps), pc,
                                          float(tol), ctypes.byref(options), int(probe_iters),
                                          path, ctypes.byref(best), ctypes.byref(ms))
        self._raise(rc)
        return best.as_dict(), ms.value

    # -- instrumentation ----------------------------------------------------
    def kernel_timing(self, classes="all"):
        """Time launches of the given kernel classes ("all", "off", a name or a list)."""
        if classes == "all":
            mask = (1 << len(KERNEL_CLASSES)) - 1
        elif classes in ("off", None):
            mask = 0
        else:
            names = [classes] if isinstance(classes, str) else classes
            mask = 0
            for nm in names:
                mask |= 1 << KERNEL_CLASSES[nm]
        self._raise(self._lib.lpu_kernel_timing(self._h, mask))

    def kernel_timing_report(self):
        out = {}
        for name, k in KERNEL_CLASSES.items():
            ms, n = ctypes.c_double(), ctypes.c_longlong()
            b, f = ctypes.c_double(), ctypes.c_double()
            self._raise(self._lib.lpu_kernel_timing_get(self._h, k, ctypes.byref(ms), ctypes.byref(n),
                                                        ctypes.byref(b), ctypes.byref(f)))
            if ms.value > 0 or n.value > 0:
                out[name] = {"ms": ms.value, "launches": n.value, "bytes": b.value,
                             "flops": f.value}
        return out

    # -- single steps -------------------------------------------------------
    def wrapped_differences(self, psi):
        M, N = psi.shape
        _check_dev(psi, torch.float64, M * N, "psi")
        dx = torch.empty_like(psi)
        dy = torch.empty_like(psi)
        self._raise(self._lib.lpu_wrapped_differences(self._h, M, N, _ptr(psi), _ptr(dx), _ptr(dy)))
        return dx, dy

    @staticmethod
    def _dtype(precision):
        return torch.float64 if precision in ("fp64", 0) else torch.float32

    @staticmethod
    def _prec(precision):
        return PRECISIONS[precision] if isinstance(precision, str) else precision

    def weights(self, phi, dx, dy, mask=None, *, p=0.0, tau=0.01, precision="fp64"):
        M, N = phi.shape
        dt = self._dtype(precision)
        U = torch.empty((M, N), dtype=dt, device=phi.device)
        V = torch.empty_like(U)
        _check_dev(mask, torch.float32, M * N, "mask")
        self._raise(self._lib.lpu_weights(self._h, M, N, self._prec(precision), _ptr(phi), _ptr(dx),
                                          _ptr(dy), _ptr(mask), float(p), float(tau), _ptr(U),
                                          _ptr(V)))
        return U, V

    def apply_A(self, U, V, x, precision="fp64"):
        M, N = x.shape
        y = torch.empty_like(x)
        self._raise(self._lib.lpu_apply_A(self._h, M, N, self._prec(precision), _ptr(U), _ptr(V),
                                          _ptr(x), _ptr(y)))
        return y

    def rhs(self, U, V, dx, dy, precision="fp64"):
        M, N = dx.shape
        b = torch.empty_like(dx)
        self._raise(self._lib.lpu_rhs(self._h, M, N, self._prec(precision), _ptr(U), _ptr(V),
                                      _ptr(dx), _ptr(dy), _ptr(b)))
        return b

    def debug_force_breakdown(self, iteration: int):
        """Testing hook: PCG iteration `iteration` of every later inner solve
        reports a breakdown (0 switches it off)."""
        self._raise(self._lib.lpu_debug_force_breakdown(self._h, int(iteration)))

    def precond_apply(self, U, V, r, preconditioner, *, precision="fp64", dct_mode="split_bf16",
                      omega=1.0):
        M, N = r.shape
        s = torch.empty_like(r)
        pc = PRECONDITIONERS[preconditioner] if isinstance(preconditioner, str) else preconditioner
        dm = DCT_MODES[dct_mode] if isinstance(dct_mode, str) else dct_mode
        self._raise(self._lib.lpu_precond_apply(self._h, M, N, self._prec(precision), pc, dm,
                                                float(omega), _ptr(U), _ptr(V), _ptr(r), _ptr(s)))
        return s

    def precond_apply_noalloc(self, U, V, r, s, preconditioner, *, precision="fp64", omega=1.0):
        """lpu_precond_apply_noalloc: enqueue s = M^{-1} r into the caller's s
        (no allocation, no synchronisation); returns the status."""
        M, N = r.shape
        pc = PRECONDITIONERS[preconditioner] if isinstance(preconditioner, str) else preconditioner
        return self._lib.lpu_precond_apply_noalloc(self._h, M, N, self._prec(precision), pc,
                                                   float(omega), _ptr(U), _ptr(V), _ptr(r), _ptr(s))

    def ilu_pivots(self, U, V, precision="fp64"):
        M, N = U.shape
        piv = torch.empty_like(U)
        self._raise(self._lib.lpu_ilu_pivots(self._h, M, N, self._prec(precision), _ptr(U), _ptr(V),
                                             _ptr(piv)))
        return piv

