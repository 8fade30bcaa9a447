"""Entropic KL-unbalanced optimal transport on AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libuot.so`` (C ABI in ``include/uot.h``): plain Sinkhorn and
translation-invariant Sinkhorn (Sejourne, Vialard, Peyre, AISTATS 2022, Sec. 3), the dual
value, plan application and the envelope-theorem backward. Every step of the computation
runs in the library's HIP kernels; this module only marshals tensors (``data_ptr()``) and
the current HIP stream. PyTorch provides device memory and streams.

There is no CPU fallback: importing works without a GPU, but every compute call raises if
the library is missing or no GPU is visible.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

__all__ = ["UOTError", "Info", "sinkhorn", "ti_sinkhorn", "dual_value", "plan_apply", "marginals",
           "backward", "workspace_bytes", "UOTLoss", "uot_loss", "library_path", "load_library",
           "profile_enable", "profile_reset", "profile_read", "set_points_kernel",
           "ti_sinkhorn_batched", "sinkhorn_anderson", "ti_sinkhorn_anderson", "sinkhorn_phi",
           "fw1d_batched", "fw1d", "fw1d_barycenter", "batched_set_plan",
           "batched_trace", "batched_trace_read", "probe_rate", "backward_noalloc",
           "set_autotune", "batched_last_plan", "batched_autotune_reset"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libuot.so")
_lib = None

UOT_OK, UOT_ERR_INVALID, UOT_ERR_HIP, UOT_ERR_NUMERIC, UOT_ERR_WORKSPACE = range(5)
UOT_COST_DENSE, UOT_COST_POINTS = 0, 1
UOT_WS_SOLVE, UOT_WS_DUAL, UOT_WS_PLAN, UOT_WS_BACKWARD, UOT_WS_ANDERSON = range(5)


class UOTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("uot status %d: %s" % (status, message))
        self.status = status


class _Cost(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("d", ctypes.c_int32), ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("p", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("warm_start", ctypes.c_int32)]


class _Anderson(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("r", ctypes.c_double), ("normalize", ctypes.c_int32)]


class _Phi(ctypes.Structure):
    _fields_ = [("entropy", ctypes.c_int32), ("variant", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("last_change", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("points_form", ctypes.c_int32)]


@dataclass
class Info:
    iters: int
    converged: bool
    last_change: float
    lam: float
    points_form: int = -1  # p = 2 points: 0 expanded form, 1 direct differences, 2 both
    #                        (expanded, then direct to the tolerance); else -1


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libuot.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libuot.so is not built; run `python -m paper_2201_00730_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, S, I32, I64, D = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    CP = ctypes.POINTER(_Cost)
    lib.uot_workspace_bytes.argtypes = [CP, I32]
    lib.uot_workspace_bytes.restype = S
    for name in ("uot_sinkhorn", "uot_ti_sinkhorn"):
        fn = getattr(lib, name)
        fn.argtypes = [CP, P, P, ctypes.POINTER(_Params), P, P, P, S, ctypes.POINTER(_Info), P]
        fn.restype = ctypes.c_int
    for name in ("uot_sinkhorn_anderson", "uot_ti_sinkhorn_anderson"):
        fn = getattr(lib, name)
        fn.argtypes = [CP, P, P, ctypes.POINTER(_Params), ctypes.POINTER(_Anderson), P, P, P, S,
                       ctypes.POINTER(_Info), P]
        fn.restype = ctypes.c_int
    lib.uot_sinkhorn_phi.argtypes = [CP, P, P, ctypes.POINTER(_Params), ctypes.POINTER(_Phi), P, P,
                                     P, S, ctypes.POINTER(_Info), P]
    lib.uot_sinkhorn_phi.restype = ctypes.c_int
    lib.uot_dual_value.argtypes = [CP, P, P, D, D, D, P, P, P, S, ctypes.POINTER(D), P]
    lib.uot_dual_value.restype = ctypes.c_int
    lib.uot_plan_apply.argtypes = [CP, P, P, D, P, P, I32, P, I32, I64, P, I64, P, S, P]
    lib.uot_plan_apply.restype = ctypes.c_int
    lib.uot_backward.argtypes = [CP, P, P, D, D, D, P, P, D, P, P, P, P, P, S, P]
    lib.uot_backward.restype = ctypes.c_int
    lib.uot_backward_noalloc.argtypes = [CP, P, P, D, D, D, P, P, D, P, P, P, P, P]
    lib.uot_backward_noalloc.restype = ctypes.c_int
    lib.uot_status_string.argtypes = [ctypes.c_int]
    lib.uot_status_string.restype = ctypes.c_char_p
    lib.uot_last_error.argtypes = []
    lib.uot_last_error.restype = ctypes.c_char_p
    lib.uot_profile_enable.argtypes = [I32]
    lib.uot_profile_enable.restype = None
    lib.uot_profile_reset.argtypes = []
    lib.uot_profile_reset.restype = None
    lib.uot_profile_read.argtypes = [I32, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.uot_profile_read.restype = I64
    lib.uot_batched_last_plan.argtypes = [ctypes.POINTER(I32), ctypes.POINTER(I32),
                                          ctypes.POINTER(D)]
    lib.uot_batched_last_plan.restype = I32
    lib.uot_batched_autotune_reset.argtypes = []
    lib.uot_batched_autotune_reset.restype = None
    lib.uot_set_autotune.argtypes = [I32]
    lib.uot_set_autotune.restype = I32
    lib.uot_probe_rate.argtypes = [I32, ctypes.POINTER(D), P]
    lib.uot_probe_rate.restype = I32
    lib.uot_set_points_kernel.argtypes = [I32]
    lib.uot_set_points_kernel.restype = I32
    lib.uot_set_grad_kernel.argtypes = [I32]
    lib.uot_set_grad_kernel.restype = I32
    lib.uot_ti_sinkhorn_batched.argtypes = [I32, P, P, I32, D, P, P, P, P, P, P, P, I32, D, I32,
                                            P, P, P, P, P, S, P]
    lib.uot_ti_sinkhorn_batched.restype = ctypes.c_int
    lib.uot_fw1d_batched.argtypes = [I32, P, P, P, P, P, P, P, P, D, I32, I32, D, P, P, P, P, P,
                                     P, S, P]
    lib.uot_fw1d_batched.restype = ctypes.c_int
    lib.uot_fw1d_barycenter.argtypes = [I32, I32, P, P, P, P, P, I32, D, P, P, P, P, P, P, P, S, P]
    lib.uot_fw1d_barycenter.restype = ctypes.c_int
    lib.uot_fw1d_barycenter_workspace_bytes.argtypes = [I32, I32, P]
    lib.uot_fw1d_barycenter_workspace_bytes.restype = S
    lib.uot_fw1d_workspace_bytes.argtypes = [I32, P, P]
    lib.uot_fw1d_workspace_bytes.restype = S
    lib.uot_batched_workspace_bytes.argtypes = [I32, P, P, I32]
    lib.uot_batched_workspace_bytes.restype = S
    lib.uot_batched_set_plan.argtypes = [I32]
    lib.uot_batched_set_plan.restype = I32
    lib.uot_batched_trace_enable.argtypes = [I32]
    lib.uot_batched_trace_enable.restype = None
    lib.uot_batched_trace_read.argtypes = [P, I32]
    lib.uot_batched_trace_read.restype = I32
    _lib = lib
    return lib


def _check(status: int):
    if status != UOT_OK:
        lib = load_library()
        raise UOTError(status, (lib.uot_last_error() or b"").decode() or
                       lib.uot_status_string(status).decode())


def _require_gpu():
    load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the UOT kernels only run on the GPU")


def _f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    return t.contiguous()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _CostRef:
    """A uot_cost struct plus the tensors it points into (kept alive)."""

    def __init__(self, C=None, x=None, y=None, p: float = 2.0):
        s = _Cost()
        self.keep = []
        if C is not None:
            if x is not None or y is not None:
                raise ValueError("give either C or (x, y)")
            C = C if C.stride(-1) == 1 else C.contiguous()
            if C.dim() != 2 or C.dtype != torch.float32 or not C.is_cuda:
                raise ValueError("C must be a 2-D float32 device tensor")
            s.kind, s.n, s.m, s.d = UOT_COST_DENSE, C.shape[0], C.shape[1], 0
            s.C, s.ldc = C.data_ptr(), C.stride(0)
            s.x = s.y = None
            s.p = 1.0
            self.keep.append(C)
        else:
            x, y = _f32(x, "x"), _f32(y, "y")
            if x.dim() == 1:
                x = x[:, None].contiguous()
            if y.dim() == 1:
                y = y[:, None].contiguous()
            if x.shape[1] != y.shape[1]:
                raise ValueError("x and y dimensions differ")
            s.kind, s.n, s.m, s.d = UOT_COST_POINTS, x.shape[0], y.shape[0], x.shape[1]
            s.C, s.ldc = None, 0
            s.x, s.y, s.p = x.data_ptr(), y.data_ptr(), float(p)
            self.keep += [x, y]
        self.s = s

    @property
    def n(self):
        return self.s.n

    @property
    def m(self):
        return self.s.m

    @property
    def device(self):
        return self.keep[0].device


PROFILE_POINTS, PROFILE_DENSE_COLS, PROFILE_DENSE_ROWS, PROFILE_GRAD = 0, 1, 2, 3
PROFILE_POINTS_DIRECT = 4  # points softmin on direct differences (p = 2 direct form, other p)


def profile_enable(on=True, period: int = 1):
    """Time every `period`-th softmin launch of the solvers with HIP events on the call's
    stream (on=False disables)."""
    load_library().uot_profile_enable(int(period) if on else 0)


def profile_reset():
    load_library().uot_profile_reset()


def profile_read(kind: int):
    """(launches, total_ms, total_entries) accumulated for a softmin kernel kind."""
    ms, ent = ctypes.c_double(0.0), ctypes.c_double(0.0)
    n = load_library().uot_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(ent))
    return int(n), ms.value, ent.value


def set_autotune(on: bool) -> bool:
    """Kernel-shape autotuning of the solvers' softmin split counts (on by default); returns
    the previous setting."""
    return bool(load_library().uot_set_autotune(1 if on else 0))


def batched_last_plan():
    """(start level, end level, tau) of this thread's last batched solve under the automatic
    plan (item levels 0, 1, 2: up to 256, 128, 64 targets per item; 3: 64-target items with
    their sources split into ranges of 512), or None."""
    a, b, t = ctypes.c_int32(-1), ctypes.c_int32(-1), ctypes.c_double(-1.0)
    ok = load_library().uot_batched_last_plan(ctypes.byref(a), ctypes.byref(b), ctypes.byref(t))
    return (a.value, b.value, t.value) if ok else None


def batched_autotune_reset():
    """Forget the batched solver's autotuned switch thresholds."""
    load_library().uot_batched_autotune_reset()


PROBE_EXP2, PROBE_FMA32, PROBE_FMA64 = 0, 1, 2
PROBE_MFMA_F64, PROBE_MFMA_F32, PROBE_MFMA_BF16 = 3, 4, 5


def probe_rate(kind: int) -> float:
    """Measured chip-wide rate of one instruction kind on the current device: lane-operations
    per second for PROBE_EXP2 (v_exp_f32), PROBE_FMA32 and PROBE_FMA64; flop/s for the
    matrix-core kinds PROBE_MFMA_F64 (16x16x4 f64), PROBE_MFMA_F32 (16x16x4 f32) and
    PROBE_MFMA_BF16 (32x32x16 bf16)."""
    _require_gpu()
    out = ctypes.c_double(0.0)
    _check(load_library().uot_probe_rate(int(kind), ctypes.byref(out), _stream()))
    return out.value


POINTS_KERNEL_AUTO, POINTS_KERNEL_VALU, POINTS_KERNEL_MFMA_F32, POINTS_KERNEL_MFMA_BF16 = 0, 1, 2, 3
POINTS_KERNEL_DIRECT = 4  # p = 2 through the differences x - y (no expanded-form rounding)


GRAD_KERNEL_MFMA, GRAD_KERNEL_VALU = 0, 1


def set_grad_kernel(variant: int) -> int:
    """Select the backward's per-entry pass for dimensions 1 to 16 (0 matrix cores, the
    default; 1 vector ALU); returns the previous setting."""
    prev = load_library().uot_set_grad_kernel(int(variant))
    if prev < 0:
        raise ValueError("unknown backward kernel variant %r" % (variant,))
    return prev


def set_points_kernel(variant: int) -> int:
    """Select the p = 2 points-softmin implementation (0 auto, 1 VALU, 2 matrix cores on
    the float32 exponent, 3 matrix cores on its bf16 split, 4 VALU on the differences x - y);
    returns the previous setting."""
    prev = load_library().uot_set_points_kernel(int(variant))
    if prev < 0:
        raise ValueError("unknown points kernel variant %r" % (variant,))
    return prev


def workspace_bytes(which: int = UOT_WS_SOLVE, *, C=None, x=None, y=None, p: float = 2.0) -> int:
    lib = load_library()
    cr = _CostRef(C, x, y, p)
    return int(lib.uot_workspace_bytes(ctypes.byref(cr.s), int(which)))


def _workspace(lib, cr: _CostRef, which: int):
    nb = int(lib.uot_workspace_bytes(ctypes.byref(cr.s), int(which)))
    if nb == 0:
        _check(UOT_ERR_INVALID)
    return torch.empty(nb, dtype=torch.uint8, device=cr.device)


def _solve(name: str, alpha, beta, *, C=None, x=None, y=None, p: float = 2.0, eps: float,
           rho1: float, rho2: float | None = None, max_iter: int = 1000, tol: float = 0.0,
           check_every: int = 10, f0=None, workspace=None, anderson=None, phi=None):
    _require_gpu()
    lib = load_library()
    cr = _CostRef(C, x, y, p)
    alpha, beta = _f32(alpha, "alpha"), _f32(beta, "beta")
    if alpha.numel() != cr.n or beta.numel() != cr.m:
        raise ValueError("alpha/beta sizes do not match the cost")
    rho2 = rho1 if rho2 is None else rho2
    f = torch.empty(cr.n, dtype=torch.float32, device=alpha.device)
    g = torch.empty(cr.m, dtype=torch.float32, device=alpha.device)
    if f0 is not None:
        f.copy_(_f32(f0, "f0").reshape(-1))
    prm = _Params(float(eps), float(rho1), float(rho2), int(max_iter), float(tol), int(check_every),
                  int(f0 is not None))
    which = UOT_WS_SOLVE if anderson is None else UOT_WS_ANDERSON
    ws = workspace if workspace is not None else _workspace(lib, cr, which)
    info = _Info()
    args = [ctypes.byref(cr.s), _ptr(alpha), _ptr(beta), ctypes.byref(prm)]
    if anderson is not None:
        args.append(ctypes.byref(_Anderson(int(anderson[0]), float(anderson[1]),
                                           int(bool(anderson[2])))))
    if phi is not None:
        args.append(ctypes.byref(_Phi(int(phi[0]), int(phi[1]))))
    st = getattr(lib, name)(*args, _ptr(f), _ptr(g), _ptr(ws), ws.numel(), ctypes.byref(info),
                            _stream())
    _check(st)
    return f, g, Info(info.iters, bool(info.converged), info.last_change, info.lambda_,
                      info.points_form)


def sinkhorn(alpha, beta, **kw):
    """Plain (F-) Sinkhorn (Sec. 3). Keyword args: C | (x, y, p), eps, rho1, rho2,
    max_iter, tol, check_every, f0. Returns (f, g, Info)."""
    return _solve("uot_sinkhorn", alpha, beta, **kw)


def ti_sinkhorn(alpha, beta, **kw):
    """Translation-invariant (H-) Sinkhorn (Sec. 3, Prop. 4; App. B for rho1 != rho2).
    Returns the translated potentials Phi(fb, gb) = (f, g) and Info."""
    return _solve("uot_ti_sinkhorn", alpha, beta, **kw)


ENTROPIES = {"kl": 0, "berg": 1}
VARIANTS = {"F": 0, "G": 1}


def sinkhorn_phi(alpha, beta, *, entropy: str = "kl", variant: str = "F", **kw):
    """F- or G-Sinkhorn (Sec. 3) with the KL or the Berg entropy for both marginal penalties
    (rho1, rho2 may differ). Other keyword args as ``sinkhorn``. Returns the F-potentials
    (f, g, Info); Info.lam is the last lambda* for G-Sinkhorn."""
    if entropy not in ENTROPIES or variant not in VARIANTS:
        raise ValueError("entropy must be one of %s and variant one of %s"
                         % (sorted(ENTROPIES), sorted(VARIANTS)))
    return _solve("uot_sinkhorn_phi", alpha, beta, phi=(ENTROPIES[entropy], VARIANTS[variant]), **kw)


def sinkhorn_anderson(alpha, beta, *, K: int = 4, r: float = 1e-7, normalize: bool = False, **kw):
    """Plain Sinkhorn with Anderson extrapolation of f every K iterations (appendix on
    Anderson acceleration; the paper's experiment uses K = 4, r = 1e-7). normalize=True
    divides the Gram matrix by its Frobenius norm before adding r. Other keyword args as
    ``sinkhorn``. Returns (f, g, Info)."""
    return _solve("uot_sinkhorn_anderson", alpha, beta, anderson=(K, r, normalize), **kw)


def ti_sinkhorn_anderson(alpha, beta, *, K: int = 4, r: float = 1e-7, normalize: bool = False,
                         **kw):
    """Translation-invariant Sinkhorn with Anderson extrapolation of fb every K iterations
    (normalize as in ``sinkhorn_anderson``). Other keyword args as ``ti_sinkhorn``. Returns
    the translated (f, g, Info)."""
    return _solve("uot_ti_sinkhorn_anderson", alpha, beta, anderson=(K, r, normalize), **kw)


def dual_value(alpha, beta, f, g, *, C=None, x=None, y=None, p: float = 2.0, eps: float,
               rho1: float, rho2: float | None = None) -> float:
    """F_eps(f, g) of the dual problem (eq. dual-uot-kl)."""
    _require_gpu()
    lib = load_library()
    cr = _CostRef(C, x, y, p)
    rho2 = rho1 if rho2 is None else rho2
    alpha, beta, f, g = (_f32(alpha, "alpha"), _f32(beta, "beta"), _f32(f, "f"), _f32(g, "g"))
    ws = _workspace(lib, cr, UOT_WS_DUAL)
    out = ctypes.c_double(0.0)
    _check(lib.uot_dual_value(ctypes.byref(cr.s), _ptr(alpha), _ptr(beta), float(eps), float(rho1),
                              float(rho2), _ptr(f), _ptr(g), _ptr(ws), ws.numel(), ctypes.byref(out),
                              _stream()))
    return out.value


def plan_apply(alpha, beta, f, g, V=None, *, transpose: bool = False, C=None, x=None, y=None,
               p: float = 2.0, eps: float):
    """pi V (or pi^T V) with pi_ij = alpha_i beta_j exp((f_i + g_j - C_ij)/eps); V = None
    applies to a column of ones (the marginals). Returns [rows, k] (or [rows] for V = None
    or a 1-D V)."""
    _require_gpu()
    lib = load_library()
    cr = _CostRef(C, x, y, p)
    alpha, beta, f, g = (_f32(alpha, "alpha"), _f32(beta, "beta"), _f32(f, "f"), _f32(g, "g"))
    rows = cr.m if transpose else cr.n
    squeeze = V is None or V.dim() == 1
    if V is not None:
        V = _f32(V, "V")
        if V.dim() == 1:
            V = V[:, None].contiguous()
        k, ldv = V.shape[1], V.stride(0)
    else:
        k, ldv = 1, 1
    out = torch.empty((rows, k), dtype=torch.float32, device=alpha.device)
    ws = _workspace(lib, cr, UOT_WS_PLAN)
    _check(lib.uot_plan_apply(ctypes.byref(cr.s), _ptr(alpha), _ptr(beta), float(eps), _ptr(f), _ptr(g),
                              int(bool(transpose)), _ptr(V), int(k), int(ldv), _ptr(out), int(k),
                              _ptr(ws), ws.numel(), _stream()))
    return out[:, 0] if squeeze else out


def marginals(alpha, beta, f, g, **kw):
    """(pi 1, pi^T 1)."""
    return (plan_apply(alpha, beta, f, g, None, transpose=False, **kw),
            plan_apply(alpha, beta, f, g, None, transpose=True, **kw))


def backward(alpha, beta, f, g, *, C=None, x=None, y=None, p: float = 2.0, eps: float, rho1: float,
             rho2: float | None = None, grad_out: float = 1.0, need_dx: bool = True,
             need_dy: bool = True, need_dalpha: bool = True, need_dbeta: bool = True):
    """Envelope gradients of UOT at (f, g): returns (dx, dy, dalpha, dbeta), None where not
    requested (dx, dy are None for a dense cost)."""
    _require_gpu()
    lib = load_library()
    cr = _CostRef(C, x, y, p)
    rho2 = rho1 if rho2 is None else rho2
    alpha, beta, f, g = (_f32(alpha, "alpha"), _f32(beta, "beta"), _f32(f, "f"), _f32(g, "g"))
    dev = alpha.device
    pts = cr.s.kind == UOT_COST_POINTS
    dx = torch.empty((cr.n, cr.s.d), dtype=torch.float32, device=dev) if pts and need_dx else None
    dy = torch.empty((cr.m, cr.s.d), dtype=torch.float32, device=dev) if pts and need_dy else None
    da = torch.empty(cr.n, dtype=torch.float32, device=dev) if need_dalpha else None
    db = torch.empty(cr.m, dtype=torch.float32, device=dev) if need_dbeta else None
    ws = _workspace(lib, cr, UOT_WS_BACKWARD)
    _check(lib.uot_backward(ctypes.byref(cr.s), _ptr(alpha), _ptr(beta), float(eps), float(rho1),
                            float(rho2), _ptr(f), _ptr(g), float(grad_out), _ptr(dx), _ptr(dy), _ptr(da),
                            _ptr(db), _ptr(ws), ws.numel(), _stream()))
    return dx, dy, da, db


def backward_noalloc(alpha, beta, f, g, *, C=None, x=None, y=None, p: float = 2.0, eps: float,
                     rho1: float, rho2: float | None = None, grad_out: float = 1.0,
                     need_dx: bool = True, need_dy: bool = True, need_dalpha: bool = True,
                     need_dbeta: bool = True, out=None):
    """backward() through uot_backward_noalloc: no workspace, the library's scratch array.
    out: optional (dx, dy, dalpha, dbeta) tensors to write (None entries are allocated here,
    outside the call, as in backward())."""
    _require_gpu()
    lib = load_library()
    cr = _CostRef(C, x, y, p)
    rho2 = rho1 if rho2 is None else rho2
    alpha, beta, f, g = (_f32(alpha, "alpha"), _f32(beta, "beta"), _f32(f, "f"), _f32(g, "g"))
    dev = alpha.device
    pts = cr.s.kind == UOT_COST_POINTS
    dx, dy, da, db = out if out is not None else (None, None, None, None)
    if dx is None and pts and need_dx:
        dx = torch.empty((cr.n, cr.s.d), dtype=torch.float32, device=dev)
    if dy is None and pts and need_dy:
        dy = torch.empty((cr.m, cr.s.d), dtype=torch.float32, device=dev)
    if da is None and need_dalpha:
        da = torch.empty(cr.n, dtype=torch.float32, device=dev)
    if db is None and need_dbeta:
        db = torch.empty(cr.m, dtype=torch.float32, device=dev)
    _check(lib.uot_backward_noalloc(ctypes.byref(cr.s), _ptr(alpha), _ptr(beta), float(eps),
                                    float(rho1), float(rho2), _ptr(f), _ptr(g), float(grad_out),
                                    _ptr(dx), _ptr(dy), _ptr(da), _ptr(db), _stream()))
    return dx, dy, da, db


BATCH_CONVERGED, BATCH_MAX_ITER, BATCH_INVALID, BATCH_NUMERIC = 0, 1, 2, 3


def ti_sinkhorn_batched(offN, offM, x, y, alpha, beta, eps, rho1, rho2=None, *, p: float = 2.0,
                        max_iter: int = 10000, tol: float = 1e-6, check_every: int = 10,
                        workspace=None):
    """Batched translation-invariant Sinkhorn over packed problems.

    offN, offM: host int64 sequences [B+1] (CSR offsets of the x and y sides); x [sum N, d],
    y [sum M, d], alpha, beta: float32 device tensors; eps, rho1, rho2: float64 device
    tensors [B], host sequences of B values, or scalars (the same for every problem).
    Returns (f, g, iters, status) as device tensors."""
    _require_gpu()
    lib = load_library()
    offN = np.ascontiguousarray(np.asarray(offN, dtype=np.int64))
    offM = np.ascontiguousarray(np.asarray(offM, dtype=np.int64))
    B = len(offN) - 1
    if len(offM) != B + 1:
        raise ValueError("offN and offM lengths differ")
    x, y = _f32(x, "x"), _f32(y, "y")
    if x.dim() == 1:
        x = x[:, None].contiguous()
    if y.dim() == 1:
        y = y[:, None].contiguous()
    alpha, beta = _f32(alpha, "alpha"), _f32(beta, "beta")
    dev = x.device

    def _d64(v):
        if isinstance(v, torch.Tensor):
            return v.to(device=dev, dtype=torch.float64).contiguous()
        return torch.as_tensor(np.asarray(v, dtype=np.float64), device=dev)

    def per_problem(v, name):
        if isinstance(v, torch.Tensor):
            t = v.to(device=dev, dtype=torch.float64).contiguous().reshape(-1)
        elif np.ndim(v) == 0:
            t = torch.full((B,), float(v), dtype=torch.float64, device=dev)
        else:
            t = _d64(v).reshape(-1)
        if t.numel() != B:
            raise ValueError("%s has %d entries, %d problems" % (name, t.numel(), B))
        return t

    if x.shape[0] != offN[-1] or alpha.numel() != offN[-1]:
        raise ValueError("x and alpha must have offN[-1] = %d rows" % int(offN[-1]))
    if y.shape[0] != offM[-1] or beta.numel() != offM[-1]:
        raise ValueError("y and beta must have offM[-1] = %d rows" % int(offM[-1]))
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y dimensions differ")
    eps_t, r1_t = per_problem(eps, "eps"), per_problem(rho1, "rho1")
    r2_t = r1_t if rho2 is None else per_problem(rho2, "rho2")
    f = torch.empty(int(offN[-1]), dtype=torch.float32, device=dev)
    g = torch.empty(int(offM[-1]), dtype=torch.float32, device=dev)
    iters = torch.empty(B, dtype=torch.int32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    pN, pM = offN.ctypes.data_as(ctypes.c_void_p), offM.ctypes.data_as(ctypes.c_void_p)
    if workspace is None:
        nb = int(lib.uot_batched_workspace_bytes(B, pN, pM, x.shape[1]))
        if nb == 0:
            _check(UOT_ERR_INVALID)
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check(lib.uot_ti_sinkhorn_batched(B, pN, pM, x.shape[1], float(p), _ptr(x), _ptr(y), _ptr(alpha),
                                       _ptr(beta), _ptr(eps_t), _ptr(r1_t), _ptr(r2_t), int(max_iter),
                                       float(tol), int(check_every), _ptr(f), _ptr(g), _ptr(iters),
                                       _ptr(status), _ptr(workspace), workspace.numel(), _stream()))
    return f, g, iters, status


BATCH_PLAN_AUTO, BATCH_PLAN_COARSE, BATCH_PLAN_FINE, BATCH_PLAN_SWITCH = 0, 1, 2, 3
BATCH_PLAN_FINEST = 4
BATCH_PLAN_SPLIT = 5  # 64-target items with their sources split into ranges of 512


def batched_set_plan(plan: int) -> int:
    """Work-item plan of the batched solver (see uot_batched_set_plan); returns the previous."""
    prev = load_library().uot_batched_set_plan(int(plan))
    if prev < 0:
        raise ValueError("unknown batched plan %r" % (plan,))
    return prev


def batched_trace(on: bool = True):
    """Enable (or disable) the per-chunk load statistics of the batched solver."""
    load_library().uot_batched_trace_enable(int(bool(on)))


def batched_trace_read():
    """Rows of the last batched solve's trace as a dict of numpy arrays (see
    uot_batched_trace_read)."""
    lib = load_library()
    n = int(lib.uot_batched_trace_read(None, 0))
    buf = np.zeros((max(n, 1), 9), dtype=np.float64)
    lib.uot_batched_trace_read(buf.ctypes.data_as(ctypes.c_void_p), n)
    keys = ("chunk", "fine", "running", "items_g", "items_f", "work", "busy_ticks", "ticks",
            "resident_waves")
    return {k: buf[:n, i].copy() for i, k in enumerate(keys)}


def fw1d_batched(offN, offM, x, y, alpha, beta, rho1, rho2=None, *, p: float = 2.0,
                 line_search: bool = False, max_iter: int = 1000, tol: float = 0.0):
    """Frank-Wolfe for unregularised 1-D KL-UOT (Sec. 4) on B problems with sorted supports
    (see uot_fw1d_batched). offN, offM: host int64 [B+1]; x, y, alpha, beta: float32 device
    [total]; rho1, rho2: float64 device [B] (or scalars). Returns (f, g, iters, gap, status)."""
    _require_gpu()
    lib = load_library()
    offN = np.ascontiguousarray(np.asarray(offN, dtype=np.int64))
    offM = np.ascontiguousarray(np.asarray(offM, dtype=np.int64))
    B = len(offN) - 1
    x, y = _f32(x, "x").reshape(-1), _f32(y, "y").reshape(-1)
    alpha, beta = _f32(alpha, "alpha"), _f32(beta, "beta")
    dev = alpha.device

    def per_problem(v, name):
        if isinstance(v, torch.Tensor):
            return v.to(device=dev, dtype=torch.float64).contiguous().reshape(-1)
        return torch.full((B,), float(v), dtype=torch.float64, device=dev)
    r1 = per_problem(rho1, "rho1")
    r2 = per_problem(rho1 if rho2 is None else rho2, "rho2")
    f = torch.empty(int(offN[-1]), dtype=torch.float32, device=dev)
    g = torch.empty(int(offM[-1]), dtype=torch.float32, device=dev)
    iters = torch.empty(B, dtype=torch.int32, device=dev)
    gap = torch.empty(B, dtype=torch.float64, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    nb = int(lib.uot_fw1d_workspace_bytes(B, offN.ctypes.data, offM.ctypes.data))
    if nb == 0:
        _check(UOT_ERR_INVALID)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    st = lib.uot_fw1d_batched(B, offN.ctypes.data, offM.ctypes.data, _ptr(x), _ptr(y), _ptr(alpha),
                              _ptr(beta), _ptr(r1), _ptr(r2), float(p), int(bool(line_search)),
                              int(max_iter), float(tol), _ptr(f), _ptr(g), _ptr(iters), _ptr(gap),
                              _ptr(status), _ptr(ws), ws.numel(), _stream())
    _check(st)
    return f, g, iters, gap, status


def fw1d_barycenter(off, K: int, x, alpha, w, rho, *, max_iter: int = 1000, tol: float = 0.0):
    """Unregularised 1-D unbalanced barycenters (Sec. 5) of K measures for B problems (see
    uot_fw1d_barycenter). off: host int64 [B*K+1]; x, alpha: float32 device; w: float64
    device [B*K]; rho: float64 device [B] (or a scalar). Returns (f, bary_x, bary_w, iters,
    gap, status); problem b's barycenter starts at off[b*K] - b*K + b."""
    _require_gpu()
    lib = load_library()
    off = np.ascontiguousarray(np.asarray(off, dtype=np.int64))
    B = (len(off) - 1) // K
    x, alpha = _f32(x, "x").reshape(-1), _f32(alpha, "alpha")
    dev = alpha.device
    w = w.to(device=dev, dtype=torch.float64).contiguous().reshape(-1)
    rho = (rho.to(device=dev, dtype=torch.float64).contiguous().reshape(-1)
           if isinstance(rho, torch.Tensor) else torch.full((B,), float(rho), dtype=torch.float64, device=dev))
    tot = int(off[-1])
    f = torch.empty(tot, dtype=torch.float32, device=dev)
    bx = torch.empty(tot - B * K + B, dtype=torch.float32, device=dev)
    bw = torch.empty(tot - B * K + B, dtype=torch.float32, device=dev)
    iters = torch.empty(B, dtype=torch.int32, device=dev)
    gap = torch.empty(B, dtype=torch.float64, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    nb = int(lib.uot_fw1d_barycenter_workspace_bytes(B, K, off.ctypes.data))
    if nb == 0:
        _check(UOT_ERR_INVALID)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    st = lib.uot_fw1d_barycenter(B, K, off.ctypes.data, _ptr(x), _ptr(alpha), _ptr(w), _ptr(rho),
                                 int(max_iter), float(tol), _ptr(f), _ptr(bx), _ptr(bw), _ptr(iters),
                                 _ptr(gap), _ptr(status), _ptr(ws), ws.numel(), _stream())
    _check(st)
    return f, bx, bw, iters, gap, status


def fw1d(x, y, alpha, beta, rho1: float, rho2: float | None = None, **kw):
    """One 1-D problem (sorted supports) by fw1d_batched; returns (f, g, iters, gap, status)."""
    n, m = int(np.prod(tuple(x.shape))), int(np.prod(tuple(y.shape)))
    f, g, it, gap, st = fw1d_batched([0, n], [0, m], x, y, alpha, beta, rho1, rho2, **kw)
    return f, g, int(it[0].item()), float(gap[0].item()), int(st[0].item())


class UOTLoss(torch.autograd.Function):
    """UOT(alpha, beta; x, y) as a differentiable scalar: the forward runs TI Sinkhorn and
    evaluates the dual value; the backward applies the envelope theorem (gradients of
    F_eps at the optimal potentials), with the plan recomputed by the backward kernel."""

    @staticmethod
    def forward(ctx, x, y, alpha, beta, eps, rho1, rho2, p, max_iter, tol, check_every):
        f, g, info = ti_sinkhorn(alpha.detach(), beta.detach(), x=x.detach(), y=y.detach(), p=p,
                                 eps=eps, rho1=rho1, rho2=rho2, max_iter=max_iter, tol=tol,
                                 check_every=check_every)
        val = dual_value(alpha.detach(), beta.detach(), f, g, x=x.detach(), y=y.detach(), p=p,
                         eps=eps, rho1=rho1, rho2=rho2)
        ctx.save_for_backward(x, y, alpha, beta, f, g)
        ctx.cfg = (eps, rho1, rho2, p)
        return torch.tensor(val, dtype=torch.float32, device=x.device)

    @staticmethod
    def backward(ctx, gout):
        x, y, alpha, beta, f, g = ctx.saved_tensors
        eps, rho1, rho2, p = ctx.cfg
        go = float(gout.item())
        dx, dy, da, db = backward(alpha.detach(), beta.detach(), f, g, x=x.detach(), y=y.detach(), p=p,
                                  eps=eps, rho1=rho1, rho2=rho2, grad_out=go,
                                  need_dx=ctx.needs_input_grad[0], need_dy=ctx.needs_input_grad[1],
                                  need_dalpha=ctx.needs_input_grad[2],
                                  need_dbeta=ctx.needs_input_grad[3])
        return dx, dy, da, db, None, None, None, None, None, None, None


def uot_loss(x, y, alpha, beta, *, eps: float, rho1: float, rho2: float | None = None, p: float = 2.0,
             max_iter: int = 10000, tol: float = 1e-6, check_every: int = 10):
    """Differentiable UOT value between point clouds (see UOTLoss)."""
    rho2 = rho1 if rho2 is None else rho2
    return UOTLoss.apply(x, y, alpha, beta, eps, rho1, rho2, p, max_iter, tol, check_every)
