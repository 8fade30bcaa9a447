"""FP64 CPU oracle for entropic KL-unbalanced OT (plain and translation-invariant Sinkhorn).

TEST INFRASTRUCTURE ONLY. Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product library
(``paper_2201_00730_amd``) never imports, links or calls it, and it shares no code
with the GPU path: the arithmetic lives in ``uot_oracle.c`` (plain C, double
precision, built with gcc, no fast-math) and in ``newton.py`` (numpy).

Paper: Sejourne, Vialard, Peyre, "Faster Unbalanced Optimal Transport: Translation
invariant Sinkhorn and 1-D Frank-Wolfe", AISTATS 2022.

Every function takes float64 numpy arrays. Inputs that the GPU path also sees are
generated in float32 and upcast here, so both sides start from the same values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uot_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile ``uot_oracle.c`` into ``liboracle.so`` with gcc (-O2, OpenMP, IEEE math)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cost(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("m", ctypes.c_int), ("d", ctypes.c_int),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_long),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("p", ctypes.c_double)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            D = ctypes.c_double
            I = ctypes.c_int
            CP = ctypes.POINTER(_Cost)
            lib.or_set_threads.argtypes = [I]
            lib.or_set_threads.restype = None
            lib.or_max_threads.argtypes = []
            lib.or_max_threads.restype = I
            lib.or_smin_vec.argtypes = [I, P, P, D]
            lib.or_smin_vec.restype = D
            lib.or_smin_cols.argtypes = [CP, P, P, D, P]
            lib.or_smin_rows.argtypes = [CP, P, P, D, P]
            lib.or_lambda_star.argtypes = [I, I, P, P, P, P, D, D]
            lib.or_lambda_star.restype = D
            lib.or_sinkhorn.argtypes = [CP, P, P, D, D, D, I, I, D, I, I, P, P, P, P, P, P, P]
            lib.or_sinkhorn.restype = I
            lib.or_phistar.argtypes = [I, D, D]
            lib.or_phistar.restype = D
            lib.or_phistar_prime.argtypes = [I, D, D]
            lib.or_phistar_prime.restype = D
            lib.or_dual_update.argtypes = [I, D, D, D]
            lib.or_dual_update.restype = D
            lib.or_lambda_star_div.argtypes = [I, I, I, P, P, P, P, D, D]
            lib.or_lambda_star_div.restype = D
            lib.or_dual_value_div.argtypes = [CP, P, P, D, D, D, I, P, P]
            lib.or_dual_value_div.restype = D
            lib.or_sinkhorn_div.argtypes = [CP, P, P, D, D, D, I, I, I, D, I, P, P, P, P]
            lib.or_sinkhorn_div.restype = I
            lib.or_solve_ot_1d.argtypes = [I, I, P, P, P, P, D, P, P, P, P]
            lib.or_solve_ot_1d.restype = D
            lib.or_h0.argtypes = [I, I, P, P, P, P, D, D, P]
            lib.or_h0.restype = D
            lib.or_fw_1d.argtypes = [I, I, P, P, P, P, D, D, D, I, I, D, P, P, P, P]
            lib.or_fw_1d.restype = I
            lib.or_solve_mot_1d.argtypes = [I, P, P, P, P, P, P, P]
            lib.or_solve_mot_1d.restype = D
            lib.or_mm_lambda.argtypes = [I, P, P, P, P, D, P]
            lib.or_mm_dual.argtypes = [I, P, P, P, P, D]
            lib.or_mm_dual.restype = D
            lib.or_fw_barycenter.argtypes = [I, P, P, P, P, D, I, D, P, P, P, P]
            lib.or_fw_barycenter.restype = I
            lib.or_anderson_mix.argtypes = [I, I, P, D, I, P, P]
            lib.or_anderson_mix.restype = I
            lib.or_sinkhorn_anderson.argtypes = [CP, P, P, D, D, D, I, I, D, I, I, D, I, I, P, P, P,
                                                 P, P]
            lib.or_sinkhorn_anderson.restype = I
            lib.or_plan_apply.argtypes = [CP, P, P, D, P, P, I, P, I, P]
            lib.or_dual_value.argtypes = [CP, P, P, D, D, D, P, P]
            lib.or_dual_value.restype = D
            lib.or_primal_value.argtypes = [CP, P, P, D, D, D, P, P]
            lib.or_primal_value.restype = D
            lib.or_h_value.argtypes = [CP, P, P, D, D, D, P, P]
            lib.or_h_value.restype = D
            lib.or_gradients.argtypes = [CP, P, P, D, D, D, P, P, D, P, P, P, P]
            _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Run the oracle's OpenMP loops on n threads; returns the previous maximum."""
    lib = _load()
    prev = int(lib.or_max_threads())
    lib.or_set_threads(int(n))
    return prev


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Cost:
    """Cost description: a dense matrix ``C`` [n, m], or points ``x`` [n, d], ``y`` [m, d]
    with C_ij = ||x_i - y_j||_2^p (Sec. 1: C_ij = d(x_i, y_j)^p)."""
    C: np.ndarray | None = None
    x: np.ndarray | None = None
    y: np.ndarray | None = None
    p: float = 2.0

    def __post_init__(self):
        if self.C is not None:
            self.C = _f64(self.C)
            if self.C.ndim != 2:
                raise ValueError("C must be 2-D")
        else:
            if self.x is None or self.y is None:
                raise ValueError("give C or both x and y")
            self.x = _f64(self.x)
            self.y = _f64(self.y)
            if self.x.ndim == 1:
                self.x = self.x[:, None].copy()
            if self.y.ndim == 1:
                self.y = self.y[:, None].copy()
            if self.x.shape[1] != self.y.shape[1]:
                raise ValueError("x and y must share their dimension")

    @property
    def n(self) -> int:
        return self.C.shape[0] if self.C is not None else self.x.shape[0]

    @property
    def m(self) -> int:
        return self.C.shape[1] if self.C is not None else self.y.shape[0]

    @property
    def d(self) -> int:
        return 0 if self.C is not None else self.x.shape[1]

    def _struct(self) -> _Cost:
        s = _Cost()
        s.n, s.m, s.d = self.n, self.m, self.d
        if self.C is not None:
            s.C, s.ldc = _ptr(self.C), self.C.shape[1]
            s.x = s.y = None
            s.p = 0.0
        else:
            s.C, s.ldc = None, 0
            s.x, s.y, s.p = _ptr(self.x), _ptr(self.y), float(self.p)
        return s

    def dense(self) -> np.ndarray:
        """The full FP64 cost matrix (only for small problems)."""
        if self.C is not None:
            return self.C
        diff = self.x[:, None, :] - self.y[None, :, :]
        s = np.sum(diff * diff, axis=-1)
        return s if self.p == 2.0 else np.sqrt(s) ** self.p


def _logw(w: np.ndarray) -> np.ndarray:
    with np.errstate(divide="ignore"):
        return np.log(w)


def smin_vec(w, h, s: float) -> float:
    """Softmin of Sec. 3 on a vector: Smin_w^s(h) = -s log sum_k w_k exp(-h_k/s)."""
    w, h = _f64(w), _f64(h)
    lw = _logw(w)
    return _load().or_smin_vec(len(w), _ptr(lw), _ptr(h), float(s))


def smin_cols(cost: Cost, alpha, h, eps: float) -> np.ndarray:
    """out_j = Smin_alpha^eps(C_{:,j} - h) = -eps log sum_i alpha_i exp((h_i - C_ij)/eps)."""
    la, h = _logw(_f64(alpha)), _f64(h)
    out = np.empty(cost.m)
    cs = cost._struct()
    _load().or_smin_cols(ctypes.byref(cs), _ptr(la), _ptr(h), float(eps), _ptr(out))
    return out


def smin_rows(cost: Cost, beta, h, eps: float) -> np.ndarray:
    """out_i = Smin_beta^eps(C_{i,:} - h) = -eps log sum_j beta_j exp((h_j - C_ij)/eps)."""
    lb, h = _logw(_f64(beta)), _f64(h)
    out = np.empty(cost.n)
    cs = cost._struct()
    _load().or_smin_rows(ctypes.byref(cs), _ptr(lb), _ptr(h), float(eps), _ptr(out))
    return out


def lambda_star(alpha, beta, fb, gb, rho1: float, rho2: float) -> float:
    """Optimal translation of Prop. 2, lambda* = tau1 Smin_beta^rho2(gb) - tau2 Smin_alpha^rho1(fb)."""
    la, lb = _logw(_f64(alpha)), _logw(_f64(beta))
    fb, gb = _f64(fb), _f64(gb)
    return _load().or_lambda_star(len(la), len(lb), _ptr(la), _ptr(lb), _ptr(fb), _ptr(gb),
                                  float(rho1), float(rho2))


@dataclass
class SinkhornResult:
    f: np.ndarray
    g: np.ndarray
    iters: int
    last_delta: float
    lam: float
    hist_delta: np.ndarray | None = None
    hist_f: np.ndarray | None = None
    hist_g: np.ndarray | None = None


def sinkhorn(cost: Cost, alpha, beta, eps: float, rho1: float, rho2: float, *, ti: bool,
             max_iter: int, tol: float = 0.0, check_every: int = 1, f0=None,
             history: bool = False, history_potentials: bool = False) -> SinkhornResult:
    """Plain (F-) Sinkhorn of Sec. 3 (``ti=False``) or H-Sinkhorn of Prop. 4 / App. B
    (``ti=True``); returns the translated potentials Phi(fb, gb) for TI.

    One iteration = a g-step then an f-step, from f_0 = 0 (or ``f0``). With ``tol > 0`` it
    stops at the first iteration t with t % check_every == 0 and
    max(||f_t - f_{t-1}||_inf, ||g_t - g_{t-1}||_inf) < tol.
    """
    alpha, beta = _f64(alpha), _f64(beta)
    n, m = cost.n, cost.m
    if alpha.shape != (n,) or beta.shape != (m,):
        raise ValueError("alpha/beta shape mismatch")
    f = _f64(f0).copy() if f0 is not None else np.zeros(n)
    g = np.zeros(m)
    lam = ctypes.c_double(0.0)
    last = ctypes.c_double(0.0)
    hd = np.empty(max_iter) if history else None
    hf = np.empty((max_iter, n)) if history_potentials else None
    hg = np.empty((max_iter, m)) if history_potentials else None
    cs = cost._struct()
    it = _load().or_sinkhorn(ctypes.byref(cs), _ptr(alpha), _ptr(beta), float(eps), float(rho1),
                             float(rho2), int(bool(ti)), int(max_iter), float(tol), int(check_every),
                             int(f0 is not None), _ptr(f), _ptr(g), ctypes.byref(lam),
                             ctypes.byref(last), _ptr(hd), _ptr(hf), _ptr(hg))
    return SinkhornResult(f=f, g=g, iters=it, last_delta=last.value, lam=lam.value,
                          hist_delta=None if hd is None else hd[:it].copy(),
                          hist_f=None if hf is None else hf[:it].copy(),
                          hist_g=None if hg is None else hg[:it].copy())


def anderson_mix(X, r: float, normalize: bool = False):
    """Anderson extrapolation of the appendix on accelerating Sinkhorn: rows of X are the
    iterates x_0 .. x_K of a map (x_{k+1} = T(x_k)); the residuals x_{k+1} - x_k form U;
    c = (G + rI)^{-1} 1 / (1^T (G + rI)^{-1} 1) with G = U^T U (normalize=True: G divided
    by its Frobenius norm first); returns (c, sum_k c_k x_{k+1})."""
    X = np.ascontiguousarray(_f64(X))
    K = X.shape[0] - 1
    c = np.empty(K)
    out = np.empty(X.shape[1])
    if _load().or_anderson_mix(X.shape[1], K, _ptr(X), float(r), int(bool(normalize)), _ptr(c),
                               _ptr(out)) != 0:
        raise ValueError("singular Anderson system")
    return c, out


def sinkhorn_anderson(cost: Cost, alpha, beta, eps: float, rho1: float, rho2: float, *, ti: bool,
                      K: int, r: float, max_iter: int, tol: float = 0.0, check_every: int = 1,
                      f0=None, history: bool = False, normalize: bool = False) -> SinkhornResult:
    """``sinkhorn`` with Anderson extrapolation of f (plain) or fb (TI) every K iterations
    (see ``anderson_mix``, including ``normalize``); the change is +inf at the first
    iteration after an extrapolation."""
    alpha, beta = _f64(alpha), _f64(beta)
    n, m = cost.n, cost.m
    if alpha.shape != (n,) or beta.shape != (m,):
        raise ValueError("alpha/beta shape mismatch")
    f = _f64(f0).copy() if f0 is not None else np.zeros(n)
    g = np.zeros(m)
    lam = ctypes.c_double(0.0)
    last = ctypes.c_double(0.0)
    hd = np.empty(max_iter) if history else None
    cs = cost._struct()
    it = _load().or_sinkhorn_anderson(ctypes.byref(cs), _ptr(alpha), _ptr(beta), float(eps),
                                      float(rho1), float(rho2), int(bool(ti)), int(K), float(r),
                                      int(bool(normalize)), int(max_iter), float(tol), int(check_every),
                                      int(f0 is not None), _ptr(f), _ptr(g), ctypes.byref(lam),
                                      ctypes.byref(last), _ptr(hd))
    if it < 0:
        raise ValueError("K must be in 1..16")
    return SinkhornResult(f=f, g=g, iters=it, last_delta=last.value, lam=lam.value,
                          hist_delta=None if hd is None else hd[:it].copy())


DIVERGENCES = {"kl": 0, "berg": 1}


def _div(div) -> int:
    if div not in DIVERGENCES:
        raise ValueError("divergence must be one of %s" % sorted(DIVERGENCES))
    return DIVERGENCES[div]


def phistar(div: str, rho: float, x: float) -> float:
    """phi*(x): KL rho (e^{x/rho} - 1); Berg -rho log(1 - x/rho) (x < rho)."""
    return _load().or_phistar(_div(div), float(rho), float(x))


def phistar_prime(div: str, rho: float, x: float) -> float:
    return _load().or_phistar_prime(_div(div), float(rho), float(x))


def dual_update(div: str, rho: float, eps: float, S: float) -> float:
    """g = -aprox_{phi*}(-S): the root of e^{(g - S)/eps} = phi*'(-g) (Sec. 3)."""
    return _load().or_dual_update(_div(div), float(rho), float(eps), float(S))


def lambda_star_div(div: str, alpha, beta, fb, gb, rho1: float, rho2: float) -> float:
    """lambda*(fb, gb): root of <alpha, phi1*'(-fb - l)> = <beta, phi2*'(-gb + l)>."""
    a, b, fb, gb = _f64(alpha), _f64(beta), _f64(fb), _f64(gb)
    return _load().or_lambda_star_div(_div(div), len(a), len(b), _ptr(a), _ptr(b), _ptr(fb),
                                      _ptr(gb), float(rho1), float(rho2))


def dual_value_div(cost: Cost, alpha, beta, eps, rho1, rho2, div: str, f, g) -> float:
    """F_eps(f, g) with the entropy's phi*."""
    a, b, f, g = _f64(alpha), _f64(beta), _f64(f), _f64(g)
    cs = cost._struct()
    return _load().or_dual_value_div(ctypes.byref(cs), _ptr(a), _ptr(b), float(eps), float(rho1),
                                     float(rho2), _div(div), _ptr(f), _ptr(g))


def sinkhorn_div(cost: Cost, alpha, beta, eps: float, rho1: float, rho2: float, *, div: str,
                 variant: str, max_iter: int, tol: float = 0.0,
                 check_every: int = 1) -> SinkhornResult:
    """F-Sinkhorn (``variant="F"``) or G-Sinkhorn (``"G"``) of Sec. 3 for the entropy ``div``
    ("kl" or "berg"), from zero potentials; G reports (fb + lambda, gb - lambda)."""
    if variant not in ("F", "G"):
        raise ValueError("variant must be F or G")
    alpha, beta = _f64(alpha), _f64(beta)
    f, g = np.empty(cost.n), np.empty(cost.m)
    lam, last = ctypes.c_double(0.0), ctypes.c_double(0.0)
    cs = cost._struct()
    it = _load().or_sinkhorn_div(ctypes.byref(cs), _ptr(alpha), _ptr(beta), float(eps), float(rho1),
                                 float(rho2), _div(div), int(variant == "G"), int(max_iter),
                                 float(tol), int(check_every), _ptr(f), _ptr(g), ctypes.byref(lam),
                                 ctypes.byref(last))
    return SinkhornResult(f=f, g=g, iters=it, last_delta=last.value, lam=lam.value)


def solve_ot_1d(x, y, a, b, p: float):
    """Balanced 1-D OT between sorted supports (Sec. 4, the linear oracle of Frank-Wolfe):
    monotone coupling and its complementary-slackness dual. Returns (cost, r, s, cells, mass)."""
    x, y, a, b = _f64(x), _f64(y), _f64(a), _f64(b)
    n, m = len(x), len(y)
    r, s = np.empty(n), np.empty(m)
    cells = np.empty(2 * (n + m - 1), dtype=np.int32)
    mass = np.empty(n + m - 1)
    cost = _load().or_solve_ot_1d(n, m, _ptr(x), _ptr(y), _ptr(a), _ptr(b), float(p), _ptr(r),
                                  _ptr(s), cells.ctypes.data_as(ctypes.c_void_p), _ptr(mass))
    return cost, r, s, cells.reshape(-1, 2), mass


def h0(alpha, beta, fb, gb, rho1: float, rho2: float):
    """H_0(fb, gb) = F_0(fb + lambda*, gb - lambda*) for KL; returns (value, lambda*)."""
    a, b, fb, gb = _f64(alpha), _f64(beta), _f64(fb), _f64(gb)
    lam = ctypes.c_double(0.0)
    v = _load().or_h0(len(a), len(b), _ptr(a), _ptr(b), _ptr(fb), _ptr(gb), float(rho1),
                      float(rho2), ctypes.byref(lam))
    return v, lam.value


@dataclass
class FWResult:
    f: np.ndarray
    g: np.ndarray
    iters: int
    gap: float
    hist_gap: np.ndarray | None = None


def fw_1d(x, y, alpha, beta, rho1: float, rho2: float, *, p: float = 2.0,
          line_search: bool = False, max_iter: int = 1000, tol: float = 0.0,
          history: bool = False) -> FWResult:
    """Frank-Wolfe on H_0 for 1-D KL-UOT with eps = 0 (Sec. 4) on sorted supports; step
    2/(2+t) or line search. Returns the reported potentials (fb + lambda*, gb - lambda*)."""
    x, y, a, b = _f64(x), _f64(y), _f64(alpha), _f64(beta)
    n, m = len(x), len(y)
    f, g = np.empty(n), np.empty(m)
    gap = ctypes.c_double(0.0)
    hg = np.empty(max_iter) if history else None
    it = _load().or_fw_1d(n, m, _ptr(x), _ptr(y), _ptr(a), _ptr(b), float(rho1), float(rho2),
                          float(p), int(bool(line_search)), int(max_iter), float(tol), _ptr(f),
                          _ptr(g), ctypes.byref(gap), _ptr(hg))
    return FWResult(f=f, g=g, iters=it, gap=gap.value,
                    hist_gap=None if hg is None else hg[:it].copy())


def _off(off):
    return np.ascontiguousarray(np.asarray(off, dtype=np.int64))


def solve_mot_1d(off, x, a, w):
    """Balanced 1-D multi-marginal OT (Sec. 5), squared distance, measures k on
    [off[k], off[k+1]) with sorted supports and equal masses: returns (cost, f, bary_x, bary_m)."""
    off, x, a, w = _off(off), _f64(x), _f64(a), _f64(w)
    K = len(off) - 1
    f = np.empty(int(off[-1]))
    nb = int(off[-1]) - K + 1
    bx, bm = np.empty(nb), np.empty(nb)
    cost = _load().or_solve_mot_1d(K, off.ctypes.data_as(ctypes.c_void_p), _ptr(x), _ptr(a), _ptr(w),
                                   _ptr(f), _ptr(bx), _ptr(bm))
    return cost, f, bx, bm


def mm_lambda(off, a, fb, w, rho: float) -> np.ndarray:
    """Closed-form optimal translation of the multi-marginal dual (KL, Sec. 5)."""
    off, a, fb, w = _off(off), _f64(a), _f64(fb), _f64(w)
    lam = np.empty(len(off) - 1)
    _load().or_mm_lambda(len(off) - 1, off.ctypes.data_as(ctypes.c_void_p), _ptr(a), _ptr(fb),
                         _ptr(w), float(rho), _ptr(lam))
    return lam


def mm_dual(off, a, f, w, rho: float) -> float:
    off, a, f, w = _off(off), _f64(a), _f64(f), _f64(w)
    return _load().or_mm_dual(len(off) - 1, off.ctypes.data_as(ctypes.c_void_p), _ptr(a), _ptr(f),
                              _ptr(w), float(rho))


@dataclass
class BarycenterResult:
    f: np.ndarray
    bary_x: np.ndarray
    bary_m: np.ndarray
    iters: int
    gap: float


def fw_barycenter(off, x, a, w, rho: float, *, max_iter: int = 1000, tol: float = 0.0) -> BarycenterResult:
    """Frank-Wolfe on the translation-invariant multi-marginal dual (Sec. 5): unbalanced 1-D
    barycenter of K measures (sorted supports), KL penalty rho, weights w; step 2/(2+t)."""
    off, x, a, w = _off(off), _f64(x), _f64(a), _f64(w)
    K = len(off) - 1
    f = np.empty(int(off[-1]))
    nb = int(off[-1]) - K + 1
    bx, bm = np.empty(nb), np.empty(nb)
    gap = ctypes.c_double(0.0)
    it = _load().or_fw_barycenter(K, off.ctypes.data_as(ctypes.c_void_p), _ptr(x), _ptr(a), _ptr(w),
                                  float(rho), int(max_iter), float(tol), _ptr(f), _ptr(bx), _ptr(bm),
                                  ctypes.byref(gap))
    return BarycenterResult(f=f, bary_x=bx, bary_m=bm, iters=it, gap=gap.value)


def plan_apply(cost: Cost, alpha, beta, eps: float, f, g, V, transpose: bool = False) -> np.ndarray:
    """out = pi V (or pi^T V) with pi_ij = alpha_i beta_j exp((f_i + g_j - C_ij)/eps)."""
    alpha, beta, f, g = _f64(alpha), _f64(beta), _f64(f), _f64(g)
    V = _f64(V)
    squeeze = V.ndim == 1
    if squeeze:
        V = V[:, None].copy()
    rows = cost.m if transpose else cost.n
    out = np.empty((rows, V.shape[1]))
    cs = cost._struct()
    _load().or_plan_apply(ctypes.byref(cs), _ptr(alpha), _ptr(beta), float(eps), _ptr(f), _ptr(g),
                          int(bool(transpose)), _ptr(V), V.shape[1], _ptr(out))
    return out[:, 0] if squeeze else out


def marginals(cost: Cost, alpha, beta, eps: float, f, g):
    """(pi_1, pi_2) = (pi 1, pi^T 1)."""
    return (plan_apply(cost, alpha, beta, eps, f, g, np.ones(cost.m)),
            plan_apply(cost, alpha, beta, eps, f, g, np.ones(cost.n), transpose=True))


def dual_value(cost: Cost, alpha, beta, eps, rho1, rho2, f, g) -> float:
    """F_eps(f, g) of eq. (dual-uot-kl) with rho KL penalties."""
    cs = cost._struct()
    a, b, f, g = _f64(alpha), _f64(beta), _f64(f), _f64(g)
    return _load().or_dual_value(ctypes.byref(cs), _ptr(a), _ptr(b), float(eps), float(rho1),
                                 float(rho2), _ptr(f), _ptr(g))


def primal_value(cost: Cost, alpha, beta, eps, rho1, rho2, f, g) -> float:
    """Primal objective of eq. (primal-uot-kl) at the plan built from (f, g)."""
    cs = cost._struct()
    a, b, f, g = _f64(alpha), _f64(beta), _f64(f), _f64(g)
    return _load().or_primal_value(ctypes.byref(cs), _ptr(a), _ptr(b), float(eps), float(rho1),
                                   float(rho2), _ptr(f), _ptr(g))


def h_value(cost: Cost, alpha, beta, eps, rho1, rho2, fb, gb) -> float:
    """Translation-invariant dual H_eps(fb, gb) of Prop. 3."""
    cs = cost._struct()
    a, b, fb, gb = _f64(alpha), _f64(beta), _f64(fb), _f64(gb)
    return _load().or_h_value(ctypes.byref(cs), _ptr(a), _ptr(b), float(eps), float(rho1),
                              float(rho2), _ptr(fb), _ptr(gb))


def gradients(cost: Cost, alpha, beta, eps, rho1, rho2, f, g, gout: float = 1.0):
    """Envelope gradients (dx, dy, dalpha, dbeta) of UOT at optimal (f, g), scaled by gout.
    dx/dy are None for a dense cost."""
    cs = cost._struct()
    a, b, f, g = _f64(alpha), _f64(beta), _f64(f), _f64(g)
    da = np.empty(cost.n)
    db = np.empty(cost.m)
    dx = np.empty((cost.n, cost.d)) if cost.d else None
    dy = np.empty((cost.m, cost.d)) if cost.d else None
    _load().or_gradients(ctypes.byref(cs), _ptr(a), _ptr(b), float(eps), float(rho1), float(rho2),
                         _ptr(f), _ptr(g), float(gout), _ptr(dx), _ptr(dy), _ptr(da), _ptr(db))
    return dx, dy, da, db


def hilbert_norm(v) -> float:
    """Hilbert pseudo-norm ||v||_star = (max v - min v)/2 (App. B, closed form lemma)."""
    v = _f64(v)
    return 0.5 * (float(v.max()) - float(v.min()))


def empirical_rate(hist_f: np.ndarray, f_star: np.ndarray, floor: float = 1e-13) -> float:
    """Rate estimator of Sec. 3 (empirical study): exp of the median over t of
    log||f_{t+1} - f*||_inf - log||f_t - f*||_inf, over iterates whose error is above ``floor``."""
    err = np.max(np.abs(hist_f - f_star[None, :]), axis=1)
    keep = err > floor
    err = err[keep]
    if len(err) < 3:
        raise ValueError("not enough iterates above the floor")
    return float(np.exp(np.median(np.diff(np.log(err)))))


from .newton import newton_dual  # noqa: E402  (numpy-only, no dependency on the C library)

__all__ = ["build", "Cost", "smin_vec", "smin_cols", "smin_rows", "lambda_star", "sinkhorn",
           "SinkhornResult", "plan_apply", "marginals", "dual_value", "primal_value", "h_value",
           "gradients", "hilbert_norm", "empirical_rate", "newton_dual"]
