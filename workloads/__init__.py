"""Seeded synthetic inputs for the unbalanced-OT solvers.

This module only draws inputs (point clouds, weights, parameters, and the stored cost
matrix of the dense workload); it holds none of the solver's arithmetic. The GPU tests,
the oracle tests and the benchmark all take their inputs from here, so both sides of
every parity check start from identical float32 arrays (the oracle upcasts them).

Values are drawn in float64 with ``numpy.random.default_rng(seed)`` and rounded once to
float32. The five workloads mirror the experiment settings of the paper (1-D measures of
Sec. 3's empirical study and Sec. 4's comparison with N = M = 200, rho = 1) and the larger
synthetic stand-ins for its GPU runs; the single-cell dataset of the paper is not used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One KL-UOT instance. Either ``C`` (dense, float32 [n, m]) or points ``x`` [n, d],
    ``y`` [m, d] with cost ||x - y||^p. Weights are float32."""
    name: str
    alpha: np.ndarray
    beta: np.ndarray
    eps: float
    rho1: float
    rho2: float
    x: np.ndarray | None = None
    y: np.ndarray | None = None
    p: float = 2.0
    C: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.alpha.shape[0])

    @property
    def m(self) -> int:
        return int(self.beta.shape[0])

    @property
    def d(self) -> int:
        return 0 if self.x is None else int(self.x.shape[1])


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def dense_cost_f32(x: np.ndarray, y: np.ndarray, p: float, rows_per_chunk: int = 1024) -> np.ndarray:
    """Stored cost C_ij = ||x_i - y_j||_2^p evaluated in float64 from the float32 points and
    rounded once to float32 (input preparation for the stored-cost workload)."""
    x64 = x.astype(np.float64)
    y64 = y.astype(np.float64)
    out = np.empty((x.shape[0], y.shape[0]), dtype=np.float32)
    for r0 in range(0, x.shape[0], rows_per_chunk):
        xs = x64[r0:r0 + rows_per_chunk]
        s = np.zeros((xs.shape[0], y64.shape[0]))
        for t in range(x64.shape[1]):
            u = xs[:, t:t + 1] - y64[None, :, t]
            s += u * u
        out[r0:r0 + rows_per_chunk] = (s if p == 2.0 else np.sqrt(s) ** p).astype(np.float32)
    return out


def oned(n: int = 200, m: int = 200, seed: int = 1, eps: float = 1e-2, rho: float = 1.0,
         mass_a: float = 1.0, mass_b: float = 1.5) -> Problem:
    """1-D measures: x ~ U[0,1]; y ~ 0.5 N(0.3, 0.05^2) + 0.5 N(0.7, 0.1^2) clipped to [0, 1];
    uniform weights of masses 1 and 1.5; C = |x - y|^2; eps = 1e-2, rho = 1 (N = M = 200)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=n)
    comp = rng.uniform(size=m) < 0.5
    y = np.where(comp, rng.normal(0.3, 0.05, size=m), rng.normal(0.7, 0.1, size=m))
    y = np.clip(y, 0.0, 1.0)
    return Problem("oned", alpha=_f32(np.full(n, mass_a / n)), beta=_f32(np.full(m, mass_b / m)),
                   eps=eps, rho1=rho, rho2=rho, x=_f32(x[:, None]), y=_f32(y[:, None]), p=2.0,
                   meta={"seed": seed})


CLOUD3D_EPS = (1e-1, 1e-2)
CLOUD3D_RHO = (0.1, 1.0, 10.0)


def cloud3d(n: int = 20000, m: int = 20000, seed: int = 2, eps: float = 1e-2, rho: float = 1.0) -> Problem:
    """3-D clouds: x ~ U[0,1]^3; y ~ N(0.5, 0.15^2 I) (not clipped); alpha uniform of mass 1;
    beta = 2 w / sum w with w ~ LogNormal(0, 0.5); squared Euclidean cost on the fly."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 3))
    y = rng.normal(0.5, 0.15, size=(m, 3))
    w = rng.lognormal(0.0, 0.5, size=m)
    return Problem("cloud3d", alpha=_f32(np.full(n, 1.0 / n)), beta=_f32(2.0 * w / w.sum()),
                   eps=eps, rho1=rho, rho2=rho, x=_f32(x), y=_f32(y), p=2.0, meta={"seed": seed})


def stored8d(n: int = 16384, m: int = 16384, seed: int = 3, eps: float = 5e-3, rho: float = 0.5,
             materialize: bool = True) -> Problem:
    """Stored dense cost: x, y ~ U[0,1]^8, C = ||x - y||^1.5 in float32 (1 GiB at 16384^2);
    uniform weights of masses 1 and 0.7; eps = 5e-3, rho = 0.5."""
    rng = np.random.default_rng(seed)
    x = _f32(rng.uniform(0.0, 1.0, size=(n, 8)))
    y = _f32(rng.uniform(0.0, 1.0, size=(m, 8)))
    C = dense_cost_f32(x, y, 1.5) if materialize else None
    return Problem("stored8d", alpha=_f32(np.full(n, 1.0 / n)), beta=_f32(np.full(m, 0.7 / m)),
                   eps=eps, rho1=rho, rho2=rho, x=x, y=y, p=1.5, C=C, meta={"seed": seed})


def highdim16(n: int = 50000, m: int = 50000, seed: int = 5, eps: float = 0.05, rho: float = 1.0) -> Problem:
    """D = 16 clouds: x ~ N(0, I), y ~ N(0.5 * 1, I); uniform weights of masses 1 and 1.3;
    squared Euclidean cost; eps = 0.05, rho = 1."""
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, 1.0, size=(n, 16))
    y = rng.normal(0.5, 1.0, size=(m, 16))
    return Problem("highdim16", alpha=_f32(np.full(n, 1.0 / n)), beta=_f32(np.full(m, 1.3 / m)),
                   eps=eps, rho1=rho, rho2=rho, x=_f32(x), y=_f32(y), p=2.0, meta={"seed": seed})


def highdim16_subset(k: int = 64) -> Problem:
    """The first k points of each cloud of ``highdim16`` (the same draws), with uniform weights
    of masses 1 and 1.3 on the subset: the finite-difference check of the D = 16 loss."""
    full = highdim16()
    return Problem("highdim16_subset", alpha=_f32(np.full(k, 1.0 / k)),
                   beta=_f32(np.full(k, 1.3 / k)), eps=full.eps, rho1=full.rho1, rho2=full.rho2,
                   x=np.ascontiguousarray(full.x[:k]), y=np.ascontiguousarray(full.y[:k]), p=2.0,
                   meta={"seed": full.meta["seed"], "subset": k})


@dataclass
class Batch:
    """Many independent KL-UOT problems packed back to back (CSR-style offsets)."""
    offN: np.ndarray   # int64 [B+1]
    offM: np.ndarray   # int64 [B+1]
    x: np.ndarray      # float32 [sum N, d]
    y: np.ndarray      # float32 [sum M, d]
    alpha: np.ndarray  # float32 [sum N]
    beta: np.ndarray   # float32 [sum M]
    eps: np.ndarray    # float64 [B]
    rho1: np.ndarray   # float64 [B]
    rho2: np.ndarray   # float64 [B]
    p: float = 2.0

    @property
    def B(self) -> int:
        return int(self.offN.shape[0] - 1)

    def problem(self, b: int) -> Problem:
        n0, n1 = int(self.offN[b]), int(self.offN[b + 1])
        m0, m1 = int(self.offM[b]), int(self.offM[b + 1])
        return Problem("batch[%d]" % b, alpha=self.alpha[n0:n1].copy(), beta=self.beta[m0:m1].copy(),
                       eps=float(self.eps[b]), rho1=float(self.rho1[b]), rho2=float(self.rho2[b]),
                       x=self.x[n0:n1].copy(), y=self.y[m0:m1].copy(), p=self.p)


def batch2d(B: int = 4096, nmin: int = 64, nmax: int = 4096, seed: int = 4,
            eps_range=(1e-3, 1e-1), rho_range=(0.1, 10.0)) -> Batch:
    """B problems with N_p, M_p integer-uniform in [nmin, nmax]; D = 2 points ~ U[0,1]^2;
    uniform weights with masses ~ U[0.5, 2] (independently for alpha and beta); eps and rho
    log-uniform in their ranges; rho1 = rho2."""
    rng = np.random.default_rng(seed)
    N = rng.integers(nmin, nmax + 1, size=B)
    M = rng.integers(nmin, nmax + 1, size=B)
    ma = rng.uniform(0.5, 2.0, size=B)
    mb = rng.uniform(0.5, 2.0, size=B)
    eps = np.exp(rng.uniform(np.log(eps_range[0]), np.log(eps_range[1]), size=B))
    rho = np.exp(rng.uniform(np.log(rho_range[0]), np.log(rho_range[1]), size=B))
    offN = np.concatenate([[0], np.cumsum(N)]).astype(np.int64)
    offM = np.concatenate([[0], np.cumsum(M)]).astype(np.int64)
    x = rng.uniform(0.0, 1.0, size=(int(offN[-1]), 2))
    y = rng.uniform(0.0, 1.0, size=(int(offM[-1]), 2))
    alpha = np.repeat(ma / N, N)
    beta = np.repeat(mb / M, M)
    return Batch(offN=offN, offM=offM, x=_f32(x), y=_f32(y), alpha=_f32(alpha), beta=_f32(beta),
                 eps=eps.astype(np.float64), rho1=rho.astype(np.float64), rho2=rho.astype(np.float64))


def fw1d_batch(B: int = 4096, nmin: int = 64, nmax: int = 4096, seed: int = 6,
               rho_range=(0.1, 10.0)) -> Batch:
    """B 1-D problems for the unregularised Frank-Wolfe solver: N_p, M_p integer-uniform in
    [nmin, nmax]; x ~ U[0,1], y ~ N(0.5, 0.2^2), each sorted ascending within its problem;
    positive random weights (U[0.2, 1] / size) with masses ~ U[0.5, 2]; rho log-uniform,
    rho1 = rho2; eps unused (0)."""
    rng = np.random.default_rng(seed)
    N = rng.integers(nmin, nmax + 1, size=B)
    M = rng.integers(nmin, nmax + 1, size=B)
    ma = rng.uniform(0.5, 2.0, size=B)
    mb = rng.uniform(0.5, 2.0, size=B)
    rho = np.exp(rng.uniform(np.log(rho_range[0]), np.log(rho_range[1]), size=B))
    offN = np.concatenate([[0], np.cumsum(N)]).astype(np.int64)
    offM = np.concatenate([[0], np.cumsum(M)]).astype(np.int64)
    x = np.empty(int(offN[-1]))
    y = np.empty(int(offM[-1]))
    alpha = np.empty(int(offN[-1]))
    beta = np.empty(int(offM[-1]))
    for b in range(B):
        n0, n1, m0, m1 = offN[b], offN[b + 1], offM[b], offM[b + 1]
        x[n0:n1] = np.sort(rng.uniform(0.0, 1.0, size=n1 - n0))
        y[m0:m1] = np.sort(rng.normal(0.5, 0.2, size=m1 - m0))
        wa = rng.uniform(0.2, 1.0, size=n1 - n0)
        wb = rng.uniform(0.2, 1.0, size=m1 - m0)
        alpha[n0:n1] = wa * ma[b] / wa.sum()
        beta[m0:m1] = wb * mb[b] / wb.sum()
    return Batch(offN=offN, offM=offM, x=_f32(x), y=_f32(y), alpha=_f32(alpha), beta=_f32(beta),
                 eps=np.zeros(B), rho1=rho.astype(np.float64), rho2=rho.astype(np.float64))


def bary_mixtures(B: int = 1, K: int = 8, nmin: int = 2000, nmax: int = 2000, seed: int = 7,
                  rho: float = 0.1):
    """Barycenter inputs: B problems of K random mixtures on [0, 1] (two Gaussian components
    with centres ~ U[0.2, 0.8] and std 0.06, clipped), sizes integer-uniform in [nmin, nmax],
    sorted supports, positive random weights with masses ~ U[0.7, 1.4]; uniform barycenter
    weights 1/K; KL penalty rho. Returns (off [B*K+1], x, alpha, w [B*K], rho [B])."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=B * K)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x = np.empty(int(off[-1]))
    a = np.empty(int(off[-1]))
    for m in range(B * K):
        n = int(sizes[m])
        c = rng.uniform(0.2, 0.8, 2)
        comp = rng.integers(0, 2, n)
        x[off[m]:off[m + 1]] = np.sort(np.clip(rng.normal(c[comp], 0.06), 0.0, 1.0))
        wv = rng.uniform(0.2, 1.0, n)
        a[off[m]:off[m + 1]] = wv * rng.uniform(0.7, 1.4) / wv.sum()
    return off, _f32(x), _f32(a), np.full(B * K, 1.0 / K), np.full(B, float(rho))


def random_small(n: int, m: int, d: int = 2, seed: int = 0, eps: float = 0.1, rho1: float = 1.0,
                 rho2: float = 1.0, mass_a: float = 1.0, mass_b: float = 1.5, dense: bool = False,
                 p: float = 2.0, weight_jitter: bool = True) -> Problem:
    """Small random instance for tests: x, y ~ U[0,1]^d; weights positive with the given
    masses (random when ``weight_jitter``); optionally with the cost stored densely."""
    rng = np.random.default_rng(seed)
    x = _f32(rng.uniform(0.0, 1.0, size=(n, d)))
    y = _f32(rng.uniform(0.0, 1.0, size=(m, d)))
    wa = rng.uniform(0.5, 1.5, size=n) if weight_jitter else np.ones(n)
    wb = rng.uniform(0.5, 1.5, size=m) if weight_jitter else np.ones(m)
    pr = Problem("small", alpha=_f32(mass_a * wa / wa.sum()), beta=_f32(mass_b * wb / wb.sum()),
                 eps=eps, rho1=rho1, rho2=rho2, x=x, y=y, p=p, meta={"seed": seed})
    if dense:
        pr.C = dense_cost_f32(x, y, p)
    return pr
