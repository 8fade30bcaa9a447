"""Dense Newton ascent on the concave dual F_eps for tiny problems (test infrastructure only).

This is a second, independent way to reach the optimum of eq. (dual-uot-kl): it never
calls a softmin or a Sinkhorn update, it maximises F_eps(f, g) over R^{n+m} directly with
its exact gradient and Hessian and a backtracking line search. F_eps is strictly concave
for rho KL penalties (its Hessian below is negative definite when all weights are
positive), so the maximiser is unique (Sec. 1: unique dual maximisers when phi* is strictly
convex).

  F(f, g) = rho1 <alpha, 1 - e^{-f/rho1}> + rho2 <beta, 1 - e^{-g/rho2}>
            - eps <alpha x beta, e^{(f + g - C)/eps} - 1>
  dF/df_i = alpha_i e^{-f_i/rho1} - pi1_i,          pi_ij = alpha_i beta_j e^{(f_i+g_j-C_ij)/eps}
  dF/dg_j = beta_j e^{-g_j/rho2} - pi2_j
  d2F/df_i^2 = -alpha_i e^{-f_i/rho1}/rho1 - pi1_i/eps,  d2F/df_i dg_j = -pi_ij/eps,
  d2F/dg_j^2 = -beta_j e^{-g_j/rho2}/rho2 - pi2_j/eps,   other entries 0.
"""
from __future__ import annotations

import numpy as np


def _value(C, a, b, eps, r1, r2, f, g):
    with np.errstate(over="ignore", invalid="ignore"):
        pi = a[:, None] * b[None, :] * np.exp((f[:, None] + g[None, :] - C) / eps)
        v = (r1 * np.sum(a * (1.0 - np.exp(-f / r1))) + r2 * np.sum(b * (1.0 - np.exp(-g / r2)))
             - eps * (np.sum(pi) - np.sum(a) * np.sum(b)))
    return v if np.isfinite(v) else -np.inf


def newton_dual(C, alpha, beta, eps: float, rho1: float, rho2: float, *, tol: float = 1e-14,
                max_iter: int = 500):
    """Maximise F_eps by Newton's method from (0, 0). Returns (f, g, grad_inf_norm, iters)."""
    C = np.asarray(C, dtype=np.float64)
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    n, m = C.shape
    if np.any(a <= 0) or np.any(b <= 0):
        raise ValueError("dense Newton needs strictly positive weights")
    f = np.zeros(n)
    g = np.zeros(m)
    gn = np.inf
    for it in range(1, max_iter + 1):
        pi = a[:, None] * b[None, :] * np.exp((f[:, None] + g[None, :] - C) / eps)
        p1, p2 = pi.sum(axis=1), pi.sum(axis=0)
        ea, eb = a * np.exp(-f / rho1), b * np.exp(-g / rho2)
        grad = np.concatenate([ea - p1, eb - p2])
        gn = float(np.max(np.abs(grad)))
        if gn < tol:
            return f, g, gn, it
        H = np.zeros((n + m, n + m))
        H[np.arange(n), np.arange(n)] = -ea / rho1 - p1 / eps
        H[n + np.arange(m), n + np.arange(m)] = -eb / rho2 - p2 / eps
        H[:n, n:] = -pi / eps
        H[n:, :n] = -pi.T / eps
        step = np.linalg.solve(H, -grad)  # ascent direction for concave F
        v0 = _value(C, a, b, eps, rho1, rho2, f, g)
        slope = float(grad @ step)
        t = 1.0
        while t > 1e-12:
            fn, gn_ = f + t * step[:n], g + t * step[n:]
            if _value(C, a, b, eps, rho1, rho2, fn, gn_) >= v0 + 1e-4 * t * slope - 1e-15 * abs(v0):
                break
            t *= 0.5
        f, g = f + t * step[:n], g + t * step[n:]
    return f, g, gn, max_iter
