"""Pins of the FP64 oracle to what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: a closed form, a second
independent algorithm (dense Newton), an exact identity the paper proves, a limit case
reducing to a textbook routine, or a finite-difference derivative. Together they are
chosen so that a dropped term, a wrong sign, a swapped rho or a transposed operand in the
oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.helpers import oracle_cost, rel_inf

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _solve(cost, a, b, eps, r1, r2, ti=True, tol=1e-14, max_iter=200000, **kw):
    return oracle.sinkhorn(cost, a, b, eps, r1, r2, ti=ti, max_iter=max_iter, tol=tol,
                           check_every=1, **kw)


# ---------------------------------------------------------------------------------------
# P9: N = M = 1 closed form. Minimising the primal of eq. (primal-uot-kl) over a scalar
# pi >= 0 gives (eps + rho1 + rho2) log pi = (eps + rho1) log a + (eps + rho2) log b - c;
# the optimality condition pi_1 = a e^{-f/rho1} gives f = -rho1 log(pi/a) (and g alike);
# substituting the first-order condition into the primal gives
# UOT = rho1 (a - pi) + rho2 (b - pi) + eps (a b - pi).
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("ti", [False, True])
@pytest.mark.parametrize("a,b,c,eps,r1,r2", [
    (0.7, 1.9, 0.3, 0.1, 1.0, 2.5),
    (1.0, 1.5, 2.0, 0.5, 0.2, 0.2),
    (2.0, 0.3, 0.0, 0.05, 3.0, 0.7),
])
def test_p9_one_point_closed_form(ti, a, b, c, eps, r1, r2):
    pi = math.exp(((eps + r1) * math.log(a) + (eps + r2) * math.log(b) - c) / (eps + r1 + r2))
    f_cf = -r1 * math.log(pi / a)
    g_cf = -r2 * math.log(pi / b)
    val_cf = r1 * (a - pi) + r2 * (b - pi) + eps * (a * b - pi)
    cost = oracle.Cost(C=np.array([[c]]))
    r = _solve(cost, [a], [b], eps, r1, r2, ti=ti)
    assert abs(r.f[0] - f_cf) <= 1e-12 * max(1.0, abs(f_cf))
    assert abs(r.g[0] - g_cf) <= 1e-12 * max(1.0, abs(g_cf))
    assert abs(oracle.dual_value(cost, [a], [b], eps, r1, r2, r.f, r.g) - val_cf) <= 1e-12
    assert abs(oracle.primal_value(cost, [a], [b], eps, r1, r2, r.f, r.g) - val_cf) <= 1e-12


# ---------------------------------------------------------------------------------------
# P10: tiny problems, Sinkhorn fixed point == dense Newton maximiser of F_eps.
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("n,m", [(1, 2), (2, 1), (2, 3), (3, 5), (5, 4), (8, 7), (8, 8)])
@pytest.mark.parametrize("ti", [False, True])
def test_p10_newton_matches_sinkhorn(n, m, ti):
    rng = np.random.default_rng(100 * n + m)
    C = rng.uniform(0.0, 2.0, size=(n, m))  # not symmetric, not square: catches transposes
    a = rng.uniform(0.2, 1.0, size=n)
    b = rng.uniform(0.2, 1.5, size=m)
    eps, r1, r2 = 0.3, 0.7, 2.0  # rho1 != rho2: catches a swapped penalty
    fN, gN, gradn, _ = oracle.newton_dual(C, a, b, eps, r1, r2)
    assert gradn < 1e-13
    r = _solve(oracle.Cost(C=C), a, b, eps, r1, r2, ti=ti)
    assert np.max(np.abs(r.f - fN)) < 1e-11
    assert np.max(np.abs(r.g - gN)) < 1e-11


# ---------------------------------------------------------------------------------------
# P1 (same fixed point, Thm. of App. B), P2 (marginals at optimum), P3 (zero duality gap).
# ---------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def medium():
    pr = workloads.random_small(37, 29, d=2, seed=7, eps=0.05, rho1=0.4, rho2=1.7,
                                mass_a=1.0, mass_b=1.6)
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    plain = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=False)
    ti = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True)
    return pr, cost, a, b, plain, ti


def test_p1_plain_and_ti_same_fixed_point(medium):
    pr, cost, a, b, plain, ti = medium
    assert plain.last_delta < 1e-14 and ti.last_delta < 1e-14
    assert np.max(np.abs(plain.f - ti.f)) < 1e-12
    assert np.max(np.abs(plain.g - ti.g)) < 1e-12
    assert ti.iters < plain.iters  # TI is faster (Thm. 1)


def test_p2_marginals_at_optimum(medium):
    pr, cost, a, b, plain, ti = medium
    p1, p2 = oracle.marginals(cost, a, b, pr.eps, ti.f, ti.g)
    assert np.max(np.abs(p1 - a * np.exp(-ti.f / pr.rho1))) < 1e-13
    assert np.max(np.abs(p2 - b * np.exp(-ti.g / pr.rho2))) < 1e-13


def test_p3_zero_duality_gap(medium):
    pr, cost, a, b, plain, ti = medium
    P = oracle.primal_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti.f, ti.g)
    F = oracle.dual_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti.f, ti.g)
    assert P - F > -1e-12
    assert P - F < 1e-12
    # a non-optimal pair leaves a strictly positive gap
    F0 = oracle.dual_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti.f + 0.05, ti.g)
    P0 = oracle.primal_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti.f + 0.05, ti.g)
    assert P0 - F0 > 1e-6


def test_p3_monotone_dual_along_iterates():
    """Both algorithms are exact block maximisations: F increases along plain iterates, and
    H = F o Phi increases along TI iterates (Sec. 3)."""
    pr = workloads.random_small(12, 9, d=2, seed=3, eps=0.05, rho1=1.0, rho2=0.5)
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    for ti in (False, True):
        r = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=ti, max_iter=60,
                            history_potentials=True)
        vals = [oracle.dual_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, r.hist_f[t], r.hist_g[t])
                for t in range(r.iters)]
        assert np.all(np.diff(vals) >= -1e-13), (ti, np.min(np.diff(vals)))


# ---------------------------------------------------------------------------------------
# P4: plain Sinkhorn started at f* + tau: f_t = f* + (k1 k2)^t tau exactly (Sec. 1 example).
# P5: TI started at f* + tau is back at (f*, g*) after one iteration (Psi(f + tau) = Psi(f) - tau).
# ---------------------------------------------------------------------------------------
def test_p4_translation_mode_of_plain_sinkhorn(medium):
    pr, cost, a, b, plain, ti = medium
    k = pr.rho1 / (pr.eps + pr.rho1) * pr.rho2 / (pr.eps + pr.rho2)
    tau = 0.37
    r = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=False, max_iter=25,
                        f0=ti.f + tau, history_potentials=True)
    for t in range(1, 26):
        expect = ti.f + k ** t * tau
        assert np.max(np.abs(r.hist_f[t - 1] - expect)) < 1e-13
        # g_t = g* - k2 (k1 k2)^{t-1} tau
        k2 = pr.rho2 / (pr.eps + pr.rho2)
        assert np.max(np.abs(r.hist_g[t - 1] - (ti.g - k2 * k ** (t - 1) * tau))) < 1e-13


@pytest.mark.parametrize("tau", [-3.0, 0.0, 0.5, 11.0])
def test_p5_ti_translation_invariance(medium, tau):
    pr, cost, a, b, plain, ti = medium
    r = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, max_iter=1, f0=ti.f + tau)
    assert np.max(np.abs(r.f - ti.f)) < 1e-13
    assert np.max(np.abs(r.g - ti.g)) < 1e-13


# ---------------------------------------------------------------------------------------
# P6: the empirical rate (median estimator of Sec. 3) of plain Sinkhorn equals
# (rho/(eps+rho))^2 on the 1-D measures, and TI's rate is strictly smaller.
# ---------------------------------------------------------------------------------------
def test_p6_empirical_rates_oned():
    pr = workloads.oned()
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    star = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True)
    assert star.last_delta < 1e-14
    rp = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=False, max_iter=1500,
                         history_potentials=True)
    rt = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, max_iter=400,
                         history_potentials=True)
    kp = oracle.empirical_rate(rp.hist_f, star.f, floor=1e-11)
    kt = oracle.empirical_rate(rt.hist_f, star.f, floor=1e-11)
    expect = (pr.rho1 / (pr.eps + pr.rho1)) ** 2
    assert abs(kp - expect) < 1e-4, (kp, expect)
    assert kt < kp - 0.01, (kt, kp)


# ---------------------------------------------------------------------------------------
# P7: Prop. 1/2 (equal tilted masses at lambda*), Prop. 3 (H = F o Phi), H invariance.
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p7_lambda_star_and_h(seed):
    rng = np.random.default_rng(seed)
    pr = workloads.random_small(9, 11, d=3, seed=seed, eps=0.2, rho1=0.3 + seed, rho2=1.1)
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    fb = rng.normal(size=9)
    gb = rng.normal(size=11)
    lam = oracle.lambda_star(a, b, fb, gb, pr.rho1, pr.rho2)
    ma = np.sum(a * np.exp(-(fb + lam) / pr.rho1))
    mb = np.sum(b * np.exp(-(gb - lam) / pr.rho2))
    assert abs(ma - mb) < 1e-13 * max(ma, mb)
    H = oracle.h_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, fb, gb)
    F = oracle.dual_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, fb + lam, gb - lam)
    assert abs(H - F) < 1e-13 * max(1.0, abs(F))
    H2 = oracle.h_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, fb + 1.7, gb - 1.7)
    assert abs(H2 - H) < 1e-13 * max(1.0, abs(H))
    # lambda* maximises G(lambda) = F(fb + lambda, gb - lambda)
    for dl in (-1e-3, 1e-3):
        assert oracle.dual_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, fb + lam + dl, gb - lam - dl) < F


# ---------------------------------------------------------------------------------------
# P8: one TI iteration is non-expansive: by the chain of App. B (Phi 1-Lipschitz into the
# (**)-norm, Upsilon 2-Lipschitz from the Hilbert norm, Psi contracting by rho/(eps+rho)),
# ||f_1 - f_1'||_inf + ||g_1 - g_1'||_inf <= 2 (rho/(eps+rho)) ||fb_0 - fb_0'||_star.
# ---------------------------------------------------------------------------------------
def test_p8_ti_iteration_lipschitz():
    pr = workloads.random_small(14, 10, d=2, seed=11, eps=0.1, rho1=0.8, rho2=0.8)
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    rng = np.random.default_rng(5)
    kfac = pr.rho1 / (pr.eps + pr.rho1)
    for _ in range(20):
        f0 = rng.normal(size=14)
        f1 = f0 + rng.normal(scale=rng.uniform(0.01, 1.0), size=14)
        r0 = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, max_iter=1, f0=f0)
        r1 = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, max_iter=1, f0=f1)
        lhs = np.max(np.abs(r0.f - r1.f)) + np.max(np.abs(r0.g - r1.g))
        assert lhs <= 2 * kfac * oracle.hilbert_norm(f0 - f1) + 1e-14


# ---------------------------------------------------------------------------------------
# P11: rho -> infinity recovers balanced entropic OT (Sec. 1), solved here by the textbook
# scaling iteration u = a / (K v), v = b / (K^T u) with Gibbs kernel K = exp(-C/eps).
# ---------------------------------------------------------------------------------------
def test_p11_large_rho_is_balanced():
    pr = workloads.random_small(15, 12, d=2, seed=21, eps=0.1, rho1=1e6, rho2=1e6,
                                mass_a=1.0, mass_b=1.0)
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    b = b * (a.sum() / b.sum())  # equal masses exactly in float64
    C = cost.dense()
    K = np.exp(-C / pr.eps)
    v = np.ones(len(b))
    for _ in range(20000):
        u = a / (K @ v)
        v = b / (K.T @ u)
    pi_bal = u[:, None] * K * v[None, :]
    r = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, tol=1e-13)
    pi = a[:, None] * b[None, :] * np.exp((r.f[:, None] + r.g[None, :] - C) / pr.eps)
    assert np.sum(np.abs(pi - pi_bal)) < 1e-5


# ---------------------------------------------------------------------------------------
# P12: envelope gradients equal central finite differences of the converged value.
# ---------------------------------------------------------------------------------------
def _uot_value(x, y, a, b, eps, r1, r2):
    cost = oracle.Cost(x=x, y=y, p=2.0)
    r = _solve(cost, a, b, eps, r1, r2, ti=True, tol=1e-15, max_iter=100000)
    return oracle.dual_value(cost, a, b, eps, r1, r2, r.f, r.g)


def test_p12_envelope_gradients_match_finite_differences():
    pr = workloads.random_small(6, 5, d=2, seed=4, eps=0.2, rho1=0.9, rho2=1.4)
    x, y = pr.x.astype(np.float64), pr.y.astype(np.float64)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    cost = oracle.Cost(x=x, y=y, p=2.0)
    r = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, tol=1e-15)
    gout = 1.7
    dx, dy, da, db = oracle.gradients(cost, a, b, pr.eps, pr.rho1, pr.rho2, r.f, r.g, gout)
    h = 1e-5
    args = (pr.eps, pr.rho1, pr.rho2)
    for i in range(6):
        e = np.zeros(6); e[i] = h
        fd = (_uot_value(x, y, a + e, b, *args) - _uot_value(x, y, a - e, b, *args)) / (2 * h)
        assert abs(gout * fd - da[i]) < 1e-7 * max(1.0, abs(da[i]))
        for t in range(2):
            ex = np.zeros_like(x); ex[i, t] = h
            fd = (_uot_value(x + ex, y, a, b, *args) - _uot_value(x - ex, y, a, b, *args)) / (2 * h)
            assert abs(gout * fd - dx[i, t]) < 1e-7 * max(1.0, abs(dx[i, t]))
    for j in range(5):
        e = np.zeros(5); e[j] = h
        fd = (_uot_value(x, y, a, b + e, *args) - _uot_value(x, y, a, b - e, *args)) / (2 * h)
        assert abs(gout * fd - db[j]) < 1e-7 * max(1.0, abs(db[j]))
        for t in range(2):
            ey = np.zeros_like(y); ey[j, t] = h
            fd = (_uot_value(x, y + ey, a, b, *args) - _uot_value(x, y - ey, a, b, *args)) / (2 * h)
            assert abs(gout * fd - dy[j, t]) < 1e-7 * max(1.0, abs(dy[j, t]))


def test_p12_dense_alpha_gradient_general_p():
    """Dense cost with p = 1.5 (the stored-cost workload's exponent): dalpha, dbeta by FD."""
    pr = workloads.random_small(5, 4, d=3, seed=8, eps=0.15, rho1=0.5, rho2=0.5, p=1.5, dense=True)
    C = pr.C.astype(np.float64)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)

    def val(a_, b_):
        cost = oracle.Cost(C=C)
        r = _solve(cost, a_, b_, pr.eps, pr.rho1, pr.rho2, ti=True, tol=1e-15)
        return oracle.dual_value(cost, a_, b_, pr.eps, pr.rho1, pr.rho2, r.f, r.g)

    cost = oracle.Cost(C=C)
    r = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, tol=1e-15)
    _, _, da, db = oracle.gradients(cost, a, b, pr.eps, pr.rho1, pr.rho2, r.f, r.g)
    h = 1e-5
    for i in range(5):
        e = np.zeros(5); e[i] = h
        assert abs((val(a + e, b) - val(a - e, b)) / (2 * h) - da[i]) < 1e-7
    for j in range(4):
        e = np.zeros(4); e[j] = h
        assert abs((val(a, b + e) - val(a, b - e)) / (2 * h) - db[j]) < 1e-7


def test_p12_point_gradient_general_p():
    """Points with p = 1.5: dx by FD (checks the p ||x-y||^{p-2} (x-y) factor)."""
    pr = workloads.random_small(4, 5, d=2, seed=9, eps=0.2, rho1=1.0, rho2=1.0, p=1.5)
    x, y = pr.x.astype(np.float64), pr.y.astype(np.float64)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)

    def val(x_):
        cost = oracle.Cost(x=x_, y=y, p=1.5)
        r = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, tol=1e-15)
        return oracle.dual_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, r.f, r.g)

    cost = oracle.Cost(x=x, y=y, p=1.5)
    r = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, tol=1e-15)
    dx, _, _, _ = oracle.gradients(cost, a, b, pr.eps, pr.rho1, pr.rho2, r.f, r.g)
    h = 1e-6
    for i in range(4):
        for t in range(2):
            e = np.zeros_like(x); e[i, t] = h
            assert abs((val(x + e) - val(x - e)) / (2 * h) - dx[i, t]) < 1e-7


# ---------------------------------------------------------------------------------------
# P13: Hilbert-metric contraction of the softmin (Birkhoff): for K = exp(-C/eps),
# ||Smin(C - f) - Smin(C - f')||_star <= tanh(Delta/4) ||f - f'||_star,
# Delta = max_{i,k,j,l} (C_il + C_kj - C_ij - C_kl)/eps  (the (1-eta)/(1+eta) reading).
# ---------------------------------------------------------------------------------------
def test_p13_birkhoff_contraction():
    pr = workloads.random_small(7, 6, d=2, seed=13, eps=0.5)
    cost = oracle_cost(pr)
    a = pr.alpha.astype(np.float64)
    C = cost.dense()
    D4 = C[:, None, None, :] + C[None, :, :, None] - C[:, None, :, None] - C[None, :, None, :]
    # D4[i, k, j, l] = C_il + C_kj - C_ij - C_kl
    Delta = np.max(D4) / pr.eps
    bound = math.tanh(Delta / 4)
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(50):
        f = rng.normal(size=7)
        f2 = f + rng.normal(scale=0.3, size=7)
        s1 = oracle.smin_cols(cost, a, f, pr.eps)
        s2 = oracle.smin_cols(cost, a, f2, pr.eps)
        ratio = oracle.hilbert_norm(s1 - s2) / oracle.hilbert_norm(f - f2)
        worst = max(worst, ratio)
    assert worst <= bound + 1e-12
    assert worst > 0.1 * bound  # the bound is not vacuous on this problem


# ---------------------------------------------------------------------------------------
# Softmin special cases and plan-apply adjoint identity.
# ---------------------------------------------------------------------------------------
def test_softmin_special_cases():
    # one point: Smin_w^s(h) = h - s log w
    assert abs(oracle.smin_vec([0.3], [1.2], 0.7) - (1.2 - 0.7 * math.log(0.3))) < 1e-15
    # constant h: Smin_w^s(c) = c - s log m(w)
    w = np.array([0.1, 0.5, 0.7])
    assert abs(oracle.smin_vec(w, [2.0, 2.0, 2.0], 0.3) - (2.0 - 0.3 * math.log(w.sum()))) < 1e-14
    # small s tends to the min; a zero weight drops its entry
    assert abs(oracle.smin_vec([1.0, 1.0], [0.5, 3.0], 1e-3) - 0.5) < 1e-12
    assert abs(oracle.smin_vec([0.0, 1.0], [-5.0, 3.0], 0.2) - 3.0) < 1e-15
    # column/row softmins on a dense matrix against the vector softmin per column/row
    rng = np.random.default_rng(1)
    C = rng.uniform(size=(4, 3))
    a, b = rng.uniform(0.1, 1, 4), rng.uniform(0.1, 1, 3)
    h, k = rng.normal(size=4), rng.normal(size=3)
    cols = oracle.smin_cols(oracle.Cost(C=C), a, h, 0.2)
    rows = oracle.smin_rows(oracle.Cost(C=C), b, k, 0.2)
    for j in range(3):
        assert abs(cols[j] - oracle.smin_vec(a, C[:, j] - h, 0.2)) < 1e-14
    for i in range(4):
        assert abs(rows[i] - oracle.smin_vec(b, C[i, :] - k, 0.2)) < 1e-14


def test_plan_apply_adjoint_and_points_vs_dense():
    pr = workloads.random_small(9, 7, d=3, seed=2, eps=0.3)
    cost = oracle_cost(pr)
    dense = oracle.Cost(C=cost.dense())
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    rng = np.random.default_rng(0)
    f, g = rng.normal(size=9) * 0.1, rng.normal(size=7) * 0.1
    V = rng.normal(size=(7, 2))
    U = rng.normal(size=(9, 2))
    PV = oracle.plan_apply(cost, a, b, pr.eps, f, g, V)
    PtU = oracle.plan_apply(cost, a, b, pr.eps, f, g, U, transpose=True)
    assert abs(np.sum(U * PV) - np.sum(PtU * V)) < 1e-13
    assert rel_inf(oracle.plan_apply(dense, a, b, pr.eps, f, g, V), PV) < 1e-13
    # pi_ij from basis vectors matches the one-point closed form structure a_i b_j e^{...}
    e = np.zeros(7); e[3] = 1.0
    col = oracle.plan_apply(cost, a, b, pr.eps, f, g, e)
    C = cost.dense()
    assert abs(col[5] - a[5] * b[3] * math.exp((f[5] + g[3] - C[5, 3]) / pr.eps)) < 1e-15


def test_zero_weight_convention():
    """A zero weight drops its point from every sum (nu_i = 0 convention, Sec. 1): the
    solution on the other points equals the solution of the problem without it."""
    pr = workloads.random_small(6, 5, d=2, seed=17, eps=0.1, rho1=0.6, rho2=0.9)
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64).copy(), pr.beta.astype(np.float64)
    a[2] = 0.0
    r = _solve(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True)
    keep = [0, 1, 3, 4, 5]
    cost2 = oracle.Cost(x=pr.x.astype(np.float64)[keep], y=pr.y.astype(np.float64), p=2.0)
    r2 = _solve(cost2, a[keep], b, pr.eps, pr.rho1, pr.rho2, ti=True)
    assert np.max(np.abs(r.f[keep] - r2.f)) < 1e-12
    assert np.max(np.abs(r.g - r2.g)) < 1e-12
    assert np.isfinite(r.f[2])


# ---------------------------------------------------------------------------------------
# Anderson extrapolation (appendix on combining Sinkhorn with Anderson acceleration).
# ---------------------------------------------------------------------------------------
def _linear_iterates(A, b, x0, K):
    X = [x0]
    for _ in range(K):
        X.append(A @ X[-1] + b)
    return np.array(X)


@pytest.mark.parametrize("symmetric", [True, False])
def test_anderson_mix_is_exact_on_linear_maps(symmetric):
    # For T(x) = A x + b with I - A invertible, the residuals are u_k = (A - I) A^k e_0
    # (e_0 = x_0 - x*). With K = n + 1 of them in R^n some c with sum 1 has U c = 0, and then
    # sum_k c_k x_{k+1} = x* + A sum_k c_k A^k e_0 = x*: the unregularised (r = 0) mix returns
    # the fixed point exactly. A wrong residual index, a combination of x_k instead of
    # x_{k+1}, or a transposed Gram fails this.
    rng = np.random.default_rng(7 if symmetric else 8)
    n = 5
    if symmetric:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        A = Q @ np.diag(rng.uniform(-0.9, 0.9, n)) @ Q.T
    else:
        A = rng.standard_normal((n, n))
        A *= 0.8 / np.max(np.abs(np.linalg.eigvals(A)))
    b = rng.standard_normal(n)
    xs = np.linalg.solve(np.eye(n) - A, b)
    X = _linear_iterates(A, b, rng.standard_normal(n), n + 1)
    c, out = oracle.anderson_mix(X, 0.0)
    assert abs(c.sum() - 1.0) < 1e-12
    assert np.max(np.abs(out - xs)) < 1e-7 * max(1.0, np.max(np.abs(xs)))


def test_anderson_mix_two_step_closed_form():
    # K = 1: one residual, c = [1], the mix is T(x_0). K = 2 with r = 0: minimising
    # |c0 u0 + c1 u1|^2 on c0 + c1 = 1 gives c0 = (u1.u1 - u0.u1) / |u0 - u1|^2.
    rng = np.random.default_rng(9)
    X = rng.standard_normal((2, 6))
    c, out = oracle.anderson_mix(X, 1e-7)
    assert np.array_equal(c, [1.0]) and np.array_equal(out, X[1])
    X = rng.standard_normal((3, 6))
    u0, u1 = X[1] - X[0], X[2] - X[1]
    c0 = (u1 @ u1 - u0 @ u1) / ((u0 - u1) @ (u0 - u1))
    c, out = oracle.anderson_mix(X, 0.0)
    assert np.allclose(c, [c0, 1.0 - c0], rtol=0, atol=1e-12)
    assert np.allclose(out, c0 * X[1] + (1.0 - c0) * X[2], rtol=0, atol=1e-12)


def test_anderson_mix_two_step_closed_form_regularised():
    # The appendix's regularised weights for K = 2: with a = |u0|^2, b = u0.u1, d = |u1|^2,
    # (G + rI)^{-1} 1 is proportional to (d + r - b, a + r - b) (2 x 2 inverse by cofactors),
    # so c0 = (d + r - b) / (a + d + 2r - 2b). r is comparable to the Gram entries here, so a
    # dropped or misplaced r (or a normalised Gram) moves c far beyond the tolerance.
    rng = np.random.default_rng(11)
    X = 0.01 * rng.standard_normal((3, 8))
    u0, u1 = X[1] - X[0], X[2] - X[1]
    a, b, d = u0 @ u0, u0 @ u1, u1 @ u1
    r = 0.5 * (a + d)
    c0 = (d + r - b) / (a + d + 2 * r - 2 * b)
    c, out = oracle.anderson_mix(X, r)
    assert np.allclose(c, [c0, 1.0 - c0], rtol=0, atol=1e-13)
    assert np.allclose(out, c0 * X[1] + (1.0 - c0) * X[2], rtol=0, atol=1e-13)
    cn, _ = oracle.anderson_mix(X, r, normalize=True)
    assert np.max(np.abs(cn - c)) > 1e-3  # the variant is a different mix


@pytest.mark.parametrize("normalize", [False, True])
def test_anderson_weights_minimise_the_regularised_energy(normalize):
    # c* minimises c^T (G + rI) c over 1^T c = 1 (the appendix's definition; G = U^T U, or
    # U^T U / ||U^T U||_F for the variant): every feasible direction v (1^T v = 0) raises
    # the energy, checked against an independent least-squares solve of the KKT system.
    rng = np.random.default_rng(12)
    X = rng.standard_normal((6, 30))
    U = np.diff(X, axis=0).T
    G = U.T @ U
    if normalize:
        G = G / np.linalg.norm(G)
    r = 1e-2
    K = G.shape[0]
    kkt = np.block([[2 * (G + r * np.eye(K)), np.ones((K, 1))], [np.ones((1, K)), np.zeros((1, 1))]])
    ref = np.linalg.lstsq(kkt, np.concatenate([np.zeros(K), [1.0]]), rcond=None)[0][:K]
    c, _ = oracle.anderson_mix(X, r, normalize=normalize)
    assert np.max(np.abs(c - ref)) < 1e-10
    energy = lambda v: v @ (G + r * np.eye(K)) @ v
    for _ in range(20):
        v = rng.standard_normal(K)
        v -= v.mean()
        assert energy(c + 1e-3 * v) > energy(c)


def test_anderson_printed_form_averages_small_residuals():
    # With the appendix's form a fixed r dominates U^T U once the residuals are small
    # against sqrt(r): the weights tend to the plain average 1/K. The normalised variant
    # does not depend on the scale of the residuals (an affine map of the iterates maps the
    # mix alike).
    rng = np.random.default_rng(10)
    X = rng.standard_normal((5, 40))
    a = rng.standard_normal(40)
    small = a + 1e-6 * (X - a)
    c_small, _ = oracle.anderson_mix(small, 1e-3)
    assert np.max(np.abs(c_small - 0.25)) < 1e-6
    c1, o1 = oracle.anderson_mix(X, 1e-3, normalize=True)
    c2, o2 = oracle.anderson_mix(a + 1e-5 * (X - a), 1e-3, normalize=True)
    assert np.max(np.abs(c1 - c2)) < 1e-8
    assert np.max(np.abs(a + 1e-5 * (o1 - a) - o2)) < 1e-12


@pytest.mark.parametrize("ti", [False, True])
def test_anderson_k1_reproduces_sinkhorn(ti):
    pr = workloads.oned()
    cost = oracle_cost(pr)
    base = oracle.sinkhorn(cost, pr.alpha, pr.beta, pr.eps, pr.rho1, pr.rho2, ti=ti, max_iter=50)
    k1 = oracle.sinkhorn_anderson(cost, pr.alpha, pr.beta, pr.eps, pr.rho1, pr.rho2, ti=ti, K=1,
                                  r=1e-7, max_iter=50)
    assert np.array_equal(base.f, k1.f) and np.array_equal(base.g, k1.g)


@pytest.mark.parametrize("ti", [False, True])
@pytest.mark.parametrize("normalize", [False, True])
def test_anderson_reaches_the_fixed_point(ti, normalize):
    # The F-potentials are unique, so the accelerated iteration must converge to the same
    # (f*, g*), with either form of the mix (K = 4, r = 1e-7, the appendix's setting). The
    # appendix's form accelerates the first cycles; near the optimum its residuals fall
    # below sqrt(r) and the weights become an average of K images, which lags behind the
    # plain iteration (to 1e-12 here: 1540 against 1120 iterations plain, 390 against 280
    # TI). The normalised variant keeps accelerating (less than half the iterations).
    pr = workloads.oned()
    cost = oracle_cost(pr)
    star = _solve(cost, pr.alpha, pr.beta, pr.eps, pr.rho1, pr.rho2, ti=True)
    kw = dict(ti=ti, max_iter=20000, tol=1e-12, check_every=10)
    acc = oracle.sinkhorn_anderson(cost, pr.alpha, pr.beta, pr.eps, pr.rho1, pr.rho2, K=4,
                                   r=1e-7, normalize=normalize, **kw)
    std = oracle.sinkhorn(cost, pr.alpha, pr.beta, pr.eps, pr.rho1, pr.rho2, **kw)
    assert rel_inf(acc.f, star.f) < 1e-8 and rel_inf(acc.g, star.g) < 1e-8
    if normalize:
        assert acc.iters < std.iters / 2
    else:
        early = oracle.sinkhorn_anderson(cost, pr.alpha, pr.beta, pr.eps, pr.rho1, pr.rho2, ti=ti,
                                         K=4, r=1e-7, max_iter=20)
        plain20 = oracle.sinkhorn(cost, pr.alpha, pr.beta, pr.eps, pr.rho1, pr.rho2, ti=ti,
                                  max_iter=20)
        assert np.max(np.abs(early.f - star.f)) < 0.5 * np.max(np.abs(plain20.f - star.f))


# ---------------------------------------------------------------------------------------
# Generic entropies (Sec. 3: F- and G-Sinkhorn for smooth phi*; the Berg entropy of the
# experiments of Sec. 3).
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("div", ["kl", "berg"])
@pytest.mark.parametrize("eps,rho,S", [(0.01, 1.0, 0.3), (0.1, 0.5, -2.0), (0.05, 2.0, 5.0),
                                       (1.0, 0.1, 0.7), (0.02, 10.0, -0.4)])
def test_dual_update_minimises_the_aprox_objective(div, eps, rho, S):
    # aprox_{phi*}(x) = argmin_y eps e^{(x - y)/eps} + phi*(y), and the update is
    # g = -aprox(-S): a direct bounded minimisation of the objective (no optimality
    # condition involved) must land on -g.
    from scipy.optimize import minimize_scalar
    g = oracle.dual_update(div, rho, eps, S)
    obj = lambda y: eps * math.exp(min((-S - y) / eps, 700.0)) + oracle.phistar(div, rho, y)
    hi = min(rho - 1e-12, abs(S) + 1.0) if div == "berg" else abs(S) + 1.0
    res = minimize_scalar(obj, bounds=(-abs(S) - 1.0, hi), method="bounded",
                          options={"xatol": 1e-13})
    assert abs(g + res.x) < 1e-6 * max(1.0, abs(g))
    if div == "kl":
        assert g == rho / (eps + rho) * S


def test_berg_update_tends_to_kl_for_small_potentials():
    # phi*'(0) = 1 and phi*''(0) = 1/rho for both entropies, so the updates agree to second
    # order in S/rho: |U_berg(S) - U_kl(S)| = O(S^2 / rho).
    eps, rho = 0.05, 2.0
    for S in (1e-2, 1e-3, 1e-4):
        d = abs(oracle.dual_update("berg", rho, eps, S) - oracle.dual_update("kl", rho, eps, S))
        assert d < 2.0 * S * S / rho


@pytest.mark.parametrize("div", ["kl", "berg"])
def test_lambda_star_div_maximises_g(div):
    # lambda* = argmax_l G_eps(fb, gb, l) = F_eps(fb + l, gb - l); the entropic term is
    # invariant under the translation, so a direct maximisation of
    # -<alpha, phi1*(-fb - l)> - <beta, phi2*(-gb + l)> must give the same l.
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(21)
    a, b = rng.uniform(0.1, 1.0, 7), rng.uniform(0.1, 1.0, 5)
    fb, gb = rng.uniform(-0.3, 0.5, 7), rng.uniform(-0.2, 0.6, 5)
    r1, r2 = 0.8, 1.7
    lam = oracle.lambda_star_div(div, a, b, fb, gb, r1, r2)
    obj = lambda l: sum(ai * oracle.phistar(div, r1, -fi - l) for ai, fi in zip(a, fb)) + \
        sum(bj * oracle.phistar(div, r2, -gj + l) for bj, gj in zip(b, gb))
    lo, hi = (-r1 - fb.min() + 1e-9, r2 + gb.min() - 1e-9) if div == "berg" else (-5.0, 5.0)
    res = minimize_scalar(obj, bounds=(lo, hi), method="bounded", options={"xatol": 1e-13})
    assert abs(lam - res.x) < 1e-6
    c = 0.37
    assert abs(oracle.lambda_star_div(div, a, b, fb + c, gb - c, r1, r2) - (lam - c)) < 1e-12


def test_kl_f_variant_is_plain_sinkhorn():
    pr = workloads.oned()
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    base = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=False, max_iter=40)
    r = oracle.sinkhorn_div(cost, a, b, pr.eps, pr.rho1, pr.rho2, div="kl", variant="F", max_iter=40)
    assert np.array_equal(base.f, r.f) and np.array_equal(base.g, r.g)


def test_berg_fixed_point_maximises_the_dual():
    # Tiny problem: a direct numerical maximisation of the concave Berg dual F_eps over
    # (f, g) (L-BFGS-B inside the domain f > -rho1, g > -rho2) must reach the potentials
    # of the Sinkhorn fixed point; F- and G-Sinkhorn share that fixed point.
    from scipy.optimize import minimize
    pr = workloads.random_small(3, 4, d=2, seed=5, eps=0.2, rho1=0.7, rho2=1.3)
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    kw = dict(div="berg", max_iter=100000, tol=1e-14, check_every=1)
    F = oracle.sinkhorn_div(cost, a, b, pr.eps, pr.rho1, pr.rho2, variant="F", **kw)
    G = oracle.sinkhorn_div(cost, a, b, pr.eps, pr.rho1, pr.rho2, variant="G", **kw)
    neg = lambda z: -oracle.dual_value_div(cost, a, b, pr.eps, pr.rho1, pr.rho2, "berg", z[:3], z[3:])
    bounds = [(-pr.rho1 + 1e-6, None)] * 3 + [(-pr.rho2 + 1e-6, None)] * 4
    res = minimize(neg, np.zeros(7), method="L-BFGS-B", bounds=bounds,
                   options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 10000})
    assert np.max(np.abs(res.x[:3] - F.f)) < 1e-5 and np.max(np.abs(res.x[3:] - F.g)) < 1e-5
    assert np.max(np.abs(G.f - F.f)) < 1e-11 and np.max(np.abs(G.g - F.g)) < 1e-11


@pytest.mark.parametrize("div", ["kl", "berg"])
def test_g_sinkhorn_is_faster_when_eps_below_rho(div):
    # Sec. 3 reports G-Sinkhorn faster than F-Sinkhorn in the regime eps <= rho, for KL and
    # the Berg entropy, towards the same optimum.
    pr = workloads.oned()
    cost = oracle_cost(pr)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    for rho in (1.0, 10.0):
        kw = dict(div=div, max_iter=100000, tol=1e-10, check_every=10)
        F = oracle.sinkhorn_div(cost, a, b, pr.eps, rho, rho, variant="F", **kw)
        G = oracle.sinkhorn_div(cost, a, b, pr.eps, rho, rho, variant="G", **kw)
        assert G.iters < F.iters / 3, (rho, F.iters, G.iters)
        assert rel_inf(G.f, F.f) < 1e-7


# ---------------------------------------------------------------------------------------
# 1-D Frank-Wolfe for unregularised KL-UOT (Sec. 4).
# ---------------------------------------------------------------------------------------
def _sorted_problem(n, m, seed):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0.0, 1.0, n))
    y = np.sort(rng.uniform(0.0, 1.0, m))
    return x, y, rng.uniform(0.2, 1.0, n), rng.uniform(0.2, 1.0, m)


@pytest.mark.parametrize("n,m,p", [(1, 1, 2.0), (1, 6, 1.0), (5, 1, 1.5), (4, 5, 2.0),
                                   (9, 7, 1.0), (12, 17, 1.5)])
def test_solve_ot_1d_is_an_optimal_primal_dual_pair(n, m, p):
    # Against a linear program (scipy's HiGHS) on the full n x m cost: same optimal cost;
    # the walk's plan has the prescribed marginals; the potentials are dual feasible and
    # their dual value equals the cost (strong duality), so both are optimal.
    from scipy.optimize import linprog
    x, y, a, b = _sorted_problem(n, m, 100 + n * m)
    a, b = a / a.sum(), b / b.sum()
    C = np.abs(x[:, None] - y[None, :]) ** p
    cost, r, s, cells, mass = oracle.solve_ot_1d(x, y, a, b, p)
    A = np.zeros((n + m, n * m))
    for i in range(n):
        A[i, i * m:(i + 1) * m] = 1.0
    for j in range(m):
        A[n + j, j::m] = 1.0
    lp = linprog(C.reshape(-1), A_eq=A, b_eq=np.concatenate([a, b]), bounds=(0, None),
                 method="highs")
    assert abs(cost - lp.fun) <= 1e-12 * max(1.0, abs(lp.fun))
    pi = np.zeros((n, m))
    for (i, j), w in zip(cells, mass):
        pi[i, j] += w
    assert np.allclose(pi.sum(1), a, rtol=0, atol=1e-14) and np.allclose(pi.sum(0), b, rtol=0, atol=1e-14)
    assert np.max(r[:, None] + s[None, :] - C) <= 1e-14
    assert abs(r @ a + s @ b - cost) <= 1e-13


def test_fw_reaches_the_unregularised_optimum():
    # A direct constrained maximisation of F_0(f, g) = rho1 <alpha, 1 - e^{-f/rho1}> +
    # rho2 <beta, 1 - e^{-g/rho2}> over f_i + g_j <= C_ij (SLSQP on a 4 x 5 problem) and
    # Frank-Wolfe on H_0 (both step rules) give the same potentials.
    from scipy.optimize import minimize
    x, y, a, b = _sorted_problem(4, 5, 3)
    r1, r2, p = 0.3, 0.7, 2.0
    n, m = 4, 5
    C = np.abs(x[:, None] - y[None, :]) ** p
    neg = lambda z: -(r1 * np.sum(a * (1 - np.exp(-z[:n] / r1))) + r2 * np.sum(b * (1 - np.exp(-z[n:] / r2))))
    cons = [{"type": "ineq", "fun": (lambda z, i=i, j=j: C[i, j] - z[i] - z[n + j])}
            for i in range(n) for j in range(m)]
    res = minimize(neg, np.zeros(n + m), method="SLSQP", constraints=cons,
                   options={"ftol": 1e-15, "maxiter": 1000})
    assert res.success
    for ls, tol in ((True, 1e-13), (False, 1e-10)):
        fw = oracle.fw_1d(x, y, a, b, r1, r2, p=p, line_search=ls, max_iter=200000, tol=tol)
        assert fw.gap <= tol
        assert np.max(np.abs(fw.f - res.x[:n])) < 1e-6 and np.max(np.abs(fw.g - res.x[n:])) < 1e-6


def test_fw_gap_bounds_the_suboptimality():
    # The Frank-Wolfe gap at an iterate bounds H_0* - H_0(iterate) (concavity of H_0); and
    # H_0 of the reported pair equals F_0 there (lambda* folded in).
    pr = workloads.oned()
    x, y = np.sort(pr.x.reshape(-1).astype(np.float64)), np.sort(pr.y.reshape(-1).astype(np.float64))
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    rho = 0.5
    star = oracle.fw_1d(x, y, a, b, rho, rho, line_search=True, max_iter=3000, tol=1e-14)
    h_star, _ = oracle.h0(a, b, star.f, star.g, rho, rho)
    for K in (1, 3, 10, 40):
        it = oracle.fw_1d(x, y, a, b, rho, rho, max_iter=K)  # iterate K (K steps)
        gap = oracle.fw_1d(x, y, a, b, rho, rho, max_iter=K + 1, history=True).hist_gap[K]
        h, lam = oracle.h0(a, b, it.f, it.g, rho, rho)
        assert abs(lam) < 1e-12  # the reported pair is already optimally translated
        assert 0.0 <= h_star - h <= gap + 1e-12, (K, h_star - h, gap)


# ---------------------------------------------------------------------------------------
# Unbalanced 1-D barycenters by Frank-Wolfe on the multi-marginal dual (Sec. 5).
# ---------------------------------------------------------------------------------------
def test_mot_two_marginals_is_pairwise_ot():
    # K = 2, w = (1/2, 1/2): min_b (x - b)^2/2 + (y - b)^2/2 = |x/2 - y/2|^2, so the
    # multi-marginal walk is the pairwise coupling on the halved supports: same cost, same
    # potentials up to the translation (f_0 + c, f_1 - c).
    rng = np.random.default_rng(5)
    n, m = 7, 9
    x, y = np.sort(rng.uniform(0, 1, n)), np.sort(rng.uniform(0, 1, m))
    a, b = rng.uniform(0.2, 1, n), rng.uniform(0.2, 1, m)
    a, b = a / a.sum(), b / b.sum()
    cost, f, bx, bm = oracle.solve_mot_1d([0, n, n + m], np.concatenate([x, y]),
                                          np.concatenate([a, b]), [0.5, 0.5])
    c2, r, s, _, _ = oracle.solve_ot_1d(x / 2, y / 2, a, b, 2.0)
    assert abs(cost - c2) <= 1e-15
    assert np.ptp(f[:n] - r) < 1e-14 and np.ptp(f[n:] - s) < 1e-14
    assert abs((f[:n] - r)[0] + (f[n:] - s)[0]) < 1e-14
    assert abs(bm.sum() - 1.0) < 1e-14 and np.all(bm >= 0)


def test_mot_three_marginals_is_an_optimal_primal_dual_pair():
    # Against a linear program on the full tensor of tuples (HiGHS): same cost, dual
    # feasibility on every tuple, strong duality; the barycenter points are the barycentric
    # maps of the visited tuples.
    import itertools
    from scipy.optimize import linprog
    rng = np.random.default_rng(6)
    Ns = [3, 4, 3]
    xs = [np.sort(rng.uniform(0, 1, k)) for k in Ns]
    ws = [rng.uniform(0.2, 1, k) for k in Ns]
    ws = [v / v.sum() for v in ws]
    w = np.array([0.2, 0.5, 0.3])
    off = np.concatenate([[0], np.cumsum(Ns)])
    X, A = np.concatenate(xs), np.concatenate(ws)
    cost, f, bx, bm = oracle.solve_mot_1d(off, X, A, w)
    tuples = list(itertools.product(*[range(k) for k in Ns]))
    bar = lambda t: sum(w[k] * xs[k][t[k]] for k in range(3)) / w.sum()
    Cc = np.array([sum(w[k] * (xs[k][t[k]] - bar(t)) ** 2 for k in range(3)) for t in tuples])
    Aeq = np.zeros((sum(Ns), len(tuples)))
    for col, t in enumerate(tuples):
        for k in range(3):
            Aeq[off[k] + t[k], col] = 1.0
    lp = linprog(Cc, A_eq=Aeq, b_eq=A, bounds=(0, None), method="highs")
    assert abs(cost - lp.fun) <= 1e-12
    viol = max(sum(f[off[k] + t[k]] for k in range(3)) - Cc[c] for c, t in enumerate(tuples))
    assert viol <= 1e-14
    assert abs(f @ A - cost) <= 1e-13
    assert len(bx) == sum(Ns) - 3 + 1 and abs(bm.sum() - 1.0) < 1e-14
    assert np.all(np.diff(bx) >= -1e-15)  # the monotone walk visits tuples in order
    # the returned barycenter is the image of the LP's optimal plan under the barycentric
    # map: the same measure (compared through its quantile function)
    px = np.array([bar(t) for t in tuples])
    u = _mid_levels([np.cumsum(bm), np.cumsum(lp.x[np.argsort(px, kind="stable")])])
    assert np.max(np.abs(_quantile(bx, bm, u) - _quantile(px, lp.x, u))) < 1e-12


def _quantile(x, m, u):
    """Quantile function of the discrete measure sum_i m_i delta_{x_i} (sum m = 1) at levels
    u in (0, 1): the smallest support point whose cumulative mass reaches u."""
    order = np.argsort(x, kind="stable")
    xs, cs = np.asarray(x)[order], np.cumsum(np.asarray(m)[order])
    return xs[np.minimum(np.searchsorted(cs, u, side="left"), len(xs) - 1)]


def _mid_levels(cumsums):
    """Midpoints between the distinct cumulative-mass levels of several measures (levels
    closer than 1e-12 merged), where every quantile function is away from its jumps."""
    lv = np.unique(np.concatenate([[0.0, 1.0]] + [np.clip(c, 0.0, 1.0) for c in cumsums]))
    lv = lv[np.concatenate([[True], np.diff(lv) > 1e-12])]
    return 0.5 * (lv[1:] + lv[:-1])


@pytest.mark.parametrize("Ns,iters", [([5, 9, 7], 1), ([5, 9, 7], 40), ([12, 3, 8, 6], 25),
                                      ([1, 6], 10)])
def test_barycenter_output_is_the_quantile_average(Ns, iters):
    # On the line, the barycenter for the cost sum_k w_k (z_k - b)^2 of K probability
    # measures has the quantile function sum_k w_k Q_k / sum_k w_k (the comonotone coupling
    # is optimal and the barycentric map acts on it level by level), a closed form that
    # does not use the multi-marginal walk. The solver returns the barycenter of its final
    # tilted marginals a_k e^{-f_k / (w_k rho)} (f the reported potentials): their masses
    # are equal (the optimal translation of Sec. 5), the barycenter carries that mass, its
    # normalised quantile function is the weighted average of theirs, and so its mean is
    # the weighted mean of their means.
    rng = np.random.default_rng(sum(Ns) + iters)
    K = len(Ns)
    xs = [np.sort(rng.normal(rng.uniform(-1, 1), rng.uniform(0.1, 0.5), k)) for k in Ns]
    As = [rng.uniform(0.2, 1.0, k) * rng.uniform(0.5, 2.0) / k for k in Ns]
    w = rng.uniform(0.2, 1.0, K)
    rho = 0.6
    off = np.concatenate([[0], np.cumsum(Ns)])
    res = oracle.fw_barycenter(off, np.concatenate(xs), np.concatenate(As), w, rho,
                               max_iter=iters)
    tilted = [As[k] * np.exp(-res.f[off[k]:off[k + 1]] / (w[k] * rho)) for k in range(K)]
    q = np.array([t.sum() for t in tilted])
    assert np.max(np.abs(q - q[0])) < 1e-12 * q[0]
    bm = res.bary_m
    assert len(res.bary_x) == off[-1] - K + 1 and np.all(bm >= 0)
    assert abs(bm.sum() - q[0]) < 1e-12 * q[0]
    probs = [t / t.sum() for t in tilted]
    u = _mid_levels([np.cumsum(p) for p in probs] + [np.cumsum(bm) / bm.sum()])
    avg = sum(w[k] * _quantile(xs[k], probs[k], u) for k in range(K)) / w.sum()
    assert np.max(np.abs(_quantile(res.bary_x, bm / bm.sum(), u) - avg)) < 1e-12
    mean = sum(w[k] * probs[k] @ xs[k] for k in range(K)) / w.sum()
    assert abs(res.bary_x @ bm / bm.sum() - mean) < 1e-12


def test_mm_lambda_maximises_the_translated_dual():
    # lambda* maximises F(fb + lambda) over sum lambda = 0 (Prop. on the multi-marginal
    # translation); checked by a direct unconstrained maximisation over K - 1 free values.
    from scipy.optimize import minimize
    rng = np.random.default_rng(7)
    Ns = [3, 4, 3]
    off = np.concatenate([[0], np.cumsum(Ns)])
    A = rng.uniform(0.2, 1.0, off[-1])
    fb = rng.uniform(-0.3, 0.3, off[-1])
    w, rho = np.array([0.2, 0.5, 0.3]), 0.7
    lam = oracle.mm_lambda(off, A, fb, w, rho)

    def neg(l2):
        lv = np.array([l2[0], l2[1], -l2[0] - l2[1]])
        return -oracle.mm_dual(off, A, fb + np.repeat(lv, Ns), w, rho)
    res = minimize(neg, [0.0, 0.0], method="BFGS", options={"gtol": 1e-12})
    assert abs(lam.sum()) < 1e-15
    assert np.max(np.abs(lam[:2] - res.x)) < 1e-7


def test_barycenter_fw_two_marginals_is_pairwise_fw():
    # K = 2, w = (1/2, 1/2), penalty rho: the multi-marginal dual is the pairwise F_0 with
    # rho1 = rho2 = rho/2 on the halved supports, and lambda* coincides with Prop. 2, so the
    # reported potentials of both Frank-Wolfe solvers agree iterate by iterate.
    rng = np.random.default_rng(8)
    n, m = 7, 9
    x, y = np.sort(rng.uniform(0, 1, n)), np.sort(rng.uniform(0, 1, m))
    a, b = rng.uniform(0.2, 1, n) / n, rng.uniform(0.2, 1, m) * 1.4 / m
    rho = 0.8
    for iters in (1, 5, 50):
        fb = oracle.fw_barycenter([0, n, n + m], np.concatenate([x, y]), np.concatenate([a, b]),
                                  [0.5, 0.5], rho, max_iter=iters)
        fw = oracle.fw_1d(x / 2, y / 2, a, b, rho / 2, rho / 2, max_iter=iters)
        assert np.max(np.abs(fb.f[:n] - fw.f)) < 1e-13 and np.max(np.abs(fb.f[n:] - fw.g)) < 1e-13
        assert abs(fb.gap - fw.gap) < 1e-13
