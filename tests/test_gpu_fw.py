"""GPU parity of the 1-D Frank-Wolfe solver for unregularised KL-UOT (Sec. 4) against the
oracle's ``fw_1d`` (both in double precision), through the C ABI.

Tolerance: relative 1e-5 (||a - b||_inf / ||b||_inf) on the reported potentials, which the
GPU returns in float32. Iteration parity uses random weights: with exactly tied cumulative
masses the monotone coupling has several optimal duals and the two sides may pick different
ones (their CDFs are summed in different orders), so problems with tied masses (uniform
weights on equal sizes) are compared at convergence, where the optimum is unique.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2201_00730_amd as uot
import workloads
from tests.helpers import rel_inf

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=dtype))).to("cuda")


def random_problem(n, m, seed, p=2.0):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0.0, 1.0, n)).astype(np.float32)
    y = np.sort(rng.normal(0.5, 0.2, m)).astype(np.float32)
    a = (rng.uniform(0.2, 1.0, n) / n).astype(np.float32)
    b = (rng.uniform(0.2, 1.0, m) * 1.3 / m).astype(np.float32)
    return x, y, a, b


def oracle_fw(x, y, a, b, rho1, rho2, **kw):
    f64 = lambda v: np.asarray(v, dtype=np.float64)
    return oracle.fw_1d(f64(x), f64(y), f64(a), f64(b), rho1, rho2, **kw)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uot.load_library()


@pytest.mark.parametrize("line_search", [False, True])
@pytest.mark.parametrize("iters", [1, 2, 5, 40, 300])
@pytest.mark.parametrize("p", [2.0, 1.5, 1.0])
def test_fw_iteration_parity(line_search, iters, p):
    x, y, a, b = random_problem(211, 173, seed=int(10 * p) + iters, p=p)
    rho1, rho2 = 0.4, 1.1
    _say("fw parity ls=%s iters=%d p=%g" % (line_search, iters, p))
    f, g, it, gap, st = uot.fw1d(dev(x), dev(y), dev(a), dev(b), rho1, rho2, p=p,
                                 line_search=line_search, max_iter=iters)
    r = oracle_fw(x, y, a, b, rho1, rho2, p=p, line_search=line_search, max_iter=iters)
    f, g = f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    _say("  rel f %.3g g %.3g gap %.6g / %.6g" % (rel_inf(f, r.f), rel_inf(g, r.g), gap, r.gap))
    assert it == r.iters == iters and st == 1  # UOT_BATCH_MAX_ITER
    assert rel_inf(f, r.f) < TOL and rel_inf(g, r.g) < TOL, (rel_inf(f, r.f), rel_inf(g, r.g))
    assert abs(gap - r.gap) <= 1e-9 + 1e-6 * abs(r.gap)


@pytest.mark.parametrize("rho", [1.0, 0.1])
def test_fw_converged_oned(rho):
    """The 1-D measures of the Sinkhorn tests (sorted; uniform weights on equal sizes, so the
    cumulative masses tie exactly and the linear oracle has several optimal duals; the two
    sides may pick different ones). Line search to gap <= 1e-9 on both sides: what is unique
    is compared — the stopping iteration (within two), the value H_0 (within the gap of the
    optimum on each side) — and the GPU's potentials are checked to be feasible."""
    pr = workloads.oned()
    x = np.sort(pr.x.reshape(-1)).astype(np.float32)
    y = np.sort(pr.y.reshape(-1)).astype(np.float32)
    _say("fw oned converged rho=%g" % rho)
    f, g, it, gap, st = uot.fw1d(dev(x), dev(y), dev(pr.alpha), dev(pr.beta), rho, rho,
                                 line_search=True, max_iter=20000, tol=1e-9)
    rule = oracle_fw(x, y, pr.alpha, pr.beta, rho, rho, line_search=True, max_iter=20000,
                     tol=1e-9)
    same = oracle_fw(x, y, pr.alpha, pr.beta, rho, rho, line_search=True, max_iter=it)
    f, g = f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    h_gpu, lam = oracle.h0(pr.alpha.astype(np.float64), pr.beta.astype(np.float64), f, g, rho, rho)
    h_orc, _ = oracle.h0(pr.alpha.astype(np.float64), pr.beta.astype(np.float64), rule.f, rule.g, rho, rho)
    C = np.abs(x.astype(np.float64)[:, None] - y.astype(np.float64)[None, :]) ** 2
    _say("  iters %d gap %.3g; oracle %d gap %.3g; H0 %.12g / %.12g; rel f (same iteration) %.3g"
         % (it, gap, rule.iters, rule.gap, h_gpu, h_orc, rel_inf(f, same.f)))
    assert st == 0 and gap <= 1e-9
    assert abs(rule.iters - it) <= 2, (rule.iters, it)
    assert abs(h_gpu - h_orc) <= 2e-9 + 1e-7 * abs(h_orc), (h_gpu, h_orc)
    assert abs(lam) < 1e-6 * max(1.0, np.max(np.abs(f)))  # reported pair optimally translated
    assert np.max(f[:, None] + g[None, :] - C) <= 1e-6  # f (+) g <= C up to float32 output


def test_fw_batched_ragged_and_invalid():
    """64 problems of ragged sizes (1 point on a side included), zero weights, one unsorted
    problem (reported invalid, the others unaffected); each against the oracle."""
    rng = np.random.default_rng(77)
    sizes = [(int(rng.integers(1, 300)), int(rng.integers(1, 300))) for _ in range(64)]
    sizes[0], sizes[1] = (1, 1), (1, 40)
    xs, ys, As, Bs = [], [], [], []
    for k, (n, m) in enumerate(sizes):
        x, y, a, b = random_problem(n, m, seed=1000 + k)
        if k == 5 and n > 3:
            a[1] = 0.0
        if k == 9 and n > 2:
            x = x[::-1].copy()  # unsorted: invalid
        xs.append(x); ys.append(y); As.append(a); Bs.append(b)
    offN = np.concatenate([[0], np.cumsum([n for n, _ in sizes])]).astype(np.int64)
    offM = np.concatenate([[0], np.cumsum([m for _, m in sizes])]).astype(np.int64)
    rho1 = rng.uniform(0.1, 2.0, 64)
    rho2 = rng.uniform(0.1, 2.0, 64)
    for ls in (False, True):
        _say("fw batched ragged ls=%s" % ls)
        f, g, it, gap, st = uot.fw1d_batched(offN, offM, dev(np.concatenate(xs)), dev(np.concatenate(ys)),
                                             dev(np.concatenate(As)), dev(np.concatenate(Bs)),
                                             dev(rho1, np.float64), dev(rho2, np.float64),
                                             line_search=ls, max_iter=25)
        f, g = f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
        it, st = it.cpu().numpy(), st.cpu().numpy()
        worst = 0.0
        for k in range(64):
            fk, gk = f[offN[k]:offN[k + 1]], g[offM[k]:offM[k + 1]]
            if k == 9 and sizes[k][0] > 2:
                assert st[k] == 2 and np.all(np.isnan(fk))
                continue
            r = oracle_fw(xs[k], ys[k], As[k], Bs[k], rho1[k], rho2[k], line_search=ls, max_iter=25)
            assert st[k] == 1 and it[k] == 25
            worst = max(worst, rel_inf(fk, r.f), rel_inf(gk, r.g))
        _say("  worst rel %.3g" % worst)
        assert worst < TOL


def test_fw_batched_large_problems():
    """6 problems with 700..3000 points a side (each thread of the workgroup owns several
    points in every loop, scan and merge share), against the oracle."""
    rng = np.random.default_rng(78)
    sizes = [(int(rng.integers(700, 3000)), int(rng.integers(700, 3000))) for _ in range(6)]
    xs, ys, As, Bs = [], [], [], []
    for k, (n, m) in enumerate(sizes):
        x, y, a, b = random_problem(n, m, seed=2000 + k)
        xs.append(x); ys.append(y); As.append(a); Bs.append(b)
    offN = np.concatenate([[0], np.cumsum([n for n, _ in sizes])]).astype(np.int64)
    offM = np.concatenate([[0], np.cumsum([m for _, m in sizes])]).astype(np.int64)
    rho1 = rng.uniform(0.1, 2.0, 6)
    rho2 = rng.uniform(0.1, 2.0, 6)
    for ls in (False, True):
        _say("fw batched large ls=%s" % ls)
        f, g, it, gap, st = uot.fw1d_batched(offN, offM, dev(np.concatenate(xs)), dev(np.concatenate(ys)),
                                             dev(np.concatenate(As)), dev(np.concatenate(Bs)),
                                             dev(rho1, np.float64), dev(rho2, np.float64),
                                             line_search=ls, max_iter=30)
        f, g = f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
        it, st = it.cpu().numpy(), st.cpu().numpy()
        worst = 0.0
        for k in range(6):
            r = oracle_fw(xs[k], ys[k], As[k], Bs[k], rho1[k], rho2[k], line_search=ls, max_iter=30)
            assert st[k] == 1 and it[k] == 30
            worst = max(worst, rel_inf(f[offN[k]:offN[k + 1]], r.f), rel_inf(g[offM[k]:offM[k + 1]], r.g))
        _say("  worst rel %.3g" % worst)
        assert worst < TOL
