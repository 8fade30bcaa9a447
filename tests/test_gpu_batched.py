"""GPU parity of the batched TI solver against the FP64 oracle, problem by problem."""
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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uot.load_library()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run_batched(bt, iters, tol=0.0, ce=1):
    f, g, it, st = uot.ti_sinkhorn_batched(bt.offN, bt.offM, dev(bt.x), dev(bt.y), dev(bt.alpha),
                                           dev(bt.beta), bt.eps, bt.rho1, bt.rho2, p=bt.p,
                                           max_iter=iters, tol=tol, check_every=ce)
    torch.cuda.synchronize()
    return (f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64),
            it.cpu().numpy(), st.cpu().numpy())


def oracle_problem(bt, b, iters, tol=0.0, ce=1):
    pr = bt.problem(b)
    cost = oracle.Cost(x=pr.x.astype(np.float64), y=pr.y.astype(np.float64), p=pr.p)
    return oracle.sinkhorn(cost, pr.alpha.astype(np.float64), pr.beta.astype(np.float64), pr.eps,
                           pr.rho1, pr.rho2, ti=True, max_iter=iters, tol=tol, check_every=ce)


def small_batch(B=23, nmin=1, nmax=300, seed=31, d=2, p=2.0, eps=(2e-2, 2e-1), rho=(0.1, 10.0)):
    bt = workloads.batch2d(B=B, nmin=nmin, nmax=nmax, seed=seed, eps_range=eps, rho_range=rho)
    if d != 2:
        rng = np.random.default_rng(seed)
        bt.x = rng.uniform(0, 1, size=(int(bt.offN[-1]), d)).astype(np.float32)
        bt.y = rng.uniform(0, 1, size=(int(bt.offM[-1]), d)).astype(np.float32)
    bt.p = p
    # unequal penalties on half of the problems
    bt.rho2 = bt.rho2 * np.where(np.arange(B) % 2 == 0, 1.0, 2.5)
    return bt


class _plan:
    """Context manager that sets the batched work-item plan and restores the previous one."""

    def __init__(self, plan):
        self.plan = plan

    def __enter__(self):
        self.prev = uot.batched_set_plan(self.plan)

    def __exit__(self, *exc):
        uot.batched_set_plan(self.prev)


PLANS = {"auto": uot.BATCH_PLAN_AUTO, "coarse": uot.BATCH_PLAN_COARSE,
         "fine": uot.BATCH_PLAN_FINE, "finest": uot.BATCH_PLAN_FINEST, "split": uot.BATCH_PLAN_SPLIT}


@pytest.mark.parametrize("plan", ["coarse", "fine", "finest", "split", "auto"])
@pytest.mark.parametrize("d,p,nmax", [(2, 2.0, 300), (3, 2.0, 300), (1, 2.0, 300), (5, 1.5, 300),
                                       (8, 2.0, 300), (2, 2.0, 1100), (3, 1.5, 700)])
def test_batched_iteration_parity(d, p, nmax, plan):
    """Sizes 1..nmax under each work-item plan: coarse items of <= 64 targets (one per lane),
    65..128 (two per lane), 129..256 (four per lane) and problems split into several items;
    fine items of <= 128 targets; split items (64 targets, sources in ranges of 512: the
    nmax = 700 and 1100 batches split their larger problems into two or three ranges)."""
    bt = small_batch(B=23 if nmax <= 300 else 9, nmax=nmax, d=d, p=p, seed=40 + d + nmax)
    print("batched d=%d p=%g B=%d plan=%s" % (d, p, bt.B, plan), file=sys.stderr, flush=True)
    T = 12
    with _plan(PLANS[plan]):
        f, g, it, st = run_batched(bt, T)
    assert np.all(it == T) and np.all(st == uot.BATCH_MAX_ITER)
    for b in range(bt.B):
        r = oracle_problem(bt, b, T)
        fb = f[bt.offN[b]:bt.offN[b + 1]]
        gb = g[bt.offM[b]:bt.offM[b + 1]]
        assert rel_inf(fb, r.f) < TOL and rel_inf(gb, r.g) < TOL, (b, rel_inf(fb, r.f), rel_inf(gb, r.g))


@pytest.mark.parametrize("plan", [uot.BATCH_PLAN_AUTO, uot.BATCH_PLAN_SWITCH, uot.BATCH_PLAN_SPLIT])
def test_batched_converges_per_problem(plan):
    """Each problem stops at its own first passing check; at its stopping iteration it matches
    the oracle run for that many iterations, and the oracle's own stopping iteration is close.
    The second plan starts on coarse items and moves to fine items after the first chunk, in
    the middle of every problem's solve (active lists rebuilt, item partials re-indexed)."""
    bt = small_batch(B=17, nmin=5, nmax=600, seed=7)
    with _plan(plan):
        f, g, it, st = run_batched(bt, 5000, tol=1e-6, ce=10)
    assert np.all(st == uot.BATCH_CONVERGED), st
    assert len(set(it.tolist())) > 1  # problems converge at different iterations
    for b in range(bt.B):
        r = oracle_problem(bt, b, int(it[b]))
        fb = f[bt.offN[b]:bt.offN[b + 1]]
        gb = g[bt.offM[b]:bt.offM[b + 1]]
        assert rel_inf(fb, r.f) < TOL and rel_inf(gb, r.g) < TOL, b
        rr = oracle_problem(bt, b, 5000, tol=1e-6, ce=10)
        assert abs(int(it[b]) - rr.iters) <= 20, (b, it[b], rr.iters)


def test_batched_matches_single_problem_solver():
    bt = small_batch(B=9, nmin=50, nmax=400, seed=3)
    f, g, _, _ = run_batched(bt, 30)
    for b in range(bt.B):
        pr = bt.problem(b)
        fs, gs, info = uot.ti_sinkhorn(dev(pr.alpha), dev(pr.beta), x=dev(pr.x), y=dev(pr.y), eps=pr.eps,
                                       rho1=pr.rho1, rho2=pr.rho2, max_iter=30)
        assert rel_inf(f[bt.offN[b]:bt.offN[b + 1]], fs.cpu().numpy()) < TOL
        assert rel_inf(g[bt.offM[b]:bt.offM[b + 1]], gs.cpu().numpy()) < TOL


def test_batched_bad_problems_are_isolated():
    bt = small_batch(B=6, nmin=3, nmax=40, seed=5)
    a = bt.alpha.copy()
    a[bt.offN[1]] = -1.0                      # problem 1: negative weight
    bt.beta[bt.offM[3]:bt.offM[4]] = 0.0      # problem 3: zero mass
    eps = bt.eps.copy()
    eps[4] = -0.1                             # problem 4: bad eps
    bt.alpha = a
    bt.eps = eps
    f, g, it, st = run_batched(bt, 10)
    assert st[1] == uot.BATCH_INVALID and st[3] == uot.BATCH_INVALID and st[4] == uot.BATCH_INVALID
    for b in (0, 2, 5):
        assert st[b] == uot.BATCH_MAX_ITER
        r = oracle_problem(bt, b, 10)
        assert rel_inf(f[bt.offN[b]:bt.offN[b + 1]], r.f) < TOL


def test_batched_sampled_full_size():
    """The full 4096-problem batch (N, M up to 4096, eps down to 1e-3): a fixed number of
    iterations, then sampled problems checked against the oracle run for as many iterations."""
    bt = workloads.batch2d()
    T = 6
    f, g, it, st = run_batched(bt, T)
    assert np.all(it == T)
    rng = np.random.default_rng(0)
    for b in rng.choice(bt.B, size=6, replace=False):
        r = oracle_problem(bt, int(b), T)
        fb = f[bt.offN[b]:bt.offN[b + 1]]
        gb = g[bt.offM[b]:bt.offM[b + 1]]
        assert rel_inf(fb, r.f) < TOL and rel_inf(gb, r.g) < TOL, (b, rel_inf(fb, r.f))


def test_batched_low_eps_converged():
    """The smallest-eps problems of the 4096-problem batch (eps from 1e-3): the whole batch runs
    to change < 1e-6, then the 8 smallest-eps problems with N_p M_p <= 1.5e6 (the oracle's cost
    stays in seconds) are compared with the oracle run to the GPU's stopping iteration. The
    p = 2 cost is taken through the differences x - y, so its rounding stays relative to each
    entry's own cost (the expanded form would add 2^-24 (d + 4) span^2 per softmin, not small
    against potentials of 0.05-0.2 at these eps)."""
    bt = workloads.batch2d()
    f, g, it, st = run_batched(bt, 100000, tol=1e-6, ce=10)
    assert np.all(st == uot.BATCH_CONVERGED)
    NM = np.diff(bt.offN) * np.diff(bt.offM)
    order = [int(b) for b in np.argsort(bt.eps, kind="stable") if NM[b] <= 1.5e6][:8]
    print("low-eps problems %s, eps %s, iters %s" % (order, bt.eps[order], it[order]),
          file=sys.stderr, flush=True)
    for b in order:
        r = oracle_problem(bt, b, int(it[b]))
        fb = f[bt.offN[b]:bt.offN[b + 1]]
        gb = g[bt.offM[b]:bt.offM[b + 1]]
        assert rel_inf(fb, r.f) < TOL and rel_inf(gb, r.g) < TOL, (b, rel_inf(fb, r.f), rel_inf(gb, r.g))


def test_batched_load_statistics():
    """The per-chunk trace: the work of the running problems never grows, the busy wave time
    of a chunk fits in its duration times the resident waves, and it ends with no problem
    running."""
    bt = small_batch(B=40, nmin=20, nmax=900, seed=11)
    uot.batched_trace(True)
    try:
        run_batched(bt, 5000, tol=1e-6, ce=10)
        tr = uot.batched_trace_read()
    finally:
        uot.batched_trace(False)
    assert len(tr["chunk"]) >= 2 and tr["running"][0] == bt.B and tr["running"][-1] == 0
    assert np.all(np.diff(tr["work"]) <= 0)
    assert np.all(tr["busy_ticks"][1:] <= tr["ticks"][1:] * tr["resident_waves"][1:] * 1.01 + 10)
    assert np.sum(tr["busy_ticks"]) > 0


def test_batched_autotuned_plan():
    """The automatic plan explores one candidate per call for a new size signature (nine:
    item levels and switch points from 256-target items throughout to split items in the
    tail), then keeps the fastest; the potentials agree across every candidate (the plan
    changes only how targets are grouped into work items) and with the oracle."""
    bt = small_batch(B=40, nmin=64, nmax=700, seed=57)
    uot.batched_autotune_reset()
    with _plan(uot.BATCH_PLAN_AUTO):
        runs, plans = [], []
        for _ in range(10):
            runs.append(run_batched(bt, 12))
            plans.append(uot.batched_last_plan())
    assert plans[:9] == [(0, 0, 0.0), (0, 1, 2.0), (0, 1, 8.0), (1, 1, 0.0), (1, 2, 2.0),
                         (1, 2, 8.0), (2, 2, 0.0), (1, 3, 2.0), (1, 3, 0.5)], plans
    assert plans[9] in plans[:9]
    f0, g0 = runs[0][0], runs[0][1]
    for f, g, it, st in runs[1:]:
        assert rel_inf(f, f0) < 1e-6 and rel_inf(g, g0) < 1e-6
        assert np.all(it == 12)
    for b in (0, 17, 39):
        r = oracle_problem(bt, b, 12)
        n0, n1 = bt.offN[b], bt.offN[b + 1]
        m0, m1 = bt.offM[b], bt.offM[b + 1]
        assert rel_inf(f0[n0:n1], r.f) < TOL and rel_inf(g0[m0:m1], r.g) < TOL
    with _plan(uot.BATCH_PLAN_COARSE):
        run_batched(bt, 2)
        assert uot.batched_last_plan() is None
