"""Run-to-run determinism on the GPU: the same call on the same inputs returns bitwise the same
results. Every reduction of the hot path has a fixed order (split partials merged in split
order, block partials in block order, batched item partials in slot order; no float atomics),
so a difference between two runs would point at a race. The first solve of a large shape
times its split counts (the autotuner), so the comparisons start from the second call, when the
shape is cached; the batched solver runs under a fixed work-item plan for the same reason."""
import sys

import numpy as np
import pytest
import torch

import paper_2201_00730_amd as uot
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uot.load_library()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _same(a, b, what):
    a = [t.cpu().numpy() for t in a if t is not None]
    b = [t.cpu().numpy() for t in b if t is not None]
    for x, y in zip(a, b):
        assert x.shape == y.shape and np.array_equal(x.view(np.uint32), y.view(np.uint32)), what


@pytest.mark.parametrize("ti", [True, False])
def test_points_solve_is_deterministic(ti):
    pr = workloads.random_small(3000, 2500, d=3, seed=5, eps=0.02, rho1=0.5, rho2=2.0)
    fn = uot.ti_sinkhorn if ti else uot.sinkhorn
    kw = dict(x=dev(pr.x), y=dev(pr.y), eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2, max_iter=60)
    a, b = dev(pr.alpha), dev(pr.beta)
    fn(a, b, **kw)  # first call of the shape: split counts tuned
    r1 = fn(a, b, **kw)[:2]
    print("points solve ti=%s" % ti, file=sys.stderr, flush=True)
    r2 = fn(a, b, **kw)[:2]
    _same(r1, r2, "points solve")


def test_dense_solve_is_deterministic():
    pr = workloads.random_small(1000, 1200, d=4, seed=6, eps=0.05, rho1=1.0, rho2=1.0, dense=True)
    kw = dict(C=dev(pr.C), eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2, max_iter=40)
    a, b = dev(pr.alpha), dev(pr.beta)
    uot.ti_sinkhorn(a, b, **kw)
    r1 = uot.ti_sinkhorn(a, b, **kw)[:2]
    r2 = uot.ti_sinkhorn(a, b, **kw)[:2]
    _same(r1, r2, "dense solve")


@pytest.mark.parametrize("d", [3, 16])
def test_backward_and_plan_apply_are_deterministic(d):
    pr = workloads.random_small(700, 600, d=d, seed=7 + d, eps=0.05, rho1=0.8, rho2=1.6)
    a, b, x, y = dev(pr.alpha), dev(pr.beta), dev(pr.x), dev(pr.y)
    f, g, _ = uot.ti_sinkhorn(a, b, x=x, y=y, eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2, max_iter=200)
    kw = dict(x=x, y=y, eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2)
    _same(uot.backward(a, b, f, g, **kw), uot.backward(a, b, f, g, **kw), "backward")
    V = torch.randn(pr.m, 20, device="cuda")
    p1 = uot.plan_apply(a, b, f, g, V, x=x, y=y, eps=pr.eps)
    p2 = uot.plan_apply(a, b, f, g, V, x=x, y=y, eps=pr.eps)
    _same([p1], [p2], "plan apply")


def test_batched_solve_is_deterministic():
    bt = workloads.batch2d(B=64, nmin=16, nmax=900, seed=3)
    prev = uot.batched_set_plan(uot.BATCH_PLAN_FINE)
    try:
        runs = []
        for _ in range(2):
            f, g, it, st = uot.ti_sinkhorn_batched(bt.offN, bt.offM, dev(bt.x), dev(bt.y),
                                                   dev(bt.alpha), dev(bt.beta), bt.eps, bt.rho1,
                                                   bt.rho2, p=bt.p, max_iter=300, tol=1e-6,
                                                   check_every=10)
            runs.append((f, g, it, st))
    finally:
        uot.batched_set_plan(prev)
    _same(runs[0][:2], runs[1][:2], "batched potentials")
    assert torch.equal(runs[0][2], runs[1][2]) and torch.equal(runs[0][3], runs[1][3])
