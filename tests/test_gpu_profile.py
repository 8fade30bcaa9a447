"""Kernel timing of the solvers (uot_profile_*): with every launch timed, a solve to a
tolerance reports exactly two timed softmins per iteration, each with the entries of the
cost. The solver queues one chunk of iterations past the device's convergence flag, and
those kernels return at once; they are left out, since they would enter the averages with
the full entry count and almost no time."""
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


@pytest.mark.parametrize("dense", [False, True])
def test_profile_counts_working_launches(dense):
    pr = workloads.random_small(900, 700, d=3, seed=21, eps=0.05, rho1=1.0, rho2=1.0, dense=dense)
    kw = dict(C=dev(pr.C)) if dense else dict(x=dev(pr.x), y=dev(pr.y))
    a, b = dev(pr.alpha), dev(pr.beta)
    args = dict(eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2, tol=1e-6, check_every=10, **kw)
    uot.ti_sinkhorn(a, b, max_iter=20, **args)  # the shape's first solve (split counts)
    print("profile dense=%s" % dense, file=sys.stderr, flush=True)
    uot.profile_reset()
    uot.profile_enable(True, period=1)
    try:
        f, g, info = uot.ti_sinkhorn(a, b, max_iter=5000, **args)
        torch.cuda.synchronize()
    finally:
        uot.profile_enable(False)
    kinds = ((uot.PROFILE_DENSE_COLS, uot.PROFILE_DENSE_ROWS) if dense
             else (uot.PROFILE_POINTS, uot.PROFILE_POINTS_DIRECT))
    reads = [uot.profile_read(k) for k in kinds]
    uot.profile_reset()
    n = sum(r[0] for r in reads)
    ent = sum(r[2] for r in reads)
    assert info.converged and info.iters % 10 == 0, info
    assert n == 2 * info.iters, (n, info.iters)
    assert ent == 2.0 * info.iters * pr.n * pr.m, (ent, info.iters)
    assert all(r[1] > 0.0 for r in reads if r[0] > 0)
