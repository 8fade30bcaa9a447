"""Envelope backward of the D = 16 differentiable loss, checked with FP64 finite differences
on a 64-point subset (the first 64 points of each cloud of the 50,000-point configuration,
uniform weights of masses 1 and 1.3, eps = 0.05, rho = 1).

Three links, each against something other than the kernel itself:
 1. the oracle's envelope formula (oracle.gradients at its converged FP64 potentials) against
    central differences of its converged value UOT(x, y, alpha, beta), on all 1,024
    coordinates of x, all 64 alpha_i and all 64 beta_j (relative 1e-6 of the largest
    entry): the formula is the derivative of the value;
 2. the GPU backward against that formula at the same float32 potentials (relative 1e-5);
 3. the GPU backward at the GPU's own converged potentials against the finite differences,
    within 1e-5 plus the derived effect of float32 potentials: a potential error delta moves
    every plan entry by a factor e^{delta/eps}, and delta is at least the float32 rounding of
    |f| (2^-24 |f|, |f| ~ 23 here) plus the stopping tolerance.
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
H = 1e-5  # central-difference step


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uot.load_library()


def _value(pr, x, y, a, b, f0):
    cost = oracle.Cost(x=x, y=y, p=2.0)
    r = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, max_iter=100000, tol=1e-14,
                        check_every=1, f0=f0)
    return oracle.dual_value(cost, a, b, pr.eps, pr.rho1, pr.rho2, r.f, r.g)


def test_highdim16_subset_backward_against_finite_differences():
    pr = workloads.highdim16_subset(64)
    x, y = pr.x.astype(np.float64), pr.y.astype(np.float64)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    cost = oracle.Cost(x=x, y=y, p=2.0)
    star = oracle.sinkhorn(cost, a, b, pr.eps, pr.rho1, pr.rho2, ti=True, max_iter=100000,
                           tol=1e-14, check_every=1)
    print("highdim16 subset: FD over 1,152 inputs", file=sys.stderr, flush=True)
    fdx = np.empty_like(x)
    for i in range(x.shape[0]):
        for k in range(x.shape[1]):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += H
            xm[i, k] -= H
            fdx[i, k] = (_value(pr, xp, y, a, b, star.f) - _value(pr, xm, y, a, b, star.f)) / (2 * H)
    fda = np.empty_like(a)
    for i in range(a.size):
        ap, am = a.copy(), a.copy()
        ap[i] += H * a[i]
        am[i] -= H * a[i]
        fda[i] = (_value(pr, x, y, ap, b, star.f) - _value(pr, x, y, am, b, star.f)) / (2 * H * a[i])
    fdb = np.empty_like(b)
    for j in range(b.size):
        bp, bm = b.copy(), b.copy()
        bp[j] += H * b[j]
        bm[j] -= H * b[j]
        fdb[j] = (_value(pr, x, y, a, bp, star.f) - _value(pr, x, y, a, bm, star.f)) / (2 * H * b[j])
    # 1. the formula is the derivative of the value
    ox, oy, oa, ob = oracle.gradients(cost, a, b, pr.eps, pr.rho1, pr.rho2, star.f, star.g)
    assert rel_inf(ox, fdx) < 1e-6 and rel_inf(oa, fda) < 1e-6 and rel_inf(ob, fdb) < 1e-6, \
        (rel_inf(ox, fdx), rel_inf(oa, fda), rel_inf(ob, fdb))
    # 2. the kernel is the formula (same float32 potentials)
    f32, g32 = star.f.astype(np.float32), star.g.astype(np.float32)
    rx, ry, ra, rb = oracle.gradients(cost, a, b, pr.eps, pr.rho1, pr.rho2, f32.astype(np.float64),
                                      g32.astype(np.float64))
    kw = dict(x=_dev(pr.x), y=_dev(pr.y), p=2.0, eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2)
    gx, gy, ga, gb = (v.cpu().numpy() for v in uot.backward(_dev(pr.alpha), _dev(pr.beta),
                                                            _dev(f32), _dev(g32), **kw))
    errs = (rel_inf(gx, rx), rel_inf(gy, ry), rel_inf(ga, ra), rel_inf(gb, rb))
    print("  kernel vs formula at the same potentials: %s" % (errs,), file=sys.stderr, flush=True)
    assert max(errs) < 1e-5, errs
    # 3. the whole float32 chain: GPU solve, then GPU backward, against the differences
    tol = 1e-5
    f, g, info = uot.ti_sinkhorn(_dev(pr.alpha), _dev(pr.beta), max_iter=5000, tol=tol,
                                 check_every=10, **kw)
    hx, hy, ha, hb = (v.cpu().numpy() for v in uot.backward(_dev(pr.alpha), _dev(pr.beta), f, g, **kw))
    fmax = float(np.max(np.abs(star.f)))
    bound = 1e-5 + 4.0 * (2.0 ** -24 * fmax + tol) / pr.eps
    errs = (rel_inf(hx, fdx), rel_inf(ha, fda), rel_inf(hb, fdb))
    print("  GPU chain vs finite differences: %s (bound %.3g, %d iterations)"
          % (errs, bound, info.iters), file=sys.stderr, flush=True)
    assert info.converged and max(errs) < bound, (errs, bound)
