"""The allocation-free backward (uot_backward_noalloc), called through the C ABI, against
uot_backward on the same inputs: two calls in a row on the same device, the second with a
smaller problem (the scratch array keeps the first call's contents)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2201_00730_amd as uot
import workloads
from tests.helpers import oracle_cost, rel_inf

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uot.load_library()


def _case(n, m, d, seed):
    pr = workloads.random_small(n, m, d=d, seed=seed, eps=0.05, rho1=0.8, rho2=1.6)
    r = oracle.sinkhorn(oracle_cost(pr), pr.alpha.astype(np.float64), pr.beta.astype(np.float64),
                        pr.eps, pr.rho1, pr.rho2, ti=True, max_iter=100000, tol=1e-12)
    return pr, r.f.astype(np.float32), r.g.astype(np.float32)


def _noalloc(pr, f, g, gout):
    """uot_backward_noalloc through ctypes, outputs allocated before the call."""
    lib = uot.load_library()
    x, y = _dev(pr.x), _dev(pr.y)
    cost = uot._Cost()
    cost.kind, cost.n, cost.m, cost.d = uot.UOT_COST_POINTS, pr.n, pr.m, pr.x.shape[1]
    cost.C, cost.ldc, cost.p = None, 0, pr.p
    cost.x, cost.y = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    a, b, fd, gd = _dev(pr.alpha), _dev(pr.beta), _dev(f), _dev(g)
    outs = [torch.full((pr.n, cost.d), np.nan, device="cuda"),
            torch.full((pr.m, cost.d), np.nan, device="cuda"),
            torch.full((pr.n,), np.nan, device="cuda"), torch.full((pr.m,), np.nan, device="cuda")]
    torch.cuda.synchronize()
    st = lib.uot_backward_noalloc(ctypes.byref(cost), ctypes.c_void_p(a.data_ptr()),
                                  ctypes.c_void_p(b.data_ptr()), pr.eps, pr.rho1, pr.rho2,
                                  ctypes.c_void_p(fd.data_ptr()), ctypes.c_void_p(gd.data_ptr()),
                                  gout, *[ctypes.c_void_p(o.data_ptr()) for o in outs],
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == uot.UOT_OK, lib.uot_last_error()
    return [o.cpu().numpy() for o in outs]


def test_noalloc_backward_matches_backward_twice():
    for n, m, d, seed in ((1500, 1211, 3, 71), (333, 257, 3, 72)):
        print("noalloc backward n=%d m=%d d=%d" % (n, m, d), file=sys.stderr, flush=True)
        pr, f, g = _case(n, m, d, seed)
        got = _noalloc(pr, f, g, 0.7)
        ref = uot.backward(_dev(pr.alpha), _dev(pr.beta), _dev(f), _dev(g), x=_dev(pr.x),
                           y=_dev(pr.y), p=pr.p, eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2,
                           grad_out=0.7)
        for a, b in zip(got, ref):
            b = b.cpu().numpy()
            assert np.all(np.isfinite(a))
            assert rel_inf(a, b) < TOL, rel_inf(a, b)

