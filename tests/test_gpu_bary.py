"""GPU parity of the 1-D unbalanced barycenter solver (Frank-Wolfe on the multi-marginal
dual, Sec. 5) against the oracle's ``fw_barycenter`` (both double precision), through the C
ABI.

Tolerance: relative 1e-5 (||a - b||_inf / ||b||_inf) on the reported potentials and the
barycenter's points, and 1e-5 of the total mass on its weights (all returned in float32).
Random weights, so that no two cumulative masses tie (with exact ties the balanced
multi-marginal problem has several optimal duals and the two sides may pick different ones).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2201_00730_amd as uot
from tests.helpers import rel_inf

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=dtype))).to("cuda")


def mixtures(K, sizes, seed):
    """K random two-component mixtures on [0, 1] (sorted supports, random weights)."""
    rng = np.random.default_rng(seed)
    xs, ws = [], []
    for k in range(K):
        n = sizes[k]
        c = rng.uniform(0.2, 0.8, 2)
        comp = rng.integers(0, 2, n)
        x = np.clip(rng.normal(c[comp], 0.06), 0.0, 1.0)
        xs.append(np.sort(x).astype(np.float32))
        ws.append((rng.uniform(0.2, 1.0, n) * rng.uniform(0.7, 1.4) / n).astype(np.float32))
    return xs, ws


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uot.load_library()


def _check_problem(f, bx, bw, xs, ws, w, rho, iters, tag):
    off = np.concatenate([[0], np.cumsum([len(x) for x in xs])])
    r = oracle.fw_barycenter(off, np.concatenate(xs).astype(np.float64),
                             np.concatenate(ws).astype(np.float64), w, rho, max_iter=iters)
    ef, ex = rel_inf(f, r.f), rel_inf(bx, r.bary_x)
    ew = np.max(np.abs(bw - r.bary_m)) / r.bary_m.sum()
    _say("  %s rel f %.3g bary x %.3g w %.3g gap %.6g" % (tag, ef, ex, ew, r.gap))
    assert ef < TOL and ex < TOL and ew < TOL, (ef, ex, ew)
    return r


@pytest.mark.parametrize("K", [2, 3, 5])
@pytest.mark.parametrize("iters", [1, 3, 30])
def test_barycenter_parity(K, iters):
    sizes = [37 + 29 * k for k in range(K)]
    xs, ws = mixtures(K, sizes, seed=10 * K + iters)
    w = np.linspace(1.0, 2.0, K)
    w /= w.sum()
    rho = 0.6
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    _say("barycenter K=%d iters=%d" % (K, iters))
    f, bx, bw, it, gap, st = uot.fw1d_barycenter(off, K, dev(np.concatenate(xs)),
                                                 dev(np.concatenate(ws)), dev(w, np.float64), rho,
                                                 max_iter=iters)
    assert int(st[0]) == 1 and int(it[0]) == iters
    r = _check_problem(f.cpu().numpy().astype(np.float64), bx.cpu().numpy().astype(np.float64),
                       bw.cpu().numpy().astype(np.float64), xs, ws, w, rho, iters, "K=%d" % K)
    assert abs(float(gap[0]) - r.gap) <= 1e-9 + 1e-6 * abs(r.gap)


def test_barycenter_batched_ragged_and_invalid():
    """12 problems of K = 4 measures with ragged sizes (single points included) and one
    unsorted measure (reported invalid, the others unaffected)."""
    K, B = 4, 12
    rng = np.random.default_rng(31)
    all_x, all_w, per = [], [], []
    for b in range(B):
        sizes = [int(v) for v in rng.integers(1, 120, K)]
        if b == 0:
            sizes = [1, 1, 1, 1]
        xs, ws = mixtures(K, sizes, seed=300 + b)
        if b == 7 and sizes[2] > 2:
            xs[2] = xs[2][::-1].copy()
        per.append((xs, ws))
        all_x += xs
        all_w += ws
    off = np.concatenate([[0], np.cumsum([len(x) for x in all_x])]).astype(np.int64)
    W = rng.uniform(0.5, 1.5, (B, K))
    W /= W.sum(1, keepdims=True)
    rho = rng.uniform(0.2, 2.0, B)
    _say("barycenter batched")
    f, bx, bw, it, gap, st = uot.fw1d_barycenter(off, K, dev(np.concatenate(all_x)),
                                                 dev(np.concatenate(all_w)),
                                                 dev(W.reshape(-1), np.float64),
                                                 dev(rho, np.float64), max_iter=20)
    f, bx, bw = (v.cpu().numpy().astype(np.float64) for v in (f, bx, bw))
    st = st.cpu().numpy()
    for b in range(B):
        xs, ws = per[b]
        lo, hi = off[b * K], off[(b + 1) * K]
        blo = lo - b * K + b
        bhi = blo + (hi - lo) - K + 1
        if b == 7 and len(xs[2]) > 2:
            assert st[b] == 2 and np.all(np.isnan(f[lo:hi]))
            continue
        assert st[b] == 1
        _check_problem(f[lo:hi], bx[blo:bhi], bw[blo:bhi], xs, ws, W[b], rho[b], 20, "b=%d" % b)


def test_barycenter_more_problems_than_cus():
    """300 problems of K = 3 small measures: more problems than CUs, so each workgroup of the
    narrower launch shape takes several problems in turn."""
    K, B = 3, 300
    rng = np.random.default_rng(77)
    all_x, all_w, per = [], [], []
    for b in range(B):
        sizes = [int(v) for v in rng.integers(1, 40, K)]
        xs, ws = mixtures(K, sizes, seed=1000 + b)
        per.append((xs, ws))
        all_x += xs
        all_w += ws
    off = np.concatenate([[0], np.cumsum([len(x) for x in all_x])]).astype(np.int64)
    W = rng.uniform(0.5, 1.5, (B, K))
    W /= W.sum(1, keepdims=True)
    rho = rng.uniform(0.2, 2.0, B)
    _say("barycenter 300 problems")
    f, bx, bw, it, gap, st = uot.fw1d_barycenter(off, K, dev(np.concatenate(all_x)),
                                                 dev(np.concatenate(all_w)),
                                                 dev(W.reshape(-1), np.float64),
                                                 dev(rho, np.float64), max_iter=15)
    f, bx, bw = (v.cpu().numpy().astype(np.float64) for v in (f, bx, bw))
    assert np.all(st.cpu().numpy() == 1)
    for b in range(0, B, 7):
        xs, ws = per[b]
        lo, hi = off[b * K], off[(b + 1) * K]
        blo = lo - b * K + b
        bhi = blo + (hi - lo) - K + 1
        _check_problem(f[lo:hi], bx[blo:bhi], bw[blo:bhi], xs, ws, W[b], rho[b], 15, "b=%d" % b)


def test_barycenter_sixteen_measures():
    """K = 16, the largest number of measures per problem."""
    K = 16
    sizes = [20 + 3 * k for k in range(K)]
    xs, ws = mixtures(K, sizes, seed=99)
    w = np.linspace(1.0, 3.0, K)
    w /= w.sum()
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    _say("barycenter K=16")
    f, bx, bw, it, gap, st = uot.fw1d_barycenter(off, K, dev(np.concatenate(xs)),
                                                 dev(np.concatenate(ws)), dev(w, np.float64), 0.8,
                                                 max_iter=12)
    assert int(st[0]) == 1 and int(it[0]) == 12
    _check_problem(f.cpu().numpy().astype(np.float64), bx.cpu().numpy().astype(np.float64),
                   bw.cpu().numpy().astype(np.float64), xs, ws, w, 0.8, 12, "K=16")
