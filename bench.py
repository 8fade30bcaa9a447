"""Benchmark: C-entry softmin updates/s and time to 1e-6 tolerance, TI vs plain Sinkhorn,
one MI355X.

Workload (one "step"): the 3-D clouds N = M = 20,000 (x ~ U[0,1]^3, y ~ N(0.5, 0.15^2 I),
alpha uniform of mass 1, beta lognormal weights of mass 2, squared Euclidean cost on the
fly, float32). For each (eps, rho) in {1e-1, 1e-2} x {0.1, 1, 10}: translation-invariant
Sinkhorn and plain Sinkhorn from f = 0 to a max potential change < 1e-6 (checked every 10
iterations, cap 100,000), then at the TI solution the dual value, both plan marginals and
the envelope backward (dx, dy, dalpha, dbeta).

value = (sum over the step's solves of 2 N M iterations) / step wall time, i.e. C-entry
softmin updates per second of the whole step. Inputs are resident in HBM before timing.

Also reported: per-(eps, rho) iterations and wall time to tolerance for TI and plain, the
live duration of the dominant kernel (points softmin, timed with HIP events on the solver's
stream) against the transcendental-rate roofline, and the FP64 CPU oracle timed on a
bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EPS_LIST = (1e-1, 1e-2)
RHO_LIST = (0.1, 1.0, 10.0)
TOL = 1e-6
CHECK_EVERY = 10
MAX_ITER = 100000

# MI355X: 256 CUs x 2.4 GHz; the transcendental unit retires 32 v_exp_f32 lanes per clock
# per CU (half the 64-lane FP32 FMA rate), and every C-entry softmin update needs one exp.
PEAK_EXP_PER_S = 256 * 2.4e9 * 32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="", help="restrict to one eps,rho pair, e.g. 0.01,1")
    ap.add_argument("--points-kernel", choices=("auto", "valu", "mfma-f32", "mfma-bf16"),
                    default="auto",
                    help="p = 2 softmin implementation")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--workload", default="cloud3d",
                    choices=("cloud3d", "oned", "stored8d", "batch2d", "highdim16", "anderson",
                             "phi", "fw1d", "bary", "probes"),
                    help="cloud3d (default) is the benchmark step above; the others print one "
                         "JSON line of their own measurement (see extra_workload)")
    return ap.parse_args()


def one_step(uot, torch, tens, pairs, record):
    x, y, a, b = tens["x"], tens["y"], tens["a"], tens["b"]
    n, m = x.shape[0], y.shape[0]
    updates = 0.0
    for eps, rho in pairs:
        for ti in (True, False):
            fn = uot.ti_sinkhorn if ti else uot.sinkhorn
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f, g, info = fn(a, b, x=x, y=y, p=2.0, eps=eps, rho1=rho, rho2=rho, max_iter=MAX_ITER,
                            tol=TOL, check_every=CHECK_EVERY)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            updates += 2.0 * n * m * info.iters
            if record is not None:
                record.append({"eps": eps, "rho": rho, "solver": "ti" if ti else "plain",
                               "iters": info.iters, "converged": info.converged,
                               "last_change": info.last_change, "seconds": dt})
            if ti:
                fti, gti = f, g
        uot.dual_value(a, b, fti, gti, x=x, y=y, eps=eps, rho1=rho, rho2=rho)
        uot.marginals(a, b, fti, gti, x=x, y=y, eps=eps)
        uot.backward(a, b, fti, gti, x=x, y=y, eps=eps, rho1=rho, rho2=rho)
    torch.cuda.synchronize()
    return updates


# Sources compiled into the points softmin kernel (its code, the side reduction it runs, and
# the argument and state layouts): the committed counters hold while these are unchanged.
KERNEL_SOURCES = ("kernels_points.hip", "uot_mx.cuh", "uot_epilogue.cuh", "uot_internal.h")
DENSE_SOURCES = ("kernels_dense.hip", "uot_internal.h")


def profiled_traffic(summary_name="points_softmin_cloud3d_hbm_bytes.md", sources=KERNEL_SOURCES):
    """HBM bytes per launch of a softmin kernel from its committed counter summary, or None
    when the kernel sources have changed since the counters were taken."""
    import hashlib
    import re
    summary = os.path.join(ROOT, "profiles", summary_name)
    csrc = os.path.join(ROOT, "paper_2201_00730_amd", "csrc")
    try:
        text = open(summary).read()
        h = hashlib.sha256()
        for name in sources:
            h.update(open(os.path.join(csrc, name), "rb").read())
        sha = h.hexdigest()
    except OSError:
        return None
    m_sha = re.search(r"source_sha256 \(%s\): ([0-9a-f]{64})" % re.escape(" + ".join(sources)), text)
    m_tr = re.search(r"traffic_bytes_per_launch: ([0-9.]+)", text)
    if not m_sha or not m_tr or m_sha.group(1) != sha:
        return None
    return float(m_tr.group(1))


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def _profiled(uot, kinds):
    """(launches, total ms, total entries) summed over the given profile kinds."""
    n, ms, ent = 0, 0.0, 0.0
    for k in kinds:
        a, b, c = uot.profile_read(k)
        n, ms, ent = n + a, ms + b, ent + c
    return n, ms, ent


RATE_RHOS = (0.01, 0.1, 1.0, 10.0)
RATE_T = 100        # iterations whose errors enter the rate estimate
RATE_FLOOR = 1e-5   # errors below this (float32 potentials) are left out


def kappa(errs, floor=RATE_FLOOR):
    """Contraction rate as the paper's empirical study estimates it (Sec. 3): exp of the
    median over t of log e_{t+1} - log e_t, e_t = ||f_t - f*||_inf, over the pairs above the
    floor."""
    import numpy as np
    d = [np.log(errs[i + 1]) - np.log(errs[i]) for i in range(len(errs) - 1)
         if errs[i] > floor and errs[i + 1] > floor]
    return float(np.exp(np.median(d))) if d else None


def contraction_rates(uot, np, pr, kw, a, b):
    """F- (plain), H- (TI) and G-Sinkhorn (KL and Berg entropies) on the 1-D measures at
    eps = 1e-2 as rho varies: the rate kappa, the iterations to ||f_t - f*|| < 1e-6 and, at
    rho = 1, the error curve. f* is each solver's own limit (run to change < 1e-8), f_t the
    potentials after t iterations from zero."""
    solvers = {
        "F": lambda **k: uot.sinkhorn(a, b, **k),
        "H": lambda **k: uot.ti_sinkhorn(a, b, **k),
        "G_kl": lambda **k: uot.sinkhorn_phi(a, b, entropy="kl", variant="G", **k),
        "G_berg": lambda **k: uot.sinkhorn_phi(a, b, entropy="berg", variant="G", **k),
    }
    out = {}
    for rho in RATE_RHOS:
        kk = dict(kw, rho1=rho, rho2=rho)
        for name, fn in solvers.items():
            fstar = fn(max_iter=MAX_ITER, tol=1e-8, check_every=10, **kk)[0].cpu().numpy().astype(np.float64)
            errs = [float(np.max(np.abs(fn(max_iter=t, tol=0.0, **kk)[0].cpu().numpy().astype(np.float64) - fstar)))
                    for t in range(1, RATE_T + 1)]
            row = {"kappa": kappa(errs),
                   "iters_to_err_1e-6": next((t + 1 for t, e in enumerate(errs) if e < 1e-6), None)}
            if rho == 1.0:
                row["err_t"] = {str(t): errs[t - 1] for t in (1, 2, 5, 10, 20, 50, 100)}
            out.setdefault(name, {})[str(rho)] = row
        print("rates rho=%g %s" % (rho, {n: out[n][str(rho)]["kappa"] for n in solvers}),
              file=sys.stderr, flush=True)
    return out


def extra_workload(args, uot, torch, np, workloads):
    """One JSON line for a workload other than the benchmark step:
    oned      N=M=200 1-D measures: latency per iteration (2000 iterations from 0, TI and
              plain) and time to change < 1e-6; the empirical contraction rates of F-, H- and
              G-Sinkhorn as rho varies (see contraction_rates); the FP64 oracle runs the same
              2000 iterations.
    stored8d  stored 16384^2 float32 cost (||x-y||^1.5, D=8): TI, exactly 500 iterations;
              HBM roofline of the stored-cost softmin kernels (4 bytes of C per entry).
    batch2d   4096 problems, N_p, M_p ~ U{64..4096}, D=2: batched TI to change < 1e-6;
              updates/s = sum_p 2 N_p M_p iters_p / wall.
    highdim16 N=M=50,000, D=16: TI forward to change < 1e-6, then the envelope backward.
    anderson  the benchmark's 3-D clouds and six (eps, rho): time and iterations to change
              < 1e-6 of TI and plain Sinkhorn with and without Anderson extrapolation
              (K = 4, r = 1e-7), with the appendix's mix and with the Gram matrix
              normalised; and the iterations on the 1-D measures of Sec. 3.
    phi       the same clouds at eps = 0.01, rho in {0.1, 1, 10}: time and iterations to change
              < 1e-6 of F- and G-Sinkhorn with the KL and the Berg entropy.
    fw1d      1-D Frank-Wolfe for unregularised UOT: the sorted 1-D measures N=M=200, rho=1,
              5000 iterations with step 2/(2+t) (microseconds per iteration, FP64 oracle on the
              same iterations); and 4096 problems, N_p, M_p ~ U{64..4096}, line search to gap
              1e-9 (point-iterations/s = sum_p (N_p + M_p) iters_p / wall).
    bary      unbalanced 1-D barycenter of K = 8 random mixtures of 2000 points (rho = 0.1),
              1000 Frank-Wolfe iterations (microseconds per iteration, FP64 oracle on 50 of
              them); and 512 such problems with 64..512 points per measure, 500 iterations.
    probes    measured issue rates of v_exp_f32, float32 FMA and double FMA (uot_probe_rate)
              beside the spec-sheet figures the rooflines use."""
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    if args.calibrate_copy:  # a plain 256 MiB device copy, the yardstick of the byte counters
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = {"n_gpus": 1, "dtype": "f32", "data": "synthetic", "vs_baseline": None,
           "higher_is_better": True, "scaling": "weak"}
    if args.workload == "probes":
        rates = issue_rates(uot)
        out.update({"metric": "issue rate", "unit": "lane-ops/s", "value": rates["exp2"],
                    "config": {"workload": "issue-rate probes: 2048 blocks x 256 lanes, 8 "
                                           "independent chains of 2048 steps per lane"},
                    "rates": rates,
                    "spec": {"exp2": PEAK_EXP_PER_S, "fma32": 256 * 4 * 16 * 2.4e9,
                             "fma64": 256 * 4 * 16 * 2.4e9, "mfma_f64_flops": 78.6e12,
                             "mfma_f32_flops": 157.3e12, "mfma_bf16_flops": 2.5e15},
                    "roofline": None})
        print(json.dumps(out))
        return
    if args.workload == "oned":
        pr = workloads.oned()
        a, b, x, y = t(pr.alpha), t(pr.beta), t(pr.x), t(pr.y)
        kw = dict(x=x, y=y, p=2.0, eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2)
        res = {}
        for name, fn in (("ti", uot.ti_sinkhorn), ("plain", uot.sinkhorn)):
            fn(a, b, max_iter=10, **kw)  # warm
            _, dt = _timed(torch, lambda: fn(a, b, max_iter=2000, tol=0.0, **kw))
            (_, _, info), dt_tol = _timed(torch, lambda: fn(a, b, max_iter=MAX_ITER, tol=TOL,
                                                           check_every=1, **kw))
            res[name] = {"us_per_iteration": dt / 2000 * 1e6, "iters_to_tol": info.iters,
                         "seconds_to_tol": dt_tol}
        rates = contraction_rates(uot, np, pr, kw, a, b)
        import oracle
        cost = oracle.Cost(x=pr.x.astype(np.float64), y=pr.y.astype(np.float64), p=2.0)
        t0 = time.perf_counter()
        for ti in (True, False):
            oracle.sinkhorn(cost, pr.alpha.astype(np.float64), pr.beta.astype(np.float64),
                            pr.eps, pr.rho1, pr.rho2, ti=ti, max_iter=2000)
        cpu = (time.perf_counter() - t0) / 4000 * 1e6
        out.update({"metric": "microseconds per Sinkhorn iteration (latency bound)",
                    "value": res["ti"]["us_per_iteration"], "unit": "us/iteration",
                    "higher_is_better": False,
                    "config": {"workload": "1-D measures N=M=200, eps=1e-2, rho=1"},
                    "solvers": res, "contraction_rates": rates, "roofline": None,
                    "cpu_baseline": {"value": cpu, "unit": "us/iteration", "kind": "oracle",
                                     "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                                     "sample": "FP64 C oracle, 2000 iterations each of TI and plain"}})
    elif args.workload == "stored8d":
        pr = workloads.stored8d()
        a, b, C = t(pr.alpha), t(pr.beta), t(pr.C)
        kw = dict(C=C, eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2)
        uot.ti_sinkhorn(a, b, max_iter=5, **kw)
        uot.profile_reset()
        uot.profile_enable(True, period=PROFILE_PERIOD)
        (_, _, info), dt = _timed(torch, lambda: uot.ti_sinkhorn(a, b, max_iter=500, tol=0.0, **kw))
        uot.profile_enable(False)
        n, ms, ent = _profiled(uot, (uot.PROFILE_DENSE_COLS, uot.PROFILE_DENSE_ROWS))
        gbs = 4.0 * ent / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out.update({"metric": "C-entry softmin updates/s", "unit": "C-entry softmin updates/s",
                    "value": 2.0 * pr.n * pr.m * info.iters / dt, "ms_per_500_iterations": dt * 1e3,
                    "config": {"workload": "stored cost 16384^2 float32 (||x-y||^1.5, D=8), "
                                           "eps=5e-3, rho=0.5, TI 500 iterations"},
                    "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                                 "frac": gbs / 8000.0,
                                 "traffic": profiled_traffic("dense_softmin_stored8d_hbm_bytes.md",
                                                             DENSE_SOURCES),
                                 "kernel": "k_dense_cols_partial + k_dense_rows (4 B of C per entry)",
                                 "launches": n, "avg_launch_ms": ms / n if n else None}})
    elif args.workload == "batch2d":
        bt = workloads.batch2d()
        x, y, a, b = t(bt.x), t(bt.y), t(bt.alpha), t(bt.beta)
        run = lambda: uot.ti_sinkhorn_batched(bt.offN, bt.offM, x, y, a, b, bt.eps, bt.rho1,
                                              bt.rho2, max_iter=MAX_ITER, tol=TOL,
                                              check_every=CHECK_EVERY)
        # the first calls of this size signature explore the autotuned plan switch (one
        # candidate threshold each); the timed call then runs the fastest
        explore = []
        for _ in range(10):
            _, dte = _timed(torch, run)
            lv0, lv1, tau = uot.batched_last_plan()
            explore.append({"levels": [lv0, lv1], "threshold": tau, "seconds": dte})
        (f, g, iters, status), dt = _timed(torch, run)
        chosen = uot.batched_last_plan()
        it = iters.cpu().numpy().astype(np.float64)
        N = np.diff(bt.offN).astype(np.float64)
        M = np.diff(bt.offM).astype(np.float64)
        ups = float((2.0 * N * M * it).sum())
        hist = np.percentile(it, [0, 50, 90, 99, 100]).tolist()
        edges = [0, 20, 50, 100, 200, 500, 1000, 2000, 5000, 100000]
        counts, _ = np.histogram(it, bins=edges)
        # a second, traced run: per-chunk load statistics (two clock reads per work item)
        uot.batched_trace(True)
        try:
            _, dt_tr = _timed(torch, run)
            tr = uot.batched_trace_read()
        finally:
            uot.batched_trace(False)
        ticks, busy, waves = tr["ticks"][1:], tr["busy_ticks"][1:], tr["resident_waves"][1:]
        util = np.where(ticks > 0, busy / np.maximum(ticks * waves, 1.0), 0.0)
        load = {"wave_slot_utilisation": float(busy.sum() / max((ticks * waves).sum(), 1.0)),
                "time_fraction_at_least_90pct_busy": float(ticks[util >= 0.9].sum() / max(ticks.sum(), 1.0)),
                "time_fraction_under_50pct_busy": float(ticks[util < 0.5].sum() / max(ticks.sum(), 1.0)),
                "chunks": int(len(ticks)), "resident_waves": int(waves[0]) if len(waves) else None,
                "traced_seconds": dt_tr,
                "running_at_chunk": {str(int(c)): int(r) for c, r in
                                     zip(tr["chunk"], tr["running"]) if int(c) in
                                     (0, 1, 2, 5, 10, 20, 50, 100)},
                "seconds_by_running": {}}
        for lo, hi in ((1025, 1 << 30), (257, 1024), (33, 256), (1, 32)):
            sel = (tr["running"][1:] >= lo) & (tr["running"][1:] <= hi)
            load["seconds_by_running"]["%d-%d" % (lo, min(hi, bt.B))] = \
                float(ticks[sel].sum() / max(ticks.sum(), 1.0) * dt_tr)
        out.update({"metric": "C-entry softmin updates/s", "unit": "C-entry softmin updates/s",
                    "value": ups / dt, "seconds": dt,
                    "config": {"workload": "4096 problems, N_p,M_p ~ U{64..4096}, D=2, "
                                           "eps log-U[1e-3,1e-1], rho log-U[0.1,10], TI to 1e-6"},
                    "autotune": {"item_levels": "0: <= 256 targets per item, 1: <= 128, 2: <= 64, "
                                                "3: 64 with sources split in ranges of 512",
                                 "explored": explore[:9],
                                 "chosen": {"levels": list(chosen[:2]), "threshold": chosen[2]}},
                    "iterations_percentiles_0_50_90_99_100": hist,
                    "iterations_histogram": {"%d-%d" % (edges[i], edges[i + 1] - 1): int(counts[i])
                                             for i in range(len(counts)) if counts[i]},
                    "load": load,
                    "status_counts": {str(k): int(v) for k, v in
                                      zip(*np.unique(status.cpu().numpy(), return_counts=True))},
                    "roofline": {"bound": "alu", "achieved": ups / dt / 1e9,
                                 "peak": PEAK_EXP_PER_S / 1e9, "unit": "Gexp/s",
                                 "frac": ups / dt / PEAK_EXP_PER_S, "traffic": None,
                                 "kernel": "k_batched_half (whole solve wall time, not per launch)"}})
    elif args.workload == "anderson":
        res = {}
        total = {"ti": 0.0, "ti_anderson": 0.0, "ti_anderson_normalised": 0.0, "plain": 0.0,
                 "plain_anderson": 0.0, "plain_anderson_normalised": 0.0}
        acc = dict(K=4, r=1e-7)
        accn = dict(K=4, r=1e-7, normalize=True)
        variants = (("ti", uot.ti_sinkhorn, {}), ("ti_anderson", uot.ti_sinkhorn_anderson, acc),
                    ("ti_anderson_normalised", uot.ti_sinkhorn_anderson, accn),
                    ("plain", uot.sinkhorn, {}), ("plain_anderson", uot.sinkhorn_anderson, acc),
                    ("plain_anderson_normalised", uot.sinkhorn_anderson, accn))
        pr1 = workloads.oned()
        kw1 = dict(x=t(pr1.x), y=t(pr1.y), p=2.0, eps=pr1.eps, rho1=pr1.rho1, rho2=pr1.rho2,
                   max_iter=MAX_ITER, tol=TOL, check_every=CHECK_EVERY)
        oned_iters = {name: fn(t(pr1.alpha), t(pr1.beta), **kw1, **extra)[2].iters
                      for name, fn, extra in variants}
        print("anderson oned iterations %s" % oned_iters, file=sys.stderr, flush=True)
        for eps in (1e-1, 1e-2):
            for rho in (0.1, 1.0, 10.0):
                pr = workloads.cloud3d(n=args.n, m=args.n, eps=eps, rho=rho)
                a, b, x, y = t(pr.alpha), t(pr.beta), t(pr.x), t(pr.y)
                kw = dict(x=x, y=y, p=2.0, eps=eps, rho1=rho, rho2=rho, max_iter=MAX_ITER, tol=TOL,
                          check_every=CHECK_EVERY)
                row = {}
                if not res:  # first launches of each entry point, untimed
                    for fn in (uot.ti_sinkhorn, uot.sinkhorn):
                        fn(a, b, **dict(kw, max_iter=5))
                    for fn in (uot.ti_sinkhorn_anderson, uot.sinkhorn_anderson):
                        fn(a, b, K=4, r=1e-7, **dict(kw, max_iter=5))
                for name, fn, extra in variants:
                    (_, _, info), dt = _timed(torch, lambda: fn(a, b, **kw, **extra))
                    row[name] = {"iters": info.iters, "seconds": round(dt, 5),
                                 "converged": info.converged}
                    total[name] += dt
                res["eps=%g,rho=%g" % (eps, rho)] = row
                print("anderson eps=%g rho=%g %s" % (eps, rho, row), file=sys.stderr, flush=True)
        out.update({"metric": "seconds to change < 1e-6, TI with Anderson extrapolation, summed "
                              "over six (eps, rho)", "unit": "s", "higher_is_better": False,
                    "value": total["ti_anderson"], "totals_seconds": total,
                    "oned_iterations_to_tol": oned_iters,
                    "config": {"workload": "3-D clouds N=M=%d, eps in {0.1,0.01} x rho in "
                                           "{0.1,1,10}, K=4, r=1e-7, change checked every %d"
                                           % (args.n, CHECK_EVERY)},
                    "time_to_tol": res, "roofline": None})
    elif args.workload == "phi":
        res = {}
        total = {}
        for rho in (0.1, 1.0, 10.0):
            pr = workloads.cloud3d(n=args.n, m=args.n, eps=1e-2, rho=rho)
            a, b, x, y = t(pr.alpha), t(pr.beta), t(pr.x), t(pr.y)
            kw = dict(x=x, y=y, p=2.0, eps=1e-2, rho1=rho, rho2=rho, max_iter=MAX_ITER, tol=TOL,
                      check_every=CHECK_EVERY)
            if not res:  # first launches, untimed
                for ent in ("kl", "berg"):
                    for var in ("F", "G"):
                        uot.sinkhorn_phi(a, b, entropy=ent, variant=var, **dict(kw, max_iter=5))
            row = {}
            for ent in ("kl", "berg"):
                for var in ("F", "G"):
                    (_, _, info), dt = _timed(torch, lambda: uot.sinkhorn_phi(
                        a, b, entropy=ent, variant=var, **kw))
                    name = "%s_%s" % (ent, var)
                    row[name] = {"iters": info.iters, "seconds": round(dt, 5),
                                 "converged": info.converged}
                    total[name] = total.get(name, 0.0) + dt
            res["eps=0.01,rho=%g" % rho] = row
            print("phi rho=%g %s" % (rho, row), file=sys.stderr, flush=True)
        out.update({"metric": "seconds to change < 1e-6, G-Sinkhorn with the Berg entropy, summed "
                              "over rho in {0.1, 1, 10}", "unit": "s", "higher_is_better": False,
                    "value": total["berg_G"], "totals_seconds": total,
                    "config": {"workload": "3-D clouds N=M=%d, eps=0.01, rho in {0.1,1,10}, KL "
                                           "and Berg entropies, F- and G-Sinkhorn, change "
                                           "checked every %d" % (args.n, CHECK_EVERY)},
                    "time_to_tol": res, "roofline": None})
    elif args.workload == "fw1d":
        import oracle
        pr = workloads.oned()
        xs = np.sort(pr.x.reshape(-1)).astype(np.float32)
        ys = np.sort(pr.y.reshape(-1)).astype(np.float32)
        a, b, x, y = t(pr.alpha), t(pr.beta), t(xs), t(ys)
        uot.fw1d(x, y, a, b, 1.0, 1.0, max_iter=10)  # warm
        _, dt = _timed(torch, lambda: uot.fw1d(x, y, a, b, 1.0, 1.0, max_iter=5000))
        t0 = time.perf_counter()
        oracle.fw_1d(xs.astype(np.float64), ys.astype(np.float64), pr.alpha.astype(np.float64),
                     pr.beta.astype(np.float64), 1.0, 1.0, max_iter=5000)
        cpu = (time.perf_counter() - t0) / 5000 * 1e6
        bt = workloads.fw1d_batch()
        args_b = (bt.offN, bt.offM, t(bt.x), t(bt.y), t(bt.alpha), t(bt.beta),
                  torch.from_numpy(bt.rho1).to(dev), torch.from_numpy(bt.rho2).to(dev))
        uot.fw1d_batched(*args_b, line_search=True, max_iter=2)  # warm
        (f, g, iters, gap, status), dtb = _timed(torch, lambda: uot.fw1d_batched(
            *args_b, line_search=True, max_iter=2000, tol=1e-9))
        it = iters.cpu().numpy().astype(np.float64)
        pts = np.diff(bt.offN) + np.diff(bt.offM)
        out["dtype"] = "f64"
        out.update({"metric": "microseconds per Frank-Wolfe iteration, 1-D N=M=200 (latency bound)",
                    "value": dt / 5000 * 1e6, "unit": "us/iteration", "higher_is_better": False,
                    "config": {"workload": "sorted 1-D measures N=M=200, rho=1, eps=0, 5000 "
                                           "iterations, step 2/(2+t); and 4096 problems "
                                           "N_p,M_p ~ U{64..4096}, line search to gap 1e-9"},
                    "batched": {"seconds": dtb, "point_iterations_per_s": float((pts * it).sum()) / dtb,
                                "iterations_percentiles_0_50_90_99_100":
                                    np.percentile(it, [0, 50, 90, 99, 100]).tolist(),
                                "status_counts": {str(k): int(v) for k, v in
                                                  zip(*np.unique(status.cpu().numpy(), return_counts=True))}},
                    "roofline": None,
                    "cpu_baseline": {"value": cpu, "unit": "us/iteration", "kind": "oracle", "cores": 1,
                                     "sample": "FP64 C oracle, the same 5000 iterations"}})
    elif args.workload == "bary":
        import oracle
        off, x, a, w, rho = workloads.bary_mixtures()
        K = 8
        xd, ad, wd, rd = t(x), t(a), torch.from_numpy(w).to(dev), torch.from_numpy(rho).to(dev)
        uot.fw1d_barycenter(off, K, xd, ad, wd, rd, max_iter=5)  # warm
        (f, bx, bw, it, gap, st), dt = _timed(torch, lambda: uot.fw1d_barycenter(
            off, K, xd, ad, wd, rd, max_iter=1000))
        t0 = time.perf_counter()
        oracle.fw_barycenter(off, x.astype(np.float64), a.astype(np.float64), w, float(rho[0]),
                             max_iter=50)
        cpu = (time.perf_counter() - t0) / 50 * 1e6
        offb, xb, ab, wb, rb = workloads.bary_mixtures(B=512, nmin=64, nmax=512, seed=8)
        argsb = (offb, K, t(xb), t(ab), torch.from_numpy(wb).to(dev), torch.from_numpy(rb).to(dev))
        uot.fw1d_barycenter(*argsb, max_iter=2)
        (_, _, _, itb, gapb, stb), dtb = _timed(torch, lambda: uot.fw1d_barycenter(*argsb, max_iter=500))
        out["dtype"] = "f64"
        out.update({"metric": "microseconds per Frank-Wolfe barycenter iteration, K=8 x 2000 points",
                    "value": dt / 1000 * 1e6, "unit": "us/iteration", "higher_is_better": False,
                    "config": {"workload": "unbalanced 1-D barycenter of 8 random mixtures x 2000 "
                                           "points, rho=0.1, 1000 iterations; and 512 problems of "
                                           "8 measures x 64..512 points, 500 iterations"},
                    "gap_after_1000": float(gap[0].item()), "status": int(st[0].item()),
                    "batched": {"seconds": dtb, "point_iterations_per_s":
                                float(int(offb[-1]) * 500) / dtb,
                                "gap_median": float(gapb.median().item())},
                    "roofline": None,
                    "cpu_baseline": {"value": cpu, "unit": "us/iteration", "kind": "oracle", "cores": 1,
                                     "sample": "FP64 C oracle, 50 iterations of the same problem"}})
    else:  # highdim16
        pr = workloads.highdim16()
        a, b, x, y = t(pr.alpha), t(pr.beta), t(pr.x), t(pr.y)
        kw = dict(x=x, y=y, p=2.0, eps=pr.eps, rho1=pr.rho1, rho2=pr.rho2)
        uot.ti_sinkhorn(a, b, max_iter=3, **kw)
        uot.profile_reset()
        uot.profile_enable(True, period=PROFILE_PERIOD)
        (f, g, info), dt = _timed(torch, lambda: uot.ti_sinkhorn(
            a, b, max_iter=MAX_ITER, tol=TOL, check_every=CHECK_EVERY, **kw))
        uot.profile_enable(False)
        n, ms, ent = _profiled(uot, (uot.PROFILE_POINTS,))          # expanded form
        nd, msd, entd = _profiled(uot, (uot.PROFILE_POINTS_DIRECT,))  # direct differences
        uot.backward(a, b, f, g, **kw)  # warm
        uot.profile_reset()
        uot.profile_enable(True, period=1)
        _, dtb = _timed(torch, lambda: uot.backward(a, b, f, g, **kw))
        uot.profile_enable(False)
        nb, msb, entb = _profiled(uot, (uot.PROFILE_GRAD,))
        # backward work per entry (one pass per side, p = 2, k_grad_mfma): the inner product
        # <t', s'> on double-precision MFMAs (2 D flops), the gradient sums q s'_k on float32
        # MFMAs (2 D flops); on the vector ALU one add and one FMA in double and one exp2.
        # Peak: the published MFMA peaks (FP64 78.6, FP32 157.3 TFLOP/s), weighted by the time
        # each share takes at its own peak (neither co-executes with vector instructions).
        rates = issue_rates(uot)
        f64, f32 = 2 * pr.d, 2 * pr.d
        peak_b = (f64 + f32) / (f64 / 78.6e12 + f32 / 157.3e12)
        peak_m = (f64 + f32) / (f64 / rates["mfma_f64_flops"] + f32 / rates["mfma_f32_flops"])
        flops_b = (f64 + f32) * entb / (msb * 1e-3) if msb > 0 else 0.0
        ach = ent / (ms * 1e-3) if ms > 0 else 0.0
        achd = entd / (msd * 1e-3) if msd > 0 else 0.0
        direct = info.points_form in (1, 2)
        # forward softmin: the direct form (k_points_partial, p = 2 compiled apart) is float32
        # vector work, D subtractions and D FMAs per entry plus an FMA and an add (3 D + 3
        # flops) against the float32 vector peak; the expanded form is bounded by its exp2.
        # A two-phase solve (points_form 2) runs both: the expanded form while the change is
        # large, the direct form to the tolerance; the line's roofline is the direct kernel's.
        flops_f = (3 * pr.d + 3) * achd
        mx_roof = {"bound": "alu", "achieved": ach / 1e9, "peak": PEAK_EXP_PER_S / 1e9,
                   "unit": "Gexp/s", "frac": ach / PEAK_EXP_PER_S, "traffic": None,
                   "kernel": "k_points_mfma<16,Bf16Form<16>>", "launches": n,
                   "avg_launch_ms": ms / n if n else None}
        fwd_roof = ({"bound": "alu", "achieved": flops_f / 1e12, "peak": 157.3, "unit": "TFLOP/s",
                     "frac": flops_f / 157.3e12, "traffic": None,
                     "kernel": "k_points_partial<16,2,2,true> (direct differences, 3D+3 flops "
                               "per entry)", "launches": nd,
                     "avg_launch_ms": msd / nd if nd else None,
                     "exp_frac": achd / PEAK_EXP_PER_S}
                    if direct else mx_roof)
        if info.points_form == 2:
            fwd_roof["expanded_phase"] = mx_roof
        out.update({"metric": "C-entry softmin updates/s", "unit": "C-entry softmin updates/s",
                    "value": 2.0 * pr.n * pr.m * info.iters / dt,
                    "config": {"workload": "D=16 clouds N=M=50,000, eps=0.05, rho=1, TI to 1e-6 "
                                           "then the envelope backward"},
                    "iters": info.iters, "converged": info.converged, "forward_seconds": dt,
                    "points_form": {0: "expanded", 1: "direct",
                                    2: "expanded, then direct to the tolerance"}[info.points_form],
                    "backward_seconds": dtb,
                    "backward_roofline": {
                        "bound": "mfma", "achieved": flops_b / 1e12, "peak": peak_b / 1e12,
                        "unit": "TFLOP/s", "frac": flops_b / peak_b, "traffic": None,
                        "frac_of_measured_mfma_rates": flops_b / peak_m,
                        "kernel": "k_grad_mfma<16,true,true> (2D FP64 + 2D FP32 MFMA flop + 1 "
                                  "exp2 per entry, both sides)",
                        "launches": nb, "avg_launch_ms": msb / nb if nb else None,
                        "exp_per_s": entb / (msb * 1e-3) if msb > 0 else None,
                        "exp_frac": entb / (msb * 1e-3) / PEAK_EXP_PER_S if msb > 0 else None,
                        "measured_issue_rates": rates},
                    "roofline": fwd_roof})
    print(json.dumps(out))


def issue_rates(uot):
    """Measured chip-wide rates of v_exp_f32, float32 FMA and double FMA (lane-operations/s)
    and of the double, float32 and bf16 MFMAs the kernels use (flop/s)."""
    return {"exp2": uot.probe_rate(uot.PROBE_EXP2), "fma32": uot.probe_rate(uot.PROBE_FMA32),
            "fma64": uot.probe_rate(uot.PROBE_FMA64),
            "mfma_f64_flops": uot.probe_rate(uot.PROBE_MFMA_F64),
            "mfma_f32_flops": uot.probe_rate(uot.PROBE_MFMA_F32),
            "mfma_bf16_flops": uot.probe_rate(uot.PROBE_MFMA_BF16)}


def cpu_baseline(pr, seconds):
    """FP64 oracle TI Sinkhorn on the same inputs for a bounded number of iterations, on all
    the host cores the process may use (OpenMP) and on one core."""
    import numpy as np
    import oracle
    cost = oracle.Cost(x=pr.x.astype(np.float64), y=pr.y.astype(np.float64), p=2.0)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)

    def timed(budget, threads):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.sinkhorn(cost, a, b, 1e-2, 1.0, 1.0, ti=True, max_iter=1)
        t1 = time.perf_counter() - t0
        iters = max(1, int(budget / max(t1, 1e-3)))
        t0 = time.perf_counter()
        oracle.sinkhorn(cost, a, b, 1e-2, 1.0, 1.0, ti=True, max_iter=iters)
        return iters, time.perf_counter() - t0

    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)) or 1))
    prev = oracle.set_threads(cores)
    try:
        iters, dt = timed(seconds, cores)
        iters1, dt1 = timed(max(2.0, seconds / 3.0), 1)
    finally:
        oracle.set_threads(prev)
    return {"value": 2.0 * pr.n * pr.m * iters / dt, "unit": "C-entry softmin updates/s",
            "cores": cores, "kind": "oracle",
            "sample": "FP64 C oracle (OpenMP, %d threads), TI Sinkhorn on the same 3-D clouds "
                      "N=M=%d, eps=1e-2 rho=1, %d iterations from f=0, %.1f s" % (cores, pr.n, iters, dt),
            "single_core": {"value": 2.0 * pr.n * pr.m * iters1 / dt1, "cores": 1,
                            "sample": "the same, one thread, %d iterations, %.1f s" % (iters1, dt1)}}


PROFILE_PERIOD = 15


def kernel_name(variant: str) -> str:
    """Name of the timed softmin kernel of the 3-D workload."""
    if variant == "valu":
        return "k_points_partial<3,kSqEuc,4>"
    return "k_points_mfma<3,%s<3>>" % ("F32Form" if variant == "mfma-f32" else "Bf16Form")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (there is no multi-GPU path); got --gpus %d"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2201_00730_amd as uot
    import workloads

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    uot.load_library()
    uot.set_points_kernel({"auto": 0, "valu": 1, "mfma-f32": 2, "mfma-bf16": 3}[args.points_kernel])
    if args.workload != "cloud3d":
        extra_workload(args, uot, torch, np, workloads)
        return
    pr = workloads.cloud3d(n=args.n, m=args.n)
    dev = torch.device("cuda:0")
    tens = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev)
            for k, v in (("x", pr.x), ("y", pr.y), ("a", pr.alpha), ("b", pr.beta))}
    pairs = [(e, r) for e in EPS_LIST for r in RHO_LIST]
    if args.only:
        e, r = (float(v) for v in args.only.split(","))
        pairs = [(e, r)]

    if args.calibrate_copy:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for w in range(args.warmup):
        one_step(uot, torch, tens, pairs, None)
        print("warmup step %d done" % w, file=sys.stderr, flush=True)

    uot.profile_reset()
    # every 15th softmin launch carries start/stop events on its dispatch (an odd period
    # samples both half-steps; reading the events back synchronises when the ring wraps)
    uot.profile_enable(True, period=PROFILE_PERIOD)
    record = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0.0
    for s in range(args.steps):
        updates += one_step(uot, torch, tens, pairs, record if s == 0 else None)
        print("step %d done" % s, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    uot.profile_enable(False)
    launches, kms, kentries = uot.profile_read(uot.PROFILE_POINTS)

    value = updates / wall
    achieved = kentries / (kms * 1e-3) if kms > 0 else 0.0
    roofline = {"bound": "alu", "achieved": achieved / 1e9, "peak": PEAK_EXP_PER_S / 1e9,
                "unit": "Gexp/s", "frac": achieved / PEAK_EXP_PER_S, "traffic": profiled_traffic(),
                "kernel": kernel_name(args.points_kernel),
                "launches": launches,
                "avg_launch_ms": kms / launches if launches else None,
                "entries_per_launch": kentries / launches if launches else None}
    by_pair = {}
    for r in record:
        key = "eps=%g,rho=%g" % (r["eps"], r["rho"])
        by_pair.setdefault(key, {})[r["solver"]] = {
            "iters": r["iters"], "seconds": round(r["seconds"], 5), "converged": r["converged"]}
    out = {
        "metric": "C-entry softmin updates/s + time to 1e-6 tol, TI vs plain Sinkhorn, 1 GPU",
        "value": value,
        "unit": "C-entry softmin updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3-D clouds N=M=%d, squared Euclidean cost on the fly, "
                               "eps in {0.1,0.01} x rho in {0.1,1,10}, TI and plain to 1e-6"
                               % args.n,
                   "n": args.n, "m": args.n, "d": 3, "tol": TOL, "check_every": CHECK_EVERY},
        "time_to_tol": by_pair,
        "roofline": roofline,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pr, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
