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


def profiled_traffic():
    """HBM bytes per launch of the points softmin from the committed counter summary, or None
    when the kernel source has changed since the counters were taken."""
    import hashlib
    import re
    summary = os.path.join(ROOT, "profiles", "points_softmin_cloud3d_hbm_bytes.md")
    src = os.path.join(ROOT, "paper_2201_00730_amd", "csrc", "kernels_points.hip")
    try:
        text = open(summary).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m_sha = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    m_tr = re.search(r"traffic_bytes_per_launch: ([0-9.]+)", text)
    if not m_sha or not m_tr or m_sha.group(1) != sha:
        return None
    return float(m_tr.group(1))


def cpu_baseline(pr, seconds):
    """FP64 oracle TI Sinkhorn on the same inputs for a bounded number of iterations."""
    import numpy as np
    import oracle
    cost = oracle.Cost(x=pr.x.astype(np.float64), y=pr.y.astype(np.float64), p=2.0)
    a, b = pr.alpha.astype(np.float64), pr.beta.astype(np.float64)
    t0 = time.perf_counter()
    oracle.sinkhorn(cost, a, b, 1e-2, 1.0, 1.0, ti=True, max_iter=1)
    t1 = time.perf_counter() - t0
    iters = max(1, int(seconds / max(t1, 1e-3)))
    t0 = time.perf_counter()
    oracle.sinkhorn(cost, a, b, 1e-2, 1.0, 1.0, ti=True, max_iter=iters)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 2.0 * pr.n * pr.m * iters / dt, "unit": "C-entry softmin updates/s",
            "cores": cores, "kind": "oracle",
            "sample": "FP64 C oracle (OpenMP), TI Sinkhorn on the same 3-D clouds N=M=%d, "
                      "eps=1e-2 rho=1, %d iterations from f=0, %.1f s" % (pr.n, iters, dt)}


PROFILE_PERIOD = 15


def kernel_name(variant: str) -> str:
    """Name of the timed softmin kernel of the 3-D workload."""
    if variant == "valu":
        return "k_points_partial<3,kSqEuc,4>"
    return "k_points_mfma<3,%s<3>>" % ("F32Form" if variant == "mfma-f32" else "Bf16Form")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d"
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
