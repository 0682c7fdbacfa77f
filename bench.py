"""Throughput benchmark of the GP population evaluator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one evaluation of a resident population on a resident case matrix:
the evaluation kernel (decode, 2D-stack interpretation, per-case error,
per-tile partial sums) and the fixed-order fitness reduction.  Programs and
cases are uploaded before the timed region.  Prints one JSON line.

Workloads (synthetic, seeded):
  scale-tree   4096 PTC2 trees of 1-256 nodes over {+,-,*,/p,sin,cos,exp,log},
               8 features x 65536 cases ~U(-5,5), MSE                (default)
  arith-tree   the same shapes over {+,-,*}
  linear       4096 register programs of 32-256 instructions, 8 registers,
               16 features x 1,048,576 cases ~N(0,1), hit count
  tiny-tree    100 ramped half-and-half trees, 1024 cases, sum |error|
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_T = 157.3   # MI355X vector FP32 peak, TFLOP/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import synth
    if name == "scale-tree":
        return synth.scale_tree_workload()
    if name == "arith-tree":
        return synth.scale_tree_workload(fset=synth.ARITH3)
    if name == "tiny-tree":
        return synth.tiny_tree_workload()
    if name == "linear":
        return synth.linear_workload()
    raise SystemExit("unknown workload " + name)


def gpu_targets(w, Xd):
    """Target values of the workload's target tree, computed by the library
    itself (the first candidate whose values are finite and below 1e6)."""
    import torch
    import paper_1601_00221_amd as gp
    for i in range(w.target.n_prog):
        t = w.target.subset([i])
        out = torch.empty((1, Xd.shape[1]), dtype=torch.float32, device="cuda")
        gp.gp_eval_tree(t.tok, t.cst, t.off, Xd, None, "cases", out)
        v = out[0]
        if bool(torch.isfinite(v).all()) and float(v.abs().max()) < 1e6:
            return (v + torch.from_numpy(w.noise).cuda()).contiguous()
    raise RuntimeError("no acceptable target tree")


def cpu_baseline(w, y_host, budget_s=10.0):
    """The oracle as it stands, on the host cores, on a bounded sample of
    the same workload: every k-th program over all cases."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    tree = hasattr(w, "target")
    P = w.pop.n_prog
    N = w.X.shape[1]

    def run(idx):
        sub = w.pop.subset(idx)
        t0 = time.perf_counter()
        if tree:
            oracle.eval_tree(sub.tok, sub.cst, sub.off, w.X, y_host, w.kind, threads=cores)
            ops = int(np.sum(sub.sizes())) * N
        else:
            oracle.eval_linear(sub.code, sub.off, sub.cst, sub.cst_off, sub.n_reg, w.X, y_host, w.kind,
                               threads=cores)
            ops = int(np.sum(sub.sizes())) * N
        return ops, time.perf_counter() - t0

    probe = np.linspace(0, P - 1, min(P, 2 * cores)).astype(int)
    ops, dt = run(probe)
    rate = ops / max(dt, 1e-9)
    want_ops = rate * budget_s
    mean_ops = ops / len(probe)
    n = int(min(P, max(len(probe), want_ops / max(mean_ops, 1))))
    idx = np.linspace(0, P - 1, n).astype(int)
    ops, dt = run(idx)
    return {"value": ops / dt, "unit": "GPop/s", "cores": cores, "kind": "oracle",
            "sample": "%d of %d programs (evenly spaced) x all %d cases, %.3g GPop in %.1f s"
                      % (n, P, N, ops, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="scale-tree")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the evaluator is built and measured on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1601_00221_amd as gp

    log("workload", args.workload)
    w = make_workload(args.workload)
    N = w.X.shape[1]
    P = w.pop.n_prog
    Xd = torch.from_numpy(w.X).cuda()
    tree = hasattr(w, "target")
    if tree:
        yd = gpu_targets(w, Xd)
        ps = gp.ProgSet.tree(w.pop.tok, w.pop.cst, w.pop.off, w.X.shape[0])
    else:
        yd = torch.from_numpy(w.y).cuda()
        ps = gp.ProgSet.linear(w.pop.code, w.pop.off, w.pop.cst, w.pop.cst_off, w.pop.n_reg, w.X.shape[0])
    info = ps.info()
    gpop_per_step = info["n_gpop"] * N
    out = gp.out_tensor(w.kind, P, N)
    for _ in range(args.warmup):
        ps.eval(Xd, yd, w.kind, out)
    torch.cuda.synchronize()
    gp.timing_read(reset=True)
    gp.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ps.eval(Xd, yd, w.kind, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gp.timing_enable(False)
    n_launch, kernel_ms = gp.timing_read(reset=True)
    step_s = (t1 - t0) / args.steps
    value = gpop_per_step / step_s
    kern_s = kernel_ms / 1e3 / max(n_launch, 1)
    achieved = gpop_per_step / kern_s / 1e12
    log("step %.3f ms, kernel %.3f ms, %.3f T GPop/s" % (step_s * 1e3, kern_s * 1e3, value / 1e12))

    # the same evaluation through the one-shot call: host lowering + PCIe upload included
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        if tree:
            gp.gp_eval_tree(w.pop.tok, w.pop.cst, w.pop.off, Xd, yd, w.kind, out)
        else:
            gp.gp_eval_linear(w.pop.code, w.pop.off, w.pop.cst, w.pop.cst_off, w.pop.n_reg, Xd, yd, w.kind, out)
    torch.cuda.synchronize()
    call_s = (time.perf_counter() - c0) / reps

    res = {
        "metric": "GPop/s (GP ops/sec) + % vector-FP32 peak",
        "value": value,
        "unit": "GPop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_prog": P, "n_cases": N, "n_feat": int(w.X.shape[0]),
                   "fitness": w.kind, "gpop_per_step": gpop_per_step},
        "pct_vector_fp32_peak": 100.0 * value / (PEAK_FP32_T * 1e12),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_T, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_T, "traffic": None,
                     "kernel": "k_eval", "kernel_ms": kern_s * 1e3},
        "call_gpops_per_s": gpop_per_step / call_s,
    }
    if not args.no_cpu:
        y_host = yd.cpu().numpy()
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(w, y_host, args.cpu_budget)
    ps.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
