"""Throughput benchmark of the GP population evaluator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one evaluation of a resident population on a resident case matrix:
the evaluation kernel (decode, 2D-stack interpretation, per-case error,
per-block partial sums) and the fixed-order fitness reduction.  Programs and
cases are uploaded before the timed region.  Prints one JSON line.

Workloads (synthetic, seeded):
  scale-tree   4096 PTC2 trees of 1-256 nodes over {+,-,*,/p,sin,cos,exp,log},
               8 features x 65536 cases ~U(-5,5), MSE                (default)
  arith-tree   the same shapes over {+,-,*}
  linear       4096 register programs of 32-256 instructions, 8 registers,
               16 features x 1,048,576 cases ~N(0,1), hit count
  tiny-tree    100 ramped half-and-half trees, 1024 cases, sum |error|
  shuttle      4096 PTC2 trees of 1-256 nodes over {*,/,+,-,>,<,==,AND,OR,IF},
               58,000 Shuttle-shaped cases x 9 inputs, 10 classes, incorrect
               classifications
  kdd          the same over {+,-,*,/,>,<,==,AND,OR,IF,sin,cos,log,exp},
               494,021 KDD-Cup-99-shaped cases x 41 inputs, 22 classes
  batched      10,000 programs in 40 populations (trees and register programs,
               lognormal lengths 8-1024) over three resident case matrices of
               4096 / 65536 / 1,048,576 cases x 8 features, one autotuned
               persistent launch per step; compared with one launch per
               population
  served       32 concurrent GP runs in a closed loop submitting population
               evaluations to the continuous-batching server; p50/p99 latency
               and throughput, compared with one launch per request
  mux20        the 20-multiplexer: 4096 PTC2 trees of 1-256 nodes over
               {AND,OR,NAND,NOR} and the 20 inputs, all 2^20 cases bit-packed
               into 32,768 words per input, hit count (sub-machine-code GP)
  gp-run       whole GP runs with the paper's Table 2 parameters (population
               1000, 50 generations, tournament 7, crossover 0.95, mutation
               0.2): the sextic regression on 100,000 cases and the
               20-multiplexer; GPop/s over the whole run, as the paper counts
  compare-1d   kernel GPop/s of the 2D-stack evaluator against the
               one-dimensional-stack (BlockGP) comparator in postfix and
               stack-operand form, on the scale-tree and arith-tree workloads
  copy-calibration
               a plain 256 MiB device copy, three times: the reference for
               scaling the FETCH_SIZE / WRITE_SIZE counters to bytes

The roofline's HBM traffic comes from the counter records under profiles/
(lines starting "traffic-record:"); a record only counts when it names this
workload and the digest of the kernel's current sources.
"""
import argparse
import glob
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_T = 157.3   # MI355X vector FP32 peak, TFLOP/s (one GP operation counted as one FP32 operation)
# 32-bit vector logic: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, 32 cases per lane-operation
PEAK_BITOP_T = 256 * 4 * 16 * 2.4e9 * 32 / 1e12


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
    if name == "shuttle":
        return synth.shuttle_workload()
    if name == "kdd":
        return synth.kdd_workload()
    raise SystemExit("unknown workload " + name)


def gpu_targets(target, X, noise):
    """Target values: the first candidate target tree whose values on X are
    all finite and below 1e6 in magnitude, computed by the library itself,
    plus the noise."""
    import torch
    import paper_1601_00221_amd as gp
    for i in range(target.n_prog):
        t = target.subset([i])
        out = torch.empty((1, X.shape[1]), dtype=torch.float32, device="cuda")
        gp.gp_eval_tree(t.tok, t.cst, t.off, X, None, "cases", out)
        v = out[0]
        if bool(torch.isfinite(v).all()) and float(v.abs().max()) < 1e6:
            return (v + torch.from_numpy(noise).cuda()).contiguous()
    raise RuntimeError("no acceptable target tree")


def host_cores():
    """Threads the oracle may use: the CPUs this process may run on (at most 16)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return max(1, min(cores, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, y_host, budget_s=10.0):
    """The oracle as it stands, on a bounded sample of the same workload
    (evenly spaced programs over all cases): on all the host cores it may use
    (`value`, `cores`) and on one core (`single_thread`)."""
    import oracle
    tree = hasattr(w.pop, "tok")
    P = w.pop.n_prog
    N = w.X.shape[1]

    def run(idx, threads):
        sub = w.pop.subset(idx)
        t0 = time.perf_counter()
        if tree:
            oracle.eval_tree(sub.tok, sub.cst, sub.off, w.X, y_host, w.kind, threads=threads)
        else:
            oracle.eval_linear(sub.code, sub.off, sub.cst, sub.cst_off, sub.n_reg, w.X, y_host, w.kind,
                               threads=threads)
        return int(np.sum(sub.sizes())) * N, time.perf_counter() - t0

    def timed(threads, budget):
        probe = np.linspace(0, P - 1, min(P, 2 * threads)).astype(int)
        ops, dt = run(probe, threads)
        want_ops = ops / max(dt, 1e-9) * budget
        n = int(min(P, max(len(probe), want_ops / max(ops / len(probe), 1))))
        idx = np.linspace(0, P - 1, n).astype(int)
        ops, dt = run(idx, threads)
        return ops / dt, "%d of %d programs (evenly spaced) x all %d cases, %.3g GPop in %.1f s" % (n, P, N, ops, dt)

    cores = host_cores()
    v_all, s_all = timed(cores, budget_s)
    v_one, s_one = timed(1, budget_s / 2)
    return {"value": v_all, "unit": "GPop/s", "cores": cores, "kind": "oracle", "sample": s_all,
            "single_thread": {"value": v_one, "unit": "GPop/s", "cores": 1, "sample": s_one},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def traffic_record(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from a committed counter
    summary measured with the kernel's current sources, else None."""
    import paper_1601_00221_amd as gp
    digest = gp.kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                line = line.strip().strip("`")
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:] if "=" in x)
                if kv.get("workload") == workload and kv.get("kernel") == kernel and kv.get("source") == digest:
                    return int(kv["bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def counter_record(workload, kernel, tag="valu-record"):
    """Instruction counts per launch of `kernel` on `workload` from a committed
    counter summary measured with the kernel's current sources, else None."""
    import paper_1601_00221_amd as gp
    digest = gp.kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                line = line.strip().strip("`")
                if not line.startswith(tag + ":"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:] if "=" in x)
                if kv.get("workload") == workload and kv.get("kernel") == kernel and kv.get("source") == digest:
                    return kv, os.path.relpath(path, ROOT)
    return None, None


# vector ALU issue rate of the chip: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz
VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4


def op_mix_ceiling(gpop_per_launch, launch_s, kernel, workload):
    """The GPop/s this kernel would reach on this workload if its vector ALUs
    issued on every cycle: GP operations per launch over the time its own
    measured vector instructions take at the full issue rate (their count per
    launch from the committed counter summary of the current sources), and
    the measured rate as a fraction of it."""
    kv, src = counter_record(workload, kernel)
    if kv is None:
        return None
    valu = float(kv["valu_insts"])
    ceil = gpop_per_launch / (valu / VALU_WAVE_INSTS_PER_S)
    achieved = gpop_per_launch / launch_s
    return {"gpops": ceil, "frac": achieved / ceil, "valu_insts_per_launch": valu,
            "gpop_per_valu_lane_op": gpop_per_launch / (valu * 64), "source": src}


def roofline(gpop_per_launch, launch_s, kernel, workload):
    achieved = gpop_per_launch / launch_s / 1e12
    traffic, src = traffic_record(workload, kernel)
    r = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_T, "unit": "TFLOP/s",
         "frac": achieved / PEAK_FP32_T, "traffic": traffic, "kernel": kernel,
         "kernel_ms": launch_s * 1e3}
    if traffic is not None:
        r["traffic_source"] = src
        r["hbm_gbs"] = traffic / launch_s / 1e9
    return r


def base_result(args, value, step_s, config):
    return {
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
        "config": config,
        "pct_vector_fp32_peak": 100.0 * value / (PEAK_FP32_T * 1e12),
    }


def kernel_name(vi):
    import paper_1601_00221_amd as gp
    return gp.variants()[vi]["kernel"] if vi >= 0 else "k_core"


# ----------------------------------------------------------------------------
# one population on one case matrix
# ----------------------------------------------------------------------------
UNPACKED_CEILING_NOTE = ("this path runs unpacked FP32 (packed FP32 is switched off in every build) with terminals "
                         "folded into operands: on {+,-,*} trees it performs about 1.54 GP operations per "
                         "vector lane-operation, so its own ceiling is 39.3 T lane-op/s x 1.54 = 61 T GPop/s")
UNPACKED_CEILING_T = 61.0


def time_population(args, w, steps, warmup):
    """Evaluate a resident population on resident data: warm-up, then `steps`
    timed steps; per-step times from events on the launch stream, the
    evaluation kernel's mean time from the library's own events."""
    import torch
    import paper_1601_00221_amd as gp
    N = w.X.shape[1]
    P = w.pop.n_prog
    Xd = torch.from_numpy(w.X).cuda()
    tree = hasattr(w.pop, "tok")
    if tree:
        yd = gpu_targets(w.target, Xd, w.noise) if hasattr(w, "target") else torch.from_numpy(w.y).cuda()
        ps = gp.ProgSet.tree(w.pop.tok, w.pop.cst, w.pop.off, w.X.shape[0])
    else:
        yd = torch.from_numpy(w.y).cuda()
        ps = gp.ProgSet.linear(w.pop.code, w.pop.off, w.pop.cst, w.pop.cst_off, w.pop.n_reg, w.X.shape[0])
    info = ps.info()
    gpop_per_step = info["n_gpop"] * N
    out = gp.out_tensor(w.kind, P, N)
    for _ in range(warmup):
        ps.eval(Xd, yd, w.kind, out)
    torch.cuda.synchronize()
    gp.timing_read(reset=True)
    gp.timing_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        ps.eval(Xd, yd, w.kind, out)
        ev[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gp.timing_enable(False)
    n_launch, kernel_ms = gp.timing_read(reset=True)
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return dict(ps=ps, Xd=Xd, yd=yd, out=out, info=info, gpop_per_step=gpop_per_step,
                step_s=(t1 - t0) / steps, kern_s=kernel_ms / 1e3 / max(n_launch, 1),
                step_ms_median=float(np.median(step_ms)), step_ms_p10=float(np.percentile(step_ms, 10)),
                step_ms_p90=float(np.percentile(step_ms, 90)))


def bench_single(args):
    import torch
    import paper_1601_00221_amd as gp

    w = make_workload(args.workload)
    N = w.X.shape[1]
    P = w.pop.n_prog
    tree = hasattr(w.pop, "tok")
    m = time_population(args, w, args.steps, args.warmup)
    ps, Xd, yd, out, info = m["ps"], m["Xd"], m["yd"], m["out"], m["info"]
    gpop_per_step, step_s, kern_s = m["gpop_per_step"], m["step_s"], m["kern_s"]
    value = gpop_per_step / step_s
    log("step %.3f ms (median %.3f, p10 %.3f, p90 %.3f), kernel %.3f ms, %.3f T GPop/s"
        % (step_s * 1e3, m["step_ms_median"], m["step_ms_p10"], m["step_ms_p90"], kern_s * 1e3, value / 1e12))

    # the same evaluation through the one-shot call: host lowering, translation and upload included
    def call():
        if tree:
            gp.gp_eval_tree(w.pop.tok, w.pop.cst, w.pop.off, Xd, yd, w.kind, out)
        else:
            gp.gp_eval_linear(w.pop.code, w.pop.off, w.pop.cst, w.pop.cst_off, w.pop.n_reg, Xd, yd, w.kind, out)
    # isolated: each call from an idle device, as in a GP run whose next generation waits for this one's fitness
    iso = []
    for _ in range(5):
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        call()
        torch.cuda.synchronize()
        iso.append(time.perf_counter() - c0)
    iso_s = float(np.median(iso))
    # back to back: calls are asynchronous, so each call's host work overlaps the kernel before it
    # (independent populations, or one population on several datasets)
    reps = max(args.steps, 3)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    call_s = (time.perf_counter() - c0) / reps
    log("one-shot call: isolated %.3f ms, back to back %.3f ms per call" % (iso_s * 1e3, call_s * 1e3))

    config = {"workload": w.name, "n_prog": P, "n_cases": N, "n_feat": int(w.X.shape[0]),
              "fitness": w.kind, "gpop_per_step": gpop_per_step}
    res = base_result(args, value, step_s, config)
    res["step_ms"] = {"median": m["step_ms_median"], "p10": m["step_ms_p10"], "p90": m["step_ms_p90"],
                      "mean": step_s * 1e3, "steps": args.steps}
    kname = kernel_name(info["variant"])
    res["roofline"] = roofline(gpop_per_step, kern_s, kname, w.name)
    res["op_mix_ceiling"] = op_mix_ceiling(gpop_per_step, kern_s, kname, w.name)
    res["call_gpops_per_s"] = gpop_per_step / call_s
    res["call_isolated_gpops_per_s"] = gpop_per_step / iso_s
    ps.close()
    if args.workload == "scale-tree" and not args.no_arith:
        # the same tree shapes over {+,-,*}: the workload on which the 40 % reading is claimed
        wa = make_workload("arith-tree")
        ma = time_population(args, wa, args.steps, args.warmup)
        ka = kernel_name(ma["info"]["variant"])
        va = ma["gpop_per_step"] / ma["step_s"]
        log("arith-tree: step %.3f ms, kernel %.3f ms, %.3f T GPop/s" % (ma["step_s"] * 1e3, ma["kern_s"] * 1e3,
                                                                       va / 1e12))
        ra = roofline(ma["gpop_per_step"], ma["kern_s"], ka, wa.name)
        ra["frac_of_unpacked_ceiling"] = ma["gpop_per_step"] / ma["kern_s"] / (UNPACKED_CEILING_T * 1e12)
        ra["unpacked_ceiling_tgpops"] = UNPACKED_CEILING_T
        ra["unpacked_ceiling_note"] = UNPACKED_CEILING_NOTE
        res["arith"] = {"workload": wa.name, "value": va, "unit": "GPop/s", "ms_per_step": ma["step_s"] * 1e3,
                        "step_ms": {"median": ma["step_ms_median"], "p10": ma["step_ms_p10"],
                                    "p90": ma["step_ms_p90"]},
                        "pct_vector_fp32_peak": 100.0 * va / (PEAK_FP32_T * 1e12), "roofline": ra,
                        "op_mix_ceiling": op_mix_ceiling(ma["gpop_per_step"], ma["kern_s"], ka, wa.name)}
        ma["ps"].close()
    if not args.no_cpu:
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(w, yd.cpu().numpy(), args.cpu_budget)
    return res


# ----------------------------------------------------------------------------
# batched: several populations and case matrices in one persistent launch
# ----------------------------------------------------------------------------
def bench_batched(args):
    import torch
    import paper_1601_00221_amd as gp
    import synth

    w = synth.batched_workload()
    dd = []
    for X, tgt, noise in zip(w.X, w.target, w.noise):
        Xd = torch.from_numpy(X).cuda()
        dd.append((Xd, gpu_targets(tgt, Xd, noise)))
    Ns = [X.shape[1] for X in w.X]
    outs = [gp.out_tensor(j.kind, j.pop.n_prog, 0) for j in w.jobs]
    jobs = [gp.make_job(j.pop, j.dataset, j.kind, o) for j, o in zip(w.jobs, outs)]
    gpop_per_step = sum(int(j.pop.sizes().sum()) * Ns[j.dataset] for j in w.jobs)

    log("autotuning ...")
    best, best_ms = gp.gp_tune_batch(dd, jobs, reps=3)
    log("tuned", best.as_dict(), "%.3f ms" % best_ms)
    for _ in range(args.warmup):
        gp.gp_eval_batch(dd, jobs)
    torch.cuda.synchronize()
    gp.timing_read(reset=True)
    gp.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gp.gp_eval_batch(dd, jobs)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    gp.timing_enable(False)
    n_launch, kernel_ms = gp.timing_read(reset=True)
    kern_s = kernel_ms / 1e3 / max(n_launch, 1)
    batched = [o.clone() for o in outs]

    # the comparison: one launch per population, serialised on one stream
    def unbatched():
        for j, o in zip(w.jobs, outs):
            X, y = dd[j.dataset]
            p = j.pop
            if hasattr(p, "tok"):
                gp.gp_eval_tree(p.tok, p.cst, p.off, X, y, j.kind, o)
            else:
                gp.gp_eval_linear(p.code, p.off, p.cst, p.cst_off, p.n_reg, X, y, j.kind, o)
    unbatched()
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 5))
    u0 = time.perf_counter()
    for _ in range(reps):
        unbatched()
    torch.cuda.synchronize()
    unb_s = (time.perf_counter() - u0) / reps
    same = all(torch.equal(a.view(torch.int32), b.view(torch.int32)) for a, b in zip(batched, outs))
    # latency of each population's fitness from the start of a step: every population of the batched step is
    # ready when its one launch ends; one launch per population finishes them one after another
    e0 = torch.cuda.Event(enable_timing=True)
    ends = [torch.cuda.Event(enable_timing=True) for _ in w.jobs]
    torch.cuda.synchronize()
    e0.record()
    for (j, o), ev in zip(zip(w.jobs, outs), ends):
        X, y = dd[j.dataset]
        p = j.pop
        if hasattr(p, "tok"):
            gp.gp_eval_tree(p.tok, p.cst, p.off, X, y, j.kind, o)
        else:
            gp.gp_eval_linear(p.code, p.off, p.cst, p.cst_off, p.n_reg, X, y, j.kind, o)
        ev.record()
    torch.cuda.synchronize()
    lat_unb = np.array([e0.elapsed_time(ev) for ev in ends])
    b_ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    torch.cuda.synchronize()
    for k in range(5):
        b_ev[k].record()
        gp.gp_eval_batch(dd, jobs)
    b_ev[5].record()
    torch.cuda.synchronize()
    lat_b = np.array([b_ev[k].elapsed_time(b_ev[k + 1]) for k in range(5)])
    value = gpop_per_step / step_s
    log("batched %.3f ms/step (%.3f T GPop/s), one launch per population %.3f ms, identical=%s"
        % (step_s * 1e3, value / 1e12, unb_s * 1e3, same))
    config = {"workload": w.name, "n_prog": w.meta["n_prog"], "n_jobs": w.meta["n_jobs"],
              "n_cases": Ns, "n_feat": w.meta["n_feat"], "fitness": "mse", "gpop_per_step": gpop_per_step,
              "tuned": best.as_dict()}
    res = base_result(args, value, step_s, config)
    res["roofline"] = roofline(gpop_per_step, kern_s, kernel_name(best.variant), w.name)
    res["unbatched"] = {"gpops_per_s": gpop_per_step / unb_s, "ms_per_step": unb_s * 1e3,
                        "launches_per_step": len(jobs), "speedup_of_batched": unb_s / step_s,
                        "fitness_identical": same}
    # per population, from the start of a step to its fitness (batched: five steps' durations)
    res["latency_ms"] = {"batched": {"p50": float(np.percentile(lat_b, 50)), "p99": float(np.percentile(lat_b, 99))},
                         "unbatched": {"p50": float(np.percentile(lat_unb, 50)),
                                       "p99": float(np.percentile(lat_unb, 99))}}
    log("latency per population: batched p50 %.2f p99 %.2f ms, one launch per population p50 %.2f p99 %.2f ms"
        % (res["latency_ms"]["batched"]["p50"], res["latency_ms"]["batched"]["p99"],
           res["latency_ms"]["unbatched"]["p50"], res["latency_ms"]["unbatched"]["p99"]))
    return res


# ----------------------------------------------------------------------------
# served: closed-loop GP runs against the continuous-batching server
# ----------------------------------------------------------------------------
def bench_served(args):
    import torch
    import paper_1601_00221_amd as gp
    import synth

    w = synth.served_workload(n_req=args.requests)
    log("served workload generated")
    data = []
    for r in w.runs:
        Xd = torch.from_numpy(r.X).cuda()
        data.append((Xd, gpu_targets(r.target, Xd, r.noise)))
    reqs = []      # per run: list of (pop, gpop)
    for ri, r in enumerate(w.runs):
        F, N = r.X.shape
        lst = []
        for form, start, P in r.requests:
            pool = w.tree_pool if form == 0 else w.lin_pool
            pop = synth.remap_features(synth.pool_slice(pool, start, P), F)
            lst.append((pop, int(pop.sizes().sum()) * N))
        reqs.append(lst)
    total_gpop = sum(g for lst in reqs for _, g in lst)
    n_warm = max(0, min(args.warmup, args.requests - 1))

    def run_mode(batching, budget=0):
        srv = gp.Server(batching=batching, memory_budget=budget,
                        hip_streams=args.hip_streams if batching else 0)
        ids = [srv.add_dataset(X, y) for X, y in data]
        lat = []
        gpop_meas = [0]
        lock = threading.Lock()
        t_first = [None]
        t_last = [0.0]
        errors = []
        results = {}
        done = [0]

        def client(ri):
            try:
                for k, (pop, g) in enumerate(reqs[ri]):
                    out = gp.out_tensor("mse", pop.n_prog, 0)
                    job = gp.make_job(pop, ids[ri], "mse", out)
                    t0 = time.perf_counter()
                    tk = srv.submit(job)
                    rc = srv.wait(tk)
                    t1 = time.perf_counter()
                    if rc != 0:
                        raise gp.GPError(rc, gp.last_error())
                    srv.release(tk)
                    results[(ri, k)] = out
                    with lock:
                        done[0] += 1
                        if done[0] % 32 == 0:
                            log("  %s: %d requests done" % ("served" if batching else "one launch per request",
                                                           done[0]))
                    if k >= n_warm:
                        with lock:
                            lat.append(t1 - t0)
                            gpop_meas[0] += g
                            if t_first[0] is None or t0 < t_first[0]:
                                t_first[0] = t0
                            t_last[0] = max(t_last[0], t1)
                    time.sleep(float(w.runs[ri].think_s[k]))
            except Exception as e:   # reported after the join
                errors.append(repr(e))

        th = [threading.Thread(target=client, args=(ri,)) for ri in range(len(w.runs))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        st = srv.stats()
        srv.close()
        if errors:
            raise RuntimeError("served run failed: " + errors[0])
        lat = np.sort(np.array(lat))
        span = t_last[0] - t_first[0]
        return {"gpops_per_s": gpop_meas[0] / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "requests": int(len(lat)),
                "span_s": span, "mean_batch": st["mean_batch"], "batches": st["batches"]}, results

    def run_open(batching, rate, seed=55):
        """Open loop: the measured requests (those after each run's warm-up)
        arrive as one Poisson stream of `rate` requests per second, taken
        round robin over the runs, whether or not earlier ones are done."""
        srv = gp.Server(batching=batching, hip_streams=args.hip_streams if batching else 0)
        ids = [srv.add_dataset(X, y) for X, y in data]
        order = [(ri, k) for k in range(n_warm, args.requests) for ri in range(len(w.runs))]
        at = np.cumsum(synth.rng_for(seed).exponential(1.0 / rate, len(order)))
        pending = []
        lock = threading.Lock()
        lat, results, errors = [], {}, []
        gpop_meas = [0]
        t_done = [0.0]

        def waiter(ri, k, tk, t_arr, out):
            # one thread per request, started at its arrival: completion is seen when it happens
            try:
                rc = srv.wait(tk)
                t1 = time.perf_counter()
                if rc != 0:
                    raise gp.GPError(rc, gp.last_error())
                srv.release(tk)
                with lock:
                    lat.append(t1 - t_arr)
                    gpop_meas[0] += reqs[ri][k][1]
                    t_done[0] = max(t_done[0], t1)
                    results[(ri, k)] = out
            except Exception as e:   # reported after the join
                errors.append(repr(e))

        t0 = time.perf_counter()
        for i, (ri, k) in enumerate(order):
            dt = t0 + at[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            pop = reqs[ri][k][0]
            out = gp.out_tensor("mse", pop.n_prog, 0)
            t_arr = time.perf_counter()
            tk = srv.submit(gp.make_job(pop, ids[ri], "mse", out))
            th = threading.Thread(target=waiter, args=(ri, k, tk, t_arr, out))
            th.start()
            pending.append(th)
            if (i + 1) % 256 == 0:
                log("  %s: %d requests submitted" % ("served" if batching else "one launch per request", i + 1))
        for th in pending:
            th.join()
        st = srv.stats()
        srv.close()
        if errors:
            raise RuntimeError("open-loop run failed: " + errors[0])
        lat = np.sort(np.array(lat))
        span = t_done[0] - t0
        return {"gpops_per_s": gpop_meas[0] / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "requests": int(len(lat)),
                "span_s": span, "offered_requests_per_s": rate, "mean_batch": st["mean_batch"],
                "batches": st["batches"]}, results

    gp.timing_read(reset=True)
    gp.timing_enable(True)
    served, res_b = run_mode(True)
    torch.cuda.synchronize()
    gp.timing_enable(False)
    n_launch, kernel_ms = gp.timing_read(reset=True)
    log("served", served)
    single, res_s = run_mode(False)
    log("one launch per request", single)
    same = all(torch.equal(res_b[k].view(torch.int32), res_s[k].view(torch.int32)) for k in res_b)
    open_loop = None
    if args.open_load > 0:
        # offered load: a fraction of the closed loop's served throughput, in requests per second
        mean_gpop = float(np.mean([g for lst in reqs for _, g in lst[n_warm:]]))
        rate = args.open_load * served["gpops_per_s"] / mean_gpop
        log("open loop at %.2f requests/s (%.0f %% of the served closed-loop rate)" % (rate, 100 * args.open_load))
        o_b, ob_res = run_open(True, rate)
        log("open loop, served", o_b)
        o_s, os_res = run_open(False, rate)
        log("open loop, one launch per request", o_s)
        open_loop = {"load_fraction": args.open_load, "served": o_b,
                     "unbatched": dict(o_s, speedup_of_served=o_b["gpops_per_s"] / o_s["gpops_per_s"]),
                     "fitness_identical": all(torch.equal(ob_res[k].view(torch.int32), os_res[k].view(torch.int32))
                                              for k in ob_res) and
                                          all(torch.equal(ob_res[k].view(torch.int32), res_b[k].view(torch.int32))
                                              for k in ob_res)}
    admission = None
    if args.budget_frac > 0:
        # device bytes a request holds while in flight (the server's own estimate, restated): core code,
        # program records and groups, fp64 partial sums per 256-case block, units
        def req_bytes(pop, N):
            n_instr = int(pop.sizes().sum()) + pop.n_prog
            return 16 * n_instr + 40 * pop.n_prog + 8 * pop.n_prog * ((N + 255) // 256) + 4096
        per_run = [max(req_bytes(pop, w.runs[ri].X.shape[1]) for pop, _ in reqs[ri]) for ri in range(len(w.runs))]
        working_set = sum(per_run)
        budget = int(max(args.budget_frac * working_set, 1.25 * max(per_run)))
        log("admission: budget %.1f MB = %.0f %% of the %.1f MB working set (every run's largest request in flight)"
            % (budget / 1e6, 100 * budget / working_set, working_set / 1e6))
        adm, res_a = run_mode(True, budget)
        log("served under the budget", adm)
        admission = dict(adm, budget_bytes=budget, working_set_bytes=working_set,
                         budget_fraction=budget / working_set,
                         fitness_identical=all(torch.equal(res_a[k].view(torch.int32), res_b[k].view(torch.int32))
                                               for k in res_a))
    config = {"workload": w.name, "n_runs": len(w.runs), "requests_per_run": args.requests,
              "warmup_requests_per_run": n_warm, "gpop_total": total_gpop, "fitness": "mse",
              "arrivals": "closed loop, Exp(2 ms) think time", "hip_streams": args.hip_streams}
    res = base_result(args, served["gpops_per_s"], served["span_s"] / max(served["requests"], 1), config)
    res["steps"] = served["requests"]
    res["served"] = served
    res["unbatched"] = dict(single, speedup_of_served=served["gpops_per_s"] / single["gpops_per_s"],
                            fitness_identical=same)
    if open_loop is not None:
        res["open_loop"] = open_loop
    if admission is not None:
        res["admission"] = admission
    # kernel time over all batched launches of the served run (warm-up included)
    all_gpop = total_gpop
    res["roofline"] = roofline(all_gpop / max(n_launch, 1), kernel_ms / 1e3 / max(n_launch, 1), "k_core", w.name)
    res["roofline"]["note"] = "mean over the served run's %d launches, several kernel variants" % n_launch
    return res


# ----------------------------------------------------------------------------
# 2D stack against the one-dimensional-stack (BlockGP) comparator
# ----------------------------------------------------------------------------
PAPER_2D_OVER_1D = {"rpn": 1.14, "lgp": 1.40}   # section 4.2 and 5: Tables 4 over 3, 8 over 7 (GTX 670)


def bench_compare_1d(args):
    """Kernel time of the 2D-stack evaluator and of the 1D comparator in its
    postfix (RPN) and stack-operand (LGP) forms on the same population,
    cases and targets; GPop/s from HIP events around each launch."""
    import torch
    import paper_1601_00221_amd as gp
    out_all = {}
    value = None
    step_2d = None
    for base in ("scale-tree", "arith-tree"):
        w = make_workload(base)
        N, P = w.X.shape[1], w.pop.n_prog
        Xd = torch.from_numpy(w.X).cuda()
        yd = gpu_targets(w.target, Xd, w.noise)
        ps = gp.ProgSet.tree(w.pop.tok, w.pop.cst, w.pop.off, w.X.shape[0])
        gpop = ps.info()["n_gpop"] * N
        out = gp.out_tensor(w.kind, P, N)
        runs = {"2d": lambda: ps.eval(Xd, yd, w.kind, out)}
        for form in ("rpn", "lgp"):
            runs["1d_" + form] = (lambda f: lambda: gp.gp_eval_tree_1d(w.pop.tok, w.pop.cst, w.pop.off, Xd, yd,
                                                                      w.kind, out, form=f))(form)
        res = {}
        fits = {}
        for name, fn in runs.items():
            steps = args.steps if name == "2d" else max(1, min(args.steps, 5))
            for _ in range(max(1, args.warmup)):
                fn()
            torch.cuda.synchronize()
            gp.timing_read(reset=True)
            gp.timing_enable(True)
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            gp.timing_enable(False)
            n_launch, ms = gp.timing_read(reset=True)
            kern_s = ms / 1e3 / max(n_launch, 1)
            res[name] = {"gpops": gpop / kern_s, "kernel_ms": kern_s * 1e3, "launches": n_launch}
            fits[name] = out.cpu().numpy().copy()
            log("%s %s: %.3f ms, %.4f T GPop/s" % (base, name, kern_s * 1e3, gpop / kern_s / 1e12))
        for form in ("rpn", "lgp"):
            res["2d_over_1d_" + form] = res["2d"]["gpops"] / res["1d_" + form]["gpops"]
            f1, f2 = fits["1d_" + form], fits["2d"]
            res["max_rel_fitness_diff_" + form] = float(np.nanmax(np.abs(f1 - f2) / np.maximum(np.abs(f2), 1e-30)))
        res.update({"n_prog": P, "n_cases": N, "gpop_per_step": gpop})
        out_all[w.name] = res
        if value is None:
            value, step_2d = res["2d"]["gpops"], res["2d"]["kernel_ms"] / 1e3
            kernel = kernel_name(ps.info()["variant"])
            roof = roofline(gpop, step_2d, kernel, w.name)
        ps.close()
    config = {"workload": "compare-1d", "bases": list(out_all)}
    r = base_result(args, value, step_2d, config)
    r["roofline"] = roof
    r["compare_1d"] = out_all
    r["paper_2d_over_1d"] = PAPER_2D_OVER_1D
    return r


# ----------------------------------------------------------------------------
# Boolean trees over bit-packed cases (sub-machine-code GP, 20-multiplexer)
# ----------------------------------------------------------------------------
def bench_mux20(args):
    import torch
    import paper_1601_00221_amd as gp
    import synth
    w = synth.mux_workload()
    P, n = w.pop.n_prog, w.n_cases
    Xd = torch.from_numpy(w.Xw.view(np.int32)).cuda()
    yd = torch.from_numpy(w.yw.view(np.int32)).cuda()
    ps = gp.ProgSet.boolean(w.pop.tok, w.pop.off, w.Xw.shape[0])
    info = ps.info()
    gpop_per_step = info["n_gpop"] * n
    out = torch.empty(P, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        ps.eval(Xd, yd, "hits", out, n_cases=n)
    torch.cuda.synchronize()
    gp.timing_read(reset=True)
    gp.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ps.eval(Xd, yd, "hits", out, n_cases=n)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gp.timing_enable(False)
    n_launch, kernel_ms = gp.timing_read(reset=True)
    step_s = (t1 - t0) / args.steps
    kern_s = kernel_ms / 1e3 / max(n_launch, 1)
    value = gpop_per_step / step_s
    log("step %.3f ms, kernel %.3f ms, %.1f T GPop/s" % (step_s * 1e3, kern_s * 1e3, value / 1e12))
    config = {"workload": w.name, "n_prog": P, "n_cases": n, "n_feat": int(w.Xw.shape[0]), "fitness": "hits",
              "gpop_per_step": gpop_per_step, "cases_per_word": 32}
    res = base_result(args, value, step_s, config)
    res["dtype"] = "u32"
    res.pop("pct_vector_fp32_peak", None)
    kernel = kernel_name(info["variant"])
    achieved = gpop_per_step / kern_s / 1e12
    traffic, src = traffic_record(w.name, kernel)
    res["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_BITOP_T, "unit": "T bit-op/s",
                       "frac": achieved / PEAK_BITOP_T, "traffic": traffic, "kernel": kernel,
                       "kernel_ms": kern_s * 1e3}
    if traffic is not None:
        res["roofline"]["traffic_source"] = src
    res["paper_gpops"] = 1.411185e12   # the paper's best 20-multiplexer rate (GTX 670), for context
    if not args.no_cpu:
        import oracle
        log("cpu baseline ...")
        # programs in an evenly spread order until the time budget is spent
        idx = np.argsort((np.arange(P) * 2654435761) % P, kind="stable")
        t = time.perf_counter()
        k = 0
        ops = 0
        while k < len(idx) and time.perf_counter() - t < args.cpu_budget:
            sub = w.pop.subset(idx[k:k + 1])
            oracle.eval_bool(sub.tok, sub.off, w.Xw, n, w.yw)
            ops += int(np.sum(sub.sizes())) * n
            k += 1
        dt = time.perf_counter() - t
        res["cpu_baseline"] = {"value": ops / dt, "unit": "GPop/s", "cores": 1, "kind": "oracle",
                               "sample": "%d programs (spread over the population) x all %d cases, %.3g GPop in %.1f s"
                                         % (k, n, ops, dt)}
    ps.close()
    return res


# ----------------------------------------------------------------------------
# whole GP runs (evaluation plus breeding), as the paper measures GPop/s
# ----------------------------------------------------------------------------
PAPER_RUN_GPOPS = {"sextic": 53.193e9, "mux20": 1411.185e9, "shuttle": 55.734e9}   # best of Table 10 (GTX 670)


def bench_gp_run(args):
    import torch
    import paper_1601_00221_amd as gp
    import synth
    runs = {}
    # sextic regression: x^6 - 2x^4 + x^2 on 100,000 cases x ~ U(-1, 1); terminal set {x}
    rng = synth.rng_for(7)
    x = rng.uniform(-1, 1, 100000)
    y = (x ** 6 - 2 * x ** 4 + x ** 2).astype(np.float32)
    Xd = torch.from_numpy(x.astype(np.float32)[None, :]).cuda()
    yd = torch.from_numpy(y).cuda()
    fset = (synth.MUL, synth.PDIV, synth.ADD, synth.SUB, synth.SIN, synth.COS, synth.PLOG, synth.EXPC)
    cfg = gp.evolve_config(fset, kind="mse", seed=11)
    for _ in range(max(0, args.warmup)):
        gp.evolve(gp.evolve_config(fset, kind="mse", pop_size=100, generations=1, seed=1), Xd, yd)
    torch.cuda.synchronize()
    log("sextic run ...")
    r = gp.evolve(cfg, Xd, yd)
    runs["sextic-1000x50-N100000"] = r
    # the 20-multiplexer, all 2^20 cases bit-packed
    Xw, yw, n = synth.mux_cases(4)
    Xb = torch.from_numpy(Xw.view(np.int32)).cuda()
    yb = torch.from_numpy(yw.view(np.int32)).cuda()
    log("20-multiplexer run ...")
    rb = gp.evolve(gp.evolve_config(synth.BOOL_SET, kind="hits", seed=12), Xb, yb, n_cases=n)
    runs["mux20-1000x50"] = rb
    # the Shuttle-shaped classification problem: 58,000 cases x 9 inputs, constants in [-200, 200]
    ws = synth.shuttle_workload(n_prog=1)
    Xs = torch.from_numpy(ws.X).cuda()
    ys = torch.from_numpy(ws.y).cuda()
    log("shuttle-shaped run ...")
    rs = gp.evolve(gp.evolve_config(synth.SHUTTLE_SET, kind="class_err", p_const=0.1, const_range=(-200.0, 200.0),
                                    seed=13), Xs, ys)
    runs["shuttle-1000x50-N58000"] = rs
    out = {}
    for name, v in runs.items():
        out[name] = {"gpops_whole_run": v["gp_ops"] / v["total_seconds"],
                     "gpops_evaluation": v["gp_ops"] / v["eval_seconds"],
                     "gp_ops": v["gp_ops"], "total_s": v["total_seconds"], "eval_s": v["eval_seconds"],
                     "breed_s": v["breed_seconds"], "best_fitness": v["best_fitness"],
                     "best_generation": v["best_generation"], "best_size": v["best_size"],
                     "paper_gpops": PAPER_RUN_GPOPS[name.split("-")[0]]}
        log("%s: %.3f s, %.1f G GPop/s whole run, %.1f G GPop/s evaluation, best %.4g" % (
            name, v["total_seconds"], out[name]["gpops_whole_run"] / 1e9, out[name]["gpops_evaluation"] / 1e9,
            v["best_fitness"]))
    s = out["sextic-1000x50-N100000"]
    config = {"workload": "gp-run", "runs": list(out), "pop_size": 1000, "generations": 50}
    res = base_result(args, s["gpops_whole_run"], s["total_s"], config)
    res["steps"] = 1
    res.pop("pct_vector_fp32_peak", None)
    res["gp_runs"] = out
    return res


def copy_calibration():
    """A plain device copy of known size for scaling the HBM counters."""
    import torch
    n = 64 << 20
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="scale-tree")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-arith", action="store_true", help="scale-tree: skip the {+,-,*} sub-measurement")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--hip-streams", type=int, default=0,
                    help="served: HIP streams for the server's two launch slots (0: the server's default, one "
                         "stream with launches back to back; 2: one each)")
    ap.add_argument("--budget-frac", type=float, default=0.0,
                    help="served: also run under a device-memory budget of this fraction of the working set")
    ap.add_argument("--requests", type=int, default=10, help="served: requests per run")
    ap.add_argument("--open-load", type=float, default=0.0,
                    help="served: also run an open loop at this fraction of the closed loop's served rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the evaluator is built and measured on a single MI355X "
              "(--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    log("workload", args.workload)
    if args.workload == "copy-calibration":
        res = copy_calibration()
    elif args.workload == "batched":
        res = bench_batched(args)
    elif args.workload == "served":
        res = bench_served(args)
    elif args.workload == "compare-1d":
        res = bench_compare_1d(args)
    elif args.workload == "mux20":
        res = bench_mux20(args)
    elif args.workload == "gp-run":
        res = bench_gp_run(args)
    else:
        res = bench_single(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
