#!/usr/bin/env python3
"""Throughput of batched fitness evaluation on one MI355X.

Workload (default): the full-generation configuration -- 100,000 random
postfix programs (lengths uniform 3..64, ops + - * protected-/ sin cos exp
protected-log sqrt|.| abs), 5 input variables, 4,096 fitness cases, MSE plus
a 1e-3 per-node length tax.  Inputs are resident in HBM before the timed
region; one step = one complete gp_eval call (device-side validation and
staging, depth-class partition, evaluation, fp64 reduction).

Prints one JSON line.  --gpus above 1 is refused: this build runs on one
GPU only.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_LANE_OPS = 256 * 64 * 2.4e9      # fp32 VALU lane-slots per second (non-packed)


def cpu_baseline(w, budget_s=15.0):
    """The fp64 oracle on the host cores, on a bounded sample of programs."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    P = w.pop.n_programs
    # grow the sample until it takes a few seconds, then time a sample sized
    # for the budget
    n = 200
    while True:
        idx = np.arange(min(n, P))
        sub = w.pop.take(idx)
        t0 = time.perf_counter()
        _, _, _, threads = oracle.fitness(sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y,
                                          w.tax, w.allowed_mask, return_threads=True)
        dt = time.perf_counter() - t0
        if dt > 2.0 or n >= P:
            break
        n *= 4
    node_evals = int(sub.offsets[-1]) * w.data.n_cases
    rate = node_evals / dt
    target = min(P, int(n * budget_s / max(dt, 1e-9)))
    if target > n:
        idx = np.arange(target)
        sub = w.pop.take(idx)
        t0 = time.perf_counter()
        _, _, _, threads = oracle.fitness(sub.nodes, sub.offsets, sub.consts, w.data.X, w.data.y,
                                          w.tax, w.allowed_mask, return_threads=True)
        dt = time.perf_counter() - t0
        node_evals = int(sub.offsets[-1]) * w.data.n_cases
        rate = node_evals / dt
    return {"value": rate / 1e9, "unit": "GPOPs", "cores": int(threads), "kind": "oracle",
            "sample": "first %d of %d programs x %d cases (%.3g node-evals, %.1f s)"
                      % (sub.n_programs, P, w.data.n_cases, node_evals, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2607_06731_amd as gp
    from paper_2607_06731_amd import synth

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    gp.lib()
    w = synth.make_config(args.config)
    print("[bench] config %d: %d programs, %d nodes, %d cases, %d vars"
          % (args.config, w.pop.n_programs, int(w.pop.offsets[-1]), w.data.n_cases,
             w.data.n_vars), file=sys.stderr, flush=True)
    pop = gp.DevicePopulation(w.pop.nodes, w.pop.offsets, w.pop.consts)
    data = gp.DeviceDataset(w.data.X, w.data.y)
    out = torch.empty(pop.n_programs, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        gp.gp_eval(pop.nodes, pop.offsets, pop.consts, data.X, data.y, w.tax, out,
                   allowed_op_mask=w.allowed_mask, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: events on the stream the kernels run on
    gp.timing_reset()
    gp.timing_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    gp.timing_enable(False)
    ms_total = start.elapsed_time(stop)
    phases, n_calls = gp.timing_read()
    F = out.cpu().numpy()

    node_evals = w.node_evals
    ms_step = ms_total / args.steps
    gpops = node_evals / (ms_step * 1e-3) / 1e9

    # dominant kernel: evaluation of the depth <= 8 class
    status, maxd, _ = gp.gp_validate(w.pop.nodes, w.pop.offsets, w.pop.consts.size,
                                     w.data.n_vars, w.allowed_mask)
    lens = w.pop.lengths
    cls0 = (status == 0) & (maxd <= 8)
    evals0 = int(lens[cls0].sum()) * w.data.n_cases
    ms0 = phases["eval_d8"] / max(n_calls, 1)
    achieved = evals0 / (ms0 * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_eval<8,4> (depth<=8 class)",
                "achieved": round(achieved, 4), "peak": round(PEAK_LANE_OPS / 1e12, 4),
                "unit": "T node-evals/s vs T fp32 VALU lane-ops/s",
                "frac": round(achieved * 1e12 / PEAK_LANE_OPS, 4), "traffic": None,
                "kernel_ms": round(ms0, 4), "node_evals_per_launch": evals0}
    phase_ms = {k: round(v / max(n_calls, 1), 4) for k, v in phases.items()}

    rec = {
        "metric": "program-node evals/sec (GPOPs)",
        "value": round(gpops, 3),
        "unit": "GPOPs",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config%d: %d programs x %d cases, %d vars, mean len %.1f"
                               % (args.config, w.pop.n_programs, w.data.n_cases,
                                  w.data.n_vars, lens.mean()),
                   "node_evals_per_step": node_evals},
        "frac_of_fp32_valu_lane_peak": round(gpops * 1e9 / PEAK_LANE_OPS, 4),
        "phase_ms": phase_ms,
        "roofline": roofline,
        "n_inf": int(np.isinf(F).sum()),
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
