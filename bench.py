#!/usr/bin/env python3
"""Throughput of the SAIM sampling path on one MI355X: p-bit spin updates/s.

A step is one round of Algorithm 1 for every replica: the annealing run
(T sweeps over all N_ext spins, the field/decision/residual work of every
visit), the round epilogue (scores, best feasible sample, residual sums) and
the multiplier step.  One spin update is one visit of one site of one replica
(slack spins counted, padding not).  Inputs are resident in HBM before the
timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2]

Prints one JSON line.  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# Algorithmic integer ALU work of one spin update outside the field dot product
# (which the int8 matrix cores do): a quarter of a Philox4x32-10 block
# (10 rounds x 8 32-bit ops / 4), the field combination and beta-grid index
# (8), the threshold compare (2) and the state/residual update (2 + 2M).
ALU_OPS_RNG = 20
ALU_OPS_FIXED = 12
# 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz 32-bit lane-ops per second (the fp32
# vector peak of 157.3 TFLOP/s counts an FMA as two operations).
ALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9


def alu_ops_per_update(m: int) -> int:
    return ALU_OPS_RNG + ALU_OPS_FIXED + 2 * m


def cpu_baseline(prob, par, seconds_target: float = 10.0):
    """The plain CPU oracle on a bounded sample of the same workload: the first
    round of a few replicas with the full sweep count."""
    from oracle import oracle as O
    threads = max(1, min(16, os.cpu_count() or 1))
    prog = O.build_program(prob, par)
    # calibrate on one replica per thread, then size the sample to ~seconds_target
    t0 = time.perf_counter()
    O.sa_round(prog, [0] * prog.m, 0, 0, threads, threads)
    dt = time.perf_counter() - t0
    reps = threads * max(1, min(8, int(seconds_target / max(dt, 1e-3))))
    t0 = time.perf_counter()
    O.sa_round(prog, [0] * prog.m, 0, threads, reps, threads)
    dt = time.perf_counter() - t0
    visits = reps * prog.n_ext * prog.T
    return {"value": visits / dt, "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"round 0 of {reps} replicas x {prog.T} sweeps x {prog.n_ext} spins "
                      f"({visits:.3g} updates, {dt:.1f} s)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=2, choices=[0, 1, 2])
    ap.add_argument("--instance", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sampler shards by replicas and instances, see DESIGN.md)", file=sys.stderr)
        return 2

    import torch
    from paper_2501_04971_amd import binding as B
    from paper_2501_04971_amd import generators as G

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    B.lib()
    prob, par, _ = G.workload(args.workload, args.instance)
    inst = B.Instance(prob, par)
    info = inst.info
    stream = torch.cuda.current_stream()

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        inst.sample_round()
        inst.update_lambda()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        ev[k][0].record(stream)
        inst.sample_round()
        ev[k][1].record(stream)
        inst.update_lambda()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(end)
    round_ms = [a.elapsed_time(b) for a, b in ev]
    sweep_ms = sum(round_ms) / len(round_ms)

    updates_per_step = par.replicas * info.n_ext * par.sweeps
    value = updates_per_step * args.steps / (total_ms / 1e3)
    ops = alu_ops_per_update(info.m) * updates_per_step
    achieved = ops / (sweep_ms / 1e3)
    best = inst.best_feasible()
    inst.close()

    out = {
        "metric": "p-bit spin updates/s",
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int64 exact integer (int8 pair profits)",
        "data": "synthetic (seeded generators of the paper's instance families)",
        "config": {
            "workload": {0: "QKP N=100 d=0.25", 1: "MKP N=250 M=10",
                         2: "QKP N=300 d=1.0"}[args.workload],
            "n_ext": info.n_ext, "constraints": info.m, "replicas": par.replicas,
            "sweeps_per_round": par.sweeps, "updates_per_step": updates_per_step,
            "parallelism": "one GPU, replicas across lanes",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "sweep (annealing run) + round epilogue, per launch",
            "achieved": achieved / 1e12,
            "peak": ALU_PEAK_OPS / 1e12,
            "unit": "Tops/s (32-bit integer)",
            "frac": achieved / ALU_PEAK_OPS,
            "traffic": None,
            "ops_per_update": alu_ops_per_update(info.m),
            "launch_ms": sweep_ms,
        },
        "wall_s": wall,
        "best_feasible_profit": None if best is None else best[0],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, par)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
