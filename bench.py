#!/usr/bin/env python3
"""Throughput of the SAIM sampling path on one MI355X: p-bit spin updates/s.

A step is one round of Algorithm 1 for every replica: the annealing run
(T sweeps over all N_ext spins, the field/decision/residual work of every
visit), the round epilogue (scores, best feasible sample, residual sums) and
the multiplier step.  One spin update is one visit of one site of one replica
(slack spins counted, padding not).  Inputs are resident in HBM before the
timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2]

Workloads: 0 QKP N=100 d=0.25 (64 replicas, 1000 sweeps), 1 MKP N=250 M=10
(1024 replicas, 2000 sweeps), 2 QKP N=300 d=1 (4096 replicas, 5000 sweeps,
the default), 3 the 512-instance mixed batch (256 QKP N in U{100..300},
256 MKP N in {100,250,500} x M in {5,10,30}, 256 replicas each; one step =
one graph replay of a round of every member).

Prints one JSON line.  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# The concurrent-instances leg runs four instances on four streams besides the
# default one; with four hardware queues per process (HIP's default) two of
# them can land on one queue and run one after the other.  Eight queues, set
# before the HIP runtime starts, give every stream its own.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

# Algorithmic integer ALU work of one spin update outside the field dot product
# (which the int8 matrix cores do for the quadratic kernel): a quarter of a
# Philox4x32-10 block (10 rounds x 8 32-bit ops / 4), the field combination
# and beta-grid index (8), the threshold compare (2) and the state/residual
# update (2 + 2M).
ALU_OPS_RNG = 20
ALU_OPS_FIXED = 12
# 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz 32-bit lane-ops per second (the fp32
# vector peak of 157.3 TFLOP/s counts an FMA as two operations).
ALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
SIMDS = 256 * 4
# int8 matrix-core peak (dense) and LDS bandwidth (128 B/clk/CU)
MFMA_I8_PEAK = 5.0e15
LDS_PEAK = 256 * 128 * 2.4e9

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = os.path.join(ROOT, "paper_2501_04971_amd", "csrc")


def kernel_source_hash() -> str:
    """sha256 over the library's kernel sources (every .h and .hip file, in name
    order): a counter figure recorded for another build of the kernels does not
    describe this one."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_SOURCES)):
        if name.endswith((".h", ".hip")):
            h.update(name.encode())
            with open(os.path.join(KERNEL_SOURCES, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def recorded_counters(kernel: str, workload: int):
    """Counter figures of this kernel build from the rocprofv3 summaries under
    profiles/ (a `bench-counters` block naming the kernel, the workload and the
    source hash they were taken on), or None when no summary matches the
    current sources."""
    import glob
    want = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read()
        start = text.find("<!-- bench-counters")
        if start < 0:
            continue
        block = text[start:text.find("-->", start)]
        rec = {}
        for line in block.splitlines()[1:]:
            if ":" in line:
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        if rec.get("kernel") == kernel and rec.get("workload") == str(workload) and rec.get("sources") == want:
            out = {"file": os.path.relpath(path, ROOT)}
            for k, v in rec.items():
                if k not in ("kernel", "workload", "sources"):
                    out[k] = float(v)
            return out
    return None


WORKLOAD_NAMES = {0: "QKP N=100 d=0.25", 1: "MKP N=250 M=10", 2: "QKP N=300 d=1.0",
                  3: "mixed batch: 256 QKP + 256 MKP, 256 replicas each"}


def alu_ops_per_update(m: int) -> int:
    return ALU_OPS_RNG + ALU_OPS_FIXED + 2 * m


def linear_split_lds(info, n):
    """LDS bytes of the split linear kernel (threshold table, ring, per-site
    constants, coefficient columns, state words)."""
    owords = (n + 31) // 32
    return 18448 + 2 * 32 * 64 * 8 + (32 * info.words + 32) * 16 + owords * 32 * info.m * 4 + info.words * 64 * 4


def quad_secondary(info, updates, seconds):
    """int8 matrix-core ops and LDS bytes per update of the quadratic kernel:
    every block of 32 visits runs 2 NB 32x32x32 int8 products per 64 replicas
    (4096 NB ops per visit-of-64, i.e. 64 NB per update), and reads per visit
    and wave the slab operands (32 x 32 NB bytes per 32 visits), the
    threshold word (256 B) and the site record (32 B, broadcast)."""
    nb = info.n_pad // 32
    mfma_ops = 64 * nb * updates
    lds_bytes = (32 * nb + 256 + 32) / 64 * updates
    return {"mfma_int8": {"achieved": mfma_ops / seconds / 1e12, "peak": MFMA_I8_PEAK / 1e12,
                          "unit": "TOP/s", "frac": mfma_ops / seconds / MFMA_I8_PEAK},
            "lds": {"achieved": lds_bytes / seconds / 1e9, "peak": LDS_PEAK / 1e9, "unit": "GB/s",
                    "frac": lds_bytes / seconds / LDS_PEAK}}


def host_cpu():
    """(logical CPUs of the machine, CPUs this process may run on, CPU model)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return os.cpu_count() or 1, usable, model


# The CPU leg uses every host CPU this process may run on, up to 16 (the share
# a one-GPU host grants a process, whatever the machine has).
HOST_CPU_SHARE = 16


def cpu_baseline(members, seconds_target: float = 15.0):
    """The plain CPU oracle on a bounded sample of the same workload: round 0
    of a few replicas (full sweep count) of the first member(s), one thread
    per usable host CPU."""
    from oracle import oracle as O
    nproc, usable, model = host_cpu()
    threads = max(1, min(HOST_CPU_SHARE, usable))
    t_all, visits_all, desc = 0.0, 0, []
    for prob, par in members:
        prog = O.build_program(prob, par)
        t0 = time.perf_counter()
        O.sa_round(prog, [0] * prog.m, 0, 0, threads, threads)
        dt = time.perf_counter() - t0
        budget = seconds_target / len(members)
        reps = threads * max(1, min(64, int(budget / max(dt, 1e-3))))
        t0 = time.perf_counter()
        O.sa_round(prog, [0] * prog.m, 0, threads, reps, threads)
        dt = time.perf_counter() - t0
        t_all += dt
        visits_all += reps * prog.n_ext * prog.T
        desc.append(f"{reps} replicas x {prog.T} sweeps x {prog.n_ext} spins")
    return {"value": visits_all / t_all, "unit": "spin-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"round 0 of: {'; '.join(desc)} ({visits_all:.3g} updates, {t_all:.1f} s)",
            "host": {"nproc": nproc, "usable_cpus": usable, "model": model,
                     "threads_rule": f"min(usable CPUs, {HOST_CPU_SHARE})"}}


def learned_start_summary(count: int = 400, rounds: int = 300):
    """Samples to reach the plain loop's best feasible profit (less 0.1 %) on
    held-out QKP N=300 d=1 instances (the throughput workload's generator,
    Table 1's QKP settings): plain start (lambda_0 = 0) against the shipped set
    encoder's start and against the scale-only start (the analytic scale times
    the training targets' median), with 95 % bootstrap intervals of the
    geometric-mean ratios over the instances that have a plain feasible sample."""
    from paper_2501_04971_amd import learn as L
    import numpy as np
    if not os.path.exists(L.DEFAULT_WEIGHTS):
        return None
    ms = [L.learn_instance(L.EVAL_SEED_BASE + 20000 + 4 * i) for i in range(count)]  # index % 4 == 0
    probs, pars = [p for p, _ in ms], [q for _, q in ms]
    lam0 = L.predict_lambda0(probs, pars).cpu().numpy().reshape(count, 32)
    lam_c = L.scale_only_lambda0(probs, pars)
    quiet = lambda *a: None  # noqa: E731
    plain = L.run_loop(probs, pars, rounds, log=quiet)
    learned = L.run_loop(probs, pars, rounds, lambda0=lam0, log=quiet)
    const = L.run_loop(probs, pars, rounds, lambda0=lam_c, log=quiet)
    R = pars[0].replicas
    return {"instances": count, "replicas": R, "sweeps": pars[0].sweeps, "rounds": rounds,
            "unit": "samples (annealing runs of 1000 sweeps)",
            "learned": L.compare(plain, learned, rounds, R), "scale_only": L.compare(plain, const, rounds, R),
            "learned_vs_scale_only": L.compare(const, learned, rounds, R)}


def tempering_leg(workload: int, slots: int, rounds: int):
    """The same instance with parallel tempering as the sampler (chains of
    `slots` replicas on a linear beta ladder, exchanges after every sweep; the
    plain kernel, every lane at its own temperature): spin updates/s over
    `rounds` rounds, exchanges included, HIP events on the launch stream."""
    import dataclasses
    import torch
    from paper_2501_04971_amd import binding as B
    from paper_2501_04971_amd import generators as G
    prob, par, _ = G.workload(workload, 0)
    par = dataclasses.replace(par, pt_slots=slots)
    inst = B.Instance(prob, par)
    inst.sample_round()
    inst.update_lambda()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(rounds):
        inst.sample_round()
        inst.update_lambda()
    b.record(s)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / rounds
    updates = par.replicas * inst.info.n_ext * par.sweeps
    inst.close()
    return {"slots": slots, "chains": par.replicas // slots, "rounds": rounds, "ms_per_round": ms,
            "spin_updates_per_s": updates / (ms / 1e3)}


def concurrent_instances(workload: int, count: int, rounds: int):
    """count instances of the workload (indices 0 .. count-1), each on a stream
    of its own, all rounds queued before any is waited on: the chip-level rate
    for the workload's own shape (one instance of the QKP N=300 workload holds
    64 of the 256 CUs).  Streams keep the default priority."""
    import torch
    from paper_2501_04971_amd import binding as B
    from paper_2501_04971_amd import generators as G
    streams = [torch.cuda.Stream() for _ in range(count)]
    insts, updates = [], 0
    for i, st in enumerate(streams):
        prob, par, _ = G.workload(workload, i)
        with torch.cuda.stream(st):
            inst = B.Instance(prob, par, stream=st)
        insts.append(inst)
        updates += par.replicas * inst.info.n_ext * par.sweeps
    for inst in insts:  # warm-up round
        inst.sample_round()
        inst.update_lambda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        for inst in insts:
            inst.sample_round()
            inst.update_lambda()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for inst in insts:
        inst.close()
    return {"instances": count, "rounds": rounds, "ms_per_round": dt / rounds * 1e3,
            "spin_updates_per_s": updates * rounds / dt,
            "timing": "host wall clock around all streams (synchronised before and after)"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=2, choices=[0, 1, 2, 3])
    ap.add_argument("--instance", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the samples-to-target comparison")
    ap.add_argument("--pt-slots", type=int, default=32,
                    help="also time the QKP workload with parallel tempering, chains of this many replicas (0: skip)")
    ap.add_argument("--concurrent", type=int, default=4,
                    help="also time this many instances of the workload side by side (0: skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sampler would shard by replicas and instances across GPUs)", file=sys.stderr)
        return 2

    import torch
    from paper_2501_04971_amd import binding as B
    from paper_2501_04971_amd import generators as G

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    B.lib()
    stream = torch.cuda.current_stream()

    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    batch = args.workload == 3
    if batch:
        from paper_2501_04971_amd import autotune as A
        members = [G.workload(3, i) for i in range(512)]
        mprobs, mpars = [p for p, _, _ in members], [q for _, q, _ in members]
        # the layout the autotuner picks for this batch shape (timed now if not cached)
        tuned = A.load_cache().get(A.batch_key(mprobs, mpars)) or A.tune_batch(mprobs, mpars)
        runner = B.Batch(mprobs, mpars, rounds=[1 << 30] * len(members), layout=tuned["layout"])
        infos = [m.info for m in runner.members]
        updates_per_step = sum(q.replicas * i.n_ext * q.sweeps for (_, q, _), i in zip(members, infos))
        ops_per_step = sum(alu_ops_per_update(p.m) * q.replicas * i.n_ext * q.sweeps
                           for (p, q, _), i in zip(members, infos))

        def step():
            runner.run(1, use_graph=True)
    else:
        prob, par, _ = G.workload(args.workload, args.instance)
        runner = B.Instance(prob, par)
        info = runner.info
        updates_per_step = par.replicas * info.n_ext * par.sweeps
        ops_per_step = alu_ops_per_update(info.m) * updates_per_step

        def step():
            runner.sample_round()

    for _ in range(args.warmup):
        step()
        if not batch:
            runner.update_lambda()
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
        step()
        ev[k][1].record(stream)
        if not batch:
            runner.update_lambda()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = start.elapsed_time(end)
    launch_ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps

    value = updates_per_step * args.steps / (total_ms / 1e3)
    achieved = ops_per_step / (launch_ms / 1e3)
    if batch:
        waves = sum((q.replicas + 255) // 256 * 4 for _, q, _ in members)
        best = None
        kernel = "sweep_batch + round epilogue + multiplier step (one graph replay)"
        secondary = {}
        cfg = {"workload": WORKLOAD_NAMES[3], "instances": len(members), "replicas_each": 256,
               "sweeps_per_round": "QKP 1000, MKP 2000", "updates_per_step": updates_per_step,
               "parallelism": "one GPU, persistent work queue over (instance, 256-replica tile)",
               "layout": {"requested": tuned["layout"], "used": runner.layout(),
                          "probe_ms": tuned["probe_ms"]}}
    else:
        # the layout pbit_sample_round picks by default: the split form whenever
        # one wave per 64 replicas leaves CUs idle and (linear kernel) its LDS fits
        groups = (par.replicas + 63) // 64
        fits = info.variant == 0 or linear_split_lds(info, prob.n) <= 160 * 1024
        split = groups <= torch.cuda.get_device_properties(0).multi_processor_count and fits
        nb = info.n_pad // 32
        producers = 6 if info.variant == 0 else 3  # the library's default for the split form
        waves = (8 if producers == 6 else 4) * groups if split else groups
        best = runner.best_feasible()
        wide = "true" if info.variant == 2 else "false"
        kernel = (f"sweep_quad_pc<{nb}, {producers}>" if split else f"sweep_quad<{nb}>") if info.variant == 0 else \
            (f"sweep_linear_pc<{info.m}, {wide}>" if split else f"sweep_linear<{info.m}, {wide}, ...>")
        secondary = quad_secondary(info, updates_per_step, launch_ms / 1e3) if info.variant == 0 else {}
        cfg = {"workload": WORKLOAD_NAMES[args.workload], "n_ext": info.n_ext, "constraints": info.m,
               "replicas": par.replicas, "sweeps_per_round": par.sweeps,
               "updates_per_step": updates_per_step, "parallelism": "one GPU, replicas across lanes"}
    runner.close()
    # counters are not measured by this run: they are the rocprofv3 figures
    # recorded under profiles/ for these exact kernel sources, if any
    counters = recorded_counters(kernel, args.workload)

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
        "config": cfg,
        "roofline": {
            "bound": "alu",
            "kernel": kernel,
            "achieved": achieved / 1e12,
            "peak": ALU_PEAK_OPS / 1e12,
            "unit": "Tops/s (32-bit integer)",
            "frac": achieved / ALU_PEAK_OPS,
            "traffic": None if counters is None else counters.get("traffic_bytes"),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "ops_per_update": None if batch else alu_ops_per_update(info.m),
            "launch_ms": launch_ms,
            "waves": waves,
            "frac_of_occupied_simds": achieved / (ALU_PEAK_OPS * min(1.0, waves / SIMDS)),
            "secondary": secondary,
            "recorded_counters": counters,
        },
        "wall_s": wall,
        "best_feasible_profit": None if best is None else best[0],
    }
    if args.concurrent > 1 and not batch:
        out["concurrent"] = concurrent_instances(args.workload, args.concurrent, max(2, min(args.steps, 5)))
    if args.pt_slots > 0 and args.workload in (0, 2):
        out["parallel_tempering"] = tempering_leg(args.workload, args.pt_slots, max(2, min(args.steps, 3)))
    if not args.no_learned and args.workload == 2:
        out["samples_to_target"] = learned_start_summary()
    if not args.no_cpu_baseline:
        if batch:
            out["cpu_baseline"] = cpu_baseline([members[0][:2], members[1][:2]])
        else:
            out["cpu_baseline"] = cpu_baseline([(prob, par)])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
