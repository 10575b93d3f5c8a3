"""Launch-layout autotuner for the sampling kernels.

Every layout the library offers gives bit-identical results (one replica per
lane, the same Philox counters and the same visit order), so the choice is
purely a speed question, answered by measurement:

* single instances: waves of 64 replicas per workgroup (quadratic kernel 1 or
  4; linear kernel 1..4), for the linear kernel whether the per-site
  constants are staged in LDS or read from global memory, and the
  producer/consumer split (for the quadratic kernel with three or six
  producer waves);
* batches: the persistent grid size.

A probe run with a reduced sweep count times each candidate (the cost of a
sweep does not depend on the sweep count) and the fastest is cached per shape
key in a JSON file (PBIT_TUNE_CACHE, default ~/.cache/pbit/tiling.json).

Fixed by design rather than tuned: replica tiles narrower than a wave (a wave
visits its sites in sequence, so fewer replicas per wave never shortens a
round), the dense-row field update (the block refresh on the int8 matrix
cores replaces it), and the threshold table's placement (always LDS).
"""
from __future__ import annotations

import dataclasses
import json
import os
import statistics

from . import binding as B


def cache_path() -> str:
    return os.environ.get("PBIT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pbit", "tiling.json"))


def _bucket_pow2(v: int) -> int:
    b = 1
    while b < v:
        b <<= 1
    return b


def shape_key(info, replicas: int) -> str:
    """Instances that share a key share a best layout: kernel variant, padded
    spin count, constraint count and replica count rounded up to a power of 2."""
    return f"v{info.variant}-n{info.n_pad}-m{info.m}-r{_bucket_pow2(replicas)}"


def candidates(info):
    """(waves per workgroup, LDS residency, split) triples."""
    if info.variant == 0:
        return [(1, -1, 0), (4, -1, 0), (4, -1, 1), (4, -1, 2)]
    return [(w, r, 0) for w in (1, 2, 3, 4) for r in (0, 1)] + [(4, 1, 1)]


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_rounds(run, reps: int) -> float:
    import torch
    s = torch.cuda.current_stream()
    run()  # warm-up
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        run()
        b.record(s)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune_instance(prob, par, probe_sweeps: int = 40, reps: int = 3, path: str | None = None) -> dict:
    """Times every layout for (prob, par) and caches the fastest."""
    probe = dataclasses.replace(par, sweeps=min(par.sweeps, probe_sweeps))
    inst = B.Instance(prob, probe)
    key = shape_key(inst.info, par.replicas)
    timings = {}
    for wpb, res, split in candidates(inst.info):
        try:
            inst.set_tiling(wpb, res, split)
        except B.PbitError:
            continue  # does not fit this shape
        timings[f"{wpb},{res},{split}"] = _time_rounds(inst.sample_round, reps)
    inst.close()
    best = min(timings, key=timings.get)
    w, r, sp = (int(v) for v in best.split(","))
    entry = {"waves_per_block": w, "lds_resident": r, "split": sp, "probe_ms": timings,
             "probe_sweeps": probe.sweeps}
    cache = load_cache(path)
    cache[key] = entry
    save_cache(cache, path)
    return entry


def apply(inst, prob, par, tune_missing: bool = True, path: str | None = None) -> dict | None:
    """Sets inst's layout from the cache (tuning the shape first if it is
    missing and tune_missing is set)."""
    key = shape_key(inst.info, par.replicas)
    entry = load_cache(path).get(key)
    if entry is None and tune_missing:
        entry = tune_instance(prob, par, path=path)
    if entry is not None:
        inst.set_tiling(entry["waves_per_block"], entry["lds_resident"], entry.get("split", -1))
    return entry


def tune_batch(probs, pars, probe_sweeps: int = 40, reps: int = 2, path: str | None = None) -> dict:
    """Times persistent grid sizes for a batch shape and caches the fastest
    under a key of the member count and the largest member."""
    probe = [dataclasses.replace(q, sweeps=min(q.sweeps, probe_sweeps)) for q in pars]
    timings = {}
    n_cu = None
    for blocks in (0, 128, 192, 384):
        b = B.Batch(probs, probe, blocks=blocks)
        items, nblk, _ = b.shape()
        n_cu = n_cu or nblk
        if str(nblk) in timings:
            b.close()
            continue
        timings[str(nblk)] = _time_rounds(lambda: b.run(1, use_graph=True), reps)
        b.close()
    best = min(timings, key=timings.get)
    key = f"batch-{len(probs)}-r{_bucket_pow2(max(q.replicas for q in pars))}"
    entry = {"blocks": int(best), "probe_ms": timings, "probe_sweeps": probe_sweeps}
    cache = load_cache(path)
    cache[key] = entry
    save_cache(cache, path)
    return entry
