"""Launch-layout autotuner for the sampling kernels.

Every layout the library offers gives bit-identical results (one replica per
lane, the same Philox counters and the same visit order), so the choice is
purely a speed question, answered by measurement:

* single instances: waves of 64 replicas per workgroup (quadratic kernel 1 or
  4; linear kernel 1..4), for the linear kernel whether the per-site
  constants are staged in LDS or read from global memory, and the
  producer/consumer split (for the quadratic kernel with three or six
  producer waves);
* batches: the rule that decides which linear members run as split tiles and
  the linear family's persistent grid (timed on a probe of the whole batch
  with every member's sweep count scaled down by one common factor).

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


def batch_key(probs, pars) -> str:
    """Batches that share a key share a best layout: the member count and the
    multiset of member shapes (kernel variant, padded spins, constraints,
    256-replica tiles, sweeps)."""
    import hashlib
    shapes = sorted((int(i.variant), int(i.n_pad), int(i.m), (q.replicas + 255) // 256, int(q.sweeps))
                    for i, q in ((B.pbit_plan(p, q), q) for p, q in zip(probs, pars)))
    return f"batch-{len(probs)}-{hashlib.sha1(repr(shapes).encode()).hexdigest()[:12]}"


def batch_candidates():
    """Layouts tried for a batch: the split rule for linear members (200 % of
    the average linear load per CU, the default, or 150 / 300 %, or no split)
    and the linear family's grid (one workgroup per resident slot, or 224)."""
    return [{"blocks_quad": 0, "blocks_linear": bl, "split_percent": sp}
            for sp in (200, 150, 300, 0) for bl in (0, 224)]


def probe_params(pars, probe_sweeps: int):
    """Every member's sweep count divided by one common factor, so that the
    members keep their relative costs (a sweep's cost does not depend on the
    sweep count)."""
    f = max(1, max(q.sweeps for q in pars) // probe_sweeps)
    return [dataclasses.replace(q, sweeps=max(1, q.sweeps // f)) for q in pars]


def tune_batch(probs, pars, probe_sweeps: int = 80, reps: int = 2, path: str | None = None) -> dict:
    """Times every candidate layout on a probe of the batch (all members, sweep
    counts scaled down together) and caches the fastest under batch_key."""
    probe = probe_params(pars, probe_sweeps)
    timings = {}
    for cand in batch_candidates():
        b = B.Batch(probs, probe, layout=cand)
        used = b.layout()
        tag = f"{cand['split_percent']},{used['blocks_linear']}"
        if tag not in timings:
            timings[tag] = _time_rounds(lambda: b.run(1, use_graph=True), reps)
        b.close()
    best = min(timings, key=timings.get)
    sp, bl = (int(v) for v in best.split(","))
    entry = {"layout": {"blocks_quad": 0, "blocks_linear": bl, "split_percent": sp}, "probe_ms": timings,
             "probe_sweeps": [q.sweeps for q in probe[:1]] + [max(q.sweeps for q in probe)]}
    cache = load_cache(path)
    cache[batch_key(probs, pars)] = entry
    save_cache(cache, path)
    return entry


def batch_layout(probs, pars, tune_missing: bool = True, path: str | None = None) -> dict | None:
    """The cached layout for this batch shape (tuned first if missing and
    tune_missing is set), as the layout argument of binding.Batch."""
    entry = load_cache(path).get(batch_key(probs, pars))
    if entry is None and tune_missing:
        entry = tune_batch(probs, pars, path=path)
    return None if entry is None else dict(entry["layout"])
