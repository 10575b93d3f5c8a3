"""Evaluation drivers: the penalty-method baseline, the accuracy metric against
exact optima, and the dual-update variants, on synthetic stand-ins for the
paper's benchmark instances.

    python -m paper_2501_04971_amd.experiments qkp100 --out F.json   (GPU)
    python -m paper_2501_04971_amd.experiments mkp100 --out F.json   (GPU)
    python -m paper_2501_04971_amd.experiments report F.json ...     (host: exact
                                                   optima, accuracy tables)

qkp100 reproduces the shape of the paper's comparison of SAIM with the
penalty method (Sec. IV-A, Table 2) on 20 synthetic QKP instances with N = 100
(10 at d = 0.25, 10 at d = 0.5):
  saim      Algorithm 1 itself, one chain per instance: 2000 annealing runs of
            1000 MCS, lambda stepped after each (Table 1: P = 2dN, beta_max 10,
            eta 20);
  p2dn      the penalty method at SAIM's P = 2dN (lambda = 0, eta = 0, 2000
            independent runs of 1000 MCS): shows that P is sub-critical and
            gives the critical-penalty estimate below;
  tuned     the penalty method with 10 runs of 2*10^5 MCS at a P raised from
            2dN over a coarse ladder until at least 20 % of the runs are
            feasible (Sec. IV-A's tuning protocol);
  penalty   the penalty method in SAIM's run structure, 2000 runs of 1000 MCS,
            at the tuned P (the paper's same-budget comparison).
mkp100 runs Algorithm 1 on 10 synthetic MKP instances with N = 100, M = 5
(Table 1: P = 5dN, beta_max 50, eta 0.05, 5000 runs of 1000 MCS) and the
remedies the paper names for the low MKP feasibility (Sec. IV-B) plus the
diminishing step of Sec. III-A's surrogate-gradient argument:
  saim       as above;
  decay      eta_k = eta H / (H + k), H = 500;
  tight      capacities B' = floor(0.97 B) in the sampler (a B'-feasible sample
             is B-feasible, and it is scored on B);
  p10        the penalty rule with alpha = 10 instead of 5.
Every arm of every instance runs as one member of a batch (one chain per
member, all members in one launch per round); per-round statistics come from
the batch snapshots (best feasible profit, feasible count, sum of the feasible
samples' profits).  The report step computes the exact optima (branch and
bound, exact.py) and prints the accuracy tables: best = 100 * best feasible
profit / OPT, avg = mean over the feasible samples of 100 * profit / OPT, and
the feasible share of all samples.  It also gives, per QKP instance, an
estimate of the critical penalty from the penalty arm's samples:
P_hat = max over sampled x with g != 0 and profit(x) > OPT of
(profit(x) - OPT) s_g^2 / (s_f |g|^2) (normalised units); such an x has a
lower energy than the optimum at every P below its term, so P_hat <= P_C.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from fractions import Fraction

import numpy as np

from . import binding as B
from . import generators as G

QKP_SAIM = dict(sweeps=1000, beta=Fraction(10), eta=Fraction(20), alpha=Fraction(2))
MKP_SAIM = dict(sweeps=1000, beta=Fraction(50), eta=Fraction(1, 20), alpha=Fraction(5))
TUNE_LADDER = [2, 5, 10, 20, 40, 70, 100, 150, 200, 300, 500, 700, 1000]  # P / (d N)


def qkp100_instances():
    return [G.qkp(100, Fraction(1, 4) if i < 10 else Fraction(1, 2), G.rng_for(5, i),
                  f"qkp-100-{25 if i < 10 else 50}-{i % 10 + 1}") for i in range(20)]


def mkp100_instances():
    return [G.mkp(100, 5, G.rng_for(6, i), f"mkp-100-5-{i + 1}") for i in range(10)]


def tighten(prob: G.Problem, num: int, den: int) -> G.Problem:
    """Same items with capacities floor(num/den * b)."""
    cap = (np.asarray(prob.capacity, dtype=np.int64) * num) // den
    return G.Problem(prob.kind, prob.profit, prob.weight, cap, prob.density, prob.name + f"-tight{num}/{den}")


def run_chains(probs, pars, rounds: int, log=print):
    """Runs every member for `rounds` rounds in one batch; returns per-round
    arrays [rounds, count]: best feasible profit so far (INT64_MIN if none),
    feasible samples, sum of the feasible samples' profits."""
    import torch
    count = len(probs)
    batch = B.Batch(probs, pars, rounds=[rounds] * count)
    snap = torch.empty((rounds, count * B.SNAPSHOT_BYTES), dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    for k in range(rounds):
        batch.run(1, use_graph=True)
        batch.snapshot(snap[k])
        if (k + 1) % 250 == 0:
            torch.cuda.synchronize()
            log(f"  round {k + 1}/{rounds}  {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    raw = snap.cpu().numpy()
    batch.close()
    recs = [B.decode_snapshot(raw[k], count) for k in range(rounds)]
    return {"best": np.stack([r["best"] for r in recs]).tolist(),
            "feasible": np.stack([r["feasible_last"] for r in recs]).tolist(),
            "feasible_profit_sum": np.stack([r["feasible_profit_sum"] for r in recs]).tolist(),
            "seconds": time.perf_counter() - t0}


def run_samples(probs, pars):
    """One round of every member (lambda = 0); per-replica profit, feasibility
    and |g|^2 of each member's samples."""
    import torch
    batch = B.Batch(probs, pars, rounds=[1] * len(probs))
    batch.run(1, use_graph=False)
    torch.cuda.synchronize()
    out = []
    for mem, p in zip(batch.members, probs):
        o = mem.round_outputs()
        g = o["g"][:, :p.m].astype(np.int64)
        out.append({"profit": o["profit"].tolist(), "feasible": o["feasible"].astype(int).tolist(),
                    "g2": (g * g).sum(axis=1).tolist()})
    batch.close()
    return out


def cmd_qkp100(args):
    probs = qkp100_instances()[:args.instances]
    res = {"experiment": "qkp100", "instances": [p.name for p in probs], "arms": {}}
    plans = [B.pbit_plan(p, G.Params(replicas=1, **QKP_SAIM)) for p in probs]
    res["n_ext"] = [int(pl.n_ext) for pl in plans]
    res["s_f"] = [int(pl.s_f) for pl in plans]
    res["s_g"] = [int(pl.s_g) for pl in plans]
    res["p_q_rule"] = [int(pl.p_q) for pl in plans]

    print("saim: Algorithm 1, one chain per instance", flush=True)
    pars = [G.Params(replicas=1, instance_id=i, **QKP_SAIM) for i in range(len(probs))]
    res["arms"]["saim"] = dict(run_chains(probs, pars, args.rounds), replicas=1, rounds=args.rounds)

    print("p2dn: penalty method at P = 2dN, lambda = 0", flush=True)
    pars = [G.Params(replicas=args.rounds, sweeps=1000, beta=Fraction(10), eta=Fraction(0), alpha=Fraction(2),
                     instance_id=i) for i in range(len(probs))]
    res["arms"]["p2dn"] = {"samples": run_samples(probs, pars), "replicas": args.rounds}

    print("tuned: 10 runs of 2e5 MCS, P raised until >= 20 % feasible", flush=True)
    chosen = [None] * len(probs)
    samples = [None] * len(probs)
    last = [None] * len(probs)      # (P / dN, samples) of the largest P tried
    exhausted = [False] * len(probs)
    for c in TUNE_LADDER:
        todo, pars = [], []
        for i in range(len(probs)):
            if chosen[i] is not None or exhausted[i]:
                continue
            # P = c d N_ext on the 2^-8 grid
            pq = round(Fraction(256 * c) * probs[i].density * res["n_ext"][i])
            par = G.Params(replicas=10, sweeps=args.tuned_sweeps, beta=Fraction(10), eta=Fraction(0),
                           p_q=int(pq), instance_id=1000 + i)
            try:
                B.pbit_plan(probs[i], par)
            except B.PbitError:
                exhausted[i] = True  # P beyond the exact integer range of the kernels
                continue
            todo.append(i)
            pars.append(par)
        if not todo:
            break
        t0 = time.perf_counter()
        got = run_samples([probs[i] for i in todo], pars)
        for i, s in zip(todo, got):
            last[i] = (c, s)
            if sum(s["feasible"]) >= 2:
                chosen[i], samples[i] = c, s
        print(f"  P = {c} dN: {len(todo)} runs, {sum(ch == c for ch in chosen)} accepted, "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
    # instances that never reached 20 % report their largest P
    for i in range(len(probs)):
        if chosen[i] is None and last[i] is not None:
            samples[i] = last[i][1]
    res["arms"]["tuned"] = {"p_over_dn": chosen, "samples": samples, "replicas": 10,
                            "sweeps": args.tuned_sweeps,
                            "largest_tried": [None if l is None else l[0] for l in last]}

    print("penalty: 2000 runs of 1000 MCS at the tuned P", flush=True)
    todo, pars = [], []
    for i in range(len(probs)):
        c = chosen[i] if chosen[i] is not None else (last[i][0] if last[i] is not None else None)
        if c is None:
            continue
        pq = round(Fraction(256 * c) * probs[i].density * res["n_ext"][i])
        todo.append(i)
        pars.append(G.Params(replicas=args.rounds, sweeps=1000, beta=Fraction(10), eta=Fraction(0), p_q=int(pq),
                             instance_id=2000 + i))
    got = run_samples([probs[i] for i in todo], pars)
    pen = [None] * len(probs)
    for i, s_ in zip(todo, got):
        pen[i] = s_
    res["arms"]["penalty"] = {"samples": pen, "replicas": args.rounds}
    with open(args.out, "w") as f:
        json.dump(res, f)
    print(json.dumps({"out": args.out}), flush=True)


def cmd_mkp100(args):
    base = mkp100_instances()[:args.instances]
    arms = {
        "saim": (lambda p: p, {}),
        "decay": (lambda p: p, {"eta_decay": 500}),
        "tight": (lambda p: tighten(p, 97, 100), {}),
        "p10": (lambda p: p, {"alpha": Fraction(10)}),
    }
    probs, pars, tags = [], [], []
    for name, (tf, extra) in arms.items():
        for i, p in enumerate(base):
            kw = dict(MKP_SAIM)
            kw.update(extra)
            probs.append(tf(p))
            pars.append(G.Params(replicas=1, instance_id=i, **kw))
            tags.append((name, i))
    print(f"mkp100: {len(probs)} chains x {args.rounds} rounds", flush=True)
    run = run_chains(probs, pars, args.rounds)
    res = {"experiment": "mkp100", "instances": [p.name for p in base], "arms": {}, "seconds": run["seconds"]}
    for a in arms:
        cols = [j for j, (name, _) in enumerate(tags) if name == a]
        res["arms"][a] = {k: [[row[j] for j in cols] for row in run[k]] for k in
                          ("best", "feasible", "feasible_profit_sum")}
        res["arms"][a]["rounds"] = args.rounds
    with open(args.out, "w") as f:
        json.dump(res, f)
    print(json.dumps({"out": args.out}), flush=True)


# ---------------------------------------------------------------------------
# report (host only)

def _chain_stats(arm, j, opt):
    best = np.asarray(arm["best"], dtype=np.int64)[:, j]
    feas = np.asarray(arm["feasible"], dtype=np.int64)[:, j]
    psum = np.asarray(arm["feasible_profit_sum"], dtype=np.int64)[:, j]
    n_feas = int(feas.sum())
    found = best[-1] > np.iinfo(np.int64).min
    return {"best": 100.0 * best[-1] / opt if found else None,
            "avg": 100.0 * psum.sum() / (n_feas * opt) if n_feas else None,
            "feasible": 100.0 * n_feas / len(feas), "optimal": bool(found and best[-1] == opt)}


def _sample_stats(s, opt):
    prof = np.asarray(s["profit"], dtype=np.int64)
    feas = np.asarray(s["feasible"], dtype=bool)
    if not feas.any():
        return {"best": None, "avg": None, "feasible": 0.0, "optimal": False}
    return {"best": 100.0 * prof[feas].max() / opt, "avg": 100.0 * prof[feas].mean() / opt,
            "feasible": 100.0 * feas.mean(), "optimal": bool(prof[feas].max() == opt)}


def _fmt(st):
    if st["best"] is None:
        return "— | — (0)"
    return f"{st['best']:.2f} | {st['avg']:.1f} ({st['feasible']:.0f})"


def _mean(vals):
    v = [x for x in vals if x is not None]
    return float(np.mean(v)) if v else float("nan")


def solve_all(probs, jobs: int, cache_path=None):
    """Exact optima of probs (parallel branch and bound), memoised by instance
    name in an optional JSON file."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    from . import exact as E
    cache = json.load(open(cache_path)) if cache_path and os.path.exists(cache_path) else {}
    todo = [p for p in probs if p.name not in cache]
    if todo:
        with ProcessPoolExecutor(max_workers=jobs) as ex:
            for p, o in zip(todo, ex.map(E.solve, todo)):
                cache[p.name] = {"profit": o.profit, "proven": o.proven, "seconds": o.seconds,
                                 "x": o.x.tolist() if o.x is not None else None}
        if cache_path:
            json.dump(cache, open(cache_path, "w"))
    out = []
    for p in probs:
        c = cache[p.name]
        x = np.asarray(c["x"], dtype=np.uint8)
        # re-score the stored assignment: it must be feasible and give the stored profit
        assert E.feasible(p, x) and E.profit_of(p, x) == c["profit"], p.name
        out.append(E.Optimum(c["profit"], x, c["proven"], float("nan"), c["seconds"]))
    return out


def cmd_report(args):
    for path in args.files:
        res = json.load(open(path))
        exp = res["experiment"]
        base = (qkp100_instances() if exp == "qkp100" else mkp100_instances())[:len(res["instances"])]
        opts = solve_all(base, args.jobs, args.opt_cache)
        if not all(o.proven for o in opts):
            print("warning: some optima are not proven", [o.proven for o in opts])
        print(f"\n## {exp}: exact optima (branch and bound): "
              f"{', '.join(str(o.profit) for o in opts)}; seconds {', '.join(f'{o.seconds:.0f}' for o in opts)}\n")
        if exp == "qkp100":
            rows = []
            print("| instance | OPT | SAIM best | avg (feas %) | penalty best | avg (feas %) | tuned best | avg (feas %) "
                  "| tuned P/dN | P=2dN feas % | P_hat_C / dN | 2dN / P_hat_C |")
            print("|---|---|---|---|---|---|---|---|---|---|---|---|")
            for j, name in enumerate(res["instances"]):
                opt = opts[j].profit
                a = _chain_stats(res["arms"]["saim"], j, opt)
                ps = res["arms"]["penalty"]["samples"][j]
                b = _sample_stats(ps, opt) if ps else {"best": None, "avg": None, "feasible": 0.0, "optimal": False}
                ts = res["arms"]["tuned"]["samples"][j]
                c = _sample_stats(ts, opt) if ts else {"best": None, "avg": None, "feasible": 0.0, "optimal": False}
                # critical-penalty estimate from the penalty arm's samples
                s = res["arms"]["p2dn"]["samples"][j]
                feas2 = 100.0 * np.mean(s["feasible"])
                prof = np.asarray(s["profit"], dtype=np.int64)
                g2 = np.asarray(s["g2"], dtype=np.int64)
                sel = (g2 > 0) & (prof > opt)
                sf, sg = res["s_f"][j], res["s_g"][j]
                phat = max((Fraction(int(p) - opt) * sg * sg / (sf * int(q)) for p, q in zip(prof[sel], g2[sel])),
                           default=None)
                dn = base[j].density * res["n_ext"][j]
                p_rule = Fraction(res["p_q_rule"][j], 256)
                rows.append((a, b, c, res["arms"]["tuned"]["p_over_dn"][j], phat, dn, p_rule, feas2))
                tp = res["arms"]["tuned"]["p_over_dn"][j]
                if tp is None:
                    tp = f"({res['arms']['tuned']['largest_tried'][j]}, < 20 %)"
                print(f"| {name} | {opt} | {_fmt(a)} | {_fmt(b)} | {_fmt(c)} | {tp} | {feas2:.0f} | "
                      f"{'—' if phat is None else f'{float(phat / dn):.1f}'} | "
                      f"{'—' if phat is None else f'{float(p_rule / phat):.3f}'} |")
            for key, label in (("best", "best"), ("avg", "avg"), ("feasible", "feasible %")):
                print(f"mean {label}: SAIM {_mean([r[0][key] for r in rows]):.2f}, "
                      f"penalty {_mean([r[1][key] for r in rows]):.2f}, tuned {_mean([r[2][key] for r in rows]):.2f}")
            print(f"optimal found: SAIM {sum(r[0]['optimal'] for r in rows)}/{len(rows)}, "
                  f"penalty {sum(r[1]['optimal'] for r in rows)}/{len(rows)}, "
                  f"tuned {sum(r[2]['optimal'] for r in rows)}/{len(rows)}")
            tuned = [r[3] for r in rows if r[3] is not None]
            print(f"tuned P: mean {np.mean(tuned):.0f} dN over {len(tuned)} instances")
        else:
            arms = list(res["arms"])
            print("| instance | OPT | " + " | ".join(f"{a} best | avg (feas %)" for a in arms) + " |")
            print("|---|---|" + "---|---|" * len(arms))
            allst = {a: [] for a in arms}
            for j, name in enumerate(res["instances"]):
                opt = opts[j].profit
                cells = []
                for a in arms:
                    st = _chain_stats(res["arms"][a], j, opt)
                    allst[a].append(st)
                    cells.append(_fmt(st))
                print(f"| {name} | {opt} | " + " | ".join(cells) + " |")
            for a in arms:
                st = allst[a]
                print(f"{a}: mean best {_mean([s['best'] for s in st]):.2f}, mean avg {_mean([s['avg'] for s in st]):.2f}, "
                      f"feasible {_mean([s['feasible'] for s in st]):.2f} %, optimal {sum(s['optimal'] for s in st)}"
                      f"/{len(st)}")


def cmd_optima(args):
    probs = qkp100_instances() if args.experiment == "qkp100" else mkp100_instances()
    opts = solve_all(probs, args.jobs, args.opt_cache)
    for p, o in zip(probs, opts):
        print(f"{p.name}: {o.profit} proven={o.proven} {o.seconds:.0f} s", flush=True)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    q = sub.add_parser("qkp100")
    q.add_argument("--out", required=True)
    q.add_argument("--instances", type=int, default=20)
    q.add_argument("--rounds", type=int, default=2000)
    q.add_argument("--tuned-sweeps", type=int, default=200000)
    m = sub.add_parser("mkp100")
    m.add_argument("--out", required=True)
    m.add_argument("--instances", type=int, default=10)
    m.add_argument("--rounds", type=int, default=5000)
    r = sub.add_parser("report")
    r.add_argument("files", nargs="+")
    r.add_argument("--jobs", type=int, default=4)
    r.add_argument("--opt-cache", default=None, help="JSON file memoising the exact optima by instance name")
    o = sub.add_parser("optima", help="exact optima of an experiment's instances (host only)")
    o.add_argument("experiment", choices=["qkp100", "mkp100"])
    o.add_argument("--jobs", type=int, default=4)
    o.add_argument("--opt-cache", required=True)
    args = ap.parse_args(argv)
    {"qkp100": cmd_qkp100, "mkp100": cmd_mkp100, "report": cmd_report, "optima": cmd_optima}[args.cmd](args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
