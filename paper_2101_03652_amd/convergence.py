"""l1 error against time and against residue updates for the FP64 path's
schedules (the two convergence views of Section 8), on a seeded Chung-Lu
graph.

Schedules, all through ppr_query_trace on the same query:

- powerpush:        local phase, then threshold-0 global sweeps (the default);
- powerpush-epochs: local phase, then Algorithm 3's epoch thresholds;
- powitr:           power iteration (no local phase; Eqs. 3-6);
- fwdpush:          the level-synchronous forward push to the end (Algorithm 2).

As in Section 8, the query shown is the source whose default query time is
the median among the sampled sources.  Each iteration's residue sum is the
exact l1 error of its estimate (residues stay >= 0).  Output: one JSON object
with, per schedule, the time and the residue updates (in units of m) at which
the error first falls to 1e-1, 1e-2, ..., lambda, and the full trace.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


SCHEDULES = {
    "powerpush": {},
    "powerpush-epochs": {"global_rule": 1},
    "powitr": {"switch_param": 1e30},
    "fwdpush": {"switch_param": 0.0},
}


def crossings(tr, m: int, lam: float) -> list:
    """First (ms, updates / m) at which the error is <= 10^-k, k = 1.. while
    10^-k >= lambda."""
    out = []
    k = 1
    while 10.0 ** -k >= lam * (1 - 1e-12):
        level = 10.0 ** -k
        hit = np.nonzero(tr["r_sum"] <= level)[0]
        if len(hit):
            i = int(hit[0])
            out.append({"l1": level, "ms": round(float(tr["ms"][i]), 3),
                        "updates_over_m": round(float(tr["edge_pushes"][i]) / m, 3)})
        else:
            out.append({"l1": level, "ms": None, "updates_over_m": None})
        k += 1
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=4_000_000)
    ap.add_argument("--m", type=int, default=70_000_000)
    ap.add_argument("--gamma", type=float, default=2.1)
    ap.add_argument("--alpha", type=float, default=0.2)
    ap.add_argument("--lam", type=float, default=1e-8)
    ap.add_argument("--sources", type=int, default=9, help="sampled sources; the median-time one is traced")
    ap.add_argument("--schedules", default=",".join(SCHEDULES))
    ap.add_argument("--full-trace", type=int, default=0, help="1: include every trace point in the output")
    args = ap.parse_args()

    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth
    import paper_2101_03652_amd as P

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = synth.chunglu(args.n, args.m, args.gamma)
    G = P.Graph.from_synth(g, trust_input=True)
    print(f"[conv] graph n={g.n} m={g.m} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    srcs = [int(s) for s in synth.sources(g.n, args.sources)]
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    G.query(srcs[0], args.alpha, args.lam, P.FP64, out=out)          # warm-up (graph capture, contexts)
    times = []
    for s in srcs:
        _, st = G.query(s, args.alpha, args.lam, P.FP64, out=out)
        times.append(st["ms"])
    order = np.argsort(times)
    s_med = srcs[int(order[len(order) // 2])]
    print(f"[conv] default query ms per source {np.round(times, 1).tolist()}, median source {s_med}",
          file=sys.stderr, flush=True)

    res = {"graph": {"n": g.n, "m": g.m, "gamma": args.gamma}, "alpha": args.alpha, "lambda": args.lam,
           "source": s_med, "schedules": {}}
    for name in args.schedules.split(","):
        opt = SCHEDULES[name]
        G.query_trace(s_med, args.alpha, args.lam, out=out, capacity=1 << 16, **opt)   # warm-up
        _, tr, st = G.query_trace(s_med, args.alpha, args.lam, out=out, capacity=1 << 16, **opt)
        entry = {"ms": round(float(tr["ms"][-1]), 3), "untraced_ms": None,
                 "local_levels": st["local_levels"], "global_iterations": st["sweeps"],
                 "updates_over_m": round(st["edge_pushes"] / g.m, 3), "final_l1": float(tr["r_sum"][-1]),
                 "to_l1": crossings(tr, g.m, args.lam)}
        _, su = G.query(s_med, args.alpha, args.lam, P.FP64, out=out, **opt)
        entry["untraced_ms"] = round(su["ms"], 3)
        if args.full_trace:
            entry["trace"] = {k: tr[k].tolist() for k in tr.dtype.names}
        res["schedules"][name] = entry
        print(f"[conv] {name}: {entry['ms']:.1f} ms traced ({entry['untraced_ms']:.1f} untraced), "
              f"{entry['local_levels']} levels + {entry['global_iterations']} global, "
              f"{entry['updates_over_m']} m updates", file=sys.stderr, flush=True)
    G.close()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
