#!/usr/bin/env python3
"""Benchmark: high-precision SSPPR queries/s on one MI355X.

Workload: directed Chung-Lu graph n = 4,000,000, m = 70,000,000 (out/in
exponent 2.1, min out-degree 1, no duplicates; synthetic stand-in for the
LiveJournal-sized graphs of the paper's evaluation), alpha = 0.2,
lambda = 1e-8, 128 seeded uniform sources.

One step answers all 128 sources with the batched mixed-precision path
(an n x B block: FP32 arithmetic on bf16-stored residues in over-relaxed block
Gauss-Seidel push sweeps, an FP32 stage accumulator, FP64 reserves, FP64
refreshes), every result certified ||pi_hat - pi_s||_1 <= lambda by the
library's FP64 certificate.  The graph and its CSC are resident in HBM before
the timed region; the outputs go to a device buffer.

Also reported (outside the timed steps): the plain FP64 single-query path on
the same graph; the global sweep's and the refresh's HBM bytes against their
measured durations (HIP events on the library's stream); a serving leg
(three resident graphs, continuous batching, Poisson arrivals: p50/p99 beside
queries/s); and the FP64 oracle (Algorithm 3, one query per host thread) on a
bounded sample, every answer certified.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def compulsory_sweep_bytes(n: int, m: int, width: int, offset_bytes: int = 4) -> int:
    """Compulsory bytes of one global sweep of a mixed n x B block, the
    yardstick the roofline fraction is quoted against: in-edge indices (4 m),
    per node an offset and a degree ((O + 4) n), and per node and column 24
    bytes (residue read and written, 4 + 4, and a reserve pair read and
    written, 16)."""
    return 4 * m + (offset_bytes + 4) * n + 24 * n * width


def refresh_bytes(n: int, m: int, width: int) -> int:
    """Compulsory bytes of one FP64 refresh pass: in-edge indices (4 m), per
    node an offset and a degree (8 n), per node and column the gathered FP32
    stage accumulator read once (4), its own accumulator, reserve and
    in-neighbour sum read (4 + 8 + 8) and the reserve, the in-neighbour sum
    and the residue written (8 + 8 + 2 at most 4)."""
    return 4 * m + 8 * n + 40 * n * width


def sweep_bytes(n: int, m: int, width: int, over_relaxed: bool = False, residue_bytes: int = 4) -> int:
    """Bytes this implementation's batched global sweep must move (all its
    row chunks), averaged over a pair of sweeps: in-edge indices (4 m), per-node CSC offset
    and FP32 scale (8 n), and per (node, column): the residue row read once
    and the new residue written (residue_bytes each: 4 in FP32, 2 in bf16),
    the FP32 per-stage reserve accumulator read and written by every second
    sweep (4 on average), which also reads the row's own input residue; an
    over-relaxed sweep reads that residue every time (its previous push)."""
    own = residue_bytes if over_relaxed else residue_bytes // 2
    per = 2 * residue_bytes + 4 + own
    return 4 * m + 8 * n + per * n * width


def fp64_sweep_bytes(n: int, m: int) -> int:
    """Plain FP64 sweep: 4 m index bytes, 8 n offset + degree, and per node the
    residue read once (8), the new residue written (8), the reserve read and
    written (16)."""
    return 4 * m + 8 * n + 32 * n


def kernel_source_digest() -> str:
    """Digest of the batched-path kernel sources: counter readings are valid
    only for the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in ("mixed_kernels.hip", "mixed_internal.h"):
        with open(os.path.join(ROOT, "paper_2101_03652_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(width: int, chunks: int, residues: str, tile: int):
    """HBM bytes per global sweep (its sweep_k and combine_k launches) from
    the committed rocprofv3 counter runs (FETCH_SIZE + WRITE_SIZE, each scaled
    by the same counter's reading for a plain 1 GiB copy), or None when they
    were taken on another kernel build, width, chunk count, residue storage
    or row tile."""
    path = os.path.join(ROOT, "profiles", "sweep_k_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("source_digest") != kernel_source_digest() or t.get("batch_cols") != width
            or t.get("sweep_chunks") != chunks or t.get("residues") != residues
            or t.get("sweep_tile_bytes") != tile):
        return None
    return t.get("bytes_per_sweep")


def cpu_model() -> str:
    """The host CPU as lscpu reports it: model name, family / model / stepping,
    sockets, cores per socket, threads per core (else /proc/cpuinfo's name)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        f = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f[k.strip()] = v.strip()
        if "Model name" in f:
            extra = ", ".join(f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping", "Socket(s)",
                                                                "Core(s) per socket", "Thread(s) per core",
                                                                "CPU max MHz") if k in f)
            return f"{f['Model name']} ({extra})" if extra else f["Model name"]
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def serve_leg(args, P, synth, torch, g_main, G_main) -> dict:
    """Continuous batching over three resident graphs (the step's graph is
    reused for its n:m): every query queued at once gives the saturated
    throughput of the mix, then Poisson arrivals at a fraction of it give
    p50/p99 latency (arrival to result in pinned host memory) beside
    queries/s.  lambda is 1e-6 or 1e-8 by seed, the graph uniform by seed."""
    import numpy as np
    from paper_2101_03652_amd import serve
    Gs, own = [], []
    for spec in args.serve_graphs.split(","):
        n, m = (int(x) for x in spec.split(":"))
        if (n, m) == (g_main.n, g_main.m):
            Gs.append(G_main)
            continue
        t0 = time.time()
        gg = synth.chunglu(n, m, 2.1)
        G = P.Graph.from_synth(gg, trust_input=True)
        del gg
        Gs.append(G)
        own.append(G)
        print(f"[bench] serve graph n={n} m={m} resident ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    free, _ = torch.cuda.mem_get_info()
    resident = sum(G.info()["device_bytes"] for G in Gs)
    budget = resident + int(0.9 * free)
    srv = serve.Server(Gs, budget, slots=32, alpha=args.alpha, sweeps_per_step=32)
    q = args.serve_queries
    pools = [synth.sources(G.n, q, seed=3652 + i) for i, G in enumerate(Gs)]

    def pick(gid):
        return [int(pools[int(gi)][k]) for k, gi in enumerate(gid)]

    _, gid, lam = serve.poisson_trace(1e9, q, len(Gs), seed=1)
    sat = serve.replay(srv, np.zeros(q), gid, lam, pick(gid), progress=100)
    print(f"[bench] serving saturated: {sat}", file=sys.stderr, flush=True)
    rate = args.serve_rate * sat["qps"]
    t_off, gid, lam = serve.poisson_trace(rate, q, len(Gs), seed=int(args.serve_rate * 1000) + 11)
    r = serve.replay(srv, t_off, gid, lam, pick(gid), progress=100)
    print(f"[bench] serving at {args.serve_rate}x: {r}", file=sys.stderr, flush=True)
    peak = srv.peak_committed
    srv.close()
    for G in own:
        G.close()
    return {"graphs": args.serve_graphs, "slots_per_graph": 32, "alpha": args.alpha, "lambdas": [1e-6, 1e-8],
            "budget_bytes": budget, "peak_committed_bytes": peak,
            "saturated": {k: sat[k] for k in ("queries", "served", "qps", "p50_ms", "p99_ms", "refused",
                                               "not_converged", "max_cert_l1")},
            "poisson": {"rate_frac": args.serve_rate, "offered_qps": round(rate, 3),
                        **{k: r[k] for k in ("queries", "served", "qps", "p50_ms", "p99_ms", "refused",
                                             "not_converged", "max_cert_l1")}}}


def large_leg(args, P, synth, torch) -> dict | None:
    """Directed Chung-Lu n = 40M, m = 1.4B (exponent 2.0, int32 indices):
    16 sources at B = 16 (one warm-up batch of 4, then the timed batch) and one
    FP64 single-source query, device outputs, every result certified.  Global
    sweep time from HIP events; bytes per sweep on the compulsory model.
    Skipped (with the reason) when the host or the device lacks the memory."""
    n, m = 40_000_000, 1_400_000_000
    host = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES")
    free, _ = torch.cuda.mem_get_info()
    if host < 96 * 2 ** 30 or free < 64 * 10 ** 9:
        return {"skipped": f"needs 96 GiB host and 64 GB free device memory (host {host >> 30} GiB, "
                           f"device {free / 1e9:.0f} GB free)"}
    t0 = time.time()
    gl = synth.chunglu(n, m, 2.0, cache=False)
    gen_s = time.time() - t0
    GL = P.Graph.from_synth(gl, trust_input=True)
    info = GL.info()
    del gl
    srcs = synth.sources(n, 16).tolist()
    out = torch.empty((16, n), dtype=torch.float64, device="cuda")
    GL.query_batch(srcs[:4], args.alpha, args.lam, P.MIXED, batch_cols=16, out=out[:4])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, st = GL.query_batch(srcs, args.alpha, args.lam, P.MIXED, batch_cols=16, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    per = st[0]["sweep_ms"] / max(st[0]["sweep_launches"], 1)
    sums = out.sum(dim=1).cpu().numpy()
    one = torch.empty(n, dtype=torch.float64, device="cuda")
    t2 = time.perf_counter()
    _, s64 = GL.query(srcs[0], args.alpha, args.lam, P.FP64, out=one, certify=1)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t2
    per64 = s64["sweep_ms"] / max(s64["sweep_launches"], 1)
    res = {"workload": f"chung-lu n={n} m={m} gamma=2.0 alpha={args.alpha} lambda={args.lam:g}",
           "generate_s": round(gen_s, 1), "graph_create_ms": round(info["build_ms"], 1),
           "graph_device_bytes": info["device_bytes"],
           "batched": {"sources": 16, "batch_cols": 16, "value": round(16 / dt, 3), "unit": "queries/s",
                       "residues": "bf16" if st[0]["residue_format"] == P.RESIDUE_BF16 else "f32",
                       "sweeps_per_query": round(sum(s["sweeps"] for s in st) / 16, 2),
                       "refreshes_per_query": round(sum(s["refreshes"] for s in st) / 16, 2),
                       "ms_per_sweep": round(per, 3),
                       "sweep_GBps_compulsory": round(compulsory_sweep_bytes(n, m, 16) / (per * 1e-3) / 1e9, 1),
                       "max_cert_l1": max(s["cert_l1"] for s in st),
                       "max_mass_error": float(abs(sums - 1.0).max())},
           "fp64_single": {"value": round(1 / dt64, 3), "unit": "queries/s", "sweeps": s64["sweeps"],
                           "ms_per_sweep": round(per64, 3),
                           "sweep_GBps_compulsory": round((4 * m + 8 * n + 32 * n) / (per64 * 1e-3) / 1e9, 1),
                           "cert_l1": s64["cert_l1"]}}
    if not (res["batched"]["max_cert_l1"] <= args.lam and s64["cert_l1"] <= args.lam):
        raise RuntimeError(f"large-graph answers not certified: {res}")
    print(f"[bench] large graph: {res}", file=sys.stderr, flush=True)
    GL.close()
    del out, one
    torch.cuda.empty_cache()
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4_000_000)
    ap.add_argument("--m", type=int, default=70_000_000)
    ap.add_argument("--gamma", type=float, default=2.1)
    ap.add_argument("--sources", type=int, default=128)
    ap.add_argument("--lam", type=float, default=1e-8)
    ap.add_argument("--alpha", type=float, default=0.2)
    ap.add_argument("--batch-cols", type=int, default=0, help="0 = autotuned")
    ap.add_argument("--sweep-tile", type=int, default=0,
                    help="LDS stage bytes of a sweep block (0 = the autotuner's choice, else 16384)")
    ap.add_argument("--fp64-queries", type=int, default=8)
    ap.add_argument("--fp64-epoch-queries", type=int, default=4,
                    help="FP64 queries with Algorithm 3's epoch thresholds in the global phase")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--approx-queries", type=int, default=8,
                    help="SpeedPPR queries timed per eps and mode (0: skip)")
    ap.add_argument("--f32-leg", type=int, default=1,
                    help="1: also time one step with FP32 residue storage (0: skip)")
    ap.add_argument("--extra-widths", default="8,32",
                    help="also time one step at these block widths (empty: skip)")
    ap.add_argument("--single-sources", type=int, default=32,
                    help="sources answered one at a time by the FP64 and the mixed path (0: skip)")
    ap.add_argument("--host-output", type=int, default=1,
                    help="1: also time one step into pinned and one into pageable host memory (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also copy a 1 GiB device buffer (reference for the HBM byte counters)")
    ap.add_argument("--serve-queries", type=int, default=400,
                    help="serving leg: queries per arrival pattern (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=0.7,
                    help="serving leg: Poisson arrival rate as a fraction of the measured saturation")
    ap.add_argument("--serve-graphs", default="1000000:15000000,4000000:70000000,16000000:300000000",
                    help="serving leg: n:m of the resident graphs")
    ap.add_argument("--large", type=int, default=1,
                    help="1: also run the large-graph leg (n=40M, m=1.4B, exponent 2.0: 16 sources at B=16 and "
                         "one FP64 query) when host and device memory allow (0: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the queries shard across GPUs with no exchange "
              "(the graph is replicated), so run one process per GPU; --gpus must be 1",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import synth
    import paper_2101_03652_amd as P

    torch.cuda.set_device(0)
    t0 = time.time()
    g = synth.chunglu(args.n, args.m, args.gamma)
    gen_s = time.time() - t0
    t0 = time.time()
    G = P.Graph.from_synth(g)
    info = G.info()
    create_s = time.time() - t0
    srcs = synth.sources(g.n, args.sources).tolist()
    print(f"[bench] graph n={g.n} m={g.m} max_in={info['max_in_degree']} gen={gen_s:.1f}s "
          f"create={create_s*1e3:.0f}ms", file=sys.stderr, flush=True)

    width = args.batch_cols
    tune = None
    if width == 0:
        tune = G.autotune(alpha=args.alpha)
        width = tune["best"]
    print(f"[bench] width={width} tune={tune}", file=sys.stderr, flush=True)

    out = torch.empty((args.sources, g.n), dtype=torch.float64, device="cuda")

    def step():
        return G.query_batch(srcs, args.alpha, args.lam, P.MIXED, out=out, batch_cols=width,
                             sweep_tile=args.sweep_tile)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats_all = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats_all.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    q = args.sources * args.steps
    qps = q / dt
    edges = sum(s["edge_pushes"] for st in stats_all for s in st)
    max_cert = max(s["cert_l1"] for st in stats_all for s in st)
    # sweep kernel timing (HIP events in the library), one entry per block
    sweep_ms = sweep_n = 0.0
    for st in stats_all:
        seen = set()
        for s in st:
            key = (s["batch_cols"], s["sweep_ms"], s["sweep_launches"])
            if key in seen:
                continue
            seen.add(key)
            sweep_ms += s["sweep_ms"]
            sweep_n += s["sweep_launches"]
    avg_sweep_ms = sweep_ms / max(sweep_n, 1)
    over_relaxed = any(s["sor_omega"] > 1.0 for st in stats_all for s in st)
    bf16 = stats_all[0][0]["residue_format"] == P.RESIDUE_BF16
    off_bytes = 8 if info["offsets_64bit"] else 4
    bytes_comp = compulsory_sweep_bytes(g.n, g.m, width, off_bytes)
    bytes_impl = sweep_bytes(g.n, g.m, width, over_relaxed, 2 if bf16 else 4)
    achieved = bytes_comp / (avg_sweep_ms * 1e-3) / 1e9
    # refresh passes (HIP events on the library's stream), one entry per block
    ref_ms = ref_n = 0.0
    for st in stats_all:
        ref_ms += st[0]["refresh_ms"]
        ref_n += st[0]["refresh_launches"]
    avg_refresh_ms = ref_ms / max(ref_n, 1)
    print(f"[bench] mixed: {qps:.1f} q/s, {dt/args.steps*1e3:.1f} ms/step, sweep {avg_sweep_ms:.3f} ms avg "
          f"over {int(sweep_n)} launches, max cert {max_cert:.3e}", file=sys.stderr, flush=True)

    # plain FP64 single-query path on the same graph
    fp64 = None
    f64_qps = None
    if args.fp64_queries > 0:
        out1 = torch.empty((1, g.n), dtype=torch.float64, device="cuda")
        G.query_batch([srcs[0]], args.alpha, args.lam, P.FP64, out=out1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f64_stats = []
        for s in srcs[:args.fp64_queries]:
            f64_stats.append(G.query_batch([s], args.alpha, args.lam, P.FP64, out=out1)[1][0])
        torch.cuda.synchronize()
        f64_dt = time.perf_counter() - t1
        f64_qps = args.fp64_queries / f64_dt
        f64_sweep_ms = sum(s["sweep_ms"] for s in f64_stats) / max(sum(s["sweep_launches"] for s in f64_stats), 1)
        f64_gbs = fp64_sweep_bytes(g.n, g.m) / (f64_sweep_ms * 1e-3) / 1e9
        f64_gteps = sum(s["edge_pushes"] for s in f64_stats) / f64_dt / 1e9
        fp64 = {"value": round(f64_qps, 3), "unit": "queries/s", "gteps": round(f64_gteps, 3),
                "sweep_ms": round(f64_sweep_ms, 4), "sweep_gbs": round(f64_gbs, 1),
                "queries": args.fp64_queries}
        print(f"[bench] fp64: {f64_qps:.1f} q/s, sweep {f64_sweep_ms:.3f} ms", file=sys.stderr, flush=True)
    if args.fp64_epoch_queries > 0 and fp64 is not None:
        # Algorithm 3's epochs; scans direction-optimizing (default), all pull, all push
        out1 = torch.empty((1, g.n), dtype=torch.float64, device="cuda")
        for key, form in (("epochs", P.SCAN_AUTO), ("epochs_pull", P.SCAN_PULL), ("epochs_push", P.SCAN_PUSH)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ep = [G.query_batch([s_], args.alpha, args.lam, P.FP64, out=out1, global_rule=P.GLOBAL_EPOCHS,
                                scan_form=form)[1][0] for s_ in srcs[:args.fp64_epoch_queries]]
            torch.cuda.synchronize()
            ep_dt = time.perf_counter() - t1
            fp64[key] = {"value": round(len(ep) / ep_dt, 3), "unit": "queries/s",
                         "scans_per_query": round(sum(e["sweeps"] for e in ep) / len(ep), 1),
                         "push_scans_per_query": round(sum(e["push_scans"] for e in ep) / len(ep), 1),
                         "edge_pushes_per_query_over_m": round(sum(e["edge_pushes"] for e in ep) / len(ep) / g.m, 2),
                         "queries": len(ep)}
            print(f"[bench] fp64 {key}: {fp64[key]}", file=sys.stderr, flush=True)
        fp64["epochs"]["threshold0_sweeps_per_query"] = round(sum(e["sweeps"] for e in f64_stats) / len(f64_stats), 1)

    # the same step with FP32 residue storage (one timed step)
    f32_leg = None
    if bf16 and args.f32_leg:
        step_f = lambda: G.query_batch(srcs, args.alpha, args.lam, P.MIXED, out=out, batch_cols=width,
                                       residue_format=P.RESIDUE_F32)[1]
        step_f()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_f = step_f()
        torch.cuda.synchronize()
        dt_f = time.perf_counter() - t1
        f32_leg = {"value": round(args.sources / dt_f, 3), "unit": "queries/s",
                   "ms_per_sweep": round(st_f[0]["sweep_ms"] / max(st_f[0]["sweep_launches"], 1), 4),
                   "sweeps_per_query": round(sum(s["sweeps"] for s in st_f) / len(st_f), 2),
                   "refreshes_per_query": round(sum(s["refreshes"] for s in st_f) / len(st_f), 2),
                   "max_cert_l1": max(s["cert_l1"] for s in st_f)}
        print(f"[bench] FP32 residues: {f32_leg}", file=sys.stderr, flush=True)

    # the same step at other block widths (one timed step each)
    widths = {}
    for w in [int(x) for x in args.extra_widths.split(",") if x.strip()]:
        if w == width:
            continue
        step_w = lambda: G.query_batch(srcs, args.alpha, args.lam, P.MIXED, out=out, batch_cols=w)[1]
        step_w()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_w = step_w()
        torch.cuda.synchronize()
        dt_w = time.perf_counter() - t1
        per_w = st_w[0]["sweep_ms"] / max(st_w[0]["sweep_launches"], 1)
        widths[str(w)] = {"value": round(args.sources / dt_w, 3), "unit": "queries/s",
                          "ms_per_sweep": round(per_w, 4),
                          "sweep_GBps_algorithmic": round(sweep_bytes(g.n, g.m, w, any(s["sor_omega"] > 1.0 for s in st_w),
                                                                      2 if st_w[0]["residue_format"] == 1 else 4)
                                                          / (per_w * 1e-3) / 1e9, 1),
                          "residues": "bf16" if st_w[0]["residue_format"] == 1 else "f32"}
        print(f"[bench] width {w}: {widths[str(w)]}", flush=True, file=sys.stderr)

    # the same step with the results delivered to host memory (device staging
    # plus a PCIe copy of 8 n bytes per query); reported beside the device-resident rate
    host_out = None
    if args.host_output:
        host_out = {}
        for kind in ("pinned", "pageable"):
            if kind == "pinned":
                hbuf = torch.empty((args.sources, g.n), dtype=torch.float64, pin_memory=True)
            else:
                hbuf = np.empty((args.sources, g.n), dtype=np.float64)
                hbuf.fill(0.0)                     # first touch outside the timed step
            G.query_batch(srcs, args.alpha, args.lam, P.MIXED, out=hbuf, batch_cols=width)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st_h = G.query_batch(srcs, args.alpha, args.lam, P.MIXED, out=hbuf, batch_cols=width)[1]
            torch.cuda.synchronize()
            dt_h = time.perf_counter() - t1
            host_out[kind] = {"value": round(args.sources / dt_h, 3), "unit": "queries/s",
                              "ms_per_step": round(dt_h * 1e3, 2),
                              "bytes_to_host": 8 * args.sources * g.n,
                              "max_cert_l1": max(s_["cert_l1"] for s_ in st_h)}
            del hbuf
        print(f"[bench] host output: {host_out}", file=sys.stderr, flush=True)

    # approximate queries (SpeedPPR, Algorithm 4): index-free and with the walk index
    approx = None
    if args.approx_queries > 0:
        approx = {"mu": "1/n", "queries": args.approx_queries}
        ms_idx = G.build_walk_index(args.alpha, seed=1)
        approx["index_build_ms"] = round(ms_idx, 1)
        approx["index_bytes"] = 4 * g.m
        one = torch.empty(g.n, dtype=torch.float64, device="cuda")
        for eps in (0.5, 0.1):
            row = {}
            for use_index in (False, True):
                G.query_approx(srcs[0], args.alpha, eps, seed=1, use_index=use_index, out=one)   # warm-up
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sts = [G.query_approx(s_, args.alpha, eps, seed=1, use_index=use_index, out=one)[1]
                       for s_ in srcs[:args.approx_queries]]
                torch.cuda.synchronize()
                dt1 = time.perf_counter() - t1
                mean = lambda k: sum(x[k] for x in sts) / len(sts)
                row["index" if use_index else "index_free"] = {
                    "value": round(len(sts) / dt1, 2), "unit": "queries/s", "W": sts[0]["W"],
                    "lambda": sts[0]["lambda"], "sweeps": mean("sweeps"), "refine_levels": mean("refine_levels"),
                    "walks": mean("walks"), "ms_push": round(mean("ms_push"), 2),
                    "ms_refine": round(mean("ms_refine"), 2), "ms_walks": round(mean("ms_walks"), 2)}
            approx[f"eps={eps:g}"] = row
            print(f"[bench] speedppr eps={eps:g}: {row}", file=sys.stderr, flush=True)

    # sources one at a time: plain FP64 path against the mixed path (one column)
    single = {}
    if args.single_sources > 0:
        one = torch.empty((1, g.n), dtype=torch.float64, device="cuda")
        ss = srcs[:args.single_sources]
        for lam in (1e-6, 1e-8):
            row = {}
            for name, prec, extra in (("fp64", P.FP64, {}), ("mixed", P.MIXED, {"batch_cols": 4})):
                G.query_batch([ss[0]], args.alpha, lam, prec, out=one, **extra)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                certs = []
                for s_ in ss:
                    st1 = G.query_batch([s_], args.alpha, lam, prec, out=one, certify=1, **extra)[1][0]
                    certs.append(st1["cert_l1"])
                torch.cuda.synchronize()
                dt1 = time.perf_counter() - t1
                row[name] = {"value": round(len(ss) / dt1, 3), "unit": "queries/s",
                             "max_cert_l1": max(certs)}
            single[f"{lam:g}"] = row
            print(f"[bench] one at a time, lambda={lam:g}: {row}", flush=True, file=sys.stderr)

    if args.calibrate_copy:
        x = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
        x.fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    # serving leg: continuous batching over three resident graphs
    serving = None
    if args.serve_queries > 0:
        serving = serve_leg(args, P, synth, torch, g, G)

    # large-graph leg (the Twitter-sized configuration)
    large = None
    if args.large:
        large = large_leg(args, P, synth, torch)

    chunks = stats_all[0][0]["sweep_chunks"]
    omegas = sorted({round(s["sor_omega"], 4) for sts in stats_all for s in sts})
    sk_name = (f"sweep_k<C={width // (8 if bf16 else 4)}{', over-relaxed' if over_relaxed else ''}"
               f"{', bf16 residues' if bf16 else ''}>")
    tile = stats_all[0][0]["sweep_tile_bytes"]
    traffic = measured_traffic(width, chunks, "bf16" if bf16 else "f32", tile)

    cpu = None
    if args.cpu_baseline:
        import oracle
        threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        threads = max(1, min(threads, os.cpu_count() or 1))
        sample = srcs[:threads]
        t2 = time.perf_counter()
        pis, ost = oracle.powerpush_many(g, sample, args.alpha, args.lam, threads)
        c_dt = time.perf_counter() - t2
        # every CPU answer certified (outside the timed region): ||pi_hat - pi_s||_1 <= lambda
        cpu_cert = max(oracle.certificate(g, int(s_), args.alpha, pis[k]) for k, s_ in enumerate(sample))
        if not cpu_cert <= args.lam * (1 + 1e-9):
            raise RuntimeError(f"oracle answer not certified: {cpu_cert} > {args.lam}")
        cpu = {"value": round(len(sample) / c_dt, 4), "unit": "queries/s", "cores": threads,
               "cpu_model": cpu_model(), "kind": "oracle", "max_cert_l1": cpu_cert,
               "sample": f"{len(sample)} of the step's sources on the same graph, Algorithm 3 in FP64, "
                         f"one query per host thread, {c_dt:.1f} s wall"}
        print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)

    rec = {
        "metric": "SSPPR queries/s at lambda=1e-8 (batched mixed precision)",
        "value": round(qps, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"chung-lu n={g.n} m={g.m} gamma={args.gamma} alpha={args.alpha} "
                        f"lambda={args.lam:g}, {args.sources} sources per step, batched mixed, B={width}, "
                        f"{chunks} sweep chunks, over-relaxation {'/'.join(str(w) for w in omegas)}, "
                        f"{'bf16' if bf16 else 'FP32'} residue storage (FP32 arithmetic, FP64 certificate)",
            "n": g.n, "m": g.m, "sources_per_step": args.sources, "batch_cols": width, "sweep_chunks": chunks,
            "sor_omega_final": omegas, "residue_storage": "bf16" if bf16 else "f32",
            "sweep_tile_bytes": tile,
            "alpha": args.alpha, "lambda": args.lam,
        },
        "gteps": round(edges / dt / 1e9, 3),
        "max_cert_l1": max_cert,
        "fp64_plain": fp64,
        "speedup_vs_fp64_plain": round(qps / f64_qps, 2) if f64_qps else None,
        # one "launch" here is one global sweep: `chunks` launches of sweep_k
        # (block Gauss-Seidel row chunks) and their combine_k launches, timed
        # together with HIP events on the library's stream.  achieved/frac:
        # the compulsory bytes of a sweep, 4 m + (O + 4) n + 24 n B; the
        # implementation's own byte model and the counted traffic beside it
        "roofline": {"bound": "hbm", "kernel": f"{sk_name} x{chunks} chunks + combine_k",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_GBps": round(traffic / (avg_sweep_ms * 1e-3) / 1e9, 1) if traffic else None,
                     "bytes_per_launch": bytes_comp, "avg_launch_ms": round(avg_sweep_ms, 4),
                     "launch": "one global sweep",
                     "bytes_model": "compulsory 4m + (O+4)n + 24nB",
                     "impl_bytes_per_launch": bytes_impl,
                     "impl_frac": round(bytes_impl / (avg_sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic_over_compulsory": round(traffic / bytes_comp, 3) if traffic else None,
                     "traffic_over_impl": round(traffic / bytes_impl, 3) if traffic else None,
                     "target_frac": 0.6, "target_met": achieved / HBM_PEAK_GBS >= 0.6},
        "refresh": {"kernel": "refresh_k + reduce_cols_k (FP64 residual, S += T)",
                    "avg_launch_ms": round(avg_refresh_ms, 4), "launches_per_step": round(ref_n / args.steps, 2),
                    "bytes_per_launch": refresh_bytes(g.n, g.m, width),
                    "achieved": round(refresh_bytes(g.n, g.m, width) / (avg_refresh_ms * 1e-3) / 1e9, 1)
                    if ref_n else None, "unit": "GB/s",
                    "frac": round(refresh_bytes(g.n, g.m, width) / (avg_refresh_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                    if ref_n else None,
                    "share_of_step": round(ref_ms / (dt * 1e3), 4)},
        "sweeps_per_query": round(sum(s["sweeps"] for st in stats_all for s in st) / q, 2),
        "refreshes_per_query": round(sum(s["refreshes"] for st in stats_all for s in st) / q, 2),
        "f32_residues": f32_leg,
        "approx_speedppr": approx,
        "batched_widths": widths,
        "host_output": host_out,
        "single_source": single,
        "serving": serving,
        "large_graph": large,
        "cpu_baseline": cpu,
        "paper_context": {"figure": "PowerPush < 40 s per query (no GPU or throughput figures in the paper)",
                          "hardware": "one Intel 2.0 GHz CPU server, 144 GB RAM, sequential C++ (GCC 9.3 -O3)",
                          "precision": "FP64", "workload": "Orkut, n=3.07M, m=234M, alpha=0.2, lambda=min(1e-8, 1/m)"},
        "graph_create_ms": round(info["build_ms"], 1),
    }
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
