"""Serving loop: continuous batching of high-precision SSPPR queries over
graphs resident in device memory.

Policy lives here; the mechanism (query slots, sweeps, FP64 refreshes,
certified retirement) is libppr's serving block (ppr_block_* / ppr_slot_*).

- Each resident graph gets at most one block of query slots, created when its
  first query arrives.  A block's slots run independently: a finished query
  is retired (its certified pi_hat copied to host memory) and its slot takes
  the next queued query while the others keep sweeping.
- Admission is by device-memory footprint: the graphs plus every block's
  state must fit the budget.  A block is created at the widest slot count
  that fits (halving down to 4), after destroying idle blocks of other graphs
  if that is what it takes.  A query whose graph cannot get even a 4-slot
  block within the budget, or that finds the graph's queue full, is refused.
- Blocks of different graphs run on their own streams, each driven by its
  own worker thread, so one block's waits never hold up another's work.

Latency is measured from a query's arrival to its result in host memory.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from collections import deque
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------- policy helpers (host only)

def choose_slots(free_bytes: int, footprint, max_slots: int) -> int:
    """Widest power-of-two slot count in [4, max_slots] whose block footprint
    fits free_bytes; 0 if none does.  footprint(slots) -> bytes."""
    w = 1 << int(math.floor(math.log2(max(4, max_slots))))
    while w >= 4:
        if footprint(w) <= free_bytes:
            return w
        w //= 2
    return 0


def percentile(xs, q: float) -> float:
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    if len(xs) == 0:
        return float("nan")
    a = np.sort(np.asarray(xs, dtype=np.float64))
    pos = (len(a) - 1) * q / 100.0
    lo = int(math.floor(pos))
    hi = min(lo + 1, len(a) - 1)
    return float(a[lo] + (a[hi] - a[lo]) * (pos - lo))


def poisson_trace(rate: float, count: int, n_graphs: int, lambdas=(1e-6, 1e-8), seed: int = 3652):
    """Seeded open-loop arrivals: exponential inter-arrival gaps of mean
    1/rate seconds; the graph is uniform over n_graphs and lambda is drawn
    uniformly from `lambdas`.  Returns (t_offsets[count], graph[count],
    lambda[count])."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    gid = rng.integers(0, n_graphs, size=count)
    lam = np.asarray(lambdas, dtype=np.float64)[rng.integers(0, len(lambdas), size=count)]
    return t, gid, lam


# ---------------------------------------------------------------- server

@dataclass
class Request:
    rid: int
    graph: int
    source: int
    lam: float
    t_arrival: float
    alpha: float = 0.0          # the query's stop probability (0: the server's alpha)
    future: Future = field(default_factory=Future)


class Refused(RuntimeError):
    pass


class Server:
    """Continuous-batching server over resident graphs (one block per graph).

    graphs: list of paper_2101_03652_amd.Graph.  budget_bytes: device memory
    the graphs and blocks may hold together.  keep_results: resolve futures
    with (pi_hat copy, stats) instead of stats alone.

    One worker thread per graph drives that graph's block: wait for the
    block's enqueued work, retire the finished slots, refill the free slots
    from the graph's queue, enqueue the next sweeps.  The library calls
    release the interpreter lock, so one block's waits (and the local phase
    of newly admitted queries) never hold up the others.  A step runs until
    the longest current stage among its running slots ends, at most
    sweeps_per_step sweeps; the default 32 lies above the usual stage
    length, so a stage is not split across host round trips."""

    def __init__(self, graphs, budget_bytes: int, slots: int = 32, alpha: float = 0.2,
                 sweeps_per_step: int = 32, max_queue: int = 100000, keep_results: bool = False):
        import threading
        import torch
        import paper_2101_03652_amd as P
        self.P = P
        self.graphs = list(graphs)
        self.budget = int(budget_bytes)
        self.max_slots = int(slots)
        self.alpha = float(alpha)
        self.sweeps_per_step = int(sweeps_per_step)
        self.max_queue = int(max_queue)
        self.keep_results = keep_results
        self.graph_bytes = sum(int(g.info()["device_bytes"]) for g in self.graphs)
        if self.graph_bytes > self.budget:
            raise ValueError(f"the graphs alone ({self.graph_bytes} B) exceed the budget ({self.budget} B)")
        k = len(self.graphs)
        self.blocks = [None] * k
        self.block_bytes = [0] * k
        self.slot_req = [dict() for _ in self.graphs]        # slot -> Request
        self.queues = [deque() for _ in self.graphs]
        self._in_use = [False] * k                           # a worker is inside its block's step
        self.committed = self.graph_bytes
        self.peak_committed = self.committed
        self.refused = 0
        self.failed = 0
        self.completed = []                                   # (Request, latency_ms, stats)
        self._rid = 0
        self._error = None
        self._stop = False
        self._cv = threading.Condition()
        # one pinned host buffer per graph receives retired results
        self._host = [torch.empty(g.n, dtype=torch.float64, pin_memory=True) for g in self.graphs]
        self._workers = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(k)]
        for t in self._workers:
            t.start()

    # -------------------------------------------------------- admission
    def submit(self, graph: int, source: int, lam: float, t_arrival: float | None = None,
               alpha: float | None = None) -> Future:
        """Queue a query (alpha None: the server's alpha; each slot of a block
        has its own alpha and lambda)."""
        req = Request(self._rid, int(graph), int(source), float(lam),
                      time.perf_counter() if t_arrival is None else t_arrival,
                      0.0 if alpha is None else float(alpha))
        g = self.graphs[req.graph]
        small = self.P.Block.footprint(g, 4)
        with self._cv:
            self._rid += 1
            if self.blocks[req.graph] is None and self.graph_bytes + small > self.budget:
                self._refuse(req, "no block of this graph fits the memory budget")
            elif len(self.queues[req.graph]) >= self.max_queue:
                self._refuse(req, "queue full")
            else:
                self.queues[req.graph].append(req)
                self._cv.notify_all()
        return req.future

    def _refuse(self, req: Request, why: str) -> None:
        self.refused += 1
        req.future.set_exception(Refused(why))

    def _idle(self, i: int) -> bool:
        return (self.blocks[i] is not None and not self.slot_req[i] and not self.queues[i]
                and not self._in_use[i])

    def _open_block(self, i: int) -> bool:
        """With the lock held: create graph i's block within the budget."""
        g = self.graphs[i]
        fp = lambda w: self.P.Block.footprint(g, w)
        w = choose_slots(self.budget - self.committed, fp, self.max_slots)
        if w == 0:
            # free the budget held by idle blocks of other graphs
            for j in range(len(self.graphs)):
                if j != i and self._idle(j):
                    self._close_block(j)
            w = choose_slots(self.budget - self.committed, fp, self.max_slots)
            if w == 0:
                return False
        self.blocks[i] = self.P.Block(g, w, self.alpha)
        self.block_bytes[i] = fp(w)
        self.committed += self.block_bytes[i]
        self.peak_committed = max(self.peak_committed, self.committed)
        return True

    def _close_block(self, i: int) -> None:
        self.blocks[i].close()
        self.blocks[i] = None
        self.committed -= self.block_bytes[i]
        self.block_bytes[i] = 0

    # -------------------------------------------------------- workers
    def _worker(self, i: int) -> None:
        try:
            while True:
                with self._cv:
                    while not self._stop and not self.queues[i] and not self.slot_req[i]:
                        self._cv.wait()
                    if self._stop:
                        return
                    if self.blocks[i] is None and not self._open_block(i):
                        self._cv.wait(0.01)          # budget held by other graphs' blocks
                        continue
                    blk = self.blocks[i]
                    self._in_use[i] = True
                try:
                    self._serve(i, blk)
                finally:
                    with self._cv:
                        self._in_use[i] = False
                        self._cv.notify_all()
        except BaseException as e:                    # surfaced by run_until_idle / replay
            with self._cv:
                self._error = e
                self._cv.notify_all()

    def _serve(self, i: int, blk) -> None:
        st = blk.poll(wait=True)
        for slot in st["done"]:
            req = self.slot_req[i][slot]
            try:
                _, stats = blk.retire(slot, out=self._host[i])
                err = None
            except self.P.PPRError as e:              # reached its sweep cap uncertified
                stats, err = None, e
            t_done = time.perf_counter()
            with self._cv:
                del self.slot_req[i][slot]
                if err is not None:
                    self.failed += 1
                else:
                    self.completed.append((req, (t_done - req.t_arrival) * 1e3, stats))
            if err is not None:
                req.future.set_exception(err)
            elif self.keep_results:
                req.future.set_result((self._host[i].numpy().copy(), stats))
            else:
                req.future.set_result(stats)
        with self._cv:
            take = []
            while self.queues[i] and len(self.slot_req[i]) + len(take) < blk.slots:
                take.append(self.queues[i].popleft())
        for req in take:
            slot = blk.admit(req.source, req.lam, alpha=req.alpha or None)
            with self._cv:
                self.slot_req[i][slot] = req
        if self.slot_req[i]:
            blk.step(self.sweeps_per_step)

    # -------------------------------------------------------- control
    def busy(self) -> bool:
        with self._cv:
            return any(self.queues) or any(self.slot_req)

    def _check(self) -> None:
        if self._error is not None:
            raise RuntimeError("serving worker failed") from self._error

    def pump(self) -> bool:
        """Returns True while anything is queued or running (the workers do the work)."""
        self._check()
        return self.busy()

    def run_until_idle(self, timeout_s: float = 600.0) -> None:
        t_end = time.perf_counter() + timeout_s
        with self._cv:
            while any(self.queues) or any(self.slot_req) or any(self._in_use):
                if self._error is not None:
                    break
                if time.perf_counter() > t_end:
                    raise TimeoutError("server did not drain")
                self._cv.wait(0.05)
        self._check()

    def close(self) -> None:
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._workers:
            t.join()
        with self._cv:
            for i in range(len(self.graphs)):
                if self.blocks[i] is not None:
                    self._close_block(i)


# ---------------------------------------------------------------- measurement

def replay(server: Server, t_off, gid, lam, sources, timeout_s: float = 900.0, progress: int = 0) -> dict:
    """Open-loop replay of an arrival trace; returns latency percentiles (ms)
    over the trace's queries, throughput, refusals and failures.  progress > 0
    prints a line to stderr every `progress` completed queries."""
    n0 = len(server.completed)
    r0 = server.refused
    f0 = server.failed
    shown = 0
    start = time.perf_counter()
    N = len(t_off)
    t_end = start + timeout_s
    for k in range(N):
        delay = start + float(t_off[k]) - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        server.submit(int(gid[k]), int(sources[k]), float(lam[k]), t_arrival=start + float(t_off[k]))
        done = len(server.completed) - n0
        if progress and done >= shown + progress:
            shown = done - done % progress
            print(f"[serve] {done}/{N} served, {time.perf_counter() - start:.1f} s", file=sys.stderr, flush=True)
    while server.pump():
        if time.perf_counter() > t_end:
            raise TimeoutError("replay did not finish")
        time.sleep(0.005)
        done = len(server.completed) - n0
        if progress and done >= shown + progress:
            shown = done - done % progress
            print(f"[serve] {done}/{N} served, {time.perf_counter() - start:.1f} s", file=sys.stderr, flush=True)
    server.run_until_idle()
    wall = time.perf_counter() - start
    lats = [lat for _, lat, _ in server.completed[n0:]]
    return {"queries": N, "served": len(lats), "refused": server.refused - r0,
            "not_converged": server.failed - f0, "wall_s": round(wall, 3),
            "qps": round(len(lats) / wall, 3), "p50_ms": round(percentile(lats, 50), 3),
            "p99_ms": round(percentile(lats, 99), 3), "max_cert_l1": max((s["cert_l1"] for _, _, s in
                                                                          server.completed[n0:]), default=None)}


def main() -> int:
    ap = argparse.ArgumentParser(description="continuous-batching serving over three resident graphs")
    ap.add_argument("--graphs", default="1000000:15000000,4000000:70000000,16000000:300000000",
                    help="n:m pairs of the resident Chung-Lu graphs (exponent 2.1)")
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--alpha", type=float, default=0.2)
    ap.add_argument("--queries", type=int, default=400, help="queries per arrival rate")
    ap.add_argument("--rates", default="0.3,0.7,1.0", help="fractions of the saturated throughput")
    ap.add_argument("--sweeps-per-step", type=int, default=32)
    ap.add_argument("--budget-gib", type=float, default=0.0, help="0 = 90%% of free device memory")
    args = ap.parse_args()

    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth
    import paper_2101_03652_amd as P

    torch.cuda.set_device(0)
    Gs = []
    for spec in args.graphs.split(","):
        n, m = (int(x) for x in spec.split(":"))
        g = synth.chunglu(n, m, 2.1)
        Gs.append(P.Graph.from_synth(g, trust_input=True))
        del g
        print(f"[serve] graph n={n} m={m} resident", file=sys.stderr, flush=True)
    free, _ = torch.cuda.mem_get_info()
    resident = sum(G.info()["device_bytes"] for G in Gs)
    budget = int(args.budget_gib * 2**30) if args.budget_gib > 0 else resident + int(0.9 * free)
    srv = Server(Gs, budget, slots=args.slots, alpha=args.alpha, sweeps_per_step=args.sweeps_per_step)

    # per graph a pool of seeded uniform sources; query k takes entry k of its graph's pool
    pools = [synth.sources(G.n, args.queries, seed=3652 + i) for i, G in enumerate(Gs)]

    def pick(gid):
        return [int(pools[int(gi)][k]) for k, gi in enumerate(gid)]

    # saturated throughput of the mix: every query queued at once
    t_off, gid, lam = poisson_trace(1e9, args.queries, len(Gs), seed=1)
    sat = replay(srv, np.zeros(args.queries), gid, lam, pick(gid), progress=50)
    print(f"[serve] saturated: {sat}", file=sys.stderr, flush=True)
    out = {"graphs": args.graphs, "slots": args.slots, "alpha": args.alpha, "budget_bytes": budget,
           "saturated": sat, "rates": []}
    for frac in (float(x) for x in args.rates.split(",")):
        rate = frac * sat["qps"]
        t_off, gid, lam = poisson_trace(rate, args.queries, len(Gs), seed=int(frac * 1000) + 11)
        r = replay(srv, t_off, gid, lam, pick(gid), progress=50)
        r["rate_frac"] = frac
        r["rate_qps"] = round(rate, 3)
        out["rates"].append(r)
        print(f"[serve] rate {frac}: {r}", file=sys.stderr, flush=True)
    out["peak_committed_bytes"] = srv.peak_committed
    srv.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
