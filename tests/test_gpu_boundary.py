"""The boundary's stream, per-query alpha and footprint calls on the GPU,
through the C ABI.

- Caller streams (ppr_options.use_stream / stream): a query runs after the
  torch work enqueued before it on the same stream (it overwrites a buffer
  that torch work on that stream filled), on a side stream and on the null
  stream, with the same result as on the library's own stream (the same
  sweeps; the local phase's FP64 atomic adds land in any order, so the last
  bits vary from run to run: FP64 values to rtol 1e-11, mixed results, whose
  FP32 sweeps start from those values, to 1e-9 in l1); a serving
  block's step is enqueued on the caller's stream (an event recorded there
  after the step completes only after the block's work).
- Per-slot alpha (ppr_slot_admit): queries with three stop probabilities in
  one block, each within lambda + 1e-9 of power-iteration truth at its own
  alpha (Eq. 1), certified by the oracle at its own alpha, and equal (the
  same sweeps and refreshes, l1 <= 1e-9) to the query alone in a block whose
  reference alpha is its own.
- ppr_footprint_bytes: the graph-free sizes equal what ppr_graph_create and
  ppr_block_footprint report for a created graph.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2101_03652_amd")

pytestmark = pytest.mark.gpu
SLACK = 1e-9


@pytest.fixture(scope="module")
def c1():
    return synth.chunglu(10_000, 100_000, 2.1)


def _truth_iters(alpha):
    # (1 - alpha)^K <= 1e-13 (Eq. 6)
    return int(np.ceil(np.log(1e-13) / np.log(1.0 - alpha)))


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_query_on_caller_stream(c1, precision):
    print(f"[gpu] caller stream precision={precision}", flush=True)
    G = P.Graph.from_synth(c1)
    srcs = [int(s) for s in synth.sources(c1.n, 4)]
    base, bst = G.query_batch(srcs, 0.2, 1e-8, precision)
    side = torch.cuda.Stream()
    out = torch.empty((len(srcs), c1.n), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(side):
        # keep the stream busy, then fill the output: the query must come after both
        a = torch.rand((2048, 2048), device="cuda")
        for _ in range(8):
            a = a @ a
            a = a / a.norm()
        out.fill_(float("nan"))
        got, st = G.query_batch(srcs, 0.2, 1e-8, precision, out=out, stream=side)
    torch.cuda.synchronize()
    def same(res):
        assert not np.isnan(res).any()
        if precision == P.FP64:
            np.testing.assert_allclose(res, base, rtol=1e-11, atol=1e-20)
        else:
            assert np.abs(res - base).sum(axis=1).max() <= SLACK

    same(out.cpu().numpy())
    assert [s["sweeps"] for s in st] == [s["sweeps"] for s in bst]
    assert all(s["cert_l1"] <= 1e-8 for s in st) or precision == P.FP64
    # the null stream (torch's default stream is handle 0)
    out.fill_(float("nan"))
    G.query_batch(srcs, 0.2, 1e-8, precision, out=out, stream=torch.cuda.default_stream())
    same(out.cpu().numpy())
    G.close()


def test_block_steps_on_caller_stream(c1):
    print("[gpu] block on caller stream", flush=True)
    G = P.Graph.from_synth(c1)
    srcs = [int(s) for s in synth.sources(c1.n, 8)]
    side = torch.cuda.Stream()
    blk = P.Block(G, 8, 0.2, stream=side)
    for s in srcs:
        blk.admit(s, 1e-8)
    results = {}
    steps = 0
    while len(results) < len(srcs):
        blk.step(4)
        steps += 1
        ev = torch.cuda.Event()
        ev.record(side)
        ev.synchronize()
        # everything the step enqueued sits before the event on the same stream
        st = blk.poll(wait=False)
        assert st["ready"], "the block's work was not on the caller's stream"
        for slot in st["done"]:
            results[slot] = blk.retire(slot)
        assert steps < 1000
    blk.close()
    alone, _ = G.query_batch(srcs, 0.2, 1e-8, P.MIXED, batch_cols=8)
    for slot, (out, stats) in results.items():
        k = srcs.index(stats["source"])
        assert stats["cert_l1"] <= 1e-8
        assert np.abs(out - alone[k]).sum() <= SLACK
    G.close()


def test_stream_option_errors(c1):
    G = P.Graph.from_synth(c1)
    with pytest.raises(P.PPRError):
        G.query_batch([0], 0.2, 1e-8, P.FP64, use_stream=2)
    with pytest.raises(P.PPRError):          # a block runs the mixed path only
        lib = P.load()
        import ctypes
        o = P.options(precision=P.FP64)
        h = ctypes.c_void_p()
        P._check(lib.ppr_block_create(G.handle, 8, 0.2, ctypes.byref(o), ctypes.byref(h)))
    G.close()


def test_per_slot_alpha(c1):
    print("[gpu] per-slot alpha", flush=True)
    G = P.Graph.from_synth(c1)
    srcs = [int(s) for s in synth.sources(c1.n, 6)]
    alphas = [0.2, 0.15, 0.3, 0.2, 0.3, 0.15]
    lams = [1e-8, 1e-8, 1e-6, 1e-6, 1e-8, 1e-6]
    blk = P.Block(G, 8, 0.2, sweep_chunks=4)
    slot_of = {}
    for k, s in enumerate(srcs):
        slot_of[blk.admit(s, lams[k], alpha=alphas[k])] = k
    results = {}
    while len(results) < len(srcs):
        st = blk.poll(wait=True)
        for slot in st["done"]:
            results[slot_of[slot]] = blk.retire(slot)
        if len(results) < len(srcs):
            blk.step(8)
    blk.close()
    for k, s in enumerate(srcs):
        out, stats = results[k]
        a = alphas[k]
        assert stats["cert_l1"] <= lams[k]
        cert = oracle.certificate(c1, s, a, out)
        assert cert <= lams[k] * (1 + 1e-6) + 1e-15
        assert abs(cert - stats["cert_l1"]) <= 1e-6 * lams[k]
        truth = oracle.powitr(c1, s, a, _truth_iters(a))
        assert np.abs(out - truth).sum() <= lams[k] + SLACK, (k, a)
        # alone, in a block whose reference alpha is the query's own (factor 1)
        b1 = P.Block(G, 8, a, sweep_chunks=4)
        slot = b1.admit(s, lams[k])
        while not b1.poll(wait=True)["done"]:
            b1.step(8)
        out1, st1 = b1.retire(slot)
        b1.close()
        assert st1["sweeps"] == stats["sweeps"] and st1["refreshes"] == stats["refreshes"], k
        assert np.abs(out1 - out).sum() <= SLACK, k
    with pytest.raises(P.PPRError):
        b2 = P.Block(G, 4, 0.2)
        b2.admit(srcs[0], 1e-8, alpha=1.0)
    G.close()


@pytest.mark.parametrize("wide", [False, True])
def test_footprint_before_the_graph(c1, wide):
    G = P.Graph.from_synth(c1, wide_offsets=wide)
    info = G.info()
    for slots in (4, 32, 128):
        gb, sb = P.footprint_bytes(c1.n, c1.m, slots, P.MIXED)
        assert sb == P.Block.footprint(G, slots)
        if not wide:                       # forced int64 offsets are a flag, not a size
            assert gb == info["device_bytes"]
        else:
            assert gb + 4 * (c1.n + 1) == info["device_bytes"]
    gb1, s1 = P.footprint_bytes(c1.n, c1.m, 1, P.FP64)
    gb3, s3 = P.footprint_bytes(c1.n, c1.m, 3, P.FP64)
    assert gb1 == gb3 and s3 == 3 * s1 and s1 >= 64 * c1.n
    G.close()
