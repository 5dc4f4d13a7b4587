"""Serving blocks (continuous batching) on the GPU, through the C ABI.

- A query's result is the same alone and inside a block whose other slots
  hold other queries with other lambdas, admitted and retired at other times:
  <= 1e-9 in l1 (FP32 summation order of the block width is the only
  difference), the same sweep and refresh counts, and each certificate
  <= its lambda, re-checked by the oracle on the exported vector.
- Slots are refilled while other slots are still sweeping.
- The server never holds more device memory than its budget.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2101_03652_amd")

pytestmark = pytest.mark.gpu
ALPHA = 0.2
SLACK = 1e-9


@pytest.fixture(scope="module")
def c1():
    return synth.chunglu(10_000, 100_000, 2.1)


def test_block_refill_and_alone_equals_in_mix(c1):
    print("[gpu] serve block refill c1", flush=True)
    G = P.Graph.from_synth(c1)
    srcs = [int(s) for s in synth.sources(c1.n, 12)]
    lams = [1e-8 if k % 2 == 0 else 1e-6 for k in range(12)]
    blk = P.Block(G, 4, ALPHA, sweep_chunks=4)
    pending = list(range(12))
    slot_of = {}
    results = {}
    refilled_while_running = 0
    steps = 0
    while len(results) < 12:
        st = blk.poll(wait=True)
        for slot in st["done"]:
            k = slot_of.pop(slot)
            out, stats = blk.retire(slot)
            results[k] = (out, stats)
        running = len(slot_of)
        while pending and len(slot_of) < 4:
            k = pending.pop(0)
            slot = blk.admit(srcs[k], lams[k])
            assert slot not in slot_of
            slot_of[slot] = k
            if running > 0 and steps > 0:
                refilled_while_running += 1
        if slot_of:
            blk.step(3)
            steps += 1
        assert steps < 10000
    assert refilled_while_running >= 4
    with pytest.raises(P.PPRError):           # every slot busy
        b2 = P.Block(G, 4, ALPHA)
        for k in range(5):
            b2.admit(srcs[0], 1e-6)
    b2 = None
    blk.close()
    for k in range(12):
        out, stats = results[k]
        assert stats["source"] == srcs[k]
        assert stats["cert_l1"] <= lams[k]
        cert = oracle.certificate(c1, srcs[k], ALPHA, out)
        assert cert <= lams[k] * (1 + 1e-6) + 1e-15
        truth = oracle.powitr(c1, srcs[k], ALPHA, 135)
        assert np.abs(out - truth).sum() <= lams[k] + SLACK
        alone, sal = G.query_batch([srcs[k]], ALPHA, lams[k], P.MIXED, batch_cols=4, sweep_chunks=4)
        assert np.abs(alone[0] - out).sum() <= SLACK, k
        assert sal[0]["sweeps"] == stats["sweeps"]
        assert sal[0]["refreshes"] == stats["refreshes"]
    G.close()


def test_block_arguments_and_lifetime(c1):
    G = P.Graph.from_synth(c1)
    with pytest.raises(P.PPRError):
        P.Block(G, 6, ALPHA)
    with pytest.raises(P.PPRError):
        P.Block(G, 4, 1.5)
    blk = P.Block(G, 8, ALPHA)
    with pytest.raises(P.PPRError):
        blk.admit(c1.n, 1e-6)
    with pytest.raises(P.PPRError):
        blk.admit(0, 0.0)
    with pytest.raises(P.PPRError):
        blk.retire(0)                          # nothing certified yet
    with pytest.raises(P.PPRError):
        blk.retire(8)                          # out of range
    with pytest.raises(P.PPRError):
        blk.step(0)
    # a graph with a live block refuses destruction
    rc = P.load().ppr_graph_destroy(G.handle)
    assert rc == -8
    s = blk.admit(5, 1e-6)
    while True:
        blk.step(64)
        if blk.poll(wait=True)["n_done"] == 1:
            break
    out = torch.empty(c1.n, dtype=torch.float64, device="cuda")
    _, stats = blk.retire(s, out=out)                  # device destination
    assert stats["cert_l1"] <= 1e-6
    assert blk.poll()["n_busy"] == 0
    blk.close()
    assert P.Block.footprint(G, 8) > 16 * c1.n * 8
    G.close()


def test_server_two_graphs_budget_and_results(c1):
    from paper_2101_03652_amd.serve import Server
    print("[gpu] serve server two graphs", flush=True)
    g2 = synth.chunglu(20_000, 160_000, 2.1, seed=77)
    G1, G2 = P.Graph.from_synth(c1), P.Graph.from_synth(g2)
    graphs = [G1, G2]
    gb = sum(G.info()["device_bytes"] for G in graphs)
    fp = lambda G, w: P.Block.footprint(G, w)
    # room for the 32-slot block of one graph and a narrower block of the other
    budget = gb + fp(G2, 32) + fp(G1, 8)
    srv = Server(graphs, budget, slots=32, alpha=ALPHA, sweeps_per_step=4, keep_results=True)
    rng = np.random.default_rng(4)
    futs = []
    for k in range(40):
        gi = int(rng.integers(0, 2))
        gh = (c1, g2)[gi]
        s = int(rng.integers(0, gh.n))
        lam = (1e-6, 1e-8)[k % 2]
        futs.append((gi, s, lam, srv.submit(gi, s, lam)))
        if k % 5 == 0:
            srv.pump()
    srv.run_until_idle(timeout_s=300)
    assert srv.peak_committed <= budget
    assert srv.refused == 0
    for gi, s, lam, f in futs:
        pi, stats = f.result(timeout=0)
        gh = (c1, g2)[gi]
        assert stats["cert_l1"] <= lam
        assert oracle.certificate(gh, s, ALPHA, pi) <= lam * (1 + 1e-6) + 1e-15
    srv.close()
    # a budget below the smallest block of a graph refuses its queries
    srv = Server([G1], G1.info()["device_bytes"] + fp(G1, 4) - 1, slots=8, alpha=ALPHA)
    f = srv.submit(0, 1, 1e-6)
    assert srv.refused == 1
    with pytest.raises(Exception):
        f.result(timeout=0)
    srv.close()
    G1.close()
    G2.close()


def test_sweep_cap_is_per_query(c1):
    """max_sweeps caps each query, not the block's lifetime: a block that has
    run many more sweeps than the cap in total still finishes new queries
    (regression: a block-wide count stopped all sweeping once it passed the
    cap), and a query that reaches the cap uncertified is retired with
    PPR_ERR_NOT_CONVERGED and frees its slot."""
    print("[gpu] serve sweep cap per query", flush=True)
    G = P.Graph.from_synth(c1)
    srcs = [int(s) for s in synth.sources(c1.n, 10)]
    blk = P.Block(G, 4, ALPHA, max_sweeps=120)
    total = 0
    for k in range(6):                      # ~62 sweeps each at lambda = 1e-6
        slot = blk.admit(srcs[k], 1e-6)
        for _ in range(1000):
            blk.step(16)
            if blk.poll(wait=True)["n_done"] == 1:
                break
        out, st = blk.retire(slot)
        total += st["sweeps"]
        assert st["cert_l1"] <= 1e-6
        assert st["sweeps"] <= 120
    assert total > 120
    slot = blk.admit(srcs[7], 1e-10)        # needs ~100 sweeps: cap below that
    blk.close()
    blk = P.Block(G, 4, ALPHA, max_sweeps=20)
    slot = blk.admit(srcs[7], 1e-10)
    for _ in range(1000):
        blk.step(16)
        if blk.poll(wait=True)["n_done"] == 1:
            break
    with pytest.raises(P.PPRError) as ei:
        blk.retire(slot)
    assert ei.value.status == -7
    assert blk.poll()["n_busy"] == 0
    blk.close()
    G.close()
