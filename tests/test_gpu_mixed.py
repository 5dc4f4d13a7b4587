"""GPU parity of the batched mixed-precision path against the FP64 oracle.

Contract (per column): ||pi_hat - pi_s||_1 <= lambda + 1e-9 against the
converged FP64 power iteration, where the slack 1e-9 is measurement slack for
the FP32 residues; the path itself stops only when its FP64 certificate
||rt||_1 (computed in FP64 from the FP64 reserves) is <= lambda, and the
certificate is re-checked here by the oracle on the exported vector.
Column independence: a source answered alone (batch width 4) and inside a
batch agree to <= 1e-9 in l1 (the block width changes the FP32 summation
order, nothing else).
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


@pytest.fixture(scope="module")
def c1_truth(c1):
    srcs = [int(s) for s in synth.sources(c1.n, 40)]
    return {s: oracle.powitr(c1, s, ALPHA, 135) for s in set(srcs)}


def _check_batch(g, srcs, out, stats, lam, truth):
    for b, s in enumerate(srcs):
        t = truth[s] if truth is not None and s in truth else oracle.powitr(g, s, ALPHA, 135)
        err = np.abs(out[b] - t).sum()
        assert err <= lam + SLACK, (b, s, err)
        cert = oracle.certificate(g, s, ALPHA, out[b])
        assert stats[b]["cert_l1"] <= lam
        assert cert <= lam * (1 + 1e-6) + 1e-15, (b, s, cert)
        assert stats[b]["cert_l1"] == pytest.approx(cert, rel=1e-6, abs=1e-14)
        assert stats[b]["source"] == s


@pytest.mark.parametrize("chunks", [1, 4])
@pytest.mark.parametrize("width", [4, 8, 16, 32, 64, 128])
def test_batch_widths_c1(c1, c1_truth, width, chunks):
    """chunks = 1: every sweep is one Eq. 7 step; chunks = 4: block
    Gauss-Seidel sweeps over four row chunks."""
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:width]
    print(f"[gpu] mixed c1 width={width} chunks={chunks}", flush=True)
    G = P.Graph.from_synth(c1)
    out, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=width, sweep_chunks=chunks)
    _check_batch(c1, srcs, out, st, 1e-8, c1_truth)
    assert all(s["refreshes"] >= 1 for s in st)


def test_ragged_batch_and_duplicates(c1, c1_truth):
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:13]
    srcs[5] = srcs[2]               # the same source twice in one block
    G = P.Graph.from_synth(c1)
    out, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=8)   # blocks of 8 + 5
    _check_batch(c1, srcs, out, st, 1e-8, c1_truth)
    # both columns are certified within lambda of the truth
    assert np.abs(out[5] - out[2]).sum() <= 2e-8 + SLACK


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
@pytest.mark.parametrize("chunks", [1, 4])
def test_alone_equals_in_mix(c1, chunks, fmt):
    """A column's sweep budget depends on its own error only, so a source
    answered alone (the narrowest block of its storage format) and inside a
    block of 32 runs the same schedule; the two results differ only by FP32
    summation order."""
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:32]
    G = P.Graph.from_synth(c1)
    rf = P.RESIDUE_F32 if fmt == "f32" else P.RESIDUE_BF16
    mix, smix = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=32, sweep_chunks=chunks, residue_format=rf)
    for b in (0, 7, 31):
        alone, sal = G.query_batch([srcs[b]], ALPHA, 1e-8, P.MIXED, batch_cols=4 if fmt == "f32" else 8,
                                   sweep_chunks=chunks, residue_format=rf)
        assert sal[0]["sweeps"] == smix[b]["sweeps"]
        assert sal[0]["refreshes"] == smix[b]["refreshes"]
        assert np.abs(alone[0] - mix[b]).sum() <= SLACK


def test_mixed_vs_fp64_path(c1):
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:8]
    G = P.Graph.from_synth(c1)
    mix, _ = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=8, sweep_chunks=4)
    f64, _ = G.query_batch(srcs, ALPHA, 1e-8, P.FP64)
    for b in range(8):
        assert np.abs(mix[b] - f64[b]).sum() <= 2e-8 + SLACK


@pytest.mark.parametrize("lam", [1e-4, 1e-6, 1e-10])
def test_lambda_range(c1, lam):
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:8]
    G = P.Graph.from_synth(c1)
    out, st = G.query_batch(srcs, ALPHA, lam, P.MIXED, batch_cols=8, sweep_chunks=4)
    _check_batch(c1, srcs, out, st, lam, None)


def test_small_graphs_and_hubs():
    a = 1 - ALPHA
    g = synth.cycle(37)
    x = np.array([ALPHA * a ** ((v - 5) % 37) / (1 - a ** 37) for v in range(37)])
    G = P.Graph.from_synth(g)
    out, st = G.query_batch([5, 5, 5, 5], ALPHA, 1e-10, P.MIXED, batch_cols=4)
    for b in range(4):
        assert np.abs(out[b] - x).sum() <= 1e-10 + SLACK
    g = synth.fig1()
    G = P.Graph.from_synth(g)
    out, st = G.query_batch([0, 1, 2, 3, 4], ALPHA, 1e-9, P.MIXED, batch_cols=8)
    for b in range(5):
        t = oracle.powitr(g, b, ALPHA, 200)
        assert np.abs(out[b] - t).sum() <= 1e-9 + SLACK
    # hub rows: long-row blocks in the sweep and in the refresh
    from test_gpu_fp64 import _hub_graph
    h = _hub_graph()
    G = P.Graph.from_synth(h)
    srcs = [0, 1, 2, 12345, 777, 19999, 3, 4]
    for width in (8, 128):
        for chunks in (1, 3):
            out, st = G.query_batch(srcs, ALPHA, 1e-9, P.MIXED, batch_cols=width, sweep_chunks=chunks)
            _check_batch(h, srcs, out, st, 1e-9, None)
    # int64 CSC offsets (the layout of graphs with m >= 2^32)
    Gw = P.Graph.from_synth(h, wide_offsets=True)
    out, st = Gw.query_batch(srcs, ALPHA, 1e-9, P.MIXED, batch_cols=32, sweep_chunks=3)
    _check_batch(h, srcs, out, st, 1e-9, None)


def _no_in_edges_graph(n=3000, head=400, seed=11):
    """Nodes 0 .. head-1 have out-edges only (into the rest), so whole sweep
    and refresh schedule blocks at the start hold rows without in-edges; the
    rest is a random graph of out-degree 5 on itself."""
    rng = np.random.default_rng(seed)
    edges = []
    for u in range(head):
        for v in rng.choice(np.arange(head, n), size=3, replace=False):
            edges.append((u, int(v)))
    for u in range(head, n):
        for v in rng.choice(np.arange(head, n - 1), size=5, replace=False):
            edges.append((u, int(v) if v < u else int(v) + 1))
    return synth.from_edges(n, edges, "no-in-edges head")


def test_blocks_of_rows_without_in_edges():
    """Schedule blocks whose rows have no in-edges (ne = 0): the refresh's
    pipelined loop loads the next block's descriptor after such a block too,
    and the sweeps leave those rows' residue at zero after the first push."""
    g = _no_in_edges_graph()
    G = P.Graph.from_synth(g)
    srcs = [0, 7, 399, 400, 1234, 2999, 5, 2000]
    for width in (8, 32, 128):
        for chunks in (1, 3):
            out, st = G.query_batch(srcs, ALPHA, 1e-9, P.MIXED, batch_cols=width, sweep_chunks=chunks)
            _check_batch(g, srcs, out, st, 1e-9, None)


@pytest.mark.parametrize("width", [8, 32])
def test_outputs_device_and_residual(c1, width):
    """The FP64 residual output (the flush) equals the oracle's residual of the
    exported estimate, in FP32 (width 8) and bf16 (width 32) residue storage."""
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:width]
    G = P.Graph.from_synth(c1)
    out = torch.empty((width, c1.n), dtype=torch.float64, device="cuda")
    r_out = torch.empty((width, c1.n), dtype=torch.float64, device="cuda")
    _, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=width, out=out, r_out=r_out)
    assert all(s["residue_format"] == (P.RESIDUE_BF16 if width >= 32 else P.RESIDUE_F32) for s in st)
    pi = out.cpu().numpy()
    r = r_out.cpu().numpy()
    for b, s in enumerate(srcs[:8]):
        cert, rt = oracle.certificate(c1, s, ALPHA, pi[b], want_residual=True)
        # rt is a difference of terms of size pi_hat(u) / alpha <= 5: FP64
        # cancellation leaves an absolute error of a few 1e-16
        np.testing.assert_allclose(r[b], rt, rtol=1e-6, atol=2e-15)
        assert np.abs(r[b]).sum() <= 1e-8


def test_not_converged_and_bad_width(c1):
    G = P.Graph.from_synth(c1)
    with pytest.raises(P.PPRError) as ei:
        G.query_batch([1, 2], ALPHA, 1e-10, P.MIXED, batch_cols=4, max_sweeps=5)
    assert ei.value.status == -7
    with pytest.raises(P.PPRError) as ei:
        G.query_batch([1, 2], ALPHA, 1e-8, P.MIXED, batch_cols=12)
    assert ei.value.status == -1
    # the graph still answers after the failures
    out, st = G.query_batch([1, 2], ALPHA, 1e-8, P.MIXED, batch_cols=4)
    assert st[0]["cert_l1"] <= 1e-8


def test_graph_recreated_between_batches(c1):
    """Regression: batched query state (with its captured sweep graphs) belongs
    to its graph and is released with it; a graph created afterwards, possibly
    at the same host address, starts from fresh state."""
    import gc
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:8]
    first = None
    for rep in range(3):
        G = P.Graph.from_synth(c1)
        out, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=8)
        assert max(s["cert_l1"] for s in st) <= 1e-8
        if first is None:
            first = out.copy()
        else:
            assert np.abs(out - first).sum(axis=1).max() <= 2e-8 + SLACK
        G.close()
        del G
        gc.collect()


def test_autotune_picks_a_width_and_queries_use_it(c1):
    """The autotuner times each (width, residue storage) end to end; later
    queries with batch_cols = 0 use the chosen width and that width's
    storage, an explicit storage overrides it, and every result stays
    certified."""
    G = P.Graph.from_synth(c1)
    res = G.autotune(ALPHA, 1e-8, widths=[4, 16])
    assert res["best"] in (4, 16)
    assert all(v > 0 for v in res["us_per_query"].values())
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:6]
    out, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED)          # batch_cols = 0: tuned width
    assert all(s["batch_cols"] == res["best"] for s in st)
    assert max(s["cert_l1"] for s in st) <= 1e-8
    if res["best"] == 4:
        assert all(s["residue_format"] == P.RESIDUE_F32 for s in st)
    _, st16 = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=16, residue_format=P.RESIDUE_F32)
    assert all(s["residue_format"] == P.RESIDUE_F32 for s in st16)
    _, st16 = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=16, residue_format=P.RESIDUE_BF16)
    assert all(s["residue_format"] == P.RESIDUE_BF16 for s in st16)
    with pytest.raises(P.PPRError):
        G.autotune(ALPHA, 0.0, widths=[4])


@pytest.mark.parametrize("self_loops", [False, True])
@pytest.mark.parametrize("chunks", [1, 5])
def test_random_small_graphs_vs_dense_solve(self_loops, chunks):
    """Section 2 allows self-loops (d_v counts them): the batched path on small
    random graphs against numpy's dense solve of Eq. 1, every source."""
    from conftest import dense_ppr_matrix
    for n, p, seed in ((30, 0.2, 1), (120, 0.05, 2), (200, 0.03, 3)):
        g = synth.random_small(n, p, seed, self_loops=self_loops)
        Pi = dense_ppr_matrix(g, ALPHA)
        G = P.Graph.from_synth(g)
        srcs = list(range(n))
        out, st = G.query_batch(srcs, ALPHA, 1e-10, P.MIXED, batch_cols=32, sweep_chunks=chunks)
        err = np.abs(out - Pi).sum(axis=1)
        assert err.max() <= 1e-10 + SLACK, (n, int(err.argmax()), err.max())
        assert max(s["cert_l1"] for s in st) <= 1e-10
        G.close()


def test_concurrent_queries_on_one_graph(c1):
    """Queries on one graph from several host threads at once (each call takes
    its own state and stream from the graph's pools) give the results of the
    same queries run one after another."""
    import threading
    srcs = [int(s) for s in synth.sources(c1.n, 40)]
    G = P.Graph.from_synth(c1)
    jobs = [("mixed", srcs[8 * k:8 * k + 8]) for k in range(4)] + [("fp64", [srcs[k]]) for k in range(4)]

    def run(kind, ss):
        if kind == "mixed":
            return G.query_batch(ss, ALPHA, 1e-8, P.MIXED, batch_cols=8, sweep_chunks=2)[0]
        return G.query_batch(ss, ALPHA, 1e-8, P.FP64)[0]

    seq = [run(k, ss) for k, ss in jobs]
    res = [None] * len(jobs)
    errs = []

    def worker(i):
        try:
            for _ in range(3):
                res[i] = run(*jobs[i])
        except Exception as e:          # surfaced below
            errs.append(e)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(len(jobs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for i in range(len(jobs)):
        # FP64 atomics in the local phase may reorder additions: a few ulps
        assert np.abs(res[i] - seq[i]).sum(axis=1).max() <= 1e-12, i


@pytest.mark.parametrize("omega", [1.15, 1.25])
def test_over_relaxed_sweeps_certified(c1, c1_truth, omega):
    """sor_omega > 1 with block Gauss-Seidel chunks: every column still ends
    certified within lambda of the truth, a column's schedule still depends
    on its own source only (alone vs in a block of 32), and fewer sweeps are
    needed than without over-relaxation on this power-law graph."""
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:32]
    G = P.Graph.from_synth(c1)
    out, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=32, sweep_chunks=4, sor_omega=omega)
    _check_batch(c1, srcs, out, st, 1e-8, c1_truth)
    _, st1 = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=32, sweep_chunks=4, sor_omega=1.0)
    assert np.mean([s["sweeps"] for s in st]) < np.mean([s["sweeps"] for s in st1])
    for b in (0, 13):
        alone, sal = G.query_batch([srcs[b]], ALPHA, 1e-8, P.MIXED, batch_cols=8, sweep_chunks=4,
                                   sor_omega=omega, residue_format=st[b]["residue_format"])
        assert sal[0]["sweeps"] == st[b]["sweeps"]
        assert np.abs(alone[0] - out[b]).sum() <= SLACK
    G.close()


def test_automatic_over_relaxation(c1):
    """sor_omega = 0 (the default) over-relaxes with 1.2 when a sweep has
    more than one chunk and not at all with one chunk."""
    srcs = [int(s) for s in synth.sources(c1.n, 9)][:8]
    G = P.Graph.from_synth(c1)
    for chunks, same in ((4, 1.2), (1, 1.0)):
        out, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=8, sweep_chunks=chunks)
        ref, sref = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=8, sweep_chunks=chunks, sor_omega=same)
        assert [s["sweeps"] for s in st] == [s["sweeps"] for s in sref]
        np.testing.assert_array_equal(out, ref)
        if chunks == 1:
            assert all(s["sor_omega"] == 1.0 for s in st)
    with pytest.raises(P.PPRError):
        G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, sor_omega=0.9)
    G.close()


@pytest.mark.parametrize("chunks,lam", [(1, 1e-8), (4, 1e-8), (4, 1e-6)])
def test_bf16_residues_certified(c1, c1_truth, chunks, lam):
    """bf16 residue storage: every column still ends certified within lambda
    of the truth (the FP64 refresh measures what the storage rounding left
    behind), with more refresh stages than FP32 storage needs, and a column's
    result does not depend on the block it ran in."""
    srcs = [int(s) for s in synth.sources(c1.n, 40)][:32]
    print(f"[gpu] bf16 residues c1 chunks={chunks} lam={lam}", flush=True)
    G = P.Graph.from_synth(c1)
    out, st = G.query_batch(srcs, ALPHA, lam, P.MIXED, batch_cols=32, sweep_chunks=chunks,
                            residue_format=P.RESIDUE_BF16)
    _check_batch(c1, srcs, out, st, lam, c1_truth)
    _, st32 = G.query_batch(srcs, ALPHA, lam, P.MIXED, batch_cols=32, sweep_chunks=chunks,
                            residue_format=P.RESIDUE_F32)
    assert np.mean([s["refreshes"] for s in st]) > np.mean([s["refreshes"] for s in st32])
    for b in (0, 17):
        alone, sal = G.query_batch([srcs[b]], ALPHA, lam, P.MIXED, sweep_chunks=chunks,
                                   residue_format=P.RESIDUE_BF16)         # default width: 8 columns
        assert sal[0]["batch_cols"] == 8
        assert sal[0]["sweeps"] == st[b]["sweeps"] and sal[0]["refreshes"] == st[b]["refreshes"]
        assert np.abs(alone[0] - out[b]).sum() <= SLACK
    G.close()


def test_bf16_serving_block(c1, c1_truth):
    """A serving block with bf16 residues: slots refilled as they retire, every
    result certified."""
    G = P.Graph.from_synth(c1)
    srcs = [int(s) for s in synth.sources(c1.n, 10)]
    with pytest.raises(P.PPRError):                  # bf16 vectors hold 8 columns
        P.Block(G, 4, ALPHA, residue_format=P.RESIDUE_BF16)
    blk = P.Block(G, 8, ALPHA, sweep_chunks=4, residue_format=P.RESIDUE_BF16)
    pending, slot_of, res = list(range(10)), {}, {}
    steps = 0
    while len(res) < 10:
        for slot in blk.poll(wait=True)["done"]:
            k = slot_of.pop(slot)
            res[k] = blk.retire(slot)
        while pending and len(slot_of) < 6:
            k = pending.pop(0)
            slot_of[blk.admit(srcs[k], 1e-8)] = k
        if slot_of:
            blk.step(5)
            steps += 1
        assert steps < 10000
    blk.close()
    _check_batch(c1, srcs, np.stack([res[k][0] for k in range(10)]), [res[k][1] for k in range(10)], 1e-8,
                 c1_truth)
    G.close()


def test_over_relaxation_falls_back_on_a_cycle():
    """On a directed cycle over-relaxed pushes make the residue grow; the
    refresh that ends the first stage measures it and the column continues
    with omega = 1, still certified.  (switch_param = 1e30 skips the local
    phase, which would otherwise finish a cycle on its own.)"""
    a = 1 - ALPHA
    n = 1000
    g = synth.cycle(n)
    x = np.array([ALPHA * a ** ((v - 5) % n) / (1 - a ** n) for v in range(n)])
    G = P.Graph.from_synth(g)
    out, st = G.query_batch([5, 17], ALPHA, 1e-8, P.MIXED, batch_cols=4, sweep_chunks=4, sor_omega=1.25,
                            switch_param=1e30)
    assert st[0]["local_levels"] == 0
    assert st[0]["cert_l1"] <= 1e-8
    assert np.abs(out[0] - x).sum() <= 1e-8 + SLACK
    assert st[0]["refreshes"] >= 2
    assert st[0]["sor_omega"] == 1.0            # fell back
    G.close()

