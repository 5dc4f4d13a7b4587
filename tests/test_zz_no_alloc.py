"""The allocation-free FP64 query (ppr_query_fp64_noalloc) against the
entry point it varies, ppr_query with PPR_FP64, and against the oracle.

Both run the same kernels in the same order; they differ only in where the
working state lives (a static device array instead of a pooled context) and
in how the sweeps are launched (one by one instead of a captured graph), so
the statistics are equal and the vectors agree to FP64 rounding order (the
local phase's atomic adds), rtol 1e-11 as for every FP64 parity test.  Two
calls in a row, the second on a smaller graph, show that nothing of the
first call's state leaks into the second.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2101_03652_amd")

pytestmark = pytest.mark.gpu
ALPHA = 0.2
RTOL = 1e-11
ATOL = 1e-20


def _check_against_entry_point(G, g, s, lam, stream=None):
    out_ref = torch.empty(g.n, dtype=torch.float64, device="cuda")
    _, st_ref = G.query(s, ALPHA, lam, P.FP64, out=out_ref)
    out = torch.full((g.n,), float("nan"), dtype=torch.float64, device="cuda")
    if stream is not None:
        # the caller's stream first overwrites the output; the call's kernels
        # run after that work, in stream order
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            out.fill_(-1.0)
    st = G.query_noalloc(s, ALPHA, lam, out, stream=stream)
    torch.cuda.synchronize()
    pi = out.cpu().numpy()
    ref = out_ref.cpu().numpy()
    assert np.isfinite(pi).all()
    for k in ("local_levels", "sweeps", "edge_pushes"):
        assert st[k] == st_ref[k], (k, st[k], st_ref[k])
    assert st["r_sum"] <= lam
    np.testing.assert_allclose(pi, ref, rtol=RTOL, atol=ATOL)
    # and the oracle's level-synchronous schedule (the FP64 path's parity reference)
    pio, _, sto, _, _ = oracle.powerpush_sync(g, s, ALPHA, lam, oracle.SWITCH_EDGES, 32.0)
    assert st["local_levels"] == sto["local_levels"] and st["sweeps"] == sto["sweeps"]
    np.testing.assert_allclose(pi, pio, rtol=RTOL, atol=ATOL)
    assert oracle.certificate(g, s, ALPHA, pi) <= lam
    return st


def test_two_calls_in_a_row_the_second_smaller():
    big = synth.chunglu(60_000, 700_000, 2.1, seed=17)
    small = synth.chunglu(10_000, 100_000, 2.1)
    Gb = P.Graph.from_synth(big)
    s1 = int(synth.sources(big.n, 1)[0])
    print(f"[gpu] noalloc call 1: n={big.n} m={big.m} s={s1}", flush=True)
    _check_against_entry_point(Gb, big, s1, 1e-8)
    Gs = P.Graph.from_synth(small)
    s2 = int(synth.sources(small.n, 2)[1])
    print(f"[gpu] noalloc call 2: n={small.n} m={small.m} s={s2}", flush=True)
    _check_against_entry_point(Gs, small, s2, 1e-8)
    # and the first graph again, after the smaller one overwrote part of the array
    print(f"[gpu] noalloc call 3: n={big.n} s={s1}, lambda 1e-6", flush=True)
    _check_against_entry_point(Gb, big, s1, 1e-6)


def test_on_a_caller_stream():
    g = synth.chunglu(10_000, 100_000, 2.1)
    G = P.Graph.from_synth(g)
    st = torch.cuda.Stream()
    for s in synth.sources(g.n, 3).tolist():
        print(f"[gpu] noalloc on a caller stream: s={s}", flush=True)
        _check_against_entry_point(G, g, int(s), 1e-8, stream=st)


def test_limits_and_arguments():
    # one node over the limit: refused before anything runs
    n = P.NOALLOC_MAX_NODES + 1
    row_ptr = np.arange(n + 1, dtype=np.int64)
    col = ((np.arange(n) + 1) % n).astype(np.int32)
    G = P.Graph(row_ptr, col, n)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    print(f"[gpu] noalloc limit: n={n}", flush=True)
    with pytest.raises(P.PPRError) as e:
        G.query_noalloc(0, ALPHA, 1e-8, out)
    assert e.value.status == -1 and "at most" in str(e.value)
    g = synth.fig1()
    G = P.Graph.from_synth(g)
    with pytest.raises(P.PPRError) as e:                  # host output
        G.query_noalloc(0, ALPHA, 1e-8, np.zeros(g.n))
    assert e.value.status == -1
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    for bad in ((g.n, ALPHA, 1e-8), (-1, ALPHA, 1e-8), (0, 0.0, 1e-8), (0, ALPHA, 0.0), (0, ALPHA, 2.0)):
        with pytest.raises(P.PPRError) as e:
            G.query_noalloc(bad[0], bad[1], bad[2], out)
        assert e.value.status == -1
    # Figure 1, exact answer (numpy's dense solve of Eq. 1)
    st = G.query_noalloc(0, ALPHA, 1e-12, out)
    x = np.array([0.29366106, 0.27166882, 0.23285899, 0.14747736, 0.05433376])
    assert np.abs(out.cpu().numpy() - x).sum() <= 1e-7
    assert st["r_sum"] <= 1e-12
