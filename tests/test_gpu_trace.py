"""Convergence traces of the FP64 path (ppr_query_trace) against the oracle's
level-synchronous schedule and against closed forms.

Each point is the residue sum after one iteration.  On this path residues
stay non-negative, so that sum is the l1 error of the estimate (Section 2).
Global points are exact FP64 sums, compared at rtol 1e-10 (different
summation orders); local points are the running sums the switch test uses.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2101_03652_amd")

pytestmark = pytest.mark.gpu
ALPHA = 0.2


@pytest.fixture(scope="module")
def c1():
    return synth.chunglu(10_000, 100_000, 2.1)


def _check_common(tr, st):
    assert len(tr) == st["local_levels"] + st["sweeps"]
    assert np.all(np.diff(tr["ms"]) >= 0) and tr["ms"][0] >= 0
    assert np.all(np.diff(tr["edge_pushes"]) > 0)
    assert tr["edge_pushes"][-1] == st["edge_pushes"]
    loc = tr[tr["phase"] == 0]
    glo = tr[tr["phase"] == 1]
    if len(glo):
        assert tr["r_sum"][-1] == st["r_sum"]
    else:                       # the running sum against the exact one
        assert tr["r_sum"][-1] == pytest.approx(st["r_sum"], rel=1e-10, abs=1e-14)
    assert np.all(tr["phase"][:len(loc)] == 0)          # local iterations first
    assert loc["index"].tolist() == list(range(1, len(loc) + 1))
    assert glo["index"].tolist() == list(range(1, len(glo) + 1))
    return loc, glo


def _check_local(loc, levels, rsum_after_local):
    """Local point j against the oracle's iteration j: the r_sum at the start
    of iteration j + 1 (or, after the last one, the exact sum), and the
    cumulative volume of S^(1..j)."""
    assert len(loc) == len(levels)
    vols = np.cumsum([v for _, v, _ in levels])
    assert loc["edge_pushes"].tolist() == vols.tolist()
    want = [r for _, _, r in levels[1:]] + [rsum_after_local]
    np.testing.assert_allclose(loc["r_sum"], want, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("lam", [1e-6, 1e-8])
def test_powerpush_trace_matches_oracle(c1, lam):
    G = P.Graph.from_synth(c1)
    for s in [int(x) for x in synth.sources(c1.n, 3)]:
        print(f"[gpu] trace powerpush c1 s={s} lam={lam}", flush=True)
        pi, tr, st = G.query_trace(s, ALPHA, lam)
        pio, ro, sto, otr, levels = oracle.powerpush_sync(c1, s, ALPHA, lam, P.SWITCH_EDGES, P.options().switch_param,
                                                            trace_cap=512)
        loc, glo = _check_common(tr, st)
        assert st["local_levels"] == sto["local_levels"] and st["sweeps"] == sto["sweeps"]
        _check_local(loc, levels, otr[0])
        np.testing.assert_allclose(glo["r_sum"], otr[1:], rtol=1e-10)
        # Lemma 1: each threshold-0 sweep contracts the residue sum by 1 - alpha
        ratios = glo["r_sum"][1:] / glo["r_sum"][:-1]
        np.testing.assert_allclose(ratios, 1 - ALPHA, rtol=1e-12)
        assert glo["edge_pushes"].tolist() == [loc["edge_pushes"][-1] + k * c1.m for k in range(1, len(glo) + 1)]
        # same answer as the untraced query
        pu, su = G.query(s, ALPHA, lam, P.FP64)
        np.testing.assert_allclose(pi, pu, rtol=1e-12, atol=1e-20)
        assert su["sweeps"] == st["sweeps"]
    G.close()


@pytest.mark.parametrize("slices", [0, 3, 8])
def test_power_iteration_trace_is_eq6(c1, slices):
    """switch_param = 1e30: no local phase; from e_s the residue sum after k
    sweeps is (1 - alpha)^k exactly (Eq. 6), which is also the l1 error of
    power iteration after k steps; also with the sweep split into passes over
    source slices (slices > 1)."""
    G = P.Graph.from_synth(c1, fp64_slices=slices)
    assert G.info()["fp64_slices"] == max(slices, 1)
    s = int(synth.sources(c1.n, 1)[0])
    pi, tr, st = G.query_trace(s, ALPHA, 1e-8, switch_param=1e30)
    loc, glo = _check_common(tr, st)
    assert len(loc) == 0
    k = np.arange(1, len(glo) + 1)
    np.testing.assert_allclose(glo["r_sum"], (1 - ALPHA) ** k, rtol=1e-12)
    assert len(glo) == int(np.ceil(np.log(1e-8) / np.log(1 - ALPHA)))
    G.close()


def test_forward_push_trace_matches_oracle(c1):
    """switch_param = 0: the level-synchronous forward push (Algorithm 2)
    to the end; every point is local."""
    G = P.Graph.from_synth(c1)
    s = int(synth.sources(c1.n, 2)[1])
    pi, tr, st = G.query_trace(s, ALPHA, 1e-8, switch_param=0.0)
    pio, ro, sto, otr, levels = oracle.powerpush_sync(c1, s, ALPHA, 1e-8, P.SWITCH_EDGES, 0.0, trace_cap=16,
                                                      level_cap=4096)
    loc, glo = _check_common(tr, st)
    assert len(glo) == 0
    _check_local(loc, levels, otr[0])
    assert tr["r_sum"][-1] <= 1e-8 * (1 + 1e-9)
    G.close()


def test_epoch_trace_matches_oracle(c1):
    G = P.Graph.from_synth(c1)
    s = int(synth.sources(c1.n, 3)[2])
    pi, tr, st = G.query_trace(s, ALPHA, 1e-8, global_rule=P.GLOBAL_EPOCHS)
    pio, ro, sto, otr, levels = oracle.powerpush_sync(c1, s, ALPHA, 1e-8, P.SWITCH_EDGES, P.options().switch_param, trace_cap=1024,
                                                      global_rule=oracle.GLOBAL_EPOCHS)
    loc, glo = _check_common(tr, st)
    assert st["sweeps"] == sto["sweeps"] and st["edge_pushes"] == sto["edge_pushes"]
    _check_local(loc, levels, otr[0])
    np.testing.assert_allclose(glo["r_sum"], otr[1:], rtol=1e-10)
    G.close()


def test_trace_arguments(c1):
    G = P.Graph.from_synth(c1)
    s = int(synth.sources(c1.n, 1)[0])
    with pytest.raises(P.PPRError):                    # more iterations than room
        G.query_trace(s, ALPHA, 1e-8, capacity=5)
    lib = P.load()
    out = np.empty(c1.n)
    cnt = ctypes.c_int32(-5)
    tr = np.zeros(8, dtype=P.TRACE_DTYPE)
    o = P.options(precision=P.MIXED)
    assert lib.ppr_query_trace(G.handle, s, ALPHA, 1e-8, ctypes.byref(o), P._ptr(out), P._ptr(tr), 8,
                               ctypes.byref(cnt), None) == -1
    o = P.options(precision=P.FP64)
    assert lib.ppr_query_trace(G.handle, s, ALPHA, 1e-8, ctypes.byref(o), P._ptr(out), None, 8,
                               ctypes.byref(cnt), None) == -1
    # capacity 0: only the count
    assert lib.ppr_query_trace(G.handle, s, ALPHA, 1e-8, ctypes.byref(o), P._ptr(out), None, 0,
                               ctypes.byref(cnt), None) == 0
    _, tr_full, st = G.query_trace(s, ALPHA, 1e-8)
    assert cnt.value == len(tr_full) == st["local_levels"] + st["sweeps"]
    G.close()
