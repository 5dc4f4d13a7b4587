"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Each test ties an oracle routine to something other than the oracle itself:
values the paper prints for its worked examples (tests/golden), closed forms
derived from the alpha-random-walk definition, numpy's dense linear solve of
Eq. 1, scipy's sparse transpose, and the bounds the paper proves.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from conftest import dense_P, dense_ppr, dense_ppr_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA = 0.2


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Worked examples printed in the paper
# --------------------------------------------------------------------------

def test_fig2_forward_push_printed_values():
    """Figure 2 (Section 3.2): pushes on v1, v3, v2 with rmax = 0.099."""
    gold = _golden("fig2_forward_push.json")
    g = synth.fig1()
    a = gold["alpha"]
    pi = np.zeros(5)
    r = np.zeros(5)
    r[gold["s"]] = 1.0
    d = g.out_degree()
    rmax = gold["rmax"]
    v1, v3, v2 = gold["order"]
    assert r[v1] > d[v1] * rmax
    oracle.push(g, a, pi, r, v1)
    p = gold["printed"]["after_push_v1"]
    assert pi[0] == pytest.approx(p["pi_v1"], abs=1e-15)
    assert r[1] == pytest.approx(p["r_v2"], abs=1e-15)
    assert r[2] == pytest.approx(p["r_v3"], abs=1e-15)
    assert r[v3] > d[v3] * rmax
    before = r.copy()
    oracle.push(g, a, pi, r, v3)
    p = gold["printed"]["after_push_v3"]
    assert pi[2] == pytest.approx(p["pi_v3"], abs=1e-15)
    assert r[1] - before[1] == pytest.approx(p["increment_to_v2_and_v4"], abs=1e-15)
    assert r[3] - before[3] == pytest.approx(p["increment_to_v2_and_v4"], abs=1e-15)
    # v2 is now the only active node
    active = [v for v in range(5) if r[v] > d[v] * rmax]
    assert active == [v2]
    oracle.push(g, a, pi, r, v2)
    assert [v for v in range(5) if r[v] > d[v] * rmax] == gold["printed"]["after_push_v2"]["active_nodes"]
    # derived final state (push definition applied by hand)
    np.testing.assert_allclose(pi, [0.2, 0.112, 0.08, 0, 0], atol=1e-15)
    np.testing.assert_allclose(r, [0.112, 0, 0.112, 0.272, 0.112], atol=1e-15)


def test_fifo_on_fig1_derived_values():
    """Algorithm 2 on the Figure 1 graph with rmax = 0.099 pops v1, v2, v3 (FIFO)."""
    g = synth.fig1()
    pi, r, st, trace = oracle.fifo_fwdpush(g, 0, ALPHA, 0.099, trace_cap=16)
    assert [v for v, _ in trace] == [0, 1, 2]
    np.testing.assert_allclose(pi, [0.2, 0.08, 0.096, 0, 0], atol=1e-15)
    np.testing.assert_allclose(r, [0.08, 0.192, 0, 0.272, 0.08], atol=1e-15)
    assert st["edge_pushes"] == 2 + 4 + 2


def test_fig3_simultaneous_push_printed_values():
    """Figure 3 (Section 4.1): r^(1) = (0, .4, .4, 0, 0); then v2 pushes .08 and
    v3 pushes .16 along each out-edge."""
    gold = _golden("fig3_sim_forward_push.json")
    g = synth.fig1()
    a = gold["alpha"]
    r0 = np.zeros(5)
    r0[0] = 1.0
    pi = np.zeros(5)
    r1 = oracle.sim_sweep(g, a, r0, pi)
    assert r1[1] == pytest.approx(gold["printed"]["r1"]["v2"], abs=1e-15)
    assert r1[2] == pytest.approx(gold["printed"]["r1"]["v3"], abs=1e-15)
    assert r1[0] == 0 and r1[3] == 0 and r1[4] == 0
    r2 = oracle.sim_sweep(g, a, r1, pi)
    inc = gold["printed"]["iteration2_push_per_edge"]
    # v1 gets only v2's push, v4 gets both, v5 only v2's, v2 only v3's, v3 only v2's
    expect = np.array([inc["v2"], inc["v3"], inc["v2"], inc["v2"] + inc["v3"], inc["v2"]])
    np.testing.assert_allclose(r2, expect, atol=1e-15)
    np.testing.assert_allclose(pi, [0.2, 0.08, 0.08, 0, 0], atol=1e-15)
    assert r2.sum() == pytest.approx(0.64, abs=1e-15)


def test_iteration_sets_of_section_4_2():
    """S^(1) = {v2, v3} and S^(2) = all five nodes for a small rmax.  The
    five-node S^(2) holds for the simultaneous reading (every node of S^(1)
    pushes the residue it held at the start of the iteration); under Algorithm
    2's strict membership test v3 is still queued when v2 pushes to it, so only
    four nodes are appended (derived)."""
    gold = _golden("fig3_sim_forward_push.json")
    g = synth.fig1()
    # rmax = lambda / m = 0.001 -> lambda = 0.013; switch rule 1 with param 0 never switches
    _, _, _, _, levels = oracle.powerpush_sync(g, 0, ALPHA, 0.001 * g.m, oracle.SWITCH_EDGES, 0.0)
    # levels[j] = (|S^(j)|, vol, r_sum); recover the sets with a direct replay
    assert levels[0][0] == 1
    assert levels[1][0] == len(gold["printed"]["S1"])
    assert levels[2][0] == len(gold["printed"]["S2_with_rmax_0.001"])
    _, _, _, trace = oracle.fifo_fwdpush(g, 0, ALPHA, 0.001, trace_cap=64)
    s1 = sorted(v for v, j in trace if j == 1)
    s2 = sorted(v for v, j in trace if j == 2)
    assert s1 == gold["printed"]["S1"]
    assert s2 == [0, 1, 3, 4]


# --------------------------------------------------------------------------
# Exact answer: dense solve of Eq. 1 and closed forms of the walk definition
# --------------------------------------------------------------------------

def test_fig1_exact_answer():
    g = synth.fig1()
    x = dense_ppr(g, 0, ALPHA)
    np.testing.assert_allclose(x, [0.29366106, 0.27166882, 0.23285899, 0.14747736, 0.05433376],
                               atol=5e-9)
    for fn in (lambda: oracle.powerpush(g, 0, ALPHA, 1e-12)[0],
               lambda: oracle.powerpush_sync(g, 0, ALPHA, 1e-12)[0],
               lambda: oracle.powitr(g, 0, ALPHA, 200)):
        assert np.abs(fn() - x).sum() <= 1e-12


def _closed_cycle(n, s, a):
    al = 1 - a
    return np.array([a * al ** ((v - s) % n) / (1 - al ** n) for v in range(n)])


@pytest.mark.parametrize("n,s", [(7, 0), (12, 5)])
def test_cycle_closed_form(n, s):
    g = synth.cycle(n)
    x = _closed_cycle(n, s, ALPHA)
    np.testing.assert_allclose(dense_ppr(g, s, ALPHA), x, atol=1e-15)
    pi, r, st, _ = oracle.powerpush(g, s, ALPHA, 1e-10)
    assert np.abs(pi - x).sum() <= 1e-10
    pi, r, st, _, _ = oracle.powerpush_sync(g, s, ALPHA, 1e-10)
    assert np.abs(pi - x).sum() <= 1e-10
    assert np.abs(oracle.powitr(g, s, ALPHA, 135) - x).sum() <= 1e-12


def test_star_closed_form():
    L = 6
    a = 1 - ALPHA
    g = synth.star(L)
    # from the centre
    x = np.full(L + 1, ALPHA * a / ((1 - a * a) * L))
    x[0] = ALPHA / (1 - a * a)
    np.testing.assert_allclose(dense_ppr(g, 0, ALPHA), x, atol=1e-15)
    assert np.abs(oracle.powerpush(g, 0, ALPHA, 1e-11)[0] - x).sum() <= 1e-11
    assert np.abs(oracle.powerpush_sync(g, 0, ALPHA, 1e-11)[0] - x).sum() <= 1e-11
    # from leaf 3
    y = np.full(L + 1, ALPHA * a * a / ((1 - a * a) * L))
    y[0] = ALPHA * a / (1 - a * a)
    y[3] = ALPHA * (1 + a * a / ((1 - a * a) * L))
    np.testing.assert_allclose(dense_ppr(g, 3, ALPHA), y, atol=1e-15)
    assert np.abs(oracle.powerpush(g, 3, ALPHA, 1e-11)[0] - y).sum() <= 1e-11
    assert np.abs(oracle.powerpush_sync(g, 3, ALPHA, 1e-11)[0] - y).sum() <= 1e-11


def test_complete_digraph_closed_form():
    n = 9
    a = 1 - ALPHA
    g = synth.complete(n)
    ps = 1.0 / n + ALPHA * (n - 1) ** 2 / (n * (n - 1 + a))
    x = np.full(n, (1 - ps) / (n - 1))
    x[2] = ps
    np.testing.assert_allclose(dense_ppr(g, 2, ALPHA), x, atol=1e-15)
    assert np.abs(oracle.powerpush(g, 2, ALPHA, 1e-11)[0] - x).sum() <= 1e-11
    assert np.abs(oracle.powerpush_sync(g, 2, ALPHA, 1e-11)[0] - x).sum() <= 1e-11


def test_self_loop_single_node():
    """The only node keeps all the mass: pi = 1.  Exercises the snapshot-then-zero
    reading of the push (the printed order would lose the self-loop's mass)."""
    g = synth.self_loop()
    for lam in (1e-3, 1e-9):
        pi, r, st, _ = oracle.powerpush(g, 0, ALPHA, lam)
        assert pi[0] + r[0] == pytest.approx(1.0, abs=1e-15)
        assert 1.0 - pi[0] <= lam
        pi, r, st, _, _ = oracle.powerpush_sync(g, 0, ALPHA, lam)
        assert pi[0] + r[0] == pytest.approx(1.0, abs=1e-15)
        assert 1.0 - pi[0] <= lam


# --------------------------------------------------------------------------
# Random small graphs against numpy's dense solve (n <= 200)
# --------------------------------------------------------------------------

GRAPHS = [(12, 0.3, 1), (40, 0.1, 2), (90, 0.05, 3), (200, 0.02, 4), (150, 0.04, 5)]


@pytest.mark.parametrize("n,p,seed", GRAPHS)
@pytest.mark.parametrize("lam", [1e-4, 1e-8])
def test_random_graphs_vs_dense_solve(n, p, seed, lam):
    g = synth.random_small(n, p, seed, self_loops=(seed % 2 == 1))
    s = seed % n
    x = dense_ppr(g, s, ALPHA)
    for name, run in (("alg3", lambda: oracle.powerpush(g, s, ALPHA, lam)[:2]),
                      ("sync", lambda: oracle.powerpush_sync(g, s, ALPHA, lam)[:2]),
                      ("sync-edges", lambda: oracle.powerpush_sync(g, s, ALPHA, lam,
                                                                   oracle.SWITCH_EDGES, 8.0)[:2]),
                      ("sync-epochs", lambda: oracle.powerpush_sync(g, s, ALPHA, lam, oracle.SWITCH_EDGES, 8.0,
                                                                    global_rule=oracle.GLOBAL_EPOCHS)[:2])):
        pi, r = run()
        err = np.abs(pi - x).sum()
        assert err <= lam, name
        # residues are non-negative, so the error equals r_sum (Section 3.2)
        assert (r >= 0).all()
        assert err == pytest.approx(r.sum(), rel=1e-9, abs=1e-15), name
        # the certificate bounds the error and is tight for r >= 0; both sides
        # carry FP64 cancellation error of a few ulps of sum(pi)/alpha ~ 1e-15
        cert = oracle.certificate(g, s, ALPHA, pi)
        assert cert >= err - 2e-15
        assert cert == pytest.approx(err, rel=1e-6, abs=2e-15)


@pytest.mark.parametrize("n,p,seed", GRAPHS[:3])
def test_invariant_pi_s_equals_reserve_plus_residue_walks(n, p, seed):
    """pi_s = pi_hat + sum_v r(v) pi_v at any intermediate state (Section 3.2)."""
    g = synth.random_small(n, p, seed)
    Pi = dense_ppr_matrix(g, ALPHA)
    s = 1
    for rmax in (0.05, 0.003):
        pi, r, _, _ = oracle.fifo_fwdpush(g, s, ALPHA, rmax)
        np.testing.assert_allclose(pi + r @ Pi, Pi[s], atol=1e-14)
    r = np.zeros(n)
    r[s] = 1.0
    pi = np.zeros(n)
    for _ in range(5):
        r = oracle.sim_sweep(g, ALPHA, r, pi)
        np.testing.assert_allclose(pi + r @ Pi, Pi[s], atol=1e-14)


def test_sim_sweep_is_one_power_iteration_step():
    """Eq. 7: r_out = (1 - alpha) r_in P, checked with numpy's matrix product."""
    g = synth.random_small(60, 0.08, 9, self_loops=True)
    P = dense_P(g)
    rng = np.random.default_rng(0)
    r_in = rng.random(60)
    pi = rng.random(60)
    pi0 = pi.copy()
    r_out = oracle.sim_sweep(g, ALPHA, r_in, pi)
    np.testing.assert_allclose(r_out, (1 - ALPHA) * r_in @ P, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(pi, pi0 + ALPHA * r_in, rtol=1e-15)


def test_powitr_error_is_exactly_geometric():
    """Eq. 6: after K iterations the l1 error is exactly (1 - alpha)^K."""
    g = synth.random_small(80, 0.06, 11)
    x = dense_ppr(g, 7, ALPHA)
    for K in (1, 5, 20, 60):
        err = np.abs(oracle.powitr(g, 7, ALPHA, K) - x).sum()
        assert err == pytest.approx((1 - ALPHA) ** K, rel=1e-10)


# --------------------------------------------------------------------------
# Rates, conservation and the paper's bounds
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    return synth.chunglu(10_000, 100_000, 2.1)


def test_threshold_zero_sweeps_contract_by_exactly_one_minus_alpha(c1):
    """Lemma 1 / Eq. 6: each rmax = 0 sweep multiplies r_sum by (1 - alpha)."""
    s = int(synth.sources(c1.n, 1)[0])
    pi, r, st, trace, levels = oracle.powerpush_sync(c1, s, ALPHA, 1e-8, trace_cap=256)
    ratios = trace[1:] / trace[:-1]
    np.testing.assert_allclose(ratios, 1 - ALPHA, rtol=1e-12)
    # sweep count follows from the closed form
    K = math.ceil(math.log(1e-8 / trace[0]) / math.log(1 - ALPHA))
    assert st["sweeps"] in (K, K + 1)
    # mass conservation
    assert pi.sum() + r.sum() == pytest.approx(1.0, abs=1e-13)


def test_eq9_per_iteration_contraction(c1):
    """Eq. 9: r_sum^(j+1) <= (1 - alpha/m * sum_{v in S^(j)} d_v) r_sum^(j) for the
    iterations of the level-synchronous local phase (S^(j) = all active nodes)."""
    for s in synth.sources(c1.n, 4):
        _, _, st, _, levels = oracle.powerpush_sync(c1, int(s), ALPHA, 1e-8, oracle.SWITCH_EDGES, 0.5)
        assert len(levels) >= 3
        for (sz, vol, rs), (_, _, rs_next) in zip(levels[:-1], levels[1:]):
            assert rs_next <= (1 - ALPHA / c1.m * vol) * rs * (1 + 1e-12)


def test_lemma3_lemma4_fifo_work_bound(c1):
    """Theorem 1: FIFO-FwdPush with rmax = lambda/m stops within
    (m/alpha) ln(1/lambda) + m + m/alpha edge pushes (Lemmas 3 and 4)."""
    lam = 1e-6
    for s in synth.sources(c1.n, 3):
        pi, r, st, _ = oracle.fifo_fwdpush(c1, int(s), ALPHA, lam / c1.m)
        bound = c1.m / ALPHA * math.log(1 / lam) + c1.m + c1.m / ALPHA
        assert st["edge_pushes"] <= bound
        d = c1.out_degree()
        assert (r <= d * (lam / c1.m)).all()
        assert r.sum() <= lam


def test_alg3_epoch_postconditions_and_truth(c1):
    """Algorithm 3: after epoch i, r_sum <= m * lambda^(i/8) / m; the result is
    within lambda of the converged power iteration (error (0.8)^135 < 1e-13)."""
    lam = 1e-8
    s = int(synth.sources(c1.n, 1)[0])
    pi, r, st, trace = oracle.powerpush(c1, s, ALPHA, lam, trace_cap=512)
    k = 1
    for i, scans in enumerate(st["scans_per_epoch"], start=1):
        k += scans
        if scans:
            assert trace[k - 1] <= c1.m * (lam ** (i / 8) / c1.m)
    truth = oracle.powitr(c1, s, ALPHA, 135)
    err = np.abs(pi - truth).sum()
    assert err <= lam
    assert err == pytest.approx(st["r_sum"], rel=1e-4)
    pi2, r2, st2, _, _ = oracle.powerpush_sync(c1, s, ALPHA, lam)
    assert np.abs(pi2 - truth).sum() <= lam


def test_certificate_equals_residue_for_exact_pushes(c1):
    """For a push-based pi_hat the certificate's residual equals the maintained
    residue r (both are e_s - pi_hat (I - (1-alpha)P)/alpha)."""
    s = int(synth.sources(c1.n, 2)[1])
    pi, r, st, _ = oracle.powerpush(c1, s, ALPHA, 1e-7)
    cert, rt = oracle.certificate(c1, s, ALPHA, pi, want_residual=True)
    np.testing.assert_allclose(rt, r, atol=1e-15)
    assert cert == pytest.approx(r.sum(), rel=1e-9)


def test_csc_matches_scipy_transpose(c1):
    sp = pytest.importorskip("scipy.sparse")
    col_ptr, row_idx, deg = oracle.csc(c1)
    A = sp.csr_matrix((np.ones(c1.m), c1.col, c1.row_ptr), shape=(c1.n, c1.n)).tocsc()
    A.sort_indices()
    np.testing.assert_array_equal(col_ptr, A.indptr)
    np.testing.assert_array_equal(row_idx, A.indices)
    np.testing.assert_array_equal(deg, np.diff(c1.row_ptr))


@pytest.mark.parametrize("n,p,seed", GRAPHS[:3])
def test_epochs_schedule_invariant_and_thresholds(n, p, seed):
    """Algorithm 3's epochs taken simultaneously: the final state satisfies the
    invariant pi_s = pi_hat + sum_v r(v) pi_v (Section 3.2) with r >= 0, the
    residue sum is <= lambda, and the scans push fewer edges than threshold-0
    sweeps to the same lambda (the point of the dynamic threshold).  The switch
    parameter 1e30 sends the query straight to the global phase."""
    from conftest import dense_ppr_matrix
    g = synth.random_small(n, p, seed, self_loops=True)
    Pi = dense_ppr_matrix(g, ALPHA)
    s = 2
    for lam in (1e-6, 1e-10):
        pi, r, st, _, _ = oracle.powerpush_sync(g, s, ALPHA, lam, oracle.SWITCH_EDGES, 1e30,
                                                global_rule=oracle.GLOBAL_EPOCHS)
        assert (r >= 0).all() and r.sum() <= lam
        np.testing.assert_allclose(pi + r @ Pi, Pi[s], atol=1e-14)
        _, _, st0, _, _ = oracle.powerpush_sync(g, s, ALPHA, lam, oracle.SWITCH_EDGES, 1e30)
        assert st["edge_pushes"] < st0["edge_pushes"]


def test_powerpush_many_rows_are_the_single_queries(c1):
    """The query-parallel form (one Algorithm 3 query per host thread) writes row i
    from sources[i]: each row and its statistics equal the single query bit for
    bit (more sources than threads, a repeated source, the first and last node),
    and each row is within lambda of the converged power iteration."""
    lam = 1e-7
    srcs = [int(s) for s in synth.sources(c1.n, 5)] + [0, c1.n - 1]
    srcs.append(srcs[1])
    pi_many, st_many = oracle.powerpush_many(c1, srcs, ALPHA, lam, threads=3)
    assert pi_many.shape == (len(srcs), c1.n)
    for i, s in enumerate(srcs):
        pi, r, st, _ = oracle.powerpush(c1, s, ALPHA, lam)
        assert np.array_equal(pi_many[i], pi), i
        assert st_many[i] == st, i
    for i in (0, len(srcs) - 2):
        truth = oracle.powitr(c1, srcs[i], ALPHA, 135)
        assert np.abs(pi_many[i] - truth).sum() <= lam


def test_powerpush_many_on_small_graphs_meets_the_dense_solve():
    """Every row of the query-parallel form against numpy's dense solve of Eq. 1
    for its own source (n <= 60, self-loops included)."""
    rng = np.random.default_rng(11)
    for trial in range(4):
        n = int(rng.integers(8, 60))
        g = synth.random_small(n, 0.15, seed=100 + trial, self_loops=True)
        X = dense_ppr_matrix(g, ALPHA)
        srcs = list(range(0, n, max(1, n // 9)))
        pi_many, _ = oracle.powerpush_many(g, srcs, ALPHA, 1e-10, threads=4)
        for i, s in enumerate(srcs):
            assert np.abs(pi_many[i] - X[s]).sum() <= 1e-10


def test_native_build_gives_the_same_answers(c1):
    """The timed CPU baseline runs an -O3 -march=native build of the same source
    (no floating-point contraction): its answers equal the test build's bit for bit."""
    srcs = [int(s) for s in synth.sources(c1.n, 3)]
    a, sa = oracle.powerpush_many(c1, srcs, ALPHA, 1e-8, threads=3)
    b, sb = oracle.powerpush_many(c1, srcs, ALPHA, 1e-8, threads=3, native=True)
    assert np.array_equal(a, b) and sa == sb
