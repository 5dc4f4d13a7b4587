"""Pins of the oracle's approximate SSPPR (SpeedPPR, Section 6, Algorithm 4):
the walk generator, the alpha-random walk, the refinement and the Monte
Carlo phase, each against something other than itself: published generator
values, closed forms, dense solves and sampling statistics."""
import math

import numpy as np
import pytest

import oracle
import synth
from conftest import dense_ppr, dense_ppr_matrix

ALPHA = 0.2
GAMMA = 0x9E3779B97F4A7C15


def test_splitmix64_published_outputs():
    """SplitMix64 seeded with 0 (Steele, Lea, Flood 2014): its first outputs."""
    assert oracle.splitmix64(0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(GAMMA) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64(2 * GAMMA % 2 ** 64) == 0x06C45D188009454F


def test_walks_on_a_cycle_stop_like_the_closed_form():
    """On a directed n-cycle a walk's stop node is (steps mod n) hops from its
    start, so the stop frequencies of many walks estimate
    pi(v_k) = alpha a^k / (1 - a^n), a = 1 - alpha (Section 2): within 5 sigma."""
    n, N = 6, 60_000
    g = synth.cycle(n)
    a = 1 - ALPHA
    want = np.array([ALPHA * a ** k / (1 - a ** n) for k in range(n)])
    cnt = np.zeros(n)
    for j in range(N):
        cnt[(oracle.walk_endpoint(g, ALPHA, 7, 2, j) - 2) % n] += 1
    f = cnt / N
    sigma = np.sqrt(want * (1 - want) / N)
    assert np.all(np.abs(f - want) <= 5 * sigma), (f, want)


def test_walks_on_fig1_match_the_dense_solve():
    """Stop frequencies of walks from v1 on the Figure 1 graph against pi_{v1}
    (dense solve of Eq. 1): this exercises the uniform choice of the next node."""
    g = synth.fig1()
    N = 60_000
    want = dense_ppr(g, 0, ALPHA)
    cnt = np.zeros(g.n)
    for j in range(N):
        cnt[oracle.walk_endpoint(g, ALPHA, 11, 0, j)] += 1
    f = cnt / N
    sigma = np.sqrt(want * (1 - want) / N)
    assert np.all(np.abs(f - want) <= 5 * sigma), (f, want)


def test_walks_depend_on_seed_node_and_index_only():
    g = synth.random_small(60, 0.08, 3)
    a = [oracle.walk_endpoint(g, ALPHA, 5, 7, j) for j in range(200)]
    assert a == [oracle.walk_endpoint(g, ALPHA, 5, 7, j) for j in range(200)]
    b = [oracle.walk_endpoint(g, ALPHA, 6, 7, j) for j in range(200)]
    assert a != b
    # max_steps = 0: every walk stops where it starts
    assert all(oracle.walk_endpoint(g, ALPHA, 5, 7, j, max_steps=0) == 7 for j in range(20))


@pytest.mark.parametrize("n,p,seed", [(40, 0.1, 1), (80, 0.05, 2)])
def test_refinement_leaves_no_active_node_and_keeps_the_invariant(n, p, seed):
    """After the refinement no node is active w.r.t. rmax; mass is conserved
    and pi_s = pi_hat + sum_v r(v) pi_v still holds (Section 3.2), checked
    against the dense solve, from a state that Algorithm 3 left behind."""
    g = synth.random_small(n, p, seed)
    Pi = dense_ppr_matrix(g, ALPHA)
    d = np.diff(g.row_ptr).astype(np.float64)
    s = 3
    pi, r, st, _ = oracle.powerpush(g, s, ALPHA, 0.05)
    before = pi.sum() + r.sum()
    rmax = 1e-4
    assert np.any(r > d * rmax)
    levels, ep = oracle.refine_sync(g, ALPHA, rmax, pi, r)
    assert levels > 0 and ep > 0
    assert not np.any(r > d * rmax)
    assert abs(pi.sum() + r.sum() - before) <= 1e-14
    np.testing.assert_allclose(pi + r @ Pi, Pi[s], atol=1e-14)


def test_walk_budget_gives_the_relative_error_of_eq8():
    """Plain Monte Carlo with W of Eq. 8 walks from s estimates every
    pi(s, v) >= mu within relative error eps (with probability 1 - 1/n)."""
    g = synth.random_small(30, 0.12, 4)
    n = g.n
    eps, mu = 0.5, 1.0 / n
    W = oracle.walk_budget(n, eps, mu)
    assert W > 0 and math.isfinite(W)
    x = dense_ppr(g, 0, ALPHA)
    Wn = int(math.ceil(W))
    cnt = np.zeros(n)
    for j in range(Wn):
        cnt[oracle.walk_endpoint(g, ALPHA, 99, 0, j)] += 1
    est = cnt / Wn
    big = x >= mu
    assert np.all(np.abs(est[big] - x[big]) <= eps * x[big])
    # and the budget grows like 1 / (eps^2 mu)
    assert oracle.walk_budget(n, eps / 2, mu) / W == pytest.approx(4 * (2 * eps / 6 + 2) / (2 * eps / 3 + 2))
    assert oracle.walk_budget(n, eps, mu / 3) / W == pytest.approx(3.0)


def test_mc_phase_counts_mass_and_is_unbiased():
    """After a refinement w.r.t. 1 / W every W_v = ceil(r(v) W) is at most d_v
    (the argument of the running-time theorem of Section 6); the phase adds
    exactly sum_v r(v) to the mass; averaged over seeds the estimate
    pi_hat + sum_v r(v) f(v, .) / W_v approaches pi_s (Eq. 10)."""
    g = synth.fig1()
    d = np.diff(g.row_ptr).astype(np.float64)
    W = 40.0
    pi = np.zeros(g.n)
    r = np.zeros(g.n)
    r[0] = 1.0
    oracle.refine_sync(g, ALPHA, 1.0 / W, pi, r)
    assert np.all(np.ceil(r * W) <= d)
    truth = dense_ppr(g, 0, ALPHA)
    acc = np.zeros(g.n)
    runs = 3000
    for seed in range(runs):
        est = pi.copy()
        walks = oracle.mc_phase(g, ALPHA, W, seed, r, est)
        assert walks == int(np.ceil(r * W)[r > 0].sum())
        assert est.sum() == pytest.approx(pi.sum() + r.sum(), abs=1e-14)
        acc += est
    mean = acc / runs
    # per node the estimate's spread is at most r_sum; the mean of `runs` draws
    assert np.all(np.abs(mean - truth) <= 5 * r.sum() / np.sqrt(runs))


@pytest.mark.parametrize("eps", [0.5, 0.2])
def test_speedppr_relative_error(eps):
    """Algorithm 4 end to end in the oracle (Algorithm 3 to lambda = m / W,
    refinement to rmax = 1 / W, Monte Carlo): every node with pi >= mu = 1/n
    within relative error eps of the dense solve."""
    g = synth.random_small(120, 0.05, 8)
    n = g.n
    mu = 1.0 / n
    W = oracle.walk_budget(n, eps, mu)
    s = 5
    pi, r, _, _ = oracle.powerpush(g, s, ALPHA, min(g.m / W, 1.0))
    oracle.refine_sync(g, ALPHA, 1.0 / W, pi, r)
    d = np.diff(g.row_ptr)
    assert np.all(np.ceil(r * W) <= d)
    oracle.mc_phase(g, ALPHA, W, 2024, r, pi)
    x = dense_ppr(g, s, ALPHA)
    big = x >= mu
    assert np.all(np.abs(pi[big] - x[big]) <= eps * x[big])


def test_walk_budget_meets_the_chernoff_tail_with_the_natural_log():
    """Eq. 8 comes from the Chernoff bound for the number X of W walks that stop
    at v (Section 6): with E X = W pi and deviation eps E X,
        P[|X - E X| >= eps E X] <= 2 exp(-eps^2 E X / (2 + 2 eps / 3))
    (the two-sided bound for sums of independent [0, 1] variables).  At the
    smallest pi that matters, pi = mu, the budget of Eq. 8 puts this tail at
    exactly 2 / n^2 when its log is the natural logarithm; a base-10 log would
    leave a tail of 2 n^(-2 / ln 10), far above it, and a base-2 log one of
    2 n^(-2 / ln 2), far below it (more walks than the bound asks for)."""
    for n, eps, mu in [(10, 0.5, 0.1), (10_000, 0.5, 1e-4), (4_000_000, 0.1, 2.5e-7),
                       (40_000_000, 0.2, 1e-5), (1000, 1.0, 1e-3)]:
        W = oracle.walk_budget(n, eps, mu)
        tail = 2.0 * math.exp(-eps * eps * W * mu / (2.0 + 2.0 * eps / 3.0))
        assert tail == pytest.approx(2.0 / n ** 2, rel=1e-9), (n, eps, mu)
        for wrong_log in (math.log10, math.log2):
            W_wrong = W * wrong_log(n) / math.log(n)
            tail_wrong = 2.0 * math.exp(-eps * eps * W_wrong * mu / (2.0 + 2.0 * eps / 3.0))
            assert abs(tail_wrong - 2.0 / n ** 2) > 0.1 * (2.0 / n ** 2)
