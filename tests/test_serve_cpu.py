"""Host-side serving policy: slot choice under a memory budget, latency
percentiles and the seeded arrival trace."""
import numpy as np
import pytest

from paper_2101_03652_amd.serve import choose_slots, percentile, poisson_trace


def test_choose_slots_widest_that_fits():
    fp = lambda w: 1000 + 100 * w
    assert choose_slots(10**9, fp, 32) == 32
    assert choose_slots(1000 + 100 * 16, fp, 32) == 16      # exactly fits 16
    assert choose_slots(1000 + 100 * 16 - 1, fp, 32) == 8
    assert choose_slots(1000 + 100 * 4, fp, 128) == 4
    assert choose_slots(1000 + 100 * 4 - 1, fp, 128) == 0   # nothing fits
    assert choose_slots(10**9, fp, 48) == 32                 # rounds down to a power of two
    for free in range(0, 20000, 37):
        w = choose_slots(free, fp, 128)
        assert w == 0 or fp(w) <= free
        if w and w < 128:
            assert fp(2 * w) > free


def test_percentile_matches_numpy_linear():
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 100, 2001):
        x = rng.exponential(size=n)
        for q in (0, 50, 90, 99, 100):
            assert percentile(x, q) == pytest.approx(np.percentile(x, q), rel=1e-12, abs=0)
    assert np.isnan(percentile([], 50))


def test_poisson_trace_is_seeded_and_has_the_rate():
    t1, g1, l1 = poisson_trace(50.0, 20000, 3, seed=9)
    t2, g2, l2 = poisson_trace(50.0, 20000, 3, seed=9)
    assert np.array_equal(t1, t2) and np.array_equal(g1, g2) and np.array_equal(l1, l2)
    assert t1[0] == 0.0 and np.all(np.diff(t1) >= 0)
    rate = (len(t1) - 1) / t1[-1]
    assert rate == pytest.approx(50.0, rel=0.03)
    assert set(np.unique(g1)) == {0, 1, 2}
    assert set(np.unique(l1)) == {1e-6, 1e-8}
    assert abs(np.mean(l1 == 1e-6) - 0.5) < 0.02
