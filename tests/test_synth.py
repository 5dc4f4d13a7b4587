"""The seeded input generator: determinism and the structural promises."""
import os
import subprocess
import sys

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check_graph(g):
    assert g.row_ptr[0] == 0 and g.row_ptr[-1] == g.m
    deg = np.diff(g.row_ptr)
    assert deg.min() >= 1                                  # no dead ends
    src = np.repeat(np.arange(g.n), deg)
    assert (src != g.col).all()                            # no self-loops
    key = src.astype(np.int64) * g.n + g.col
    assert np.all(np.diff(key) > 0)                        # rows ascending, no duplicates
    assert g.col.min() >= 0 and g.col.max() < g.n


def test_c1_shape():
    g = synth.chunglu(10_000, 100_000, 2.1, cache=False)
    assert g.m == 100_000 and len(g.col) == 100_000
    _check_graph(g)
    # heavy tail: the maximum degrees are far above the mean (10) and at most ~sqrt(m)-scale
    assert 100 < g.max_out < 2000 and 100 < g.max_in < 2000


def test_deterministic_and_thread_independent():
    a = synth.chunglu(20_000, 150_000, 2.1, seed=7, cache=False)
    b = synth.chunglu(20_000, 150_000, 2.1, seed=7, cache=False)
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.col, b.col)
    code = ("import sys, numpy as np; sys.path.insert(0, %r); import synth; "
            "g = synth.chunglu(20_000, 150_000, 2.1, seed=7, cache=False); "
            "print(int(g.row_ptr.sum() %% 1000003), int(g.col.astype(np.int64).sum()))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True,
                         env=dict(os.environ, OMP_NUM_THREADS="1")).stdout.split()
    assert int(out[0]) == int(a.row_ptr.sum() % 1000003)
    assert int(out[1]) == int(a.col.astype(np.int64).sum())
    c = synth.chunglu(20_000, 150_000, 2.1, seed=8, cache=False)
    assert not np.array_equal(a.col, c.col)


def test_degree_tail_exponent():
    """The in-degree tail follows the requested power law roughly (CCDF slope)."""
    g = synth.chunglu(200_000, 2_000_000, 2.1, cache=False)
    _check_graph(g)
    indeg = np.bincount(g.col, minlength=g.n)
    ks = np.array([20, 40, 80, 160])
    ccdf = np.array([(indeg >= k).mean() for k in ks])
    slope = np.polyfit(np.log(ks), np.log(ccdf), 1)[0]
    # CCDF ~ k^-(gamma-1) = k^-1.1 for gamma = 2.1; loose window (finite size, cap)
    assert -1.6 < slope < -0.7


def test_sources_uniform_and_seeded():
    s = synth.sources(1000, 5000)
    assert s.min() >= 0 and s.max() < 1000
    np.testing.assert_array_equal(s, synth.sources(1000, 5000))
    assert abs(s.mean() - 499.5) < 20


def test_small_fixed_graphs():
    g = synth.fig1()
    assert g.n == 5 and g.m == 13
    assert np.diff(g.row_ptr).tolist() == [2, 4, 2, 3, 2]
    assert synth.complete(4).m == 12
    assert synth.star(3).m == 6
    with pytest.raises(RuntimeError):
        synth.chunglu(10, 100, 2.1, cache=False)
