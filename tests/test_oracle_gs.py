"""Pins of the oracle's block Gauss-Seidel sweep (the batched GPU path's
global sweep): one chunk is Eq. 7; one row per chunk is sequential
Gauss-Seidel (a triangular solve); any chunking equals Algorithm 3's in-place
push scan taken a chunk at a time (push operations of Section 3.2 written
out here independently); iterated, it converges to the dense-solve PPR with
the residual contracting by at least 1 - alpha per sweep."""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from conftest import dense_P, dense_ppr

ALPHA = 0.2


def _A_and_deg(g):
    P = dense_P(g)
    d = np.diff(g.row_ptr).astype(np.float64)
    return P * d[:, None], d          # A[v, u] = number of edges v -> u


@pytest.mark.parametrize("fresh", [False, True])
def test_one_chunk_is_eq7(fresh):
    g = synth.random_small(60, 0.08, 9, self_loops=True)
    A, d = _A_and_deg(g)
    y = np.random.default_rng(1).random(g.n)
    got = oracle.block_gs_sweep(g, ALPHA, [0, g.n], y, fresh)
    np.testing.assert_allclose(got, (1 - ALPHA) / d * (A.T @ y), rtol=1e-14, atol=1e-17)


@pytest.mark.parametrize("fresh", [False, True])
def test_row_chunks_are_sequential_gauss_seidel(fresh):
    """lo = 0..n: (I - D L) y_new = D (U + fresh L) y_old with L / U the parts
    of A^T below / on-and-above the diagonal and D = (1-alpha)/d."""
    g = synth.random_small(70, 0.07, 4, self_loops=True)
    A, d = _A_and_deg(g)
    M = A.T
    L = np.tril(M, -1)
    U = M - L
    D = np.diag((1 - ALPHA) / d)
    y = np.random.default_rng(2).random(g.n)
    rhs = D @ ((U + (L if fresh else 0)) @ y)
    want = scipy.linalg.solve_triangular(np.eye(g.n) - D @ L, rhs, lower=True)
    got = oracle.block_gs_sweep(g, ALPHA, np.arange(g.n + 1), y, fresh)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-16)


def _push_scan(g, lo, r0, sweeps):
    """Algorithm 3's in-place scan in push form (Section 3.2 pushes), one chunk
    at a time: first every node pushes its fresh residue r0 simultaneously,
    then per sweep and chunk every node of the chunk pushes what it has
    received since its last push.  Returns the amounts pushed per sweep."""
    n = g.n
    d = np.diff(g.row_ptr)
    r = np.zeros(n)
    for v in range(n):                      # the fresh push at the start
        for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
            r[g.col[e]] += (1 - ALPHA) * r0[v] / d[v]
    out = []
    for _ in range(sweeps):
        pushed = np.zeros(n)
        for j in range(len(lo) - 1):
            x = {v: r[v] for v in range(lo[j], lo[j + 1])}
            for v in range(lo[j], lo[j + 1]):
                r[v] = 0.0
            for v in range(lo[j], lo[j + 1]):
                pushed[v] = x[v]
                for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
                    r[g.col[e]] += (1 - ALPHA) * x[v] / d[v]
        out.append(pushed)
    return out


@pytest.mark.parametrize("chunks", [1, 2, 5])
def test_block_gs_equals_chunked_push_scan(chunks):
    g = synth.random_small(40, 0.12, 6, self_loops=True)
    d = np.diff(g.row_ptr).astype(np.float64)
    lo = oracle.chunk_bounds(g, chunks)
    r0 = np.random.default_rng(3).random(g.n)
    pushes = _push_scan(g, lo, r0, 3)
    y = (1 - ALPHA) * r0 / d
    for k in range(3):
        y = oracle.block_gs_sweep(g, ALPHA, lo, y, fresh=(k == 0))
        np.testing.assert_allclose(y, (1 - ALPHA) * pushes[k] / d, rtol=1e-12, atol=1e-17)


@pytest.mark.parametrize("chunks", [1, 3, 7])
def test_iterated_sweeps_converge_and_contract(chunks):
    """S = y0 + y1 + ... (reserve in the y domain, pi_hat = alpha d S / (1-alpha))
    converges to pi_s; the exact residual (the certificate) falls by at least
    1 - alpha per sweep, and by exactly 1 - alpha for one chunk."""
    g = synth.random_small(120, 0.05, 8)
    s = 3
    x = dense_ppr(g, s, ALPHA)
    d = np.diff(g.row_ptr).astype(np.float64)
    lo = oracle.chunk_bounds(g, chunks)
    y = np.zeros(g.n)
    y[s] = (1 - ALPHA) / d[s]
    S = y.copy()
    prev = oracle.certificate(g, s, ALPHA, ALPHA * d * S / (1 - ALPHA))
    assert prev == pytest.approx(1 - ALPHA, rel=1e-12)
    for k in range(160):
        y = oracle.block_gs_sweep(g, ALPHA, lo, y, fresh=(k == 0))
        S += y
        cert = oracle.certificate(g, s, ALPHA, ALPHA * d * S / (1 - ALPHA))
        if prev > 1e-13:
            assert cert <= (1 - ALPHA) * prev * (1 + 1e-9) + 1e-15, (k, cert, prev)
            if chunks == 1:
                assert cert == pytest.approx((1 - ALPHA) * prev, rel=1e-8)
        prev = cert
    assert np.abs(ALPHA * d * S / (1 - ALPHA) - x).sum() <= 1e-12


def test_chunk_bounds_definition():
    g = synth.chunglu(5000, 60000, 2.1)
    col_ptr, _, _ = oracle.csc(g)
    for G in (1, 2, 7, 16):
        lo = oracle.chunk_bounds(g, G)
        assert lo[0] == 0 and lo[-1] == g.n and np.all(np.diff(lo) >= 0)
        for j in range(1, G):
            want = g.m * j // G
            assert col_ptr[lo[j]] >= want
            assert lo[j] == 0 or col_ptr[lo[j] - 1] < want


def test_sor_with_omega_one_is_the_plain_sweep():
    g = synth.random_small(80, 0.06, 12, self_loops=True)
    lo = oracle.chunk_bounds(g, 3)
    rng = np.random.default_rng(4)
    y = rng.random(g.n)
    q = rng.random(g.n) * 0.1
    for fresh in (False, True):
        ys, qs = oracle.block_sor_sweep(g, ALPHA, lo, y, fresh, 1.0, np.zeros(g.n))
        np.testing.assert_array_equal(ys, oracle.block_gs_sweep(g, ALPHA, lo, y, fresh))
        assert not qs.any()
        # one chunk, a kept residue q: every row sees the previous sweep only,
        # so y = q + the Eq. 7 value and nothing is kept
        ys, qs = oracle.block_sor_sweep(g, ALPHA, [0, g.n], y, fresh, 1.0, q)
        np.testing.assert_allclose(ys, q + oracle.block_gs_sweep(g, ALPHA, [0, g.n], y, fresh), rtol=1e-14)
        assert not qs.any()


@pytest.mark.parametrize("chunks,omega", [(1, 1.05), (4, 1.2), (9, 1.3)])
def test_sor_increments_equal_reserve_domain_sor(chunks, omega):
    """Accumulating the over-relaxed sweeps' pushes (S = sum of y) reproduces
    successive over-relaxation of the block Gauss-Seidel iteration written in
    the reserve domain with numpy (S(u) <- (1 - omega) S(u) + omega (1-alpha)/d_u
    (e_s(u) + sum_{v in N_in(u)} S(v)), earlier chunks already updated), which
    converges to the dense-solve PPR."""
    g = synth.random_small(90, 0.05, 13)
    A, d = _A_and_deg(g)
    s = 4
    sc = (1 - ALPHA) / d
    lo = oracle.chunk_bounds(g, chunks)
    e = np.zeros(g.n)
    e[s] = 1.0
    y = sc * e                              # the fresh residue: e_s in the y domain
    S = y.copy()                            # pushed at the start of the first sweep
    q = np.zeros(g.n)
    R = y.copy()                            # reserve-domain iterate after the same start
    for k in range(40):
        y, q = oracle.block_sor_sweep(g, ALPHA, lo, y, k == 0, omega, q)
        S += y
        Rn = R.copy()
        for j in range(len(lo) - 1):
            a, b = lo[j], lo[j + 1]
            gs = sc[a:b] * (e[a:b] + A.T[a:b] @ Rn)
            Rn[a:b] = (1 - omega) * R[a:b] + omega * gs
        R = Rn
        np.testing.assert_allclose(S, R, rtol=1e-11, atol=1e-15)
    for k in range(40, 400):
        y, q = oracle.block_sor_sweep(g, ALPHA, lo, y, False, omega, q)
        S += y
    x = dense_ppr(g, s, ALPHA)
    assert np.abs(ALPHA * d * S / (1 - ALPHA) - x).sum() <= 1e-11
