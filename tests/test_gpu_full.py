"""Parity at full size: the n = 4,000,000 / m = 70,000,000 Chung-Lu graph,
alpha = 0.2, lambda = 1e-8, 128 seeded sources answered in one batched call
with device outputs (the configuration the benchmark times).

The oracle cannot afford a converged power iteration per source at this
size, so the checks are ones that hold at any size:
- the CSC built on the device equals the oracle's counting-sort CSC bit for
  bit;
- the oracle's FP64 certificate of the exported vector (Eq. 1 rearranged:
  ||pi_hat - pi_s||_1 <= ||e_s - pi_hat (I - (1-alpha) P) / alpha||_1) is
  <= lambda on sampled columns, and equals the library's certificate;
- mass: sum(pi_s) = 1, so |sum(pi_hat) - 1| <= lambda for every column;
- one source in full: the FP64 path equals the oracle's level-synchronous
  schedule element by element (rtol 1e-11), with the same local levels and
  sweeps, and the batched mixed column lies within 2 lambda + 1e-9 of it
  (both are within lambda of pi_s).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2101_03652_amd")

pytestmark = pytest.mark.gpu
ALPHA = 0.2
LAM = 1e-8
N, M = 4_000_000, 70_000_000


@pytest.fixture(scope="module")
def c2():
    print("[gpu] full-size graph n=4M m=70M", flush=True)
    return synth.chunglu(N, M, 2.1)


@pytest.fixture(scope="module")
def G(c2):
    g = P.Graph.from_synth(c2)
    yield g
    g.close()


@pytest.fixture(scope="module")
def srcs(c2):
    return [int(s) for s in synth.sources(c2.n, 128)]


@pytest.fixture(scope="module")
def sync0(c2, srcs):
    print("[gpu] oracle level-synchronous schedule, source 0", flush=True)
    pi, r, st, trace, levels = oracle.powerpush_sync(c2, srcs[0], ALPHA, LAM, oracle.SWITCH_EDGES,
                                                     P.options().switch_param)
    return pi, st


def test_full_csc_bit_exact(c2, G):
    cp, ri, dg = G.csc()
    ocp, ori, odg = oracle.csc(c2)
    assert np.array_equal(cp, ocp)
    assert np.array_equal(ri, ori)
    assert np.array_equal(dg, odg)


@pytest.mark.parametrize("width", [0, 32, 128])
def test_full_batched_certified(c2, G, srcs, width):
    """width 0: the autotuned width, as the benchmark runs it."""
    if width == 0:
        width = G.autotune(alpha=ALPHA)["best"]
    print(f"[gpu] full-size batched width={width}", flush=True)
    out = torch.empty((len(srcs), c2.n), dtype=torch.float64, device="cuda")
    _, st = G.query_batch(srcs, ALPHA, LAM, P.MIXED, out=out, batch_cols=width)
    host = out.cpu().numpy()
    sums = host.sum(axis=1)
    assert np.all(np.abs(sums - 1.0) <= LAM), np.abs(sums - 1.0).max()
    assert all(s["cert_l1"] <= LAM for s in st)
    assert [s["source"] for s in st] == srcs
    assert host.min() >= -1e-15
    for b in (0, 1, 37, 64, 101, 127):
        cert = oracle.certificate(c2, srcs[b], ALPHA, host[b])
        assert cert <= LAM * (1 + 1e-6), (b, cert)
        assert st[b]["cert_l1"] == pytest.approx(cert, rel=1e-6, abs=1e-15)


def test_full_fp64_matches_oracle_sync(c2, G, srcs, sync0):
    print("[gpu] full-size FP64 vs oracle sync", flush=True)
    opi, ost = sync0
    out = torch.empty(c2.n, dtype=torch.float64, device="cuda")
    _, st = G.query(srcs[0], ALPHA, LAM, P.FP64, out=out, certify=1)
    pi = out.cpu().numpy()
    assert st["local_levels"] == ost["local_levels"]
    assert st["sweeps"] == ost["sweeps"]
    assert st["edge_pushes"] == ost["edge_pushes"]
    np.testing.assert_allclose(pi, opi, rtol=1e-11, atol=1e-20)
    assert st["cert_l1"] <= LAM
    assert oracle.certificate(c2, srcs[0], ALPHA, pi) <= LAM * (1 + 1e-9)


def test_full_mixed_column_near_oracle_sync(c2, G, srcs, sync0):
    opi, _ = sync0
    out, st = G.query_batch(srcs[:4], ALPHA, LAM, P.MIXED, batch_cols=4)
    assert np.abs(out[0] - opi).sum() <= 2 * LAM + 1e-9
