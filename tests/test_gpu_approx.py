"""Approximate SSPPR (SpeedPPR, Section 6, Algorithm 4) on the GPU against the
oracle: the walk index bit for bit (integer work), the refinement element
by element (FP64, same levels and residue updates), the Monte Carlo phase
on the same residue (the same walks, so the same estimate up to FP64
summation order), and the whole query against the truth within the
relative error eps of the Approx-SSPPR definition (Section 2)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2101_03652_amd")

pytestmark = pytest.mark.gpu
ALPHA = 0.2


@pytest.fixture(scope="module")
def graphs():
    from test_gpu_fp64 import _hub_graph
    return {"c1": synth.chunglu(10_000, 100_000, 2.1), "hub": _hub_graph()}


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("name", ["c1", "hub"])
def test_walk_index_bit_exact(graphs, name):
    """Every entry of the index (walk j from v for j < d_v) equals the oracle's
    walk with the same seed, node and index."""
    g = graphs[name]
    print(f"[gpu] walk index {name} m={g.m}", flush=True)
    G = P.Graph.from_synth(g)
    G.build_walk_index(ALPHA, seed=7)
    idx = G.walk_index()
    rp = g.row_ptr
    want = np.empty(g.m, dtype=np.int32)
    for v in range(g.n):
        for j in range(int(rp[v + 1] - rp[v])):
            want[rp[v] + j] = oracle.walk_endpoint(g, ALPHA, 7, v, j)
    np.testing.assert_array_equal(idx, want)
    G.close()


def _pushed_state(g, s, lam):
    pi, r, _, _ = oracle.powerpush(g, s, ALPHA, lam)
    return pi, r


@pytest.mark.parametrize("name,rmax,slices", [("c1", 1e-7, 0), ("c1", 1e-9, 0), ("hub", 1e-8, 0),
                                               ("c1", 1e-9, 4), ("hub", 1e-8, 3)])
def test_refinement_matches_oracle(graphs, name, rmax, slices):
    """slices > 1: the refinement's pull levels sweep over source slices."""
    g = graphs[name]
    print(f"[gpu] refinement {name} rmax={rmax} slices={slices}", flush=True)
    G = P.Graph.from_synth(g, fp64_slices=slices)
    pi0, r0 = _pushed_state(g, 3, 0.05)
    pi_d, r_d = _dev(pi0), _dev(r0)
    levels, ep = G.debug_refine(ALPHA, rmax, pi_d, r_d)
    pio, ro = pi0.copy(), r0.copy()
    lvo, epo = oracle.refine_sync(g, ALPHA, rmax, pio, ro)
    assert (levels, ep) == (lvo, epo)
    np.testing.assert_allclose(pi_d.cpu().numpy(), pio, rtol=1e-11, atol=1e-20)
    np.testing.assert_allclose(r_d.cpu().numpy(), ro, rtol=1e-11, atol=1e-20)
    d = np.diff(g.row_ptr).astype(np.float64)
    assert not np.any(r_d.cpu().numpy() > d * rmax)
    G.close()


@pytest.mark.parametrize("name,W", [("c1", 3e5), ("c1", 2e7), ("hub", 1e6)])
def test_walk_phase_matches_oracle(graphs, name, W):
    """The Monte Carlo phase on the same refined residue: the same number of
    walks, the same stop nodes, so the estimate agrees to FP64 summation
    order; read from the index it is the same again."""
    g = graphs[name]
    print(f"[gpu] walk phase {name} W={W:g}", flush=True)
    G = P.Graph.from_synth(g)
    pi0, r0 = _pushed_state(g, 5, min(g.m / W, 1.0))
    oracle.refine_sync(g, ALPHA, 1.0 / W, pi0, r0)
    d = np.diff(g.row_ptr)
    assert np.all(np.ceil(r0 * W) <= d)
    pio = pi0.copy()
    nwo = oracle.mc_phase(g, ALPHA, W, 99, r0, pio)
    pi_d = _dev(pi0)
    nw = G.debug_walks(ALPHA, W, 99, _dev(r0), pi_d)
    assert nw == nwo
    got = pi_d.cpu().numpy()
    np.testing.assert_allclose(got, pio, rtol=1e-12, atol=1e-300)
    G.build_walk_index(ALPHA, seed=99)
    pi_i = _dev(pi0)
    assert G.debug_walks(ALPHA, W, 99, _dev(r0), pi_i, use_index=True) == nw
    np.testing.assert_allclose(pi_i.cpu().numpy(), got, rtol=1e-13, atol=1e-300)
    G.close()


@pytest.mark.parametrize("eps", [0.5, 0.2])
def test_speedppr_query_within_eps(graphs, eps):
    """Every node with pi >= mu = 1/n within relative error eps of the
    power-iteration truth; the walk budget is Eq. 8's; at most m walks."""
    g = graphs["c1"]
    G = P.Graph.from_synth(g)
    for s in [int(x) for x in synth.sources(g.n, 3)]:
        print(f"[gpu] speedppr c1 s={s} eps={eps}", flush=True)
        pi, st = G.query_approx(s, ALPHA, eps, seed=11)
        assert st["W"] == pytest.approx(oracle.walk_budget(g.n, eps, 1.0 / g.n), rel=1e-14)
        assert st["lambda"] == pytest.approx(min(g.m / st["W"], 1.0), rel=1e-14)
        assert 0 < st["walks"] <= g.m
        truth = oracle.powitr(g, s, ALPHA, 135)
        big = truth >= 1.0 / g.n
        rel = np.abs(pi[big] - truth[big]) / truth[big]
        assert rel.max() <= eps, (s, rel.max())
        assert abs(pi.sum() - 1.0) <= 1e-9
    G.close()


def test_speedppr_index_gives_the_same_answer(graphs):
    g = graphs["c1"]
    G = P.Graph.from_synth(g)
    s = int(synth.sources(g.n, 1)[0])
    a, sa = G.query_approx(s, ALPHA, 0.3, seed=5)
    with pytest.raises(P.PPRError):                    # no index yet
        G.query_approx(s, ALPHA, 0.3, seed=5, use_index=True)
    G.build_walk_index(ALPHA, seed=5)
    b, sb = G.query_approx(s, ALPHA, 0.3, seed=5, use_index=True)
    assert sb["used_index"] == 1 and sb["walks"] == sa["walks"]
    np.testing.assert_allclose(b, a, rtol=1e-13, atol=1e-300)
    with pytest.raises(P.PPRError):                    # built for another seed
        G.query_approx(s, ALPHA, 0.3, seed=6, use_index=True)
    with pytest.raises(P.PPRError):
        G.query_approx(s, ALPHA, 0.0, seed=5)
    with pytest.raises(P.PPRError):
        G.query_approx(s, ALPHA, 0.3, mu=0.0, seed=5)
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    G.query_approx(s, ALPHA, 0.3, seed=5, out=out)
    np.testing.assert_allclose(out.cpu().numpy(), a, rtol=1e-13, atol=1e-300)
    G.close()
