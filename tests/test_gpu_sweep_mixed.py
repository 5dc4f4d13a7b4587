"""The batched mixed path's global sweep against the oracle, element by
element: one block Gauss-Seidel sweep (Eq. 7 for one chunk) on FP32 inputs,
computed by the library in FP32 and by the oracle in FP64 from the same
FP32 values, every column (fresh and continuing ones mixed), widths 4..128,
1..8 row chunks, long rows cut into pieces (the hub graph), every row tile.

Three checks, from exact to semantic:
- exact: with dyadic inputs (small integers times 2^-20, bf16-representable)
  every FP32 row sum is exact in any order, so one Eq. 7 sweep must equal,
  bit for bit, the FP32 product of the FP32 scale (1 - alpha) / d_u and the
  exact sum (then rounded to bf16 in bf16 storage).  A dropped or doubled
  in-edge anywhere (a round seam, a piece seam, a tile) changes the sum by at
  least one unit and fails.  A seam graph puts rows at in-degrees on both
  sides of every round and piece boundary of every tile and width.
- own inputs: each row against the oracle's Eq. 7 sweep of exactly the values
  that row pulls (the library's stored outputs of earlier chunks, plus the
  fresh residue rounded as stored, and y_in for the rest).  Only the row's
  own FP32 summation and the final product differ: at most (h + 3) u times
  the sum of the terms' magnitudes, h the depth of the row's summation in the
  sweep block (a lane's chain of ceil(min(d, piece) / T2) + rounds terms, a
  log2 T2 shuffle tree, the pieces added in order; h <= d + 6 for a row that
  fits one round); in bf16 the stored value must be the rounding of a value
  in that interval.
- semantics: against the oracle's block Gauss-Seidel sweep run from y_in
  alone, where rows also inherit the rounding of earlier chunks' outputs:
  (d_in(u) + max_in + 3) u relative (non-negative inputs).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2101_03652_amd")

pytestmark = pytest.mark.gpu
ALPHA = 0.2
U = 2.0 ** -24


TILES = (12288, 16384, 24576)


def _vectors(B, bf16):
    """16-byte vectors per row: 4 FP32 or 8 bf16 columns."""
    return B // (8 if bf16 else 4)


def _seam_degrees():
    """In-degrees on both sides of every round (kNnz in-edges) and piece
    (8 rounds) boundary of every tile and vector count, and past several
    pieces."""
    ds = set()
    for C in (1, 2, 4, 8, 16, 32):
        for L in TILES:
            k = L // (16 * C)
            pc = 8 * k
            ds.update({k - 1, k, k + 1, pc - 1, pc, pc + 1, 2 * pc, 2 * pc + 1, 3 * pc + 5})
    return sorted(d for d in ds if d >= 1)


def _seam_graph():
    """Rows 0.. get the in-degrees of _seam_degrees (distinct random
    sources); every node also gets one out-edge into the filler rows."""
    rng = np.random.default_rng(11)
    degs = _seam_degrees()
    n = max(degs) + 64
    edges = set()
    for u, d in enumerate(degs):
        for v in rng.choice(np.setdiff1d(np.arange(n), [u]), size=d, replace=False):
            edges.add((int(v), u))
    fill = np.arange(len(degs), n)
    for v in range(n):
        w = int(fill[rng.integers(0, len(fill))])
        if w != v:
            edges.add((v, w))
        else:
            edges.add((v, int(fill[0]) if w != fill[0] else int(fill[1])))
    return synth.from_edges(n, sorted(edges), "seam")


def _graphs():
    from test_gpu_fp64 import _hub_graph
    return {"c1": synth.chunglu(10_000, 100_000, 2.1), "hub": _hub_graph(), "seam": _seam_graph()}


def _depth(din, B, bf16, tile):
    """Bound on the additions a term of row u undergoes in the sweep block
    (see the module docstring)."""
    C = _vectors(B, bf16)
    knnz = tile // (16 * C)
    pc = 8 * knnz
    t2 = min(64, 256 // C)
    lg = int(np.log2(t2))
    din = din.astype(np.float64)
    long_chain = np.ceil(np.minimum(din, pc) / t2) + 8 + lg
    pieces = np.where(din > pc, np.ceil(din / pc), 0.0)
    return np.where(din <= knnz, din + 6, long_chain + pieces)


def _own_input_ref(g, csc_arrays, lo, yin, got, fresh, bf16):
    """Per row u of chunk j, the oracle's Eq. 7 sweep of the values the row
    pulls: got(v) for v in earlier chunks (plus yin(v), added in FP32 and
    stored as the block stores, for a fresh column), yin(v) otherwise.
    Returns (value, the same sweep of the terms' magnitudes)."""
    n = g.n
    ids = np.arange(n)
    early_val = got
    if fresh:
        early_val = np.float32(got) + np.float32(yin)
        if bf16:
            early_val = _bf16(early_val)
    want = np.zeros(n)
    mag = np.zeros(n)
    one = np.array([0, n], dtype=np.int32)
    for j in range(len(lo) - 1):
        a, b = int(lo[j]), int(lo[j + 1])
        if a == b:
            continue
        ymix = np.where(ids < a, early_val, yin).astype(np.float64)
        want[a:b] = oracle.block_gs_sweep(g, ALPHA, one, ymix, False, csc_arrays=csc_arrays)[a:b]
        mag[a:b] = oracle.block_gs_sweep(g, ALPHA, one, np.abs(ymix), False, csc_arrays=csc_arrays)[a:b]
    return want, mag


def _assert_own_inputs(g, csc_arrays, lo, yin, got, fresh, B, bf16, tile, omega=None, where=""):
    """got (one column) against its own-input reference; omega: over-relaxed
    (the row pushes omega * value + (1 - omega) * yin(u) unless fresh)."""
    want, mag = _own_input_ref(g, csc_arrays, lo, yin, got, fresh, bf16)
    din = np.diff(csc_arrays[0])
    tol = (_depth(din, B, bf16, tile) + 3) * U
    if omega is not None and omega != 1.0:
        k = 0.0 if fresh else (1.0 - omega)
        want = omega * want + k * yin.astype(np.float64)
        mag = abs(omega) * mag + abs(k) * np.abs(yin.astype(np.float64))
        tol = tol + 3 * U
    if not bf16:
        err = np.abs(got.astype(np.float64) - want)
        bad = err > tol * mag + 1e-38
        assert not bad.any(), (where, int(np.argmax(err - tol * mag)), int(bad.sum()))
    else:
        lo_b = _bf16(np.float32(want - tol * mag)).astype(np.float64)
        hi_b = _bf16(np.float32(want + tol * mag)).astype(np.float64)
        g64 = got.astype(np.float64)
        bad = (g64 < lo_b) | (g64 > hi_b)
        assert not bad.any(), (where, int(np.argmax(bad)), int(bad.sum()))


@pytest.fixture(scope="module")
def graphs():
    return _graphs()


@pytest.mark.parametrize("name", ["c1", "hub", "hub-wide", "seam"])
@pytest.mark.parametrize("width,chunks", [(4, 1), (4, 5), (32, 1), (32, 3), (32, 8), (128, 1), (128, 4)])
def test_sweep_matches_oracle(graphs, name, width, chunks):
    """hub-wide: the hub graph with int64 device CSC offsets."""
    g = graphs[name.split("-")[0]]
    print(f"[gpu] batched sweep parity {name} width={width} chunks={chunks}", flush=True)
    G = P.Graph.from_synth(g, wide_offsets=name.endswith("wide"))
    rng = np.random.default_rng(width * 100 + chunks)
    y = rng.random((g.n, width)).astype(np.float32)
    y[rng.random((g.n, width)) < 0.3] = 0.0             # sparse residues
    fresh = (rng.random(width) < 0.5).astype(np.int32)
    fresh[0], fresh[-1] = 1, 0
    t_out = np.empty_like(y)
    got = P.debug_sweep_mixed(G, ALPHA, y, fresh, chunks=chunks, t_out=t_out)
    csc_arrays = oracle.csc(g)
    col_ptr = csc_arrays[0]
    din = np.diff(col_ptr).astype(np.float64)
    lo = oracle.chunk_bounds(g, chunks)
    tol_rel = (din + din.max() + 3) * U
    for b in range(width):
        want = oracle.block_gs_sweep(g, ALPHA, lo, y[:, b].astype(np.float64), bool(fresh[b]),
                                     csc_arrays=csc_arrays)
        err = np.abs(got[:, b] - want)
        assert np.all(err <= tol_rel * want + 1e-38), (b, int(np.argmax(err - tol_rel * want)))
        _assert_own_inputs(g, csc_arrays, lo, y[:, b], got[:, b], bool(fresh[b]), width, False, 16384, where=b)
        # stage accumulator: the stored new residue, plus the fresh residue (FP32 add)
        t_want = (y[:, b] if fresh[b] else np.zeros(g.n, np.float32)) + got[:, b]
        np.testing.assert_array_equal(t_out[:, b], t_want.astype(np.float32))
    G.close()


@pytest.fixture(scope="module")
def devgraphs(graphs):
    gs = {k: P.Graph.from_synth(v) for k, v in graphs.items()}
    yield gs
    for G in gs.values():
        G.close()


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("name", ["c1", "hub", "seam"])
@pytest.mark.parametrize("width,fmt", [(4, "f32"), (8, "f32"), (32, "f32"), (128, "f32"),
                                       (8, "bf16"), (32, "bf16"), (128, "bf16")])
def test_dyadic_sweep_bit_exact(graphs, devgraphs, tile, name, width, fmt):
    """One Eq. 7 sweep (one chunk) on dyadic residues k 2^-20, k in [1, 255]
    (bf16-representable; every row sum below 2^24 units, so exact in FP32 in
    any order): the stored output is exactly fl32(fl32((1 - alpha) / d_u) *
    sum), rounded to bf16 in bf16 storage, and the stage accumulator exactly
    the stored value plus the fresh residue.  One dropped or doubled in-edge
    changes a row sum by at least one unit (a relative change of at least
    2^-22 here, or 1/255 of a bf16-scale term for the sparse columns) and
    fails."""
    g = graphs[name]
    G = devgraphs[name]
    bf16 = fmt == "bf16"
    print(f"[gpu] dyadic sweep {name} width={width} tile={tile} {fmt}", flush=True)
    rng = np.random.default_rng(tile + 3 * width + (1 if bf16 else 0))
    k = rng.integers(1, 256, size=(g.n, width)).astype(np.float64)
    # sparse columns: a dropped term moves a bf16 output too
    for b in range(1, width, 2):
        keep = rng.random(g.n) < 0.01
        k[~keep, b] = 0.0
        k[keep, b] = rng.integers(128, 256, size=int(keep.sum()))
    y = (k * 2.0 ** -20).astype(np.float32)
    fresh = (rng.random(width) < 0.5).astype(np.int32)
    t_out = np.empty_like(y)
    got = P.debug_sweeps_mixed(G, ALPHA, y, fresh, 1, chunks=1, t_out=t_out, sweep_tile=tile,
                               residue_format=P.RESIDUE_BF16 if bf16 else P.RESIDUE_F32)
    col_ptr, row_idx, deg = oracle.csc(g)
    assert np.diff(col_ptr).max() * 255 < 2 ** 24
    # exact row sums (float64 holds them exactly), per column
    rows = np.repeat(np.arange(g.n), np.diff(col_ptr))
    S = np.zeros((g.n, width))
    np.add.at(S, rows, y[row_idx].astype(np.float64))
    sc = np.float32((1.0 - ALPHA) / deg.astype(np.float64)).astype(np.float64)
    want = np.float32(sc[:, None] * S)          # one rounding of an exact product
    if bf16:
        want = _bf16(want)
    np.testing.assert_array_equal(got, want)
    t_want = np.where(fresh[None, :] != 0, y, np.float32(0.0)) + want
    np.testing.assert_array_equal(t_out, t_want.astype(np.float32))


def test_sweep_device_buffers_and_errors(graphs):
    g = graphs["c1"]
    G = P.Graph.from_synth(g)
    y = torch.rand((g.n, 8), dtype=torch.float32, device="cuda")
    got = P.debug_sweep_mixed(G, ALPHA, y, [1] * 8, chunks=2)
    host = P.debug_sweep_mixed(G, ALPHA, y.cpu().numpy(), [1] * 8, chunks=2)
    assert np.array_equal(got.cpu().numpy(), host)          # same kernels, same order
    with pytest.raises(P.PPRError):
        P.debug_sweep_mixed(G, ALPHA, np.zeros((g.n, 6), np.float32), [0] * 6)
    with pytest.raises(P.PPRError):
        P.debug_sweep_mixed(G, ALPHA, np.zeros((g.n, 8), np.float32), [0] * 8, chunks=0)
    G.close()


@pytest.mark.parametrize("name", ["c1", "hub"])
@pytest.mark.parametrize("width,chunks", [(4, 3), (32, 4), (128, 8)])
def test_over_relaxed_sweep_matches_oracle(graphs, name, width, chunks):
    """The over-relaxed sweep against the oracle's, per column: omega between
    1 and 1.3 (some exactly 1), fresh and continuing columns.  The kernel keeps
    no separate kept-back residue: a continuing row kept (1 - omega) / omega
    times what it pushed last (y_in), a fresh one nothing; the oracle is given
    that q explicitly.  q is negative for omega > 1, so the rounding bound is
    taken relative to the same recursion run on absolute values."""
    g = graphs[name]
    print(f"[gpu] over-relaxed sweep parity {name} width={width} chunks={chunks}", flush=True)
    G = P.Graph.from_synth(g)
    rng = np.random.default_rng(width * 7 + chunks)
    y = rng.random((g.n, width)).astype(np.float32)
    y[rng.random((g.n, width)) < 0.3] = 0.0
    fresh = (rng.random(width) < 0.5).astype(np.int32)
    om = (1.0 + 0.3 * rng.random(width)).astype(np.float32)
    om[0] = 1.0
    got = P.debug_sweep_mixed(G, ALPHA, y, fresh, chunks=chunks, omega=om)
    csc_arrays = oracle.csc(g)
    din = np.diff(csc_arrays[0]).astype(np.float64)
    lo = oracle.chunk_bounds(g, chunks)
    tol_rel = (din + din.max() + 6) * U
    for b in range(width):
        w = float(om[b])
        yb = y[:, b].astype(np.float64)
        qb = np.zeros(g.n) if fresh[b] else (1.0 - w) / w * yb
        want_y, want_q = oracle.block_sor_sweep(g, ALPHA, lo, yb, bool(fresh[b]), w, qb, csc_arrays=csc_arrays)
        mag_y, _ = oracle.block_sor_sweep(g, ALPHA, lo, yb, bool(fresh[b]), w, np.abs(qb), csc_arrays=csc_arrays)
        assert np.all(np.abs(got[:, b] - want_y) <= tol_rel * mag_y + 1e-38), b
        _assert_own_inputs(g, csc_arrays, lo, y[:, b], got[:, b], bool(fresh[b]), width, False, 16384, omega=w,
                           where=b)
        # what the row keeps is (1 - omega) / omega times what it pushes: the
        # next sweep's q, read back from y_out
        np.testing.assert_allclose(want_q, (1.0 - w) / w * want_y, rtol=1e-13, atol=1e-300)
    G.close()


def _bf16(x):
    """Round FP32 values to bf16 (nearest, ties to even), returned as FP32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


UB = 2.0 ** -8     # bf16 unit roundoff (8-bit significand)


@pytest.mark.parametrize("name", ["c1", "hub", "seam"])
@pytest.mark.parametrize("width,chunks,sor", [(8, 1, False), (8, 5, True), (32, 3, False), (128, 1, False),
                                              (128, 8, False), (32, 4, True), (128, 8, True)])
def test_bf16_sweep_matches_oracle(graphs, name, width, chunks, sor):
    """bf16 residue storage: the library rounds y_in to bf16, sweeps in FP32
    and stores every new residue as bf16; the oracle sweeps the same bf16
    inputs in FP64.  Every output is a bf16 value.  A row of chunk j reads the
    stored, rounded values of chunks < j, so by induction its value is within
    j + 1 bf16 roundings of the oracle's (relative to the same recursion on
    absolute values), plus the FP32 summation bound; a fresh column's row
    reads an earlier chunk's new value plus the fresh residue as one more
    rounded value (j + 2).  The stage accumulator holds exactly the stored
    values (plus the fresh input residue)."""
    g = graphs[name]
    print(f"[gpu] bf16 sweep parity {name} width={width} chunks={chunks} sor={sor}", flush=True)
    G = P.Graph.from_synth(g)
    rng = np.random.default_rng(width * 31 + chunks + (7 if sor else 0))
    y = rng.random((g.n, width)).astype(np.float32)
    y[rng.random((g.n, width)) < 0.3] = 0.0
    fresh = (rng.random(width) < 0.5).astype(np.int32)
    fresh[0], fresh[-1] = 1, 0
    om = None
    if sor:
        om = (1.0 + 0.3 * rng.random(width)).astype(np.float32)
        om[1] = 1.0
    t_out = np.empty_like(y)
    got = P.debug_sweep_mixed(G, ALPHA, y, fresh, chunks=chunks, t_out=t_out, omega=om,
                              residue_format=P.RESIDUE_BF16)
    assert not np.any(got.view(np.uint32) & 0xFFFF)                 # bf16 values
    yb = _bf16(y)
    csc_arrays = oracle.csc(g)
    din = np.diff(csc_arrays[0]).astype(np.float64)
    lo = oracle.chunk_bounds(g, chunks)
    chunk_of = np.searchsorted(lo, np.arange(g.n), side="right") - 1        # row -> its chunk j
    for b in range(width):
        rounds = chunk_of + 1 + (1 if fresh[b] else 0) * (chunk_of > 0)
        rel = (1.0 + UB) ** rounds - 1.0 + (din + din.max() + 6) * U
        yb_b = yb[:, b].astype(np.float64)
        if sor:
            w = float(om[b])
            q = np.zeros(g.n) if fresh[b] else (1.0 - w) / w * yb_b
            want, _ = oracle.block_sor_sweep(g, ALPHA, lo, yb_b, bool(fresh[b]), w, q, csc_arrays=csc_arrays)
            mag, _ = oracle.block_sor_sweep(g, ALPHA, lo, yb_b, bool(fresh[b]), w, np.abs(q), csc_arrays=csc_arrays)
        else:
            want = oracle.block_gs_sweep(g, ALPHA, lo, yb_b, bool(fresh[b]), csc_arrays=csc_arrays)
            mag = want
        err = np.abs(got[:, b] - want)
        assert np.all(err <= rel * mag + 1e-38), (b, int(np.argmax(err - rel * mag)))
        _assert_own_inputs(g, csc_arrays, lo, yb[:, b], got[:, b], bool(fresh[b]), width, True, 16384,
                           omega=float(om[b]) if sor else None, where=b)
        # T = (fresh input residue) + the stored value, in FP32
        t_want = (yb[:, b] if fresh[b] else np.zeros(g.n, np.float32)) + got[:, b]
        np.testing.assert_array_equal(t_out[:, b], t_want.astype(np.float32))
    G.close()


def test_bf16_device_buffers_and_errors(graphs):
    """Device and host buffers give the same bits; an unknown format is
    refused."""
    g = graphs["c1"]
    G = P.Graph.from_synth(g)
    y = torch.rand((g.n, 8), dtype=torch.float32, device="cuda")
    a = P.debug_sweep_mixed(G, ALPHA, y, [1] * 8, chunks=2, residue_format=P.RESIDUE_BF16)
    h = P.debug_sweep_mixed(G, ALPHA, y.cpu().numpy(), [1] * 8, chunks=2, residue_format=P.RESIDUE_BF16)
    assert np.array_equal(a.cpu().numpy(), h)
    with pytest.raises(P.PPRError):
        P.debug_sweep_mixed(G, ALPHA, y, [1] * 8, residue_format=5)
    with pytest.raises(P.PPRError):                      # bf16 vectors hold 8 columns
        P.debug_sweep_mixed(G, ALPHA, y[:, :4].contiguous(), [1] * 4, residue_format=P.RESIDUE_BF16)
    G.close()


def _sequence_by_single_sweeps(G, y, entry, budget, sweeps, chunks, om, fmt):
    """The stored residues y_0 (input as stored), y_1, .., y_sweeps of a
    sequence, produced one sweep at a time by the single-sweep entry point
    (fresh only on the first), a column set to 0 after its budget."""
    ys = []
    cur = y
    for k in range(sweeps):
        fr = (entry != 0).astype(np.int32) if k == 0 else np.zeros_like(entry)
        nxt = P.debug_sweep_mixed(G, ALPHA, cur, fr, chunks=chunks, omega=om, residue_format=fmt)
        nxt[:, budget <= k] = 0.0
        ys.append(nxt)
        cur = nxt
    y0 = _bf16(y) if fmt == P.RESIDUE_BF16 else y
    return [y0] + ys


@pytest.mark.parametrize("name", ["c1", "hub"])
@pytest.mark.parametrize("width,chunks,sweeps,sor,fmt", [
    (8, 3, 1, False, 0), (8, 3, 2, False, 0), (32, 4, 5, False, 0), (32, 4, 4, True, 0), (16, 1, 3, True, 0),
    (128, 8, 5, True, 1), (128, 8, 6, False, 1), (8, 2, 7, True, 1)])
def test_sweep_sequence_stage_accumulator(graphs, name, width, chunks, sweeps, sor, fmt):
    """A launch sequence of several sweeps with per-column budgets and the
    three entry kinds (continuing, fresh, fresh with the accumulator
    restarting).  The accumulator is updated by every second sweep, which
    adds its input and its output, and by the last sweep; whatever the
    pairing, it must hold t_in (unless restarting) + the fresh residue + every
    residue stored.  Checked two ways: (1) bit for bit against the same
    sweeps run one at a time through the single-sweep entry point, adding
    the stored values in the order the kernel adds them (FP32); (2) in FP32
    storage, against the oracle's block Gauss-Seidel (or over-relaxed) sweeps
    chained in FP64, within the one-sweep FP32 bound (module docstring)
    taken once per sweep."""
    g = graphs[name]
    print(f"[gpu] sweep sequence {name} width={width} chunks={chunks} sweeps={sweeps} sor={sor} fmt={fmt}",
          flush=True)
    G = P.Graph.from_synth(g)
    rng = np.random.default_rng(width * 13 + chunks * 5 + sweeps + (3 if sor else 0) + 97 * fmt)
    y = rng.random((g.n, width)).astype(np.float32)
    y[rng.random((g.n, width)) < 0.3] = 0.0
    t_in = rng.random((g.n, width)).astype(np.float32)
    entry = rng.integers(0, 3, width).astype(np.int32)
    entry[:3] = [0, 1, 2]
    budget = rng.integers(0, sweeps + 1, width).astype(np.int32)
    budget[:4] = sweeps
    budget[-1] = 0
    budget[-2] = max(sweeps - 1, 0)
    om = None
    if sor:
        om = (1.0 + 0.3 * rng.random(width)).astype(np.float32)
        om[0] = 1.0
    t_out = np.empty_like(y)
    got = P.debug_sweeps_mixed(G, ALPHA, y, entry, sweeps, budget=budget, t_in=t_in, chunks=chunks,
                               t_out=t_out, omega=om, residue_format=fmt)
    ys = _sequence_by_single_sweeps(G, y, entry, budget, sweeps, chunks, om, fmt)
    np.testing.assert_array_equal(got, ys[-1])
    # the accumulator, in the kernel's order of FP32 additions
    t = t_in.copy()
    t[:, entry == 2] = 0.0
    first = (entry != 0) & (budget > 0)
    t = t + np.where(first[None, :], ys[0], np.float32(0.0))
    for k in range(sweeps):
        if k % 2 == 1:
            t = (t + ys[k]) + ys[k + 1]
        elif k == sweeps - 1:
            t = t + ys[k + 1]
    np.testing.assert_array_equal(t_out, t)
    # every step of the sequence against the oracle on the values it pulled
    csc_arrays = oracle.csc(g)
    lo = oracle.chunk_bounds(g, chunks)
    for k in range(sweeps):
        for b in range(width):
            if budget[b] <= k:
                assert not ys[k + 1][:, b].any()
                continue
            w = float(om[b]) if sor else None
            fr = bool(entry[b]) and k == 0
            _assert_own_inputs(g, csc_arrays, lo, ys[k][:, b], ys[k + 1][:, b], fr, width, fmt == P.RESIDUE_BF16,
                               16384, omega=w, where=(k, b))
    if fmt == P.RESIDUE_F32:
        csc_arrays = oracle.csc(g)
        din = np.diff(csc_arrays[0]).astype(np.float64)
        lo = oracle.chunk_bounds(g, chunks)
        rel = sweeps * (2 * din.max() + 6) * U
        for b in range(width):
            w = float(om[b]) if sor else 1.0
            cur = y[:, b].astype(np.float64)
            q = np.zeros(g.n) if entry[b] else (1.0 - w) / w * cur
            mag, qm = cur.copy(), np.abs(q)
            t_want = (0.0 if entry[b] == 2 else t_in[:, b].astype(np.float64)) + (cur if first[b] else 0.0)
            t_mag = np.abs(t_want)
            for k in range(sweeps):
                fresh = bool(entry[b]) and k == 0
                if k >= budget[b]:
                    cur, q, mag, qm = (np.zeros(g.n),) * 4
                    break
                cur, q = oracle.block_sor_sweep(g, ALPHA, lo, cur, fresh, w, q, csc_arrays=csc_arrays)
                mag, qm = oracle.block_sor_sweep(g, ALPHA, lo, mag, fresh, w, qm, csc_arrays=csc_arrays)
                qm = np.abs(qm)                # the same recursion on absolute values
                t_want = t_want + cur
                t_mag = t_mag + mag
            assert np.all(np.abs(got[:, b] - cur) <= rel * mag + 1e-38), b
            assert np.all(np.abs(t_out[:, b] - t_want) <= (rel + (sweeps + 2) * U) * t_mag + 1e-38), b
    G.close()


def test_sweep_sequence_arguments(graphs):
    g = graphs["c1"]
    G = P.Graph.from_synth(g)
    y = np.zeros((g.n, 8), np.float32)
    for kw in ({"sweeps": 0}, {"sweeps": 65}, {"entry": [3] * 8}, {"budget": [5] * 8}, {"budget": [-1] * 8}):
        args = {"sweeps": 4, "entry": [0] * 8}
        args.update(kw)
        with pytest.raises(P.PPRError):
            P.debug_sweeps_mixed(G, ALPHA, y, args["entry"], args["sweeps"], budget=args.get("budget"))
    G.close()


@pytest.mark.parametrize("tile", [12288, 24576])
@pytest.mark.parametrize("name", ["c1", "hub", "seam"])
@pytest.mark.parametrize("width,chunks,fmt", [(32, 3, "f32"), (128, 4, "f32"), (32, 8, "bf16"), (128, 8, "bf16")])
def test_sweep_tiles_match_oracle(graphs, tile, name, width, chunks, fmt):
    """The row tiles the autotuner may pick (LDS stages of 12 and 24 KB; the
    16 KB default is the tile of the tests above) compute the same sweep:
    other in-edge counts per block, rows per block and long-row pieces, the
    same bounds as above."""
    g = graphs[name]
    print(f"[gpu] sweep tile parity tile={tile} {name} width={width} chunks={chunks} {fmt}", flush=True)
    G = P.Graph.from_synth(g)
    rng = np.random.default_rng(tile + width * 7 + chunks)
    y = rng.random((g.n, width)).astype(np.float32)
    y[rng.random((g.n, width)) < 0.3] = 0.0
    fresh = (rng.random(width) < 0.5).astype(np.int32)
    fresh[0], fresh[-1] = 1, 0
    bf16 = fmt == "bf16"
    t_out = np.empty_like(y)
    got = P.debug_sweeps_mixed(G, ALPHA, y, fresh, 1, chunks=chunks, t_out=t_out, sweep_tile=tile,
                               residue_format=P.RESIDUE_BF16 if bf16 else P.RESIDUE_F32)
    yin = _bf16(y) if bf16 else y
    csc_arrays = oracle.csc(g)
    din = np.diff(csc_arrays[0]).astype(np.float64)
    lo = oracle.chunk_bounds(g, chunks)
    chunk_of = np.searchsorted(lo, np.arange(g.n), side="right") - 1
    for b in range(width):
        want = oracle.block_gs_sweep(g, ALPHA, lo, yin[:, b].astype(np.float64), bool(fresh[b]),
                                     csc_arrays=csc_arrays)
        if bf16:
            rounds = chunk_of + 1 + (1 if fresh[b] else 0) * (chunk_of > 0)
            rel = (1.0 + UB) ** rounds - 1.0 + (din + din.max() + 6) * U
        else:
            rel = (din + din.max() + 3) * U
        err = np.abs(got[:, b] - want)
        assert np.all(err <= rel * want + 1e-38), (b, int(np.argmax(err - rel * want)))
        _assert_own_inputs(g, csc_arrays, lo, yin[:, b], got[:, b], bool(fresh[b]), width, bf16, tile, where=b)
        t_want = (yin[:, b] if fresh[b] else np.zeros(g.n, np.float32)) + got[:, b]
        np.testing.assert_array_equal(t_out[:, b], t_want.astype(np.float32))
    G.close()


def test_tiled_queries_and_tile_errors(graphs):
    """Whole batched queries at each row tile are certified and report their
    tile; the autotuner keeps one of the candidate tiles for every width it
    times and the width's queries use it; an unknown tile is an argument
    error."""
    g = graphs["hub"]
    G = P.Graph.from_synth(g)
    srcs = [int(s) for s in synth.sources(g.n, 8)]
    outs = []
    for tile in (12288, 16384, 24576):
        out, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=8, sweep_tile=tile)
        assert all(s["sweep_tile_bytes"] == tile for s in st)
        assert max(s["cert_l1"] for s in st) <= 1e-8
        outs.append(out)
    for o in outs[1:]:                       # each within lambda of pi_s, so within 2 lambda of each other
        assert np.abs(o - outs[0]).sum(axis=1).max() <= 2e-8 + 1e-9
    res = G.autotune(ALPHA, widths=[8, 32])
    for w in (8, 32):
        _, st = G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=w)
        assert st[0]["sweep_tile_bytes"] in (12288, 16384, 24576)
        assert max(s["cert_l1"] for s in st) <= 1e-8
    assert res["best"] in (8, 32)
    with pytest.raises(P.PPRError):
        G.query_batch(srcs, ALPHA, 1e-8, P.MIXED, batch_cols=8, sweep_tile=1000)
    _, st = G.query_batch(srcs[:1], ALPHA, 1e-8, P.FP64)
    assert st[0]["sweep_tile_bytes"] == 0
    G.close()


@pytest.mark.parametrize("name", ["c1", "hub", "seam"])
@pytest.mark.parametrize("width,chunks,fmt,sweeps", [(4, 3, "f32", 3), (32, 8, "bf16", 3), (128, 8, "bf16", 2),
                                                     (128, 4, "f32", 1), (64, 1, "bf16", 2)])
def test_wide_gather_addresses_same_bits(graphs, devgraphs, name, width, chunks, fmt, sweeps):
    """A block whose two residue buffers fit one buffer of < 4 GiB gathers at
    32-bit offsets from its base (the other tests); the full-address form of
    larger blocks, run here on buffers allocated apart, gives the same bits:
    outputs and stage accumulator, over chunk seams, both buffer orders
    (several sweeps) and entry and continuing columns, with over-relaxation."""
    g = graphs[name]
    G = devgraphs[name]
    print(f"[gpu] wide gather {name} width={width} chunks={chunks} {fmt} sweeps={sweeps}", flush=True)
    rng = np.random.default_rng(width * 11 + chunks + sweeps)
    y = rng.random((g.n, width)).astype(np.float32)
    y[rng.random((g.n, width)) < 0.3] = 0.0
    entry = rng.integers(0, 3, size=width).astype(np.int32)
    t_in = rng.random((g.n, width)).astype(np.float32)
    om = np.where(rng.random(width) < 0.5, 1.2, 1.0).astype(np.float32)
    fmt_id = P.RESIDUE_BF16 if fmt == "bf16" else P.RESIDUE_F32
    outs = []
    for wide in (False, True):
        t_out = np.empty_like(y)
        got = P.debug_sweeps_mixed(G, ALPHA, y, entry, sweeps, t_in=t_in, chunks=chunks, t_out=t_out, omega=om,
                                   residue_format=fmt_id, wide_gather=wide)
        outs.append((got, t_out))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    assert np.any(outs[0][0] != 0)
