"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host-side argument and CSR validation returns the documented codes
(no compute call runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2101_03652_amd as P
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = P.load()
    header = open(os.path.join(ROOT, "include", "ppr.h")).read()
    declared = set(re.findall(r"^\s*(?:ppr_status|void|const char\*|size_t)\s+(ppr_\w+)\s*\(", header, re.M))
    assert declared, "no declarations parsed"
    assert declared == set(P.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert P.version().startswith("libppr")


def test_options_default():
    o = P.options()
    assert o.precision == P.FP64 and o.switch_rule == P.SWITCH_EDGES
    assert o.switch_param == 32.0 and o.max_sweeps == 4096 and o.refresh_factor == 0.0 and o.residue_format == 2
    assert o.scan_form == P.SCAN_AUTO


def _create(row_ptr, col, n, flags=0):
    lib = P.load()
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    rc = lib.ppr_graph_create(rp.ctypes.data, c.ctypes.data if len(c) else None, n, len(c), flags,
                              ctypes.byref(h))
    return rc, h


def test_graph_flags_validation():
    """Unknown flag bits and more than 64 source slices are argument errors,
    caught before any device work."""
    rp, col = [0, 1, 2, 3], [1, 2, 0]
    assert _create(rp, col, 3, flags=1 << 20)[0] == -1
    assert _create(rp, col, 3, flags=65 << 8)[0] == -1
    assert _create(rp, col, 3, flags=255 << 8)[0] == -1


def test_csr_validation_codes():
    # non-monotone offsets
    rc, _ = _create([0, 2, 1, 3], [1, 2, 0], 3)
    assert rc == -2
    # row_ptr[0] != 0
    rc, _ = _create([1, 2, 3, 4], [1, 2, 0], 3)
    assert rc == -2
    # column index out of range
    rc, _ = _create([0, 1, 2, 3], [1, 7, 0], 3)
    assert rc == -2
    rc, _ = _create([0, 1, 2, 3], [1, -1, 0], 3)
    assert rc == -2
    # dangling node (out-degree 0)
    rc, _ = _create([0, 1, 1, 3], [1, 0, 1], 3)
    assert rc == -3
    # m < n
    rc, _ = _create([0, 1, 2, 2], [1, 2], 3)
    assert rc == -3
    # duplicate edge (unsorted row too)
    rc, _ = _create([0, 3, 4, 5], [2, 1, 2, 2, 0], 3)
    assert rc == -4
    assert b"duplicate" in P.load().ppr_last_error()
    # unknown flag bits
    g = synth.fig1()
    rc, _ = _create(g.row_ptr, g.col, g.n, flags=4)
    assert rc == -1 and b"flags" in P.load().ppr_last_error()


def test_serving_and_debug_entry_points_reject_bad_arguments():
    lib = P.load()
    h = ctypes.c_void_p()
    assert lib.ppr_block_create(None, 8, 0.2, None, ctypes.byref(h)) == -1
    assert lib.ppr_block_destroy(None) == 0
    b = ctypes.c_size_t()
    assert lib.ppr_block_footprint(None, 8, ctypes.byref(b)) == -1
    slot = ctypes.c_int32()
    assert lib.ppr_slot_admit(None, 0, 0.2, 1e-8, ctypes.byref(slot)) == -1
    assert lib.ppr_block_step(None, 4) == -1
    assert lib.ppr_block_poll(None, 0, None, None, None, None) == -1
    assert lib.ppr_slot_retire(None, 0, None, None) == -1
    assert lib.ppr_debug_sweep_mixed(None, 0.2, 8, 1, None, None, None, None, None, 0) == -1
    assert lib.ppr_debug_sweeps_mixed(None, 0.2, 8, 1, 2, None, None, None, None, None, None, None, 0, 0, 0) == -1


def test_null_and_range_arguments():
    lib = P.load()
    h = ctypes.c_void_p()
    assert lib.ppr_graph_create(None, None, 3, 3, 0, ctypes.byref(h)) == -1
    assert lib.ppr_graph_create(np.zeros(2, np.int64).ctypes.data, None, 0, 0, 0, ctypes.byref(h)) == -1
    out = np.zeros(4)
    assert lib.ppr_query(None, 0, 0.2, 1e-8, 0, out.ctypes.data, None) == -1
    assert lib.ppr_graph_destroy(None) == 0
    # a valid CSR reaches the device step and reports the missing GPU (or succeeds on a GPU host)
    g = synth.fig1()
    rc, h = _create(g.row_ptr, g.col, g.n)
    if rc == 0:
        lib.ppr_graph_destroy(h)
    else:
        assert rc == -6


def test_large_generated_graph_passes_validation_fast():
    g = synth.chunglu(200_000, 3_000_000, 2.1)
    rc, h = _create(g.row_ptr, g.col, g.n)
    assert rc in (0, -6)
    if rc == 0:
        P.load().ppr_graph_destroy(h)


def test_footprint_bytes_without_a_graph():
    """ppr_footprint_bytes is host arithmetic: it answers before any graph or
    GPU exists.  Graph: CSR (8 (n+1) + 4 m), CSC (4 or 8 bytes per offset, 4 m),
    degrees (4 n) and, above 1.5M nodes, the FP64 sweep's source slices (one
    per 12 MiB of FP64 vector, at most 16: a copy of the in-edges, the listed
    (slice, row) pairs of all slices but the last, at most min((S - 1) n, m)
    of them with a row id and an offset each, and the last slice's n + 1
    offsets; the pairs depend on the graph, so this part is an upper bound).
    A mixed block of B slots holds per (node, column) the
    FP64 local-phase scratch (16 bytes), two residue buffers (2 bytes each in
    bf16 from 32 slots up, else 4), the FP64 reserve and its in-neighbour sums
    (16) and the FP32 stage accumulator (4), plus the frontier, the
    long-row partial sums and the refresh's per-block column sums."""
    n, m = 4_000_000, 70_000_000
    for B in (4, 8, 16, 32, 64, 128):
        gb, sb = P.footprint_bytes(n, m, B, P.MIXED)
        assert gb == 8 * (n + 1) + 4 * m + 4 * (n + 1) + 4 * m + 4 * n + 4 * m + 8 * (2 * n) + 4 + 4 * (n + 1)
        per = 16 + 16 + 4 + (2 * 2 if B >= 32 else 2 * 4)
        assert per * n * B <= sb <= per * n * B * 1.15 + (64 << 20), (B, sb)
    # int64 CSC offsets from 2^32 - 1 edges on
    gb, _ = P.footprint_bytes(40_000_000, 2 ** 32 - 1, 16, P.MIXED)
    assert gb == (8 * (40_000_001) + 4 * (2 ** 32 - 1) + 8 * 40_000_001 + 4 * (2 ** 32 - 1) + 4 * 40_000_000
                  + 4 * (2 ** 32 - 1) + 12 * (15 * 40_000_000) + 8 + 8 * 40_000_001)
    # no slices while the FP64 vector fits 12 MiB; 2 from just above
    gb, _ = P.footprint_bytes(1_500_000, 5_000_000, 4, P.MIXED)
    assert gb == 8 * 1_500_001 + 4 * 5_000_000 + 4 * 1_500_001 + 4 * 5_000_000 + 4 * 1_500_000
    gb, _ = P.footprint_bytes(1_600_000, 5_000_000, 4, P.MIXED)
    assert gb == (8 * 1_600_001 + 4 * 5_000_000 + 4 * 1_600_001 + 4 * 5_000_000 + 4 * 1_600_000
                  + 4 * 5_000_000 + 8 * 1_600_000 + 4 + 4 * 1_600_001)
    gb1, s1 = P.footprint_bytes(n, m, 1, P.FP64)
    _, s2 = P.footprint_bytes(n, m, 2, P.FP64)
    assert s2 == 2 * s1 and 80 * n <= s1 <= 100 * n
    for args in ((0, 10, 4, P.MIXED), (10, 9, 4, P.MIXED), (10, 101, 4, P.MIXED), (10, 20, 6, P.MIXED),
                 (10, 20, 256, P.MIXED), (10, 20, 0, P.FP64), (10, 20, 4, 7)):
        with pytest.raises(P.PPRError):
            P.footprint_bytes(*args)


def test_options_stream_fields():
    o = P.options()
    assert o.use_stream == 0 and not o.stream
    o = P.options(stream=0)                # torch's default stream: the null stream
    assert o.use_stream == 1 and not o.stream
    o = P.options(stream=0x1234)
    assert o.use_stream == 1 and o.stream == 0x1234
