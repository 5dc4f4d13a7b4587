"""Python binding of libppr: high-precision single-source Personalized PageRank
on one MI355X (PowerPush, Wu, Gan, Wei, Zhang, SIGMOD 2021).

This module only marshals arguments to the C ABI declared in include/ppr.h;
every step of a query runs in the library's HIP kernels.  There is no CPU
fallback: if libppr.so is missing or no GPU is present, calls raise.

Buffers: graph inputs are host numpy arrays.  Outputs may be numpy arrays
(host) or torch tensors on the GPU (device pointers are passed straight
through); PyTorch serves only as a device allocator here.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppr.so")

PPR_OK = 0
STATUS = {0: "PPR_OK", -1: "PPR_ERR_ARG", -2: "PPR_ERR_CSR", -3: "PPR_ERR_DANGLING",
          -4: "PPR_ERR_DUPLICATE", -5: "PPR_ERR_OOM", -6: "PPR_ERR_DEVICE",
          -7: "PPR_ERR_NOT_CONVERGED", -8: "PPR_ERR_BUSY"}
FP64 = 0
MIXED = 1
SWITCH_NODES = 0
SWITCH_EDGES = 1
GLOBAL_SWEEPS = 0
GLOBAL_EPOCHS = 1
RESIDUE_F32 = 0
RESIDUE_BF16 = 1
RESIDUE_AUTO = 2
DEBUG_WIDE_GATHER = 1                    # ppr_debug_sweeps_mixed flag: 64-bit gather addresses
SCAN_AUTO = 0
SCAN_PULL = 1
SCAN_PUSH = 2
GRAPH_TRUST_INPUT = 1
GRAPH_WIDE_OFFSETS = 2
NOALLOC_MAX_NODES = 1 << 20          # ppr_query_fp64_noalloc's node limit

# every symbol include/ppr.h declares (checked by the CPU tests)
EXPORTS = [
    "ppr_options_default", "ppr_graph_create", "ppr_graph_destroy", "ppr_graph_get_info",
    "ppr_graph_copy_csc", "ppr_query", "ppr_query_batch", "ppr_query_ex",
    "ppr_debug_sweep_fp64", "ppr_version", "ppr_last_error", "ppr_autotune",
    "ppr_block_create", "ppr_block_destroy", "ppr_block_footprint", "ppr_slot_admit",
    "ppr_block_step", "ppr_block_poll", "ppr_slot_retire", "ppr_debug_sweep_mixed", "ppr_query_trace",
    "ppr_query_approx", "ppr_walk_index_build", "ppr_walk_index_copy", "ppr_debug_refine", "ppr_debug_walks",
    "ppr_debug_sweeps_mixed", "ppr_query_fp64_noalloc", "ppr_footprint_bytes",
]


class PPRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [("local_levels", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("refreshes", ctypes.c_int32), ("source", ctypes.c_int32),
                ("edge_pushes", ctypes.c_int64), ("r_sum", ctypes.c_double),
                ("cert_l1", ctypes.c_double), ("ms", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int32),
                ("batch_cols", ctypes.c_int32), ("sweep_chunks", ctypes.c_int32),
                ("sor_omega", ctypes.c_double), ("residue_format", ctypes.c_int32),
                ("push_scans", ctypes.c_int32), ("sweep_tile_bytes", ctypes.c_int32),
                ("refresh_ms", ctypes.c_double), ("refresh_launches", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ApproxStats(ctypes.Structure):
    _fields_ = [("source", ctypes.c_int32), ("local_levels", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("refine_levels", ctypes.c_int32), ("refine_edge_pushes", ctypes.c_int64),
                ("walks", ctypes.c_int64), ("W", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("r_sum", ctypes.c_double), ("ms_push", ctypes.c_double), ("ms_refine", ctypes.c_double),
                ("ms_walks", ctypes.c_double), ("ms", ctypes.c_double), ("used_index", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["lambda"] = d.pop("lambda_")
        return d


# one ppr_trace_point
TRACE_DTYPE = np.dtype([("ms", np.float64), ("r_sum", np.float64), ("edge_pushes", np.int64),
                        ("phase", np.int32), ("index", np.int32)])


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("switch_rule", ctypes.c_int32),
                ("switch_param", ctypes.c_double), ("max_sweeps", ctypes.c_int32),
                ("certify", ctypes.c_int32), ("refresh_factor", ctypes.c_double),
                ("batch_cols", ctypes.c_int32), ("sweep_chunks", ctypes.c_int32),
                ("global_rule", ctypes.c_int32), ("sor_omega", ctypes.c_double),
                ("residue_format", ctypes.c_int32), ("scan_form", ctypes.c_int32),
                ("sweep_tile", ctypes.c_int32), ("use_stream", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("max_in_degree", ctypes.c_int32), ("m", ctypes.c_int64),
                ("max_out_degree", ctypes.c_int32), ("offsets_64bit", ctypes.c_int32),
                ("build_ms", ctypes.c_double), ("device_bytes", ctypes.c_size_t),
                ("fp64_slices", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libppr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    sig = {
        "ppr_options_default": (None, [vp]),
        "ppr_graph_create": (st, [vp, vp, i32, i64, ctypes.c_uint32, ctypes.POINTER(vp)]),
        "ppr_graph_destroy": (st, [vp]),
        "ppr_graph_get_info": (st, [vp, vp]),
        "ppr_graph_copy_csc": (st, [vp, vp, vp, vp]),
        "ppr_query": (st, [vp, i32, f64, f64, ctypes.c_int, vp, vp]),
        "ppr_query_batch": (st, [vp, vp, i32, f64, f64, ctypes.c_int, vp, vp]),
        "ppr_query_ex": (st, [vp, vp, i32, f64, f64, vp, vp, vp, vp]),
        "ppr_query_trace": (st, [vp, i32, f64, f64, vp, vp, vp, i32, vp, vp]),
        "ppr_query_approx": (st, [vp, i32, f64, f64, f64, ctypes.c_uint64, i32, vp, vp, vp]),
        "ppr_walk_index_build": (st, [vp, f64, ctypes.c_uint64, vp]),
        "ppr_walk_index_copy": (st, [vp, vp]),
        "ppr_debug_refine": (st, [vp, f64, f64, vp, vp, vp, vp]),
        "ppr_debug_walks": (st, [vp, f64, f64, ctypes.c_uint64, i32, vp, vp, vp]),
        "ppr_debug_sweep_fp64": (st, [vp, f64, vp, vp, vp, vp]),
        "ppr_autotune": (st, [vp, f64, f64, vp, i32, vp, vp]),
        "ppr_debug_sweep_mixed": (st, [vp, f64, i32, i32, vp, vp, vp, vp, vp, i32]),
        "ppr_debug_sweeps_mixed": (st, [vp, f64, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i32, i32, i32]),
        "ppr_block_create": (st, [vp, i32, f64, vp, ctypes.POINTER(vp)]),
        "ppr_block_destroy": (st, [vp]),
        "ppr_block_footprint": (st, [vp, i32, vp]),
        "ppr_slot_admit": (st, [vp, i32, f64, f64, vp]),
        "ppr_footprint_bytes": (st, [i32, i64, i32, ctypes.c_int, vp, vp]),
        "ppr_block_step": (st, [vp, i32]),
        "ppr_block_poll": (st, [vp, i32, vp, vp, vp, vp]),
        "ppr_slot_retire": (st, [vp, i32, vp, vp]),
        "ppr_query_fp64_noalloc": (st, [vp, i32, f64, f64, vp, vp, vp]),
        "ppr_version": (ctypes.c_char_p, []),
        "ppr_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != PPR_OK:
        raise PPRError(rc, (load().ppr_last_error() or b"").decode())


def _ptr(x):
    """Raw address of a numpy array or a torch tensor (host or device)."""
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(f"unsupported buffer type {type(x)}")


def stream_handle(stream):
    """The hipStream_t of a torch.cuda.Stream (or a raw integer handle)."""
    return int(stream) if isinstance(stream, int) else int(stream.cuda_stream)


def options(**kw) -> Options:
    """ppr_options with the defaults, then the given fields.  stream=<a
    torch.cuda.Stream or a raw handle> sets use_stream = 1 and the handle
    (torch's default stream is the null stream, handle 0)."""
    o = Options()
    load().ppr_options_default(ctypes.byref(o))
    if kw.get("stream") is not None:
        o.use_stream = 1
        o.stream = stream_handle(kw.pop("stream"))
    kw.pop("stream", None)
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def footprint_bytes(n: int, m: int, slots: int, precision: int = MIXED) -> tuple[int, int]:
    """(graph bytes, state bytes) on the device for a graph of n nodes and m
    edges and `slots` query slots (ppr_footprint_bytes), before any graph
    exists."""
    gb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().ppr_footprint_bytes(int(n), int(m), int(slots), int(precision), ctypes.byref(gb),
                                      ctypes.byref(sb)))
    return gb.value, sb.value


class Graph:
    """A device-resident graph (CSC built on the GPU from CSR out-edges)."""

    def __init__(self, row_ptr: np.ndarray, col: np.ndarray, n: int | None = None,
                 trust_input: bool = False, wide_offsets: bool = False, fp64_slices: int = 0):
        """fp64_slices: source slices of the FP64 sweep (0: the library's choice)."""
        lib = load()
        self._row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self._col = np.ascontiguousarray(col, dtype=np.int32)
        self.n = int(len(self._row_ptr) - 1 if n is None else n)
        self.m = int(len(self._col))
        h = ctypes.c_void_p()
        _check(lib.ppr_graph_create(_ptr(self._row_ptr), _ptr(self._col) if self.m else None,
                                    self.n, self.m,
                                    (GRAPH_TRUST_INPUT if trust_input else 0) |
                                    (GRAPH_WIDE_OFFSETS if wide_offsets else 0) |
                                    ((int(fp64_slices) & 0xff) << 8),
                                    ctypes.byref(h)))
        self._h = h
        del self._row_ptr, self._col

    @classmethod
    def from_synth(cls, g, trust_input: bool = False, wide_offsets: bool = False,
                   fp64_slices: int = 0) -> "Graph":
        return cls(g.row_ptr, g.col, g.n, trust_input=trust_input, wide_offsets=wide_offsets,
                   fp64_slices=fp64_slices)

    @property
    def handle(self):
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().ppr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        gi = GraphInfo()
        _check(load().ppr_graph_get_info(self._h, ctypes.byref(gi)))
        return {k: getattr(gi, k) for k, _ in gi._fields_}

    def csc(self):
        """Host copies of (col_ptr int64[n+1], row_idx int32[m], deg_out int32[n])."""
        col_ptr = np.empty(self.n + 1, dtype=np.int64)
        row_idx = np.empty(max(self.m, 1), dtype=np.int32)
        deg = np.empty(self.n, dtype=np.int32)
        _check(load().ppr_graph_copy_csc(self._h, _ptr(col_ptr), _ptr(row_idx), _ptr(deg)))
        return col_ptr, row_idx[:self.m], deg

    # ---- queries
    def query(self, s: int, alpha: float = 0.2, lam: float = 1e-8, precision: int = FP64,
              out=None, **opt):
        """pi_hat for source s (numpy float64[n] unless `out` is given)."""
        res = self.query_batch([s], alpha, lam, precision, out=out, **opt)
        return (res[0][0] if out is None else res[0]), res[1][0]

    def query_batch(self, sources, alpha: float = 0.2, lam: float = 1e-8, precision: int = FP64,
                    out=None, r_out=None, **opt):
        """pi_hat for every source: float64[B, n] (host array or device tensor `out`)."""
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1))
        B = len(src)
        if out is None:
            out = np.empty((B, self.n), dtype=np.float64)
        st = (Stats * B)()
        o = options(precision=precision, **opt)
        rc = load().ppr_query_ex(self._h, _ptr(src), B, float(alpha), float(lam), ctypes.byref(o),
                                 _ptr(out), _ptr(r_out) if r_out is not None else None, st)
        _check(rc)
        return out, [s.as_dict() for s in st]

    def query_noalloc(self, s: int, alpha: float, lam: float, out, stream=None) -> dict:
        """The allocation-free FP64 query (ppr_query_fp64_noalloc): pi_hat into
        `out`, a float64[n] device tensor; `stream`: a torch.cuda.Stream (None:
        the null stream).  Returns the statistics."""
        st = Stats()
        h = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(load().ppr_query_fp64_noalloc(self._h, int(s), float(alpha), float(lam), h, _ptr(out),
                                             ctypes.byref(st)))
        return st.as_dict()

    def query_trace(self, s: int, alpha: float = 0.2, lam: float = 1e-8, out=None, capacity: int = 4096,
                    **opt):
        """One FP64 query with its convergence trace.  Returns (pi_hat, trace,
        stats); trace is a structured array with fields ms, r_sum (= the l1
        error), edge_pushes, phase (0 local, 1 global) and index, one row per
        iteration."""
        if out is None:
            out = np.empty(self.n, dtype=np.float64)
        tr = np.zeros(capacity, dtype=TRACE_DTYPE)
        cnt = ctypes.c_int32()
        st = Stats()
        o = options(precision=FP64, **opt)
        _check(load().ppr_query_trace(self._h, int(s), float(alpha), float(lam), ctypes.byref(o), _ptr(out),
                                      _ptr(tr), int(capacity), ctypes.byref(cnt), ctypes.byref(st)))
        if cnt.value > capacity:
            raise PPRError(-1, f"trace needs {cnt.value} points, capacity is {capacity}")
        return out, tr[:cnt.value].copy(), st.as_dict()

    def query_approx(self, s: int, alpha: float = 0.2, eps: float = 0.5, mu: float | None = None,
                     seed: int = 0, use_index: bool = False, out=None, **opt):
        """Approximate query (SpeedPPR, Algorithm 4): relative error eps on
        every node with pi >= mu (default 1/n) with probability 1 - 1/n.
        Keyword options go to the phase-1 PowerPush (default: Algorithm 3's
        epoch thresholds).  Returns (pi_hat, stats)."""
        if out is None:
            out = np.empty(self.n, dtype=np.float64)
        opt.setdefault("global_rule", GLOBAL_EPOCHS)
        st = ApproxStats()
        mu = 1.0 / self.n if mu is None else mu
        o = options(precision=FP64, **opt)
        _check(load().ppr_query_approx(self._h, int(s), float(alpha), float(eps), float(mu),
                                       ctypes.c_uint64(seed), 1 if use_index else 0, ctypes.byref(o), _ptr(out),
                                       ctypes.byref(st)))
        return out, st.as_dict()

    def build_walk_index(self, alpha: float = 0.2, seed: int = 0) -> float:
        """Pre-compute d_v walks per node (m in all); returns the build time (ms)."""
        ms = ctypes.c_double()
        _check(load().ppr_walk_index_build(self._h, float(alpha), ctypes.c_uint64(seed), ctypes.byref(ms)))
        return ms.value

    def walk_index(self) -> np.ndarray:
        out = np.empty(max(self.m, 1), dtype=np.int32)
        _check(load().ppr_walk_index_copy(self._h, _ptr(out)))
        return out[:self.m]

    def debug_refine(self, alpha: float, rmax: float, pi, r):
        """Refinement in place on device tensors; returns (levels, edge_pushes)."""
        lv = ctypes.c_int32()
        ep = ctypes.c_int64()
        _check(load().ppr_debug_refine(self._h, float(alpha), float(rmax), _ptr(pi), _ptr(r), ctypes.byref(lv),
                                       ctypes.byref(ep)))
        return lv.value, ep.value

    def debug_walks(self, alpha: float, W: float, seed: int, r, pi, use_index: bool = False) -> int:
        """Monte Carlo phase on device tensors (adds into pi); returns the walks."""
        nw = ctypes.c_int64()
        _check(load().ppr_debug_walks(self._h, float(alpha), float(W), ctypes.c_uint64(seed),
                                      1 if use_index else 0, _ptr(r), _ptr(pi), ctypes.byref(nw)))
        return nw.value

    def autotune(self, alpha: float = 0.2, lam: float = 1e-8, widths=None) -> dict:
        """Pick the batched block width, the residue storage per width and
        the sweep row tile per (width, storage) by timing sweeps and one batch
        of queries end to end per candidate on this graph; the choices become
        the defaults of later batched queries (and the tiles of serving
        blocks)."""
        w = None if widths is None else np.ascontiguousarray(widths, dtype=np.int32)
        cnt = 5 if w is None else len(w)
        cost = np.zeros(cnt, dtype=np.float64)
        best = ctypes.c_int32()
        _check(load().ppr_autotune(self._h, float(alpha), float(lam), _ptr(w) if w is not None else None,
                                   cnt, ctypes.byref(best), _ptr(cost)))
        ws = [8, 16, 32, 64, 128] if w is None else w.tolist()
        return {"best": best.value, "us_per_query": dict(zip(ws, cost.round(3).tolist()))}

    def debug_sweep(self, alpha: float, r_in, r_out, pi) -> float:
        """One Eq. 7 sweep on device tensors: r_out = (1-alpha) r_in P, pi += alpha r_in."""
        rs = ctypes.c_double()
        _check(load().ppr_debug_sweep_fp64(self._h, float(alpha), _ptr(r_in), _ptr(r_out), _ptr(pi),
                                           ctypes.byref(rs)))
        return rs.value


class Block:
    """A serving block: `slots` query slots on one graph (continuous batching).

    admit() puts a (source, lambda) query into a free slot, step() advances
    every running slot, poll() collects finished work, retire() copies a
    certified result out and frees its slot for the next query."""

    def __init__(self, graph: Graph, slots: int, alpha: float = 0.2, **opt):
        """opt: ppr_options fields; stream=<torch.cuda.Stream> runs the block
        on that stream."""
        self.graph = graph          # keeps the graph alive while the block exists
        self.slots = int(slots)
        self.alpha = float(alpha)
        o = options(precision=MIXED, **opt)
        h = ctypes.c_void_p()
        _check(load().ppr_block_create(graph.handle, self.slots, self.alpha, ctypes.byref(o),
                                       ctypes.byref(h)))
        self._h = h
        self._done = np.zeros(self.slots, dtype=np.uint8)

    @staticmethod
    def footprint(graph: Graph, slots: int) -> int:
        b = ctypes.c_size_t()
        _check(load().ppr_block_footprint(graph.handle, int(slots), ctypes.byref(b)))
        return b.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().ppr_block_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, source: int, lam: float, alpha: float | None = None) -> int:
        """Admit a query; alpha None takes the block's reference alpha."""
        slot = ctypes.c_int32(-1)
        _check(load().ppr_slot_admit(self._h, int(source), 0.0 if alpha is None else float(alpha), float(lam),
                                     ctypes.byref(slot)))
        return slot.value

    def step(self, max_sweeps: int = 16) -> None:
        _check(load().ppr_block_step(self._h, int(max_sweeps)))

    def poll(self, wait: bool = False) -> dict:
        nd, nb, rd = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().ppr_block_poll(self._h, 1 if wait else 0, _ptr(self._done), ctypes.byref(nd),
                                     ctypes.byref(nb), ctypes.byref(rd)))
        return {"done": np.flatnonzero(self._done).tolist(), "n_done": nd.value, "n_busy": nb.value,
                "ready": bool(rd.value)}

    def retire(self, slot: int, out=None):
        if out is None:
            out = np.empty(self.graph.n, dtype=np.float64)
        st = Stats()
        _check(load().ppr_slot_retire(self._h, int(slot), _ptr(out), ctypes.byref(st)))
        return out, st.as_dict()


def debug_sweep_mixed(graph: "Graph", alpha: float, y_in, fresh, chunks: int = 1, t_out=None,
                      omega=None, residue_format: int = RESIDUE_F32):
    """One batched global sweep (block Gauss-Seidel over `chunks` row chunks;
    over-relaxed when `omega`, B factors, is given) with the residue block
    stored as `residue_format` (FP32 unless asked).  y_in: float32[n, B]
    (numpy or device tensor); fresh: B flags.  Returns y_out (same kind as
    y_in)."""
    B = int(y_in.shape[1])
    fr = np.ascontiguousarray(np.asarray(fresh, dtype=np.int32).reshape(-1))
    if len(fr) != B:
        raise ValueError("fresh needs one flag per column")
    if isinstance(y_in, np.ndarray):
        y_out = np.empty_like(y_in)
    else:
        y_out = y_in.new_empty(y_in.shape)
    om = None if omega is None else np.ascontiguousarray(np.asarray(omega, dtype=np.float32).reshape(-1))
    if om is not None and len(om) != B:
        raise ValueError("omega needs one factor per column")
    _check(load().ppr_debug_sweep_mixed(graph.handle, float(alpha), B, int(chunks), _ptr(y_in), _ptr(fr),
                                        _ptr(y_out), _ptr(t_out) if t_out is not None else None,
                                        _ptr(om) if om is not None else None, int(residue_format)))
    return y_out


def debug_sweeps_mixed(graph: "Graph", alpha: float, y_in, entry, sweeps: int, budget=None, t_in=None,
                       chunks: int = 1, t_out=None, omega=None, residue_format: int = RESIDUE_F32,
                       sweep_tile: int = 0, wide_gather: bool = False):
    """One launch sequence of `sweeps` batched global sweeps carrying the
    stage accumulator.  entry: B flags (0 continuing, 1 fresh, 2 fresh with
    the accumulator restarting); budget: B sweep counts in [0, sweeps] (None:
    all); t_in: float32[n, B] initial accumulator (None: 0); sweep_tile: LDS
    stage bytes of a sweep block (0: the graph's choice).  Returns y_out
    (same kind as y_in); t_out, if given, receives the accumulator.
    wide_gather: run the sweeps on residue buffers allocated apart (64-bit
    gather addresses instead of 32-bit offsets; same results)."""
    B = int(y_in.shape[1])
    en = np.ascontiguousarray(np.asarray(entry, dtype=np.int32).reshape(-1))
    if len(en) != B:
        raise ValueError("entry needs one flag per column")
    kb = None if budget is None else np.ascontiguousarray(np.asarray(budget, dtype=np.int32).reshape(-1))
    if kb is not None and len(kb) != B:
        raise ValueError("budget needs one count per column")
    if isinstance(y_in, np.ndarray):
        y_out = np.empty_like(y_in)
    else:
        y_out = y_in.new_empty(y_in.shape)
    om = None if omega is None else np.ascontiguousarray(np.asarray(omega, dtype=np.float32).reshape(-1))
    if om is not None and len(om) != B:
        raise ValueError("omega needs one factor per column")
    _check(load().ppr_debug_sweeps_mixed(graph.handle, float(alpha), B, int(chunks), int(sweeps), _ptr(y_in),
                                         _ptr(en), _ptr(kb) if kb is not None else None,
                                         _ptr(t_in) if t_in is not None else None, _ptr(y_out),
                                         _ptr(t_out) if t_out is not None else None,
                                         _ptr(om) if om is not None else None, int(residue_format),
                                         int(sweep_tile), DEBUG_WIDE_GATHER if wide_gather else 0))
    return y_out


def version() -> str:
    return load().ppr_version().decode()
