"""FP64 CPU oracle for high-precision single-source PPR -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2101_03652_amd``), and the GPU library never imports it.

The arithmetic lives in ``oracle.c`` (plain sequential C, double precision);
this module only marshals numpy arrays to it.  Each routine states the passage
of the paper it restates:

- ``csc``              -- in-edge lists by counting sort (Section 2's graph, transposed)
- ``push``             -- the push operation (Section 3.2)
- ``fifo_fwdpush``     -- Algorithm 2, with the iteration sets S^(j) of Section 4.2
- ``powerpush``        -- Algorithm 3 (queue-ordered local phase, epochs of sequential scans)
- ``powerpush_sync``   -- the level-synchronous schedule of the GPU path:
                          iterations S^(j) pushed simultaneously, then Eq. 7 sweeps, or
                          Algorithm 3's epochs with each scan taken simultaneously
- ``sim_sweep``        -- one Simultaneous Forward Push iteration (Eq. 7)
- ``block_gs_sweep``   -- one global sweep in block Gauss-Seidel order (Algorithm 3's
                          in-place scan taken a chunk of rows at a time; Eq. 7 for one chunk)
- ``chunk_bounds``     -- the row chunks of about m / chunks in-edges that sweep uses
- ``block_sor_sweep``  -- that sweep over-relaxed (successive over-relaxation of it)
- ``powitr``           -- power iteration (Eqs. 3-5), compensated, used as truth
- ``certificate``      -- ||e_s - pi_hat (I - (1-alpha) P)/alpha||_1 (from Eq. 1)

Parity pins (tests/test_oracle_*.py) tie each routine to values the paper
prints, closed forms, a dense linear solve and the paper's bounds.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_NATIVE_PATH = os.path.join(_HERE, "liboracle_native.so")
_lib = None
_native = None


class Stats(ctypes.Structure):
    _fields_ = [("pushes", ctypes.c_int64), ("edge_pushes", ctypes.c_int64),
                ("local_levels", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("scans_per_epoch", ctypes.c_int32 * 8), ("switched", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("r_sum", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {"pushes": self.pushes, "edge_pushes": self.edge_pushes,
                "local_levels": self.local_levels, "sweeps": self.sweeps,
                "scans_per_epoch": list(self.scans_per_epoch), "switched": self.switched,
                "r_sum": self.r_sum}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain x86-64, -O2) for the tests."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_native() -> str:
    """Compile the same source for the host it runs on (-O3 -march=native, no
    floating-point contraction, so the arithmetic stays plain double): the
    build the timed CPU baseline uses.  Built where it is timed, never shipped:
    a -march=native object from another machine may not run."""
    tmp = _NATIVE_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-Wall", os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"])
    os.replace(tmp, _NATIVE_PATH)
    return _NATIVE_PATH


def _p(a):
    return a.ctypes.data


def _load(native: bool = False):
    global _lib, _native
    if native:
        if _native is None:
            _native = _bind(ctypes.CDLL(build_native()))
        return _native
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(lib):
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.oracle_sum.restype = f64
    lib.oracle_sum.argtypes = [i64, vp]
    lib.oracle_csc.restype = ctypes.c_int
    lib.oracle_csc.argtypes = [i32, i64, vp, vp, vp, vp, vp]
    lib.oracle_block_gs_sweep.restype = None
    lib.oracle_block_gs_sweep.argtypes = [i32, vp, vp, vp, f64, i32, vp, vp, ctypes.c_int, vp]
    lib.oracle_block_sor_sweep.restype = None
    lib.oracle_block_sor_sweep.argtypes = [i32, vp, vp, vp, f64, i32, vp, vp, ctypes.c_int, f64, vp, vp, vp]
    lib.oracle_push.restype = None
    lib.oracle_push.argtypes = [vp, vp, f64, vp, vp, i32]
    lib.oracle_fifo_fwdpush.restype = i64
    lib.oracle_fifo_fwdpush.argtypes = [i32, vp, vp, i32, f64, f64, vp, vp, vp, vp, i64, vp]
    lib.oracle_powerpush.restype = ctypes.c_int
    lib.oracle_powerpush.argtypes = [i32, i64, vp, vp, i32, f64, f64, vp, vp, vp, vp, i32]
    lib.oracle_powerpush_sync.restype = ctypes.c_int
    lib.oracle_powerpush_sync.argtypes = [i32, i64, vp, vp, i32, f64, f64, ctypes.c_int, f64, ctypes.c_int,
                                          vp, vp, vp, vp, i32, vp, vp, vp, i32]
    lib.oracle_sim_sweep.restype = None
    lib.oracle_sim_sweep.argtypes = [i32, vp, vp, f64, vp, vp, vp]
    lib.oracle_powitr.restype = ctypes.c_int
    lib.oracle_powitr.argtypes = [i32, vp, vp, i32, f64, i32, vp]
    lib.oracle_certificate.restype = f64
    lib.oracle_certificate.argtypes = [i32, vp, vp, i32, f64, vp, vp]
    u64 = ctypes.c_uint64
    lib.oracle_walk_budget.restype = f64
    lib.oracle_walk_budget.argtypes = [i32, f64, f64]
    lib.oracle_splitmix64.restype = u64
    lib.oracle_splitmix64.argtypes = [u64]
    lib.oracle_walk_endpoint.restype = i32
    lib.oracle_walk_endpoint.argtypes = [vp, vp, f64, u64, i32, ctypes.c_uint32, i32]
    lib.oracle_refine_sync.restype = i32
    lib.oracle_refine_sync.argtypes = [i32, vp, vp, f64, f64, vp, vp, vp]
    lib.oracle_mc_phase.restype = i64
    lib.oracle_mc_phase.argtypes = [i32, vp, vp, f64, f64, u64, i32, vp, vp]
    lib.oracle_powerpush_many.restype = ctypes.c_int
    lib.oracle_powerpush_many.argtypes = [i32, i64, vp, vp, vp, i32, f64, f64, vp, vp, vp, i32]
    return lib


def _g(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    return rp, col


def rsum(x: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return _load().oracle_sum(len(x), _p(x))


def csc(g):
    """(col_ptr int64[n+1], row_idx int32[m], deg_out int32[n])."""
    rp, col = _g(g)
    col_ptr = np.empty(g.n + 1, dtype=np.int64)
    row_idx = np.empty(max(g.m, 1), dtype=np.int32)
    deg = np.empty(g.n, dtype=np.int32)
    rc = _load().oracle_csc(g.n, g.m, _p(rp), _p(col), _p(col_ptr), _p(row_idx), _p(deg))
    if rc != 0:
        raise RuntimeError(f"oracle_csc failed ({rc})")
    return col_ptr, row_idx[:g.m], deg


def push(g, alpha: float, pi: np.ndarray, r: np.ndarray, v: int) -> None:
    """In-place push on v (Section 3.2)."""
    rp, col = _g(g)
    assert pi.dtype == np.float64 and r.dtype == np.float64
    _load().oracle_push(_p(rp), _p(col), alpha, _p(pi), _p(r), int(v))


def fifo_fwdpush(g, s: int, alpha: float, rmax: float, trace_cap: int = 0):
    """Algorithm 2.  Returns (pi, r, stats, trace) with trace a list of
    (node, iteration j) in pop order (at most trace_cap entries)."""
    rp, col = _g(g)
    pi = np.zeros(g.n)
    r = np.zeros(g.n)
    tn = np.zeros(max(trace_cap, 1), dtype=np.int32)
    tl = np.zeros(max(trace_cap, 1), dtype=np.int32)
    st = Stats()
    k = _load().oracle_fifo_fwdpush(g.n, _p(rp), _p(col), int(s), alpha, rmax, _p(pi), _p(r),
                                    _p(tn) if trace_cap else None, _p(tl) if trace_cap else None,
                                    trace_cap, ctypes.byref(st))
    if k < 0:
        raise MemoryError("oracle_fifo_fwdpush")
    cnt = min(int(k), trace_cap)
    return pi, r, st.as_dict(), list(zip(tn[:cnt].tolist(), tl[:cnt].tolist()))


def powerpush(g, s: int, alpha: float, lam: float, trace_cap: int = 0):
    """Algorithm 3.  Returns (pi, r, stats, rsum_trace)."""
    rp, col = _g(g)
    pi = np.zeros(g.n)
    r = np.zeros(g.n)
    tr = np.zeros(max(trace_cap, 1))
    st = Stats()
    k = _load().oracle_powerpush(g.n, g.m, _p(rp), _p(col), int(s), alpha, lam, _p(pi), _p(r),
                                 ctypes.byref(st), _p(tr) if trace_cap else None, trace_cap)
    if k < 0:
        raise MemoryError("oracle_powerpush")
    return pi, r, st.as_dict(), tr[:k].copy()


SWITCH_NODES = 0   # continue the local phase while 4|S| <= n (Algorithm 3)
SWITCH_EDGES = 1   # continue while param * vol(S) <= m


GLOBAL_SWEEPS = 0   # global phase: threshold-0 sweeps (Eq. 7)
GLOBAL_EPOCHS = 1   # global phase: Algorithm 3's epochs, each scan taken simultaneously


def powerpush_sync(g, s: int, alpha: float, lam: float, switch_rule: int = SWITCH_NODES,
                   switch_param: float = 1.0, trace_cap: int = 0, level_cap: int = 64,
                   global_rule: int = GLOBAL_SWEEPS):
    """Level-synchronous schedule.  Returns (pi, r, stats, rsum_trace, levels) where
    levels is a list of (|S^(j)|, vol(S^(j)), r_sum at the start of iteration j)."""
    rp, col = _g(g)
    pi = np.zeros(g.n)
    r = np.zeros(g.n)
    tr = np.zeros(max(trace_cap, 1))
    ls = np.zeros(max(level_cap, 1), dtype=np.int32)
    lv = np.zeros(max(level_cap, 1), dtype=np.int64)
    lr = np.zeros(max(level_cap, 1), dtype=np.float64)
    st = Stats()
    k = _load().oracle_powerpush_sync(g.n, g.m, _p(rp), _p(col), int(s), alpha, lam,
                                      int(switch_rule), float(switch_param), int(global_rule), _p(pi), _p(r),
                                      ctypes.byref(st), _p(tr) if trace_cap else None, trace_cap,
                                      _p(ls), _p(lv), _p(lr), level_cap)
    if k < 0:
        raise MemoryError("oracle_powerpush_sync")
    nl = min(st.local_levels, level_cap)
    return pi, r, st.as_dict(), tr[:k].copy(), list(zip(ls[:nl].tolist(), lv[:nl].tolist(),
                                                        lr[:nl].tolist()))


def sim_sweep(g, alpha: float, r_in: np.ndarray, pi: np.ndarray):
    """One Eq. 7 iteration.  Returns r_out; pi is updated in place."""
    rp, col = _g(g)
    r_in = np.ascontiguousarray(r_in, dtype=np.float64)
    r_out = np.empty(g.n)
    assert pi.dtype == np.float64 and pi.flags.c_contiguous
    _load().oracle_sim_sweep(g.n, _p(rp), _p(col), alpha, _p(r_in), _p(r_out), _p(pi))
    return r_out


def chunk_bounds(g, chunks: int) -> np.ndarray:
    """Row chunks of about m / chunks in-edges: lo[j] = the first row whose
    CSC offset reaches floor(m j / chunks); lo[0] = 0, lo[chunks] = n."""
    col_ptr, _, _ = csc(g)
    want = (np.int64(g.m) * np.arange(chunks + 1, dtype=np.int64)) // chunks
    lo = np.searchsorted(col_ptr, want, side="left").astype(np.int64)
    lo = np.minimum(lo, g.n)
    lo[0], lo[-1] = 0, g.n
    return np.maximum.accumulate(lo).astype(np.int32)


def block_gs_sweep(g, alpha: float, lo, y_old, fresh: bool = False, csc_arrays=None) -> np.ndarray:
    """One global sweep in block Gauss-Seidel order over the row chunks lo
    (y domain; see oracle_block_gs_sweep).  Returns y_new."""
    col_ptr, row_idx, deg = csc_arrays if csc_arrays is not None else csc(g)
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    y_old = np.ascontiguousarray(y_old, dtype=np.float64)
    y_new = np.zeros(g.n)
    _load().oracle_block_gs_sweep(g.n, _p(col_ptr), _p(row_idx), _p(deg), alpha, len(lo) - 1, _p(lo),
                                  _p(y_old), 1 if fresh else 0, _p(y_new))
    return y_new


def block_sor_sweep(g, alpha: float, lo, y_old, fresh: bool, omega: float, q_in, csc_arrays=None):
    """One over-relaxed block Gauss-Seidel sweep (see oracle_block_sor_sweep).
    Returns (y_new, q_out)."""
    col_ptr, row_idx, deg = csc_arrays if csc_arrays is not None else csc(g)
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    y_old = np.ascontiguousarray(y_old, dtype=np.float64)
    q_in = np.ascontiguousarray(q_in, dtype=np.float64)
    y_new = np.zeros(g.n)
    q_out = np.zeros(g.n)
    _load().oracle_block_sor_sweep(g.n, _p(col_ptr), _p(row_idx), _p(deg), alpha, len(lo) - 1, _p(lo),
                                   _p(y_old), 1 if fresh else 0, float(omega), _p(q_in), _p(q_out), _p(y_new))
    return y_new, q_out


def powitr(g, s: int, alpha: float, K: int = 135) -> np.ndarray:
    """Power iteration estimate after K iterations (error (1-alpha)^K, Eq. 6)."""
    rp, col = _g(g)
    pi = np.zeros(g.n)
    rc = _load().oracle_powitr(g.n, _p(rp), _p(col), int(s), alpha, int(K), _p(pi))
    if rc != 0:
        raise MemoryError("oracle_powitr")
    return pi


def certificate(g, s: int, alpha: float, pi_hat: np.ndarray, want_residual: bool = False):
    """||rt||_1 with rt = e_s - (pi_hat - (1-alpha) pi_hat P)/alpha; an upper
    bound on ||pi_hat - pi_s||_1."""
    rp, col = _g(g)
    pi_hat = np.ascontiguousarray(pi_hat, dtype=np.float64)
    rt = np.empty(g.n) if want_residual else None
    l1 = _load().oracle_certificate(g.n, _p(rp), _p(col), int(s), alpha, _p(pi_hat),
                                    _p(rt) if want_residual else None)
    if l1 < 0:
        raise MemoryError("oracle_certificate")
    return (l1, rt) if want_residual else l1


def powerpush_many(g, sources, alpha: float, lam: float, threads: int, native: bool = False):
    """Algorithm 3 on several sources, one query per thread.  Returns (pi[count, n], stats).
    native: run the -O3 -march=native build of the same source (built here first)."""
    rp, col = _g(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    cnt = len(src)
    pi = np.zeros((cnt, g.n))
    r = np.zeros((cnt, g.n))
    st = (Stats * cnt)()
    rc = _load(native).oracle_powerpush_many(g.n, g.m, _p(rp), _p(col), _p(src), cnt, alpha, lam,
                                       _p(pi), _p(r), st, int(threads))
    if rc != 0:
        raise MemoryError("oracle_powerpush_many")
    return pi, [s.as_dict() for s in st]


# ---------------------------------------------------------------- SpeedPPR (Section 6)
MAX_WALK_STEPS = 4096     # a walk alive after this many steps stops where it is


def walk_budget(n: int, eps: float, mu: float) -> float:
    """W of Eq. 8 (natural logarithm)."""
    return _load().oracle_walk_budget(int(n), float(eps), float(mu))


def splitmix64(z: int) -> int:
    return int(_load().oracle_splitmix64(ctypes.c_uint64(z & (2 ** 64 - 1))))


def walk_endpoint(g, alpha: float, seed: int, v: int, j: int, max_steps: int = MAX_WALK_STEPS) -> int:
    """Stop node of walk j from v (see oracle_walk_endpoint)."""
    rp, col = _g(g)
    return int(_load().oracle_walk_endpoint(_p(rp), _p(col), alpha, ctypes.c_uint64(seed), int(v), int(j),
                                            int(max_steps)))


def refine_sync(g, alpha: float, rmax: float, pi: np.ndarray, r: np.ndarray):
    """Algorithm 4's refinement, level-synchronous, in place on (pi, r).
    Returns (levels, edge_pushes)."""
    rp, col = _g(g)
    assert pi.dtype == np.float64 and r.dtype == np.float64 and pi.flags.c_contiguous and r.flags.c_contiguous
    ep = ctypes.c_int64()
    lv = _load().oracle_refine_sync(g.n, _p(rp), _p(col), alpha, rmax, _p(pi), _p(r), ctypes.byref(ep))
    if lv < 0:
        raise MemoryError("oracle_refine_sync")
    return int(lv), int(ep.value)


def mc_phase(g, alpha: float, W: float, seed: int, r: np.ndarray, pi: np.ndarray,
             max_steps: int = MAX_WALK_STEPS) -> int:
    """Algorithm 4's Monte Carlo phase: adds the walks' estimates to pi in
    place.  Returns the number of walks."""
    rp, col = _g(g)
    r = np.ascontiguousarray(r, dtype=np.float64)
    assert pi.dtype == np.float64 and pi.flags.c_contiguous
    return int(_load().oracle_mc_phase(g.n, _p(rp), _p(col), alpha, float(W), ctypes.c_uint64(seed),
                                       int(max_steps), _p(r), _p(pi)))

