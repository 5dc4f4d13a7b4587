"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds only input generation: directed Chung-Lu scale-free graphs (C, OpenMP,
counter-based SplitMix64 so the output is independent of the thread count),
uniform query sources, and a few small fixed graphs used as worked examples.
None of the PPR method's arithmetic lives here.

The graph shapes stand in for the SNAP datasets of the paper's evaluation
(Section 8, Table 1), which are not available: n=4M/m=70M has the shape of
LiveJournal, n=40M/m=1.4B that of Twitter.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

GRAPH_SEED = 2101
SOURCE_SEED = 3652
GEN_VERSION = 1


def build(force: bool = True) -> str:
    """Compile the generator with gcc (plain x86-64 code, portable across hosts)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               os.path.join(_HERE, "chunglu.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_chunglu.restype = ctypes.c_int
        lib.synth_chunglu.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_sources.restype = None
        lib.synth_sources.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """CSR of out-edges: row_ptr[n+1] int64, col[m] int32, rows ascending."""
    n: int
    m: int
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""
    max_out: int = 0
    max_in: int = 0

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def from_edges(n: int, edges, name: str = "") -> Graph:
    """CSR from an (src, dst) edge list; rows sorted ascending, duplicates kept."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    order = np.lexsort((e[:, 1], e[:, 0]))
    e = e[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, e[:, 0] + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    col = e[:, 1].astype(np.int32)
    deg = np.diff(row_ptr)
    indeg = np.bincount(col, minlength=n) if len(col) else np.zeros(n, dtype=np.int64)
    return Graph(n, int(len(col)), row_ptr, np.ascontiguousarray(col), name,
                 int(deg.max()) if n else 0, int(indeg.max()) if n else 0)


def _cache_dir() -> str:
    d = os.environ.get("PPR_GRAPH_CACHE", "/tmp/ppr_graph_cache")
    os.makedirs(d, exist_ok=True)
    return d


def chunglu(n: int, m: int, gamma_out: float = 2.1, gamma_in: float | None = None,
            seed: int = GRAPH_SEED, cache: bool = True) -> Graph:
    """Directed Chung-Lu graph with exactly m edges, min out-degree 1, no
    self-loops, no duplicate edges (see chunglu.c for the model)."""
    if gamma_in is None:
        gamma_in = gamma_out
    name = f"cl_{n}_{m}_{gamma_out:g}_{gamma_in:g}_{seed}_v{GEN_VERSION}"
    if cache:
        base = os.path.join(_cache_dir(), name)
        if os.path.exists(base + ".col.npy") and os.path.exists(base + ".meta.npy"):
            meta = np.load(base + ".meta.npy")
            return Graph(n, m, np.load(base + ".rowptr.npy"), np.load(base + ".col.npy"), name,
                         int(meta[0]), int(meta[1]))
    lib = _load()
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(m, dtype=np.int32)
    mo = ctypes.c_int32(0)
    mi = ctypes.c_int32(0)
    rc = lib.synth_chunglu(n, m, gamma_out, gamma_in, seed, row_ptr.ctypes.data, col.ctypes.data,
                           ctypes.byref(mo), ctypes.byref(mi))
    if rc != 0:
        raise RuntimeError(f"synth_chunglu failed with code {rc} for n={n} m={m}")
    g = Graph(n, m, row_ptr, col, name, mo.value, mi.value)
    if cache:
        base = os.path.join(_cache_dir(), name)
        for suffix, arr in ((".rowptr.npy", row_ptr), (".col.npy", col),
                            (".meta.npy", np.array([mo.value, mi.value], dtype=np.int64))):
            tmp = base + suffix + f".tmp{os.getpid()}.npy"
            np.save(tmp, arr)
            os.replace(tmp, base + suffix)
    return g


def sources(n: int, count: int, seed: int = SOURCE_SEED) -> np.ndarray:
    """count query sources, uniform in [0, n), from the counter-based generator."""
    lib = _load()
    out = np.empty(count, dtype=np.int32)
    lib.synth_sources(n, count, seed, out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Small fixed graphs (inputs of worked examples and closed-form cases)
# ---------------------------------------------------------------------------

def fig1() -> Graph:
    """The 5-node example graph of the paper's Figure 1 (v1..v5 -> ids 0..4),
    read off its printed transition matrix."""
    out = {0: [1, 2], 1: [0, 2, 3, 4], 2: [1, 3], 3: [0, 1, 2], 4: [1, 2]}
    return from_edges(5, [(v, u) for v, us in out.items() for u in us], "fig1")


def cycle(n: int) -> Graph:
    """Directed cycle 0 -> 1 -> ... -> n-1 -> 0."""
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], f"cycle{n}")


def star(leaves: int) -> Graph:
    """Bidirected star: centre 0, leaves 1..L, edges both ways."""
    e = [(0, i) for i in range(1, leaves + 1)] + [(i, 0) for i in range(1, leaves + 1)]
    return from_edges(leaves + 1, e, f"star{leaves}")


def complete(n: int) -> Graph:
    """Complete digraph without self-loops."""
    return from_edges(n, [(i, j) for i in range(n) for j in range(n) if i != j], f"K{n}")


def self_loop() -> Graph:
    """A single node with a self-loop."""
    return from_edges(1, [(0, 0)], "loop1")


def random_small(n: int, p: float, seed: int, self_loops: bool = False) -> Graph:
    """Erdos-Renyi-style digraph on n nodes (edge prob. p), plus one forced
    out-edge per node so no node is a dead end; no duplicates."""
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) < p
    if not self_loops:
        np.fill_diagonal(a, False)
    for v in range(n):
        if not a[v].any():
            choices = [u for u in range(n) if self_loops or u != v]
            a[v, choices[int(rng.integers(len(choices)))]] = True
    src, dst = np.nonzero(a)
    return from_edges(n, zip(src.tolist(), dst.tolist()), f"er{n}_{p:g}_{seed}")
