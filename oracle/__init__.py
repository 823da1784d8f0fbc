"""TCR-network oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the two
share no code: the only common input source is the ``synth`` generator, which
holds none of the method's arithmetic.

Contents
  oracle.c   full O(m n) dynamic-programming Levenshtein over all O(N^2) pairs
             (paper, Methods: "Levenshtein distance", "TCR network",
             "Adjacency matrix", "Overview of network theory concepts")
  k1.c       an independent closed-form witness for threshold 1 (no DP)
  graph.c    breadth-first connected components and site percolation
  checks.py  pure-Python brute force over the edit graph on tiny alphabets

``build_lib()`` compiles the C files into ``liboracle.so`` with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "k1.c"), os.path.join(_HERE, "graph.c")]


def build_lib(out: str = LIB_PATH, extra_flags=()) -> str:
    """Compile the oracle with gcc (OpenMP).  Returns the library path."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           *extra_flags, *SOURCES, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_u8p = ctypes.c_void_p
_lib = None


def _bind(lib):
    lib.oracle_lev.restype = ctypes.c_int
    lib.oracle_lev.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_int]
    lib.oracle_build_rows.restype = ctypes.c_int
    lib.oracle_build_rows.argtypes = [_u8p, _u8p, ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]
    lib.oracle_row.restype = ctypes.c_int64
    lib.oracle_row.argtypes = [_u8p, _u8p, ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint32,
                               ctypes.c_int, ctypes.c_void_p]
    lib.oracle_query.restype = ctypes.c_int
    lib.oracle_query.argtypes = [_u8p, _u8p, ctypes.c_uint32, _u8p, _u8p, ctypes.c_uint32,
                                 ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                 ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]
    lib.oracle_free.restype = None
    lib.oracle_free.argtypes = [ctypes.c_void_p]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_threads.argtypes = [ctypes.c_int]
    lib.oracle_exit_step.restype = ctypes.c_int
    lib.oracle_exit_step.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_int, ctypes.c_int]
    lib.oracle_exit_steps.restype = None
    lib.oracle_exit_steps.argtypes = [_u8p, _u8p, _u8p, _u8p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int,
                                      ctypes.c_void_p]
    lib.k1_build.restype = ctypes.c_int
    lib.k1_build.argtypes = [_u8p, _u8p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p),
                             ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]
    lib.k1_adjacent.restype = ctypes.c_int
    lib.k1_adjacent.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_int]
    lib.k1_free.restype = None
    lib.k1_free.argtypes = [ctypes.c_void_p]
    lib.oracle_components.restype = ctypes.c_int64
    lib.oracle_components.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p]
    lib.oracle_robustness.restype = ctypes.c_int
    lib.oracle_robustness.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, _u8p, _u8p, ctypes.c_uint32,
                                      ctypes.c_void_p]
    return lib


def load(path: str = LIB_PATH):
    """Load (building first if absent) the oracle library."""
    global _lib
    if path != LIB_PATH:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib()
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _as_bytes(s) -> bytes:
    return s.encode("ascii") if isinstance(s, str) else bytes(s)


def _take_pairs(lib, ptr, n, free) -> np.ndarray:
    n = int(n)
    if n == 0:
        free(ptr)
        return np.zeros((0, 2), dtype=np.uint32)
    buf = (ctypes.c_uint32 * (2 * n)).from_address(ptr)
    arr = np.frombuffer(buf, dtype=np.uint32).reshape(n, 2).copy()
    free(ptr)
    return arr


class Oracle:
    """ctypes view of liboracle.so; ``nthreads=0`` means all OpenMP threads."""

    def __init__(self, path: str = LIB_PATH, nthreads: int = 0):
        self.lib = load(path)
        self.nthreads = nthreads

    def threads(self) -> int:
        return self.lib.oracle_threads(self.nthreads)

    def lev(self, a, b) -> int:
        a, b = _as_bytes(a), _as_bytes(b)
        return self.lib.oracle_lev(a, len(a), b, len(b))

    def build(self, seqs, k: int, row_lo: int = 0, row_hi: int | None = None):
        """Edges (E, 2) uint32 sorted, degree int32 (true degree only for the
        whole network, i.e. row_lo=0 and row_hi=n)."""
        n = seqs.n
        row_hi = n if row_hi is None else row_hi
        deg = np.zeros(max(1, n), dtype=np.int32)
        ptr = ctypes.c_void_p()
        cnt = ctypes.c_uint64()
        chars = np.ascontiguousarray(seqs.chars) if seqs.chars.size else np.zeros(1, np.uint8)
        rc = self.lib.oracle_build_rows(chars.ctypes.data, seqs.offsets.ctypes.data, n, k, row_lo,
                                        row_hi, self.nthreads, ctypes.byref(ptr),
                                        ctypes.byref(cnt), deg.ctypes.data)
        if rc != 0:
            raise MemoryError("oracle_build_rows failed")
        return _take_pairs(self.lib, ptr.value, cnt.value, self.lib.oracle_free), deg[:n]

    def row(self, seqs, k: int, i: int) -> np.ndarray:
        """All j != i with lev(s_i, s_j) <= k, ascending."""
        out = np.zeros(max(1, seqs.n), dtype=np.uint32)
        chars = np.ascontiguousarray(seqs.chars) if seqs.chars.size else np.zeros(1, np.uint8)
        c = self.lib.oracle_row(chars.ctypes.data, seqs.offsets.ctypes.data, seqs.n, k, i,
                                self.nthreads, out.ctypes.data)
        if c < 0:
            raise MemoryError("oracle_row failed")
        return out[:c].copy()

    def query(self, rep, qs, k: int):
        """Pairs (q, r) with lev <= k sorted, and per-query neighbour counts."""
        cnt = np.zeros(max(1, qs.n), dtype=np.int32)
        ptr = ctypes.c_void_p()
        ne = ctypes.c_uint64()
        rc_ = np.ascontiguousarray(rep.chars) if rep.chars.size else np.zeros(1, np.uint8)
        qc_ = np.ascontiguousarray(qs.chars) if qs.chars.size else np.zeros(1, np.uint8)
        rc = self.lib.oracle_query(rc_.ctypes.data, rep.offsets.ctypes.data, rep.n,
                                   qc_.ctypes.data, qs.offsets.ctypes.data, qs.n, k,
                                   self.nthreads, ctypes.byref(ptr), ctypes.byref(ne),
                                   cnt.ctypes.data)
        if rc != 0:
            raise MemoryError("oracle_query failed")
        return _take_pairs(self.lib, ptr.value, ne.value, self.lib.oracle_free), cnt[:qs.n]

    def exit_step(self, a, b, k: int) -> int:
        """Steps of the exact final-diagonal early exit (rows = longer string)."""
        a, b = _as_bytes(a), _as_bytes(b)
        return self.lib.oracle_exit_step(a, len(a), b, len(b), k)

    def exit_steps(self, seqs, pi, pj, k: int) -> np.ndarray:
        pi = np.ascontiguousarray(pi, dtype=np.uint32)
        pj = np.ascontiguousarray(pj, dtype=np.uint32)
        out = np.zeros(max(1, len(pi)), dtype=np.int32)
        chars = np.ascontiguousarray(seqs.chars) if seqs.chars.size else np.zeros(1, np.uint8)
        self.lib.oracle_exit_steps(chars.ctypes.data, seqs.offsets.ctypes.data, pi.ctypes.data, pj.ctypes.data,
                                   len(pi), k, self.nthreads, out.ctypes.data)
        return out[:len(pi)]

    def k1_build(self, seqs):
        """Closed-form threshold-1 network (no DP): edges, degree."""
        n = seqs.n
        deg = np.zeros(max(1, n), dtype=np.int32)
        ptr = ctypes.c_void_p()
        cnt = ctypes.c_uint64()
        chars = np.ascontiguousarray(seqs.chars) if seqs.chars.size else np.zeros(1, np.uint8)
        rc = self.lib.k1_build(chars.ctypes.data, seqs.offsets.ctypes.data, n, ctypes.byref(ptr),
                               ctypes.byref(cnt), deg.ctypes.data)
        if rc == -2:
            raise ValueError("k1_build: string longer than 32")
        if rc != 0:
            raise MemoryError("k1_build failed")
        return _take_pairs(self.lib, ptr.value, cnt.value, self.lib.k1_free), deg[:n]

    def k1_adjacent(self, a, b) -> bool:
        a, b = _as_bytes(a), _as_bytes(b)
        return bool(self.lib.k1_adjacent(a, len(a), b, len(b)))


def _pairs_arg(pairs):
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.uint32).reshape(-1, 2))
    return p if p.size else np.zeros((1, 2), dtype=np.uint32), int(len(np.asarray(pairs).reshape(-1, 2)))


def components(pairs, n: int):
    """(labels, sizes, n_components, lcc): labels[i] = smallest id of i's
    component; sizes[i] = size of the component labelled i (0 if none)."""
    lib = load()
    p, E = _pairs_arg(pairs)
    labels = np.zeros(max(1, n), dtype=np.uint32)
    sizes = np.zeros(max(1, n), dtype=np.uint32)
    nc = ctypes.c_uint32()
    lcc = lib.oracle_components(p.ctypes.data, E, n, labels.ctypes.data, sizes.ctypes.data, ctypes.byref(nc))
    if lcc < 0:
        raise MemoryError("oracle_components failed")
    return labels[:n], sizes[:n], nc.value, int(lcc)


def robustness(pairs, n: int, order, removed):
    """LCC size after removing order[:r] for each r in removed."""
    lib = load()
    p, E = _pairs_arg(pairs)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    removed = np.ascontiguousarray(removed, dtype=np.uint32)
    out = np.zeros(max(1, len(removed)), dtype=np.uint32)
    rc = lib.oracle_robustness(p.ctypes.data, E, n, order.ctypes.data if n else None, removed.ctypes.data,
                               len(removed), out.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle_robustness failed")
    return out[:len(removed)]


def lcc_norm1(lcc, removed, n: int):
    """Paper, Methods, "Computing LCC": LCC(p) / ((1 - p) N), p = removed / N."""
    lcc = np.asarray(lcc, dtype=np.float64)
    alive = n - np.asarray(removed, dtype=np.float64)
    return np.where(alive > 0, lcc / np.maximum(alive, 1), 0.0)


def lcc_norm2(lcc, removed, n: int):
    """LCC_norm,1(p) / LCC_norm,1(0); removed[0] must be 0."""
    r = np.asarray(removed)
    assert r[0] == 0
    v = lcc_norm1(lcc, removed, n)
    return v / v[0] if v[0] > 0 else v


def graph_stats(pairs, n: int, hist_len: int | None = None):
    """Degree statistics, assortativity and clustering (see graph.c)."""
    lib = load()
    if not hasattr(lib, "_stats_bound"):
        lib.oracle_graph_stats.restype = ctypes.c_int64
        lib.oracle_graph_stats.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32] + [ctypes.c_void_p] * 3 + \
            [ctypes.c_uint32] + [ctypes.c_void_p] * 5
        lib._stats_bound = True
    p, E = _pairs_arg(pairs)
    hist_len = hist_len or (n + 1)
    deg = np.zeros(max(1, n), dtype=np.int32)
    cnt = np.zeros(max(1, hist_len), dtype=np.uint64)
    nbr = np.zeros(max(1, hist_len), dtype=np.uint64)
    tri = np.zeros(max(1, n), dtype=np.uint64)
    clu = np.zeros(max(1, n), dtype=np.float64)
    r = ctypes.c_double()
    avg = ctypes.c_double()
    t3 = ctypes.c_uint64()
    maxd = lib.oracle_graph_stats(p.ctypes.data, E, n, deg.ctypes.data, cnt.ctypes.data, nbr.ctypes.data, hist_len,
                                  tri.ctypes.data, clu.ctypes.data, ctypes.byref(r), ctypes.byref(avg),
                                  ctypes.byref(t3))
    if maxd == -1:
        raise MemoryError("oracle_graph_stats failed")
    if maxd == -2:
        raise ValueError("hist_len too small")
    return {"degree": deg[:n], "max_degree": int(maxd), "count": cnt[:maxd + 1], "nbr_sum": nbr[:maxd + 1],
            "triangles_per_node": tri[:n], "clustering": clu[:n], "assortativity": r.value,
            "avg_clustering": avg.value, "triangles": t3.value}
