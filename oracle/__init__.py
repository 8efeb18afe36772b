"""ctypes access to the CPU oracle (centra_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  The oracle is a
plain, slow implementation of the CentRA hot path written from the paper
(Pellegrina, KDD 2023); see centra_oracle.c for the readings it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "centra_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_centra.so")
_lib = None

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("directed", ctypes.c_uint32), ("n_arcs", ctypes.c_uint64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("rrow_ptr", ctypes.c_void_p), ("rcol_idx", ctypes.c_void_p)]


class SampleInfo(ctypes.Structure):
    _fields_ = [("s", ctypes.c_uint32), ("t", ctypes.c_uint32), ("dist", ctypes.c_uint32),
                ("len", ctypes.c_uint32), ("arcs_scanned", ctypes.c_uint64),
                ("nodes_visited", ctypes.c_uint64)]


class BoundOut(ctypes.Structure):
    _fields_ = [("c_hat", ctypes.c_double), ("amcera", ctypes.c_double), ("wimpy", ctypes.c_double),
                ("xi", ctypes.c_double), ("nu", ctypes.c_double), ("rtilde", ctypes.c_double),
                ("r", ctypes.c_double), ("eta", ctypes.c_double), ("certified", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("n_picked", ctypes.c_uint32), ("iterations", ctypes.c_uint32),
                ("certified", ctypes.c_int), ("coverage", ctypes.c_uint64), ("m_final", ctypes.c_uint64),
                ("c_hat", ctypes.c_double), ("amcera", ctypes.c_double), ("wimpy", ctypes.c_double),
                ("xi", ctypes.c_double), ("nu", ctypes.c_double), ("rtilde", ctypes.c_double),
                ("r", ctypes.c_double), ("eta", ctypes.c_double)]


def build() -> str:
    """Compiles the oracle library in place (plain C, gcc) and returns its path."""
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                           _SRC, "-o", _LIB + ".tmp", "-lm"])
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    c = ctypes
    lib.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.orc_philox4x64_10.restype = None
    lib.orc_bounded_many.argtypes = [c.c_uint64, c.c_uint64, c.c_uint64, c.c_uint64, c.c_uint64,
                                     c.c_uint64, _u64p]
    lib.orc_bounded_many.restype = None
    lib.orc_graph_check.argtypes = [c.POINTER(Graph)]
    lib.orc_graph_check.restype = c.c_int
    lib.orc_count_bits.argtypes = [c.POINTER(Graph)]
    lib.orc_count_bits.restype = c.c_uint32
    lib.orc_sample_path.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_uint64, c.c_uint32, c.c_uint64,
                                    _u32p, c.POINTER(SampleInfo)]
    lib.orc_sample_path.restype = c.c_uint32
    lib.orc_sample_paths.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_uint64, c.c_uint32, c.c_uint64,
                                     c.c_uint64, _u64p, _u32p, c.c_uint64, c.c_void_p]
    lib.orc_sample_paths.restype = c.c_uint64
    lib.orc_count_bits_out.argtypes = [c.POINTER(Graph)]
    lib.orc_count_bits_out.restype = c.c_uint32
    lib.orc_sample_paths_bidir.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_uint32, c.c_uint64, c.c_uint32,
                                           c.c_uint64, c.c_uint64, _u64p, _u32p, c.c_uint64, c.c_void_p]
    lib.orc_sample_paths_bidir.restype = c.c_uint64
    lib.orc_bfs_counts.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_uint32, _u32p, _u64p]
    lib.orc_bfs_counts.restype = None
    lib.orc_greedy_cover.argtypes = [c.c_uint32, c.c_uint64, _u64p, _u32p, c.c_uint32, _u32p, _u64p]
    lib.orc_greedy_cover.restype = c.c_uint32
    lib.orc_rademacher.argtypes = [c.c_uint64, c.c_uint32, c.c_uint64, c.c_uint32]
    lib.orc_rademacher.restype = c.c_int
    lib.orc_rade_sums.argtypes = [c.c_uint32, c.c_uint64, _u64p, _u32p, c.c_uint64, c.c_uint32,
                                  c.c_uint32, _i64p]
    lib.orc_rade_sums.restype = None
    lib.orc_mcera.argtypes = [c.c_uint32, c.c_uint64, _u64p, _u32p, c.c_uint64, c.c_uint32, c.c_uint32,
                              c.c_uint32, _i64p, c.POINTER(c.c_uint64), c.POINTER(c.c_uint32)]
    lib.orc_mcera.restype = c.c_double
    lib.orc_bound.argtypes = [c.c_uint64, c.c_uint64, c.c_int64, c.c_uint32, c.c_uint64, c.c_uint32,
                              c.c_double, c.c_double, c.POINTER(BoundOut)]
    lib.orc_bound.restype = None
    lib.orc_progressive.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_uint32, c.c_uint32, c.c_double,
                                    c.c_double, c.c_uint64, c.c_uint32, c.c_uint64, c.c_uint64,
                                    c.c_uint32, c.c_uint32, c.c_uint32, c.c_uint32, c.c_uint32, c.c_uint32,
                                    _u32p, c.POINTER(Result), _u64p, c.c_uint32]
    lib.orc_log_sets.argtypes = [c.c_uint64, c.c_uint32]
    lib.orc_log_sets.restype = c.c_double
    lib.orc_hedge_bound.argtypes = [c.c_uint64, c.c_uint64, c.c_uint64, c.c_uint32, c.c_double, c.c_double,
                                    c.POINTER(BoundOut)]
    lib.orc_hedge_bound.restype = None
    lib.orc_vc_dims.argtypes = [c.c_uint64, c.c_uint32, c.c_uint64, c.POINTER(c.c_uint32), c.POINTER(c.c_uint64),
                                c.POINTER(c.c_uint64)]
    lib.orc_vc_dims.restype = c.c_int
    lib.orc_kpath.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_uint64, c.c_uint32, c.c_uint64, _u32p,
                              c.POINTER(c.c_uint32), c.POINTER(c.c_uint32)]
    lib.orc_kpath.restype = c.c_uint32
    lib.orc_sample_kpaths.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_uint64, c.c_uint32, c.c_uint64,
                                      c.c_uint64, _u64p, _u32p]
    lib.orc_sample_kpaths.restype = c.c_int
    lib.orc_triangles.argtypes = [c.POINTER(Graph), c.c_void_p, c.c_uint64]
    lib.orc_triangles.restype = c.c_uint64
    lib.orc_row_triangles.argtypes = [c.POINTER(Graph), c.c_uint32, c.c_void_p, c.c_uint64]
    lib.orc_row_triangles.restype = c.c_uint64
    lib.orc_sample_triangles.argtypes = [c.POINTER(Graph), c.c_uint64, c.c_uint32, c.c_uint64, c.c_uint64,
                                         _u64p, _u32p]
    lib.orc_sample_triangles.restype = c.c_int
    lib.orc_next_sample_size.argtypes = [c.c_uint64, c.c_double, c.c_double, c.c_double, c.c_uint32,
                                         c.c_uint32, c.c_uint64, c.c_uint32]
    lib.orc_next_sample_size.restype = c.c_uint64
    lib.orc_progressive.restype = c.c_int
    _lib = lib
    return lib


class OracleGraph:
    """Keeps the numpy arrays alive behind the C graph struct."""

    def __init__(self, g):
        self.g = g
        self._keep = [np.ascontiguousarray(g.row_ptr, dtype=np.uint32),
                      np.ascontiguousarray(g.col_idx, dtype=np.uint32)]
        if g.directed:
            self._keep += [np.ascontiguousarray(g.rrow_ptr, dtype=np.uint32),
                           np.ascontiguousarray(g.rcol_idx, dtype=np.uint32)]
        ptrs = [a.ctypes.data for a in self._keep]
        self.c = Graph(g.n, 1 if g.directed else 0, int(g.row_ptr[-1]), ptrs[0], ptrs[1],
                       ptrs[2] if g.directed else None, ptrs[3] if g.directed else None)


def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64_10(np.asarray(ctr, dtype=np.uint64), np.asarray(key, dtype=np.uint64), out)
    return out


def bounded_many(seed, c1, c2, c3, W, count):
    out = np.zeros(count, dtype=np.uint64)
    _load().orc_bounded_many(seed, c1, c2, c3, W, count, out)
    return out


def graph_check(g) -> int:
    og = OracleGraph(g)
    return _load().orc_graph_check(ctypes.byref(og.c))


def count_bits(g) -> int:
    og = OracleGraph(g)
    return _load().orc_count_bits(ctypes.byref(og.c))


def sample_path(g, seed, instance, sample, c_bits=None, og=None):
    """Returns (hyperedge nodes as np.uint32 array, SampleInfo)."""
    og = og or OracleGraph(g)
    lib = _load()
    if c_bits is None:
        c_bits = lib.orc_count_bits(ctypes.byref(og.c))
    h = np.zeros(g.n, dtype=np.uint32)
    info = SampleInfo()
    ln = lib.orc_sample_path(ctypes.byref(og.c), c_bits, seed, instance, sample, h, ctypes.byref(info))
    return h[:ln].copy(), info


def sample_paths(g, seed, instance, first, count, c_bits=None, with_info=False):
    """Samples [first, first+count): returns (he_off u64[count+1], he_nodes u32[I][, infos])."""
    og = OracleGraph(g)
    lib = _load()
    if c_bits is None:
        c_bits = lib.orc_count_bits(ctypes.byref(og.c))
    cap = max(16, count * 8)
    while True:
        he_off = np.zeros(count + 1, dtype=np.uint64)
        he_nodes = np.zeros(cap, dtype=np.uint32)
        infos = (SampleInfo * max(1, count))() if with_info else None
        tot = lib.orc_sample_paths(ctypes.byref(og.c), c_bits, seed, instance, first, count, he_off,
                                   he_nodes, cap, ctypes.cast(infos, ctypes.c_void_p) if with_info else None)
        if tot != 2**64 - 1:
            break
        cap *= 4
    res = (he_off, he_nodes[:tot].copy())
    if with_info:
        return res + (list(infos)[:count],)
    return res


def count_bits_out(g) -> int:
    og = OracleGraph(g)
    return _load().orc_count_bits_out(ctypes.byref(og.c))


def sample_paths_bidir(g, seed, instance, first, count, c_f=None, c_b=None, with_info=False):
    """The balanced bidirectional sampler (reading R16): samples [first,
    first+count) -> (he_off u64[count+1], he_nodes u32[I][, infos])."""
    og = OracleGraph(g)
    lib = _load()
    if c_f is None:
        c_f = lib.orc_count_bits(ctypes.byref(og.c))
    if c_b is None:
        c_b = lib.orc_count_bits_out(ctypes.byref(og.c))
    cap = max(16, count * 8)
    while True:
        he_off = np.zeros(count + 1, dtype=np.uint64)
        he_nodes = np.zeros(cap, dtype=np.uint32)
        infos = (SampleInfo * max(1, count))() if with_info else None
        tot = lib.orc_sample_paths_bidir(ctypes.byref(og.c), c_f, c_b, seed, instance, first, count, he_off,
                                         he_nodes, cap, ctypes.cast(infos, ctypes.c_void_p) if with_info else None)
        if tot != 2**64 - 1:
            break
        cap *= 4
    res = (he_off, he_nodes[:tot].copy())
    if with_info:
        return res + (list(infos)[:count],)
    return res


def bfs_counts(g, s, c_bits=None):
    og = OracleGraph(g)
    lib = _load()
    if c_bits is None:
        c_bits = lib.orc_count_bits(ctypes.byref(og.c))
    level = np.zeros(g.n, dtype=np.uint32)
    sigma = np.zeros(g.n, dtype=np.uint64)
    lib.orc_bfs_counts(ctypes.byref(og.c), c_bits, s, level, sigma)
    return level, sigma


def greedy_cover(n, he_off, he_nodes, k):
    m = len(he_off) - 1
    picks = np.zeros(max(1, k), dtype=np.uint32)
    cov = np.zeros(max(1, k), dtype=np.uint64)
    cnt = _load().orc_greedy_cover(n, m, np.ascontiguousarray(he_off, dtype=np.uint64),
                                   np.ascontiguousarray(he_nodes, dtype=np.uint32), k, picks, cov)
    return picks[:cnt].copy(), cov[:cnt].copy()


def rademacher(seed, instance, s, j) -> int:
    return _load().orc_rademacher(seed, instance, s, j)


def rade_sums(n, he_off, he_nodes, seed, instance, t):
    m = len(he_off) - 1
    R = np.zeros(n * t, dtype=np.int64)
    _load().orc_rade_sums(n, m, np.ascontiguousarray(he_off, dtype=np.uint64),
                          np.ascontiguousarray(he_nodes, dtype=np.uint32), seed, instance, t, R)
    return R.reshape(n, t)


def mcera(n, he_off, he_nodes, seed, instance, t, k):
    """Returns (amcera, topk_sum int64[t], deg_topk, b_max)."""
    m = len(he_off) - 1
    topk = np.zeros(t, dtype=np.int64)
    dk = ctypes.c_uint64()
    bm = ctypes.c_uint32()
    a = _load().orc_mcera(n, m, np.ascontiguousarray(he_off, dtype=np.uint64),
                          np.ascontiguousarray(he_nodes, dtype=np.uint32), seed, instance, t, k, topk,
                          ctypes.byref(dk), ctypes.byref(bm))
    return a, topk, dk.value, bm.value


def bound(m, cov, sum_topk, t, deg_topk, b_max, eps, delta_i) -> BoundOut:
    out = BoundOut()
    _load().orc_bound(m, cov, sum_topk, t, deg_topk, b_max, eps, delta_i, ctypes.byref(out))
    return out


SCHEDULE_GEOMETRIC, SCHEDULE_ADAPTIVE, SCHEDULE_FIXED = 0, 1, 2


def next_sample_size(m_i, c_hat, eps, delta_next, growth_num, growth_den, m_max, schedule):
    """samplingSchedule of Algorithm 1: m_{i+1} after an iteration at m_i."""
    return int(_load().orc_next_sample_size(m_i, c_hat, eps, delta_next, growth_num, growth_den, m_max,
                                            schedule))


SPACE_SHORTEST_PATHS, SPACE_TRIANGLES, SPACE_KPATHS, SPACE_PATHS_BIDIR = 0, 1, 2, 3


def triangles(g):
    """All triangles (a < b < c) in rank order, as an int array of shape
    (T, 3); None for a directed graph."""
    og = OracleGraph(g)
    lib = _load()
    T = lib.orc_triangles(ctypes.byref(og.c), None, 0)
    if T == 2**64 - 1:
        return None
    tri = np.zeros(3 * max(1, T), dtype=np.uint32)
    lib.orc_triangles(ctypes.byref(og.c), tri.ctypes.data, T)
    return tri[: 3 * T].reshape(T, 3)


def row_triangle_count(g, a, og=None):
    """Number of triangles whose smallest node is a (None if directed)."""
    og = og or OracleGraph(g)
    T = _load().orc_row_triangles(ctypes.byref(og.c), a, None, 0)
    return None if T == 2**64 - 1 else T


def sample_triangles(g, seed, instance, first, count):
    """Triangle hyperedges [first, first+count): (he_off, he_nodes); None if
    the graph is directed or has no triangle."""
    og = OracleGraph(g)
    off = np.zeros(count + 1, dtype=np.uint64)
    nodes = np.zeros(3 * max(1, count), dtype=np.uint32)
    rc = _load().orc_sample_triangles(ctypes.byref(og.c), seed, instance, first, count, off, nodes)
    return None if rc else (off, nodes[: 3 * count])


def vc_dims(b, k, n):
    """(d1, dk_lemma, dk_union) of Sec. 4.3's VC bounds; None if b, k or n is 0."""
    d1, dl, du = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    if _load().orc_vc_dims(b, k, n, ctypes.byref(d1), ctypes.byref(dl), ctypes.byref(du)):
        return None
    return d1.value, dl.value, du.value


def kpath(g, kappa, seed, instance, sample, og=None):
    """Sample `sample` of the kappa-path space: (walk after its start as a
    np.uint32 array, start s, drawn length l)."""
    og = og or OracleGraph(g)
    h = np.zeros(max(1, kappa), dtype=np.uint32)
    s_out, l_out = ctypes.c_uint32(), ctypes.c_uint32()
    ln = _load().orc_kpath(ctypes.byref(og.c), kappa, seed, instance, sample, h, ctypes.byref(s_out),
                           ctypes.byref(l_out))
    return h[:ln].copy(), s_out.value, l_out.value


def sample_kpaths(g, kappa, seed, instance, first, count):
    """kappa-path hyperedges [first, first+count): (he_off, he_nodes); None
    if kappa == 0."""
    og = OracleGraph(g)
    off = np.zeros(count + 1, dtype=np.uint64)
    nodes = np.zeros(max(1, count * kappa), dtype=np.uint32)
    rc = _load().orc_sample_kpaths(ctypes.byref(og.c), kappa, seed, instance, first, count, off, nodes)
    return None if rc else (off, nodes[: int(off[-1])])


def log_sets(n, k) -> float:
    return _load().orc_log_sets(n, k)


def hedge_bound(m, cov, n, k, eps, delta_i) -> BoundOut:
    o = BoundOut()
    _load().orc_hedge_bound(m, cov, n, k, eps, delta_i, ctypes.byref(o))
    return o


METHOD_CENTRA, METHOD_HEDGE_P = 0, 1


def progressive(g, k, t, eps, delta, seed, instance, m_init, m_max, growth_num=2, growth_den=1,
                c_bits=None, schedule=SCHEDULE_GEOMETRIC, with_m_log=False, space=SPACE_SHORTEST_PATHS,
                kappa=0, method=METHOD_CENTRA):
    """Algorithm 1; returns (rc, picks, Result) and, with with_m_log, the
    sample size of every iteration."""
    og = OracleGraph(g)
    lib = _load()
    if c_bits is None:
        c_bits = lib.orc_count_bits(ctypes.byref(og.c))
    picks = np.zeros(max(1, k), dtype=np.uint32)
    res = Result()
    m_log = np.zeros(256, dtype=np.uint64)
    rc = lib.orc_progressive(ctypes.byref(og.c), c_bits, k, t, eps, delta, seed, instance, m_init, m_max,
                             growth_num, growth_den, schedule, space, kappa, method, picks, ctypes.byref(res), m_log,
                             len(m_log))
    out = (rc, picks[: res.n_picked].copy(), res)
    if with_m_log:
        out = out + ([int(x) for x in m_log[: min(res.iterations, len(m_log))]],)
    return out
