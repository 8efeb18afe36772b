"""Seeded synthetic inputs: graphs in CSR form and synthetic hyperedge sets.

The paper's experiments (Sec. 5 and the graph table of the appendix) run on
SNAP / KONECT networks that are not available here.  These generators stand
in for them with the same shapes (Barabasi-Albert for the scale-free
undirected graphs, R-MAT for the skewed directed ones, 2D grids for long
diameters).  They use their own generator (SplitMix64), hold none of the
method's arithmetic, and feed the HIP path and the oracle alike.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compiles the generator library in place and returns its path."""
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"])
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.gg_ba_arcs.restype = ctypes.c_uint64
    lib.gg_ba_arcs.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.gg_ba.restype = ctypes.c_uint64
    lib.gg_ba.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, _u32p, _u32p]
    lib.gg_grid.restype = ctypes.c_uint64
    lib.gg_grid.argtypes = [ctypes.c_uint32, _u32p, _u32p]
    lib.gg_rmat.restype = ctypes.c_uint64
    lib.gg_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, _u32p, _u32p]
    lib.gg_reverse.restype = None
    lib.gg_reverse.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u32p, _u32p]
    lib.gg_hyperedges.restype = ctypes.c_uint64
    lib.gg_hyperedges.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint64, _u64p, _u32p]
    _lib = lib
    return lib


@dataclasses.dataclass
class CSRGraph:
    """CSR graph: rows sorted ascending, no duplicates, no self loops.

    For a directed graph ``rrow_ptr``/``rcol_idx`` hold the in-neighbours;
    for an undirected graph they are None (the in-rows are the out-rows).
    """
    n: int
    directed: bool
    row_ptr: np.ndarray
    col_idx: np.ndarray
    rrow_ptr: np.ndarray | None = None
    rcol_idx: np.ndarray | None = None
    name: str = ""

    @property
    def n_arcs(self) -> int:
        return int(self.row_ptr[-1])

    def in_rows(self):
        if self.directed:
            return self.rrow_ptr, self.rcol_idx
        return self.row_ptr, self.col_idx


def from_edges(n: int, src, dst, directed: bool, name: str = "") -> CSRGraph:
    """CSR from an edge list (undirected edges are stored both ways)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if not directed:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    keep = src != dst
    key = np.unique(src[keep] * n + dst[keep])
    s = (key // n).astype(np.uint32)
    d = (key % n).astype(np.uint32)
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    np.add.at(row_ptr, s.astype(np.int64) + 1, 1)
    row_ptr = np.cumsum(row_ptr, dtype=np.uint64).astype(np.uint32)
    g = CSRGraph(n, directed, row_ptr, np.ascontiguousarray(d), name=name)
    if directed:
        g.rrow_ptr, g.rcol_idx = reverse(n, g.row_ptr, g.col_idx)
    return g


def reverse(n: int, row_ptr: np.ndarray, col_idx: np.ndarray):
    lib = _load()
    rrow = np.zeros(n + 1, dtype=np.uint32)
    rcol = np.zeros(max(1, int(row_ptr[-1])), dtype=np.uint32)
    lib.gg_reverse(n, row_ptr, col_idx, rrow, rcol)
    return rrow, rcol[: int(row_ptr[-1])]


def ba_graph(n: int, m0: int = 5, seed: int = 1) -> CSRGraph:
    """Undirected Barabasi-Albert graph (clique on 0..m0, then m0 edges per node)."""
    lib = _load()
    arcs = int(lib.gg_ba_arcs(n, m0))
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    col_idx = np.zeros(arcs, dtype=np.uint32)
    got = int(lib.gg_ba(n, m0, seed, row_ptr, col_idx))
    assert got == arcs, (got, arcs)
    return CSRGraph(n, False, row_ptr, col_idx, name=f"ba_n{n}_m{m0}_s{seed}")


def grid_graph(L: int) -> CSRGraph:
    """L x L 4-neighbour grid, undirected, node id r*L + c."""
    lib = _load()
    n = L * L
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    col_idx = np.zeros(max(1, 4 * L * (L - 1)), dtype=np.uint32)
    got = int(lib.gg_grid(L, row_ptr, col_idx))
    return CSRGraph(n, False, row_ptr, col_idx[:got], name=f"grid_{L}")


def rmat_graph(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1) -> CSRGraph:
    """Directed R-MAT graph, self loops and duplicates removed, with reverse CSR."""
    lib = _load()
    n = 1 << scale
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    col_idx = np.zeros(edge_factor << scale, dtype=np.uint32)
    got = int(lib.gg_rmat(scale, edge_factor, a, b, c, seed, row_ptr, col_idx))
    col_idx = np.ascontiguousarray(col_idx[:got])
    rrow, rcol = reverse(n, row_ptr, col_idx)
    return CSRGraph(n, True, row_ptr, col_idx, rrow, rcol, name=f"rmat_s{scale}_s{seed}")


def hyperedges(n: int, m: int, max_len: int = 8, skew: int = 3, seed: int = 1):
    """Synthetic hyperedge set (he_off u64[m+1], he_nodes u32[I]) shaped like
    shortest-path samples on a scale-free graph."""
    lib = _load()
    he_off = np.zeros(m + 1, dtype=np.uint64)
    he_nodes = np.zeros(max(1, m * max_len), dtype=np.uint32)
    total = int(lib.gg_hyperedges(n, m, max_len, skew, seed, he_off, he_nodes))
    return he_off, np.ascontiguousarray(he_nodes[:total])


def layered_dag(layers: int = 40, width: int = 12, max_in: int = 8, hub_out: int = 600,
                seed: int = 1) -> CSRGraph:
    """Directed layered graph whose maximum in-degree differs from its maximum
    out-degree: node 0 feeds every node of layer 1; each node of a later
    layer has 1..max_in in-neighbours drawn from the layer before (numpy
    generator of `seed`); a separate hub feeds `hub_out` leaves.  Path
    counts grow about max_in/2-fold per layer, so long pairs exceed 2^C."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    first = 1
    for v in range(first, first + width):
        src.append(0); dst.append(v)
    for L in range(1, layers):
        prev = first + (L - 1) * width
        cur = first + L * width
        for v in range(cur, cur + width):
            k = int(rng.integers(1, max_in + 1))
            for u in rng.choice(width, size=k, replace=False):
                src.append(prev + int(u)); dst.append(v)
    hub = first + layers * width
    for j in range(hub_out):
        src.append(hub); dst.append(hub + 1 + j)
    n = hub + 1 + hub_out
    return from_edges(n, src, dst, directed=True, name=f"layered_{layers}x{width}_s{seed}")


def uneven_instances(count: int = 256, seed: int = 1, ba_n=(1000, 100_000), grid_side=(64, 1024),
                     k=(5, 50)):
    """The uneven-instances mix: per instance, a Bernoulli(1/2) choice of a
    Barabasi-Albert graph (n uniform in ba_n, attachment 5) or an L x L grid
    (L uniform in grid_side), and k uniform in k (bounds inclusive); numpy
    generator of `seed`.  Returns [(kind, size, graph_seed, k)]; build the
    graphs with instance_graph."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if rng.random() < 0.5:
            out.append(("ba", int(rng.integers(ba_n[0], ba_n[1] + 1)), 1000 + i, int(rng.integers(k[0], k[1] + 1))))
        else:
            out.append(("grid", int(rng.integers(grid_side[0], grid_side[1] + 1)), 0, int(rng.integers(k[0], k[1] + 1))))
    return out


def instance_graph(kind: str, size: int, graph_seed: int) -> CSRGraph:
    return ba_graph(size, 5, graph_seed) if kind == "ba" else grid_graph(size)
