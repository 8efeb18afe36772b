"""Pins for the oracle's hyperedge sampler (Sec. 3.1 hyperedge space, Sec. 5
sampling procedure; readings R3-R6).

Levels are pinned to networkx distances, path counts to enumeration of all
shortest paths and to the grid closed form C(r+c, r), sampled hyperedges to
being internal nodes of a shortest s-t path, and the sampling distribution to
uniformity over pairs and over the shortest paths of a fixed pair.  The set
betweenness estimate is pinned to the exact value computed by enumeration.
"""
import itertools
import math

import networkx as nx
import numpy as np
import pytest

import oracle
from paper_2306_03651_amd import inputs

UNSEEN = 0xFFFFFFFF


def to_nx(g):
    G = nx.DiGraph() if g.directed else nx.Graph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            G.add_edge(u, int(g.col_idx[e]))
    return G


def random_digraph(n, p, seed):
    rng = np.random.default_rng(seed)
    src, dst = np.nonzero(rng.random((n, n)) < p)
    return inputs.from_edges(n, src, dst, directed=True)


GRAPHS = {
    "ba200": lambda: inputs.ba_graph(200, 3, 7),
    "grid6": lambda: inputs.grid_graph(6),
    "dir60": lambda: random_digraph(60, 0.05, 3),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_graph_contract(name):
    assert oracle.graph_check(GRAPHS[name]()) == 0


@pytest.mark.parametrize("name", list(GRAPHS))
def test_levels_and_exact_counts_match_enumeration(name):
    g = GRAPHS[name]()
    G = to_nx(g)
    for s in [0, 5, g.n - 1]:
        level, sigma = oracle.bfs_counts(g, s)
        dist = nx.single_source_shortest_path_length(G, s)
        for v in range(g.n):
            if v in dist:
                assert level[v] == dist[v]
            else:
                assert level[v] == UNSEEN and sigma[v] == 0
        # counts are exact here (no level needs more than C bits)
        for v in list(dist)[:40]:
            if v == s:
                assert sigma[v] == 1
                continue
            npaths = sum(1 for _ in nx.all_shortest_paths(G, s, v))
            assert sigma[v] == npaths, (s, v)


def test_grid_counts_closed_form():
    L = 20
    g = inputs.grid_graph(L)
    level, sigma = oracle.bfs_counts(g, 0)
    for r in range(L):
        for c in range(L):
            v = r * L + c
            assert level[v] == r + c
            assert int(sigma[v]) == math.comb(r + c, r)


@pytest.mark.parametrize("c_bits", [4, 8, 13])
def test_grid_normalised_counts(c_bits):
    # With a small count budget C the counts of a level whose largest raw
    # count needs b > C bits are shifted right by b - C and clamped to >= 1
    # (reading R4).  On a grid the raw counts follow Pascal's rule along
    # anti-diagonals; recompute them that way with Python integers.
    L = 24
    g = inputs.grid_graph(L)
    level, sigma = oracle.bfs_counts(g, 0, c_bits=c_bits)
    norm = {(0, 0): 1}
    for d in range(1, 2 * L - 1):
        cells = [(r, d - r) for r in range(max(0, d - L + 1), min(d, L - 1) + 1)]
        raw = {(r, c): norm.get((r - 1, c), 0) + norm.get((r, c - 1), 0) for r, c in cells}
        shift = max(0, max(raw.values()).bit_length() - c_bits)
        for cell, x in raw.items():
            norm[cell] = max(1, x >> shift)
    for (r, c), x in norm.items():
        assert int(sigma[r * L + c]) == x
        assert 1 <= x < 2**c_bits
    # the first diagonal that needs a shift keeps the exact binomials' top bits
    first = next(d for d in range(2 * L - 1) if math.comb(d, d // 2).bit_length() > c_bits)
    sh = math.comb(first, first // 2).bit_length() - c_bits
    for r in range(max(0, first - L + 1), min(first, L - 1) + 1):
        assert int(sigma[r * L + first - r]) == max(1, math.comb(first, r) >> sh)


def test_count_bits():
    g = inputs.ba_graph(2000, 5, 1)
    dmax = int(np.diff(g.row_ptr.astype(np.int64)).max())
    assert oracle.count_bits(g) == 63 - dmax.bit_length()


def test_count_bits_directed_uses_in_degree():
    # Reading R4 budgets the counts by the largest in-degree (a level's raw
    # count is a sum over in-neighbours).  On this directed graph the
    # largest in-degree (8, from the transpose) is far below the largest
    # out-degree (600), so C = 59, not 52; the counts from node 0 cross
    # 2^C, and every normalised count equals a recomputation with Python
    # integers level by level (BFS levels over out-arcs, raw sums over
    # in-neighbours one level up, the level's shift, the clamp to 1).
    g = inputs.layered_dag()
    indeg = np.bincount(g.col_idx.astype(np.int64), minlength=g.n)
    outdeg = np.diff(g.row_ptr.astype(np.int64))
    assert indeg.max() == 8 and outdeg.max() == 600
    C = 63 - int(indeg.max()).bit_length()
    assert oracle.count_bits(g) == C == 59
    level, sigma = oracle.bfs_counts(g, 0)
    # Python reference, independent of the oracle's BFS
    preds = [[] for _ in range(g.n)]
    for u in range(g.n):
        for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            preds[int(g.col_idx[e])].append(u)
    lev = {0: 0}
    frontier, d = [0], 0
    while frontier:
        nxt = []
        for u in frontier:
            for e in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
                v = int(g.col_idx[e])
                if v not in lev:
                    lev[v] = d + 1
                    nxt.append(v)
        frontier, d = nxt, d + 1
    norm = {0: 1}
    shifted = 0
    for L in range(1, d):
        cells = [v for v, x in lev.items() if x == L]
        raw = {v: sum(norm[w] for w in preds[v] if lev.get(w) == L - 1) for v in cells}
        shift = max(0, max(raw.values()).bit_length() - C)
        shifted += shift > 0
        for v, x in raw.items():
            norm[v] = max(1, x >> shift)
    assert shifted >= 5
    for v, L in lev.items():
        assert int(level[v]) == L
        assert int(sigma[v]) == norm[v], v
    # with the out-degree budget (C = 52) the counts would differ
    level52, sigma52 = oracle.bfs_counts(g, 0, c_bits=63 - int(outdeg.max()).bit_length())
    assert any(int(sigma52[v]) != norm[v] for v in lev)


BAD_GRAPHS = {
    "n_below_2": lambda g: inputs.CSRGraph(1, False, np.array([0, 0], np.uint32), np.zeros(0, np.uint32)),
    "unsorted_row": lambda g: _with_col(g, lambda c: c.__setitem__(slice(0, 2), c[[1, 0]])),
    "duplicate": lambda g: _with_col(g, lambda c: c.__setitem__(1, c[0])),
    "self_loop": lambda g: _with_col(g, lambda c: c.__setitem__(0, 0)),
    "out_of_range": lambda g: _with_col(g, lambda c: c.__setitem__(len(c) - 1, g.n)),
}


def _with_col(g, edit):
    col = g.col_idx.copy()
    edit(col)
    return inputs.CSRGraph(g.n, False, g.row_ptr, col)


@pytest.mark.parametrize("name", list(BAD_GRAPHS))
def test_graph_check_rejects(name):
    # a star rooted at 0 whose row 0 is 1, 2, ... : each edit breaks one
    # rule of the graph contract (rows sorted ascending, no duplicates, no
    # self loops, ids below n, n >= 2)
    g = inputs.from_edges(20, np.zeros(19, np.int64), np.arange(1, 20), directed=False)
    assert oracle.graph_check(g) == 0
    assert oracle.graph_check(BAD_GRAPHS[name](g)) != 0


def test_graph_check_rejects_wrong_reverse_rows():
    d = random_digraph(40, 0.1, 1)
    assert oracle.graph_check(d) == 0
    # a reverse CSR with one in-arc moved to another row
    rrow = d.rrow_ptr.copy()
    v = int(np.argmax(np.diff(rrow.astype(np.int64)) > 0))
    rrow[v + 1] -= 1
    bad = inputs.CSRGraph(d.n, True, d.row_ptr, d.col_idx, rrow, d.rcol_idx)
    assert oracle.graph_check(bad) != 0
    # a sorted in-row with one source replaced by a node that has no such arc
    rcol = d.rcol_idx.copy()
    row = set(int(x) for x in rcol[d.rrow_ptr[v]:d.rrow_ptr[v + 1]])
    repl = next(u for u in range(d.n) if u not in row and u != v)
    rcol[d.rrow_ptr[v]] = repl
    rcol[d.rrow_ptr[v]:d.rrow_ptr[v + 1]] = np.sort(rcol[d.rrow_ptr[v]:d.rrow_ptr[v + 1]])
    bad = inputs.CSRGraph(d.n, True, d.row_ptr, d.col_idx, d.rrow_ptr, rcol)
    assert oracle.graph_check(bad) != 0


@pytest.mark.parametrize("name", list(GRAPHS))
def test_sampled_hyperedges_are_shortest_path_interiors(name):
    g = GRAPHS[name]()
    G = to_nx(g)
    off, nodes, infos = oracle.sample_paths(g, 17, 0, 0, 400, with_info=True)
    for i, inf in enumerate(infos):
        h = [int(x) for x in nodes[int(off[i]):int(off[i + 1])]]
        assert inf.s != inf.t
        if not nx.has_path(G, inf.s, inf.t):
            assert inf.dist == UNSEEN and h == []
            continue
        d = nx.shortest_path_length(G, inf.s, inf.t)
        assert inf.dist == d
        assert len(h) == max(0, d - 1)
        # backtrack order: t's neighbour first
        path = [inf.t] + h + [inf.s]
        for a, b in zip(path[1:], path[:-1]):
            assert G.has_edge(a, b)
        assert len(set(h)) == len(h)


def test_pair_uniform():
    g = inputs.grid_graph(3)
    n = g.n
    _, _, infos = oracle.sample_paths(g, 5, 0, 0, 36000, with_info=True)
    counts = np.zeros((n, n))
    for inf in infos:
        counts[inf.s, inf.t] += 1
    assert np.all(np.diag(counts) == 0)
    cells = counts[~np.eye(n, dtype=bool)]
    exp = len(infos) / (n * (n - 1))
    chi2 = ((cells - exp) ** 2 / exp).sum()
    dof = n * (n - 1) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_paths_uniform_for_fixed_pair():
    # 3x3 grid, corner 0 -> corner 8: C(4,2) = 6 shortest paths.
    g = inputs.grid_graph(3)
    _, nodes_all, infos = None, None, None
    off, nodes, infos = oracle.sample_paths(g, 23, 1, 0, 72000, with_info=True)
    seen = {}
    for i, inf in enumerate(infos):
        if (inf.s, inf.t) == (0, 8):
            key = tuple(int(x) for x in nodes[int(off[i]):int(off[i + 1])])
            seen[key] = seen.get(key, 0) + 1
    assert len(seen) == 6
    c = np.array(list(seen.values()), dtype=float)
    exp = c.sum() / 6
    assert ((c - exp) ** 2 / exp).sum() < 5 + 6 * math.sqrt(10)


def test_paths_uniform_with_unequal_counts():
    # A graph where predecessors carry different path counts: s=0 reaches
    # node 4 via 1 path (0-1-4) and via node 5 with 2 paths (0-2-5, 0-3-5),
    # and 4, 5 both precede t=6.  Three shortest 0->6 paths, each must get
    # probability 1/3.
    edges = [(0, 1), (0, 2), (0, 3), (1, 4), (2, 5), (3, 5), (4, 6), (5, 6)]
    src, dst = zip(*edges)
    g = inputs.from_edges(7, src, dst, directed=True)
    off, nodes, infos = oracle.sample_paths(g, 3, 0, 0, 120000, with_info=True)
    seen = {}
    for i, inf in enumerate(infos):
        if (inf.s, inf.t) == (0, 6):
            key = tuple(int(x) for x in nodes[int(off[i]):int(off[i + 1])])
            seen[key] = seen.get(key, 0) + 1
    assert set(seen) == {(4, 1), (5, 2), (5, 3)}
    c = np.array([seen[(4, 1)], seen[(5, 2)], seen[(5, 3)]], dtype=float)
    exp = c.sum() / 3
    assert ((c - exp) ** 2 / exp).sum() < 2 + 6 * 2


def test_unreachable_and_adjacent_give_empty():
    # directed path 0 -> 1 -> 2 plus isolated node 3
    g = inputs.from_edges(4, [0, 1], [1, 2], directed=True)
    off, nodes, infos = oracle.sample_paths(g, 8, 0, 0, 2000, with_info=True)
    for i, inf in enumerate(infos):
        h = [int(x) for x in nodes[int(off[i]):int(off[i + 1])]]
        if (inf.s, inf.t) == (0, 2):
            assert h == [1]
        else:
            assert h == []


def exact_set_betweenness(G, n, S):
    """C(S) by enumeration over all ordered pairs and all shortest paths (Sec. 3.1)."""
    tot = 0.0
    for u, v in itertools.permutations(range(n), 2):
        if not nx.has_path(G, u, v):
            continue
        paths = list(nx.all_shortest_paths(G, u, v))
        hit = sum(1 for p in paths if any(x in S for x in p[1:-1]))
        tot += hit / len(paths)
    return tot / (n * (n - 1))


def test_estimator_matches_exact_set_betweenness():
    g = inputs.ba_graph(40, 2, 3)
    G = to_nx(g)
    m = 20000
    off, nodes = oracle.sample_paths(g, 99, 0, 0, m)
    for S in [{0}, {1, 2}, {5, 9, 13}]:
        exact = exact_set_betweenness(G, g.n, S)
        hits = sum(1 for i in range(m) if any(int(x) in S for x in nodes[int(off[i]):int(off[i + 1])]))
        est = hits / m
        sd = math.sqrt(exact * (1 - exact) / m)
        assert abs(est - exact) < 5 * sd + 1e-9, (S, est, exact)


def test_sample_stream_prefix_property():
    g = inputs.ba_graph(300, 3, 2)
    off_a, nodes_a = oracle.sample_paths(g, 4, 1, 0, 500)
    off_b, nodes_b = oracle.sample_paths(g, 4, 1, 0, 230)
    off_c, nodes_c = oracle.sample_paths(g, 4, 1, 230, 270)
    assert np.array_equal(nodes_a, np.concatenate([nodes_b, nodes_c]))
    assert np.array_equal(off_a[:231], off_b)
    assert np.array_equal(off_a[230:] - off_a[230], off_c)
