"""Pins of the oracle's triangle hyperedges (Sec. 3.1: the triangle
centrality's space of node sets of triangles, drawn uniformly): the ranked
triangle list against brute force and a closed form, the draw against the
bounded-draw definition, uniformity, the estimator against the exact
triangle centrality, and the progressive loop on this space."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2306_03651_amd import inputs


def gnp(n, p, seed):
    rng = np.random.default_rng(seed)
    a, b = np.nonzero(np.triu(rng.random((n, n)) < p, 1))
    return inputs.from_edges(n, a, b, directed=False)


def brute_triangles(g):
    adj = [set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
    return [t for t in itertools.combinations(range(g.n), 3)
            if t[1] in adj[t[0]] and t[2] in adj[t[0]] and t[2] in adj[t[1]]]


@pytest.mark.parametrize("n", [3, 4, 7, 12])
def test_complete_graph_closed_form(n):
    g = inputs.from_edges(n, *zip(*itertools.combinations(range(n), 2)), directed=False)
    tri = oracle.triangles(g)
    assert len(tri) == math.comb(n, 3)
    # rank order is lexicographic: the r-th 3-combination
    assert [tuple(t) for t in tri.tolist()] == list(itertools.combinations(range(n), 3))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_graph_brute_force(seed):
    g = gnp(40, 0.3, seed)
    assert [tuple(t) for t in oracle.triangles(g).tolist()] == brute_triangles(g)


def test_no_triangles_and_directed():
    grid = inputs.grid_graph(6)   # bipartite: no triangle
    assert len(oracle.triangles(grid)) == 0
    assert oracle.sample_triangles(grid, 1, 0, 0, 10) is None
    d = inputs.from_edges(3, [0, 1, 2], [1, 2, 0], directed=True)
    assert oracle.triangles(d) is None
    assert oracle.sample_triangles(d, 1, 0, 0, 10) is None


def test_draw_is_the_ranked_triangle():
    g = gnp(30, 0.3, 4)
    tri = oracle.triangles(g)
    off, nodes = oracle.sample_triangles(g, 9, 2, 100, 50)
    assert np.array_equal(off, 3 * np.arange(51))
    for i in range(50):
        r = int(oracle.bounded_many(9, 100 + i, 2, 5, len(tri), 1)[0])
        assert nodes[3 * i: 3 * i + 3].tolist() == tri[r].tolist()


def test_uniform_over_triangles():
    g = gnp(16, 0.4, 3)
    tri = oracle.triangles(g)
    T = len(tri)
    assert 20 <= T <= 200
    m = 200 * T
    off, nodes = oracle.sample_triangles(g, 5, 0, 0, m)
    index = {tuple(t): i for i, t in enumerate(tri.tolist())}
    counts = np.bincount([index[tuple(x)] for x in nodes.reshape(-1, 3).tolist()], minlength=T)
    assert stats.chisquare(counts).pvalue > 1e-4


def test_estimator_matches_exact_triangle_centrality():
    g = gnp(60, 0.2, 8)
    tri = oracle.triangles(g)
    S = {0, 5, 17}
    exact = np.mean([bool(S & set(t)) for t in tri.tolist()])
    m = 20000
    off, nodes = oracle.sample_triangles(g, 3, 0, 0, m)
    est = np.mean([bool(S & set(x)) for x in nodes.reshape(-1, 3).tolist()])
    assert abs(est - exact) <= 5 * math.sqrt(exact * (1 - exact) / m) + 1e-12


def test_progressive_on_triangles_matches_its_parts():
    g = gnp(200, 0.08, 6)
    k, t, eps, delta, seed = 4, 8, 0.2, 0.1, 2
    rc, picks, res, mlog = oracle.progressive(g, k, t, eps, delta, seed, 0, 1000, 64000,
                                              space=oracle.SPACE_TRIANGLES, with_m_log=True)
    assert rc in (0, 1) and res.iterations >= 1
    m = res.m_final
    off, nodes = oracle.sample_triangles(g, seed, 0, 0, m)
    p2, cov = oracle.greedy_cover(g.n, off, nodes, k)
    assert np.array_equal(picks, p2) and res.coverage == cov[-1]
    am, topk, dk, bm = oracle.mcera(g.n, off, nodes, seed, 0, t, k)
    assert bm == 3
    o = oracle.bound(m, int(cov[-1]), int(topk.sum()), t, dk, bm, eps, delta / 2**res.iterations)
    assert res.eta == o.eta and (rc == 0) == bool(o.certified)


def test_row_counts_partition_the_ranked_list():
    # the per-row enumeration is the ranked list sliced by smallest node
    g = gnp(40, 0.3, 7)
    brute = brute_triangles(g)
    og = oracle.OracleGraph(g)
    per_row = [oracle.row_triangle_count(g, a, og=og) for a in range(g.n)]
    assert per_row == [sum(1 for t in brute if t[0] == a) for a in range(g.n)]
    assert sum(per_row) == len(oracle.triangles(g))
    d = inputs.from_edges(3, [0, 1, 2], [1, 2, 0], directed=True)
    assert oracle.row_triangle_count(d, 0) is None
