"""Pins for the oracle's balanced bidirectional sampler (the sampling
procedure of Sec. 5; reading R16): every hyperedge is the interior of a
shortest s-t path (networkx), in t-to-s order, empty when t is unreachable
or adjacent; the pair is uniform; for a fixed pair every shortest path is
equally likely (chi-square over the enumerated paths, including pairs whose
meeting nodes carry unequal products of counts); the set-betweenness
estimate agrees with the exact value by enumeration; small count budgets
keep every path a shortest one; the search scans far fewer arcs than a
whole-level BFS from s."""
import math

import networkx as nx
import numpy as np
import pytest

import oracle
from paper_2306_03651_amd import inputs
from tests.test_oracle_sampler import GRAPHS, exact_set_betweenness, random_digraph, to_nx

UNSEEN = 0xFFFFFFFF

CASES = dict(GRAPHS)
CASES["layered"] = lambda: inputs.layered_dag(layers=12, width=5, max_in=3, hub_out=20)
CASES["two_parts"] = lambda: inputs.from_edges(30, list(range(14)), list(range(1, 15)), directed=False)


def check_paths(g, off, nodes, infos):
    G = to_nx(g)
    for i, inf in enumerate(infos):
        h = [int(x) for x in nodes[int(off[i]):int(off[i + 1])]]
        assert inf.s != inf.t
        if not nx.has_path(G, inf.s, inf.t):
            assert inf.dist == UNSEEN and h == []
            continue
        d = nx.shortest_path_length(G, inf.s, inf.t)
        assert inf.dist == d
        assert len(h) == max(0, d - 1)
        path = [inf.t] + h + [inf.s]   # t's neighbour first
        for a, b in zip(path[1:], path[:-1]):
            assert G.has_edge(a, b)
        assert len(set(path)) == len(path)


@pytest.mark.parametrize("name", list(CASES))
def test_hyperedges_are_shortest_path_interiors(name):
    g = CASES[name]()
    off, nodes, infos = oracle.sample_paths_bidir(g, 17, 0, 0, 400, with_info=True)
    check_paths(g, off, nodes, infos)


def test_small_budgets_keep_paths_shortest():
    # counts shifted at almost every level on both sides
    g = inputs.grid_graph(20)
    off, nodes, infos = oracle.sample_paths_bidir(g, 3, 2, 0, 300, c_f=3, c_b=3, with_info=True)
    check_paths(g, off, nodes, infos)
    assert max(i.dist for i in infos if i.dist != UNSEEN) > 20


def test_pair_uniform():
    g = inputs.grid_graph(3)
    n = g.n
    _, _, infos = oracle.sample_paths_bidir(g, 5, 0, 0, 36000, with_info=True)
    counts = np.zeros((n, n))
    for inf in infos:
        counts[inf.s, inf.t] += 1
    assert np.all(np.diag(counts) == 0)
    cells = counts[~np.eye(n, dtype=bool)]
    exp = len(infos) / (n * (n - 1))
    dof = n * (n - 1) - 1
    assert ((cells - exp) ** 2 / exp).sum() < dof + 6 * math.sqrt(2 * dof)


def path_counts(g, off, nodes, infos, pair):
    seen = {}
    for i, inf in enumerate(infos):
        if (inf.s, inf.t) == pair:
            key = tuple(int(x) for x in nodes[int(off[i]):int(off[i + 1])])
            seen[key] = seen.get(key, 0) + 1
    return seen


def chi2_uniform(c):
    c = np.asarray(c, dtype=float)
    exp = c.sum() / len(c)
    return ((c - exp) ** 2 / exp).sum(), len(c) - 1


@pytest.mark.parametrize("pair", [(0, 8), (2, 6), (8, 0)])
def test_paths_uniform_for_fixed_pair(pair):
    # 3x3 grid, corner to corner: 6 shortest paths; the meeting level's
    # nodes carry products 1x1, 2x2, 1x1 when the sides meet in the middle
    g = inputs.grid_graph(3)
    off, nodes, infos = oracle.sample_paths_bidir(g, 23, 1, 0, 72000, with_info=True)
    seen = path_counts(g, off, nodes, infos, pair)
    G = to_nx(g)
    want = {tuple(p[1:-1][::-1]) for p in nx.all_shortest_paths(G, *pair)}
    assert set(seen) == want
    chi2, dof = chi2_uniform(list(seen.values()))
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_paths_uniform_with_unequal_counts():
    # s = 0 reaches 4 by one path and 5 by two; both precede t = 6, which
    # has one more layer behind (so the sides meet at 4 and 5 with unequal
    # forward counts): three shortest 0 -> 7 paths, each 1/3
    edges = [(0, 1), (0, 2), (0, 3), (1, 4), (2, 5), (3, 5), (4, 6), (5, 6), (6, 7)]
    src, dst = zip(*edges)
    g = inputs.from_edges(8, src, dst, directed=True)
    off, nodes, infos = oracle.sample_paths_bidir(g, 3, 0, 0, 200000, with_info=True)
    seen = path_counts(g, off, nodes, infos, (0, 7))
    assert set(seen) == {(6, 4, 1), (6, 5, 2), (6, 5, 3)}
    chi2, dof = chi2_uniform(list(seen.values()))
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_paths_uniform_on_a_wide_diamond():
    # 0 -> {1..4} -> {5..8} (complete) -> 9 -> 10, plus 0 -> 11 -> 5:
    # 17 shortest 0 -> 10 paths of length 4 through 9... counts differ per
    # middle node (5 has 5 predecessors, 6..8 have 4)
    edges = [(0, i) for i in range(1, 5)] + [(i, j) for i in range(1, 5) for j in range(5, 9)]
    edges += [(j, 9) for j in range(5, 9)] + [(9, 10), (0, 11), (11, 5)]
    src, dst = zip(*edges)
    g = inputs.from_edges(12, src, dst, directed=True)
    off, nodes, infos = oracle.sample_paths_bidir(g, 7, 4, 0, 400000, with_info=True)
    seen = path_counts(g, off, nodes, infos, (0, 10))
    G = to_nx(g)
    want = {tuple(p[1:-1][::-1]) for p in nx.all_shortest_paths(G, 0, 10)}
    assert len(want) == 17 and set(seen) == want
    chi2, dof = chi2_uniform(list(seen.values()))
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_unreachable_and_adjacent_give_empty():
    g = inputs.from_edges(4, [0, 1], [1, 2], directed=True)
    off, nodes, infos = oracle.sample_paths_bidir(g, 8, 0, 0, 2000, with_info=True)
    for i, inf in enumerate(infos):
        h = [int(x) for x in nodes[int(off[i]):int(off[i + 1])]]
        assert h == ([1] if (inf.s, inf.t) == (0, 2) else [])


def test_estimator_matches_exact_set_betweenness():
    g = inputs.ba_graph(40, 2, 3)
    G = to_nx(g)
    m = 20000
    off, nodes = oracle.sample_paths_bidir(g, 99, 0, 0, m)
    for S in [{0}, {1, 2}, {5, 9, 13}]:
        exact = exact_set_betweenness(G, g.n, S)
        hits = sum(1 for i in range(m) if any(int(x) in S for x in nodes[int(off[i]):int(off[i + 1])]))
        est = hits / m
        sd = math.sqrt(exact * (1 - exact) / m)
        assert abs(est - exact) < 5 * sd + 1e-9, (S, est, exact)


def test_prefix_property_and_fewer_arcs():
    g = inputs.ba_graph(3000, 4, 2)
    off_a, nodes_a, inf_a = oracle.sample_paths_bidir(g, 4, 1, 0, 600, with_info=True)
    off_b, nodes_b = oracle.sample_paths_bidir(g, 4, 1, 0, 250)
    off_c, nodes_c = oracle.sample_paths_bidir(g, 4, 1, 250, 350)
    assert np.array_equal(nodes_a, np.concatenate([nodes_b, nodes_c]))
    _, _, inf_u = oracle.sample_paths(g, 4, 1, 0, 600, with_info=True)
    # the balanced search scans a small fraction of a whole-level BFS
    assert sum(i.arcs_scanned for i in inf_a) * 5 < sum(i.arcs_scanned for i in inf_u)


def test_progressive_on_bidir_matches_its_parts():
    # Algorithm 1 with the bidirectional sampler: the result equals greedy,
    # the AMCERA and the bound recomputed on its final sample
    g = inputs.ba_graph(400, 3, 6)
    k, t, eps, delta, seed = 5, 8, 0.2, 0.1, 2
    rc, picks, res, mlog = oracle.progressive(g, k, t, eps, delta, seed, 0, 1000, 64000,
                                              space=oracle.SPACE_PATHS_BIDIR, with_m_log=True)
    assert rc in (0, 1) and res.iterations >= 1
    m = res.m_final
    off, nodes = oracle.sample_paths_bidir(g, seed, 0, 0, m)
    p2, cov = oracle.greedy_cover(g.n, off, nodes, k)
    assert np.array_equal(picks, p2) and res.coverage == cov[-1]
    am, topk, dk, bm = oracle.mcera(g.n, off, nodes, seed, 0, t, k)
    o = oracle.bound(m, int(cov[-1]), int(topk.sum()), t, dk, bm, eps, delta / 2**res.iterations)
    assert res.eta == o.eta and (rc == 0) == bool(o.certified)
