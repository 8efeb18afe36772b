"""Pins of the oracle's kappa-path hyperedges (Sec. 3.1 names the space of
node sets of simple paths of length at most kappa; the sampler is the
random simple walk of the kappa-path centrality, a reading): every walk is a
simple path that stops only at its drawn length or a dead end; the sampled
walks follow the exact distribution enumerated over every random choice;
closed forms on complete graphs; the estimator against the exact kappa-path
set centrality; and the progressive loop on this space."""
import math
from collections import defaultdict

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2306_03651_amd import inputs
from tests.test_oracle_triangles import gnp


def out_rows(g):
    rp = g.row_ptr.astype(np.int64)
    return [g.col_idx[rp[v]:rp[v + 1]].tolist() for v in range(g.n)]


def exact_walks(g, kappa):
    """Probability of every (s, walk) by enumeration of every choice: s
    uniform, l uniform in 1..kappa, each step uniform over the current
    node's out-neighbours not yet on the walk, stopping at l steps or when
    there is none."""
    adj = out_rows(g)
    dist = defaultdict(float)

    def rec(s, walk, left, p):
        v = walk[-1] if walk else s
        free = [w for w in adj[v] if w != s and w not in walk] if left else []
        if not free:
            dist[(s,) + tuple(walk)] += p
            return
        for w in free:
            rec(s, walk + [w], left - 1, p / len(free))

    for s in range(g.n):
        for l in range(1, kappa + 1):
            rec(s, [], l, 1.0 / (g.n * kappa))
    return dist


def small_graphs():
    # a house with a chord (undirected), and a small directed graph with a
    # dead end and a cycle
    house = inputs.from_edges(6, [0, 0, 1, 1, 2, 3, 4], [1, 2, 2, 3, 4, 4, 5], directed=False)
    dg = inputs.from_edges(6, [0, 0, 1, 2, 2, 3, 4, 5], [1, 2, 3, 3, 4, 0, 5, 2], directed=True)
    return {"house": house, "directed": dg}


@pytest.mark.parametrize("kappa", [1, 3, 6])
def test_walks_are_simple_paths_that_stop_only_at_a_dead_end(kappa):
    for g in [gnp(60, 0.08, 1), inputs.ba_graph(500, 3, 2), inputs.rmat_graph(10, 8, seed=3)]:
        adj = [set(r) for r in out_rows(g)]
        og = oracle.OracleGraph(g)
        for x in range(1500):
            h, s, l = oracle.kpath(g, kappa, 7, 1, x, og=og)
            h = h.tolist()
            assert 1 <= l <= kappa and len(h) <= l
            assert len(set(h)) == len(h) and s not in h
            prev = s
            for v in h:
                assert v in adj[prev]
                prev = v
            if len(h) < l:   # stopped early: every out-neighbour is on the walk
                assert adj[prev] <= set(h) | {s}


@pytest.mark.parametrize("name", ["house", "directed"])
def test_exact_walk_distribution(name):
    g = small_graphs()[name]
    kappa = 3
    dist = exact_walks(g, kappa)
    assert abs(sum(dist.values()) - 1.0) < 1e-12
    keys = sorted(dist)
    index = {k: i for i, k in enumerate(keys)}
    N = 60000
    og = oracle.OracleGraph(g)
    counts = np.zeros(len(keys))
    for x in range(N):
        h, s, l = oracle.kpath(g, kappa, 3, 0, x, og=og)
        counts[index[(s,) + tuple(h.tolist())]] += 1
    expected = N * np.array([dist[k] for k in keys])
    assert stats.chisquare(counts, expected).pvalue > 1e-4


def test_complete_graph_closed_forms():
    # On K_n with kappa < n no walk meets a dead end: the length is the
    # drawn l, uniform on 1..kappa, and the first step is uniform over the
    # n - 1 other nodes.
    n, kappa, N = 9, 5, 20000
    g = inputs.from_edges(n, *zip(*[(a, b) for a in range(n) for b in range(a + 1, n)]), directed=False)
    og = oracle.OracleGraph(g)
    lens = np.zeros(kappa + 1)
    first = np.zeros(n - 1)
    for x in range(N):
        h, s, l = oracle.kpath(g, kappa, 5, 2, x, og=og)
        assert len(h) == l
        lens[len(h)] += 1
        first[(int(h[0]) - s - 1) % n] += 1
    assert lens[0] == 0
    assert stats.chisquare(lens[1:]).pvalue > 1e-4
    assert stats.chisquare(first).pvalue > 1e-4


def test_estimator_matches_exact_kpath_centrality():
    g = gnp(14, 0.3, 4)
    kappa = 4
    dist = exact_walks(g, kappa)
    S = {2, 7, 11}
    exact = sum(p for k, p in dist.items() if S & set(k[1:]))
    m = 30000
    off, nodes = oracle.sample_kpaths(g, kappa, 9, 0, 0, m)
    hits = sum(bool(S & set(nodes[int(off[i]):int(off[i + 1])].tolist())) for i in range(m))
    assert abs(hits / m - exact) <= 5 * math.sqrt(exact * (1 - exact) / m) + 1e-12


def test_batch_equals_single_samples_and_errors():
    g = inputs.ba_graph(300, 3, 5)
    off, nodes = oracle.sample_kpaths(g, 4, 2, 1, 100, 400)
    og = oracle.OracleGraph(g)
    for i in range(400):
        h, s, l = oracle.kpath(g, 4, 2, 1, 100 + i, og=og)
        assert nodes[int(off[i]):int(off[i + 1])].tolist() == h.tolist()
    assert oracle.sample_kpaths(g, 0, 2, 1, 0, 10) is None


def test_progressive_on_kpaths_matches_its_parts():
    g = inputs.ba_graph(400, 3, 6)
    k, t, eps, delta, seed, kappa = 5, 8, 0.2, 0.1, 2, 4
    rc, picks, res, mlog = oracle.progressive(g, k, t, eps, delta, seed, 0, 1000, 64000,
                                              space=oracle.SPACE_KPATHS, kappa=kappa, with_m_log=True)
    assert rc in (0, 1) and res.iterations >= 1
    m = res.m_final
    off, nodes = oracle.sample_kpaths(g, kappa, seed, 0, 0, m)
    p2, cov = oracle.greedy_cover(g.n, off, nodes, k)
    assert np.array_equal(picks, p2) and res.coverage == cov[-1]
    am, topk, dk, bm = oracle.mcera(g.n, off, nodes, seed, 0, t, k)
    assert bm <= kappa
    o = oracle.bound(m, int(cov[-1]), int(topk.sum()), t, dk, bm, eps, delta / 2**res.iterations)
    assert res.eta == o.eta and (rc == 0) == bool(o.certified)
    rc0, _, _ = oracle.progressive(g, k, t, eps, delta, seed, 0, 1000, 64000, space=oracle.SPACE_KPATHS, kappa=0)
    assert rc0 == -1
