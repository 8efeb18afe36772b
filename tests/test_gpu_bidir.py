"""GPU parity of centra_sample_paths_bidir (the balanced bidirectional
sampler of Sec. 5, reading R16) against the oracle: bit-exact hyperedges,
pairs and distances on the sampler's test graphs (hubs, count shifts on both
sides, unreachable targets, long diameters), batch splits, the large sparse
configuration on sampled indices, and Algorithm 1 on this sampler."""
import numpy as np
import pytest
import torch

import oracle
from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import check_graph_info, nodes_np, off_np, say
from tests.test_gpu_sampler import CASES

pytestmark = pytest.mark.gpu


def budgets(g, cbo):
    c_f, c_b = oracle.count_bits(g), oracle.count_bits_out(g)
    if cbo:
        c_f, c_b = min(c_f, cbo), min(c_b, cbo)
    return c_f, c_b


def check_batch(ctx, g, cbo, seed, inst, first, count):
    dg = binding.DeviceGraph(ctx, g, count_bits_override=cbo)
    try:
        off, nodes, st, dist = binding.sample_paths(ctx, dg, seed, inst, first, count, with_st=True, bidir=True)
        torch.cuda.synchronize()
        check_graph_info(dg, g, cbo)
    finally:
        dg.release()
    c_f, c_b = budgets(g, cbo)
    want_off, want_nodes, infos = oracle.sample_paths_bidir(g, seed, inst, first, count, c_f=c_f, c_b=c_b,
                                                            with_info=True)
    assert np.array_equal(off_np(off), want_off)
    assert np.array_equal(nodes_np(nodes), want_nodes)
    st = st.cpu().numpy().view(np.uint32)[: 2 * count]
    dist = dist.cpu().numpy().view(np.uint32)[:count]
    assert np.array_equal(st[0::2], np.array([i.s for i in infos], dtype=np.uint32))
    assert np.array_equal(st[1::2], np.array([i.t for i in infos], dtype=np.uint32))
    assert np.array_equal(dist, np.array([i.dist for i in infos], dtype=np.uint32))


@pytest.mark.parametrize("name", list(CASES))
def test_bidir_bit_exact(ctx, name):
    build, cbo = CASES[name]
    g = build()
    count = 3000 if g.n > 2 else 500
    say(f"bidir parity {name}: n={g.n} arcs={g.n_arcs} count={count} cbo={cbo}")
    check_batch(ctx, g, cbo, seed=7, inst=1, first=0, count=count)


def test_bidir_grid_small_budget(ctx):
    # counts shifted at almost every level of both sides
    check_batch(ctx, inputs.grid_graph(60), 6, seed=3, inst=2, first=100, count=2000)


def test_bidir_batch_split_and_relabelling(ctx, monkeypatch):
    g = inputs.ba_graph(3000, 4, 2)
    dg = binding.DeviceGraph(ctx, g)
    try:
        off_a, nodes_a = binding.sample_paths(ctx, dg, 5, 0, 0, 4000, bidir=True)
        off_b, nodes_b = binding.sample_paths(ctx, dg, 5, 0, 0, 1500, bidir=True)
        off_c, nodes_c = binding.sample_paths(ctx, dg, 5, 0, 1500, 2500, bidir=True)
    finally:
        dg.release()
    assert np.array_equal(nodes_np(nodes_a), np.concatenate([nodes_np(nodes_b), nodes_np(nodes_c)]))
    monkeypatch.setenv("CENTRA_RELABEL", "0")
    say("bidir parity without relabelling")
    check_batch(ctx, inputs.rmat_graph(12, 8, seed=3), 0, seed=7, inst=1, first=0, count=3000)


def test_bidir_large_sparse_sampled(ctx):
    # BA n = 10^6: 100,000 samples; 300 spread indices recomputed by the oracle
    g = inputs.ba_graph(1_000_000, 5, 1)
    dg = binding.DeviceGraph(ctx, g)
    count = 100_000
    try:
        say("bidir sampler: 100000 samples on BA n=1e6")
        binding.centra_sampler_stats_get(ctx, reset=True)
        off, nodes, st, dist = binding.sample_paths(ctx, dg, 1, 0, 0, count, with_st=True, bidir=True)
        torch.cuda.synchronize()
        stats = binding.centra_sampler_stats_get(ctx)
        check_graph_info(dg, g)
    finally:
        dg.release()
    say(f"  {stats.kernel_ms:.1f} ms, {stats.arcs / count:.0f} arcs and {stats.nodes / count:.0f} nodes per path")
    off, nodes = off_np(off), nodes_np(nodes)
    idx = np.linspace(0, count - 1, 300).astype(np.int64)
    c_f, c_b = budgets(g, 0)
    for i in idx:
        w_off, w_nodes = oracle.sample_paths_bidir(g, 1, 0, int(i), 1, c_f=c_f, c_b=c_b)
        assert np.array_equal(nodes[int(off[i]):int(off[i + 1])], w_nodes), i


@pytest.mark.parametrize("name,m_init,m_max,k", [("ba2000", 5000, 40000, 10), ("dir300", 2000, 16000, 5)])
def test_progressive_on_bidir(ctx, name, m_init, m_max, k):
    build, cbo = CASES[name]
    g = build()
    dg = binding.DeviceGraph(ctx, g)
    try:
        say(f"progressive with the bidirectional sampler on {name}")
        rc, picks, res, log = binding.centra_progressive(ctx, dg.handle, k, 10, 0.1, 0.1, 3, 0, m_init, m_max,
                                                         space=binding.CENTRA_SPACE_PATHS_BIDIR)
    finally:
        dg.release()
    wrc, wpicks, wres = oracle.progressive(g, k, 10, 0.1, 0.1, 3, 0, m_init, m_max, space=oracle.SPACE_PATHS_BIDIR)
    assert rc == wrc and np.array_equal(picks, wpicks)
    assert (res.iterations, res.m_final, res.coverage) == (wres.iterations, wres.m_final, wres.coverage)
    assert res.eta == pytest.approx(wres.eta, rel=1e-12)
