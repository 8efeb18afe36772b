"""GPU parity of centra_sample_paths against the oracle: bit-exact hyperedges,
pairs and distances on graphs spanning the sampler's code paths (multi-chunk
frontiers, hubs wider than a workgroup, count normalisation, unreachable
targets, long diameters that overflow the staging area), batch splits, the
first configuration in full and the large sparse configuration on sampled
indices."""
import contextlib
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import check_graph_info, nodes_np, off_np, oracle_paths, say

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def monkeypatch_env(key, value):
    old = os.environ.get(key)
    os.environ[key] = value
    try:
        yield
    finally:
        if old is None:
            del os.environ[key]
        else:
            os.environ[key] = old


def random_digraph(n, p, seed):
    rng = np.random.default_rng(seed)
    src, dst = np.nonzero(rng.random((n, n)) < p)
    return inputs.from_edges(n, src, dst, directed=True)


def star(n):
    return inputs.from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n), directed=False)


def chain(n):
    return inputs.from_edges(n, np.arange(n - 1), np.arange(1, n), directed=False)


def funnel(seed, fan_src=20, fan_t1=20):
    # Directed: a strongly connected blob (0..999); sources 1000..1499 (no
    # in-neighbours) feeding tier 1 (1500..1599, whose ancestors are sources
    # only: depth 1) and the blob; tier 2 (1600..1699, ancestors tier 1 and
    # sources: depth 2); and 1700..2999, fed by the blob.  Pairs from the
    # blob into the tiers are unreachable; pairs from sources reach them at
    # distance 1 or 2.  With small fans (fan_src, fan_t1) a tier-2 target's
    # pairs fit one chunk, so its ancestor depth is known up front.
    rng = np.random.default_rng(seed)
    src, dst = [], []
    a, b = np.nonzero(rng.random((1000, 1000)) < 0.01)
    src += list(a); dst += list(b)
    for v in range(1000, 1500):
        for w in rng.choice(np.arange(1500, 1600), fan_src, replace=False):
            src.append(v); dst.append(w)
        for w in rng.choice(1000, 2, replace=False):
            src.append(v); dst.append(w)
    for v in range(1500, 1600):
        for w in rng.choice(np.arange(1600, 1700), fan_t1, replace=False):
            src.append(v); dst.append(w)
    for v in range(1700, 3000):
        for w in rng.choice(1000, 2, replace=False):
            src.append(w); dst.append(v)
    e = np.unique(np.array([src, dst]).T, axis=0)
    e = e[e[:, 0] != e[:, 1]]
    return inputs.from_edges(3000, e[:, 0], e[:, 1], directed=True)


CASES = {
    "ba2000": (lambda: inputs.ba_graph(2000, 5, 1), 0),
    "grid40_c8": (lambda: inputs.grid_graph(40), 8),
    "grid40": (lambda: inputs.grid_graph(40), 0),
    "dir300": (lambda: random_digraph(300, 0.01, 5), 0),
    "rmat12": (lambda: inputs.rmat_graph(12, 8, seed=3), 0),
    "star3000": (lambda: star(3000), 0),
    "chain1500": (lambda: chain(1500), 0),
    "dense1200": (lambda: random_digraph(1200, 0.5, 8), 0),   # every target has > 512 in-neighbours
    "funnel3000": (lambda: funnel(2), 0),   # targets whose ancestors end within 1 or 2 hops
    "funnel3000s": (lambda: funnel(3, 1, 2), 0),
    "pair": (lambda: inputs.from_edges(2, [0], [1], directed=False), 0),
    "empty2": (lambda: inputs.from_edges(2, [], [], directed=True), 0),
    # directed; largest in-degree 8, largest out-degree 600: the library's
    # own C (59) shifts the counts of long pairs
    "layered": (lambda: inputs.layered_dag(), 0),
}


def check_batch(ctx, g, cbo, seed, inst, first, count):
    dg = binding.DeviceGraph(ctx, g, count_bits_override=cbo)
    try:
        off, nodes, st, dist = binding.sample_paths(ctx, dg, seed, inst, first, count, with_st=True)
        torch.cuda.synchronize()
        c_bits = check_graph_info(dg, g, cbo)
    finally:
        dg.release()
    want_off, want_nodes, infos = oracle.sample_paths(g, seed, inst, first, count, c_bits=c_bits, with_info=True)
    got_off, got_nodes = off_np(off), nodes_np(nodes)
    assert np.array_equal(got_off, want_off)
    assert np.array_equal(got_nodes, want_nodes)
    st = st.cpu().numpy().view(np.uint32)[: 2 * count]
    dist = dist.cpu().numpy().view(np.uint32)[:count]
    assert np.array_equal(st[0::2], np.array([i.s for i in infos], dtype=np.uint32))
    assert np.array_equal(st[1::2], np.array([i.t for i in infos], dtype=np.uint32))
    assert np.array_equal(dist, np.array([i.dist for i in infos], dtype=np.uint32))
    return got_off, got_nodes


@pytest.mark.parametrize("name", list(CASES))
def test_sampler_bit_exact(ctx, name):
    build, cbo = CASES[name]
    g = build()
    count = 3000 if g.n > 2 else 500
    say(f"sampler parity {name}: n={g.n} arcs={g.n_arcs} count={count} cbo={cbo}")
    check_batch(ctx, g, cbo, seed=7, inst=1, first=0, count=count)


@pytest.mark.parametrize("variant", ["lds", "hbm512", "hbm256", "hbm64"])
@pytest.mark.parametrize("name", ["ba2000", "grid40_c8", "rmat12", "star3000", "chain1500", "dense1200",
                                  "funnel3000"])
def test_sampler_variants_bit_exact(ctx, name, variant, monkeypatch):
    # every launch shape of the sampler (LDS bitmap with 1024-thread
    # workgroups; Bloom filter with 512/256/64 threads; the default 128 runs
    # in the tests above) gives the same hyperedges
    monkeypatch.setenv("CENTRA_SAMPLER_VARIANT", variant)
    build, cbo = CASES[name]
    g = build()
    say(f"sampler parity ({variant}) {name}")
    check_batch(ctx, g, cbo, seed=9, inst=0, first=17, count=2500)


def test_c1_configuration_full(ctx):
    # BA n=2000, m0=5, seed 1; m = 10,000 samples of seed 1, instance 0.
    g = inputs.ba_graph(2000, 5, 1)
    say("C1 sampler parity: 10000 samples")
    check_batch(ctx, g, 0, seed=1, inst=0, first=0, count=10000)


def test_batch_split_is_invariant(ctx):
    g = inputs.ba_graph(3000, 4, 2)
    dg = binding.DeviceGraph(ctx, g)
    try:
        off_a, nodes_a = binding.sample_paths(ctx, dg, 5, 0, 0, 4000)
        off_b, nodes_b = binding.sample_paths(ctx, dg, 5, 0, 0, 1234)
        off_c, nodes_c = binding.sample_paths(ctx, dg, 5, 0, 1234, 2766)
        off_d, nodes_d = binding.sample_paths(ctx, dg, 5, 0, 0, 4000)   # rerun: identical
    finally:
        dg.release()
    a = nodes_np(nodes_a)
    assert np.array_equal(a, np.concatenate([nodes_np(nodes_b), nodes_np(nodes_c)]))
    assert np.array_equal(off_np(off_a)[:1235], off_np(off_b))
    assert np.array_equal(a, nodes_np(nodes_d)) and np.array_equal(off_np(off_a), off_np(off_d))


def test_count_zero_and_enospc(ctx):
    g = inputs.ba_graph(500, 3, 1)
    dg = binding.DeviceGraph(ctx, g)
    try:
        off = torch.full((1,), 7, dtype=torch.int64, device="cuda")
        rc, need = binding.centra_sample_paths(ctx, dg.handle, 1, 0, 0, 0, off, None, 0)
        assert rc == 0 and need == 0 and int(off[0]) == 0
        off = torch.empty(401, dtype=torch.int64, device="cuda")
        small = torch.empty(3, dtype=torch.int32, device="cuda")
        rc, need = binding.centra_sample_paths(ctx, dg.handle, 1, 0, 0, 400, off, small, 3)
        assert rc == binding.CENTRA_ENOSPC
        want_off, want_nodes = oracle.sample_paths(g, 1, 0, 0, 400)
        assert need == len(want_nodes)
        assert np.array_equal(off_np(off), want_off)
    finally:
        dg.release()


def test_invalid_graphs_are_rejected(ctx):
    good = inputs.ba_graph(50, 2, 1)
    bad_rows = []
    col = good.col_idx.copy()
    col[[0, 1]] = col[[1, 0]]                       # unsorted row
    bad_rows.append(col)
    col = good.col_idx.copy()
    col[0] = 0                                      # self loop on node 0
    bad_rows.append(col)
    col = good.col_idx.copy()
    col[5] = 1000                                   # out of range
    bad_rows.append(col)
    for col in bad_rows:
        g = inputs.CSRGraph(good.n, False, good.row_ptr, col)
        with pytest.raises(binding.CentraError) as e:
            binding.DeviceGraph(ctx, g)
        assert e.value.code == binding.CENTRA_EINVAL
    d = random_digraph(40, 0.1, 1)
    rcol = d.rcol_idx.copy()
    # a wrong (but sorted) in-row: swap one source for another not adjacent
    v = int(np.argmax(np.diff(d.rrow_ptr.astype(np.int64)) > 0))
    row = set(int(x) for x in rcol[d.rrow_ptr[v]:d.rrow_ptr[v + 1]])
    repl = next(u for u in range(40) if u not in row and u != v)
    rcol[d.rrow_ptr[v]] = repl
    seg = np.sort(rcol[d.rrow_ptr[v]:d.rrow_ptr[v + 1]])
    rcol[d.rrow_ptr[v]:d.rrow_ptr[v + 1]] = seg
    g = inputs.CSRGraph(d.n, True, d.row_ptr, d.col_idx, d.rrow_ptr, rcol)
    with pytest.raises(binding.CentraError):
        binding.DeviceGraph(ctx, g)


def test_large_sparse_configuration_sampled(ctx):
    # BA n = 10^6, m0 = 5: a batch of 20,000 samples in the launch
    # configuration the benchmark uses; 1,000 indices spread over the batch
    # are recomputed one by one by the oracle (on the host's cores).
    g = inputs.ba_graph(1_000_000, 5, 1)
    dg = binding.DeviceGraph(ctx, g)
    count = 20000
    try:
        say("C2 sampler: 20000 samples on BA n=1e6")
        off, nodes, st, dist = binding.sample_paths(ctx, dg, 1, 0, 0, count, with_st=True)
        torch.cuda.synchronize()
        c_bits = check_graph_info(dg, g)
    finally:
        dg.release()
    off, nodes = off_np(off), nodes_np(nodes)
    idx = np.linspace(0, count - 1, 1000).astype(np.int64)
    say("  oracle on 1000 indices")
    for i, (h, info) in zip(idx, oracle_paths(g, 1, 0, idx, c_bits)):
        assert np.array_equal(nodes[int(off[i]):int(off[i + 1])], h), i
    # properties over the whole batch: lengths = d - 1, no repeats in a path
    d = dist.cpu().numpy().view(np.uint32)[:count]
    lens = np.diff(off.astype(np.int64))
    reach = d != 0xFFFFFFFF
    assert np.array_equal(lens[reach], np.maximum(d[reach].astype(np.int64) - 1, 0))
    assert (lens[~reach] == 0).all()


@pytest.fixture(scope="module")
def rmat22():
    return inputs.rmat_graph(22, 16, seed=1)


def check_sampled(ctx, g, seed, inst, first, count, n_check):
    """Samples a full batch on the GPU; recomputes n_check spread indices
    with the oracle and checks every hyperedge's length against its
    distance."""
    dg = binding.DeviceGraph(ctx, g)
    try:
        off, nodes, st, dist = binding.sample_paths(ctx, dg, seed, inst, first, count, with_st=True)
        torch.cuda.synchronize()
        c_bits = check_graph_info(dg, g)
    finally:
        dg.release()
    off, nodes = off_np(off), nodes_np(nodes)
    st = st.cpu().numpy().view(np.uint32)[: 2 * count]
    d = dist.cpu().numpy().view(np.uint32)[:count]
    idx = np.linspace(0, count - 1, n_check).astype(np.int64)
    say(f"  oracle on {n_check} indices")
    for i, (h, info) in zip(idx, oracle_paths(g, seed, inst, first + idx, c_bits)):
        assert np.array_equal(nodes[int(off[i]):int(off[i + 1])], h), i
        assert (st[2 * i], st[2 * i + 1], d[i]) == (info.s, info.t, info.dist), i
    lens = np.diff(off.astype(np.int64))
    reach = d != 0xFFFFFFFF
    assert np.array_equal(lens[reach], np.maximum(d[reach].astype(np.int64) - 1, 0))
    assert (lens[~reach] == 0).all()
    return off, nodes, d


def test_rmat22_configuration_sampled(ctx, rmat22):
    # The skewed directed configuration: R-MAT scale 22 (4.2M nodes, 65.2M
    # arcs after dropping duplicates and self loops), reverse CSR; half the
    # targets have no in-neighbour, and many pairs are unreachable.
    say(f"R-MAT 22: n={rmat22.n} arcs={rmat22.n_arcs}; 200000 samples")
    off, nodes, d = check_sampled(ctx, rmat22, 1, 0, 0, 200000, 200)
    say(f"  reachable fraction {np.mean(d != 0xFFFFFFFF):.3f}")


@pytest.mark.parametrize("L", [256, 1024])
def test_grid_configuration_sampled(ctx, L):
    # Grids of the uneven-instances configuration (side up to 1024, diameter
    # up to 2046): thousands of levels, count normalisation shifts, and the
    # last-level shortcut disabled once the level sums exceed 2^C.
    say(f"grid {L}x{L}: 3000 samples")
    check_sampled(ctx, inputs.grid_graph(L), 3, 5, 1000, 3000, 96)


def test_serving_graphs_sampled(ctx):
    # Graph families of the serving configuration beyond the ones above:
    # directed R-MAT scale 20 (16.1M arcs) and the 2048 x 2048 grid
    # (diameter 4,094: up to 4,094 levels per BFS, slot count capped by the
    # slot memory budget).
    g = inputs.rmat_graph(20, 16, seed=1)
    say(f"R-MAT 20 directed: n={g.n} arcs={g.n_arcs}; 100000 samples")
    check_sampled(ctx, g, 1, 0, 0, 100000, 200)
    del g
    g = inputs.grid_graph(2048)
    say(f"grid 2048x2048: n={g.n}; 600 samples")
    off, nodes, d = check_sampled(ctx, g, 4, 2, 0, 600, 48)
    say(f"  longest hyperedge {int(np.diff(off.astype(np.int64)).max())}")


def test_ba_1e5_configuration_sampled(ctx):
    say("BA n=1e5: 50000 samples")
    check_sampled(ctx, inputs.ba_graph(100_000, 5, 7), 2, 9, 0, 50000, 400)


@pytest.mark.parametrize("variant", ["hbm128", "hbm512"])
def test_hub_targets_without_ring_cache(ctx, variant, monkeypatch):
    # Targets with more in-neighbours than the ring cache (256 entries for
    # workgroups below 512 threads, 512 from 512 up) take the uncached 2-hop
    # test; with d >= 3 its first backtrack step is followed by ordinary
    # steps, which must draw from the same stream on every thread.  The
    # indices are selected from the GPU's own (s, t, d) output; every
    # selected hyperedge and (s, t, d) is recomputed by the oracle.
    monkeypatch.setenv("CENTRA_SAMPLER_VARIANT", variant)
    cache = 512 if variant == "hbm512" else 256
    g = inputs.ba_graph(1_000_000, 5, 1)
    count = 200_000
    dg = binding.DeviceGraph(ctx, g)
    try:
        say(f"hub targets ({variant}): {count} samples on BA n=1e6")
        off, nodes, st, dist = binding.sample_paths(ctx, dg, 1, 0, 0, count, with_st=True)
        torch.cuda.synchronize()
        c_bits = check_graph_info(dg, g)
    finally:
        dg.release()
    off, nodes = off_np(off), nodes_np(nodes)
    st = st.cpu().numpy().view(np.uint32)[: 2 * count]
    d = dist.cpu().numpy().view(np.uint32)[:count]
    t = st[1::2].astype(np.int64)
    indeg = (g.row_ptr[t + 1] - g.row_ptr[t]).astype(np.int64)   # undirected: in-degree = degree
    sel = np.nonzero((indeg > cache) & (d >= 3) & (d != 0xFFFFFFFF))[0][:30]
    say(f"  {len(sel)} selected samples")
    assert len(sel) >= 2
    for i, (h, info) in zip(sel, oracle_paths(g, 1, 0, sel, c_bits)):
        assert np.array_equal(nodes[int(off[i]):int(off[i + 1])], h), i
        assert (st[2 * i], st[2 * i + 1], d[i]) == (info.s, info.t, info.dist), i


@pytest.mark.parametrize("name", ["ba2000", "dir300", "rmat12", "grid40_c8", "chain1500"])
def test_sampler_without_relabelling(ctx, name, monkeypatch):
    # The sampler normally traverses a locality-relabelled copy of the
    # graph; traversing the caller's CSR directly must give the same bits.
    monkeypatch.setenv("CENTRA_RELABEL", "0")
    build, cbo = CASES[name]
    g = build()
    say(f"sampler parity without relabelling {name}")
    check_batch(ctx, g, cbo, seed=7, inst=1, first=0, count=3000)


@pytest.mark.parametrize("fans,count", [((20, 20), 20000), ((1, 2), 60000)])
def test_funnel_covers_the_ancestor_depth_cases(ctx, fans, count):
    # The funnel graphs must actually produce the cases the early stop
    # decides: unreachable targets with ancestors, and targets reached at
    # exactly their ancestor depth.
    g = funnel(2, *fans)
    _, _, infos = oracle.sample_paths(g, 7, 1, 0, count, with_info=True)
    t = np.array([i.t for i in infos]); d = np.array([i.dist for i in infos])
    tier1 = (t >= 1500) & (t < 1600)
    tier2 = (t >= 1600) & (t < 1700)
    assert ((d == 0xFFFFFFFF) & (tier1 | tier2)).sum() > 100
    assert ((d == 1) & tier1).sum() > 2 and ((d == 2) & tier2).sum() > 2
    say(f"funnel {fans}: {count} samples")
    check_batch(ctx, g, 0, seed=7, inst=1, first=0, count=count)


def test_stamp_wrap(monkeypatch):
    # The sampler's records carry 32-bit BFS stamps and are never reset
    # between samples; when the stamps would wrap, every record is cleared
    # and numbering restarts at 1.  Starting a context just below the wrap
    # crosses it within a few batches; every batch must still match the
    # oracle (a stale record would change a hyperedge or fail the backtrack).
    monkeypatch.setenv("CENTRA_STAMP_START", str(0xFFFFFFFF - 5000))
    ctx = binding.centra_create(0, 0)
    try:
        g = inputs.ba_graph(2000, 5, 1)
        dg = binding.DeviceGraph(ctx, g)
        try:
            first = 0
            for count in [3000, 3000, 3000]:   # the second batch crosses the wrap
                say(f"stamp wrap: batch at {first}")
                off, nodes = binding.sample_paths(ctx, dg, 7, 1, first, count)
                want_off, want_nodes = oracle.sample_paths(g, 7, 1, first, count)
                assert np.array_equal(off_np(off), want_off)
                assert np.array_equal(nodes_np(nodes), want_nodes)
                first += count
        finally:
            dg.release()
    finally:
        binding.centra_destroy(ctx)


def test_hbm_budget():
    # A budget too small for the graph's relabelled copy is refused with
    # CENTRA_ENOMEM; a budget that holds only a few BFS slots runs fewer
    # concurrent BFSs and gives the same hyperedges.
    g = inputs.ba_graph(2000, 5, 1)
    ctx = binding.centra_create(0, 64 << 10)
    try:
        with pytest.raises(binding.CentraError) as e:
            binding.DeviceGraph(ctx, g)
        assert e.value.code == binding.CENTRA_ENOMEM
    finally:
        binding.centra_destroy(ctx)
    ctx = binding.centra_create(0, 48 << 20)
    try:
        dg = binding.DeviceGraph(ctx, g)
        try:
            say("budgeted context: 3000 samples")
            binding.centra_sampler_stats_get(ctx, reset=True)
            off, nodes = binding.sample_paths(ctx, dg, 7, 1, 0, 3000)
            st = binding.centra_sampler_stats_get(ctx)
            assert 1 <= st.slots < 100
            want_off, want_nodes = oracle.sample_paths(g, 7, 1, 0, 3000)
            assert np.array_equal(off_np(off), want_off)
            assert np.array_equal(nodes_np(nodes), want_nodes)
        finally:
            dg.release()
    finally:
        binding.centra_destroy(ctx)


def _sample_in_fresh_context(g, count, first=0):
    ctx = binding.centra_create(0, 0)
    try:
        dg = binding.DeviceGraph(ctx, g)
        try:
            off, nodes = binding.sample_paths(ctx, dg, 1, 0, first, count)
            torch.cuda.synchronize()
            return off_np(off), nodes_np(nodes), binding.centra_context_log(ctx)
        finally:
            dg.release()
    finally:
        binding.centra_destroy(ctx)


def test_slot_placement_search(monkeypatch):
    # A fresh slot state of at least 4 GiB (BA 10^6: 61 GB) is chosen among
    # up to four allocations by timing the batch's first 65,536 samples on
    # each.  The hyperedges are those of a context without the search, and
    # of the oracle on sampled indices.
    g = inputs.ba_graph(1_000_000, 5, 1)
    count = 100_000
    monkeypatch.setenv("CENTRA_SLOT_SEARCH", "0")
    say("placement search off: 100000 samples on BA n=1e6")
    off0, nodes0, log0 = _sample_in_fresh_context(g, count)
    assert "slot placement" not in log0
    monkeypatch.delenv("CENTRA_SLOT_SEARCH")
    say("placement search on: 100000 samples on BA n=1e6")
    off1, nodes1, log1 = _sample_in_fresh_context(g, count)
    say(f"  {log1.strip()}")
    line = [x for x in log1.splitlines() if x.startswith("slot placement:")]
    assert len(line) == 1
    times = [float(x) for x in line[0].split(":")[1].split("ms")[0].split()]
    assert 1 <= len(times) <= 4 and all(t > 0 for t in times)
    assert np.array_equal(off0, off1) and np.array_equal(nodes0, nodes1)
    idx = np.linspace(0, count - 1, 200).astype(np.int64)
    for i, (h, info) in zip(idx, oracle_paths(g, 1, 0, idx, oracle.count_bits(g))):
        assert np.array_equal(nodes1[int(off1[i]):int(off1[i + 1])], h), i


def test_slot_placement_search_skipped_near_stamp_wrap(monkeypatch):
    # The search would use about 524k stamps; a context that has fewer left
    # before the 32-bit wrap skips it (the held slot states must agree with
    # the stamps), and the batches across the wrap still match the oracle.
    monkeypatch.setenv("CENTRA_STAMP_START", str(0xFFFFFFFF - 150_000))
    g = inputs.ba_graph(1_000_000, 5, 1)
    ctx = binding.centra_create(0, 0)
    try:
        dg = binding.DeviceGraph(ctx, g)
        try:
            first = 0
            for count in [100_000, 100_000]:   # the second batch crosses the wrap
                say(f"near-wrap context: batch at {first}")
                off, nodes = binding.sample_paths(ctx, dg, 1, 0, first, count)
                off, nodes = off_np(off), nodes_np(nodes)
                idx = np.linspace(0, count - 1, 50).astype(np.int64)
                for i, (h, info) in zip(idx, oracle_paths(g, 1, 0, idx + first, oracle.count_bits(g))):
                    assert np.array_equal(nodes[int(off[i]):int(off[i + 1])], h), i
                first += count
            assert "slot placement" not in binding.centra_context_log(ctx)
        finally:
            dg.release()
    finally:
        binding.centra_destroy(ctx)


@pytest.mark.parametrize("name", ["ba2000", "grid40_c8", "grid40", "rmat12", "dir300", "dense1200", "funnel3000",
                                  "layered", "star3000", "chain1500"])
def test_wide_bfs_bit_exact(ctx, name, monkeypatch):
    # With the threshold lowered to one node, nearly every BFS is handed
    # from its workgroup to the device-wide BFS, which redraws the sample
    # with full levels (no ring tests) and the same backtrack; hyperedges,
    # pairs and distances must still be the oracle's (count shifts on the
    # 8-bit grid and the layered graph, unreachable targets on the funnel).
    monkeypatch.setenv("CENTRA_WIDE_NODES", "1")
    build, cbo = CASES[name]
    g = build()
    count = 40 if name == "chain1500" else 200
    say(f"device-wide BFS parity {name}: {count} samples")
    binding.centra_sampler_stats_get(ctx, reset=True)
    check_batch(ctx, g, cbo, seed=11, inst=2, first=5, count=count)
    st = binding.centra_sampler_stats_get(ctx)
    say(f"  {st.wide} samples went wide")
    if name in ("grid40_c8", "grid40", "chain1500", "layered"):
        assert st.wide > 0


def test_wide_bfs_on_a_flood(ctx):
    # R-MAT scale 22: sample 260,231 (seed 1, instance 0) floods the ~2M
    # nodes its source reaches (63M arcs).  It goes to the device-wide BFS
    # at the default threshold; the batch around it equals the workgroup
    # kernel's (CENTRA_WIDE=0) and the oracle on sampled indices.
    g = inputs.rmat_graph(22, 16, seed=1)
    dg = binding.DeviceGraph(ctx, g)
    first, count = 260_000, 2_000
    try:
        say("R-MAT 22 batch with a flooding sample: device-wide BFS on")
        binding.centra_sampler_stats_get(ctx, reset=True)
        off1, nodes1, st1, dist1 = binding.sample_paths(ctx, dg, 1, 0, first, count, with_st=True)
        torch.cuda.synchronize()
        s1 = binding.centra_sampler_stats_get(ctx)
        off1, nodes1, dist1 = off_np(off1), nodes_np(nodes1), dist1.cpu().numpy().view(np.uint32)[:count].copy()
        say(f"  {s1.wide} wide, {s1.kernel_ms:.1f} ms")
        assert s1.wide >= 1
        say("same batch, device-wide BFS off")
        with monkeypatch_env("CENTRA_WIDE", "0"):
            binding.centra_sampler_stats_get(ctx, reset=True)
            off0, nodes0, st0, dist0 = binding.sample_paths(ctx, dg, 1, 0, first, count, with_st=True)
            torch.cuda.synchronize()
            s0 = binding.centra_sampler_stats_get(ctx)
        say(f"  {s0.wide} wide, {s0.kernel_ms:.1f} ms")
        assert s0.wide == 0
        assert np.array_equal(off1, off_np(off0)) and np.array_equal(nodes1, nodes_np(nodes0))
        assert np.array_equal(dist1, dist0.cpu().numpy().view(np.uint32)[:count])
        c_bits = check_graph_info(dg, g)
    finally:
        dg.release()
    idx = np.array([231, 0, 1999] + list(range(5, count, 97)), dtype=np.int64)
    say("  oracle on sampled indices (the flood included)")
    for i, (h, info) in zip(idx, oracle_paths(g, 1, 0, idx + first, c_bits)):
        assert np.array_equal(nodes1[int(off1[i]):int(off1[i + 1])], h), i
        assert dist1[i] == info.dist, i


def test_work_counts_are_deterministic(ctx):
    # Half the nodes of a directed R-MAT graph have no in-neighbour, so with
    # about one sample per workgroup some workgroups draw only targets that
    # need no BFS (no arc scanned); their sources' levels still count.  The
    # arcs and nodes of a launch must not depend on how the work items were
    # spread over the workgroups.
    g = inputs.rmat_graph(11, 8, seed=5)
    dg = binding.DeviceGraph(ctx, g)
    seen = set()
    try:
        for rep in range(6):
            binding.centra_sampler_stats_get(ctx, reset=True)
            binding.sample_paths(ctx, dg, 5, 2, 0, 3000)
            torch.cuda.synchronize()
            st = binding.centra_sampler_stats_get(ctx)
            seen.add((st.arcs, st.nodes))
    finally:
        dg.release()
    say(f"  work counts over 6 launches: {sorted(seen)}")
    assert len(seen) == 1
