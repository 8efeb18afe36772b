"""GPU tests of the batching and serving engine (centra_engine_*): every
query's result equals centra_progressive run alone on the same graph and
parameters (bit-exact picks, coverage, sample sizes and iteration count;
bound values to 1e-12), in batch mode over uneven instances, under a tight
memory budget, without captured graphs, with arrivals spread in time
(continuous batching), and when a pool's released levels are rebuilt; the
same query alone and in a mix gives the same result."""
import numpy as np
import pytest

import oracle
from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

FIELDS = ["c_hat", "amcera", "wimpy", "xi", "nu", "rtilde", "r", "eta"]


def standalone(ctx, dg, pool, q):
    seed, inst, t_pool, m_init, m_max = pool
    k, t, eps, delta = q
    return binding.centra_progressive(ctx, dg.handle, k, t, eps, delta, seed, inst, m_init, m_max)


def same(got, want):
    rc, picks, res = got[0], got[1], got[2]
    wrc, wpicks, wres = want[0], want[1], want[2]
    assert rc == wrc
    assert np.array_equal(picks, wpicks)
    assert (res.n_picked, res.iterations, res.certified, res.coverage, res.m_final) == \
        (wres.n_picked, wres.iterations, wres.certified, wres.coverage, wres.m_final)
    for f in FIELDS:
        assert getattr(res, f) == pytest.approx(getattr(wres, f), rel=1e-12, abs=1e-300), f


def uneven_instances(seed, count):
    """Small graphs of the uneven-instances mix (BA of a few thousand nodes,
    grids up to side 40, a directed R-MAT), with per-instance k."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = i % 4
        if kind == 0:
            g = inputs.ba_graph(int(rng.integers(1000, 5000)), 5, 100 + i)
        elif kind == 1:
            g = inputs.grid_graph(int(rng.integers(12, 41)))
        elif kind == 2:
            g = inputs.rmat_graph(11, 8, seed=200 + i)
        else:
            g = inputs.ba_graph(int(rng.integers(200, 800)), 3, 300 + i)
        out.append((g, int(rng.integers(5, 30))))
    return out


def run_batch(ctx, graphs, flags=0, budget=0, t=16, eps=0.1, delta=0.1, m_init=2000, m_max=32000):
    dgs = [binding.DeviceGraph(ctx, g) for g, _ in graphs]
    eng = binding.Engine(ctx, budget, flags)
    try:
        qids, pools = [], []
        for i, (dg, (g, k)) in enumerate(zip(dgs, graphs)):
            pool = (7, i, t, m_init, m_max)
            pid = eng.add_pool(dg.handle, *pool)
            qids.append(eng.submit(pid, k, t, eps, delta))
            pools.append(pool)
        eng.run()
        got = [eng.result(q) for q in qids]
        st = eng.stats()
        log = eng.log()
        want = [standalone(ctx, dg, pool, (k, t, eps, delta)) for dg, pool, (g, k) in zip(dgs, pools, graphs)]
    finally:
        eng.destroy()
        for dg in dgs:
            dg.release()
    return got, want, st, log


def test_batch_equals_standalone(ctx):
    graphs = uneven_instances(1, 12)
    say(f"engine batch: {len(graphs)} instances")
    got, want, st, log = run_batch(ctx, graphs)
    for g, w in zip(got, want):
        same(g, w)
    say(f"  ticks {st.ticks}, sampler launches {st.sampler_launches}, graph replays {st.graph_replays}, "
        f"tuned block {st.tuned_block}; {log.strip()}")
    assert st.graph_replays > 0 and st.tuned_block in (64, 128, 256, 512)
    assert "autotune" in log
    # fused: one sampling launch per tick at most (plus the tuner's probes)
    assert st.sampler_launches <= st.ticks


@pytest.mark.parametrize("k", [200, 600])
def test_large_k_candidate_lists(ctx, k):
    # many greedy rounds: the rounds run on candidate lists most of the time
    # (full scans only to rebuild them); picks must still be exact
    graphs = [(inputs.ba_graph(20000, 5, 31), k), (inputs.grid_graph(60), k), (inputs.rmat_graph(13, 8, seed=32), k)]
    say(f"engine batch with k={k}")
    got, want, st, _ = run_batch(ctx, graphs, t=8, eps=0.02, m_init=20000, m_max=80000)
    for g, w in zip(got, want):
        same(g, w)


def test_batch_matches_oracle(ctx):
    # one instance, checked against the oracle's progressive loop as well
    g = inputs.ba_graph(2000, 5, 1)
    got, want, st, _ = run_batch(ctx, [(g, 10)], t=10, eps=0.05, m_init=10000, m_max=40000)
    wrc, wpicks, wres = oracle.progressive(g, 10, 10, 0.05, 0.1, 7, 0, 10000, 40000)
    rc, picks, res, _ = got[0]
    assert rc == wrc and np.array_equal(picks, wpicks)
    assert res.coverage == wres.coverage and res.m_final == wres.m_final
    assert res.eta == pytest.approx(wres.eta, rel=1e-12)


def test_batch_without_graphs_and_under_budget(ctx):
    graphs = uneven_instances(2, 8)
    say("engine batch without captured graphs")
    got, want, st, _ = run_batch(ctx, graphs, flags=binding.CENTRA_ENGINE_NO_GRAPHS | binding.CENTRA_ENGINE_NO_TUNE)
    for g, w in zip(got, want):
        same(g, w)
    assert st.graph_replays == 0 and st.greedy_launches > 0 and st.tuned_block == 0
    # a budget below the unbudgeted peak: fewer queries at once, same results
    budget = int(st.peak_bytes * 0.8)
    say(f"engine batch under a budget of {budget} bytes (unbudgeted peak {st.peak_bytes})")
    got_b, _, st_b, _ = run_batch(ctx, graphs, budget=budget)
    for g, w in zip(got_b, want):
        same(g, w)
    say(f"  peak active {st_b.peak_active} (unbudgeted {st.peak_active}), peak bytes {st_b.peak_bytes}")
    assert st_b.peak_bytes <= budget and st_b.peak_active < st.peak_active


def test_serving_mix_equals_alone(ctx):
    # three resident pools, queries arriving over 0.3 s with mixed k, t
    # and eps; each result equals the query run alone (a fresh engine with
    # that query only) and centra_progressive
    gs = [inputs.ba_graph(3000, 5, 11), inputs.rmat_graph(11, 8, seed=12), inputs.grid_graph(30)]
    dgs = [binding.DeviceGraph(ctx, g) for g in gs]
    pools = [(5, 0, 32, 4000, 64000), (5, 1, 32, 4000, 64000), (5, 2, 32, 2000, 16000)]
    rng = np.random.default_rng(3)
    qs = []
    tarr = 0.0
    for i in range(16):
        tarr += float(rng.exponential(0.02))
        qs.append((int(rng.integers(3)), int(rng.integers(5, 40)), int(rng.choice([8, 16, 32])),
                   float(rng.choice([0.1, 0.05])), tarr))
    try:
        eng = binding.Engine(ctx, 0)
        try:
            pids = [eng.add_pool(dg.handle, *p) for dg, p in zip(dgs, pools)]
            qids = [eng.submit(pids[p], k, t, eps, 0.1, a) for p, k, t, eps, a in qs]
            say("engine serving: 16 queries over 3 pools, realtime")
            eng.run(realtime=True)
            mixed = [eng.result(q) for q in qids]
            st = eng.stats()
        finally:
            eng.destroy()
        say(f"  ticks {st.ticks}, peak active {st.peak_active}")
        assert st.peak_active >= 2   # queries overlapped on the device
        for (p, k, t, eps, a), got in zip(qs, mixed):
            rc, picks, res, info = got
            assert info.finished_s >= info.admitted_s >= info.arrival_s - 1e-9
            same(got, standalone(ctx, dgs[p], pools[p], (k, t, eps, 0.1)))
        # alone: the first three queries each in a fresh engine
        for (p, k, t, eps, a), got in list(zip(qs, mixed))[:3]:
            eng = binding.Engine(ctx, 0, binding.CENTRA_ENGINE_NO_TUNE)
            try:
                pid = eng.add_pool(dgs[p].handle, *pools[p])
                q = eng.submit(pid, k, t, eps, 0.1, 0.0)
                eng.run()
                alone = eng.result(q)
            finally:
                eng.destroy()
            assert alone[0] == got[0] and np.array_equal(alone[1], got[1])
            assert alone[2].eta == got[2].eta and alone[2].coverage == got[2].coverage
    finally:
        for dg in dgs:
            dg.release()


def test_released_levels_are_rebuilt(ctx):
    # a pool whose levels were released (its only query finished) serves a
    # later query by rebuilding them from its kept samples
    g = inputs.ba_graph(2500, 4, 21)
    dg = binding.DeviceGraph(ctx, g)
    pool = (9, 3, 16, 3000, 24000)
    try:
        eng = binding.Engine(ctx, 0, binding.CENTRA_ENGINE_NO_TUNE)
        try:
            pid = eng.add_pool(dg.handle, *pool)
            q1 = eng.submit(pid, 12, 16, 0.05, 0.1)
            eng.run()
            q2 = eng.submit(pid, 7, 8, 0.1, 0.1)
            eng.run()
            r1, r2 = eng.result(q1), eng.result(q2)
        finally:
            eng.destroy()
        same(r1, standalone(ctx, dg, pool, (12, 16, 0.05, 0.1)))
        same(r2, standalone(ctx, dg, pool, (7, 8, 0.1, 0.1)))
    finally:
        dg.release()


def test_engine_argument_errors(ctx):
    g = inputs.ba_graph(500, 3, 1)
    dg = binding.DeviceGraph(ctx, g)
    eng = binding.Engine(ctx, 0)
    try:
        with pytest.raises(binding.CentraError):
            eng.add_pool(dg.handle, 1, 0, 0, 100, 200)          # t = 0
        with pytest.raises(binding.CentraError):
            eng.add_pool(dg.handle, 1, 0, 8, 300, 200)          # m_max < m_init
        pid = eng.add_pool(dg.handle, 1, 0, 8, 100, 400)
        with pytest.raises(binding.CentraError):
            eng.submit(pid, 5, 9, 0.1, 0.1)                     # t above the pool's
        with pytest.raises(binding.CentraError):
            eng.submit(pid, 5, 8, 0.7, 0.1)                     # eps >= 1 - 1/e
        eng.submit(pid, 5, 8, 0.1, 0.1, 1.0)
        with pytest.raises(binding.CentraError):
            eng.submit(pid, 5, 8, 0.1, 0.1, 0.5)                # arrivals out of order
    finally:
        eng.destroy()
        dg.release()


def test_level_caches_are_exact(ctx):
    # many queries on two pools with mixed k (up to past the prefix sort's
    # 2,048: those ticks select by exact k), t and eps: the cached run
    # (greedy picks and top-k prefix sums kept per level) equals the run
    # without caches and each query alone, with fewer greedy runs
    gs = [inputs.ba_graph(2500, 4, 51), inputs.grid_graph(24)]
    dgs = [binding.DeviceGraph(ctx, g) for g in gs]
    pools = [(3, 0, 24, 2000, 32000), (3, 1, 24, 1000, 8000)]
    rng = np.random.default_rng(8)
    qs = [(int(rng.integers(2)), int(rng.choice([3, 17, 60, 250])), int(rng.choice([8, 24])),
           float(rng.choice([0.1, 0.05, 0.02]))) for _ in range(14)]
    qs.append((0, 2100, 24, 0.05))
    try:
        out = {}
        for flags in (binding.CENTRA_ENGINE_NO_TUNE, binding.CENTRA_ENGINE_NO_TUNE | binding.CENTRA_ENGINE_NO_CACHE):
            eng = binding.Engine(ctx, 0, flags)
            try:
                pids = [eng.add_pool(dg.handle, *p) for dg, p in zip(dgs, pools)]
                # two runs: the second one's queries meet the levels the
                # first one computed (the caches are kept across runs)
                qids = [eng.submit(pids[p], k, t, eps, 0.1) for p, k, t, eps in qs[:8]]
                eng.run()
                qids += [eng.submit(pids[p], k, t, eps, 0.1) for p, k, t, eps in qs[8:]]
                eng.run()
                out[flags] = ([eng.result(q) for q in qids], eng.stats())
            finally:
                eng.destroy()
        (with_c, st_c), (without, st_n) = out.values()
        say(f"engine caches: greedy runs {st_c.greedy_runs} cached, {st_n.greedy_runs} without")
        for a, b in zip(with_c, without):
            same(a, b)
        assert st_c.greedy_runs < st_n.greedy_runs
        for (p, k, t, eps), got in list(zip(qs, with_c))[:4] + [(qs[-1], with_c[-1])]:
            same(got, standalone(ctx, dgs[p], pools[p], (k, t, eps, 0.1)))
    finally:
        for dg in dgs:
            dg.release()


def test_fused_launch_after_placement_search():
    # A pool on BA 10^6 gives the fused sampling launch 49 GB of slot
    # records, so the context chooses their placement on the first fused
    # (tuner) launch; every result must still equal its standalone run.
    ctx = binding.centra_create(0, 0)
    try:
        graphs = [(inputs.ba_graph(1_000_000, 5, 1), 10), (inputs.ba_graph(2000, 5, 2), 5)]
        say("engine batch with a BA 1e6 pool (fresh context)")
        got, want, st, log = run_batch(ctx, graphs, t=8, eps=0.1, m_init=100_000, m_max=200_000)
        for g, w in zip(got, want):
            same(g, w)
        clog = binding.centra_context_log(ctx)
        say(f"  {clog.strip()}")
        assert "slot placement:" in clog
    finally:
        binding.centra_destroy(ctx)


def test_fused_launch_stages_in_one_attempt_after_plain_runs():
    # A launch's first staging size follows the entries per sample the
    # context has staged so far.  A grid's paths have tens of nodes, far
    # above the 8 entries per sample a context starts from: the plain run
    # overflows once and is redrawn, and the larger fused launch after it on
    # the same context must then stage in one attempt (the staging area the
    # plain run left is too small for it), with the standalone result.
    ctx = binding.centra_create(0, 0)
    g = inputs.grid_graph(96)
    dg = binding.DeviceGraph(ctx, g)
    eng = binding.Engine(ctx, 0, binding.CENTRA_ENGINE_NO_TUNE)
    try:
        binding.centra_progressive(ctx, dg.handle, 5, 8, 0.05, 0.1, 3, 1, 5000, 5000)
        st0 = binding.centra_sampler_stats_get(ctx)   # attempts count their samples; entries only once
        per_sample = st0.hyperedge_nodes / 5000
        say(f"plain run: {st0.launches} launch attempts, {per_sample:.1f} entries per sample")
        assert per_sample > 16 and st0.launches == 2 and st0.samples == 10000
        pool = (3, 0, 8, 40000, 40000)
        pid = eng.add_pool(dg.handle, *pool)
        qid = eng.submit(pid, 5, 8, 0.05, 0.1)
        eng.run()
        got = eng.result(qid)
        st1 = binding.centra_sampler_stats_get(ctx)
        assert eng.stats().sampler_launches == 1
        assert st1.launches - st0.launches == 1 and st1.samples - st0.samples == 40000
        same(got, standalone(ctx, dg, pool, (5, 8, 0.05, 0.1)))
    finally:
        eng.destroy()
        dg.release()
        binding.centra_destroy(ctx)
