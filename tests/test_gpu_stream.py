"""GPU tests of the stream-ordered calls (centra_sample_paths_append,
centra_extend, centra_reserve, centra_check): a chain of appends and
extensions issued on one stream without any synchronisation gives, once the
stream is drained, the store of the oracle's sampler and the oracle's
greedy cover and AMCERA ingredients of every prefix [0, m) (bit-exact);
the calls return before the stream reaches them; state is reused across
calls, rebuilt when it cannot be, and a store that overflows its capacity
stays consistent and is reported by centra_check."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import nodes_np, off_np, say

pytestmark = pytest.mark.gpu

SEED, INST = 11, 3


class Phase:
    """Device outputs of one centra_extend call."""

    def __init__(self, k, t):
        dev = "cuda"
        self.picks = torch.zeros(k, dtype=torch.int32, device=dev)
        self.cov = torch.zeros(k, dtype=torch.int64, device=dev)
        self.npk = torch.zeros(1, dtype=torch.int32, device=dev)
        self.topk = torch.zeros(max(t, 1), dtype=torch.int64, device=dev)
        self.dk = torch.zeros(1, dtype=torch.int64, device=dev)
        self.bm = torch.zeros(1, dtype=torch.int32, device=dev)

    def extend(self, ctx, n, k, m_prev, m, off, nodes, cap, t, greedy=True):
        binding.centra_extend(ctx, n, k, m_prev, m, off, nodes, cap,
                              self.picks if greedy else None, self.cov if greedy else None,
                              self.npk if greedy else None, t, SEED, INST,
                              self.topk if t else None, self.dk if t else None, self.bm if t else None)

    def check(self, n, k, t, off, nodes, m, greedy=True):
        o = off[:m + 1]
        nd = nodes[:int(o[-1])]
        if greedy:
            wp, wc = oracle.greedy_cover(n, o, nd, k)
            cnt = int(self.npk.item())
            assert cnt == len(wp)
            assert np.array_equal(self.picks.cpu().numpy()[:cnt].view(np.uint32), wp)
            assert np.array_equal(self.cov.cpu().numpy()[:cnt].astype(np.uint64), wc)
        if t:
            _, wtop, wdk, wbm = oracle.mcera(n, o, nd, SEED, INST, t, k)
            assert np.array_equal(self.topk.cpu().numpy()[:t], wtop)
            assert int(self.dk.item()) == wdk and int(self.bm.item()) == wbm


def store(m_max, cap):
    return (torch.zeros(m_max + 1, dtype=torch.int64, device="cuda"),
            torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda"))


def busy_stream(seconds_hint=0.3):
    """Enqueues matrix products that keep the current stream busy for a
    while and returns an event recorded after them."""
    a = torch.randn(4096, 4096, device="cuda")
    b = a @ a
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        b = a @ b
        b = b * (1.0 / 4096.0)
    torch.cuda.synchronize()
    one = max((time.perf_counter() - t0) / 4, 1e-4)
    reps = int(min(400, max(8, seconds_hint / one)))
    for _ in range(reps):
        b = a @ b
        b = b * (1.0 / 4096.0)
    ev = torch.cuda.Event()
    ev.record()
    return ev, reps * one


def test_chain_without_syncs_matches_oracle(ctx):
    g = inputs.ba_graph(4000, 4, 8)
    dg = binding.DeviceGraph(ctx, g)
    n, k, t = g.n, 16, 24
    batches = [3000, 5000, 8000]
    M = sum(batches)
    w_off, w_nodes = oracle.sample_paths(g, SEED, INST, 0, M)
    cap = int(w_off[-1]) + 7
    try:
        binding.centra_reserve(ctx, dg.handle, n, max(batches), M, cap, k, t)
        # warm-up chain: loads every kernel, so the timed chain only enqueues
        off, nodes = store(M, cap)
        m = 0
        for c in batches:
            binding.centra_sample_paths_append(ctx, dg.handle, SEED, INST, m, c, off[m:], nodes, cap)
            Phase(k, t).extend(ctx, n, k, m, m + c, off, nodes, cap, t)
            m += c
        assert binding.centra_check(ctx) == binding.CENTRA_OK
        say(f"stream chain: BA n={n}, batches {batches}, store cap {cap}")
        off, nodes = store(M, cap)
        totals = torch.zeros(len(batches), dtype=torch.int64, device="cuda")
        phases = [Phase(k, t) for _ in batches]
        ev, busy_s = busy_stream()
        t0 = time.perf_counter()
        m = 0
        for i, c in enumerate(batches):
            binding.centra_sample_paths_append(ctx, dg.handle, SEED, INST, m, c, off[m:], nodes, cap,
                                               totals[i:i + 1])
            phases[i].extend(ctx, n, k, m, m + c, off, nodes, cap, t)
            m += c
        host_s = time.perf_counter() - t0
        pending = not ev.query()
        say(f"  enqueued in {host_s * 1e3:.1f} ms behind ~{busy_s * 1e3:.0f} ms of queued work; "
            f"queued work still pending: {pending}")
        if host_s < 0.25 * busy_s:
            assert pending, "a stream-ordered call waited for the stream"
        assert binding.centra_check(ctx) == binding.CENTRA_OK
        got_off, got_nodes = off_np(off), nodes_np(nodes)
        assert np.array_equal(got_off, w_off)
        assert np.array_equal(got_nodes[:int(w_off[-1])], w_nodes)
        ends = np.cumsum(batches)
        assert np.array_equal(totals.cpu().numpy().astype(np.uint64), w_off[ends])
        for ph, m in zip(phases, ends):
            ph.check(n, k, t, w_off, w_nodes, int(m))
    finally:
        dg.release()


def test_state_reuse_and_rebuild(ctx):
    # the same prefixes reached by different call sequences: AMCERA counts
    # extended over two segments (a greedy-only extension in between), a
    # rebuild after another call took the incidence, a rebuild on m_prev = 0,
    # a repeated m (nothing new), and a change of (seed, t)
    g = inputs.rmat_graph(11, 8, seed=41)
    n, k, t = g.n, 9, 40
    sizes = [1500, 2600, 4000, 6100]
    M = sizes[-1]
    w_off, w_nodes = oracle.sample_paths(g, SEED, INST, 0, M)
    cap = int(w_off[-1])
    off = torch.from_numpy(w_off.view(np.int64)).cuda()
    nodes = torch.from_numpy(w_nodes.view(np.int32)).cuda() if cap else torch.zeros(1, dtype=torch.int32,
                                                                                     device="cuda")
    p = [Phase(k, t) for _ in range(8)]
    say("stream state: extend with AMCERA, greedy only, AMCERA over two segments")
    p[0].extend(ctx, n, k, 0, sizes[0], off, nodes, cap, t)
    p[1].extend(ctx, n, k, sizes[0], sizes[1], off, nodes, cap, 0)
    p[2].extend(ctx, n, k, sizes[1], sizes[2], off, nodes, cap, t)
    p[3].extend(ctx, n, k, sizes[2], sizes[2], off, nodes, cap, t)   # nothing new
    assert binding.centra_check(ctx) == binding.CENTRA_OK
    p[0].check(n, k, t, w_off, w_nodes, sizes[0])
    p[1].check(n, k, 0, w_off, w_nodes, sizes[1])
    p[2].check(n, k, t, w_off, w_nodes, sizes[2])
    p[3].check(n, k, t, w_off, w_nodes, sizes[2])
    # another call builds its own incidence: the next extension rebuilds
    o2 = off[:sizes[0] + 1].clone()
    pk = torch.zeros(k, dtype=torch.int32, device="cuda")
    cv = torch.zeros(k, dtype=torch.int64, device="cuda")
    npk = torch.zeros(1, dtype=torch.int32, device="cuda")
    binding.centra_greedy_cover(ctx, n, o2, nodes, k, pk, cv, npk)
    p[4].extend(ctx, n, k, sizes[2], sizes[3], off, nodes, cap, t)
    # m_prev = 0 rebuilds everything; a new seed rebuilds the counts
    p[5].extend(ctx, n, k, 0, sizes[3], off, nodes, cap, t)
    binding.centra_extend(ctx, n, k, sizes[3], sizes[3], off, nodes, cap, p[6].picks, p[6].cov, p[6].npk, 8,
                          SEED + 1, INST, p[6].topk, p[6].dk, p[6].bm)
    assert binding.centra_check(ctx) == binding.CENTRA_OK
    p[4].check(n, k, t, w_off, w_nodes, sizes[3])
    p[5].check(n, k, t, w_off, w_nodes, sizes[3])
    o = w_off[:sizes[3] + 1]
    _, wtop, wdk, wbm = oracle.mcera(n, o, w_nodes[:int(o[-1])], SEED + 1, INST, 8, k)
    assert np.array_equal(p[6].topk.cpu().numpy()[:8], wtop) and int(p[6].bm.item()) == wbm


def test_overflow_keeps_store_consistent(ctx):
    g = inputs.grid_graph(30)
    dg = binding.DeviceGraph(ctx, g)
    n, k, t = g.n, 6, 8
    M1, M2 = 400, 900
    w_off, w_nodes = oracle.sample_paths(g, SEED, INST, 0, M1 + M2)
    need1 = int(w_off[M1])
    try:
        cap = need1 + 10   # the second batch does not fit
        off, nodes = store(M1 + M2, cap)
        tot = torch.zeros(2, dtype=torch.int64, device="cuda")
        say(f"stream overflow: grid 30x30, store cap {cap}, second batch needs {int(w_off[-1])}")
        binding.centra_sample_paths_append(ctx, dg.handle, SEED, INST, 0, M1, off[0:], nodes, cap, tot[0:1])
        binding.centra_sample_paths_append(ctx, dg.handle, SEED, INST, M1, M2, off[M1:], nodes, cap, tot[1:2])
        ph = Phase(k, t)
        ph.extend(ctx, n, k, 0, M1 + M2, off, nodes, cap, t)   # runs on the consistent (emptied) store
        assert binding.centra_check(ctx) == binding.CENTRA_ENOSPC
        assert "capacity" in binding.centra_last_error(ctx)
        assert binding.centra_check(ctx) == binding.CENTRA_OK   # cleared
        got = off_np(off)
        assert np.array_equal(got[:M1 + 1], w_off[:M1 + 1])
        assert np.all(got[M1:] == need1)
        assert int(tot[1].item()) == int(w_off[-1])
        # the store of the first batch alone is intact
        ph.check(n, k, t, np.concatenate([w_off[:M1 + 1], np.full(M2, need1, dtype=np.uint64)]),
                 w_nodes[:need1], M1 + M2)
        # redraw into a larger store
        cap2 = int(tot[1].item())
        off2, nodes2 = store(M1 + M2, cap2)
        off2[:M1 + 1] = off[:M1 + 1]
        nodes2[:need1] = nodes[:need1]
        binding.centra_sample_paths_append(ctx, dg.handle, SEED, INST, M1, M2, off2[M1:], nodes2, cap2)
        ph2 = Phase(k, t)
        ph2.extend(ctx, n, k, 0, M1 + M2, off2, nodes2, cap2, t)
        assert binding.centra_check(ctx) == binding.CENTRA_OK
        assert np.array_equal(off_np(off2), w_off) and np.array_equal(nodes_np(nodes2)[:cap2], w_nodes)
        ph2.check(n, k, t, w_off, w_nodes, M1 + M2)
        # a capacity below the store's size: the incidence stays empty, no
        # access beyond the stated capacity, CENTRA_ENOSPC
        ph3 = Phase(k, t)
        ph3.extend(ctx, n, k, 0, M1 + M2, off2, nodes2, cap2 - 1, t)
        assert binding.centra_check(ctx) == binding.CENTRA_ENOSPC
        assert int(ph3.npk.item()) == 0
    finally:
        dg.release()


def test_extend_argument_errors(ctx):
    off = torch.zeros(11, dtype=torch.int64, device="cuda")
    nodes = torch.zeros(4, dtype=torch.int32, device="cuda")
    ph = Phase(3, 4)
    with pytest.raises(binding.CentraError):
        binding.centra_extend(ctx, 10, 3, 5, 4, off, nodes, 4, ph.picks, ph.cov, ph.npk)       # m < m_prev
    with pytest.raises(binding.CentraError):
        binding.centra_extend(ctx, 10, 3, 0, 10, off, nodes, 4, ph.picks, None, ph.npk)        # partial outputs
    with pytest.raises(binding.CentraError):
        binding.centra_extend(ctx, 10, 3, 0, 10, off, nodes, 4, t=1025, topk_sum=ph.topk, deg_topk=ph.dk,
                              b_max=ph.bm)
    with pytest.raises(binding.CentraError):
        binding.centra_extend(ctx, 10, 3, 0, 10, off, nodes, 4, t=4)                           # NULL outputs
    with pytest.raises(binding.CentraError):
        binding.centra_extend(ctx, 0, 3, 0, 10, off, nodes, 4, ph.picks, ph.cov, ph.npk)       # n == 0
    with pytest.raises(binding.CentraError):
        binding.centra_reserve(ctx, None, 0, 0, 10, 10, 3, 4)
    # an all-empty store is valid: nothing covered
    binding.centra_extend(ctx, 10, 3, 0, 10, off, nodes, 4, ph.picks, ph.cov, ph.npk)
    assert binding.centra_check(ctx) == binding.CENTRA_OK
    assert int(ph.npk.item()) == 0
