"""GPU test of centra_greedy_cover_noalloc, the greedy cover whose
workspaces come from a fixed device array instead of allocations: called
through the C ABI twice in a row (the second call on a smaller input, so it
runs over what the first left in the array), each result equal to
centra_greedy_cover's and the oracle's; sizes beyond the array are refused
before any launch."""
import numpy as np
import pytest
import torch

import oracle
from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import say, to_dev_u32, to_dev_u64

pytestmark = pytest.mark.gpu


def run(fn, n, off, nodes, k):
    picks = torch.full((k,), -1, dtype=torch.int32, device="cuda")
    cov = torch.full((k,), -1, dtype=torch.int64, device="cuda")
    npk = torch.zeros(1, dtype=torch.int32, device="cuda")
    fn(n, to_dev_u64(off), to_dev_u32(nodes), k, picks, cov, npk)
    torch.cuda.synchronize()
    c = int(npk.item())
    return picks.cpu().numpy().view(np.uint32)[:c].copy(), cov.cpu().numpy().astype(np.uint64)[:c].copy()


def test_noalloc_greedy_matches_greedy_cover(ctx):
    big_off, big_nodes = inputs.hyperedges(1_000_000, 200_000, max_len=8, skew=3, seed=5)
    g = inputs.ba_graph(2000, 5, 1)
    small_off, small_nodes = oracle.sample_paths(g, 1, 0, 0, 10000)
    cases = [("synthetic n=1e6 m=2e5 k=50", 1_000_000, big_off, big_nodes, 50),
             ("BA 2000 paths m=1e4 k=10", 2000, small_off, small_nodes, 10)]
    for name, n, off, nodes, k in cases:
        say(f"noalloc greedy: {name}")
        got = run(binding.centra_greedy_cover_noalloc, n, off, nodes, k)
        want = run(lambda *a: binding.centra_greedy_cover(ctx, *a), n, off, nodes, k)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), name
        if n == 2000:
            wp, wc = oracle.greedy_cover(n, off, nodes, k)
            assert np.array_equal(got[0], wp) and np.array_equal(got[1], wc)


def test_noalloc_greedy_refuses_oversize():
    n = 3_000_000   # 28 n bytes alone exceed the fixed array
    off = torch.zeros(11, dtype=torch.int64, device="cuda")
    picks = torch.zeros(4, dtype=torch.int32, device="cuda")
    cov = torch.zeros(4, dtype=torch.int64, device="cuda")
    npk = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.CentraError) as e:
        binding.centra_greedy_cover_noalloc(n, off, None, 4, picks, cov, npk)
    assert e.value.code == binding.CENTRA_ENOSPC
    assert "scratch" in str(e.value)
