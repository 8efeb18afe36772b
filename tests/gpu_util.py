"""Helpers for the GPU parity tests: move library outputs to numpy."""
import numpy as np
import torch


def off_np(t):
    return t.cpu().numpy().astype(np.uint64)


def nodes_np(t):
    return t.cpu().numpy().view(np.uint32)


def to_dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def to_dev_u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if a.size == 0:
        return torch.zeros(1, dtype=torch.int32, device="cuda")[:0]
    return torch.from_numpy(a.view(np.int32)).cuda()


def say(*args):
    print(*args, flush=True)


def check_graph_info(dg, g, cbo=0):
    """Asserts the library's prepared-graph info against values computed
    without it: the largest in-degree from the transpose (numpy) and the
    oracle's count bit budget C (lowered to the test override, if any).
    Returns that C, for the oracle's sampler."""
    import oracle
    indeg = np.bincount(np.asarray(g.col_idx, dtype=np.int64), minlength=g.n)
    c = oracle.count_bits(g)
    if cbo and cbo < c:
        c = cbo
    assert tuple(dg.info()) == (int(indeg.max()), c)
    return c


def oracle_paths(g, seed, inst, indices, c_bits, threads=16):
    """The oracle's hyperedges and SampleInfos of the given sample indices,
    drawn on up to `threads` host threads (the oracle's C calls release the
    GIL; each index is independent)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    og = oracle.OracleGraph(g)
    threads = max(1, min(threads, os.cpu_count() or 1))
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda i: oracle.sample_path(g, seed, inst, int(i), c_bits=c_bits, og=og), indices))
