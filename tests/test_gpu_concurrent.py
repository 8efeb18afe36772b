"""Independent contexts used at the same time from two host threads, each on
its own stream, give the same results as when run alone (the library keeps
no state outside its contexts; results are pure functions of the inputs)."""
import threading

import numpy as np
import pytest
import torch

from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

BUDGET = 8 << 30


def run_query(g, k, t, eps, delta, seed, m_init, m_max, stream=None):
    ctx = binding.centra_create(0, BUDGET)
    try:
        dg = binding.DeviceGraph(ctx, g)
        try:
            rc, picks, res, log = binding.centra_progressive(ctx, dg.handle, k, t, eps, delta, seed, 0, m_init,
                                                             m_max, 2, 1, stream=stream)
            if stream is not None:
                stream.synchronize()
            return rc, picks.tolist(), res.m_final, res.coverage, res.eta, [it.m for it in log]
        finally:
            dg.release()
    finally:
        binding.centra_destroy(ctx)


def test_two_contexts_in_parallel_match_alone():
    queries = [
        (inputs.ba_graph(2000, 5, 1), 10, 10, 0.05, 0.1, 1, 2000, 64000),
        (inputs.rmat_graph(11, 8, seed=2), 7, 33, 0.2, 0.05, 3, 3000, 24000),
    ]
    say("two contexts: standalone runs")
    alone = [run_query(*q) for q in queries]
    results = [None, None]
    errors = []

    def worker(i):
        try:
            with torch.cuda.stream(torch.cuda.Stream()):
                s = torch.cuda.current_stream()
                for _ in range(3):
                    r = run_query(*queries[i], stream=s)
                    if r != alone[i]:
                        errors.append((i, r, alone[i]))
                results[i] = r
        except Exception as e:   # surfaced below
            errors.append((i, repr(e)))

    say("two contexts: concurrent runs")
    th = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=240)
    assert not any(x.is_alive() for x in th)
    assert not errors, errors
    assert results == alone
