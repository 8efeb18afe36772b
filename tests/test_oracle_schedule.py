"""Pins of the oracle's sample schedule (samplingSchedule of Algorithm 1,
Section 4): the optimistic size against its defining property, the
geometric step and caps, and the fixed-size mode against a direct bound
evaluation with delta itself (Theorem bound_dev)."""
import math

import numpy as np
import pytest

import oracle
from paper_2306_03651_amd import inputs

A = 1.0 - math.exp(-1.0)
GEO, ADAPT, FIXED = oracle.SCHEDULE_GEOMETRIC, oracle.SCHEDULE_ADAPTIVE, oracle.SCHEDULE_FIXED


def eta_optimistic(m, L):
    # eta of Theorem bound_dev with R = 0 and nu = 1
    return math.sqrt(2.0 * L / m) + L / (3.0 * m)


@pytest.mark.parametrize("eps", [0.2, 0.05, 0.01])
@pytest.mark.parametrize("c_hat", [0.9, 0.5, 0.05, 1e-3])
@pytest.mark.parametrize("delta_next", [0.05, 0.1 / 2**7, 1e-9])
def test_optimistic_size_is_the_smallest_meeting_the_target(eps, c_hat, delta_next):
    # m_opt is the least integer m whose optimistic eta is at most
    # eps * c_hat / (1 - 1/e): checked by evaluating eta directly at m and
    # m - 1 (a different computation from the oracle's closed-form root)
    L = math.log(5.0 / delta_next)
    T = eps * c_hat / A
    m = oracle.next_sample_size(1, c_hat, eps, delta_next, 6, 5, 1 << 50, ADAPT)
    assert m > 2   # larger than the geometric step from 1
    assert eta_optimistic(m, L) <= T * (1 + 1e-12)
    assert eta_optimistic(m - 1, L) > T * (1 - 1e-12)
    # the dominant term alone gives the familiar 2L / T^2 as T -> 0
    if T < 1e-3:
        assert m == pytest.approx(2.0 * L / T**2, rel=0.05)


def test_schedule_steps_and_caps():
    # geometric: ceil(m * num / den), capped
    assert oracle.next_sample_size(1000, 0.5, 0.1, 0.01, 6, 5, 10**9, GEO) == 1200
    assert oracle.next_sample_size(1001, 0.5, 0.1, 0.01, 6, 5, 10**9, GEO) == 1202
    assert oracle.next_sample_size(1000, 0.5, 0.1, 0.01, 2, 1, 1500, GEO) == 1500
    # adaptive: never below the geometric step, no guess without coverage
    for m_i in [10, 1000, 10**6]:
        g = oracle.next_sample_size(m_i, 0.5, 0.05, 0.01, 6, 5, 10**12, GEO)
        a = oracle.next_sample_size(m_i, 0.5, 0.05, 0.01, 6, 5, 10**12, ADAPT)
        assert a >= g
    assert oracle.next_sample_size(1000, 0.0, 0.05, 0.01, 6, 5, 10**12, ADAPT) == 1200
    # a huge optimistic size is capped at m_max
    assert oracle.next_sample_size(1000, 1e-6, 0.01, 1e-6, 6, 5, 77777, ADAPT) == 77777
    # once the guess is below the geometric step, the step wins
    m_opt = oracle.next_sample_size(1, 0.5, 0.05, 0.01, 6, 5, 10**12, ADAPT)
    assert oracle.next_sample_size(m_opt, 0.5, 0.05, 0.01, 6, 5, 10**12, ADAPT) == -(-m_opt * 6 // 5)


def test_fixed_schedule_is_one_bound_with_delta():
    g = inputs.ba_graph(400, 3, 5)
    k, t, eps, delta, seed, m = 5, 8, 0.2, 0.05, 3, 3000
    rc, picks, res, mlog = oracle.progressive(g, k, t, eps, delta, seed, 0, m, 10 * m, schedule=FIXED,
                                              with_m_log=True)
    assert res.iterations == 1 and res.m_final == m and mlog == [m]
    off, nodes = oracle.sample_paths(g, seed, 0, 0, m)
    p2, cov = oracle.greedy_cover(g.n, off, nodes, k)
    am, topk, dk, bm = oracle.mcera(g.n, off, nodes, seed, 0, t, k)
    o = oracle.bound(m, int(cov[-1]), int(topk.sum()), t, dk, bm, eps, delta)   # delta, not delta / 2
    assert np.array_equal(picks, p2)
    assert res.eta == o.eta and res.xi == o.xi
    assert (rc == 0) == bool(o.certified)


def test_adaptive_schedule_run():
    # every iteration's size follows from the previous iteration's coverage:
    # replay the schedule from the oracle's own parts
    g = inputs.ba_graph(400, 3, 5)
    k, t, eps, delta, seed = 5, 8, 0.1, 0.1, 4
    rc, picks, res, mlog = oracle.progressive(g, k, t, eps, delta, seed, 0, 200, 400000, 6, 5,
                                              schedule=ADAPT, with_m_log=True)
    assert rc == 0 and len(mlog) == res.iterations >= 2
    off, nodes = oracle.sample_paths(g, seed, 0, 0, mlog[-1])
    for i in range(1, len(mlog)):
        m = mlog[i - 1]
        _, cov = oracle.greedy_cover(g.n, off[: m + 1], nodes[: int(off[m])], k)
        want = oracle.next_sample_size(m, int(cov[-1]) / m, eps, delta / 2**(i + 1), 6, 5, 400000, ADAPT)
        assert mlog[i] == want
        assert mlog[i] >= -(-m * 6 // 5)
    # the geometric schedule alone needs more iterations to certify
    rc_g, _, res_g = oracle.progressive(g, k, t, eps, delta, seed, 0, 200, 400000, 6, 5, schedule=GEO)
    assert rc_g == 0 and res_g.iterations > res.iterations


def test_bad_schedule_rejected():
    g = inputs.ba_graph(100, 2, 1)
    assert oracle.progressive(g, 3, 4, 0.1, 0.1, 1, 0, 10, 100, schedule=3)[0] < 0
