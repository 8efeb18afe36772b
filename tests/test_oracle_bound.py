"""Pins for the oracle's bound arithmetic (Theorem bound_dev, eq. epsrade;
Algorithm 1 definition of xi and stopping condition) and its progressive
loop (Algorithm 1).

The bound is pinned to the fixed points it comes from (the proofs of
Theorem selfboundingupperbound and Theorem bound_dev solve quadratic
inequalities; nu - C/a and R - R~ must be their larger roots), to a
closed-form special case, and to the chain of inequalities of the proof of
Proposition main, of which the stopping condition is the middle link.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2306_03651_amd import inputs

A = 1.0 - math.exp(-1.0)

CASES = [
    # m, cov, sum_topk, t, deg_topk, b_max, eps, delta_i
    (10000, 4826, 2187, 10, 5568, 4, 0.05, 0.05),
    (4000000, 1900000, 812345, 64, 9000000, 9, 0.01, 0.1 / 2**7),
    (100, 3, 0, 1, 3, 1, 0.3, 0.5),
    (2**40, 2**39, 2**35, 1000, 2**38, 30, 0.001, 1e-9),
]


@pytest.mark.parametrize("case", CASES)
def test_fixed_point_roots(case):
    m, cov, sk, t, dk, bm, eps, di = case
    o = oracle.bound(*case)
    L = math.log(5 / di)
    C = cov / m
    assert o.c_hat == C
    # nu - C/a = xi is the larger root of x^2 - 2(L/m)x - 2CL/(a m) = 0
    x = o.nu - C / A
    assert x == pytest.approx(o.xi, rel=1e-12)
    assert x > 0
    assert x * x - 2 * (L / m) * x - 2 * C * L / (A * m) == pytest.approx(0.0, abs=1e-9 * x * x)
    # R - R~ is the larger root of y^2 - 2(L/m)y - 2 L R~/m = 0
    y = o.r - o.rtilde
    assert y > 0
    assert y * y - 2 * (L / m) * y - 2 * L * o.rtilde / m == pytest.approx(0.0, abs=1e-9 * y * y)
    # R~ - AMCERA squared is 4 w L / (t m), with w = b_max * D_k / m
    assert o.wimpy == pytest.approx(bm * dk / m, rel=1e-15)
    assert o.amcera == pytest.approx(sk / (t * m), rel=1e-15)
    z = o.rtilde - o.amcera
    assert z * z == pytest.approx(4 * o.wimpy * L / (t * m), rel=1e-9)


def test_closed_form_when_everything_is_zero():
    # C = 0, AMCERA = 0, w = 0: xi = 2L/m, R~ = 0, R = 2L/m,
    # eta = 4L/m + sqrt(2L(2L/m + 8L/m)/m) + L/(3m) = (4 + sqrt(20) + 1/3) L/m.
    m, di = 1000, 0.01
    o = oracle.bound(m, 0, 0, 5, 0, 0, 0.1, di)
    L = math.log(5 / di)
    assert o.xi == pytest.approx(2 * L / m, rel=1e-14)
    assert o.rtilde == 0.0
    assert o.r == pytest.approx(2 * L / m, rel=1e-14)
    assert o.eta == pytest.approx((4 + math.sqrt(20) + 1 / 3) * L / m, rel=1e-14)
    assert not o.certified


@pytest.mark.parametrize("case", CASES)
def test_stop_condition_is_proof_chain_middle_link(case):
    # Proof of Proposition main: certification must be equivalent to
    # C/a + xi <= (C - eta)/(a - eps).
    m, cov, sk, t, dk, bm, eps, di = case
    o = oracle.bound(*case)
    C = cov / m
    lhs = C / A + o.xi
    rhs = (C - o.eta) / (A - eps)
    if abs(lhs - rhs) > 1e-12 * max(1.0, abs(lhs)):
        assert bool(o.certified) == (lhs <= rhs)


def test_bound_shrinks_with_m():
    etas = [oracle.bound(m, m // 2, m // 100, 10, m, 5, 0.05, 0.01).eta for m in [10**3, 10**4, 10**5, 10**6]]
    assert all(a > b for a, b in zip(etas, etas[1:]))
    # eta ~ 1/sqrt(m) asymptotically (Sec. 5: both bounds decrease as 1/sqrt(m))
    assert etas[2] / etas[3] == pytest.approx(math.sqrt(10), rel=0.2)


def test_progressive_matches_its_parts():
    g = inputs.ba_graph(400, 3, 5)
    k, t, eps, delta, seed = 5, 8, 0.2, 0.1, 3
    rc, picks, res = oracle.progressive(g, k, t, eps, delta, seed, 0, 500, 8000)
    assert res.iterations >= 1
    m = res.m_final
    # schedule 500 -> 1000 -> ... doubling, capped at 8000
    sched = [500]
    while sched[-1] < 8000:
        sched.append(min(2 * sched[-1], 8000))
    assert m == sched[res.iterations - 1]
    off, nodes = oracle.sample_paths(g, seed, 0, 0, m)
    p2, cov = oracle.greedy_cover(g.n, off, nodes, k)
    assert np.array_equal(picks, p2)
    assert res.coverage == cov[-1]
    am, topk, dk, bm = oracle.mcera(g.n, off, nodes, seed, 0, t, k)
    o = oracle.bound(m, int(cov[-1]), int(topk.sum()), t, dk, bm, eps, delta / 2**res.iterations)
    assert res.eta == o.eta and res.xi == o.xi and res.amcera == am
    assert (rc == 0) == bool(o.certified)
    if rc == 0 and res.iterations > 1:
        # the previous iteration was not certified
        mp = sched[res.iterations - 2]
        offp, nodesp = off[: mp + 1], nodes[: int(off[mp])]
        _, covp = oracle.greedy_cover(g.n, offp, nodesp, k)
        amp, topkp, dkp, bmp = oracle.mcera(g.n, offp, nodesp, seed, 0, t, k)
        op = oracle.bound(mp, int(covp[-1]), int(topkp.sum()), t, dkp, bmp, eps, delta / 2**(res.iterations - 1))
        assert not op.certified


def test_progressive_rejects_bad_parameters():
    g = inputs.ba_graph(100, 2, 1)
    assert oracle.progressive(g, 0, 4, 0.1, 0.1, 1, 0, 10, 100)[0] < 0
    assert oracle.progressive(g, 3, 4, 0.7, 0.1, 1, 0, 10, 100)[0] < 0     # eps >= 1 - 1/e
    assert oracle.progressive(g, 3, 4, 0.1, 1.0, 1, 0, 10, 100)[0] < 0


def test_proposition_main_failure_rate():
    # Prop. main: the output is a (1 - 1/e - eps)-approximation with
    # probability >= 1 - delta.  Exact C(S) on a small graph by enumeration.
    import itertools
    import networkx as nx
    from tests.test_oracle_sampler import exact_set_betweenness, to_nx
    g = inputs.ba_graph(16, 2, 9)
    G = to_nx(g)
    k, eps, delta = 2, 0.25, 0.2
    cache = {}

    def C(S):
        key = tuple(sorted(S))
        if key not in cache:
            cache[key] = exact_set_betweenness(G, g.n, set(S))
        return cache[key]

    opt = max(C(S) for S in itertools.combinations(range(g.n), k))
    fails = 0
    runs = 20
    for seed in range(runs):
        rc, picks, res = oracle.progressive(g, k, 8, eps, delta, 1000 + seed, 0, 2000, 64000)
        assert rc == 0
        if C(set(int(x) for x in picks)) < (A - eps) * opt:
            fails += 1
    assert fails <= max(1, int(delta * runs))


# ---------------------------------------------------------------------------
# HEDGE-P's union bound (reading R17)
def test_log_sets_matches_exact_binomial_sums():
    # ln sum_{j <= k} C(n, j) against Python's exact integers
    for n, k in [(2, 1), (10, 3), (40, 40), (1000, 5), (10**6, 50), (2**30, 100)]:
        exact = math.log(sum(math.comb(n, j) for j in range(min(k, n) + 1)))
        assert oracle.log_sets(n, k) == pytest.approx(exact, rel=1e-9)


def test_hedge_bound_closed_forms():
    # k = 1: N_1 = n + 1 sets, eta = sqrt(ln(2 (n + 1) / delta) / (2 m))
    n, m, delta = 1000, 50000, 0.05
    o = oracle.hedge_bound(m, 20000, n, 1, 0.1, delta)
    assert o.eta == pytest.approx(math.sqrt(math.log(2 * (n + 1) / delta) / (2 * m)), rel=1e-12)
    assert o.c_hat == 0.4
    # the stopping rule: eta <= eps (C - eta) / 2, tested on both sides of
    # the sample size that first satisfies it
    eps = 0.1
    lo = 1
    while not oracle.hedge_bound(lo, lo // 2, n, 3, eps, delta).certified:
        lo *= 2
    hi = lo
    lo //= 2
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if oracle.hedge_bound(mid, mid // 2, n, 3, eps, delta).certified:
            hi = mid
        else:
            lo = mid
    for mm, want in [(hi, True), (lo, False)]:
        o = oracle.hedge_bound(mm, mm // 2, n, 3, eps, delta)
        assert bool(o.certified) == want
        assert (o.eta <= eps * (o.c_hat - o.eta) / 2) == want
    # eta ~ 1/sqrt(m) and grows with k and 1/delta
    a = oracle.hedge_bound(10**4, 5000, n, 5, eps, delta).eta
    b = oracle.hedge_bound(4 * 10**4, 20000, n, 5, eps, delta).eta
    assert a == pytest.approx(2 * b, rel=1e-12)
    assert oracle.hedge_bound(10**4, 5000, n, 6, eps, delta).eta > a
    assert oracle.hedge_bound(10**4, 5000, n, 5, eps, delta / 10).eta > a


def test_hedge_p_progressive_matches_its_parts():
    # HEDGE-P: Algorithm 1's loop with eta^UB; the result equals greedy and
    # the union bound recomputed on the final sample, with delta_i = delta/2^i
    from paper_2306_03651_amd import inputs
    g = inputs.ba_graph(300, 3, 4)
    k, eps, delta = 5, 0.2, 0.1
    rc, picks, res, mlog = oracle.progressive(g, k, 8, eps, delta, 2, 0, 1000, 2**22, with_m_log=True,
                                              method=oracle.METHOD_HEDGE_P)
    assert rc == 0
    off, nodes = oracle.sample_paths(g, 2, 0, 0, res.m_final)
    p2, cov = oracle.greedy_cover(g.n, off, nodes, k)
    assert np.array_equal(picks, p2) and res.coverage == cov[-1]
    o = oracle.hedge_bound(res.m_final, int(cov[-1]), g.n, k, eps, delta / 2**res.iterations)
    assert o.certified and res.eta == o.eta and res.amcera == 0
    if res.iterations > 1:
        prev = mlog[-2]
        off, nodes = oracle.sample_paths(g, 2, 0, 0, prev)
        _, cov = oracle.greedy_cover(g.n, off, nodes, k)
        assert not oracle.hedge_bound(prev, int(cov[-1]), g.n, k, eps, delta / 2**(res.iterations - 1)).certified
