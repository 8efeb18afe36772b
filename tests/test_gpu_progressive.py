"""GPU parity of centra_progressive (Algorithm 1) against the oracle's progressive loop:
identical iterations, sample sizes, picks and coverage; FP64 bound values
within 1e-12 relative."""
import numpy as np
import pytest

import oracle
from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

FIELDS = ["c_hat", "amcera", "wimpy", "xi", "nu", "rtilde", "r", "eta"]


def compare(g, ctx, k, t, eps, delta, seed, inst, m_init, m_max, num=2, den=1,
            schedule=binding.CENTRA_SCHEDULE_GEOMETRIC):
    dg = binding.DeviceGraph(ctx, g)
    try:
        rc, picks, res, log = binding.centra_progressive(ctx, dg.handle, k, t, eps, delta, seed, inst, m_init,
                                                         m_max, num, den, log_cap=256, schedule=schedule)
    finally:
        dg.release()
    wrc, wpicks, wres, wlog = oracle.progressive(g, k, t, eps, delta, seed, inst, m_init, m_max, num, den,
                                                 schedule=schedule, with_m_log=True)
    assert rc == wrc
    assert np.array_equal(picks, wpicks)
    assert res.iterations == wres.iterations and res.m_final == wres.m_final
    assert res.coverage == wres.coverage and res.n_picked == wres.n_picked
    assert res.certified == wres.certified
    for f in FIELDS:
        assert getattr(res, f) == pytest.approx(getattr(wres, f), rel=1e-12, abs=1e-300), f
    assert [it.m for it in log] == wlog
    if schedule == binding.CENTRA_SCHEDULE_GEOMETRIC:
        sched = [m_init]
        while len(sched) < res.iterations:
            sched.append(min(-(-sched[-1] * num // den), m_max))
        assert wlog == sched
    assert [it.i for it in log] == list(range(1, res.iterations + 1))
    return res


def test_c1_configuration(ctx):
    # BA n=2000, m0=5; m = 10,000, k = 10, t = 10, eps = 0.05, delta = 0.1:
    # one iteration (delta_1 = 0.05).
    g = inputs.ba_graph(2000, 5, 1)
    say("progressive C1")
    res = compare(g, ctx, 10, 10, 0.05, 0.1, 1, 0, 10000, 10000)
    assert res.iterations == 1


def test_c1_continued_until_certified(ctx):
    g = inputs.ba_graph(2000, 5, 1)
    say("progressive C1 continued")
    res = compare(g, ctx, 10, 10, 0.05, 0.1, 1, 0, 10000, 1_280_000)
    assert res.certified


def test_directed_and_non_doubling_schedule(ctx):
    g = inputs.rmat_graph(11, 8, seed=2)
    say("progressive rmat11 growth 6/5")
    compare(g, ctx, 7, 33, 0.2, 0.05, 3, 2, 3000, 20000, 6, 5)


def test_many_iterations_restart_the_incidence(ctx):
    # Growth 1.05 from 1,000 to 150,000 samples: 104 iterations.  Each
    # iteration appends an incidence segment; after 64 of them the loop
    # rebuilds one segment from sample 0 and recounts the trial sums, and
    # appends again from there.
    say("progressive: 104 iterations at growth 21/20")
    compare(inputs.ba_graph(2000, 5, 1), ctx, 10, 16, 0.01, 0.1, 3, 0, 1000, 150000, 21, 20)


def test_adaptive_schedule(ctx):
    # the paper's schedule: growth 1.2 combined with the optimistic guess
    g = inputs.ba_graph(2000, 5, 1)
    say("progressive C1 adaptive")
    res = compare(g, ctx, 10, 10, 0.05, 0.1, 1, 0, 2000, 1_280_000, 6, 5, schedule=binding.CENTRA_SCHEDULE_ADAPTIVE)
    assert res.certified


def test_fixed_schedule(ctx):
    g = inputs.rmat_graph(11, 8, seed=2)
    say("progressive fixed m")
    for m in [500, 20000]:
        res = compare(g, ctx, 7, 33, 0.2, 0.05, 3, 2, m, m, schedule=binding.CENTRA_SCHEDULE_FIXED)
        assert res.iterations == 1 and res.m_final == m


def test_bad_schedule_rejected(ctx):
    g = inputs.ba_graph(300, 2, 1)
    dg = binding.DeviceGraph(ctx, g)
    try:
        with pytest.raises(binding.CentraError) as e:
            binding.centra_progressive(ctx, dg.handle, 3, 4, 0.1, 0.1, 1, 0, 10, 100, schedule=7)
        assert e.value.code == binding.CENTRA_EINVAL
    finally:
        dg.release()


@pytest.mark.parametrize("name", ["ba2000", "dir"])
def test_hedge_p_matches_oracle(ctx, name):
    # HEDGE-P (Sec. 5's comparison method): the same iterations with the
    # union bound; picks, coverage, sample sizes bit-exact and eta^UB within
    # 1e-12 of the oracle's
    g = inputs.ba_graph(2000, 5, 1) if name == "ba2000" else inputs.rmat_graph(11, 8, seed=4)
    dg = binding.DeviceGraph(ctx, g)
    try:
        say(f"HEDGE-P on {name}")
        rc, picks, res, log = binding.centra_progressive(ctx, dg.handle, 5, 8, 0.2, 0.1, 3, 0, 2000, 1 << 20,
                                                         method=binding.CENTRA_METHOD_HEDGE_P)
    finally:
        dg.release()
    wrc, wpicks, wres, wlog = oracle.progressive(g, 5, 8, 0.2, 0.1, 3, 0, 2000, 1 << 20, with_m_log=True,
                                                 method=oracle.METHOD_HEDGE_P)
    assert rc == wrc and np.array_equal(picks, wpicks)
    assert (res.iterations, res.m_final, res.coverage) == (wres.iterations, wres.m_final, wres.coverage)
    assert [it.m for it in log] == wlog
    assert res.eta == pytest.approx(wres.eta, rel=1e-12) and res.amcera == 0.0
