"""GPU tests of checkpoint / resume (centra_progressive_resumable) and of
the command-line driver: a run stopped after any iteration and resumed --
on the same context (the kept sample is extended), on a fresh context (the
sample is redrawn) or after another call took the context's state -- gives
the uninterrupted run's picks, coverage, sample sizes, bound values and
per-iteration records, bit for bit; checkpoints of another graph, other
parameters or another version are refused; the driver, killed by its
host-forced fault after iteration i, resumes to the same result and log."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2306_03651_amd import binding, inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RES_FIELDS = ["n_picked", "iterations", "certified", "coverage", "m_final", "c_hat", "amcera", "wimpy", "xi", "nu",
              "rtilde", "r", "eta"]
IT_FIELDS = ["i", "m", "coverage", "sum_topk", "deg_topk", "b_max", "delta_i", "amcera", "wimpy", "xi", "nu",
             "rtilde", "r", "eta", "certified", "arcs", "nodes"]


def mix64(z):
    m = (1 << 64) - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def graph_hash(g):
    """The fingerprint as the header defines it, from the host CSR."""
    h = mix64(g.n | ((1 if g.directed else 0) << 32))
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    ci = np.asarray(g.col_idx, dtype=np.uint64)
    src = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(rp))
    z = (src << np.uint64(32)) | ci
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return (h + int(z.sum(dtype=np.uint64))) & ((1 << 64) - 1)


def params(k=12, t=16, eps=0.01, seed=5, inst=2, m_init=2000, m_max=64000, schedule=0, space=0, kappa=0, method=0):
    return binding.Params(k, t, eps, 0.1, seed, inst, m_init, m_max, 2, 1, schedule, space, kappa, method)


def same_result(a, b):
    (rc_a, picks_a, res_a), (rc_b, picks_b, res_b) = a, b
    assert rc_a == rc_b
    assert np.array_equal(picks_a, picks_b)
    for f in RES_FIELDS:
        assert getattr(res_a, f) == getattr(res_b, f), f


def same_iteration(x, y, work=True):
    # arcs and nodes count the sampling work done, which includes the redraw
    # of samples [0, m_i) in the first iteration of a resume elsewhere
    for f in IT_FIELDS:
        if work or f not in ("arcs", "nodes"):
            assert getattr(x, f) == getattr(y, f), f


def full_run(ctx, dg, p):
    rc, picks, res, its, _ = binding.centra_progressive_resumable(ctx, dg.handle, p)
    return (rc, picks, res), its


@pytest.mark.parametrize("kind", ["ba", "rmat"])
def test_graph_hash(ctx, kind):
    g = inputs.ba_graph(3000, 4, 2) if kind == "ba" else inputs.rmat_graph(12, 8, seed=3)
    dg = binding.DeviceGraph(ctx, g)
    try:
        assert dg.hash() == graph_hash(g)
    finally:
        dg.release()


CASES = {
    "paths": dict(),
    "adaptive": dict(schedule=binding.CENTRA_SCHEDULE_ADAPTIVE, eps=0.02),
    "bidir": dict(space=binding.CENTRA_SPACE_PATHS_BIDIR),
    "triangles": dict(space=binding.CENTRA_SPACE_TRIANGLES, k=6, eps=0.02),
    "kpaths": dict(space=binding.CENTRA_SPACE_KPATHS, kappa=4, eps=0.02),
    "hedge": dict(method=binding.CENTRA_METHOD_HEDGE_P, eps=0.05),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_stop_and_resume_every_iteration(ctx, case):
    g = inputs.ba_graph(3000, 4, 9)
    dg = binding.DeviceGraph(ctx, g)
    p = params(**CASES[case])
    try:
        want, want_its = full_run(ctx, dg, p)
        n_it = want[2].iterations
        say(f"resume {case}: uninterrupted run of {n_it} iterations, m_final {want[2].m_final}")
        assert n_it >= 2
        for stop in range(1, n_it):
            # stop after `stop`, resume on the same context (kept sample)
            rc, _, res, its, ck = binding.centra_progressive_resumable(ctx, dg.handle, p, stop_after=stop)
            assert rc == binding.CENTRA_STOPPED and res.iterations == stop and ck.i == stop
            same_iteration(its[stop], want_its[stop])
            assert ck.m_i == want_its[stop].m and ck.m_next == want_its[stop + 1].m
            rc2, picks2, res2, its2, _ = binding.centra_progressive_resumable(ctx, dg.handle, p, resume=ck)
            same_result((rc2, picks2, res2), want)
            assert sorted(its2) == list(range(stop + 1, n_it + 1))
            for i, it in its2.items():
                same_iteration(it, want_its[i])
        # resume in a fresh context: the sample is redrawn
        _, _, _, _, ck = binding.centra_progressive_resumable(ctx, dg.handle, p, stop_after=n_it - 1)
        ctx2 = binding.centra_create(0, 0)
        dg2 = binding.DeviceGraph(ctx2, g)
        try:
            rc3, picks3, res3, its3, _ = binding.centra_progressive_resumable(ctx2, dg2.handle, p, resume=ck)
            same_result((rc3, picks3, res3), want)
            for i, it in its3.items():
                same_iteration(it, want_its[i], work=i > ck.i + 1)
        finally:
            dg2.release()
            binding.centra_destroy(ctx2)
    finally:
        dg.release()


def test_resume_after_other_work_and_refusals(ctx):
    import torch
    g = inputs.rmat_graph(11, 8, seed=5)
    dg = binding.DeviceGraph(ctx, g)
    p = params(k=8, t=24, eps=0.02, m_init=3000, m_max=48000)
    try:
        want, want_its = full_run(ctx, dg, p)
        _, _, _, _, ck = binding.centra_progressive_resumable(ctx, dg.handle, p, stop_after=2)
        # another call builds an incidence and AMCERA counts on the context
        off = torch.tensor([0, 2, 3], dtype=torch.int64, device="cuda")
        nodes = torch.tensor([1, 4, 4], dtype=torch.int32, device="cuda")
        tk = torch.zeros(4, dtype=torch.int64, device="cuda")
        dk = torch.zeros(1, dtype=torch.int64, device="cuda")
        bm = torch.zeros(1, dtype=torch.int32, device="cuda")
        binding.centra_mcera(ctx, 10, off, nodes, 1, 0, 4, 2, tk, dk, bm)
        rc, picks, res, its, _ = binding.centra_progressive_resumable(ctx, dg.handle, p, resume=ck)
        same_result((rc, picks, res), want)
        for i, it in its.items():
            same_iteration(it, want_its[i], work=i > ck.i + 1)
        # refusals: other parameters, another graph, another version, bad sizes
        other = params(k=8, t=24, eps=0.02, m_init=3000, m_max=48000, seed=6)
        with pytest.raises(binding.CentraError, match="parameters"):
            binding.centra_progressive_resumable(ctx, dg.handle, other, resume=ck)
        g2 = inputs.rmat_graph(11, 8, seed=6)
        dg2 = binding.DeviceGraph(ctx, g2)
        try:
            with pytest.raises(binding.CentraError, match="graph"):
                binding.centra_progressive_resumable(ctx, dg2.handle, p, resume=ck)
        finally:
            dg2.release()
        for field, value in [("version", 7), ("m_next", ck.m_i), ("i", 0)]:
            bad = binding.Checkpoint.from_dict(ck.to_dict())
            setattr(bad, field, value)
            with pytest.raises(binding.CentraError):
                binding.centra_progressive_resumable(ctx, dg.handle, p, resume=bad)
        bad = binding.Checkpoint.from_dict(ck.to_dict())
        bad.entries += 1   # the redrawn sample must have the checkpoint's entries
        ctx2 = binding.centra_create(0, 0)
        dg3 = binding.DeviceGraph(ctx2, g)
        try:
            with pytest.raises(binding.CentraError, match="entries"):
                binding.centra_progressive_resumable(ctx2, dg3.handle, p, resume=bad)
        finally:
            dg3.release()
            binding.centra_destroy(ctx2)
        fixed = params(k=8, t=24, eps=0.02, m_init=3000, m_max=48000, schedule=binding.CENTRA_SCHEDULE_FIXED)
        with pytest.raises(binding.CentraError):
            binding.centra_progressive_resumable(ctx, dg.handle, fixed, resume=ck)
    finally:
        dg.release()


def driver(tmp, extra_env=None, resume=False, name="run"):
    args = [sys.executable, "-u", "-m", "paper_2306_03651_amd.run", "--graph", "ba", "--n", "4000", "--m0", "4",
            "--k", "10", "--t", "16", "--eps", "0.01", "--m-init", "2000", "--m-max", "64000",
            "--checkpoint", str(tmp / f"{name}.ck.json"), "--log", str(tmp / f"{name}.jsonl"),
            "--result", str(tmp / f"{name}.res.json")]
    if resume:
        args.append("--resume")
    env = dict(os.environ)
    env.pop("CENTRA_FAULT_AFTER_ITER", None)
    env.update(extra_env or {})
    return subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=240)


def strip_ms(lines, redrawn_i=0):
    """Records without timings (and without the work counts of the first
    iteration of a resume, which redraws the earlier samples)."""
    out = []
    for line in lines:
        d = json.loads(line)
        for f in ("ms_sample", "ms_cover", "ms_mcera") + (("arcs", "nodes") if d["i"] == redrawn_i else ()):
            d.pop(f)
        out.append(d)
    return out


def test_driver_fault_and_resume(tmp_path):
    say("driver: uninterrupted run")
    full = driver(tmp_path, name="full")
    assert full.returncode == 0, full.stderr[-2000:]
    say("driver: run with a host-forced fault after iteration 2")
    cut = driver(tmp_path, {"CENTRA_FAULT_AFTER_ITER": "2"}, name="cut")
    assert cut.returncode == 75, (cut.returncode, cut.stderr[-2000:])
    assert "fault injected after iteration 2" in cut.stdout
    assert not (tmp_path / "cut.res.json").exists()
    ck = json.loads((tmp_path / "cut.ck.json").read_text())
    assert ck["i"] == 2
    # a log record written after the checkpoint (a fault between the two)
    # is dropped on resume
    with open(tmp_path / "cut.jsonl", "a") as f:
        f.write(json.dumps({"i": 3, "stale": True}) + "\n")
    say("driver: resumed run")
    res = driver(tmp_path, resume=True, name="cut")
    assert res.returncode == 0, res.stderr[-2000:]
    a = json.loads((tmp_path / "full.res.json").read_text())
    b = json.loads((tmp_path / "cut.res.json").read_text())
    assert a == b
    la = strip_ms((tmp_path / "full.jsonl").read_text().splitlines(), redrawn_i=3)
    lb = strip_ms((tmp_path / "cut.jsonl").read_text().splitlines(), redrawn_i=3)
    assert la == lb and [d["i"] for d in la] == list(range(1, a["iterations"] + 1))
    assert a["iterations"] >= 3 and a["rc"] in (binding.CENTRA_OK, binding.CENTRA_NOT_CERTIFIED)
