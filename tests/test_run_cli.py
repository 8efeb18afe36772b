"""CPU checks of the command-line driver's host logic: argument defaults
(the sparse benchmark configuration), the log trim a resume applies, and
that it refuses to run without a HIP device (no CPU fallback)."""
import json
import subprocess
import sys

import pytest

from paper_2306_03651_amd import binding, run


def test_defaults_are_the_benchmark_configuration():
    a = run.parse(["--checkpoint", "c", "--log", "l", "--result", "r"])
    p = run.make_params(a)
    assert (a.graph, a.n, a.m0) == ("ba", 100_000, 5)
    assert (p.k, p.t, p.eps, p.delta, p.m_init, p.m_max) == (50, 64, 0.01, 0.1, 100_000, 4_000_000)
    assert p.schedule == binding.CENTRA_SCHEDULE_GEOMETRIC and p.space == binding.CENTRA_SPACE_SHORTEST_PATHS


def test_trim_log_drops_records_after_the_checkpoint(tmp_path):
    log = tmp_path / "it.jsonl"
    log.write_text("".join(json.dumps({"i": i, "m": 10 * i}) + "\n" for i in range(1, 6)))
    run.trim_log(str(log), 3)
    assert [json.loads(x)["i"] for x in log.read_text().splitlines()] == [1, 2, 3]
    run.trim_log(str(tmp_path / "missing.jsonl"), 3)   # nothing to trim


def test_write_atomic_replaces(tmp_path):
    f = tmp_path / "ck.json"
    run.write_atomic(str(f), "a\n")
    run.write_atomic(str(f), "b\n")
    assert f.read_text() == "b\n" and not (tmp_path / "ck.json.tmp").exists()


def test_refuses_without_a_device(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    r = subprocess.run([sys.executable, "-m", "paper_2306_03651_amd.run", "--checkpoint", str(tmp_path / "c"),
                        "--log", str(tmp_path / "l"), "--result", str(tmp_path / "r")],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "HIP device" in r.stderr
