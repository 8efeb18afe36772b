"""The committed rocprofv3 summaries match the code they describe: the HBM
traffic summaries were taken on the current sampler source (bench.py reports
their traffic only then), and every summary records the command that made
it, which runs committed files only."""
import os
import re

import pytest

import bench

PROFILES = os.path.join(bench.ROOT, "profiles")


@pytest.mark.parametrize("workload", ["sparse", "skewed", "triangles", "kpaths"])
def test_traffic_summary_matches_the_sampler_source(workload):
    name = bench.WORKLOADS[workload]["traffic"]
    assert bench.read_traffic(name) is not None, f"{name} was taken on another sampler source: profile again"


def test_every_summary_gives_its_command():
    files = sorted(f for f in os.listdir(PROFILES) if f.endswith((".txt", ".md")))
    assert files
    for f in files:
        text = open(os.path.join(PROFILES, f)).read()
        cmds = re.findall(r"rocprofv3 [^\n]*-- python3 (\S+)", text)
        assert cmds, f"{f} gives no rocprofv3 command"
        for script in cmds:
            assert os.path.exists(os.path.join(bench.ROOT, script)), f"{f} runs {script}, which is not committed"
            assert not script.startswith("_work"), f"{f} runs a working file"
