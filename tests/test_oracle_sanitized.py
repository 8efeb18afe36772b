"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc): tests/oracle_sanitize.c runs every oracle function on small graphs
(a grid with shifted levels, a random directed graph, a complete graph) and
must finish with no sanitizer report, no leak and no failed check."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def sanitizers_available(tmp):
    probe = tmp / "probe.c"
    probe.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc"] + FLAGS + [str(probe), "-o", str(tmp / "probe")], capture_output=True)
    return r.returncode == 0


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    if not sanitizers_available(tmp_path):
        pytest.skip("gcc sanitizer runtimes are not installed")
    exe = tmp_path / "oracle_sanitize"
    subprocess.check_call(["gcc"] + FLAGS + ["-I", os.path.join(ROOT, "oracle"),
                                             os.path.join(ROOT, "tests", "oracle_sanitize.c"),
                                             os.path.join(ROOT, "oracle", "centra_oracle.c"), "-lm", "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failed checks" in r.stdout
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
