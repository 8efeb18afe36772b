"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every library source is compiled with the sanitizers on its host side only
(the device code is built as usual) and linked with tests/host_sanitize.cpp,
which drives the C ABI.  Without a GPU the program runs the calls that need
no device (the bound formulas, the VC-dimension bounds, the parameter hash,
argument checks, centra_create without a device); the same program run with
--gpu on a machine with one drives every device entry point as well.  A run
passes when it reports no failed check and the sanitizers report nothing.

The CPU test builds the program into tests/_san/ with a stamp of the sources
it was built from; the GPU test runs that build when the stamp matches the
sources (nothing is compiled on the GPU machine)."""
import concurrent.futures
import hashlib
import os
import shutil
import subprocess

import pytest

from paper_2306_03651_amd import _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PREBUILT_DIR = os.path.join(ROOT, "tests", "_san")
HARNESS_SRC = os.path.join(ROOT, "tests", "host_sanitize.cpp")
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def rocm() -> str:
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def sources() -> list:
    return [os.path.join(_build.CSRC, s) for s in _build.SOURCES] + [HARNESS_SRC]


def sources_stamp() -> str:
    """sha256 of every source the program is built from (library sources,
    the headers beside them and the public header, and the driver program)."""
    files = sources() + sorted(os.path.join(_build.CSRC, f) for f in os.listdir(_build.CSRC) if f.endswith(".hpp"))
    files.append(os.path.join(ROOT, "include", "centra.h"))
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()


def build_harness(out_dir: str) -> str:
    """Compiles the library sources and the driver program with host-side
    sanitizers into out_dir and links them; returns the program's path."""
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()

    def compile_one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        cmd = [_build.hipcc()] + _build.FLAGS + SANITIZE + ["-x", "hip", "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed for {src}:\n{r.stderr[-4000:]}")
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = os.path.join(out_dir, "host_sanitize")
    lib = os.path.join(rocm(), "lib")
    cmd = [os.path.join(rocm(), "llvm", "bin", "clang++"), "-fsanitize=address,undefined", "-o", exe] + objs + \
          ["-L", lib, "-lamdhip64", f"-Wl,-rpath,{lib}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    for obj in objs:
        os.remove(obj)
    return exe


# The ROCm runtime keeps a few allocations to the end of the process on
# purpose; a leak whose stack passes through it is not the library's.
LEAK_SUPPRESSIONS = "leak:libhsa-runtime64.so\nleak:libamdhip64.so\n"


def run_harness(exe: str, gpu: bool, timeout: int = 600) -> subprocess.CompletedProcess:
    supp = os.path.join(os.path.dirname(exe), "lsan.supp")
    with open(supp, "w") as f:
        f.write(LEAK_SUPPRESSIONS)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={supp}:print_suppressions=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([exe] + (["--gpu"] if gpu else []), capture_output=True, text=True, env=env,
                          timeout=timeout)


@pytest.mark.skipif(not os.path.exists(os.path.join(rocm(), "llvm", "bin", "clang++")) or shutil.which("gcc") is None,
                    reason="needs the ROCm toolchain")
def test_host_code_under_asan_and_ubsan():
    stamp = sources_stamp()
    stamp_file = os.path.join(PREBUILT_DIR, "sources.sha256")
    if os.path.exists(stamp_file):
        os.remove(stamp_file)
    exe = build_harness(PREBUILT_DIR)
    with open(stamp_file, "w") as f:
        f.write(stamp + "\n")
    check_run(run_harness(exe, gpu=False), gpu=False)


def check_run(r, gpu):
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "host checks done" in r.stdout and "0 failed checks" in r.stdout, out[-6000:]
    if gpu:
        assert "device checks done" in r.stdout, out[-6000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]


@pytest.mark.gpu
def test_host_code_under_asan_and_ubsan_on_the_device():
    exe = os.path.join(PREBUILT_DIR, "host_sanitize")
    stamp_file = os.path.join(PREBUILT_DIR, "sources.sha256")
    if not (os.path.exists(exe) and os.path.exists(stamp_file)):
        pytest.skip("the sanitized build is made by the CPU test of this file; run it first")
    with open(stamp_file) as f:
        if f.read().strip() != sources_stamp():
            pytest.skip("the sanitized build predates the current sources; run the CPU test of this file")
    print("host_sanitize --gpu: every device entry point under host ASan and UBSan", flush=True)
    check_run(run_harness(exe, gpu=True, timeout=300), gpu=True)
