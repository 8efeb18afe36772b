"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/centra.h declares, the Python binding mirrors the header, and the
host-only bound (centra_bound) agrees with the oracle to 1e-12."""
import math
import os
import re

import pytest

import oracle
from paper_2306_03651_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "centra.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"CENTRA_API\s+[\w\s\*]*?\b(centra_\w+)\s*\(", text)))


def test_header_declares_the_four_hot_path_calls():
    names = declared_functions()
    for f in ["centra_sample_paths", "centra_greedy_cover", "centra_mcera", "centra_progressive"]:
        assert f in names
    assert len(names) >= 17


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_mirrors_header():
    assert sorted(binding.SIGNATURES) == declared_functions()


def test_abi_version():
    assert binding.centra_abi_version() == 11


CASES = [
    (10000, 4826, 2187, 10, 5568, 4, 0.05, 0.05),
    (4000000, 1900000, 812345, 64, 9000000, 9, 0.01, 0.1 / 2**7),
    (100, 3, 0, 1, 3, 1, 0.3, 0.5),
    (2**40, 2**39, 2**35, 1000, 2**38, 30, 0.001, 1e-9),
    (1000, 0, 0, 5, 0, 0, 0.1, 0.01),
]


@pytest.mark.parametrize("case", CASES)
def test_host_bound_matches_oracle(case):
    got = binding.centra_bound(*case)
    want = oracle.bound(*case)
    for f in ["c_hat", "amcera", "wimpy", "xi", "nu", "rtilde", "r", "eta"]:
        a, b = getattr(got, f), getattr(want, f)
        assert a == pytest.approx(b, rel=1e-12, abs=1e-300), f
    assert got.certified == want.certified


def test_host_bound_rejects_bad_arguments():
    with pytest.raises(binding.CentraError):
        binding.centra_bound(0, 0, 0, 1, 0, 0, 0.1, 0.1)
    with pytest.raises(binding.CentraError):
        binding.centra_bound(10, 0, 0, 0, 0, 0, 0.1, 0.1)
    with pytest.raises(binding.CentraError):
        binding.centra_bound(10, 0, 0, 1, 0, 0, 0.1, 1.0)


@pytest.mark.parametrize("b", [1, 2, 3, 5, 8, 1000, 2 ** 40 + 1, 2 ** 63, 2 ** 64 - 1])
@pytest.mark.parametrize("k", [1, 2, 50, 500])
def test_vc_dims_match_oracle(b, k):
    for n in [2, 1000, 10 ** 6, 2 ** 22]:
        got = binding.centra_vc_dims(b, k, n)
        d1, dl, du = oracle.vc_dims(b, k, n)
        assert (got.d1, got.dk_lemma, got.dk_union) == (d1, dl, du)
        assert got.dk == min(dl, du)


def test_vc_dims_rejects_zeros():
    for args in [(0, 1, 1), (1, 0, 1), (1, 1, 0)]:
        with pytest.raises(binding.CentraError):
            binding.centra_vc_dims(*args)


@pytest.mark.parametrize("m,cov,n,k,eps,delta_i", [(50000, 20000, 1000, 1, 0.1, 0.05), (10**6, 512000, 10**6, 50, 0.01, 0.1 / 8),
                                                  (100, 0, 2, 2, 0.3, 0.5), (2**30, 2**29, 2**30, 500, 0.05, 1e-9)])
def test_hedge_bound_matches_oracle(m, cov, n, k, eps, delta_i):
    got = binding.centra_hedge_bound(m, cov, n, k, eps, delta_i)
    want = oracle.hedge_bound(m, cov, n, k, eps, delta_i)
    assert got.eta == pytest.approx(want.eta, rel=1e-12) and got.c_hat == want.c_hat
    assert got.certified == want.certified and got.amcera == 0.0


STRUCTS = {"centra_csr": "Csr", "centra_extend_args": "ExtendArgs", "centra_sampler_stats": "SamplerStats",
           "centra_bound_out": "BoundOut", "centra_vc_out": "VcOut", "centra_params": "Params",
           "centra_result": "Result", "centra_iteration": "Iteration", "centra_pool_params": "PoolParams",
           "centra_query_info": "QueryInfo", "centra_engine_stats": "EngineStats", "centra_checkpoint": "Checkpoint"}


def test_binding_structs_match_header_layout(tmp_path):
    # the C compiler's sizeof / offsetof of every struct of the header
    # against the ctypes mirrors (same field names, same offsets)
    import ctypes
    import subprocess
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "centra.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(binding, pyname)
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for cname, pyname in STRUCTS.items():
        cls = getattr(binding, pyname)
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, f"{cname}.{f}"
    # every struct the header defines is mirrored
    text = open(HEADER).read()
    assert sorted(re.findall(r"}\s*(centra_\w+);", text)) == sorted(STRUCTS)


def test_params_hash_is_fnv1a_of_the_fields():
    # FNV-1a 64 over each field's little-endian bytes, in declaration order
    import struct
    p = binding.Params(50, 64, 0.01, 0.1, 12345678901, 7, 100000, 4000000, 2, 1, 1, 3, 0, 1)
    data = struct.pack("<IIddQIQQIIIIII", p.k, p.t, p.eps, p.delta, p.seed, p.instance, p.m_init, p.m_max,
                       p.growth_num, p.growth_den, p.schedule, p.space, p.kappa, p.method)
    h = 0xCBF29CE484222325
    for b in data:
        h = ((h ^ b) * 0x100000001B3) & ((1 << 64) - 1)
    assert binding.centra_params_hash(p) == h
    q = binding.Params(50, 64, 0.01, 0.1, 12345678901, 7, 100000, 4000000, 2, 1, 1, 3, 0, 0)
    assert binding.centra_params_hash(q) != h
