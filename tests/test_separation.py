"""The oracle and the HIP path are independent, and the product path has no
CPU fallback: no oracle source names the library, its sources or its header;
no library source (Python, HIP, C++ or header) imports or includes the
oracle; the seeded input generators import neither side; the binding fails
loudly when the HIP library is missing instead of computing anything else."""
import ast
import os
import re

import pytest

from paper_2306_03651_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2306_03651_amd")
SOURCE_EXT = (".py", ".c", ".h", ".hpp", ".hip", ".cpp")


def sources(top):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(SOURCE_EXT):
                yield os.path.join(d, f)


def python_imports(path):
    tree = ast.parse(open(path).read(), path)
    names = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            names.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            if node.level == 0 and node.module:
                names.add(node.module.split(".")[0])
            else:   # relative: the modules named
                names.update("." + a.name for a in node.names)
    return names


def c_includes(path):
    return re.findall(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', open(path).read(), re.M)


def test_oracle_names_nothing_of_the_library():
    for path in sources(os.path.join(ROOT, "oracle")):
        text = open(path).read()
        for word in ("paper_2306_03651_amd", "centra.h", "csrc", "libcentra", "hip_runtime"):
            assert word not in text, f"{os.path.relpath(path, ROOT)} names {word}"
        if path.endswith(".py"):
            assert "paper_2306_03651_amd" not in python_imports(path)
        else:
            assert all("centra.h" not in inc and "csrc" not in inc for inc in c_includes(path))


def test_library_does_not_use_the_oracle():
    for top in (PKG, os.path.join(ROOT, "include")):
        for path in sources(top):
            rel = os.path.relpath(path, ROOT)
            if path.endswith(".py"):
                assert "oracle" not in python_imports(path), f"{rel} imports the oracle"
                assert "liboracle" not in open(path).read(), f"{rel} loads the oracle's library"
            else:
                incs = c_includes(path)
                assert not any("oracle" in inc for inc in incs), f"{rel} includes the oracle"
                assert "orc_" not in open(path).read(), f"{rel} names an oracle function"


def test_input_generators_import_neither_side():
    for path in sources(os.path.join(PKG, "inputs")):
        if path.endswith(".py"):
            imps = python_imports(path)
            assert not imps & {"oracle", "paper_2306_03651_amd", ".binding"}, (path, imps)
        else:
            assert not any("oracle" in i or "centra" in i for i in c_includes(path)), path


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "libcentra.so"))
    with pytest.raises(ImportError, match="missing"):
        binding.lib()
    with pytest.raises(ImportError):
        binding.centra_abi_version()
