"""The C-ABI library loads and exports every function include/celmi.h declares (no GPU
needed: nothing is called)."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "celmi.h")).read()
    return sorted(set(re.findall(r"^\s*(?:cel_status|void|const char\*)\s+(cel_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    lib = os.path.join(ROOT, "paper_1803_00113_amd", "libcelmi.so")
    if not os.path.exists(lib):
        from paper_1803_00113_amd import build
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (cel_\w+)$", out, re.M))
    declared = _declared()
    assert len(declared) >= 10
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    from paper_1803_00113_amd import _ffi
    assert set(_ffi.EXPORTED) == set(declared)
