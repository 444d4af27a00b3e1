"""The C ABI library loads on the CPU and exports every symbol that
include/hdarray.h declares (no compute calls: there may be no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1809_05657_amd as hd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_loads_and_exports_header_symbols():
    if not os.path.exists(hd.LIB_PATH):
        pytest.skip("libhdarray.so not built")
    lib = ctypes.CDLL(hd.LIB_PATH)
    names = hd.exported_symbols()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", hd.LIB_PATH], capture_output=True, text=True).stdout
    defined = set(re.findall(r" T (hdarray_\w+)", out))
    assert set(names) <= defined
    # the binding declares a signature for every exported function
    hd.load()


def test_header_is_plain_c():
    """No torch or HIP types in the ABI: the header compiles as C99 alone."""
    hdr = os.path.join(ROOT, "include", "hdarray.h")
    r = subprocess.run(["gcc", "-std=c99", "-fsyntax-only", "-x", "c", hdr], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    txt = open(hdr).read()
    assert "torch" not in txt and "hip_runtime" not in txt


def test_product_does_not_reference_oracle():
    """The product path never loads the oracle and has no CPU fallback."""
    pkg = os.path.join(ROOT, "paper_1809_05657_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f
