"""The C ABI header compiles on its own, as C and as C++ (it is what a
caller includes; declarations in it are checked against the library's
exports in test_lib_abi.py)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("lang,compiler", [("c", "gcc"), ("c++", "g++")])
def test_header_compiles(lang, compiler):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    r = subprocess.run([compiler, "-fsyntax-only", "-Wall", "-x", lang, os.path.join(ROOT, "include", "eipc.h")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
