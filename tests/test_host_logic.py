"""Host-side logic of the HIP library, checked on the CPU: the vertex
permutation of Algorithm 1 (a keyed Feistel network with cycle walking) is a
bijection of [0, n) and its inverse, used to pick a long batch's sources by a
scan over the vertices, undoes it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_permutation_bijection_and_inverse(tmp_path):
    exe = tmp_path / "perm_check"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2303_04934_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "perm_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert out.strip() == "ok"
