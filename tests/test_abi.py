"""The C-ABI library loads and exports every function include/hipscc.h declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hipscc.h")
LIB = os.path.join(ROOT, "paper_2303_04934_amd", "libhipscc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("scc_create", "scc_destroy", "scc_labels", "scc_reach", "scc_labels_batched",
                 "scc_policy_load", "scc_bag_selftest", "scc_last_error"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_2303_04934_amd import _native
    assert sorted(_native.EXPORTS) == declared_functions()
    lib.scc_version.restype = ctypes.c_char_p
    assert lib.scc_version().startswith(b"hipscc")


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_struct_layouts_match_header():
    # the Python mirrors must have the sizes the C compiler gives the structs
    from paper_2303_04934_amd import _native
    assert ctypes.sizeof(_native.Graph) == 8 + 4 * 8
    assert ctypes.sizeof(_native.Options) == 4 * 6 + 8 + 4 * 4 + 8 + 4 + 4 + 4 + 4 * 5
    assert ctypes.sizeof(_native.Stats) == 6 * 8 + 18 * 8 + 3 * 8 * 3 + 3 * 8


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_options_and_argument_errors_without_gpu():
    from paper_2303_04934_amd import _native
    lib = _native.load()
    o = _native.Options()
    assert lib.scc_default_options(ctypes.byref(o)) == 0
    assert (o.tau, o.lambda_log2, o.sigma) == (512, 10, 50)
    assert abs(o.beta - 1.5) < 1e-6
    assert lib.scc_default_options(None) == _native.SCC_EINVAL
    # a NULL context is rejected before any device work
    assert lib.scc_labels(None, None, None, None, None) == _native.SCC_EINVAL
    assert lib.scc_last_error(None) == b"null context"
