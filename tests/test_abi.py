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


def _c_layout(tmp_path, fields):
    """sizeof / offsetof of header structs as the C compiler lays them out."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hipscc.h"', "int main(void) {"]
    for struct, members in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (struct, struct))
        for f in members:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (struct, f, struct, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    return {k: int(v) for k, v in (ln.split() for ln in out if ln)}


def test_struct_layouts_match_header(tmp_path):
    # the Python mirrors must have the sizes and offsets the C compiler gives
    from paper_2303_04934_amd import _native
    mirrors = {"scc_graph_t": _native.Graph, "scc_options_t": _native.Options, "scc_stats_t": _native.Stats}
    fields = {k: [f for f, _ in v._fields_] for k, v in mirrors.items()}
    c = _c_layout(tmp_path, fields)
    for struct, py in mirrors.items():
        assert ctypes.sizeof(py) == c[struct], struct
        for f in fields[struct]:
            assert getattr(py, f).offset == c["%s.%s" % (struct, f)], (struct, f)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_options_and_argument_errors_without_gpu():
    from paper_2303_04934_amd import _native
    lib = _native.load()
    o = _native.Options()
    assert lib.scc_default_options(ctypes.byref(o)) == 0
    assert (o.tau, o.lambda_log2, o.sigma) == (2048, 0, 50)
    assert abs(o.beta - 2.0) < 1e-6
    assert abs(o.beta_fast - 4.0) < 1e-6 and abs(o.table_floor - 1.2) < 1e-6
    assert o.tau_single == 0 and o.union_streams == 0
    assert lib.scc_default_options(None) == _native.SCC_EINVAL
    # a NULL context is rejected before any device work
    assert lib.scc_labels(None, None, None, None, None) == _native.SCC_EINVAL
    assert lib.scc_last_error(None) == b"null context"
