"""CPU-side checks of the HIP library: it builds for gfx950, loads, exports every
entry point declared in include/mpcg.h, and its ctypes structs have the C
layout (checked against the header with the host compiler).  No GPU calls."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpcg.h")
LIB = os.path.join(ROOT, "paper_2412_08059_amd", "libmpcg.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:mpcg_status|const char \*)\s*(mpcg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__._hip_build_module().build()
    return LIB


def test_library_exports_every_declared_symbol(built):
    lib = ctypes.CDLL(built)
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    from paper_2412_08059_amd import capi
    assert sorted(capi.EXPORTED) == names


def test_strerror_without_gpu(built):
    from paper_2412_08059_amd import capi
    assert capi.mpcg_strerror(0) == "ok"
    assert "CSR" in capi.mpcg_strerror(capi.MPCG_EINVAL)
    assert capi.mpcg_strerror(12345) == "unknown status"


def test_struct_layout_matches_header(tmp_path, built):
    from paper_2412_08059_amd import capi
    src = tmp_path / "layout.c"
    src.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu\\n", sizeof(mpcg_csr), sizeof(mpcg_features_t), sizeof(mpcg_stats), sizeof(mpcg_options));
  printf("%zu %zu %zu %zu\\n", offsetof(mpcg_csr, col_idx), offsetof(mpcg_stats, feat),
         offsetof(mpcg_stats, t_total_ms), offsetof(mpcg_options, maxit2));
  printf("%zu %zu %zu\\n", sizeof(mpcg_request), offsetof(mpcg_request, eps1), offsetof(mpcg_request, user));
  printf("%zu %zu\\n", sizeof(mpcg_diam_t), offsetof(mpcg_diam_t, best_start));
  return 0;
}}""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split()
    got = [int(v) for v in out]
    exp = [ctypes.sizeof(capi.mpcg_csr), ctypes.sizeof(capi.mpcg_features_t),
           ctypes.sizeof(capi.mpcg_stats), ctypes.sizeof(capi.mpcg_options),
           capi.mpcg_csr.col_idx.offset, capi.mpcg_stats.feat.offset,
           capi.mpcg_stats.t_total_ms.offset, capi.mpcg_options.maxit2.offset,
           ctypes.sizeof(capi.mpcg_request), capi.mpcg_request.eps1.offset, capi.mpcg_request.user.offset,
           ctypes.sizeof(capi.mpcg_diam_t), capi.mpcg_diam_t.best_start.offset]
    assert got == exp


def test_product_package_does_not_reach_the_oracle():
    pkg = os.path.join(ROOT, "paper_2412_08059_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "mpcg_oracle" not in text, f
