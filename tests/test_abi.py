"""The C-ABI library loads on the CPU host and exports every entry point
that include/pw.h declares (no compute call: no GPU here)."""

import ctypes
import os
import re

import paper_1905_00473_amd as pw

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include",
                      "pw.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == pw.SYMBOLS


def test_library_exports_every_symbol():
    L = ctypes.CDLL(pw.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_version_and_error_string():
    L = pw.lib()
    assert b"gfx950" in L.pw_version()
    assert isinstance(L.pw_last_error(), bytes)


def test_problem_struct_layout():
    # int dim, int n[3], int ratio, double T, int N, mF, mC, order,
    # double tol, int dtype, comp, max_iters
    assert ctypes.sizeof(pw.Problem) == 72
    assert pw.Problem.T.offset == 24
    assert pw.Problem.svd_tol.offset == 48
