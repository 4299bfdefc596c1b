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
    """The ctypes mirror of pw_problem has the size and field offsets that
    a C compiler gives the header's struct."""
    import shutil
    import subprocess
    import tempfile
    names = [n for n, _ in pw.Problem._fields_]
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = "#include <stddef.h>\n#include <stdio.h>\n#include \"pw.h\"\n" \
          "int main(void) { printf(\"%zu\", sizeof(pw_problem));" + "".join(
              f' printf(" %zu", offsetof(pw_problem, {n}));' for n in names) + \
          " return 0; }\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", os.path.dirname(HEADER), c, "-o", exe],
                       check=True)
        got = [int(x) for x in subprocess.run([exe], check=True,
                                              capture_output=True,
                                              text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(pw.Problem)
    assert got[1:] == [getattr(pw.Problem, n).offset for n in names]


def _create(P):
    h = ctypes.c_void_p()
    arr = (pw.Problem * 1)(P)
    st = pw.lib().pw_create(arr, 1, None, ctypes.byref(h))
    return st, pw.lib().pw_last_error().decode()


def test_invalid_problems_rejected_before_any_device_work():
    """Argument validation of pw_create runs on the host before any device
    allocation (these calls make no GPU call)."""
    good = dict(shape=(40, 40), ratio=4, T=0.25, N=4, m_fine=8, m_coarse=2)
    cases = []

    def mk(**kw):
        a = dict(good)
        a.update(kw)
        return pw.Problem.make(a["shape"], a["ratio"], a["T"], a["N"],
                               a["m_fine"], a["m_coarse"],
                               a.get("order", 4), a.get("tol", 1e-10),
                               a.get("dtype", "f64"), a.get("comp", False),
                               a.get("max_iters", 2))
    cases.append((mk(ratio=3), "ratio must divide"))
    cases.append((mk(shape=(16, 16)), "at least 5 points"))
    cases.append((mk(T=0.0), "T must be positive"))
    cases.append((mk(N=0), "slice/step"))
    cases.append((mk(order=3), "grad_order"))
    cases.append((mk(order=10), "grad_order"))
    bad_interp = mk()
    bad_interp.interp = 3
    cases.append((bad_interp, "interp"))
    cases.append((mk(tol=0.0), "svd_tol"))
    cases.append((mk(comp=True), "compensation"))
    cases.append((mk(max_iters=0), "max_iters"))
    bad_dim = mk()
    bad_dim.dim = 4
    cases.append((bad_dim, "dim must be"))
    bad_axis = mk()
    bad_axis.n_fine[2] = 3
    cases.append((bad_axis, "unused axes"))
    # the absorbing layer: 2D only, width in (0, 0.5), reflection in [0, 1)
    bad_bc = mk()
    bad_bc.bc = 2
    cases.append((bad_bc, "bc must be"))
    sp1d = pw.Problem.make((64,), 4, 0.25, 4, 8, 2, sponge_width=0.1)
    cases.append((sp1d, "2D problems only"))
    wide = mk()
    wide.bc, wide.sponge_width = pw.SPONGE, 0.5
    cases.append((wide, "sponge_width"))
    refl = mk()
    refl.bc, refl.sponge_width, refl.sponge_reflection = pw.SPONGE, 0.1, 1.0
    cases.append((refl, "sponge_reflection"))
    cmax = mk()
    cmax.bc, cmax.sponge_width, cmax.sponge_cmax = pw.SPONGE, 0.1, -1.0
    cases.append((cmax, "sponge_cmax"))
    for P, msg in cases:
        st, err = _create(P)
        assert st == -1, (msg, st, err)
        assert msg in err, (msg, err)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asked for more it says so and exits 2."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_argument_checks_run_before_any_device_work():
    """The binding's tensor checks (dtype, device, shape, contiguity) reject
    a mismatched tensor with ValueError; a CPU tensor is refused here, on a
    host without a GPU, before any library call."""
    import pytest
    import torch
    t = torch.zeros((2, 3), dtype=torch.float64)
    with pytest.raises(ValueError, match="device"):
        pw.require(t, torch.float64, (2, 3), "u")
    with pytest.raises(ValueError, match="torch tensor"):
        pw.require([1.0], torch.float64, (1,), "u")


def test_keep_history_flag_validated():
    P = pw.Problem.make((40, 40), 4, 0.25, 4, 8, 2)
    P.keep_history = 2
    st, msg = _create(P)
    assert st == -1 and "keep_history" in msg
