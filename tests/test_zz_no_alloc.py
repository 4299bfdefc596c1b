"""pw_energy_noalloc, the allocation-free form of pw_energy: the same
energy and l2 sums with the reduction's partial sums in the library's fixed
device scratch instead of a context buffer.  Checked through the C ABI
against pw_energy on two calls in a row, the second on a smaller grid (and
the other state dtype), and against the oracle; the size limit is checked
on the host without a GPU."""

import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W


def _fn():
    import paper_1905_00473_amd as pw
    return pw.lib().pw_energy_noalloc


def test_rejects_grid_beyond_limit_on_host():
    """2^31 points or more: PW_EINVAL before any device call (runs without
    a GPU)."""
    import paper_1905_00473_amd as pw
    P = pw.Problem.make((2048, 1024, 1024), 4, 1.0, 4, 8, 2)
    st = _fn()(ctypes.byref(P), None, None, None, None, None, None, None)
    assert st == -1
    assert b"2^31" in pw.lib().pw_last_error()
    bad = pw.Problem.make((40, 40), 4, 1.0, 4, 8, 2)
    bad.grad_order = 3
    assert _fn()(ctypes.byref(bad), None, None, None, None, None, None,
                 None) == -1


@pytest.mark.gpu
def test_matches_pw_energy_two_calls_second_smaller():
    import torch

    import paper_1905_00473_amd as pw
    from tests.gpu_helpers import problem_pair
    cases = [(W.disc2d(n=96, ratio=4, N=4, K=1, T=0.25, dtype="f64",
                       compensated=False), "f64", 6),
             (W.disc2d(n=40, ratio=4, N=4, K=1, T=0.25, dtype="f32",
                       compensated=False), "f32", 4)]
    rng = np.random.default_rng(11)
    f = _fn()
    for w, dtype, order in cases:            # the second grid is smaller
        w.grad_order = order
        P, Q = problem_pair(w, dtype=dtype, compensated=False)
        s = pw.Solver(P)
        s.set_medium(w.c)
        td = torch.float64 if dtype == "f64" else torch.float32
        arrs = [rng.standard_normal(w.shape) for _ in range(4)]
        if dtype == "f32":
            arrs = [a.astype(np.float32).astype(np.float64) for a in arrs]
        dev = [torch.tensor(a, dtype=td, device="cuda") for a in arrs]
        c = torch.tensor(w.c, dtype=torch.float64, device="cuda")
        out = torch.full((4,), float("nan"), dtype=torch.float64,
                         device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        st = f(ctypes.byref(P), c.data_ptr(), *[d.data_ptr() for d in dev],
               out.data_ptr(), stream)
        assert st == 0, pw.lib().pw_last_error()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = s.error_norms(*dev)
        want = np.array([ref["E_diff"], ref["E_ref"], ref["l2_diff2"],
                         ref["l2_ref2"]])
        # the same kernels in the same order: the same bits
        assert np.array_equal(got, want), (got, want)
        u, p, ur, pr = arrs
        e = O.energy(u - ur, p - pr, w.c, Q.dx_fine, order)
        assert abs(got[0] - e) <= 1e-12 * e
        # without a reference: energy and sum of squares of [u, p]
        out.fill_(float("nan"))
        st = f(ctypes.byref(P), c.data_ptr(), dev[0].data_ptr(),
               dev[1].data_ptr(), None, None, out.data_ptr(), stream)
        assert st == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        e1, _ = s.energy(dev[0], dev[1])
        assert got[0] == e1 and got[1] == 0.0
        s.close()
