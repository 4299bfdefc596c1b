"""The lower-order interpolations I on the GPU (pw_problem.interp =
PW_INTERP_LINEAR, PW_INTERP_CUBIC) against the FP64 oracle: the
interpolation itself and whole runs of Algorithm 3.

Gates: interpolation 1e-13 relative (FP64); Algorithm 3, FP64 state, svd
tol 1e-6: the derived gate max(1e-12, 256 A eps, 16 S) of the other
parity tests (tests/gpu_helpers.py); FP32 compensated: 1e-5.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import (derived_gate, inputs_as, problem_pair,
                               rel_energy_err, to_np)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["linear", "cubic"])
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_interp_add_parity(dim, kind):
    import paper_1905_00473_amd as pw
    import torch
    w = {1: lambda: W.wave1d(), 2: lambda: W.disc2d(n=72, N=4, K=2, T=0.25),
         3: lambda: W.layers3d(n=40, N=4, K=2, T=0.06)}[dim]()
    P, Q = problem_pair(w, max_iters=1, dtype="f64", interp=kind)
    s = pw.Solver(P)
    rng = np.random.default_rng(5)
    du = torch.tensor(rng.standard_normal((3,) + w.coarse_shape), device="cuda")
    dp = torch.tensor(rng.standard_normal((3,) + w.coarse_shape), device="cuda")
    v = torch.tensor(rng.standard_normal((3,) + w.shape), device="cuda")
    uo, po = s.interp_add(du, dp, v, v)
    for k in range(3):
        ref = to_np(v[k]) + O.interp(to_np(du[k]), w.ratio, kind)
        np.testing.assert_allclose(to_np(uo[k]), ref, rtol=1e-13,
                                   atol=1e-13 * np.abs(ref).max())
    s.close()


def _run(w, K, dtype, tol=1e-6, kind="linear"):
    import paper_1905_00473_amd as pw
    P, Q = problem_pair(w, max_iters=max(K, 1), tol=tol, dtype=dtype,
                        interp=kind)
    s = pw.Solver(P)
    u0, p0 = inputs_as(w, dtype)
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    s.run(K)
    return s, Q, u0, p0


@pytest.mark.parametrize("kind", ["linear", "cubic"])
@pytest.mark.parametrize("case", ["wave1d", "disc2d"])
def test_algorithm3_fp64(case, kind):
    w = (W.wave1d() if case == "wave1d" else
         W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5, dtype="f64",
                  compensated=False))
    K = 4 if case == "wave1d" else 3
    s, Q, u0, p0 = _run(w, K, "f64", kind=kind)
    ref = O.theta_parareal(Q, w.c, u0, p0, K)
    gate = derived_gate(Q, w, u0, p0, K)
    worst = max(rel_energy_err(to_np(s.state(n)[0]), to_np(s.state(n)[1]),
                               ref.u[n], ref.p[n], w.c, Q.dx_fine)
                for n in range(1, Q.N + 1))
    assert worst < gate, (worst, gate)
    rho, rk = s.residuals()
    assert list(rk) == list(ref.rank)
    np.testing.assert_allclose(rho, ref.rho, rtol=1e-6)
    s.close()


@pytest.mark.parametrize("kind", ["linear", "cubic"])
def test_algorithm3_fp32(kind):
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5)
    s, Q, u0, p0 = _run(w, 3, "f32", kind=kind)
    ref = O.theta_parareal(Q, w.c, u0, p0, 3)
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        assert e < 1e-5, (n, e)
    s.close()


def test_linear_rejected_by_taped_runs():
    import paper_1905_00473_amd as pw
    s, _, _, _ = _run(W.wave1d(), 1, "f64")
    with pytest.raises(pw.PwError, match="trigonometric"):
        s.run_taped(1)
    s.close()
