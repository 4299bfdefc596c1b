"""End-to-end parity of the HIP implementation of Algorithm 3 with the FP64
oracle, exactness invariants, and the serial fine reference.

Tolerances (energy norm of the Sec. 6 error measure, per slice):
* FP64 state, svd_tol >= 1e-6: max(1e-12, 256 A eps), with A the
  amplification of a relative input perturbation through the iteration,
  measured on the oracle (about 400 on wave1d: the gate is 2.2e-11
  there).  At the paper's tol (1e-14) the
  phase corrector keeps directions with sigma_i / sigma_1 down to 1e-14,
  in which Omega is only determined to about eps * sigma_1 / sigma_i; two
  orderings of the same exact arithmetic already differ by ~1e-11 there
  (measured with the oracle against an algebraically equivalent sweep), so
  the gate is 1e-9.
* FP32 compensated state: 1e-5 against the oracle run on the same
  FP32-rounded initial data.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import (derived_gate, inputs_as, problem_pair,
                               rel_energy_err, to_np)

pytestmark = pytest.mark.gpu


def _run(w, K, tol=None, dtype=None, compensated=None):
    import paper_1905_00473_amd as pw
    dt = dtype or w.dtype
    P, Q = problem_pair(w, max_iters=max(K, 1), tol=tol, dtype=dt,
                        compensated=compensated)
    s = pw.Solver(P)
    u0, p0 = inputs_as(w, dt)
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    s.run(K)
    return s, Q, u0, p0


def _compare(s, Q, w, u0, p0, K, gate):
    ref = O.theta_parareal(Q, w.c, u0, p0, K)
    gate = derived_gate(Q, w, u0, p0, K, gate)
    worst = 0.0
    for n in range(Q.N + 1):
        u, p = s.state(n)
        if n == 0:
            assert np.array_equal(to_np(u), u0)
            continue
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        worst = max(worst, e)
    assert worst < gate, (worst, gate)
    rho, rk = s.residuals()
    assert rk == ref.rank, (rk, ref.rank)
    np.testing.assert_allclose(rho, ref.rho, rtol=1e-6)
    return worst


@pytest.mark.parametrize("tol,gate", [(1e-3, 1e-12), (1e-6, 1e-12),
                                      (1e-14, 1e-9)])
def test_wave1d_fp64_parity(tol, gate):
    w = W.wave1d()
    s, Q, u0, p0 = _run(w, w.K, tol=tol)
    _compare(s, Q, w, u0, p0, w.K, gate)


@pytest.mark.parametrize("N,K", [(100, 3), (200, 2)])
def test_many_slices_fp64_parity(N, K):
    """More than 64 slices: the orthonormalisation inside Algorithm 1 runs
    in column blocks of 64 made orthogonal by block Gram-Schmidt."""
    w = W.wave1d(n=512, N=N, K=K)
    s, Q, u0, p0 = _run(w, K, tol=1e-6)
    _compare(s, Q, w, u0, p0, K, 1e-12)
    s.close()


def test_layers3d_small_spectral_fp64():
    """Algorithm 3 with the Fourier gradient in 3D (non-power-of-two coarse
    axes: the direct DFT passes)."""
    w = W.layers3d(n=48, ratio=4, N=4, K=2, T=0.1, dtype="f64",
                   compensated=False)
    w.grad_order = "spectral"
    s, Q, u0, p0 = _run(w, 2, tol=1e-6)
    _compare(s, Q, w, u0, p0, 2, 1e-12)
    s.close()


@pytest.mark.parametrize("order", [8, "spectral"])
def test_disc2d_small_fp64_gradient_orders(order):
    """Algorithm 3 with the 8th-order and the Fourier gradient (Sec. 6.4):
    Lambda, its transpose in the sweep coordinates and the corrector."""
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5, dtype="f64",
                 compensated=False)
    w.grad_order = order
    s, Q, u0, p0 = _run(w, 3, tol=1e-6)
    _compare(s, Q, w, u0, p0, 3, 1e-12)
    s.close()


def test_many_slices_fp32():
    """100 slices with the FP32 compensated state (Cholesky QR for the
    data blocks, blocked beyond 64 columns)."""
    w = W.wave1d(n=512, N=100, K=2)
    s, Q, u0, p0 = _run(w, 2, tol=1e-6, dtype="f32", compensated=True)
    ref = O.theta_parareal(Q, w.c, u0, p0, 2)
    for n in range(1, Q.N + 1, 7):
        u, p = s.state(n)
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        assert e < 1e-5, (n, e)
    s.close()


def test_more_slices_than_rows():
    """The Sec. 6 setup at T = 15: 300 slices, 2 x 100 data rows, so the
    data matrices are wide (the QR inside Algorithm 1 factors only as many
    columns as there are rows)."""
    import paper_1905_00473_amd as pw
    n, T, N, K = 100, 15.0, 300, 2
    x = -0.5 + np.arange(n) / n
    u0 = np.cos(10 * np.pi * x) * np.exp(-100 * x ** 2)
    p0 = np.zeros(n)
    c = np.ones(n)
    P = pw.Problem.make((n,), 1, T, N, 200, 10, 2, 1e-14, "f64", False, K)
    Q = O.Problem((n,), 1, T, N, 200, 10, 2, 1e-14)
    s = pw.Solver(P)
    s.set_medium(c)
    s.set_initial(u0, p0)
    s.run(K)
    ref = O.theta_parareal(Q, c, u0, p0, K)
    worst = max(rel_energy_err(to_np(s.state(k)[0]), to_np(s.state(k)[1]),
                               ref.u[k], ref.p[k], c, Q.dx_fine, 2)
                for k in range(1, N + 1))
    assert worst < 1e-9, worst
    _, rk = s.residuals()
    assert list(rk) == list(ref.rank)
    s.close()


def test_disc2d_small_fp64_parity():
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5, dtype="f64",
                 compensated=False)
    s, Q, u0, p0 = _run(w, 3, tol=1e-6)
    _compare(s, Q, w, u0, p0, 3, 1e-12)


def test_disc2d_small_fp32_parity():
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5)
    s, Q, u0, p0 = _run(w, 3, tol=1e-6)
    ref = O.theta_parareal(Q, w.c, u0, p0, 3)
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        assert e < 1e-5, (n, e)


def test_layers3d_small_fp32_parity():
    w = W.layers3d(n=32, ratio=4, N=4, K=2, T=0.2)
    s, Q, u0, p0 = _run(w, 2, tol=1e-6)
    ref = O.theta_parareal(Q, w.c, u0, p0, 2)
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        assert e < 1e-5, (n, e)


def test_serial_fine_parity_and_exactness():
    """Slices 0..k are bit-for-bit the GPU serial fine solution after k
    iterations; with K = N every slice is."""
    import torch
    w = W.wave1d()
    for K in (1, 3, w.N):
        s, Q, u0, p0 = _run(w, K)
        for n in range(0, w.N + 1):
            uf, pf = s.serial_fine(n)
            u, p = s.state(n)
            if n <= K:
                assert torch.equal(u, uf) and torch.equal(p, pf), (K, n)
    # the GPU serial fine solution itself against the oracle
    us, ps = O.serial_fine(Q, w.c, u0, p0)
    uf, pf = s.serial_fine(w.N)
    assert rel_energy_err(to_np(uf), to_np(pf), us[-1], ps[-1], w.c,
                          Q.dx_fine) < 1e-12


def test_zero_iterations_is_coarse_solution():
    w = W.wave1d()
    s, Q, u0, p0 = _run(w, 0)
    cc = O.restrict(w.c, w.ratio)
    U, P = O.restrict(u0, w.ratio), O.restrict(p0, w.ratio)
    for n in range(1, w.N + 1):
        U, P = O.propagate(U, P, cc * cc, Q.dt_coarse, Q.dx_coarse, Q.m_coarse)
        u, p = s.state(n)
        np.testing.assert_allclose(to_np(u), O.interp(U, w.ratio), atol=1e-12)


def test_unstable_medium_rejected():
    import paper_1905_00473_amd as pw
    w = W.wave1d()
    P, _ = problem_pair(w)
    s = pw.Solver(P)
    with pytest.raises(pw.PwError) as e:
        s.set_medium(w.c * 10)
    assert e.value.status == -2
