"""The comparator iterations of Sec. 6 on the GPU against the FP64 oracle:
Omega = I (Sec. 6.2), the phase-corrected coarse propagation without the
parareal-style correction (Sec. 6.3) and plain parareal (eq.
plainparareal), each run through the same C-ABI entry point as Algorithm 3
after pw_set_variant.

Gates: FP64 state, svd tol 1e-6: max(1e-12, 256 A eps) in the energy norm
per slice, eps = 2^-52, where A is the amplification of a relative input
perturbation through the same iteration, measured on the oracle (u0
perturbed by 1e-13 relative noise).  Omega = I and plain parareal are
unstable for waves (the growth Sec. 6 reports), so rounding differences
between two correct orderings grow with A (up to ~1e4 on wave1d); 256
covers the rounding injected at every stage rather than at the input
only.  For Algorithm 3 (no correction) the gate is also at least 16
times the spread between two oracle runs that pass Algorithm 1 its data
columns in opposite orders.  FP32 compensated state: 1e-5 against the oracle on the same
FP32-rounded initial data.  Residuals to rtol 1e-6 and equal ranks (the
row count for Omega = I and plain).
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import (derived_gate, inputs_as, problem_pair,
                               rel_energy_err, to_np)

pytestmark = pytest.mark.gpu

# variant name -> oracle arguments
ORACLE_ARGS = {
    "omega_one": dict(omega="identity", correction=True),
    "no_correction": dict(omega="procrustes", correction=False),
    "plain": dict(omega="plain", correction=True),
}


def _solve(w, K, variant, dtype="f64", tol=1e-6):
    import paper_1905_00473_amd as pw
    P, Q = problem_pair(w, max_iters=max(K, 1), tol=tol, dtype=dtype)
    s = pw.Solver(P)
    u0, p0 = inputs_as(w, dtype)
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    s.set_variant(variant)
    s.run(K)
    return s, Q, u0, p0


def _compare(s, Q, w, u0, p0, K, variant, floor):
    ref = O.theta_parareal(Q, w.c, u0, p0, K, **ORACLE_ARGS[variant])
    gate = derived_gate(Q, w, u0, p0, K, floor, **ORACLE_ARGS[variant])
    worst = 0.0
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        worst = max(worst, rel_energy_err(to_np(u), to_np(p), ref.u[n],
                                          ref.p[n], w.c, Q.dx_fine))
    assert worst < gate, (variant, worst, gate)
    rho, rk = s.residuals()
    assert list(rk) == list(ref.rank), (rk, ref.rank)
    np.testing.assert_allclose(rho, ref.rho, rtol=1e-6)
    return worst


@pytest.mark.parametrize("variant", list(ORACLE_ARGS))
def test_wave1d_fp64(variant):
    w = W.wave1d()
    s, Q, u0, p0 = _solve(w, w.K, variant)
    _compare(s, Q, w, u0, p0, w.K, variant, 1e-12)
    s.close()


@pytest.mark.parametrize("variant", list(ORACLE_ARGS))
def test_disc2d_small_fp64(variant):
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5, dtype="f64",
                 compensated=False)
    s, Q, u0, p0 = _solve(w, 3, variant)
    _compare(s, Q, w, u0, p0, 3, variant, 1e-12)
    s.close()


@pytest.mark.parametrize("variant", list(ORACLE_ARGS))
def test_ragged_2d_fp64(variant):
    """Non-power-of-two coarse axes (DFT path of Lambda^dag), ragged tiles."""
    w, _, _ = W.misfit_case((60, 84), ratio=3, N=5, K=2, T=0.3, m_fine=12,
                            m_coarse=4)
    s, Q, u0, p0 = _solve(w, 2, variant)
    _compare(s, Q, w, u0, p0, 2, variant, 1e-12)
    s.close()


@pytest.mark.parametrize("variant", list(ORACLE_ARGS))
def test_layers3d_small_fp32(variant):
    w = W.layers3d(n=32, ratio=4, N=4, K=2, T=0.2)
    s, Q, u0, p0 = _solve(w, 2, variant, dtype="f32")
    ref = O.theta_parareal(Q, w.c, u0, p0, 2, **ORACLE_ARGS[variant])
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        assert e < 1e-5, (variant, n, e)
    s.close()


@pytest.mark.parametrize("variant", list(ORACLE_ARGS))
def test_single_slice(variant):
    w, _, _ = W.misfit_case((64,), ratio=4, N=1, K=2, T=0.0625, m_fine=8,
                            m_coarse=2)
    s, Q, u0, p0 = _solve(w, 2, variant)
    _compare(s, Q, w, u0, p0, 2, variant, 1e-12)
    s.close()


def test_variant_switch_back_reproduces_algorithm3():
    """Setting the default variant again gives Algorithm 3 bit for bit."""
    import torch
    w = W.wave1d()
    s, _, _, _ = _solve(w, 3, "theta")
    ref = [s.state(n) for n in range(w.N + 1)]
    s.set_variant("plain")
    s.run(3)
    s.set_variant("theta")
    s.run(3)
    for n in range(w.N + 1):
        u, p = s.state(n)
        assert torch.equal(u, ref[n][0]) and torch.equal(p, ref[n][1]), n
    s.close()


def test_variant_errors():
    import paper_1905_00473_amd as pw
    w = W.wave1d()
    s, _, _, _ = _solve(w, 1, "plain")
    for bad in (-1, 4):
        with pytest.raises(pw.PwError, match="unknown variant"):
            s.set_variant(bad)
    with pytest.raises(pw.PwError, match="Algorithm 3 only"):
        s.run_taped(1)
    s.close()


@pytest.mark.parametrize("variant", list(ORACLE_ARGS))
def test_disc2d_small_fp32(variant):
    """The comparators with the FP32 compensated state: 1e-5 in the energy
    norm relative to the oracle's result (run on the same FP32-rounded
    initial data), the FP32 gate of Algorithm 3."""
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5)
    s, Q, u0, p0 = _solve(w, 3, variant, dtype="f32")
    ref = O.theta_parareal(Q, w.c, u0, p0, 3, **ORACLE_ARGS[variant])
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        assert e < 1e-5, (variant, n, e)
    s.close()
