"""Pins of the oracle's misfit gradient (frozen corrector): dot-product
tests of every hand-written transpose and finite differences of the same
frozen forward map."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import adjoint as A


def _setup(K=2, tol=1e-6, seed=0):
    w, receivers, data = W.misfit_case(K=K, tol=tol, seed=seed)
    prob = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                     w.grad_order, w.tol)
    return prob, w.c, w.u0, w.p0, receivers, data


def test_forward_frozen_reproduces_algorithm3():
    prob, c, u0, p0, _, _ = _setup()
    K = 2
    res = O.theta_parareal(prob, c, u0, p0, K, record_correctors=True)
    corr, cc = A.record_correctors(prob, c, u0, p0, K)
    u, p = A.forward_frozen(prob, c * c, u0, p0, K, corr, cc)
    for n in range(prob.N + 1):
        np.testing.assert_allclose(u[n], res.u[n], atol=1e-13)
        np.testing.assert_allclose(p[n], res.p[n], atol=1e-12)


def test_transposes_dot_product():
    rng = np.random.default_rng(3)
    prob, c, u0, p0, _, _ = _setup()
    cs, fs = prob.coarse_shape, prob.shape
    x = rng.standard_normal(cs)
    y = rng.standard_normal(fs)
    assert np.dot(O.interp(x, 4).ravel(), y.ravel()) == pytest.approx(
        np.dot(x.ravel(), A._interp_T(y, 4, cs).ravel()), rel=1e-12)
    assert np.dot(O.restrict(y, 4).ravel(), x.ravel()) == pytest.approx(
        np.dot(y.ravel(), A._restrict_T(x, 4, fs).ravel()), rel=1e-12)
    # velocity Verlet: <J dx, l> = <dx, J^T l> (linear in the state)
    c2 = c * c
    du, dp = rng.standard_normal(fs), rng.standard_normal(fs)
    lu, lp = rng.standard_normal(fs), rng.standard_normal(fs)
    ou, op, us = A._prop_store(du, dp, c2, prob.dt_fine, prob.dx_fine, 5)
    au, ap, _ = A._prop_adjoint(us, lu, lp, c2, prob.dt_fine, prob.dx_fine)
    lhs = np.sum(ou * lu) + np.sum(op * lp)
    rhs = np.sum(du * au) + np.sum(dp * ap)
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("K", [0, 1, 2])
def test_gradient_matches_finite_differences(K):
    prob, c, u0, p0, rec, data = _setup()
    corr, cc = A.record_correctors(prob, c, u0, p0, max(K, 1))
    c2 = c * c
    J, g = A.gradient(prob, c2, u0, p0, K, corr, cc, rec, data)
    rng = np.random.default_rng(11)
    n = prob.shape[0]
    Y, X = np.meshgrid(np.arange(n) / n, np.arange(n) / n, indexing="ij")
    for t in range(3):
        e = np.cos(2 * np.pi * (rng.integers(1, 4) * X + rng.integers(0, 3) * Y)
                   + rng.uniform(0, 6)) + 0.3 * rng.standard_normal((n, n))
        eps = 1e-5
        def J_at(cc2):
            u, _ = A.forward_frozen(prob, cc2, u0, p0, K, corr, cc)
            return A.misfit(u, rec, data)
        fd = (J_at(c2 + eps * e) - J_at(c2 - eps * e)) / (2 * eps)
        ad = float(np.sum(g * e))
        assert ad == pytest.approx(fd, rel=2e-6, abs=1e-12 * abs(J)), (t, ad, fd)


@pytest.mark.parametrize("shape,ratio,m_fine,m_coarse", [
    ((64,), 4, 16, 4), ((16, 16, 16), 2, 8, 2)])
def test_gradient_fd_1d_3d(shape, ratio, m_fine, m_coarse):
    """The same finite-difference pin on a 1D and a 3D grid (the transposes
    of the separable interpolation along every axis)."""
    K = 1
    w, rec, data = W.misfit_case(shape, ratio=ratio, K=K, m_fine=m_fine,
                                 m_coarse=m_coarse)
    prob = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                     w.grad_order, w.tol)
    corr, cc = A.record_correctors(prob, w.c, w.u0, w.p0, K)
    c2 = w.c * w.c
    J, g = A.gradient(prob, c2, w.u0, w.p0, K, corr, cc, rec, data)
    e = np.random.default_rng(5).standard_normal(shape)
    eps = 1e-5

    def J_at(cc2):
        u, _ = A.forward_frozen(prob, cc2, w.u0, w.p0, K, corr, cc)
        return A.misfit(u, rec, data)

    fd = (J_at(c2 + eps * e) - J_at(c2 - eps * e)) / (2 * eps)
    assert float(np.sum(g * e)) == pytest.approx(fd, rel=2e-6,
                                                 abs=1e-12 * abs(J))


# ---- absorbing layer and point source ----------------------------------
def _forced_setup(K=2, seed=0):
    w, rec, data, fd = W.forced_misfit_case(K=K, seed=seed)
    prob = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                     w.grad_order, w.tol)
    return prob, w.c, w.u0, w.p0, rec, data, O.Forcing(**fd)


def test_damped_verlet_adjoint_dot_product():
    """<J dx, l> = <dx, J^T l> for velocity Verlet with the layer (the
    source adds a constant, so the map of a state difference is the damped
    linear one)."""
    rng = np.random.default_rng(5)
    prob, c, _, _, _, _, fo = _forced_setup()
    fs = O.forcing_setup(prob, c, fo)
    assert fs["dF"].min() < 0.9           # the layer really damps
    c2, fsh = c * c, prob.shape
    du, dp = rng.standard_normal(fsh), rng.standard_normal(fsh)
    lu, lp = rng.standard_normal(fsh), rng.standard_normal(fsh)
    ou, op, us = A._prop_store(du, dp, c2, prob.dt_fine, prob.dx_fine, 6,
                               fs["dF"])
    au, ap, _ = A._prop_adjoint(us, lu, lp, c2, prob.dt_fine, prob.dx_fine,
                                fs["dF"])
    lhs = np.sum(ou * lu) + np.sum(op * lp)
    rhs = np.sum(du * au) + np.sum(dp * ap)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_frozen_forward_is_affine_in_state_and_source():
    """With the correctors frozen, Algorithm 3 is a linear map of the
    initial state and the source jointly: the run with data and source
    equals the run with the data alone plus the run with the source alone
    (same layer).  Pins the source's handling in F, C and the sweep, where
    it must cancel in the difference theta(w) - theta(U)."""
    prob, c, _, _, _, _, fo = _forced_setup()
    rng = np.random.default_rng(2)
    u0 = rng.standard_normal(prob.shape)
    p0 = rng.standard_normal(prob.shape)
    K = 2
    corr, cc = A.record_correctors(prob, c, u0, p0, K, forcing=fo)
    layer_only = O.Forcing(width=fo.width, reflection=fo.reflection,
                           c_max=fo.c_max)
    c2 = c * c
    ua, pa = A.forward_frozen(prob, c2, u0, p0, K, corr, cc, forcing=fo)
    ub, pb = A.forward_frozen(prob, c2, u0, p0, K, corr, cc,
                              forcing=layer_only)
    z = np.zeros(prob.shape)
    uc, pc = A.forward_frozen(prob, c2, z, z, K, corr, cc, forcing=fo)
    scale = max(np.abs(x).max() for x in ua[1:])
    for n in range(1, prob.N + 1):
        np.testing.assert_allclose(ua[n], ub[n] + uc[n], atol=1e-12 * scale)
        np.testing.assert_allclose(pa[n], pb[n] + pc[n],
                                   atol=1e-12 * max(np.abs(x).max() for x in pa[1:]))
    # the source alone really drives the run
    assert max(np.abs(x).max() for x in uc[1:]) > 1e-3 * scale


@pytest.mark.parametrize("traces", ["sweep", "coupling"])
@pytest.mark.parametrize("K", [0, 2])
def test_forced_gradient_matches_finite_differences(K, traces):
    """The misfit gradient through Algorithm 3 with the layer and source
    (frozen correctors, layer held fixed by its c_max) against central
    differences of the same forward, for a record sampled every fine step
    of one more F sweep ("sweep") and at the coupling times."""
    prob, c, u0, p0, rec, data, fo = _forced_setup()
    corr, cc = A.record_correctors(prob, c, u0, p0, max(K, 1), forcing=fo)
    if traces == "coupling":
        data = data[:, -1, :]
    c2 = c * c
    J, g = A.gradient(prob, c2, u0, p0, K, corr, cc, rec, data, forcing=fo,
                      traces=traces)

    def J_at(cc2):
        u, p = A.forward_frozen(prob, cc2, u0, p0, K, corr, cc, forcing=fo)
        if traces == "coupling":
            return A.misfit(u, rec, data)
        return A.sweep_misfit(A.sweep_traces(prob, cc2, u, p, rec, fo), data,
                              prob.dt_fine)

    assert J == pytest.approx(J_at(c2), rel=1e-13)
    rng = np.random.default_rng(13)
    n = prob.shape[0]
    Y, X = np.meshgrid(np.arange(n) / n, np.arange(n) / n, indexing="ij")
    for t in range(3):
        e = np.cos(2 * np.pi * (rng.integers(1, 4) * X + rng.integers(0, 3) * Y)
                   + rng.uniform(0, 6)) + 0.3 * rng.standard_normal((n, n))
        eps = 1e-5
        fd = (J_at(c2 + eps * e) - J_at(c2 - eps * e)) / (2 * eps)
        ad = float(np.sum(g * e))
        assert ad == pytest.approx(fd, rel=2e-6, abs=1e-12 * abs(J)), (t, ad, fd)
