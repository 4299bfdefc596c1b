"""Random subsampling of the data matrices (Sec. 6.5) on the GPU against
the FP64 oracle fed the same column table.

Gate: FP64 state, svd tol 1e-6: max(1e-12, 256 A eps) in the energy norm
per slice, with A the amplification of a relative input perturbation
through the same iteration measured on the oracle (about 1e3 on wave1d,
below 10 on the 2D cases); equal ranks, rho to rtol 1e-6.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import (derived_gate, problem_pair, rel_energy_err,
                               to_np)

pytestmark = pytest.mark.gpu


def _solve(w, K, cols, tol=1e-6):
    import paper_1905_00473_amd as pw
    P, Q = problem_pair(w, max_iters=max(K, 1), tol=tol, dtype="f64")
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    s.set_sampling(cols)
    s.run(K)
    return s, Q


def _compare(s, Q, w, K, cols):
    sc = None if cols is None else list(cols)
    ref = O.theta_parareal(Q, w.c, w.u0, w.p0, K, sample_cols=sc)
    gate = derived_gate(Q, w, w.u0, w.p0, K, sample_cols=sc)
    worst = 0.0
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        worst = max(worst, rel_energy_err(to_np(u), to_np(p), ref.u[n],
                                          ref.p[n], w.c, Q.dx_fine))
    assert worst < gate, (worst, gate)
    rho, rk = s.residuals()
    assert list(rk) == list(ref.rank), (rk, ref.rank)
    np.testing.assert_allclose(rho, ref.rho, rtol=1e-6)


@pytest.mark.parametrize("n_per_iter", [1, 5, 16])
def test_wave1d_sampled(n_per_iter):
    w = W.wave1d()
    cols = W.sample_columns(w.N, n_per_iter, w.K, seed=n_per_iter)
    s, Q = _solve(w, w.K, cols)
    _compare(s, Q, w, w.K, cols)
    s.close()


def test_disc2d_small_sampled():
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5, dtype="f64",
                 compensated=False)
    cols = W.sample_columns(w.N, 3, 3, seed=11)
    s, Q = _solve(w, 3, cols)
    _compare(s, Q, w, 3, cols)
    s.close()


def test_waveguide_small_sampled():
    """The Sec. 6.5 recipe on a 40^2 / 20^2 grid with 20 slices."""
    w = W.waveguide2d(n=40, ratio=2, N=20, K=3, T=0.4, m_fine=25,
                      m_coarse=5)
    cols = W.sample_columns(w.N, 6, 3, seed=5)
    s, Q = _solve(w, 3, cols)
    _compare(s, Q, w, 3, cols)
    s.close()


@pytest.mark.parametrize("n_per_iter", [70, 100])
def test_many_slices_sampled(n_per_iter):
    """100 slices, samples of more than 64 columns (blocked
    orthonormalisation inside Algorithm 1) on the waveguide, whose data
    matrices are numerically low-rank (singular values of the sampled
    columns fall to 2e-13 of the largest, the decay Sec. 6.5 reports)."""
    w = W.waveguide2d(n=40, ratio=2, N=100, K=2, T=1.0, m_fine=10,
                      m_coarse=2)
    cols = W.sample_columns(w.N, n_per_iter, 2, seed=9)
    s, Q = _solve(w, 2, cols)
    _compare(s, Q, w, 2, cols)
    s.close()


def test_unsorted_table_and_switch_off():
    """A permuted full table gives the unsampled iteration up to rounding;
    switching sampling off gives it bit for bit."""
    import torch
    w = W.wave1d()
    rng = np.random.default_rng(2)
    perm = np.array([rng.permutation(w.N) for _ in range(3)])
    s, Q = _solve(w, 3, perm)
    _compare(s, Q, w, 3, None)
    # both runs are within the derived gate of the oracle, so within twice
    # that of each other
    gate = 2 * derived_gate(Q, w, w.u0, w.p0, 3)
    a = [s.state(n) for n in range(w.N + 1)]
    s.set_sampling(None)
    s.run(3)
    b = [s.state(n) for n in range(w.N + 1)]
    s2, _ = _solve(w, 3, None)
    for n in range(w.N + 1):
        u, p = s2.state(n)
        assert torch.equal(u, b[n][0]) and torch.equal(p, b[n][1]), n
        assert rel_energy_err(to_np(a[n][0]), to_np(a[n][1]), to_np(u),
                              to_np(p), w.c, Q.dx_fine) < gate
    s.close()
    s2.close()


def test_sampling_errors():
    import paper_1905_00473_amd as pw
    w = W.wave1d()
    P, _ = problem_pair(w, max_iters=3, tol=1e-6, dtype="f64")
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    for bad in ([[0, 0]], [[w.N]], [[-1]], np.zeros((2, w.N + 1))):
        with pytest.raises(pw.PwError):
            s.set_sampling(bad)
    s.set_sampling(W.sample_columns(w.N, 4, 2))
    with pytest.raises(pw.PwError, match="fewer iterations"):
        s.run(3)
    s.run(2)
    s.close()


def test_sampled_fp32():
    """Subsampling with the FP32 compensated state, 1e-5 against the
    oracle fed the same table and the same FP32-rounded initial data."""
    import paper_1905_00473_amd as pw
    from tests.gpu_helpers import inputs_as
    w = W.disc2d(n=96, ratio=4, N=8, K=3, T=0.5)
    cols = W.sample_columns(w.N, 4, 3, seed=13)
    P, Q = problem_pair(w, max_iters=3, tol=1e-6, dtype="f32")
    s = pw.Solver(P)
    u0, p0 = inputs_as(w, "f32")
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    s.set_sampling(cols)
    s.run(3)
    ref = O.theta_parareal(Q, w.c, u0, p0, 3, sample_cols=list(cols))
    for n in range(1, Q.N + 1):
        u, p = s.state(n)
        e = rel_energy_err(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                           Q.dx_fine)
        assert e < 1e-5, (n, e)
    s.close()
