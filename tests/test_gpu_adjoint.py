"""Parity of the HIP adjoint (pw_run_taped / pw_run_frozen / pw_traces /
pw_backward) with the FP64 oracle's hand-written adjoint of Algorithm 3 with
frozen correctors, plus finite differences through the GPU's own frozen
forward, checkpoint-interval invariance and the autograd Function.

Gates (FP64 state): traces to 1e-12 absolute (values are O(0.1)); J to
1e-10 relative; gradient max-abs error <= 1e-8 * max |oracle gradient|.
The two sides compute the correctors independently (same Algorithm 1, other
rounding); with svd_tol 1e-6 the kept directions have sigma_i / sigma_1 >=
1e-6, where rounding moves Omega by ~eps * 1e6 ~ 1e-10 relative.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import adjoint as A
from tests.gpu_helpers import to_np

pytestmark = pytest.mark.gpu

CASES = {
    "2d": dict(shape=(32, 32), ratio=4, m_fine=8, m_coarse=2),
    "1d": dict(shape=(64,), ratio=4, m_fine=16, m_coarse=4),
    "3d": dict(shape=(16, 16, 16), ratio=2, m_fine=8, m_coarse=2),
    # 2D, several tiles and a ragged tail on both axes, N = 6 slices
    "2d_ragged": dict(shape=(40, 72), ratio=4, N=6, m_fine=12, m_coarse=3,
                      T=0.375),
    # 2D with N * points = 2^18: the fine reverse steps run as row streams,
    # four steps per launch
    "2d_stream": dict(shape=(128, 128), ratio=4, N=16, m_fine=32, m_coarse=8,
                      T=0.5),
    # 1D, 100 slices (blocked QR in the taped run's Algorithm 1)
    "1d_many": dict(shape=(512,), ratio=4, N=100, m_fine=16, m_coarse=4,
                    T=1.0),
}


def _solver(w, K, dtype="f64", compensated=False):
    import paper_1905_00473_amd as pw
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, dtype, compensated, max(K, 1))
    s = pw.Solver(P)
    s.set_medium(w.c)
    if dtype == "f32":
        u0 = w.u0.astype(np.float32).astype(np.float64)
    else:
        u0 = w.u0
    s.set_initial(u0, w.p0)
    return s, u0


def _oracle(w, u0, K, rec, data):
    Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                  w.grad_order, w.tol)
    corr, cc = A.record_correctors(Q, w.c, u0, w.p0, max(K, 1))
    J, g = A.gradient(Q, w.c * w.c, u0, w.p0, K, corr, cc, rec, data)
    u, _ = A.forward_frozen(Q, w.c * w.c, u0, w.p0, K, corr, cc)
    tr = np.stack([u[n].ravel()[rec] for n in range(1, w.N + 1)])
    # rounding sensitivity of the traces: their change under a 1e-13
    # relative perturbation of u0 (frozen correctors), per unit
    eps = 1e-13
    rng = np.random.default_rng(11)
    u1 = u0 * (1 + eps * rng.standard_normal(np.shape(u0)))
    v, _ = A.forward_frozen(Q, w.c * w.c, u1, w.p0, K, corr, cc)
    tr1 = np.stack([v[n].ravel()[rec] for n in range(1, w.N + 1)])
    amp = np.abs(tr1 - tr).max() / eps
    # and to the rounding of Algorithm 1: correctors recorded with the data
    # columns in the opposite order (the same exact arithmetic)
    res2 = O.theta_parareal(Q, w.c, u0, w.p0, max(K, 1), record_correctors=True,
                            sample_cols=[np.arange(w.N)[::-1]] * max(K, 1))
    v2, _ = A.forward_frozen(Q, w.c * w.c, u0, w.p0, K, res2.correctors, cc)
    tr2 = np.stack([v2[n].ravel()[rec] for n in range(1, w.N + 1)])
    gate = max(1e-12, 256 * amp * 2.0 ** -52, 16 * np.abs(tr2 - tr).max())
    return J, g, tr, [c[0].shape[1] for c in corr[:K]], gate


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("K", [0, 1, 2])
def test_backward_matches_oracle(case, K):
    kw = dict(CASES[case])
    w, rec, data = W.misfit_case(K=K, **kw)
    print(f"adjoint parity {case} K={K} shape={w.shape}", flush=True)
    s, u0 = _solver(w, K)
    s.run_taped(K)
    tr = to_np(s.traces(rec))
    J_ref, g_ref, tr_ref, ranks_ref, gate = _oracle(w, u0, K, rec, data)
    _, ranks = s.residuals()
    assert list(ranks) == ranks_ref
    # 1e-12, or where larger (long runs: 100 slices) 256 eps times the
    # traces' sensitivity to rounding of the input, or 16 times their
    # spread over two orderings of Algorithm 1's arithmetic
    np.testing.assert_allclose(tr, tr_ref, rtol=0, atol=gate)
    seed = tr - data
    J = 0.5 * float(np.sum(seed * seed))
    assert J == pytest.approx(J_ref, rel=1e-10)
    g = to_np(s.backward(rec, seed, wrt="c2"))
    err = np.abs(g - g_ref).max()
    assert err <= 1e-8 * np.abs(g_ref).max(), (err, np.abs(g_ref).max())
    # d/dc = 2 c d/dc^2
    gc = to_np(s.backward(rec, seed, wrt="c"))
    np.testing.assert_allclose(gc, 2 * w.c * g, rtol=1e-14, atol=0)
    s.close()


@pytest.mark.parametrize("case", ["2d_ragged", "2d_stream"])
def test_checkpoint_interval_does_not_change_the_gradient(case):
    w, rec, data = W.misfit_case(K=2, **CASES[case])
    s, _ = _solver(w, 2)
    s.run_taped(2)
    seed = to_np(s.traces(rec)) - data
    g64 = to_np(s.backward(rec, seed, checkpoint_every=64))
    for ck in (1, 3, 5, 12):
        g = to_np(s.backward(rec, seed, checkpoint_every=ck))
        assert np.array_equal(g, g64), ck
    s.close()


def test_frozen_replay_reproduces_the_taped_run():
    w, rec, _ = W.misfit_case(K=2, **CASES["2d"])
    s, _ = _solver(w, 2)
    s.run_taped(2)
    a = to_np(s.traces(rec))
    u2a, p2a = s.state(w.N)
    s.run_frozen(2)
    b = to_np(s.traces(rec))
    u2b, p2b = s.state(w.N)
    assert np.array_equal(a, b)
    assert np.array_equal(to_np(u2a), to_np(u2b))
    assert np.array_equal(to_np(p2a), to_np(p2b))
    s.close()


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_gradient_matches_gpu_finite_differences(case):
    """Central differences of J through pw_run_frozen (the GPU's own frozen
    forward) against <grad, e> for random directions e."""
    K = 2
    w, rec, data = W.misfit_case(K=K, **CASES[case])
    s, _ = _solver(w, K)
    s.run_taped(K)
    seed = to_np(s.traces(rec)) - data
    J0 = 0.5 * float(np.sum(seed * seed))
    g = to_np(s.backward(rec, seed, wrt="c2"))
    rng = np.random.default_rng(7)
    c2 = w.c * w.c
    for t in range(2):
        e = rng.standard_normal(w.shape)
        eps = 1e-5

        def J_at(x):
            s.set_medium(np.sqrt(x))
            s.run_frozen(K)
            d = to_np(s.traces(rec)) - data
            return 0.5 * float(np.sum(d * d))

        fd = (J_at(c2 + eps * e) - J_at(c2 - eps * e)) / (2 * eps)
        ad = float(np.sum(g * e))
        assert ad == pytest.approx(fd, rel=1e-6, abs=1e-12 * J0), (t, ad, fd)
    s.close()


@pytest.mark.parametrize("K", [1, 2])
@pytest.mark.parametrize("case", ["2d", "1d", "3d"])
def test_fp32_compensated_gradient_close_to_oracle(case, K):
    """FP32 compensated states, FP64 adjoint: the gradient follows the
    FP64 oracle (from the same FP32-rounded initial state) to 1e-5 of its
    maximum, the FP32 tolerance of the state."""
    w, rec, data = W.misfit_case(K=K, **CASES[case])
    s, u0 = _solver(w, K, dtype="f32", compensated=True)
    s.run_taped(K)
    seed = to_np(s.traces(rec)) - data
    g = to_np(s.backward(rec, seed))
    _, g_ref, _, _, _ = _oracle(w, u0, K, rec, data)
    err = np.abs(g - g_ref).max()
    assert err <= 1e-5 * np.abs(g_ref).max(), (err, np.abs(g_ref).max())
    s.close()


def test_autograd_function():
    import torch
    import paper_1905_00473_amd as pw
    K = 1
    w, rec, data = W.misfit_case(K=K, **CASES["2d"])
    s, u0 = _solver(w, K)
    c = torch.tensor(w.c, dtype=torch.float64, device="cuda",
                     requires_grad=True)
    d = torch.tensor(data, dtype=torch.float64, device="cuda")
    tr = pw.PararealTraces.apply(c, s, rec, K)
    loss = 0.5 * ((tr - d) ** 2).sum()
    loss.backward()
    J_ref, g_ref, _, _, _ = _oracle(w, u0, K, rec, data)
    assert float(loss.detach()) == pytest.approx(J_ref, rel=1e-10)
    gc = to_np(c.grad)
    ref = 2 * w.c * g_ref
    assert np.abs(gc - ref).max() <= 1e-8 * np.abs(ref).max()
    s.close()


def test_backward_call_order_and_argument_errors():
    import paper_1905_00473_amd as pw
    w, rec, data = W.misfit_case(K=1, **CASES["2d"])
    s, _ = _solver(w, 1)
    seed = np.zeros((w.N, rec.size))
    with pytest.raises(pw.PwError, match="PW_ESTATE"):
        s.backward(rec, seed)
    with pytest.raises(pw.PwError, match="PW_ESTATE"):
        s.run_frozen(1)
    s.run_taped(1)
    with pytest.raises(pw.PwError, match="PW_EINVAL"):
        s.traces(np.array([w.npts], dtype=np.int64))
    with pytest.raises(pw.PwError, match="PW_EINVAL"):
        s.backward(np.array([-1], dtype=np.int64), np.zeros((w.N, 1)))
    with pytest.raises(pw.PwError, match="PW_ESTATE"):
        s.run_frozen(2)
    s.set_medium(w.c)
    with pytest.raises(pw.PwError, match="PW_ESTATE"):
        s.backward(rec, seed)
    # a frozen replay makes the tape current again
    s.run_frozen(1)
    g = to_np(s.backward(rec, seed))
    assert np.all(g == 0.0)
    s.close()


def test_full_size_gradient_directional_fd():
    """At the full misfit workload size (512^2, N = 32, m_F = 96, 128
    receivers recorded every fine step, absorbing layer and point source;
    FP64 states, K = 2, checkpoints every 64 steps) the oracle cannot run;
    the property checked is <grad, e> = central difference of J through the
    GPU's frozen forward, for a smooth random direction e."""
    import paper_1905_00473_amd as pw
    K = 2
    w, rec, _, fd = W.misfit2d(K=K, dtype="f64", compensated=False)
    print(f"full-size adjoint {w.shape} N={w.N} m_F={w.m_fine}", flush=True)
    data = 0.01 * np.random.default_rng(3).standard_normal(
        (w.N, w.m_fine, rec.size))
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f64", False, K,
                        sponge_width=fd["width"],
                        sponge_reflection=fd["reflection"],
                        sponge_cmax=fd["c_max"])
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_source(fd["src_pos"], fd["freq"], fd["t0"])
    s.set_initial(w.u0, w.p0)
    dt = w.T / w.N / w.m_fine
    s.run_taped(K)
    res = to_np(s.trace_sweep(rec)) - data
    J0 = 0.5 * dt * float(np.sum(res * res))
    g = to_np(s.backward_sweep(rec, dt * res, wrt="c2", checkpoint_every=64))
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0
    e = W.smooth_random_field(w.shape, 0.05, 7)
    c2 = w.c * w.c
    eps = 1e-4

    def J_at(x):
        s.set_medium(np.sqrt(x))
        s.run_frozen(K)
        d = to_np(s.trace_sweep(rec)) - data
        return 0.5 * dt * float(np.sum(d * d))

    fd_ = (J_at(c2 + eps * e) - J_at(c2 - eps * e)) / (2 * eps)
    ad = float(np.sum(g * e))
    assert ad == pytest.approx(fd_, rel=1e-5, abs=1e-12 * J0), (ad, fd_)
    s.close()


def _parity_with(w, K, rec, data, setup, oracle_kwargs):
    """Taped run + backward on the GPU after `setup(solver)`, against the
    adjoint oracle with correctors recorded the same way."""
    s, u0 = _solver(w, K)
    setup(s)
    s.run_taped(K)
    tr = to_np(s.traces(rec))
    Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                  w.grad_order, w.tol)
    corr, cc = A.record_correctors(Q, w.c, u0, w.p0, max(K, 1),
                                   **oracle_kwargs)
    J_ref, g_ref = A.gradient(Q, w.c * w.c, u0, w.p0, K, corr, cc, rec, data)
    u, _ = A.forward_frozen(Q, w.c * w.c, u0, w.p0, K, corr, cc)
    tr_ref = np.stack([u[n].ravel()[rec] for n in range(1, w.N + 1)])
    np.testing.assert_allclose(tr, tr_ref, rtol=0, atol=1e-12)
    seed = tr - data
    g = to_np(s.backward(rec, seed, wrt="c2"))
    err = np.abs(g - g_ref).max()
    assert err <= 1e-8 * np.abs(g_ref).max(), (err, np.abs(g_ref).max())
    s.close()


def test_backward_with_sampling_matches_oracle():
    """Taped run with random subsampling of the data matrices."""
    K = 2
    w, rec, data = W.misfit_case(K=K, **CASES["2d_ragged"])
    cols = W.sample_columns(w.N, 3, K, seed=17)
    _parity_with(w, K, rec, data, lambda s: s.set_sampling(cols),
                 dict(sample_cols=list(cols)))


def test_backward_spectral_gradient_matches_oracle():
    """Taped run with the Fourier gradient inside Lambda."""
    K = 2
    w, rec, data = W.misfit_case(K=K, **CASES["2d"])
    w.grad_order = "spectral"
    _parity_with(w, K, rec, data, lambda s: None, {})
