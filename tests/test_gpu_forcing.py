"""The absorbing layer and point source (PW_SPONGE, pw_set_source) on the
GPU against the oracle: the forced propagators F and C, the serial fine
solve, Algorithm 3 with forcing, the receiver record of one more F sweep
sampled every fine step (pw_trace_sweep) and its gradient
(pw_backward_sweep) with frozen correctors and a fixed layer.

Gates.  FP64 propagators and serial solve: 1e-12 relative in the energy
norm per state (rounding of m_F steps).  FP32 compensated propagators:
1e-5.  Algorithm 3: the derived per-norm gates of the other end-to-end
tests (amplification, column order, SVD driver, form of the correction).
Record: 1e-12 of its largest value (FP64; the sweep starts from the same
injected states), 1e-5 for FP32 compensated.  Gradient: as the periodic
adjoint tests, the two sides fit their correctors independently (svd tol
1e-6), record within the derived gate, J to 1e-10, gradient within 1e-8 of
the largest oracle value; plus central differences of the GPU's own frozen
forward."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import adjoint as A
from tests.gpu_helpers import derived_gates, rel_energy_err, state_errors, to_np

pytestmark = pytest.mark.gpu

CASES = {
    "2d": dict(shape=(32, 32), ratio=4, m_fine=8, m_coarse=2),
    # several column blocks and row segments with ragged tails, a box
    # longer in x than in y, ragged last launch (12 = 8 + 4 steps in FP32)
    "2d_ragged": dict(shape=(40, 72), ratio=4, N=6, m_fine=12, m_coarse=3,
                      T=0.375),
    # N * points = 2^18: the fine reverse steps run as row streams
    "2d_stream": dict(shape=(128, 128), ratio=4, N=16, m_fine=32, m_coarse=8,
                      T=0.5),
}


def _pulse(shape, seed):
    """A Gaussian pulse of random centre plus a small random field."""
    rng = np.random.default_rng(seed)
    u, p = W.random_pulses(shape, 1, seed)
    return u[0] + 0.01 * rng.standard_normal(shape), p[0]


def _setup(case, K=2, dtype="f64", comp=False, nonzero=True):
    import paper_1905_00473_amd as pw
    w, rec, data, fd = W.forced_misfit_case(K=K, **CASES[case])
    if nonzero:
        w.u0, w.p0 = _pulse(w.shape, 5)
    if dtype == "f32":
        w.u0 = w.u0.astype(np.float32).astype(np.float64)
        w.p0 = w.p0.astype(np.float32).astype(np.float64)
    fo = O.Forcing(**fd)
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, dtype, comp, max(K, 1),
                        sponge_width=fd["width"],
                        sponge_reflection=fd["reflection"],
                        sponge_cmax=fd["c_max"])
    Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                  w.grad_order, w.tol)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_source(fd["src_pos"], fd["freq"], fd["t0"])
    s.set_initial(w.u0, w.p0)
    return w, rec, data, fd, fo, s, Q


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("case", list(CASES))
def test_forced_propagators_match_oracle(case, prec):
    import torch

    import paper_1905_00473_amd as pw
    dtype, comp = ("f64", False) if prec == "f64" else ("f32", True)
    w, _, _, _, fo, s, Q = _setup(case, dtype=dtype, comp=comp)
    print(f"forced F/C {case} {prec} shape={w.shape} N={w.N}", flush=True)
    td = torch.float64 if dtype == "f64" else torch.float32
    fs = O.forcing_setup(Q, w.c, fo)
    assert fs["dF"].min() < 1.0 and fs["srcF"] is not None
    rng = np.random.default_rng(3)
    gate = 1e-12 if prec == "f64" else 1e-5
    cc = O.restrict(w.c, w.ratio)
    for grid, shape, c, h, dx, m, damp, src in (
            (pw.FINE, w.shape, w.c, Q.dt_fine, Q.dx_fine, Q.m_fine, fs["dF"],
             fs["srcF"]),
            (pw.COARSE, Q.coarse_shape, cc, Q.dt_coarse, Q.dx_coarse,
             Q.m_coarse, fs["dC"], fs["srcC"])):
        u = 0.1 * rng.standard_normal((w.N,) + shape)
        p = 0.1 * rng.standard_normal((w.N,) + shape)
        if dtype == "f32":
            u = u.astype(np.float32).astype(np.float64)
            p = p.astype(np.float32).astype(np.float64)
        uo, po = s.propagate(torch.tensor(u, dtype=td, device="cuda"),
                             torch.tensor(p, dtype=td, device="cuda"), grid)
        uo, po = to_np(uo), to_np(po)
        worst = 0.0
        for n in range(w.N):
            ru, rp = O.propagate_forced(u[n], p[n], c * c, h, dx, m, damp, src,
                                        n * Q.dt_com)
            worst = max(worst, rel_energy_err(uo[n], po[n], ru, rp, c, dx))
        print(f"  grid {grid}: worst {worst:.3g} (gate {gate:g})", flush=True)
        assert worst < gate, (grid, worst)
    s.close()


def test_forced_serial_fine_matches_oracle():
    """pw_serial_fine (one time) and pw_serial_fine_states (every coupling
    time, one chain): the same states bit for bit, and the oracle's."""
    w, _, _, _, fo, s, Q = _setup("2d_ragged")
    us, ps = O.serial_fine(Q, w.c, w.u0, w.p0, forcing=fo)
    au, ap = s.serial_fine_states()
    assert tuple(au.shape) == (w.N + 1,) + w.shape
    for n in range(w.N + 1):
        err = rel_energy_err(to_np(au[n]), to_np(ap[n]), us[n], ps[n], w.c,
                             Q.dx_fine)
        assert err < 1e-12 or n == 0 and err == 0.0, (n, err)
    for n in (1, w.N // 2, w.N):
        u, p = s.serial_fine(n)
        assert np.array_equal(to_np(u), to_np(au[n]))
        assert np.array_equal(to_np(p), to_np(ap[n]))
    s.close()


@pytest.mark.parametrize("case", ["2d", "2d_ragged"])
def test_forced_algorithm3_matches_oracle(case):
    K = 2
    w, _, _, _, fo, s, Q = _setup(case, K=K)
    s.run(K)
    ref = O.theta_parareal(Q, w.c, w.u0, w.p0, K, forcing=fo)
    gates, spread = derived_gates(Q, w, w.u0, w.p0, K, ref, forcing=fo)
    _, ranks = s.residuals()
    assert list(ranks) == list(ref.rank)
    worst = np.zeros(3)
    for n in range(1, w.N + 1):
        u, p = s.state(n)
        worst = np.maximum(worst, state_errors(to_np(u), to_np(p), ref.u[n],
                                               ref.p[n], w.c, Q.dx_fine))
    print(f"forced Algorithm 3 {case}: worst {worst} gates {gates}", flush=True)
    assert np.all(worst < gates), (worst, gates)
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("case", list(CASES))
def test_record_matches_oracle(case, prec):
    """The record of one more sweep from the same slice starts: the
    oracle's iterate injected into the GPU (pw_set_iterate)."""
    dtype, comp = ("f64", False) if prec == "f64" else ("f32", True)
    w, rec, _, _, fo, s, Q = _setup(case, K=1, dtype=dtype, comp=comp)
    ref = O.theta_parareal(Q, w.c, w.u0, w.p0, 1, forcing=fo)
    us, ps = list(ref.u), list(ref.p)
    if dtype == "f32":
        us = [x.astype(np.float32).astype(np.float64) for x in us]
        ps = [x.astype(np.float32).astype(np.float64) for x in ps]
    s.run(1)
    for n in range(1, w.N + 1):
        s.set_iterate(n, us[n], ps[n])
    got = to_np(s.trace_sweep(rec))
    want = A.sweep_traces(Q, w.c * w.c, us, ps, rec, fo)
    assert got.shape == want.shape == (w.N, w.m_fine, rec.size)
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"record {case} {prec}: {err:.3g}", flush=True)
    assert err < (1e-12 if prec == "f64" else 1e-5), err
    s.close()


def _oracle_gradient(w, rec, data, fo, Q, K):
    corr, cc = A.record_correctors(Q, w.c, w.u0, w.p0, max(K, 1), forcing=fo)
    J, g = A.gradient(Q, w.c * w.c, w.u0, w.p0, K, corr, cc, rec, data,
                      forcing=fo, traces="sweep")
    u, p = A.forward_frozen(Q, w.c * w.c, w.u0, w.p0, K, corr, cc, forcing=fo)
    tr = A.sweep_traces(Q, w.c * w.c, u, p, rec, fo)
    # rounding sensitivity of the record (frozen correctors): a 1e-13
    # relative perturbation of u0, and correctors fitted to the columns in
    # the opposite order
    eps = 1e-13
    rng = np.random.default_rng(11)
    u1 = w.u0 * (1 + eps * rng.standard_normal(w.shape))
    v, vp = A.forward_frozen(Q, w.c * w.c, u1, w.p0, K, corr, cc, forcing=fo)
    amp = np.abs(A.sweep_traces(Q, w.c * w.c, v, vp, rec, fo) - tr).max() / eps
    res2 = O.theta_parareal(Q, w.c, w.u0, w.p0, max(K, 1),
                            record_correctors=True, forcing=fo,
                            sample_cols=[np.arange(w.N)[::-1]] * max(K, 1))
    v2, vp2 = A.forward_frozen(Q, w.c * w.c, w.u0, w.p0, K, res2.correctors,
                               cc, forcing=fo)
    spread = np.abs(A.sweep_traces(Q, w.c * w.c, v2, vp2, rec, fo) - tr).max()
    gate = max(1e-12 * np.abs(tr).max(), 256 * amp * 2.0 ** -52, 16 * spread)
    return J, g, tr, gate


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("K", [0, 2])
def test_record_gradient_matches_oracle_adjoint(case, K):
    w, rec, data, _, fo, s, Q = _setup(case, K=K)
    print(f"forced adjoint {case} K={K} shape={w.shape}", flush=True)
    s.run_taped(K)
    tr = to_np(s.trace_sweep(rec))
    J_ref, g_ref, tr_ref, gate = _oracle_gradient(w, rec, data, fo, Q, K)
    np.testing.assert_allclose(tr, tr_ref, rtol=0, atol=gate)
    seed = Q.dt_fine * (tr - data)
    J = 0.5 * Q.dt_fine * float(np.sum((tr - data) ** 2))
    assert J == pytest.approx(J_ref, rel=1e-10)
    g = to_np(s.backward_sweep(rec, seed, wrt="c2"))
    err = np.abs(g - g_ref).max()
    print(f"  gradient err {err:.3g} of {np.abs(g_ref).max():.3g}", flush=True)
    assert err <= 1e-8 * np.abs(g_ref).max(), (err, np.abs(g_ref).max())
    gc = to_np(s.backward_sweep(rec, seed, wrt="c"))
    np.testing.assert_allclose(gc, 2 * w.c * g, rtol=1e-14, atol=0)
    s.close()


def test_coupling_time_gradient_with_forcing_matches_oracle():
    """pw_backward (the record at the coupling times) with the layer and
    source."""
    K = 2
    w, rec, data, _, fo, s, Q = _setup("2d_ragged", K=K)
    data = data[:, -1, :]
    s.run_taped(K)
    tr = to_np(s.traces(rec))
    corr, cc = A.record_correctors(Q, w.c, w.u0, w.p0, K, forcing=fo)
    J_ref, g_ref = A.gradient(Q, w.c * w.c, w.u0, w.p0, K, corr, cc, rec, data,
                              forcing=fo, traces="coupling")
    J = 0.5 * float(np.sum((tr - data) ** 2))
    assert J == pytest.approx(J_ref, rel=1e-10)
    g = to_np(s.backward(rec, tr - data, wrt="c2"))
    err = np.abs(g - g_ref).max()
    assert err <= 1e-8 * np.abs(g_ref).max(), (err, np.abs(g_ref).max())
    s.close()


@pytest.mark.parametrize("case", ["2d_ragged", "2d_stream"])
def test_record_gradient_finite_differences_and_checkpoints(case):
    """Central differences of the GPU's own frozen forward (pw_run_frozen +
    pw_trace_sweep) against pw_backward_sweep, and the gradient's
    independence of the checkpoint interval."""
    import torch
    K = 2
    w, rec, data, _, _, s, Q = _setup(case, K=K)
    s.run_taped(K)
    tr = to_np(s.trace_sweep(rec))
    seed = Q.dt_fine * (tr - data)
    g = to_np(s.backward_sweep(rec, seed, checkpoint_every=64))
    for ck in (1, 5):
        assert np.array_equal(to_np(s.backward_sweep(rec, seed,
                                                     checkpoint_every=ck)), g)
    rng = np.random.default_rng(2)
    ny, nx = w.shape
    Y, X = np.meshgrid(np.arange(ny) / nx, np.arange(nx) / nx, indexing="ij")
    e = np.cos(2 * np.pi * (2 * X + Y) + 0.7) + 0.3 * rng.standard_normal(w.shape)
    eps = 1e-5

    def J_at(c2):
        s.set_medium(torch.tensor(np.sqrt(c2), device="cuda"))
        s.run_frozen(K)
        r = to_np(s.trace_sweep(rec))
        return 0.5 * Q.dt_fine * float(np.sum((r - data) ** 2))

    c2 = w.c * w.c
    fd = (J_at(c2 + eps * e) - J_at(c2 - eps * e)) / (2 * eps)
    ad = float(np.sum(g * e))
    assert ad == pytest.approx(fd, rel=1e-6), (ad, fd)
    s.close()


def test_autograd_record_function():
    import torch

    import paper_1905_00473_amd as pw
    K = 1
    w, rec, data, _, _, s, Q = _setup("2d", K=K)
    c = torch.tensor(w.c, device="cuda", requires_grad=True)
    r = pw.PararealRecord.apply(c, s, rec, K)
    d = torch.tensor(data, device="cuda")
    J = 0.5 * Q.dt_fine * ((r - d) ** 2).sum()
    J.backward()
    g = to_np(s.backward_sweep(rec, Q.dt_fine * (to_np(r) - data), wrt="c"))
    np.testing.assert_allclose(to_np(c.grad), g, rtol=1e-13, atol=0)
    s.close()


def test_forcing_argument_errors():
    import paper_1905_00473_amd as pw
    w, rec, _, fd, _, s, _ = _setup("2d")
    with pytest.raises(pw.PwError, match="positive finite frequency"):
        s.set_source(fd["src_pos"], freq=0.0)
    s.set_source(fd["src_pos"], fd["freq"], fd["t0"])
    s.run(1)
    dup = np.array([rec[0], rec[0]])
    with pytest.raises(pw.PwError, match="distinct"):
        s.trace_sweep(dup)
    s.set_variant("no_correction")
    with pytest.raises(pw.PwError, match="source"):
        s.run(1)
    s.set_variant("theta")
    with pytest.raises(pw.PwError, match="batched runs"):
        s.run_batch(1)
    s.close()
    P1 = pw.Problem.make((64,), 4, 0.25, 4, 8, 2)
    s1 = pw.Solver(P1)
    with pytest.raises(pw.PwError, match="2D problems only"):
        s1.set_source((0.3,), 10.0, 0.1)
    s1.close()
