"""End-to-end parity of the benchmarked solves with the FP64 oracle.

The oracle runs Algorithm 3 step by step (tests/gpu_helpers.oracle_pool
farms the fine propagations of each iteration out to host processes, the
parfor of Algorithm 3; every other step runs in order in the test process).
Every expected value comes from oracle/; the GPU path is compared with it
slice by slice in the energy norm of the Sec. 6 preamble, and also in the
l2 norm of the displacement and pointwise (the energy is blind to a
constant shift of u).

Configurations and gates:
* disc2d at its benchmark size (512^2 / 128^2, N = 64, K = 8, svd tol
  1e-13), FP32 compensated state: every slice of every iterate k = 1..9
  within 1e-5 of the oracle run on the same FP32-rounded initial data
  (energy, l2 and max norms).
* the same solve with FP64 state, one iteration resumed from the oracle's
  own iterate u^k and corrector Omega^k (pw_set_iterate, pw_set_corrector,
  pw_continue with the corrector held): 1e-12 (this pins the rounding of
  one iteration -- F, C, the data restriction, the corrected sweep and the
  update -- independently of how Algorithm 1's rounding is amplified over
  iterations).
* disc2d at full size (K = 4) and layers3d at the reduced size 64^3 /
  16^3 (N = 32, K = 6), FP64 state, svd tol 1e-3 (Omega well
  determined): end to end in the energy and l2 norms at the gates of
  tests/gpu_helpers.derived_gates, per norm max(1e-12, 256 A eps, 16 S,
  16 D, 16 L) from four more oracle runs (input perturbation, column order,
  SVD driver, one-term form of the correction); the pointwise maximum is
  reported and bounded by 1e-10; layers3d FP64 at its run
  tol 1e-13 one iteration from the oracle's iterate and corrector, 1e-12;
  the layers3d FP32 compensated solve at tol 1e-13 within 1e-5 (energy,
  l2; pointwise 3e-5).
* layers3d at full size 256^3: F over one whole slice (76 steps) on two
  states of the coarse initialisation, FP32 compensated, 1e-5.
* the batched solve of four uneven 2D problems (grf2d recipe), K = 6,
  FP32 compensated: 1e-5 per slice of every problem.
"""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import (derived_gates, inputs_as, oracle_pool,
                               problem_pair, state_errors, to_np)

pytestmark = pytest.mark.gpu

_CACHE = {}


def _disc2d_oracle(tol, K):
    """Oracle run of the disc2d benchmark workload (FP32-rounded inputs),
    with every iterate and the corrector of every iteration."""
    key = ("disc2d", tol, K)
    if key not in _CACHE:
        w = W.disc2d()
        Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                      w.grad_order, tol)
        u0, p0 = inputs_as(w, "f32")
        print(f"oracle: disc2d {w.shape} N={w.N} K={K} tol={tol}", flush=True)
        with oracle_pool() as pm:
            ref = O.theta_parareal(Q, w.c, u0, p0, K, keep_history=True,
                                   record_correctors=True, pmap=pm)
        _CACHE[key] = (w, Q, u0, p0, ref)
    return _CACHE[key]


def _solver(w, Q, u0, p0, K, dtype, tol, keep_history=False):
    import paper_1905_00473_amd as pw
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, tol, dtype, dtype == "f32", K,
                        keep_history=keep_history)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    return s


@pytest.mark.timeout(900)
def test_disc2d_fullsize_fp32_every_iterate():
    w, Q, u0, p0, ref = _disc2d_oracle(1e-13, 8)
    s = _solver(w, Q, u0, p0, 8, "f32", 1e-13, keep_history=True)
    print("gpu: disc2d FP32 compensated K=8", flush=True)
    assert s.run(8) == 8
    worst = np.zeros(3)
    for k in range(1, 10):
        hu, hp = ref.history[k - 1]
        for n in range(1, w.N + 1):
            u, p = s.iterate(k, n)
            e = state_errors(to_np(u), to_np(p), hu[n], hp[n], w.c, Q.dx_fine)
            assert max(e) < 1e-5, (k, n, e)
            worst = np.maximum(worst, e)
    print(f"disc2d FP32 vs oracle, worst (energy, l2, max) = {worst}",
          flush=True)
    rho, rk = s.residuals()
    assert rk == ref.rank, (rk, ref.rank)
    # the residual of FP32 data carries the FP32 rounding of F (6e-8
    # relative) and its Omega-action the ill-determined directions of a
    # corrector truncated at 1e-13: a percent-level agreement only
    np.testing.assert_allclose(rho, ref.rho, rtol=5e-2)
    s.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("k", [1, 4, 7])
def test_disc2d_fullsize_fp64_one_iteration_from_oracle_state(k):
    """u^{k+1} from the oracle's u^k and Omega^k in one GPU iteration."""
    import paper_1905_00473_amd as pw
    w, Q, u0, p0, ref = _disc2d_oracle(1e-13, 8)
    s = _solver(w, Q, u0, p0, 8, "f64", 1e-13)
    s.run(k - 1)                      # any state: it is overwritten below
    hu, hp = ref.history[k - 1]      # u^k
    for n in range(1, w.N + 1):
        s.set_iterate(n, hu[n], hp[n])
    U, V = ref.correctors[k - 1]      # Omega^k (after iteration k's update)
    S = ref.sigma[k - 1]
    s.set_corrector(np.ascontiguousarray(U.T), S, np.ascontiguousarray(V.T))
    Ug, Sg, Vg = s.corrector()
    assert np.array_equal(to_np(Ug), U.T) and np.array_equal(to_np(Sg), S)
    print(f"gpu: disc2d FP64 one iteration from the oracle's u^{k}, "
          f"rank {len(S)}", flush=True)
    assert s.resume(1, update_corrector=False) == k
    nu, npp = ref.history[k]          # u^{k+1}
    worst = np.zeros(3)
    for n in range(1, w.N + 1):
        u, p = s.state(n)
        e = state_errors(to_np(u), to_np(p), nu[n], npp[n], w.c, Q.dx_fine)
        worst = np.maximum(worst, e)
    print(f"k={k}: worst (energy, l2, max) = {worst}", flush=True)
    assert worst.max() < 1e-12, worst
    s.close()
    assert isinstance(pw.DIAG_FIELDS, tuple)


@pytest.mark.timeout(900)
def test_disc2d_fullsize_fp64_end_to_end_tol_1e3():
    w, Q, u0, p0, ref = _disc2d_oracle(1e-3, 4)
    s = _solver(w, Q, u0, p0, 4, "f64", 1e-3)
    print("gpu: disc2d FP64 tol 1e-3 K=4", flush=True)
    s.run(4)
    worst = np.zeros(3)
    for n in range(1, w.N + 1):
        u, p = s.state(n)
        e = state_errors(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                         Q.dx_fine)
        worst = np.maximum(worst, e)
    with oracle_pool() as pm:
        gates, spread = derived_gates(Q, w, u0, p0, 4, ref, pmap=pm)
    print(f"disc2d FP64 tol 1e-3: worst (energy, l2, max) = {worst}, "
          f"gates {gates}, spreads {spread}", flush=True)
    assert np.all(worst[:2] < gates[:2]), (worst, gates)
    assert worst[2] < 1e-10, worst
    rho, rk = s.residuals()
    assert rk == ref.rank
    np.testing.assert_allclose(rho, ref.rho, rtol=1e-9)
    d = s.diagnostics()
    for kk in range(4):
        f2, fin2, gin2 = ref.data_norms[kk]
        assert abs(d[kk]["F2"] - f2) <= 1e-12 * f2
        assert abs(d[kk]["F_in2"] - fin2) <= 1e-12 * fin2
        assert abs(d[kk]["G_in2"] - gin2) <= 1e-12 * gin2
        trs = float(np.sum(ref.sigma[kk]))
        assert abs(d[kk]["trace_S"] - trs) <= 1e-12 * trs
        tot = sum(a[1] + a[2] for a in ref.data_norms[:kk + 1])
        r2 = tot - 2 * trs
        assert abs(d[kk]["r2_min"] - r2) <= 1e-12 * tot
    s.close()


def _layers_small():
    return W.layers3d(n=64, ratio=4, N=32, K=6, T=1.5)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-13), ("f64", 1e-3)])
def test_layers3d_reduced_end_to_end(dtype, tol):
    """FP32 compensated at the workload's svd tol (1e-13) within 1e-5; FP64
    at svd tol 1e-3, where Omega is well determined, within the derived
    gates (at the run tol the FP64 iteration is pinned one iteration at a
    time by the next test)."""
    import paper_1905_00473_amd as pw
    w = _layers_small()
    K = w.K
    P, Q = problem_pair(w, max_iters=K, dtype=dtype, tol=tol,
                        compensated=dtype == "f32")
    u0, p0 = inputs_as(w, dtype)
    print(f"layers3d {w.shape} N={w.N} K={K} {dtype} tol {tol}", flush=True)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    s.run(K)
    with oracle_pool() as pm:
        ref = O.theta_parareal(Q, w.c, u0, p0, K, pmap=pm)
        if dtype == "f32":
            # the FP32 bar is 1e-5 in the energy norm (and l2); the largest
            # pointwise difference, relative to the largest value, carries
            # the rounding where the field is largest: 3e-5
            gates, spread = np.array([1e-5, 1e-5, 3e-5]), None
        else:
            gates, spread = derived_gates(Q, w, u0, p0, K, ref, pmap=pm)
    worst = np.zeros(3)
    for n in range(1, w.N + 1):
        u, p = s.state(n)
        e = state_errors(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                         Q.dx_fine)
        worst = np.maximum(worst, e)
    print(f"layers3d {dtype}: worst (energy, l2, max) = {worst}, "
          f"gates {gates}, spreads {spread}", flush=True)
    assert np.all(worst[:2] < gates[:2]), (worst, gates)
    assert worst[2] < (3e-5 if dtype == "f32" else 1e-10), worst
    s.close()


@pytest.mark.timeout(900)
def test_layers3d_reduced_fp64_one_iteration_from_oracle_state():
    """At the run tol 1e-13: u^4 from the oracle's u^3 and Omega^3 in one
    GPU iteration, within 1e-12."""
    import paper_1905_00473_amd as pw
    w = _layers_small()
    P, Q = problem_pair(w, max_iters=4, dtype="f64", compensated=False)
    u0, p0 = inputs_as(w, "f64")
    with oracle_pool() as pm:
        ref = O.theta_parareal(Q, w.c, u0, p0, 3, keep_history=True,
                               record_correctors=True, pmap=pm)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    s.run(2)
    hu, hp = ref.history[2]
    for n in range(1, w.N + 1):
        s.set_iterate(n, hu[n], hp[n])
    U, V = ref.correctors[2]
    s.set_corrector(np.ascontiguousarray(U.T), ref.sigma[2],
                    np.ascontiguousarray(V.T))
    assert s.resume(1, update_corrector=False) == 3
    worst = np.zeros(3)
    for n in range(1, w.N + 1):
        u, p = s.state(n)
        e = state_errors(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                         Q.dx_fine)
        worst = np.maximum(worst, e)
    print(f"layers3d one iteration: worst (energy, l2, max) = {worst}",
          flush=True)
    assert worst.max() < 1e-12, worst
    s.close()


@pytest.mark.timeout(900)
def test_layers3d_fullsize_one_slice_of_F():
    import torch
    w = W.layers3d()
    P, Q = problem_pair(w, max_iters=1)
    import paper_1905_00473_amd as pw
    u0, p0 = inputs_as(w, "f32")
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(u0, p0)
    s.run(0)
    # two states of the coarse initialisation: slices 8 and 24
    picks = [8, 24]
    us, ps = zip(*[s.state(n) for n in picks])
    u = torch.stack(us).contiguous()
    p = torch.stack(ps).contiguous()
    print(f"layers3d full: F ({w.m_fine} steps of {w.shape}) on 2 states",
          flush=True)
    uo, po = s.propagate(u, p)
    # the FP32 path propagates with c^2 rounded once to FP32
    c2 = (w.c * w.c).astype(np.float32).astype(np.float64)
    h = Q.dt_fine
    args = [(to_np(u[i]), to_np(p[i]), c2, h, Q.dx_fine, w.m_fine)
            for i in range(2)]
    with oracle_pool(2) as pm:
        out = list(pm(O.propagate, args))
    for i in range(2):
        e = state_errors(to_np(uo[i]), to_np(po[i]), out[i][0], out[i][1],
                         w.c, Q.dx_fine)
        print(f"slice {picks[i]}: (energy, l2, max) = {e}", flush=True)
        assert max(e) < 1e-5, e
    s.close()


@pytest.mark.timeout(900)
def test_batch_four_uneven_problems_K6():
    import paper_1905_00473_amd as pw
    ws = [W.grf2d(n=n, ratio=4, N=8, K=6, T=0.5, seed=b, dtype="f32",
                  compensated=True)
          for b, n in enumerate([64, 96, 128, 80])]
    K = 6
    probs, Qs = [], []
    for w in ws:
        P, Q = problem_pair(w, max_iters=K)
        probs.append(P)
        Qs.append(Q)
    s = pw.Solver(probs)
    ins = []
    for i, w in enumerate(ws):
        u0, p0 = inputs_as(w, "f32")
        ins.append((u0, p0))
        s.set_medium(w.c, prob=i)
        s.set_initial(u0, p0, prob=i)
    print("batch of 4 uneven problems, K=6", flush=True)
    s.run_batch(K)
    for i, w in enumerate(ws):
        ref = O.theta_parareal(Qs[i], w.c, ins[i][0], ins[i][1], K)
        worst = np.zeros(3)
        for n in range(1, w.N + 1):
            u, p = s.state(n, prob=i)
            e = state_errors(to_np(u), to_np(p), ref.u[n], ref.p[n], w.c,
                             Qs[i].dx_fine)
            worst = np.maximum(worst, e)
        print(f"problem {i} {w.shape}: worst {worst}", flush=True)
        assert worst.max() < 1e-5, (i, worst)
        rho, rk = s.residuals(prob=i)
        assert rk == ref.rank
    s.close()
