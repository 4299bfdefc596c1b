"""Shared helpers of the GPU parity tests: build a solver and the matching
oracle problem from one seeded workload."""

import contextlib
import math
import os

import numpy as np

import oracle as O


def problem_pair(w, max_iters=None, tol=None, dtype=None, compensated=None,
                 interp="trig"):
    """(pw.Problem, oracle.Problem) for a workloads.Workload."""
    import paper_1905_00473_amd as pw
    dt = dtype or w.dtype
    comp = w.compensated if compensated is None else compensated
    t = w.tol if tol is None else tol
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, t, dt, comp and dt == "f32",
                        max_iters or w.K, interp)
    Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                  w.grad_order, t, interp=interp)
    return P, Q


def inputs_as(w, dtype):
    """Initial state rounded to the state dtype (so both sides start from
    the same numbers), returned as float64 arrays."""
    if dtype == "f32":
        return (w.u0.astype(np.float32).astype(np.float64),
                w.p0.astype(np.float32).astype(np.float64))
    return w.u0.copy(), w.p0.copy()


def rel_energy_err(u, p, ur, pr, c, dx, order=4):
    """sqrt(E(u - ur) / E(ur)) on the fine grid (Sec. 6 error measure)."""
    e = O.energy(u - ur, p - pr, c, dx, order)
    e0 = O.energy(ur, pr, c, dx, order)
    return math.sqrt(e / e0) if e0 > 0 else math.sqrt(e)


def to_np(t):
    return t.detach().double().cpu().numpy()


def amplification(Q, w, u0, p0, K, **oracle_kwargs):
    """Sensitivity of the iteration to rounding: max over slices of the
    relative energy-norm change caused by a 1e-13 relative perturbation of
    u0, divided by 1e-13 (oracle only)."""
    eps = 1e-13
    rng = np.random.default_rng(7)
    ref = O.theta_parareal(Q, w.c, u0, p0, K, **oracle_kwargs)
    u1 = u0 * (1 + eps * rng.standard_normal(np.shape(u0)))
    r1 = O.theta_parareal(Q, w.c, u1, p0, K, **oracle_kwargs)
    return max(rel_energy_err(r1.u[n], r1.p[n], ref.u[n], ref.p[n], w.c,
                              Q.dx_fine) for n in range(1, Q.N + 1)) / eps


def ordering_spread(Q, w, u0, p0, K, **oracle_kwargs):
    """Sensitivity of Algorithm 1 to the order of its data columns: max
    over slices of the relative energy-norm difference between two oracle
    runs that pass the columns of every iteration in opposite orders (the
    same exact arithmetic, two roundings; zero for the iterations without
    a fitted corrector)."""
    if oracle_kwargs.get("omega", "procrustes") != "procrustes":
        return 0.0
    kw = dict(oracle_kwargs)
    cols = kw.pop("sample_cols", None)
    if cols is None:
        cols = [np.arange(Q.N)] * K
    fwd = [np.asarray(c) for c in cols]
    rev = [c[::-1].copy() for c in fwd]
    a = O.theta_parareal(Q, w.c, u0, p0, K, sample_cols=fwd, **kw)
    b = O.theta_parareal(Q, w.c, u0, p0, K, sample_cols=rev, **kw)
    return max(rel_energy_err(b.u[n], b.p[n], a.u[n], a.p[n], w.c,
                              Q.dx_fine) for n in range(1, Q.N + 1))


def derived_gate(Q, w, u0, p0, K, floor=1e-12, **oracle_kwargs):
    """max(floor, 256 A eps, 16 S): A the amplification above, eps =
    2^-52; 256 covers the rounding injected at every stage of every
    iteration (fine and coarse sweeps, QR, SVD, recurrence: of the order
    of a hundred injections of relative size eps) rather than at the input
    only; S the column-order spread of Algorithm 1 above (the GPU's
    reductions are one more ordering of the same arithmetic)."""
    return max(floor,
               256 * amplification(Q, w, u0, p0, K, **oracle_kwargs)
               * 2.0 ** -52,
               16 * ordering_spread(Q, w, u0, p0, K, **oracle_kwargs))


def state_errors(u, p, ur, pr, c, dx, order=4):
    """(energy, l2, max) relative differences of a state against a
    reference: the Sec. 6 energy norm (blind to a constant shift of u), the
    l2 norm of the displacement and its largest pointwise difference
    relative to the largest reference value."""
    e = rel_energy_err(u, p, ur, pr, c, dx, order)
    l2 = O.l2_error(u, ur)
    m = float(np.max(np.abs(u - ur)) / max(np.max(np.abs(ur)), 1e-300))
    return e, l2, m


@contextlib.contextmanager
def oracle_pool(n=None):
    """The parfor of Algorithm 3 for the oracle: a process pool (started by
    a fork server, so the workers hold no GPU state) whose starmap runs the
    oracle's propagate on all slices of an iteration at once."""
    import multiprocessing as mp
    n = n or max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("forkserver")
    with ctx.Pool(n) as pool:
        yield pool.starmap


def derived_gates(Q, w, u0, p0, K, ref, pmap=None, floor=1e-12,
                  **oracle_kwargs):
    """Per-norm gates (energy, l2, max; see state_errors) for an FP64
    end-to-end comparison, each max(floor, 256 A eps, 16 S, 16 D, 16 L)
    with, from four more oracle runs:
    A  the amplification of a perturbation of u0 of relative size 1e-13,
       random per point plus a constant shift of 1e-13 max|u0| (rounding
       reaches every component, the mean included, which the energy norm
       does not see but l2 does);
    S  the spread of Algorithm 1 over the order of its data columns;
    D  the spread over the SVD routine of Algorithm 1 (LAPACK's QR-iteration
       driver in place of divide and conquer): both drivers are backward
       stable, so D is how far a correct SVD may move the iteration through
       the singular directions the truncation keeps but the data determine
       only to eps sigma_1 / sigma_i;
    L  the spread over the form of the correction: Omega and Lambda^dag
       applied to each of its two terms (Algorithm 3 as written) or once to
       their difference, with the mean of the difference (the GPU's form):
       in the two-term form the mean is a difference of two large sums.
    ``ref`` is the oracle run the GPU is compared with."""
    import functools

    import scipy.linalg
    eps_in = 1e-13
    rng = np.random.default_rng(7)
    u1 = u0 * (1 + eps_in * rng.standard_normal(np.shape(u0))) \
        + eps_in * float(np.max(np.abs(u0)))
    runs = {"A": O.theta_parareal(Q, w.c, u1, p0, K, pmap=pmap,
                                  **oracle_kwargs)}
    cols = [np.arange(Q.N)[::-1].copy() for _ in range(K)]
    runs["S"] = O.theta_parareal(Q, w.c, u0, p0, K, pmap=pmap,
                                 sample_cols=cols, **oracle_kwargs)
    svd = functools.partial(scipy.linalg.svd, lapack_driver="gesvd")
    runs["D"] = O.theta_parareal(Q, w.c, u0, p0, K, pmap=pmap, svd=svd,
                                 **oracle_kwargs)
    runs["L"] = O.theta_parareal(Q, w.c, u0, p0, K, pmap=pmap,
                                 sweep="difference", **oracle_kwargs)
    spread = {}
    for key, r in runs.items():
        spread[key] = np.max([state_errors(r.u[n], r.p[n], ref.u[n], ref.p[n],
                                           w.c, Q.dx_fine)
                              for n in range(1, Q.N + 1)], axis=0)
    gates = np.maximum.reduce([np.full(3, floor),
                               256 * spread["A"] / eps_in * 2.0 ** -52,
                               16 * spread["S"], 16 * spread["D"],
                               16 * spread["L"]])
    return gates, spread
