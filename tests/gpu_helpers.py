"""Shared helpers of the GPU parity tests: build a solver and the matching
oracle problem from one seeded workload."""

import math

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
