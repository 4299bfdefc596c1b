"""Shared helpers of the GPU parity tests: build a solver and the matching
oracle problem from one seeded workload."""

import math

import numpy as np

import oracle as O


def problem_pair(w, max_iters=None, tol=None, dtype=None, compensated=None):
    """(pw.Problem, oracle.Problem) for a workloads.Workload."""
    import paper_1905_00473_amd as pw
    dt = dtype or w.dtype
    comp = w.compensated if compensated is None else compensated
    t = w.tol if tol is None else tol
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, t, dt, comp and dt == "f32",
                        max_iters or w.K)
    Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                  w.grad_order, t)
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
