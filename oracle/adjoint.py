"""FP64 oracle of the misfit gradient d J / d c^2 through Algorithm 3 with the
phase corrector held fixed.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Misfit: receivers are fine-grid nodes x_r, data d_{n,r} are given at the
coupling times t_n, n = 1..N, and

    J(c^2) = 1/2 sum_{n=1..N} sum_r (u^{K+1}_n(x_r) - d_{n,r})^2 ,

where u^{K+1}_n is the iterate of Algorithm 3 after K iterations.  The
medium enters the fine propagator (c^2 on the fine grid) and the coarse
propagator (its pointwise restriction).  The corrector of each iteration,
theta^k = I Lambda^dag Omega^k Lambda of eq. thetarelation, is recorded in
a first run and then held fixed (Omega^k and the c inside Lambda and
Lambda^dag): the gradient is that of the map c^2 -> J with theta^k frozen,
the reading under which the SVD of Algorithm 1 is not differentiated.

The adjoint is written by hand in reverse order of the forward steps:
velocity Verlet reversed step by step (every forward state is stored: the
sizes here are small), the transposes of R (scatter), I (the transpose of
the separable interpolation matrices) and theta^k (the transpose of its
dense matrix).  Pinned by finite differences of the same frozen forward
(tests/test_oracle_adjoint.py).
"""

from __future__ import annotations

import numpy as np

from . import wave as O

__all__ = ["record_correctors", "forward_frozen", "misfit", "gradient",
           "theta_matrix"]


def record_correctors(prob, c, u0, p0, K, sample_cols=None):
    """Run Algorithm 3 once and return the correctors [(U_k, V_k)] and the
    coarse medium used inside Lambda / Lambda^dag (``sample_cols``: the
    subsampling table of the run, see theta_parareal)."""
    res = O.theta_parareal(prob, c, u0, p0, K, record_correctors=True,
                           sample_cols=sample_cols)
    return res.correctors, O.restrict(np.asarray(c, float), prob.ratio)


def _theta(W, Wp, UV, cc, prob):
    """theta = Lambda^dag Omega Lambda on the coarse grid (the part of
    theta^k before I), with the DC term sum(W) of the input."""
    U, V = UV
    z = O.energy_components(W, Wp, cc, prob.dx_coarse, prob.grad_order)
    y = U @ (V.T @ z)
    q, pq = O.split_components(y, prob.coarse_shape)
    return O.grad2func(q, W.sum(), prob.dx_coarse), cc * pq


def theta_matrix(UV, cc, prob):
    """Dense matrix of the coarse map (W, Wp) -> theta(W, Wp) acting on the
    stacked vector [W.ravel(); Wp.ravel()]."""
    cs = prob.coarse_shape
    nc = int(np.prod(cs))
    T = np.zeros((2 * nc, 2 * nc))
    for j in range(2 * nc):
        e = np.zeros(2 * nc)
        e[j] = 1.0
        a, b = _theta(e[:nc].reshape(cs), e[nc:].reshape(cs), UV, cc, prob)
        T[:nc, j] = a.ravel()
        T[nc:, j] = b.ravel()
    return T


def _prop_store(u, p, c2, h, dx, m):
    """velocity Verlet keeping the displacement at every step start."""
    us = [np.array(u, float)]
    u, p = np.array(u, float), np.array(p, float)
    for _ in range(m):
        u, p = O.vv_step(u, p, c2, h, dx)
        us.append(u)
    return u, p, us


def _prop_adjoint(us, lu, lp, c2, h, dx):
    """Reverse of m velocity-Verlet steps: given the adjoint (lu, lp) of the
    output and the displacements us[0..m], return the adjoint of the input
    and d J / d c^2 accumulated over the steps."""
    g = np.zeros_like(lu)
    lu, lp = lu.copy(), lp.copy()
    for i in range(len(us) - 1, 0, -1):
        # p2 = p1 + h/2 c^2 Lap u_i   (second half kick, u_i = us[i])
        lu = lu + 0.5 * h * O.laplacian(c2 * lp, dx)
        g += 0.5 * h * lp * O.laplacian(us[i], dx)
        # u_i = u_{i-1} + h p1
        lp = lp + h * lu
        # p1 = p0 + h/2 c^2 Lap u_{i-1}
        lu = lu + 0.5 * h * O.laplacian(c2 * lp, dx)
        g += 0.5 * h * lp * O.laplacian(us[i - 1], dx)
    return lu, lp, g


def _interp_matrix(nc, ratio):
    A = np.zeros((nc * ratio, nc))
    for j in range(nc):
        e = np.zeros(nc)
        e[j] = 1.0
        A[:, j] = O.interp(e, ratio)
    return A


def _interp_T(y, ratio, cshape):
    """Transpose of the separable interpolation I applied to a fine field."""
    out = np.asarray(y, float)
    for ax in range(out.ndim):
        A = _interp_matrix(cshape[ax], ratio)
        out = np.moveaxis(np.tensordot(A.T, np.moveaxis(out, ax, 0), axes=1),
                          0, ax)
    return out


def _restrict_T(Y, ratio, fshape):
    out = np.zeros(fshape)
    sl = tuple(slice(None, None, ratio) for _ in fshape)
    out[sl] = Y
    return out


def forward_frozen(prob, c2f, u0, p0, K, correctors, cc_theta, store=False):
    """Algorithm 3 with the recorded correctors theta^k (literal sweep).
    Returns the final iterates (lists over n) and, with store=True, the
    intermediate quantities the adjoint needs."""
    r, N = prob.ratio, prob.N
    c2f = np.asarray(c2f, float)
    c2c = O.restrict(c2f, r)
    hf, hc = prob.dt_fine, prob.dt_coarse
    dxf, dxc = prob.dx_fine, prob.dx_coarse
    tape = {"init": [], "iters": []}
    u = [np.array(u0, float)] + [None] * N
    p = [np.array(p0, float)] + [None] * N
    W, Wp = O.restrict(u[0], r), O.restrict(p[0], r)
    for n in range(1, N + 1):
        W2, Wp2, us = _prop_store(W, Wp, c2c, hc, dxc, prob.m_coarse)
        tape["init"].append(us)
        u[n], p[n] = O.interp(W2, r), O.interp(Wp2, r)
        W, Wp = O.restrict(u[n], r), O.restrict(p[n], r)
    for k in range(K):
        UV = correctors[k]
        it = {"F": [None] * (N + 1), "Cw": [None] * (N + 1),
              "Ct": [None] * (N + 1)}
        v, vp = [None] * (N + 1), [None] * (N + 1)
        for n in range(1, N + 1):
            v[n], vp[n], it["F"][n] = _prop_store(u[n - 1], p[n - 1], c2f,
                                                  hf, dxf, prob.m_fine)
        un, pn = [u[0]] + [None] * N, [p[0]] + [None] * N
        for n in range(1, N + 1):
            w, wp, it["Cw"][n] = _prop_store(O.restrict(un[n - 1], r),
                                             O.restrict(pn[n - 1], r), c2c,
                                             hc, dxc, prob.m_coarse)
            wt, wtp, it["Ct"][n] = _prop_store(O.restrict(u[n - 1], r),
                                               O.restrict(p[n - 1], r), c2c,
                                               hc, dxc, prob.m_coarse)
            a, b = _theta(w, wp, UV, cc_theta, prob)
            at, bt = _theta(wt, wtp, UV, cc_theta, prob)
            un[n] = v[n] + O.interp(a - at, r)
            pn[n] = vp[n] + O.interp(b - bt, r)
        tape["iters"].append(it)
        u, p = un, pn
    return (u, p, tape) if store else (u, p)


def misfit(u_list, receivers, data):
    """1/2 sum_{n>=1} sum_r (u_n(x_r) - d_{n,r})^2; receivers: flat fine
    indices, data: array (N, n_receivers)."""
    J = 0.0
    for n in range(1, len(u_list)):
        d = u_list[n].ravel()[receivers] - data[n - 1]
        J += 0.5 * float(d @ d)
    return J


def gradient(prob, c2f, u0, p0, K, correctors, cc_theta, receivers, data):
    """d J / d c^2 on the fine grid by the hand-written adjoint (frozen
    correctors).  Returns (J, grad)."""
    r, N = prob.ratio, prob.N
    fshape, cshape = prob.shape, prob.coarse_shape
    nc = int(np.prod(cshape))
    c2f = np.asarray(c2f, float)
    c2c = O.restrict(c2f, r)
    hf, hc = prob.dt_fine, prob.dt_coarse
    dxf, dxc = prob.dx_fine, prob.dx_coarse
    u, p, tape = forward_frozen(prob, c2f, u0, p0, K, correctors, cc_theta,
                                store=True)
    J = misfit(u, receivers, data)
    # seed: adjoint of u^{K+1}_n at the receivers
    lu = [np.zeros(fshape) for _ in range(N + 1)]
    lp = [np.zeros(fshape) for _ in range(N + 1)]
    for n in range(1, N + 1):
        d = u[n].ravel()[receivers] - data[n - 1]
        flat = lu[n].ravel()
        np.add.at(flat, receivers, d)
        lu[n] = flat.reshape(fshape)
    gf = np.zeros(fshape)
    gc = np.zeros(cshape)
    for k in range(K - 1, -1, -1):
        it = tape["iters"][k]
        Th = theta_matrix(correctors[k], cc_theta, prob)
        lu_old = [np.zeros(fshape) for _ in range(N + 1)]
        lp_old = [np.zeros(fshape) for _ in range(N + 1)]
        lv, lvp = [None] * (N + 1), [None] * (N + 1)
        # reverse sweep over n: un[n] = v[n] + I(theta(w_n) - theta(wt_n))
        carry_u = np.zeros(fshape)   # adjoint reaching un[n] from n+1
        carry_p = np.zeros(fshape)
        for n in range(N, 0, -1):
            Lu = lu[n] + carry_u
            Lp = lp[n] + carry_p
            lv[n], lvp[n] = Lu, Lp
            # adjoint of the correction theta(w) - theta(wt)
            y = np.concatenate([_interp_T(Lu, r, cshape).ravel(),
                                _interp_T(Lp, r, cshape).ravel()])
            z = Th.T @ y
            zu, zp = z[:nc].reshape(cshape), z[nc:].reshape(cshape)
            # w = C(R un[n-1]) : adjoint to un[n-1]
            au, ap, g1 = _prop_adjoint(it["Cw"][n], zu, zp, c2c, hc, dxc)
            # wt = C(R u[n-1]) (previous iterate), enters with a minus sign
            bu, bp, g2 = _prop_adjoint(it["Ct"][n], -zu, -zp, c2c, hc, dxc)
            gc += g1 + g2
            carry_u = _restrict_T(au, r, fshape)
            carry_p = _restrict_T(ap, r, fshape)
            lu_old[n - 1] += _restrict_T(bu, r, fshape)
            lp_old[n - 1] += _restrict_T(bp, r, fshape)
        # un[0] = u0 is fixed: carry into n = 0 is dropped
        # v[n] = F(u[n-1])
        for n in range(1, N + 1):
            a, b, g = _prop_adjoint(it["F"][n], lv[n], lvp[n], c2f, hf, dxf)
            gf += g
            lu_old[n - 1] += a
            lp_old[n - 1] += b
        lu, lp = lu_old, lp_old
    # initialisation: u^1_n = I C R u^1_{n-1}
    carry_u = np.zeros(cshape)
    carry_p = np.zeros(cshape)
    for n in range(N, 0, -1):
        Lu = _interp_T(lu[n], r, cshape) + carry_u
        Lp = _interp_T(lp[n], r, cshape) + carry_p
        au, ap, g = _prop_adjoint(tape["init"][n - 1], Lu, Lp, c2c, hc, dxc)
        gc += g
        # R I = 1: the restricted state R u^1_{n-1} is W_{n-1} itself
        carry_u, carry_p = au, ap
    gf += _restrict_T(gc, r, fshape)
    return J, gf
