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
           "theta_matrix", "sweep_traces", "sweep_misfit"]


def record_correctors(prob, c, u0, p0, K, sample_cols=None, forcing=None):
    """Run Algorithm 3 once and return the correctors [(U_k, V_k)] and the
    coarse medium used inside Lambda / Lambda^dag (``sample_cols``: the
    subsampling table of the run, see theta_parareal; ``forcing``: its
    layer and source)."""
    res = O.theta_parareal(prob, c, u0, p0, K, record_correctors=True,
                           sample_cols=sample_cols, forcing=forcing)
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


def _prop_store(u, p, c2, h, dx, m, damp=None, src=None, t_start=0.0):
    """velocity Verlet keeping the displacement at every step start; with a
    layer (damp) or a source (src) the steps of wave.propagate_forced,
    step j at time t_start + j h."""
    us = [np.array(u, float)]
    u, p = np.array(u, float), np.array(p, float)
    for j in range(m):
        if damp is None and src is None:
            u, p = O.vv_step(u, p, c2, h, dx)
        else:
            u, p = O.propagate_forced(u, p, c2, h, dx, 1, damp, src,
                                      t_start + j * h)
        us.append(u)
    return u, p, us


def _prop_adjoint(us, lu, lp, c2, h, dx, damp=None, seeds=None):
    """Reverse of m velocity-Verlet steps: given the adjoint (lu, lp) of the
    output and the displacements us[0..m], return the adjoint of the input
    and d J / d c^2 accumulated over the steps.  damp: the layer's factor
    exp(-sigma h / 2) of every half kick (a source adds a constant and
    drops out); seeds[i]: a field added to the adjoint of u_{i+1} (the
    derivative of J with respect to the displacement after step i + 1)."""
    g = np.zeros_like(lu)
    lu, lp = lu.copy(), lp.copy()
    for i in range(len(us) - 1, 0, -1):
        if seeds is not None:
            lu = lu + seeds[i - 1]
        # p2 = d p1 + h/2 (c^2 Lap u_i + f)   (second half kick, u_i = us[i])
        lu = lu + 0.5 * h * O.laplacian(c2 * lp, dx)
        g += 0.5 * h * lp * O.laplacian(us[i], dx)
        if damp is not None:
            lp = damp * lp
        # u_i = u_{i-1} + h p1
        lp = lp + h * lu
        # p1 = d p0 + h/2 (c^2 Lap u_{i-1} + f)
        lu = lu + 0.5 * h * O.laplacian(c2 * lp, dx)
        g += 0.5 * h * lp * O.laplacian(us[i - 1], dx)
        if damp is not None:
            lp = damp * lp
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


def _forcing(prob, c2f, forcing):
    """Layer factors and sources of wave.forcing_setup for the medium
    sqrt(c2f) (give forcing.c_max to hold the layer fixed under changes of
    the medium, as the gradient does)."""
    return O.forcing_setup(prob, np.sqrt(c2f), forcing)


def forward_frozen(prob, c2f, u0, p0, K, correctors, cc_theta, store=False,
                   forcing=None):
    """Algorithm 3 with the recorded correctors theta^k (literal sweep).
    Returns the final iterates (lists over n) and, with store=True, the
    intermediate quantities the adjoint needs.  forcing: the layer and
    source of wave.theta_parareal (F and C of slice n from t_{n-1})."""
    r, N = prob.ratio, prob.N
    c2f = np.asarray(c2f, float)
    c2c = O.restrict(c2f, r)
    hf, hc = prob.dt_fine, prob.dt_coarse
    dxf, dxc = prob.dx_fine, prob.dx_coarse
    fs = _forcing(prob, c2f, forcing)

    def Cst(U, P, n):
        return _prop_store(U, P, c2c, hc, dxc, prob.m_coarse, fs["dC"],
                           fs["srcC"], (n - 1) * prob.dt_com)

    tape = {"init": [], "iters": []}
    u = [np.array(u0, float)] + [None] * N
    p = [np.array(p0, float)] + [None] * N
    W, Wp = O.restrict(u[0], r), O.restrict(p[0], r)
    for n in range(1, N + 1):
        W2, Wp2, us = Cst(W, Wp, n)
        tape["init"].append(us)
        u[n], p[n] = O.interp(W2, r), O.interp(Wp2, r)
        W, Wp = O.restrict(u[n], r), O.restrict(p[n], r)
    for k in range(K):
        UV = correctors[k]
        it = {"F": [None] * (N + 1), "Cw": [None] * (N + 1),
              "Ct": [None] * (N + 1)}
        v, vp = [None] * (N + 1), [None] * (N + 1)
        for n in range(1, N + 1):
            v[n], vp[n], it["F"][n] = _prop_store(
                u[n - 1], p[n - 1], c2f, hf, dxf, prob.m_fine, fs["dF"],
                fs["srcF"], (n - 1) * prob.dt_com)
        un, pn = [u[0]] + [None] * N, [p[0]] + [None] * N
        for n in range(1, N + 1):
            w, wp, it["Cw"][n] = Cst(O.restrict(un[n - 1], r),
                                     O.restrict(pn[n - 1], r), n)
            wt, wtp, it["Ct"][n] = Cst(O.restrict(u[n - 1], r),
                                       O.restrict(p[n - 1], r), n)
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


def sweep_traces(prob, c2f, u, p, receivers, forcing=None, store=False):
    """One more F sweep from the slice starts (u[n-1], p[n-1]), n = 1..N,
    sampling u at the receivers after every fine step: array (N, m_F,
    n_rec) (the traces of a receiver record; with store=True also the
    displacements of every step, for the adjoint)."""
    c2f = np.asarray(c2f, float)
    fs = _forcing(prob, c2f, forcing)
    tr, uss = [], []
    for n in range(1, prob.N + 1):
        _, _, us = _prop_store(u[n - 1], p[n - 1], c2f, prob.dt_fine,
                               prob.dx_fine, prob.m_fine, fs["dF"],
                               fs["srcF"], (n - 1) * prob.dt_com)
        tr.append(np.stack([x.ravel()[receivers] for x in us[1:]]))
        uss.append(us)
    tr = np.stack(tr)
    return (tr, uss) if store else tr


def sweep_misfit(traces, data, dt):
    """1/2 dt sum_{n, i, r} (traces - data)^2 (the time integral of the
    squared residual of a receiver record sampled every fine step)."""
    d = np.asarray(traces) - np.asarray(data)
    return 0.5 * dt * float(np.sum(d * d))


def gradient(prob, c2f, u0, p0, K, correctors, cc_theta, receivers, data,
             forcing=None, traces="coupling"):
    """d J / d c^2 on the fine grid by the hand-written adjoint (frozen
    correctors).  Returns (J, grad).

    traces="coupling": J = misfit(u^{K+1}, receivers, data), data (N,
    n_rec) at the coupling times.  traces="sweep": J = sweep_misfit of
    sweep_traces(u^{K+1}) against data (N, m_F, n_rec).  forcing: the layer
    and source (give c_max: the layer is held fixed, not differentiated)."""
    r, N = prob.ratio, prob.N
    fshape, cshape = prob.shape, prob.coarse_shape
    nc = int(np.prod(cshape))
    c2f = np.asarray(c2f, float)
    c2c = O.restrict(c2f, r)
    hf, hc = prob.dt_fine, prob.dt_coarse
    dxf, dxc = prob.dx_fine, prob.dx_coarse
    fs = _forcing(prob, c2f, forcing)
    dF, dC = fs["dF"], fs["dC"]
    u, p, tape = forward_frozen(prob, c2f, u0, p0, K, correctors, cc_theta,
                                store=True, forcing=forcing)
    lu = [np.zeros(fshape) for _ in range(N + 1)]
    lp = [np.zeros(fshape) for _ in range(N + 1)]
    gf = np.zeros(fshape)
    if traces == "coupling":
        J = misfit(u, receivers, data)
        # seed: adjoint of u^{K+1}_n at the receivers
        for n in range(1, N + 1):
            d = u[n].ravel()[receivers] - data[n - 1]
            flat = lu[n].ravel()
            np.add.at(flat, receivers, d)
            lu[n] = flat.reshape(fshape)
    elif traces == "sweep":
        tr, uss = sweep_traces(prob, c2f, u, p, receivers, forcing,
                               store=True)
        J = sweep_misfit(tr, data, hf)
        # the sweep from u^{K+1}_{n-1}: its adjoint seeds slot n - 1
        for n in range(1, N + 1):
            seeds = []
            for i in range(prob.m_fine):
                flat = np.zeros(int(np.prod(fshape)))
                np.add.at(flat, receivers, hf * (tr[n - 1, i] - data[n - 1, i]))
                seeds.append(flat.reshape(fshape))
            a, b, g = _prop_adjoint(uss[n - 1], np.zeros(fshape),
                                    np.zeros(fshape), c2f, hf, dxf, dF, seeds)
            gf += g
            lu[n - 1] += a
            lp[n - 1] += b
    else:
        raise ValueError(traces)
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
            au, ap, g1 = _prop_adjoint(it["Cw"][n], zu, zp, c2c, hc, dxc, dC)
            # wt = C(R u[n-1]) (previous iterate), enters with a minus sign
            bu, bp, g2 = _prop_adjoint(it["Ct"][n], -zu, -zp, c2c, hc, dxc,
                                       dC)
            gc += g1 + g2
            carry_u = _restrict_T(au, r, fshape)
            carry_p = _restrict_T(ap, r, fshape)
            lu_old[n - 1] += _restrict_T(bu, r, fshape)
            lp_old[n - 1] += _restrict_T(bp, r, fshape)
        # un[0] = u0 is fixed: carry into n = 0 is dropped
        # v[n] = F(u[n-1])
        for n in range(1, N + 1):
            a, b, g = _prop_adjoint(it["F"][n], lv[n], lvp[n], c2f, hf, dxf,
                                    dF)
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
        au, ap, g = _prop_adjoint(tape["init"][n - 1], Lu, Lp, c2c, hc, dxc,
                                  dC)
        gc += g
        # R I = 1: the restricted state R u^1_{n-1} is W_{n-1} itself
        carry_u, carry_p = au, ap
    gf += _restrict_T(gc, r, fshape)
    return J, gf
