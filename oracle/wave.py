"""FP64 numpy oracle of the stabilised parareal-like method (Nguyen & Tsai,
arXiv 1905.00473).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the HIP library.

Array conventions
-----------------
* A grid function on the periodic box is a numpy array of shape
  ``(n_y, n_x)`` (2D), ``(n_z, n_y, n_x)`` (3D) or ``(n_x,)`` (1D); x is the
  last (fastest) axis.  Spatial axis ``a = 0, 1, 2`` means x, y, z, i.e. numpy
  axis ``ndim - 1 - a``.
* The box has the same length ``L = n * dx`` along every axis (``L = 1`` for
  the unit box of eq. (1)); wavenumbers are ``xi = 2*pi*k/L`` with integer
  ``k`` from ``numpy.fft.fftfreq``.
* A column of the data matrices (the energy components of eqs. matrixF /
  matrixG) is the concatenation ``[d_x U ; d_y U ; (d_z U) ; P / c]`` of
  flattened fields (x fastest), without the ``dx**d`` factor.

Parity status (what pins each routine; see tests/test_oracle_pins.py)
--------------------------------------------------------------------
* laplacian, vv_step, propagate ........ pinned (discrete closed form for
  constant c, conservation of the modified discrete energy, observed order
  2 on a plane wave, time reversibility)
* restrict, interp ...................... pinned (R I = identity, exact
  reproduction of trigonometric polynomials, I(0) = 0)
* gradient, grad2func, lambda_dag ....... pinned (per-mode multipliers of
  Lambda^dag Lambda in closed form; the paper's printed reconstruction
  errors of the Sec. 6.4 gradient-order table, third column)
* energy ................................. pinned (the Frobenius identity of
  eq. partOPP, hand-computed values)
* procrustes, update_svd ................. pinned (brute force over O(2) and
  O(3); the minimum-residual closed form; incremental == direct SVD of the
  explicitly summed correlation matrix; rank identity of Sec. 3.3.1)
* theta_parareal (and adjoint.py) ......... pinned (exactness of the first k
  slices after k iterations; reduction to textbook parareal with the
  spectral gradient, identical grids and Omega = I; energy preservation of
  the corrected coarse propagator of Sec. 6.3).  The full-loop values on
  the synthetic workloads are not printed in the paper: parity unpinned
  beyond these invariants.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "laplacian", "vv_step", "propagate", "restrict", "interp",
    "ricker", "sponge_sigma", "sponge_sigma_max", "propagate_forced",
    "Forcing", "forcing_setup", "fine_traces",
    "gradient", "FD_COEFFS", "energy_components", "split_components",
    "grad2func", "lambda_dag", "energy", "procrustes", "update_svd",
    "omega_apply", "theta_parareal", "serial_fine", "energy_error",
    "l2_error", "PararealResult",
]


# ---------------------------------------------------------------------------
# Problem description (parameter columns of the Sec. 6 tables)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """Discretisation parameters of one wave problem.

    ``shape``: fine grid, numpy order (x last).  ``ratio``: dx_coarse /
    dx_fine (coarse node J sits on fine node ratio*J, Sec. 6 "coarse grid
    nodes overlap with the fine grid nodes").  ``T``: final time, ``N``:
    number of coupling intervals of length dt_com = T/N.  ``m_fine`` /
    ``m_coarse``: steps per interval of F and C (Sec. 3.1).  ``length``: box
    length L per axis.  ``interp``: the interpolation I, trigonometric
    (the interpft of Sec. 6), periodic piecewise linear, or local cubic
    (4-point Lagrange): lower-order interpolants of the kind the numerical
    examples of Sec. 7 also use.
    """

    shape: tuple
    ratio: int
    T: float
    N: int
    m_fine: int
    m_coarse: int
    grad_order: object = 4
    tol: float = 1e-14
    length: float = 1.0
    interp: str = "trig"    # I: "trig" (interpft), "linear" or "cubic"

    @property
    def dim(self):
        return len(self.shape)

    @property
    def coarse_shape(self):
        return tuple(n // self.ratio for n in self.shape)

    @property
    def dx_fine(self):
        return self.length / self.shape[-1]

    @property
    def dx_coarse(self):
        return self.dx_fine * self.ratio

    @property
    def dt_com(self):
        return self.T / self.N

    @property
    def dt_fine(self):
        return self.dt_com / self.m_fine

    @property
    def dt_coarse(self):
        return self.dt_com / self.m_coarse


# ---------------------------------------------------------------------------
# Sec. 3.1: second-order central differences + velocity Verlet
# ---------------------------------------------------------------------------
def laplacian(u, dx):
    """Periodic second-order central-difference Laplacian: the sum over the
    axes of (u[i+1] - 2 u[i] + u[i-1]) / dx^2 (Sec. 3.1)."""
    out = np.zeros_like(u)
    for ax in range(u.ndim):
        out += (np.roll(u, -1, ax) - 2.0 * u + np.roll(u, 1, ax)) / dx ** 2
    return out


def vv_step(u, p, c2, h, dx):
    """One velocity-Verlet step of u_tt = c^2 Lap u (Sec. 3.1): half kick,
    drift, half kick."""
    p = p + 0.5 * h * c2 * laplacian(u, dx)
    u = u + h * p
    p = p + 0.5 * h * c2 * laplacian(u, dx)
    return u, p


def propagate(u, p, c2, h, dx, m):
    """m velocity-Verlet steps of size h.  With the fine grid and
    h = dt_com/m_F this is the fine propagator F; with the coarse grid,
    pointwise coarse c and h = dt_com/m_C it is the coarse propagator C
    (Sec. 3.1)."""
    u = np.array(u, dtype=np.float64, copy=True)
    p = np.array(p, dtype=np.float64, copy=True)
    for _ in range(m):
        u, p = vv_step(u, p, c2, h, dx)
    return u, p


# ---------------------------------------------------------------------------
# Absorbing layer and point source (eq. (1) names absorbing boundaries as an
# alternative to the periodic box; the forcing is an inhomogeneous term f in
# u_tt = c^2 Lap u + f).  Reading: a damping layer inside the periodic box,
# p_t = ... - sigma p, integrated exactly over each half step, and a point
# source r(t) / dx^d at one node.
# ---------------------------------------------------------------------------
def ricker(t, freq, t0):
    """Ricker wavelet (1 - 2 a) exp(-a), a = (pi f (t - t0))^2."""
    a = (np.pi * freq * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def sponge_sigma(shape, width, sigma_max, length=1.0):
    """Damping coefficient of a layer of the given width along every face of
    the box: sigma = sigma_max (d / width)^2, d the largest penetration
    max(0, width - min(x_a, L_a - x_a)) over the axes (nodes x = j dx, the
    spacing dx = length / n_x of every axis, so the box is L_a = n_a dx
    long along axis a)."""
    dx = length / shape[-1]
    d = np.zeros(shape)
    for ax, n in enumerate(shape):
        x = np.arange(n) * dx
        L = n * dx
        pen = np.maximum(0.0, width - np.minimum(x, L - x))
        sh = [1] * len(shape)
        sh[ax] = n
        d = np.maximum(d, pen.reshape(sh))
    return sigma_max * (d / width) ** 2


def sponge_sigma_max(c_max, width, reflection=1e-3):
    """sigma_max of a quadratic layer whose round trip at speed c_max damps
    the amplitude by `reflection`: (3 c_max / (2 width)) ln(1 / reflection)."""
    return 3.0 * c_max / (2.0 * width) * math.log(1.0 / reflection)


def propagate_forced(u, p, c2, h, dx, m, damp=None, src=None, t_start=0.0,
                     receivers=None):
    """m velocity-Verlet steps of u_tt = c^2 Lap u - sigma u_t + f (Sec. 3.1
    scheme).  Each half step first damps p by damp = exp(-sigma h / 2) (the
    exact solution of p_t = -sigma p over h / 2; None: no layer), then
    kicks it by (h/2) (c^2 Lap u + f(t)); f is src = (flat index, amplitude,
    freq, t0): amplitude * ricker(t) at one node (None: no source); the
    kicks of step j use t_start + j h and t_start + (j + 1) h.  With
    receivers (flat indices) also returns the (m, n_rec) samples of u after
    every step."""
    u = np.array(u, dtype=np.float64, copy=True)
    p = np.array(p, dtype=np.float64, copy=True)
    traces = [] if receivers is not None else None

    def half_kick(pp, uu, t):
        # the same expression as vv_step, then the source term
        pp = (pp if damp is None else damp * pp) + 0.5 * h * c2 * laplacian(uu, dx)
        if src is not None:
            idx, amp, freq, t0 = src
            pp.flat[idx] += 0.5 * h * amp * ricker(t, freq, t0)
        return pp

    for j in range(m):
        t0_, t1_ = t_start + j * h, t_start + (j + 1) * h
        p = half_kick(p, u, t0_)
        u = u + h * p
        p = half_kick(p, u, t1_)
        if traces is not None:
            traces.append(u.ravel()[np.asarray(receivers)].copy())
    if traces is not None:
        return u, p, np.array(traces)
    return u, p


@dataclasses.dataclass
class Forcing:
    """Absorbing layer and point source of a problem: layer width (0: none)
    and the round-trip damping it is designed for; source position in the
    box (x first; None: no source), Ricker peak frequency and peak time."""
    width: float = 0.0
    reflection: float = 1e-3
    src_pos: tuple = None
    freq: float = 10.0
    t0: float = 0.1
    c_max: float = None     # speed in sigma_max (None: the largest c given)


def _nearest_node(pos, shape, dx):
    idx = []
    for a in range(len(shape)):
        ax = len(shape) - 1 - a
        idx.append(int(round(pos[a] / dx)) % shape[ax])
    flat = 0
    for a in reversed(range(len(shape))):
        ax = len(shape) - 1 - a
        flat = flat * shape[ax] + idx[a]
    return flat


def forcing_setup(prob, c, forcing):
    """Fine and coarse damping factors exp(-sigma h / 2) (the coarse layer
    is the pointwise restriction of the fine sigma; sigma_max from the
    largest fine c) and the point sources (nearest fine / coarse node,
    amplitude 1 / dx^d) of a problem."""
    out = {"dF": None, "dC": None, "srcF": None, "srcC": None}
    if forcing is None:
        return out
    cf = np.asarray(c, dtype=np.float64)
    d = len(prob.shape)
    if forcing.width > 0:
        cmax = float(cf.max()) if forcing.c_max is None else forcing.c_max
        smax = sponge_sigma_max(cmax, forcing.width, forcing.reflection)
        sig = sponge_sigma(prob.shape, forcing.width, smax, prob.length)
        out["dF"] = np.exp(-0.5 * sig * prob.dt_fine)
        out["dC"] = np.exp(-0.5 * restrict(sig, prob.ratio) * prob.dt_coarse)
    if forcing.src_pos is not None:
        out["srcF"] = (_nearest_node(forcing.src_pos, prob.shape, prob.dx_fine),
                       prob.dx_fine ** -d, forcing.freq, forcing.t0)
        out["srcC"] = (_nearest_node(forcing.src_pos, prob.coarse_shape,
                                     prob.dx_coarse),
                       prob.dx_coarse ** -d, forcing.freq, forcing.t0)
    return out


def fine_traces(prob, c, us, ps, forcing, receivers, pmap=None):
    """Receiver samples of u after every fine step of one F sweep from the
    slice starts (us[n-1], ps[n-1]), n = 1..N: array (N, m_F, n_rec)."""
    cf = np.asarray(c, dtype=np.float64)
    fs = forcing_setup(prob, cf, forcing)
    args = [(us[n - 1], ps[n - 1], cf * cf, prob.dt_fine, prob.dx_fine,
             prob.m_fine, fs["dF"], fs["srcF"], (n - 1) * prob.dt_com,
             receivers) for n in range(1, prob.N + 1)]
    out = list(pmap(propagate_forced, args)) if pmap is not None else \
        [propagate_forced(*a) for a in args]
    return np.stack([o[2] for o in out])


# ---------------------------------------------------------------------------
# Grid transfer (Sec. 3.1; Sec. 5 "R I = 1"; Sec. 6 interpft)
# ---------------------------------------------------------------------------
def restrict(u, ratio):
    """Pointwise restriction R: the values at the fine nodes that coincide
    with coarse nodes (coarse J <-> fine ratio*J on every axis)."""
    sl = tuple(slice(None, None, ratio) for _ in range(u.ndim))
    return np.array(u[sl], copy=True)


def _interp_axis(U, ratio, ax):
    n = U.shape[ax]
    nf = n * ratio
    A = np.moveaxis(np.fft.fft(U, axis=ax), ax, -1)
    B = np.zeros(A.shape[:-1] + (nf,), dtype=complex)
    h = n // 2
    if n % 2 == 0:
        # non-negative frequencies below Nyquist, then the Nyquist
        # coefficient split equally between +n/2 and -n/2, then the
        # negative frequencies
        B[..., :h] = A[..., :h]
        B[..., h] = 0.5 * A[..., h]
        B[..., nf - h] = 0.5 * A[..., h]
        B[..., nf - h + 1:] = A[..., h + 1:]
    else:
        B[..., :h + 1] = A[..., :h + 1]
        B[..., nf - h:] = A[..., h + 1:]
    out = np.fft.ifft(B, axis=-1).real * ratio
    return np.moveaxis(out, -1, ax)


def _interp_axis_linear(U, ratio, ax):
    # fine node ratio*J + s lies at J + s/ratio in coarse units, between
    # coarse nodes J and J + 1 (periodic)
    A = np.moveaxis(U, ax, -1)
    n = A.shape[-1]
    out = np.zeros(A.shape[:-1] + (n * ratio,))
    for J in range(n):
        for s in range(ratio):
            t = s / ratio
            out[..., J * ratio + s] = (1.0 - t) * A[..., J] + t * A[..., (J + 1) % n]
    return np.moveaxis(out, -1, ax)


def _cubic_weights(t):
    # 4-point Lagrange weights of the nodes -1, 0, 1, 2 at t in [0, 1)
    return ((-t * (t - 1) * (t - 2) / 6.0, (t + 1) * (t - 1) * (t - 2) / 2.0,
             -(t + 1) * t * (t - 2) / 2.0, (t + 1) * t * (t - 1) / 6.0))


def _interp_axis_cubic(U, ratio, ax):
    # fine node ratio*J + s at J + s/ratio: the cubic through the coarse
    # nodes J - 1 .. J + 2 (periodic)
    A = np.moveaxis(U, ax, -1)
    n = A.shape[-1]
    out = np.zeros(A.shape[:-1] + (n * ratio,))
    for J in range(n):
        for s in range(ratio):
            w = _cubic_weights(s / ratio)
            out[..., J * ratio + s] = sum(w[k] * A[..., (J + k - 1) % n]
                                          for k in range(4))
    return np.moveaxis(out, -1, ax)


def interp(U, ratio, kind="trig"):
    """Interpolation I from the coarse to the fine grid, one axis at a time.
    ``kind='trig'``: trigonometric (Fourier) interpolation: the coarse
    spectrum is zero-padded, the Nyquist coefficient of an even length is
    split between +n/2 and -n/2, and the real part of the inverse transform
    is returned (the `interpft` interpolation of Sec. 6).
    ``kind='linear'``: periodic piecewise-linear interpolation between
    neighbouring coarse nodes.  ``kind='cubic'``: local cubic (4-point
    Lagrange) interpolation through the coarse nodes J - 1 .. J + 2."""
    if kind not in ("trig", "linear", "cubic"):
        raise ValueError(kind)
    out = np.asarray(U, dtype=np.float64)
    if ratio == 1:
        return np.array(out, copy=True)
    for ax in range(out.ndim):
        f = {"trig": _interp_axis, "linear": _interp_axis_linear,
             "cubic": _interp_axis_cubic}[kind]
        out = f(out, ratio, ax)
    return out


# ---------------------------------------------------------------------------
# Energy components (eqs. matrixF / matrixG, discrete-wave-energy)
# ---------------------------------------------------------------------------
#: beta_j of the central 2m-order first-derivative stencil
#: d u ~ sum_j beta_j (u[i+j] - u[i-j]) / dx (Sec. 3.4)
FD_COEFFS = {
    2: (1.0 / 2.0,),
    4: (2.0 / 3.0, -1.0 / 12.0),
    6: (3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0),
    8: (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0),
}


def _wavenumbers(n, dx):
    return 2.0 * np.pi * np.fft.fftfreq(n, d=dx)


def gradient(U, dx, order=4):
    """Numerical gradient nabla_h U as a list [d_x U, d_y U, (d_z U)]: a
    periodic central difference of the given even order, or the Fourier
    derivative real(ifft(i xi fft U)) for order 'spectral' (Sec. 3.4)."""
    U = np.asarray(U, dtype=np.float64)
    out = []
    for a in range(U.ndim):
        ax = U.ndim - 1 - a
        if order == "spectral":
            xi = _wavenumbers(U.shape[ax], dx)
            shp = [1] * U.ndim
            shp[ax] = -1
            d = np.fft.ifft(1j * xi.reshape(shp) * np.fft.fft(U, axis=ax),
                            axis=ax).real
        else:
            d = np.zeros_like(U)
            for j, b in enumerate(FD_COEFFS[order], start=1):
                d += b * (np.roll(U, -j, ax) - np.roll(U, j, ax))
            d /= dx
        out.append(d)
    return out


def energy_components(U, P, c, dx, order=4):
    """Lambda[U, P] = [nabla_h U ; P / c] as one column (eqs. matrixF /
    matrixG)."""
    g = gradient(U, dx, order)
    return np.concatenate([x.ravel() for x in g] + [(P / c).ravel()])


def split_components(z, shape):
    """Inverse of the concatenation in energy_components: returns the list
    of d gradient blocks and the momentum block."""
    n = int(np.prod(shape))
    d = len(shape)
    q = [z[a * n:(a + 1) * n].reshape(shape) for a in range(d)]
    return q, z[d * n:(d + 1) * n].reshape(shape)


def energy(u, p, c, dx, order=4):
    """Discrete wave energy (eq. discrete-wave-energy):
    1/2 sum |nabla_h u|^2 dx^d + 1/2 sum c^-2 p^2 dx^d."""
    d = np.ndim(u)
    g = gradient(u, dx, order)
    return 0.5 * (sum(np.sum(x * x) for x in g)
                  + np.sum(p * p / (c * c))) * dx ** d


# ---------------------------------------------------------------------------
# Reconstruction of the wavefield from its gradient (Sec. 3.4)
# ---------------------------------------------------------------------------
def grad2func(q, s, dx):
    """Algorithm 2 / eq. gradient2coordinate: given gradient components q
    (list of d fields) and the sum s of the sought function, return
    real(ifft(W)) with W(xi) = -i xi.fft(q) / |xi|^2 for xi != 0 and
    W(0) = s (unnormalised forward transform)."""
    shape = q[0].shape
    d = len(shape)
    num = np.zeros(shape, dtype=complex)
    xi2 = np.zeros(shape)
    for a in range(d):
        ax = d - 1 - a
        xi = _wavenumbers(shape[ax], dx)
        shp = [1] * d
        shp[ax] = -1
        xi = xi.reshape(shp)
        num = num + xi * np.fft.fftn(q[a])
        xi2 = xi2 + xi * xi
    W = np.zeros(shape, dtype=complex)
    nz = xi2 != 0
    W[nz] = -1j * num[nz] / xi2[nz]
    W[(0,) * d] = s
    return np.fft.ifftn(W).real


def lambda_dag(z, s, c, dx, shape):
    """Lambda^dag: energy components [q ; p] -> wavefield [w, w_t] with
    w = grad2func(q, s) and w_t = c p (Sec. 3.4)."""
    q, pm = split_components(z, shape)
    return grad2func(q, s, dx), c * pm


# ---------------------------------------------------------------------------
# Orthogonal Procrustes problem (Secs. 3.2, 3.3)
# ---------------------------------------------------------------------------
def procrustes(F, G):
    """Full-rank solution of min ||F - Omega G||_F over orthogonal Omega:
    Omega = X Y^T from the SVD F G^T = X Sigma Y^T, and the minimum
    residual ||F||^2 + ||G||^2 - 2 trace(Sigma) (Sec. 3.3)."""
    X, sig, Yt = np.linalg.svd(F @ G.T)
    omega = X @ Yt
    rmin2 = np.sum(F * F) + np.sum(G * G) - 2.0 * np.sum(sig)
    return omega, rmin2


def _reduced_qr(A):
    # "truncatedqr" of Algorithm 1, read as the economy-size QR
    Q, R = np.linalg.qr(A, mode="reduced")
    return Q, R


def _rank(sig, tol):
    if sig.size == 0 or sig[0] <= 0.0:
        return 0
    return int(np.sum(sig / np.max(sig) > tol))


def _range_basis(A, omega, power):
    """Randomised range finder of Halko, Martinsson and Tropp (2011,
    Algorithm 4.3 with power iterations): an orthonormal basis of the range
    of A Omega (A A^T)^q-weighted, Q = qr((A A^T)^q A Omega), each power
    step re-orthonormalised."""
    Y = A @ omega
    for _ in range(power):
        Y, _ = _reduced_qr(Y)
        Y = A @ (A.T @ Y)
    Q, _ = _reduced_qr(Y)
    return Q


def update_svd(U, S, V, F, G, tol, svd=None, sketch=None):
    """Algorithm 1: truncated SVD of M_new = U diag(S) V^T + F G^T.

    With S empty (first call): reduced QR of F and G, SVD of R_F R_G^T,
    rank = #{sigma_i / sigma_max > tol}.  Otherwise: projections U_F = U^T F
    and V_G = V^T G, reduced QR of the residuals (one classical
    Gram-Schmidt re-orthogonalisation pass against U / V, exact no-op in
    exact arithmetic), SVD of H = [U_F; R_F][V_G; R_G]^T + diag(S, 0),
    truncation, and the rotated bases [U Q_F] X_h, [V Q_G] Y_h.
    Returns (U_new, S_new, V_new).  ``svd``: the SVD routine (default
    numpy.linalg.svd, LAPACK's divide and conquer); another backward-stable
    driver gives the same exact arithmetic with other rounding.

    ``sketch = (Omega, q)``: randomised sketching of the new data (the
    randomised low-rank methods Sec. 6.5 points to), in place of the
    truncated QR of the residuals: Q_F = range basis of (F - U U_F) Omega
    with q power iterations (Halko, Martinsson, Tropp), R_F = Q_F^T (F -
    U U_F), and likewise for G with the same Omega (N x l, l <= N, a
    random draw given as input).  The core matrix is then (r + l) square.
    Exact (up to rounding) whenever the residuals have rank <= l.
    """
    svd = svd or np.linalg.svd
    F = np.asarray(F, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)

    def qr_of(A):
        if sketch is None:
            return _reduced_qr(A)
        Q = _range_basis(A, sketch[0], sketch[1])
        return Q, Q.T @ A

    if S is None or len(S) == 0:
        QF, RF = qr_of(F)
        QG, RG = qr_of(G)
        X, sig, Yt = svd(RF @ RG.T)
        r = _rank(sig, tol)
        return QF @ X[:, :r], sig[:r].copy(), QG @ Yt.T[:, :r]
    UF = U.T @ F
    VG = V.T @ G
    Fp = F - U @ UF
    Gp = G - V @ VG
    UF2 = U.T @ Fp
    Fp = Fp - U @ UF2
    UF = UF + UF2
    VG2 = V.T @ Gp
    Gp = Gp - V @ VG2
    VG = VG + VG2
    QF, RF = qr_of(Fp)
    QG, RG = qr_of(Gp)
    H = np.vstack([UF, RF]) @ np.vstack([VG, RG]).T
    r0 = len(S)
    H[:r0, :r0] += np.diag(S)
    X, sig, Yt = svd(H)
    r = _rank(sig, tol)
    Un = np.hstack([U, QF]) @ X[:, :r]
    Vn = np.hstack([V, QG]) @ Yt.T[:, :r]
    return Un, sig[:r].copy(), Vn


def omega_apply(U, V, z):
    """Action of the truncated phase corrector Omega = U V^T on z."""
    return U @ (V.T @ z)


# ---------------------------------------------------------------------------
# Algorithm 3 (eq. thetarelation)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class PararealResult:
    u: list                 # u^{K+1}_n, n = 0..N (fine grid)
    p: list
    rho: list               # ||F^k - Omega^k G^k||_F / ||F^k||_F, k = 1..K
    rank: list              # rank of Omega^k, k = 1..K
    history: list           # [(u list, p list)] for k = 1..K+1 if kept
    sigma: list             # singular values after each update
    correctors: list = None  # [(U_k, V_k)] if recorded
    data_norms: list = None  # [(||F^k||^2, ||F^k_in||^2, ||G^k_in||^2)]


def theta_parareal(prob: Problem, c, u0, p0, K, keep_history=False,
                   omega="procrustes", correction=True,
                   record_correctors=False, sample_cols=None, pmap=None,
                   svd=None, sweep="literal", sketch=None, power=0,
                   forcing=None):
    """Algorithm 3 of the paper, step by step.

    Initialisation u^1_n = I C R u^1_{n-1}; then K iterations of: parallel
    v_n = F u^k_{n-1} and U_n = C R u^k_{n-1} for n = 1..N; data matrices
    F = [Lambda R v_n], G = [Lambda U_n]; UpdateSVD; serial sweep
    w = C R u^{k+1}_{n-1}, [q,p] = Omega Lambda w, [q~,p~] = Omega Lambda U_n,
    u^{k+1}_n = v_n + I[real(grad2func(q, sum w) - grad2func(q~, sum U_n)),
    c (p - p~)].  Slice indices n = 0..N with u^k_0 = u0.

    ``omega='identity'`` uses Omega = I (Sec. 6.2); ``omega='plain'`` is
    the plain parareal method of eq. plainparareal with the coarse
    propagator I C R (no energy components, no Lambda^dag);
    ``correction=False`` drops the parareal-style additive term (Sec. 6.3).

    ``sample_cols``: random subsampling of the data matrices (Sec. 6.5).
    Entry k-1 lists the columns (0-based, column j holds slice j+1) of
    F^k and G^k that Algorithm 1 receives in iteration k; the draw is an
    input.  rho_k is still measured on all N columns.

    ``pmap``: how the parallel loop of Algorithm 3 (the parfor over slices)
    is executed: a function with the signature of ``itertools.starmap``
    applied to ``propagate`` and one argument tuple per slice (e.g. a
    process pool's ``starmap``); None runs the slices one after another.
    Every slice is computed by the same ``propagate`` call either way.
    ``svd``: the SVD routine of Algorithm 1 (see update_svd).

    ``sketch``: randomised sketching inside Algorithm 1 (see update_svd):
    entry k-1 is the N x l Gaussian test matrix of iteration k (an input);
    ``power`` power iterations.  Not combined with ``sample_cols``.

    ``forcing``: an absorbing layer and / or a point source (Forcing): F
    and C of slice n then propagate u_tt = c^2 Lap u - sigma u_t + f from
    t_{n-1} = (n - 1) dt_com (propagate_forced), the coarse layer and source
    from forcing_setup; everything else is unchanged.

    ``sweep``: "literal" applies Omega and grad2func to both terms of the
    correction, as Algorithm 3 writes it; "difference" applies them once
    to the difference Lambda(w - U_n), with the sum of w - U_n as the mean
    (the same linear map, another rounding; used only to measure how much
    rounding alone moves the iteration).
    """
    r = prob.ratio
    ik = prob.interp
    N = prob.N
    cf = np.asarray(c, dtype=np.float64)
    cc = restrict(cf, r)
    c2f, c2c = cf * cf, cc * cc
    dxf, dxc = prob.dx_fine, prob.dx_coarse
    hf, hc = prob.dt_fine, prob.dt_coarse
    cshape = prob.coarse_shape
    order = prob.grad_order

    fs = forcing_setup(prob, cf, forcing)

    def Fargs(u, p, n):
        if forcing is None:
            return (u, p, c2f, hf, dxf, prob.m_fine)
        return (u, p, c2f, hf, dxf, prob.m_fine, fs["dF"], fs["srcF"],
                (n - 1) * prob.dt_com)

    def Fprop(u, p, n):
        a = Fargs(u, p, n)
        return propagate(*a) if forcing is None else propagate_forced(*a)

    def Cprop(U, P, n):
        if forcing is None:
            return propagate(U, P, c2c, hc, dxc, prob.m_coarse)
        return propagate_forced(U, P, c2c, hc, dxc, prob.m_coarse, fs["dC"],
                                fs["srcC"], (n - 1) * prob.dt_com)

    def Lam(U, P):
        return energy_components(U, P, cc, dxc, order)

    u = [np.array(u0, dtype=np.float64)] + [None] * N
    p = [np.array(p0, dtype=np.float64)] + [None] * N
    for n in range(1, N + 1):
        W, Wp = Cprop(restrict(u[n - 1], r), restrict(p[n - 1], r), n)
        u[n], p[n] = interp(W, r, ik), interp(Wp, r, ik)
    history = [([x.copy() for x in u], [x.copy() for x in p])] \
        if keep_history else []

    Us = S = Vs = None
    rhos, ranks, sigmas, norms = [], [], [], []
    correctors = [] if record_correctors else None
    for _k in range(K):
        v, vp, Uc, Ucp = [None] * (N + 1), [None] * (N + 1), \
            [None] * (N + 1), [None] * (N + 1)
        if pmap is not None:                # the parallel loop (parfor)
            out = list(pmap(propagate if forcing is None else
                            propagate_forced,
                            [Fargs(u[n - 1], p[n - 1], n)
                             for n in range(1, N + 1)]))
            for n in range(1, N + 1):
                v[n], vp[n] = out[n - 1]
        for n in range(1, N + 1):           # the parallel loop
            if pmap is None:
                v[n], vp[n] = Fprop(u[n - 1], p[n - 1], n)
            Uc[n], Ucp[n] = Cprop(restrict(u[n - 1], r),
                                  restrict(p[n - 1], r), n)
        Fm = np.column_stack([Lam(restrict(v[n], r), restrict(vp[n], r))
                              for n in range(1, N + 1)])
        Gm = np.column_stack([Lam(Uc[n], Ucp[n]) for n in range(1, N + 1)])
        if omega not in ("procrustes", "identity", "plain"):
            raise ValueError(omega)
        if omega == "procrustes":
            if sample_cols is None:
                Fs, Gs = Fm, Gm
            else:
                cols = np.asarray(sample_cols[_k], dtype=np.int64)
                if (cols.size == 0 or cols.min() < 0 or cols.max() >= N
                        or np.unique(cols).size != cols.size):
                    raise ValueError("sample columns must be distinct "
                                     "indices in [0, N)")
                Fs, Gs = Fm[:, cols], Gm[:, cols]
            norms.append((float(np.sum(Fm * Fm)), float(np.sum(Fs * Fs)),
                          float(np.sum(Gs * Gs))))
            sk = None
            if sketch is not None:
                if sample_cols is not None:
                    raise ValueError("sketching and column sampling are "
                                     "exclusive")
                sk = (np.asarray(sketch[_k], dtype=np.float64), power)
            Us, S, Vs = update_svd(Us, S, Vs, Fs, Gs, prob.tol, svd, sk)
            if record_correctors:
                correctors.append((Us.copy(), Vs.copy()))
            res = Fm - omega_apply(Us, Vs, Gm)
            ranks.append(len(S))
            sigmas.append(S.copy())
        else:
            norms.append((float(np.sum(Fm * Fm)), 0.0, 0.0))
            res = Fm - Gm
            ranks.append(Fm.shape[0])
            sigmas.append(np.zeros(0))
        nF = np.linalg.norm(Fm)
        rhos.append(float(np.linalg.norm(res) / nF) if nF > 0 else 0.0)

        def Om(z):
            return omega_apply(Us, Vs, z) if omega == "procrustes" else z

        un = [u[0]] + [None] * N
        pn = [p[0]] + [None] * N
        for n in range(1, N + 1):            # the serial sweep
            w, wp = Cprop(restrict(un[n - 1], r), restrict(pn[n - 1], r), n)
            if omega == "plain":
                # eq. plainparareal: I C R u^{k+1}_{n-1} + F u^k_{n-1}
                #                    - I C R u^k_{n-1}
                if correction:
                    un[n] = v[n] + interp(w - Uc[n], r, ik)
                    pn[n] = vp[n] + interp(wp - Ucp[n], r, ik)
                else:
                    un[n], pn[n] = interp(w, r, ik), interp(wp, r, ik)
                continue
            if correction and sweep == "difference":
                zd = Om(Lam(w - Uc[n], wp - Ucp[n]))
                qd, pd = split_components(zd, cshape)
                un[n] = v[n] + interp(grad2func(qd, np.sum(w - Uc[n]), dxc),
                                      r, ik)
                pn[n] = vp[n] + interp(cc * pd, r, ik)
                continue
            zq = Om(Lam(w, wp))
            q, pq = split_components(zq, cshape)
            q1 = grad2func(q, np.sum(w), dxc)
            if correction:
                zt = Om(Lam(Uc[n], Ucp[n]))
                qt, pt = split_components(zt, cshape)
                qt1 = grad2func(qt, np.sum(Uc[n]), dxc)
                du = q1 - qt1
                dp = cc * (pq - pt)
                un[n] = v[n] + interp(du, r, ik)
                pn[n] = vp[n] + interp(dp, r, ik)
            else:
                un[n] = interp(q1, r, ik)
                pn[n] = interp(cc * pq, r, ik)
        u, p = un, pn
        if keep_history:
            history.append(([x.copy() for x in u], [x.copy() for x in p]))
    return PararealResult(u=u, p=p, rho=rhos, rank=ranks,
                            history=history, sigma=sigmas,
                            correctors=correctors, data_norms=norms)


def serial_fine(prob: Problem, c, u0, p0, forcing=None):
    """Serial fine reference u(t_n) = F^n [u0, p0], n = 0..N (Sec. 6: the
    reference solution is computed serially with the fine propagator)."""
    cf = np.asarray(c, dtype=np.float64)
    c2 = cf * cf
    fs = forcing_setup(prob, cf, forcing)
    us = [np.array(u0, dtype=np.float64)]
    ps = [np.array(p0, dtype=np.float64)]
    for n in range(1, prob.N + 1):
        if forcing is None:
            a, b = propagate(us[-1], ps[-1], c2, prob.dt_fine, prob.dx_fine,
                             prob.m_fine)
        else:
            a, b = propagate_forced(us[-1], ps[-1], c2, prob.dt_fine,
                                    prob.dx_fine, prob.m_fine, fs["dF"],
                                    fs["srcF"], (n - 1) * prob.dt_com)
        us.append(a)
        ps.append(b)
    return us, ps


# ---------------------------------------------------------------------------
# Error measures (Sec. 6 preamble)
# ---------------------------------------------------------------------------
def energy_error(u, p, u_ref, p_ref, c, dx, order=4):
    """sqrt(E([u - u_ref, p - p_ref]) / E([u_ref, p_ref])) on the fine grid."""
    e = energy(u - u_ref, p - p_ref, c, dx, order)
    e0 = energy(u_ref, p_ref, c, dx, order)
    return math.sqrt(e / e0) if e0 > 0 else math.sqrt(e)


def l2_error(u, u_ref):
    """||u - u_ref||_2 / ||u_ref||_2 of the displacement component."""
    n0 = np.linalg.norm(u_ref)
    return float(np.linalg.norm(u - u_ref) / n0) if n0 > 0 else \
        float(np.linalg.norm(u - u_ref))
