"""Seeded synthetic inputs shared by the oracle-side and the HIP-side tests
and by the benchmark.

This module holds no arithmetic of the method: it only builds the medium
c(x), the initial state (u0, p0) on the fine grid and the discretisation
parameters of each workload, in float64, deterministically.

Workloads (fine grid / coarse grid, unit periodic box):

* ``wave1d``  1D, 256 / 64 points, c = 1 + 0.2 sin(2 pi x),
  u0 = exp(-(x - 0.5)^2 / 0.05^2), p0 = 0, T = 1, N = 16, dt/dx = 0.5
  (m_F = 32), coarse step 4x the fine one (m_C = 8), K = 6, FP64,
  tol 1e-14.
* ``disc2d``  2D, 512^2 / 128^2, c = 1 with c = 2 inside the open disc of
  radius 0.2 centred at (0.5, 0.5), u0 = Gaussian pulse of standard
  deviation 0.03 at (0.3, 0.5), p0 = 0, T = 2, N = 64, Courant number
  c_max dt/dx = 0.5 (m_F = 64, m_C = 16), K = 8, FP32 state, tol 1e-13.
* ``layers3d`` 3D, 256^3 / 64^3, c(z) piecewise constant 1.0 / 1.5 / 2.2 /
  3.0 on four equal layers, times (1 + 0.05 eta) with eta ~ U[-1, 1] i.i.d.
  per node (seed 0), Gaussian pulse sigma = 0.04 at the centre, T = 1.5,
  N = 32, Courant number <= 0.5 with m_F a multiple of 4 (m_F = 76,
  m_C = 19), K = 6, FP32 compensated state, tol 1e-13.

* ``misfit_case`` small receiver-misfit problems in 1D/2D/3D (smooth
  medium, Ricker-shaped initial pulse, a line of receivers, random data),
  ``forced_misfit_case`` the same in 2D with an absorbing layer and a point
  source, and ``misfit2d`` the full-size one: 512^2 / 128^2, c = 1 + 2 s
  with s a min-max normalised Gaussian random field (correlation 0.1, seed
  0), zero initial state, an absorbing layer of width 0.05 (round trip
  1e-3 at c_max = 3), a Ricker source of peak frequency 10 (peak time 0.1)
  at (0.5, 0.1), 128 receivers at x = (i + 1/2)/128, y = 0.9 (nearest
  nodes) recorded every fine step, T = 1, N = 32, m_F = 96, m_C = 24,
  K = 4; target medium for the data: the same recipe, seed 1.
* ``random_pulses`` seeded Gaussian-pulse states (test inputs of the
  propagators at full size).
* ``waveguide2d`` the low-rank study of the data matrices (Sec. 6.5):
  200^2 / 100^2, c = 1 - 0.3 cos(2 pi x) on [-0.5, 0.5)^2 (here x + 1/2 on
  the unit box, i.e. c = 1 + 0.3 cos(2 pi x)), T = 4, N = 200 slices
  (dt_com = 0.02), coarse step 8e-4 (m_C = 25), fine step 8e-5
  (m_F = 250); the plane wave is a Gaussian pulse in y (sigma 0.05)
  moving in +y, p0 = -c du0/dy.  ``sample_columns`` draws the random
  slice columns of Sec. 6.5 (seeded, sorted per iteration).
* ``grf2d`` / ``batch2d``  smooth random media c = exp(0.3 g) with random
  Gaussian pulses; ``batch2d`` draws 32 such problems with fine grids from
  {256, 384, 512, 768, 1024}^2 (the batched workload).

Every generator takes the grid size, slice count and final time as
arguments, so tests run the same recipes on grids that finish in seconds.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    shape: tuple            # fine grid, numpy order (x last)
    ratio: int
    T: float
    N: int
    m_fine: int
    m_coarse: int
    K: int
    tol: float
    grad_order: int
    dtype: str              # "f64" or "f32"
    compensated: bool
    c: np.ndarray
    u0: np.ndarray
    p0: np.ndarray

    @property
    def dim(self):
        return len(self.shape)

    @property
    def coarse_shape(self):
        return tuple(n // self.ratio for n in self.shape)

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def updates_per_sweep(self):
        """Fine point-updates of one F sweep over all slices."""
        return self.N * self.m_fine * self.npts


def _axes(shape):
    """Node coordinates j/n on [0,1) per numpy axis."""
    return np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")


def _steps_for_courant(c_max, n, dt_com, courant=0.5, multiple=4):
    """Smallest m (a multiple of `multiple`) with c_max (dt_com/m) n <= courant."""
    m = math.ceil(c_max * dt_com * n / courant - 1e-12)
    return multiple * math.ceil(m / multiple)


def wave1d(n=256, ratio=4, N=16, K=6):
    x = np.arange(n) / n
    c = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    u0 = np.exp(-(x - 0.5) ** 2 / 0.05 ** 2)
    p0 = np.zeros(n)
    T = 1.0
    # dt_fine / dx_fine = 0.5 -> m_F = (T/N) / (0.5/n)
    m_f = int(round((T / N) * n / 0.5))
    return Workload("wave1d", (n,), ratio, T, N, m_f, m_f // 4, K, 1e-14, 4,
                    "f64", False, c, u0, p0)


def disc2d(n=512, ratio=4, N=64, K=8, T=2.0, dtype="f32", compensated=True):
    Y, X = _axes((n, n))
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    c = np.where(r2 < 0.2 ** 2, 2.0, 1.0)
    s = 0.03
    u0 = np.exp(-((X - 0.3) ** 2 + (Y - 0.5) ** 2) / (2 * s * s))
    p0 = np.zeros((n, n))
    m_f = _steps_for_courant(2.0, n, T / N)
    return Workload("disc2d", (n, n), ratio, T, N, m_f, m_f // 4, K, 1e-13, 4,
                    dtype, compensated, c, u0, p0)


def layers3d(n=256, ratio=4, N=32, K=6, T=1.5, dtype="f32",
             compensated=True):
    Z, Y, X = _axes((n, n, n))
    base = np.select([Z < 0.25, Z < 0.5, Z < 0.75], [1.0, 1.5, 2.2], 3.0)
    eta = np.random.default_rng(0).uniform(-1.0, 1.0, size=(n, n, n))
    c = base * (1.0 + 0.05 * eta)
    s = 0.04
    u0 = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
                / (2 * s * s))
    p0 = np.zeros((n, n, n))
    m_f = _steps_for_courant(3.0 * 1.05, n, T / N)
    return Workload("layers3d", (n, n, n), ratio, T, N, m_f, m_f // 4, K,
                    1e-13, 4, dtype, compensated, c, u0, p0)


def waveguide2d(n=200, ratio=2, N=200, K=6, T=4.0, m_fine=250, m_coarse=25,
                dtype="f64", compensated=False, tol=1e-14):
    Y, X = _axes((n, n))
    c = 1.0 + 0.3 * np.cos(2 * np.pi * X)
    s = 0.05
    u0 = np.exp(-(Y - 0.5) ** 2 / (2 * s * s))
    p0 = c * (Y - 0.5) / (s * s) * u0
    return Workload("waveguide2d", (n, n), ratio, T, N, m_fine, m_coarse, K,
                    tol, 4, dtype, compensated, c, u0, p0)


def sample_columns(N, n_per_iter, n_iters, seed=0):
    """(n_iters, n_per_iter) int32 table: per iteration n_per_iter distinct
    slice columns in [0, N), drawn uniformly without replacement and
    sorted."""
    rng = np.random.default_rng(seed)
    return np.array([np.sort(rng.choice(N, n_per_iter, replace=False))
                     for _ in range(n_iters)], dtype=np.int32).reshape(
                         n_iters, n_per_iter)


def sketch_matrices(N, l, n_iters, seed=0):
    """Standard normal test matrices of the randomised range finder, one
    N x l matrix per iteration: shape (n_iters, N, l) (seed)."""
    return np.random.default_rng(seed).standard_normal((n_iters, N, l))


def smooth_random_field(shape, corr, seed):
    """Unit-variance periodic Gaussian random field with covariance
    exp(-r^2 / (2 corr^2)), synthesised spectrally on the given grid."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    k2 = np.zeros(shape)
    for ax, n in enumerate(shape):
        k = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
        shp = [1] * len(shape)
        shp[ax] = -1
        k2 = k2 + k.reshape(shp) ** 2
    filt = np.exp(-0.25 * corr * corr * k2)
    g = np.fft.ifftn(np.fft.fftn(white) * filt).real
    g -= g.mean()
    sd = g.std()
    return g / sd if sd > 0 else g


def grf2d(n=64, ratio=4, N=8, K=3, T=0.25, seed=0, dtype="f32",
          compensated=True):
    """Smooth random medium c = exp(0.3 g), g a unit GRF of correlation
    length 0.1, with a random Gaussian pulse (the batched-problem recipe)."""
    g = smooth_random_field((n, n), 0.1, 1000 + seed)
    c = np.exp(0.3 * g)
    rng = np.random.default_rng(2000 + seed)
    x0, y0 = rng.uniform(0, 1, size=2)
    s = rng.uniform(0.02, 0.05)
    Y, X = _axes((n, n))
    dxp = (X - x0 + 0.5) % 1.0 - 0.5
    dyp = (Y - y0 + 0.5) % 1.0 - 0.5
    u0 = np.exp(-(dxp ** 2 + dyp ** 2) / (2 * s * s))
    p0 = np.zeros((n, n))
    m_f = _steps_for_courant(float(c.max()), n, T / N)
    return Workload("grf2d", (n, n), ratio, T, N, m_f, m_f // 4, K, 1e-13, 4,
                    dtype, compensated, c, u0, p0)


def batch2d(n_problems=32, sizes=(256, 384, 512, 768, 1024), N=32, K=6,
            T=1.0, seed=0, dtype="f32", compensated=True):
    """The batched-problem recipe: n_problems independent 2D problems whose
    fine grids are drawn uniformly from `sizes` (seed), each with a smooth
    random medium c = exp(0.3 g) (g a unit Gaussian random field of
    correlation length 0.1, seed 1000+b) and a random Gaussian pulse
    (centre ~ U[0,1)^2, sigma ~ U[0.02, 0.05], seed 2000+b); coarse = fine/4,
    N = 32 slices, Courant number <= 0.5 (m_F a multiple of 4, m_C = m_F/4)."""
    grids = np.random.default_rng(seed).choice(np.asarray(sizes), n_problems)
    out = []
    for b, n in enumerate(grids):
        w = grf2d(n=int(n), ratio=4, N=N, K=K, T=T, seed=b, dtype=dtype,
                  compensated=compensated)
        w.name = f"batch2d[{b}]"
        out.append(w)
    return out


def ricker_pulse(shape, centre, freq):
    """(1 - 2 a) exp(-a), a = (pi f r)^2, r the periodic distance to
    `centre` (given in numpy axis order)."""
    grids = _axes(shape)
    r2 = np.zeros(shape)
    for g, x0 in zip(grids, centre):
        d = (g - x0 + 0.5) % 1.0 - 0.5
        r2 = r2 + d * d
    a = (np.pi * freq) ** 2 * r2
    return (1.0 - 2.0 * a) * np.exp(-a)


def random_pulses(shape, n, seed, sigma=(0.02, 0.05)):
    """n seeded states (u, p) of Gaussian pulses at random centres with
    widths drawn from `sigma` (the batched-problem recipe's pulse), p a
    second pulse of random amplitude; periodic distances."""
    rng = np.random.default_rng(seed)
    grids = _axes(shape)
    us, ps = [], []
    for _ in range(n):
        fields = []
        for _ in range(2):
            x0 = rng.uniform(0, 1, size=len(shape))
            s = rng.uniform(*sigma)
            r2 = np.zeros(shape)
            for g, c in zip(grids, x0):
                d = (g - c + 0.5) % 1.0 - 0.5
                r2 = r2 + d * d
            fields.append(np.exp(-r2 / (2 * s * s)))
        us.append(fields[0])
        ps.append(rng.uniform(-2, 2) * fields[1])
    return np.stack(us), np.stack(ps)


def misfit_case(shape=(32, 32), ratio=4, N=4, K=2, T=0.25, m_fine=8,
                m_coarse=2, tol=1e-6, seed=0, dtype="f64"):
    """A small receiver-misfit problem: c = 1.2 + 0.3 prod_axes
    sin/cos(2 pi x), Ricker-shaped initial pulse (peak frequency 4) at
    0.3 along the first numpy axis and 0.5 along the others, receivers
    every second node along x at 3/4 of every other axis, data
    0.01 * N(0, 1) of shape (N, n_receivers) (seed).
    Returns (Workload, receivers (int64 flat fine indices), data)."""
    shape = tuple(int(n) for n in shape)
    grids = _axes(shape)
    prod = np.ones(shape)
    for i, g in enumerate(grids):
        prod = prod * (np.sin(2 * np.pi * g) if i % 2 == 0
                       else np.cos(2 * np.pi * g))
    c = 1.2 + 0.3 * prod
    centre = [0.3] + [0.5] * (len(shape) - 1)
    u0 = ricker_pulse(shape, centre, 4.0)
    p0 = np.zeros(shape)
    nx = shape[-1]
    base = 0
    stride = 1
    for ax in range(len(shape) - 1, -1, -1):
        if ax != len(shape) - 1:
            base += (3 * shape[ax] // 4) * stride
        stride *= shape[ax]
    receivers = (base + np.arange(0, nx, 2)).astype(np.int64)
    data = 0.01 * np.random.default_rng(seed).standard_normal(
        (N, receivers.size))
    w = Workload("misfit_case", shape, ratio, T, N, m_fine, m_coarse, K, tol,
                 4, dtype, False, c, u0, p0)
    return w, receivers, data


def forced_misfit_case(shape=(32, 32), ratio=4, N=4, K=2, T=0.25, m_fine=8,
                       m_coarse=2, tol=1e-6, seed=0, dtype="f64", width=0.2,
                       c_max=2.0):
    """A small misfit problem with an absorbing layer and a point source:
    the medium and receivers of misfit_case, zero initial state, a layer of
    the given width (sigma_max for c_max, round trip 1e-3), a Ricker source
    (peak frequency 8, peak time 0.05) at x = 0.5, y = 0.3 (2D; 0.3 along x
    in 1D) and data 0.01 * N(0, 1) of shape (N, m_fine, n_receivers) for a
    record sampled every fine step (seed).  Returns (Workload, receivers,
    data, forcing) with forcing a dict of the layer and source parameters
    (x first)."""
    w, receivers, _ = misfit_case(shape, ratio, N, K, T, m_fine, m_coarse,
                                  tol, seed, dtype)
    w.name = "forced_misfit_case"
    w.u0 = np.zeros(w.shape)
    w.p0 = np.zeros(w.shape)
    pos = (0.3,) if len(w.shape) == 1 else (0.5, 0.3) + (0.5,) * (len(w.shape) - 2)
    forcing = {"width": width, "reflection": 1e-3, "src_pos": pos,
               "freq": 8.0, "t0": 0.05, "c_max": c_max}
    data = 0.01 * np.random.default_rng(seed).standard_normal(
        (N, m_fine, receivers.size))
    return w, receivers, data, forcing


def misfit_medium(shape, seed):
    """c = 1 + 2 s, s a min-max normalised Gaussian random field of
    correlation length 0.1 (seed)."""
    g = smooth_random_field(shape, 0.1, seed)
    s = (g - g.min()) / (g.max() - g.min())
    return 1.0 + 2.0 * s


def misfit2d(n=512, ratio=4, N=32, K=4, T=1.0, dtype="f32",
             compensated=True, n_receivers=128):
    """The full-size receiver-misfit workload with an absorbing layer and a
    point source: medium seed 0 (target medium misfit_medium(shape, 1) for
    the data), zero initial state, a layer of width 0.05 on every face
    (round trip 1e-3 at c_max = 3, the medium's upper bound), a Ricker
    source of peak frequency 10 and peak time 0.1 at (0.5, 0.1), 128
    receivers at x = (i + 1/2) / 128, y = 0.9 (nearest nodes), the record
    sampled every fine step.  Returns (Workload, receivers, target medium,
    forcing) with forcing a dict of the layer and source parameters (x
    first)."""
    shape = (n, n)
    c = misfit_medium(shape, 0)
    target = misfit_medium(shape, 1)
    u0 = np.zeros(shape)
    p0 = np.zeros(shape)
    m_f = _steps_for_courant(3.0, n, T / N)
    xs = np.floor((np.arange(n_receivers) + 0.5) / n_receivers * n + 0.5)
    y = int(np.floor(0.9 * n + 0.5))
    receivers = (y * n + xs.astype(np.int64)).astype(np.int64)
    w = Workload("misfit2d", shape, ratio, T, N, m_f, m_f // 4, K, 1e-13, 4,
                 dtype, compensated, c, u0, p0)
    forcing = {"width": 0.05, "reflection": 1e-3, "src_pos": (0.5, 0.1),
               "freq": 10.0, "t0": 0.1, "c_max": 3.0}
    return w, receivers, target, forcing


BY_NAME = {"wave1d": wave1d, "disc2d": disc2d, "layers3d": layers3d,
           "grf2d": grf2d, "batch2d": batch2d, "misfit2d": misfit2d}
