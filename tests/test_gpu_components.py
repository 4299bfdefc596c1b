"""Parity of each building block of the HIP path with the FP64 oracle,
through the C ABI.  Sizes span several tiles and a ragged tail.

Tolerances: FP64 path 1e-12 relative (the bound stated for the FP64
method); FP32 path 1e-5 relative in the energy norm, with both sides
starting from the same FP32-rounded numbers.
"""

import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import problem_pair, rel_energy_err, to_np

pytestmark = pytest.mark.gpu


def _solver(w, **kw):
    import paper_1905_00473_amd as pw
    P, Q = problem_pair(w, **kw)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    return s, Q


def _rand_states(rng, n, shape, dtype):
    import torch
    u = rng.standard_normal((n,) + shape)
    p = rng.standard_normal((n,) + shape)
    td = torch.float64 if dtype == "f64" else torch.float32
    return (torch.tensor(u, dtype=td, device="cuda"),
            torch.tensor(p, dtype=td, device="cuda"))


# ---------------------------------------------------------------------------
# F and C (Sec. 3.1)
# ---------------------------------------------------------------------------
CASES = [
    ("1d-f64", lambda: W.wave1d(), "f64"),
    ("2d-f64", lambda: W.disc2d(n=72, ratio=4, N=4, K=2, T=0.25), "f64"),
    ("2d-f32c", lambda: W.disc2d(n=72, ratio=4, N=4, K=2, T=0.25), "f32"),
    ("3d-f64", lambda: W.layers3d(n=40, ratio=4, N=4, K=2, T=0.06), "f64"),
    ("3d-f32c", lambda: W.layers3d(n=40, ratio=4, N=4, K=2, T=0.06), "f32"),
]


@pytest.mark.parametrize("name,make,dtype", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("grid", ["fine", "coarse"])
def test_propagator_parity(name, make, dtype, grid):
    import paper_1905_00473_amd as pw
    w = make()
    s, Q = _solver(w, dtype=dtype, compensated=True)
    rng = np.random.default_rng(1)
    fine = grid == "fine"
    shape = w.shape if fine else w.coarse_shape
    # smooth states: a few Fourier modes (the scheme's own regime)
    nst = 3
    grids = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    us, ps = [], []
    for _ in range(nst):
        ph = sum(2 * np.pi * rng.integers(1, 4) * g for g in grids)
        us.append(np.cos(ph + rng.uniform()) + 0.1 * rng.standard_normal())
        ps.append(np.sin(ph) * rng.uniform(0.5, 2))
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    u = torch.tensor(np.stack(us), dtype=td, device="cuda")
    p = torch.tensor(np.stack(ps), dtype=td, device="cuda")
    uo, po = s.propagate(u, p, pw.FINE if fine else pw.COARSE)
    c = w.c if fine else O.restrict(w.c, w.ratio)
    dx = Q.dx_fine if fine else Q.dx_coarse
    h = Q.dt_fine if fine else Q.dt_coarse
    m = Q.m_fine if fine else Q.m_coarse
    c2 = c * c
    if dtype == "f32":
        c2 = c2.astype(np.float32).astype(np.float64)
    for k in range(nst):
        ru, rp = O.propagate(to_np(u[k]), to_np(p[k]), c2, h, dx, m)
        err = rel_energy_err(to_np(uo[k]), to_np(po[k]), ru, rp, c, dx)
        tol = 1e-12 if dtype == "f64" else 1e-5
        assert err < tol, (name, grid, k, err)
        scale = np.max(np.abs(ru))
        assert np.max(np.abs(to_np(uo[k]) - ru)) / scale < (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("m", [1, 7, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_propagator_parity_3d_ragged(dtype, m):
    """3D F on a grid of unequal sides that are not multiples of the
    streaming blocks' output columns and rows, for step counts that end on
    a partial launch (7), on whole launches (8) and within one launch (1):
    the last launch of a slice runs its own block geometry."""
    import torch
    import paper_1905_00473_amd as pw
    shape = (26, 50, 72)  # (z, y, x)
    h = 0.004  # c dt / dx <= 1.5 * 0.004 * 72 = 0.43 (3D bound 1/sqrt 3)
    P = pw.Problem.make(shape, 2, 4 * m * h, 4, m, m, 2, 1e-14, dtype,
                        dtype == "f32", 1)
    Q = O.Problem(shape, 2, 4 * m * h, 4, m, m, 2, 1e-14)
    g = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    c = 1.0 + 0.3 * np.sin(2 * np.pi * g[2]) * np.cos(2 * np.pi * g[1]) + 0.1 * g[0]
    s = pw.Solver(P)
    s.set_medium(c)
    rng = np.random.default_rng(5)
    us, ps = [], []
    for _ in range(3):
        ph = sum(2 * np.pi * rng.integers(1, 4) * x for x in g)
        us.append(np.cos(ph + rng.uniform()) + 0.1 * rng.standard_normal(shape))
        ps.append(np.sin(ph) * rng.uniform(0.5, 2))
    td = torch.float64 if dtype == "f64" else torch.float32
    u = torch.tensor(np.stack(us), dtype=td, device="cuda")
    p = torch.tensor(np.stack(ps), dtype=td, device="cuda")
    uo, po = s.propagate(u, p)
    c2 = c * c
    if dtype == "f32":
        c2 = c2.astype(np.float32).astype(np.float64)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for k in range(3):
        ru, rp = O.propagate(to_np(u[k]), to_np(p[k]), c2, Q.dt_fine, Q.dx_fine, m)
        err = rel_energy_err(to_np(uo[k]), to_np(po[k]), ru, rp, c, Q.dx_fine)
        assert err < tol, (dtype, m, k, err)
        assert np.max(np.abs(to_np(uo[k]) - ru)) / np.max(np.abs(ru)) < tol
    s.close()


def test_batched_equals_single_bitwise():
    import torch
    w = W.disc2d(n=72, ratio=4, N=4, K=2, T=0.25)
    s, _ = _solver(w, dtype="f32", compensated=True)
    rng = np.random.default_rng(2)
    u, p = _rand_states(rng, 4, w.shape, "f32")
    ub, pb = s.propagate(u, p)
    for k in range(4):
        u1, p1 = s.propagate(u[k:k + 1].contiguous(), p[k:k + 1].contiguous())
        assert torch.equal(u1[0], ub[k]) and torch.equal(p1[0], pb[k])


# ---------------------------------------------------------------------------
# restriction + energy components (eqs. matrixF / matrixG)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [2, 4, 6, 8, "spectral"])
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_energy_components_parity(dim, order):
    import paper_1905_00473_amd as pw
    import torch
    w = {1: lambda: W.wave1d(), 2: lambda: W.disc2d(n=72, N=4, K=2, T=0.25),
         3: lambda: W.layers3d(n=40, N=4, K=2, T=0.06)}[dim]()
    w.grad_order = order
    s, Q = _solver(w, dtype="f64")
    rng = np.random.default_rng(3)
    u, p = _rand_states(rng, 3, w.shape, "f64")
    cols = s.energy_components(u, p, pw.FINE)
    cc = O.restrict(w.c, w.ratio)
    for k in range(3):
        ref = O.energy_components(O.restrict(to_np(u[k]), w.ratio),
                                  O.restrict(to_np(p[k]), w.ratio), cc,
                                  Q.dx_coarse, order)
        np.testing.assert_allclose(to_np(cols[k]), ref, rtol=1e-13,
                                   atol=1e-13 * np.max(np.abs(ref)))
    Uc = torch.tensor(rng.standard_normal((2,) + w.coarse_shape), device="cuda")
    Pc = torch.tensor(rng.standard_normal((2,) + w.coarse_shape), device="cuda")
    cols = s.energy_components(Uc, Pc, pw.COARSE)
    for k in range(2):
        ref = O.energy_components(to_np(Uc[k]), to_np(Pc[k]), cc, Q.dx_coarse,
                                  order)
        np.testing.assert_allclose(to_np(cols[k]), ref, rtol=1e-13,
                                   atol=1e-13 * np.max(np.abs(ref)))


# ---------------------------------------------------------------------------
# trigonometric interpolation + update (Algorithm 3, last line)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,dtype", [(1, "f64"), (2, "f64"), (2, "f32"),
                                       (3, "f64")])
def test_interp_add_parity(dim, dtype):
    import torch
    w = {1: lambda: W.wave1d(), 2: lambda: W.disc2d(n=72, N=4, K=2, T=0.25),
         3: lambda: W.layers3d(n=40, N=4, K=2, T=0.06)}[dim]()
    s, Q = _solver(w, dtype=dtype, compensated=False)
    rng = np.random.default_rng(4)
    n = 3
    du = torch.tensor(rng.standard_normal((n,) + w.coarse_shape), device="cuda")
    dp = torch.tensor(rng.standard_normal((n,) + w.coarse_shape), device="cuda")
    td = torch.float64 if dtype == "f64" else torch.float32
    v = torch.tensor(rng.standard_normal((n,) + w.shape), dtype=td, device="cuda")
    vp = torch.tensor(rng.standard_normal((n,) + w.shape), dtype=td, device="cuda")
    uo, po = s.interp_add(du, dp, v, vp)
    for k in range(n):
        a = to_np(du[k])
        if dtype == "f32":
            a = a.astype(np.float32).astype(np.float64)
        ref = to_np(v[k]) + O.interp(a, w.ratio)
        tol = 1e-13 if dtype == "f64" else 2e-6
        np.testing.assert_allclose(to_np(uo[k]), ref, atol=tol * np.max(np.abs(ref)))
        # R I = 1 at the coarse nodes, bit for bit
        got = O.restrict(to_np(uo[k]), w.ratio)
        want = O.restrict(to_np(v[k]), w.ratio) + a
        if dtype == "f32":
            want = want.astype(np.float32).astype(np.float64)
        assert np.array_equal(got, want)
    # zero correction leaves v untouched exactly
    z = torch.zeros_like(du)
    uo, _ = s.interp_add(z, z, v, vp)
    assert torch.equal(uo, v)


# ---------------------------------------------------------------------------
# Lambda^dag (Algorithm 2)
# ---------------------------------------------------------------------------
G2F_CASES = {
    # coarse axes of power-of-two length go through the FFT, the others
    # through the direct transform
    "1d_fft": lambda: W.wave1d(),
    "2d_direct": lambda: W.disc2d(n=72, N=4, K=2, T=0.25),
    "2d_fft": lambda: W.disc2d(n=128, N=4, K=2, T=0.25),
    "2d_mixed": lambda: W.misfit_case((40, 64), ratio=4, N=4, K=1, m_fine=16,
                                      m_coarse=4)[0],
    "3d_direct": lambda: W.layers3d(n=40, N=4, K=2, T=0.06),
    "3d_fft": lambda: W.layers3d(n=32, N=4, K=2, T=0.06),
}


@pytest.mark.parametrize("case", list(G2F_CASES))
def test_grad2func_parity(case):
    import torch
    w = G2F_CASES[case]()
    dim = len(w.shape)
    s, Q = _solver(w, dtype="f64")
    rng = np.random.default_rng(5)
    n = 3
    nc = int(np.prod(w.coarse_shape))
    q = torch.tensor(rng.standard_normal((n, dim * nc)), device="cuda")
    sums = torch.tensor(rng.standard_normal(n), device="cuda")
    out = s.grad2func(q, sums)
    for k in range(n):
        qs = [to_np(q[k])[a * nc:(a + 1) * nc].reshape(w.coarse_shape)
              for a in range(dim)]
        ref = O.grad2func(qs, float(sums[k]), Q.dx_coarse)
        np.testing.assert_allclose(to_np(out[k]), ref,
                                   atol=1e-13 * max(1.0, np.max(np.abs(ref))))


# ---------------------------------------------------------------------------
# Algorithm 1: compare Omega = U V^T (unique), never U or V themselves
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_update_svd_parity(tol):
    import torch
    w = W.wave1d()
    s, Q = _solver(w, dtype="f64", tol=tol, max_iters=4)
    rows = 2 * 64
    rng = np.random.default_rng(6)
    U = S = V = None
    # data with a decaying spectrum, like the method's snapshots
    for it in range(4):
        basis = rng.standard_normal((rows, 40)) * (0.5 ** np.arange(40))
        F = basis @ rng.standard_normal((40, w.N))
        G = F + 0.05 * (basis @ rng.standard_normal((40, w.N)))
        U, S, V = O.update_svd(U, S, V, F, G, tol)
        r = s.update_svd(torch.tensor(F.T.copy(), device="cuda"),
                         torch.tensor(G.T.copy(), device="cuda"), reset=(it == 0))
        Ug, Sg, Vg = s.corrector()
        assert r == len(S), (it, r, len(S))
        np.testing.assert_allclose(to_np(Sg), S, rtol=1e-9, atol=1e-12 * S[0])
        # Omega-action on the data agrees within conditioning
        Om_ref = U @ V.T
        Om = to_np(Ug).T @ to_np(Vg)
        np.testing.assert_allclose(Om @ G, Om_ref @ G,
                                   atol=1e-9 * np.max(np.abs(G)))
        ortho = to_np(Ug) @ to_np(Ug).T
        np.testing.assert_allclose(ortho, np.eye(r), atol=1e-12)


# ---------------------------------------------------------------------------
# the orthonormalisation inside Algorithm 1 at awkward shapes: Householder
# TSQR chunking (rows below, at and just above one chunk of 256, many
# chunks), more than 64 columns (blocked), fewer rows than columns
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nc,ncols", [(50, 7), (128, 64), (129, 64),
                                      (2500, 33), (70, 65), (300, 130),
                                      (6, 24), (50, 130), (40, 100)])
def test_update_svd_qr_shapes(nc, ncols):
    """1D problems with rows = 2 nc; data with a steep spectrum (so the
    FP64 path takes the Householder TSQR), two updates against the oracle:
    singular values 1e-9, Omega-action on the data 1e-9 of its size, U
    orthonormal to 1e-12."""
    import paper_1905_00473_amd as pw
    import torch
    print(f"qr shapes nc={nc} ncols={ncols}", flush=True)
    rows = 2 * nc
    m_c = int(np.ceil(2 * nc / ncols))       # c dt / dx <= 1/2 on one grid
    P = pw.Problem.make((nc,), 1, 1.0, ncols, 4 * m_c, m_c, 4, 1e-6, "f64",
                        False, 2)
    s = pw.Solver(P)
    s.set_medium(np.ones(nc))
    rng = np.random.default_rng(nc + ncols)
    U = S = V = None
    k = min(rows, 40)
    for it in range(2):
        basis = rng.standard_normal((rows, k)) * (0.55 ** np.arange(k))
        F = basis @ rng.standard_normal((k, ncols))
        G = F + 0.05 * (basis @ rng.standard_normal((k, ncols)))
        U, S, V = O.update_svd(U, S, V, F, G, 1e-6)
        r = s.update_svd(torch.tensor(F.T.copy(), device="cuda"),
                         torch.tensor(G.T.copy(), device="cuda"),
                         reset=(it == 0))
        Ug, Sg, Vg = s.corrector()
        assert r == len(S), (it, r, len(S))
        np.testing.assert_allclose(to_np(Sg), S, rtol=1e-9, atol=1e-12 * S[0])
        Ug, Vg = to_np(Ug).T, to_np(Vg).T
        d = np.abs(Ug @ (Vg.T @ G) - U @ (V.T @ G)).max() / np.abs(G).max()
        assert d < 1e-9, (it, d)
        # with more columns than rows the new QR basis is completed by
        # noise directions that overlap the old basis; how much of them the
        # rotated basis keeps is set by the rounding of the core SVD
        # (measured 7e-12 for 2 x 40 rows and 100 columns)
        np.testing.assert_allclose(Ug.T @ Ug, np.eye(r),
                                   atol=1e-12 if rows >= ncols else 1e-10)
    s.close()


def test_update_svd_tied_norms():
    """Algorithm 1 when the core matrix has columns of equal norm (the SVD
    orders every sweep by column norm, ties by index): data F = G = 2 Q_k
    with orthonormal Q_k give a core 4 I (every norm tied, no rotation),
    then a random update mixes the tied block.  Against the oracle as
    above: singular values 1e-9, Omega-action 1e-9, U orthonormal 1e-12."""
    import paper_1905_00473_amd as pw
    import torch
    nc, ncols = 64, 48
    rows = 2 * nc
    m_c = int(np.ceil(2 * nc / ncols))
    P = pw.Problem.make((nc,), 1, 1.0, ncols, 4 * m_c, m_c, 4, 1e-6, "f64",
                        False, 3)
    s = pw.Solver(P)
    s.set_medium(np.ones(nc))
    rng = np.random.default_rng(11)
    Qm, _ = np.linalg.qr(rng.standard_normal((rows, rows)))
    data = [2.0 * Qm[:, :ncols], 2.0 * Qm[:, ncols:2 * ncols]]
    basis = rng.standard_normal((rows, 30)) * (0.6 ** np.arange(30))
    data.append(basis @ rng.standard_normal((30, ncols)))
    U = S = V = None
    for it, F in enumerate(data):
        G = F if it < 2 else F + 0.05 * (basis @ rng.standard_normal((30, ncols)))
        U, S, V = O.update_svd(U, S, V, F, G, 1e-6)
        r = s.update_svd(torch.tensor(F.T.copy(), device="cuda"),
                         torch.tensor(G.T.copy(), device="cuda"),
                         reset=(it == 0))
        Ug, Sg, Vg = s.corrector()
        assert r == len(S), (it, r, len(S))
        np.testing.assert_allclose(to_np(Sg), S, rtol=1e-9, atol=1e-12 * S[0])
        Ug, Vg = to_np(Ug).T, to_np(Vg).T
        d = np.abs(Ug @ (Vg.T @ G) - U @ (V.T @ G)).max() / np.abs(G).max()
        assert d < 1e-9, (it, d)
        np.testing.assert_allclose(Ug.T @ Ug, np.eye(r), atol=1e-12)
    s.close()
