"""Parity of the FP64 energy reductions on the fine grid (the error measure
of the Sec. 6 preamble: the discrete energy of eq. discrete-wave-energy,
and the l2 norm of the displacement) with the oracle, through pw_energy
and pw_error_norms, in 1D, 2D and 3D, for every central-difference order
and both state dtypes.  The grids have ragged sizes (no multiple of the
reduction's block size).  Gate: 1e-12 relative (FP64 sums of the same
products in another order)."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_helpers import problem_pair

pytestmark = pytest.mark.gpu

CASES = {
    "1d": lambda: W.wave1d(n=300, ratio=4, N=4, K=1),
    "2d": lambda: W.disc2d(n=72, ratio=4, N=4, K=1, T=0.25, dtype="f64",
                           compensated=False),
    "3d": lambda: W.layers3d(n=28, ratio=4, N=4, K=1, T=0.05, dtype="f64",
                             compensated=False),
}


def _fields(rng, shape, dtype, smooth):
    x = rng.standard_normal(shape)
    if smooth:
        # a few low Fourier modes plus a constant (the constant is invisible
        # to the gradient part and must show up in the l2 sums only)
        k = np.fft.fftn(x)
        mask = np.zeros(shape, bool)
        mask[tuple(slice(0, 3) for _ in shape)] = True
        x = np.fft.ifftn(np.where(mask, k, 0)).real * 5 + 0.3
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    return x


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("order", [2, 4, 6, 8])
@pytest.mark.parametrize("case", list(CASES))
def test_energy_and_l2_parity(case, order, dtype):
    import torch

    import paper_1905_00473_amd as pw
    w = CASES[case]()
    w.grad_order = order
    P, Q = problem_pair(w, dtype=dtype, compensated=False)
    s = pw.Solver(P)
    s.set_medium(w.c)
    rng = np.random.default_rng(5 + order)
    td = torch.float64 if dtype == "f64" else torch.float32
    for smooth in (False, True):
        u, p, ur, pr = (_fields(rng, w.shape, dtype, smooth) for _ in range(4))
        dev = [torch.tensor(a, dtype=td, device="cuda") for a in (u, p, ur, pr)]
        ed, er = s.energy(*dev)
        e_ref = O.energy(u - ur, p - pr, w.c, Q.dx_fine, order)
        e0_ref = O.energy(ur, pr, w.c, Q.dx_fine, order)
        assert abs(ed - e_ref) <= 1e-12 * e_ref, (ed, e_ref)
        assert abs(er - e0_ref) <= 1e-12 * e0_ref, (er, e0_ref)
        # single-state form (no reference)
        e1, _ = s.energy(dev[0], dev[1])
        e1_ref = O.energy(u, p, w.c, Q.dx_fine, order)
        assert abs(e1 - e1_ref) <= 1e-12 * e1_ref
        nm = s.error_norms(*dev)
        assert nm["E_diff"] == ed and nm["E_ref"] == er
        d2 = float(np.sum((u - ur) ** 2))
        r2 = float(np.sum(ur ** 2))
        assert abs(nm["l2_diff2"] - d2) <= 1e-12 * d2
        assert abs(nm["l2_ref2"] - r2) <= 1e-12 * r2
        assert abs(nm["l2"] - O.l2_error(u, ur)) <= 1e-12 * O.l2_error(u, ur)
        assert abs(nm["energy"] - O.energy_error(u, p, ur, pr, w.c,
                                                   Q.dx_fine, order)) \
            <= 1e-12 * nm["energy"]
    s.close()


def test_energy_blind_to_constant_shift_l2_is_not():
    """A constant offset of u is invisible to the energy semi-norm (the
    reason the end-to-end tests also compare in l2)."""
    import torch

    import paper_1905_00473_amd as pw
    w = CASES["2d"]()
    P, Q = problem_pair(w, dtype="f64", compensated=False)
    s = pw.Solver(P)
    s.set_medium(w.c)
    rng = np.random.default_rng(3)
    # values on a 2^-20 lattice, so that u + 1/4 - u is exactly 1/4
    u = np.round(rng.standard_normal(w.shape) * 2 ** 20) / 2 ** 20
    p = rng.standard_normal(w.shape)
    a = [torch.tensor(x, device="cuda") for x in (u + 0.25, p, u, p)]
    nm = s.error_norms(*a)
    assert nm["E_diff"] == 0.0
    assert abs(nm["l2_diff2"] - 0.0625 * u.size) <= 1e-12 * 0.0625 * u.size
    s.close()
