"""MI355X (gfx950) implementation of the stabilised parareal-like method for
the second-order wave equation (Nguyen & Tsai, arXiv 1905.00473).

Thin Python binding over the C ABI of ``libpwave.so`` (include/pw.h):
argument marshalling only.  Every step of the method runs in the HIP
kernels of the library; torch is used for device memory and the stream.
There is no CPU fallback: if the library is missing or fails to load, every
call raises.
"""

from __future__ import annotations

import ctypes
import os

__all__ = ["Problem", "Solver", "lib", "PwError", "LIB_PATH", "F32", "F64",
           "FINE", "COARSE", "PararealTraces", "require", "DIAG_FIELDS"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "libpwave.so")
F32, F64 = 0, 1
FINE, COARSE = 0, 1
PERIODIC, SPONGE = 0, 1

_STATUS = {0: "PW_OK", -1: "PW_EINVAL", -2: "PW_EUNSTABLE", -3: "PW_ENOMEM",
           -4: "PW_EHIP", -5: "PW_ESTATE", -6: "PW_ENUMERIC"}


class PwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    """Mirror of pw_problem (include/pw.h)."""
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n_fine", ctypes.c_int * 3),
        ("ratio", ctypes.c_int),
        ("T", ctypes.c_double),
        ("n_slices", ctypes.c_int),
        ("m_fine", ctypes.c_int),
        ("m_coarse", ctypes.c_int),
        ("grad_order", ctypes.c_int),
        ("svd_tol", ctypes.c_double),
        ("state_dtype", ctypes.c_int),
        ("compensated", ctypes.c_int),
        ("max_iters", ctypes.c_int),
        ("interp", ctypes.c_int),
        ("keep_history", ctypes.c_int),
        ("bc", ctypes.c_int),
        ("sponge_width", ctypes.c_double),
        ("sponge_reflection", ctypes.c_double),
        ("sponge_cmax", ctypes.c_double),
    ]

    @classmethod
    def make(cls, shape, ratio, T, N, m_fine, m_coarse, grad_order=4,
             tol=1e-14, dtype="f64", compensated=False, max_iters=8,
             interp="trig", keep_history=False, sponge_width=0.0,
             sponge_reflection=0.0, sponge_cmax=0.0):
        """shape: fine grid in numpy order (x last); interp: "trig",
        "linear" or "cubic"; keep_history: keep every iterate u^k_n;
        sponge_width > 0: an absorbing layer of that width (PW_SPONGE, 2D;
        reflection 0 means 1e-3, cmax 0 the medium's largest c)."""
        p = cls()
        p.dim = len(shape)
        xyz = list(reversed(shape)) + [1] * (3 - len(shape))
        for a in range(3):
            p.n_fine[a] = int(xyz[a])
        p.ratio = int(ratio)
        p.T = float(T)
        p.n_slices = int(N)
        p.m_fine = int(m_fine)
        p.m_coarse = int(m_coarse)
        p.grad_order = 0 if grad_order == "spectral" else int(grad_order)
        p.svd_tol = float(tol)
        p.state_dtype = F64 if dtype in ("f64", "float64", F64) else F32
        p.compensated = int(bool(compensated))
        p.max_iters = int(max_iters)
        p.interp = {"trig": 0, "linear": 1, "cubic": 2}.get(interp, interp)
        p.keep_history = int(bool(keep_history))
        if sponge_width > 0:
            p.bc = SPONGE
            p.sponge_width = float(sponge_width)
            p.sponge_reflection = float(sponge_reflection)
            p.sponge_cmax = float(sponge_cmax)
        return p


#: comparator iterations of Sec. 6 selectable with Solver.set_variant
VARIANTS = {"theta": 0, "omega_one": 1, "no_correction": 2, "plain": 3}

_LIB = None

_SIGS = {
    "pw_create": [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_void_p)],
    "pw_destroy": [ctypes.c_void_p],
    "pw_sync": [ctypes.c_void_p],
    "pw_set_medium": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_int],
    "pw_set_initial": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_int],
    "pw_run": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
               ctypes.POINTER(ctypes.c_int)],
    "pw_continue": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                    ctypes.c_double, ctypes.POINTER(ctypes.c_int)],
    "pw_get_iterate": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_int],
    "pw_set_iterate": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "pw_set_corrector": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                         ctypes.c_int],
    "pw_get_diagnostics": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                           ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "pw_error_norms": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p],
    "pw_save": [ctypes.c_void_p, ctypes.c_char_p],
    "pw_load": [ctypes.c_void_p, ctypes.c_char_p],
    "pw_get_tape_id": [ctypes.c_void_p, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_longlong)],
    "pw_launch_plan": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                       ctypes.POINTER(ctypes.c_int)],
    "pw_set_variant": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int],
    "pw_set_sketch": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_int, ctypes.c_int, ctypes.c_int],
    "pw_set_sampling": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                        ctypes.c_int, ctypes.c_int],
    "pw_get_state": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "pw_get_residuals": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_int)],
    "pw_serial_fine": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                       ctypes.c_void_p, ctypes.c_void_p],
    "pw_propagate": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_int],
    "pw_energy_components": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                             ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_int],
    "pw_interp_add": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "pw_grad2func": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "pw_update_svd": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                      ctypes.POINTER(ctypes.c_int)],
    "pw_get_corrector": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_int)],
    "pw_energy": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_double)],
    "pw_energy_noalloc": [ctypes.c_void_p] * 8,
    "pw_serial_fine_states": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p],
    "pw_set_source": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_double, ctypes.c_double],
    "pw_trace_sweep": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                       ctypes.c_int, ctypes.c_void_p, ctypes.c_int],
    "pw_backward_sweep": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                          ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_int, ctypes.c_int, ctypes.c_int],
    "pw_get_timings": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                       ctypes.c_int],
    "pw_run_batch": [ctypes.c_void_p, ctypes.c_int],
    "pw_batch_fine_sweeps": [ctypes.c_void_p, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_double)],
    "pw_get_batch_info": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                          ctypes.c_int],
    "pw_run_taped": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int],
    "pw_run_frozen": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int],
    "pw_traces": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_int, ctypes.c_void_p, ctypes.c_int],
    "pw_backward": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                    ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                    ctypes.c_int, ctypes.c_int, ctypes.c_int],
}

#: every symbol include/pw.h declares
SYMBOLS = sorted(list(_SIGS) + ["pw_last_error", "pw_version",
                                "pw_num_problems"])


def lib():
    """Load libpwave.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1905_00473_amd.build` (no fallback exists)")
        # torch (ROCm) carries its own HIP runtime beside the one the
        # library links; have torch's initialised before the library's is
        # loaded, the order of every torch-driven caller (loading the
        # library first has left its runtime reporting no device)
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.pw_last_error.restype = ctypes.c_char_p
        L.pw_last_error.argtypes = []
        L.pw_version.restype = ctypes.c_char_p
        L.pw_version.argtypes = []
        L.pw_num_problems.restype = ctypes.c_int
        L.pw_num_problems.argtypes = [ctypes.c_void_p]
        _LIB = L
    return _LIB


def _check(st):
    if st != 0:
        raise PwError(st, lib().pw_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


#: values per iteration of Solver.diagnostics (PW_DIAG_STRIDE)
DIAG_STRIDE = 8
DIAG_FIELDS = ("rho", "rank", "F2", "F_in2", "G_in2", "trace_S", "r2_min",
               "change")


def require(t, dtype, shape, name):
    """Check a tensor handed to the C ABI: a CUDA (HIP) tensor of the given
    torch dtype and shape, contiguous.  Raises ValueError before any device
    work (the library reads and writes exactly the sizes the problem
    implies, so a mismatch would read or write out of bounds)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device (cuda) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return t


class Solver:
    """A context of one or more wave problems on the current CUDA (HIP)
    device and stream."""

    def __init__(self, problems):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("pwave needs a GPU (torch.cuda.is_available() "
                               "is False)")
        if isinstance(problems, Problem):
            problems = [problems]
        self.problems = list(problems)
        arr = (Problem * len(self.problems))(*self.problems)
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().pw_create(arr, len(self.problems),
                               ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(h)))
        self._h = h

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().pw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers ------------------------------------------------------------
    def dtype(self, prob=0):
        import torch
        return torch.float64 if self.problems[prob].state_dtype == F64 \
            else torch.float32

    def shape(self, prob=0):
        p = self.problems[prob]
        return tuple(reversed([p.n_fine[a] for a in range(p.dim)]))

    def coarse_shape(self, prob=0):
        p = self.problems[prob]
        return tuple(n // p.ratio for n in self.shape(prob))

    def rows(self, prob=0):
        import math
        p = self.problems[prob]
        return (p.dim + 1) * math.prod(self.coarse_shape(prob))

    def _dev(self, x, dtype=None):
        import torch
        t = torch.as_tensor(x)
        return t.to(device="cuda", dtype=dtype or torch.float64).contiguous()

    # -- the method -----------------------------------------------------------
    def set_medium(self, c, prob=0):
        import torch
        t = self._dev(c, torch.float64)
        _check(lib().pw_set_medium(self._h, prob, _ptr(t), 1))

    def set_initial(self, u0, p0, prob=0):
        import torch
        a, b = self._dev(u0, torch.float64), self._dev(p0, torch.float64)
        _check(lib().pw_set_initial(self._h, prob, _ptr(a), _ptr(b), 1))

    def run(self, K, prob=0, stop_tol=0.0):
        """Algorithm 3 from u0: coarse initialisation and up to K
        iterations (stop_tol > 0: stop once the change of the iterate falls
        to stop_tol).  Returns the number of iterations run."""
        kd = ctypes.c_int()
        _check(lib().pw_run(self._h, prob, int(K), float(stop_tol),
                            ctypes.byref(kd)))
        return kd.value

    def resume(self, K, update_corrector=True, stop_tol=0.0, prob=0):
        """Continue Algorithm 3 from the current iterate for up to K more
        iterations (update_corrector=False holds the corrector fixed).
        Returns k_done after the call."""
        kd = ctypes.c_int()
        _check(lib().pw_continue(self._h, prob, int(K),
                                 int(bool(update_corrector)),
                                 float(stop_tol), ctypes.byref(kd)))
        return kd.value

    def iterate(self, k, n, prob=0):
        """u^k_n, p^k_n of the last run (k = 1: coarse initialisation)."""
        import torch
        u = torch.empty(self.shape(prob), dtype=self.dtype(prob), device="cuda")
        p = torch.empty_like(u)
        _check(lib().pw_get_iterate(self._h, prob, int(k), int(n), _ptr(u),
                                    _ptr(p), 1))
        return u, p

    def set_iterate(self, n, u, p, prob=0):
        """Overwrite slice n (1..N) of the current iterate (float64 fields)."""
        import torch
        a, b = self._dev(u, torch.float64), self._dev(p, torch.float64)
        require(a, torch.float64, self.shape(prob), "u")
        require(b, torch.float64, self.shape(prob), "p")
        _check(lib().pw_set_iterate(self._h, prob, int(n), _ptr(a), _ptr(b), 1))

    def set_corrector(self, U, S, V, prob=0):
        """Replace the corrector: U, V (rank, rows), S (rank,) float64, rows
        of U and V the singular vectors."""
        import torch
        U = self._dev(U, torch.float64)
        V = self._dev(V, torch.float64)
        S = self._dev(S, torch.float64).reshape(-1)
        r = int(S.numel())
        require(U, torch.float64, (r, self.rows(prob)), "U")
        require(V, torch.float64, (r, self.rows(prob)), "V")
        _check(lib().pw_set_corrector(self._h, prob, _ptr(U), _ptr(S), _ptr(V),
                                      r, 1))

    def diagnostics(self, prob=0, cap=256):
        """Per-iteration record: a list of dicts with the DIAG_FIELDS."""
        buf = (ctypes.c_double * (DIAG_STRIDE * cap))()
        cnt = ctypes.c_int()
        _check(lib().pw_get_diagnostics(self._h, prob, buf, cap,
                                        ctypes.byref(cnt)))
        out = []
        for k in range(min(cnt.value, cap)):
            row = buf[DIAG_STRIDE * k:DIAG_STRIDE * (k + 1)]
            d = dict(zip(DIAG_FIELDS, row))
            d["rank"] = int(d["rank"])
            out.append(d)
        return out

    def save(self, path):
        _check(lib().pw_save(self._h, os.fsencode(path)))

    def load(self, path):
        _check(lib().pw_load(self._h, os.fsencode(path)))

    def launch_plan(self, n_states, grid=FINE, prob=0):
        """(launches, steps per launch) of one propagation of n_states."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().pw_launch_plan(self._h, prob, grid, int(n_states),
                                    ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def tape_id(self, prob=0):
        v = ctypes.c_longlong()
        _check(lib().pw_get_tape_id(self._h, prob, ctypes.byref(v)))
        return v.value

    def set_sampling(self, cols, prob=0):
        """Random subsampling of the data matrices: cols is a
        (n_iters, n_per_iter) integer table of slice columns per iteration
        (None switches sampling off)."""
        import numpy as np
        if cols is None:
            _check(lib().pw_set_sampling(self._h, prob, None, 0, 0))
            return
        a = np.ascontiguousarray(np.asarray(cols, dtype=np.int32))
        if a.ndim != 2:
            raise ValueError("cols must be a 2-D table (iterations x samples)")
        _check(lib().pw_set_sampling(
            self._h, prob, a.ctypes.data_as(ctypes.c_void_p),
            int(a.shape[1]), int(a.shape[0])))

    def set_sketch(self, omega, power=0, prob=0):
        """Randomised sketching inside Algorithm 1: omega is an (n_iters, N,
        l) array of test matrices, one per iteration (None switches it
        off); power = power iterations of the range finder."""
        import numpy as np
        if omega is None:
            _check(lib().pw_set_sketch(self._h, prob, None, 0, 0, 0))
            return
        a = np.asarray(omega, dtype=np.float64)
        if a.ndim != 3 or a.shape[1] != self.problems[prob].n_slices:
            raise ValueError("omega must be (n_iters, N, l)")
        cm = np.ascontiguousarray(np.transpose(a, (0, 2, 1)))  # N x l column-major
        _check(lib().pw_set_sketch(
            self._h, prob, cm.ctypes.data_as(ctypes.c_void_p), int(a.shape[2]),
            int(a.shape[0]), int(power)))

    def set_variant(self, variant, prob=0):
        """Iteration run by `run`: 'theta' (Algorithm 3), 'omega_one'
        (Omega = I), 'no_correction' or 'plain' (plain parareal)."""
        v = VARIANTS.get(variant, variant)
        _check(lib().pw_set_variant(self._h, prob, int(v)))

    def run_batch(self, K):
        """Algorithm 3 for all problems of the context in lockstep."""
        _check(lib().pw_run_batch(self._h, int(K)))

    def batch_fine_sweeps(self, reps=3):
        ms = ctypes.c_double()
        _check(lib().pw_batch_fine_sweeps(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    def batch_info(self):
        d, ly = ctypes.c_int(), ctypes.c_int()
        ms = (ctypes.c_double * 136)()
        _check(lib().pw_get_batch_info(self._h, ctypes.byref(d),
                                       ctypes.byref(ly), ms, 136))
        c = int(ms[7])
        by_size = {int(ms[8 + 2 * i]): int(ms[9 + 2 * i]) for i in range(c)}
        return dict(depth=d.value, rows_per_stream=ly.value,
                    parallel=ms[0], corrector=ms[1], sweep=ms[2],
                    total=ms[3], tune_ms=ms[4], tuned_sweep_ms=ms[5],
                    from_cache=bool(ms[6]), rows_per_stream_by_size=by_size)

    def sync(self):
        _check(lib().pw_sync(self._h))

    def state(self, n, prob=0):
        import torch
        u = torch.empty(self.shape(prob), dtype=self.dtype(prob), device="cuda")
        p = torch.empty_like(u)
        _check(lib().pw_get_state(self._h, prob, int(n), _ptr(u), _ptr(p), 1))
        return u, p

    def residuals(self, prob=0, cap=256):
        rho = (ctypes.c_double * cap)()
        rk = (ctypes.c_int * cap)()
        cnt = ctypes.c_int()
        _check(lib().pw_get_residuals(self._h, prob, rho, rk, cap,
                                      ctypes.byref(cnt)))
        return list(rho[:cnt.value]), list(rk[:cnt.value])

    def serial_fine(self, n, prob=0):
        import torch
        u = torch.empty(self.shape(prob), dtype=self.dtype(prob), device="cuda")
        p = torch.empty_like(u)
        _check(lib().pw_serial_fine(self._h, prob, int(n), _ptr(u), _ptr(p)))
        return u, p

    def serial_fine_states(self, prob=0):
        """(N + 1, *grid) u and p: the serial fine reference at every
        coupling time t_n, n = 0..N."""
        import torch
        N = self.problems[prob].n_slices
        u = torch.empty((N + 1,) + self.shape(prob), dtype=self.dtype(prob),
                        device="cuda")
        p = torch.empty_like(u)
        _check(lib().pw_serial_fine_states(self._h, prob, _ptr(u), _ptr(p)))
        return u, p

    def timings(self, prob=0):
        ms = (ctypes.c_double * 6)()
        _check(lib().pw_get_timings(self._h, prob, ms, 6))
        return dict(parallel=ms[0], corrector=ms[1], sweep=ms[2], total=ms[3],
                    taped=ms[4], backward=ms[5])

    # -- differentiation --------------------------------------------------------
    def run_taped(self, K, prob=0):
        """Algorithm 3 recording the tape the backward pass reads."""
        _check(lib().pw_run_taped(self._h, prob, int(K)))

    def run_frozen(self, K, prob=0):
        """Algorithm 3 with the correctors of the last taped run."""
        _check(lib().pw_run_frozen(self._h, prob, int(K)))

    def _receivers(self, receivers):
        import torch
        return torch.as_tensor(receivers).to(device="cuda",
                                             dtype=torch.int64).contiguous()

    def traces(self, receivers, prob=0):
        """(N, n_rec) float64: u_n at the receivers (flat fine indices)."""
        import torch
        rec = self._receivers(receivers)
        N = self.problems[prob].n_slices
        out = torch.empty((N, rec.numel()), dtype=torch.float64, device="cuda")
        _check(lib().pw_traces(self._h, prob, _ptr(rec), rec.numel(),
                               _ptr(out), 1))
        return out

    def set_source(self, pos, freq=10.0, t0=0.1, prob=0):
        """Ricker point source at the node nearest to pos (box coordinates,
        x first; None removes it), peak frequency freq, peak time t0."""
        if pos is None:
            _check(lib().pw_set_source(self._h, prob, None, 0.0, 0.0))
            return
        arr = (ctypes.c_double * len(pos))(*[float(x) for x in pos])
        _check(lib().pw_set_source(self._h, prob, arr, float(freq), float(t0)))

    def trace_sweep(self, receivers, prob=0):
        """(N, m_fine, n_rec) float64: u at the receivers after every fine
        step of one more F sweep from the current iterate (distinct flat
        fine indices)."""
        import torch
        rec = self._receivers(receivers)
        P = self.problems[prob]
        out = torch.empty((P.n_slices, P.m_fine, rec.numel()),
                          dtype=torch.float64, device="cuda")
        _check(lib().pw_trace_sweep(self._h, prob, _ptr(rec), rec.numel(),
                                    _ptr(out), 1))
        return out

    def backward_sweep(self, receivers, seed, wrt="c2", checkpoint_every=64,
                       prob=0):
        """Vector-Jacobian product of trace_sweep() through the last taped
        or frozen run (seed: (N, m_fine, n_rec))."""
        import torch
        rec = self._receivers(receivers)
        sd = self._dev(seed, torch.float64)
        g = torch.empty(self.shape(prob), dtype=torch.float64, device="cuda")
        _check(lib().pw_backward_sweep(self._h, prob, _ptr(rec), rec.numel(),
                                       _ptr(sd), _ptr(g), 1, int(wrt == "c"),
                                       int(checkpoint_every)))
        return g

    def backward(self, receivers, seed, wrt="c2", checkpoint_every=64,
                 prob=0):
        """Vector-Jacobian product of traces() through the last taped or
        frozen run: d/d c^2 (wrt="c2") or d/dc (wrt="c") of
        sum(seed * traces), on the fine grid (float64)."""
        import torch
        rec = self._receivers(receivers)
        sd = self._dev(seed, torch.float64)
        g = torch.empty(self.shape(prob), dtype=torch.float64, device="cuda")
        _check(lib().pw_backward(self._h, prob, _ptr(rec), rec.numel(),
                                 _ptr(sd), _ptr(g), 1, int(wrt == "c"),
                                 int(checkpoint_every)))
        return g

    def _state_args(self, prob, **fields):
        sh, dt = self.shape(prob), self.dtype(prob)
        for name, t in fields.items():
            if t is not None:
                require(t, dt, sh, name)

    def energy(self, u, p, u_ref=None, p_ref=None, prob=0):
        self._state_args(prob, u=u, p=p, u_ref=u_ref, p_ref=p_ref)
        if (u_ref is None) != (p_ref is None):
            raise ValueError("u_ref and p_ref go together")
        ed, er = ctypes.c_double(), ctypes.c_double()
        _check(lib().pw_energy(self._h, prob, _ptr(u), _ptr(p), _ptr(u_ref),
                               _ptr(p_ref), ctypes.byref(ed),
                               ctypes.byref(er)))
        return ed.value, er.value

    def error_norms(self, u, p, u_ref=None, p_ref=None, prob=0):
        """dict: energy error sqrt(E(d)/E(ref)), l2 error of u, and the raw
        sums E(d), E(ref), sum (u-u_ref)^2, sum u_ref^2."""
        import math
        self._state_args(prob, u=u, p=p, u_ref=u_ref, p_ref=p_ref)
        if (u_ref is None) != (p_ref is None):
            raise ValueError("u_ref and p_ref go together")
        out = (ctypes.c_double * 4)()
        _check(lib().pw_error_norms(self._h, prob, _ptr(u), _ptr(p),
                                    _ptr(u_ref), _ptr(p_ref), out))
        e, e0, d2, r2 = out[0], out[1], out[2], out[3]
        return dict(energy=math.sqrt(e / e0) if e0 > 0 else math.sqrt(e),
                    l2=math.sqrt(d2 / r2) if r2 > 0 else math.sqrt(d2),
                    E_diff=e, E_ref=e0, l2_diff2=d2, l2_ref2=r2)

    # -- building blocks (parity checks) --------------------------------------
    def propagate(self, u, p, grid=FINE, prob=0):
        """u, p: (n_states, *grid) tensors of the state dtype."""
        import torch
        sh = self.shape(prob) if grid == FINE else self.coarse_shape(prob)
        n = int(u.shape[0]) if getattr(u, "dim", lambda: 0)() > 0 else 0
        require(u, self.dtype(prob), (n,) + sh, "u")
        require(p, self.dtype(prob), (n,) + sh, "p")
        uo, po = torch.empty_like(u), torch.empty_like(p)
        _check(lib().pw_propagate(self._h, prob, grid, _ptr(u), _ptr(p),
                                  _ptr(uo), _ptr(po), int(u.shape[0])))
        return uo, po

    def energy_components(self, u, p, grid=FINE, prob=0):
        import torch
        n = int(u.shape[0]) if getattr(u, "dim", lambda: 0)() > 0 else 0
        sh = self.shape(prob) if grid == FINE else self.coarse_shape(prob)
        require(u, self.dtype(prob), (n,) + sh, "u")
        require(p, self.dtype(prob), (n,) + sh, "p")
        out = torch.empty((n, self.rows(prob)), dtype=torch.float64,
                          device="cuda")
        _check(lib().pw_energy_components(self._h, prob, grid, _ptr(u),
                                          _ptr(p), _ptr(out), n))
        return out

    def interp_add(self, du, dp, v=None, vp=None, prob=0):
        import torch
        n = int(du.shape[0]) if getattr(du, "dim", lambda: 0)() > 0 else 0
        cs = (n,) + self.coarse_shape(prob)
        require(du, torch.float64, cs, "du")
        require(dp, torch.float64, cs, "dp")
        shp = (n,) + self.shape(prob)
        if (v is None) != (vp is None):
            raise ValueError("v and vp go together")
        if v is not None:
            require(v, self.dtype(prob), shp, "v")
            require(vp, self.dtype(prob), shp, "vp")
        uo = torch.empty(shp, dtype=self.dtype(prob), device="cuda")
        po = torch.empty_like(uo)
        _check(lib().pw_interp_add(self._h, prob, _ptr(du), _ptr(dp), _ptr(v),
                                   _ptr(vp), _ptr(uo), _ptr(po), n))
        return uo, po

    def grad2func(self, q, sums=None, prob=0):
        import math
        import torch
        n = int(q.shape[0]) if getattr(q, "dim", lambda: 0)() > 0 else 0
        d = self.problems[prob].dim
        nc = math.prod(self.coarse_shape(prob))
        require(q, torch.float64, (n, d * nc), "q")
        if sums is not None:
            require(sums, torch.float64, (n,), "sums")
        w = torch.empty((n,) + self.coarse_shape(prob), dtype=torch.float64,
                        device="cuda")
        _check(lib().pw_grad2func(self._h, prob, _ptr(q), _ptr(sums), _ptr(w),
                                  n))
        return w

    def update_svd(self, F, G, reset=False, prob=0):
        """F, G: (n_cols, rows) float64 device tensors (column j = row j)."""
        import torch
        n = int(F.shape[0]) if getattr(F, "dim", lambda: 0)() > 0 else 0
        require(F, torch.float64, (n, self.rows(prob)), "F")
        require(G, torch.float64, (n, self.rows(prob)), "G")
        rk = ctypes.c_int()
        _check(lib().pw_update_svd(self._h, prob, _ptr(F), _ptr(G),
                                   int(F.shape[0]), int(bool(reset)),
                                   ctypes.byref(rk)))
        return rk.value

    def corrector(self, prob=0):
        """(U, S, V) of the current corrector: U, V as (rank, rows) tensors
        (row j = singular vector j)."""
        import torch
        rk = ctypes.c_int()
        _check(lib().pw_get_corrector(self._h, prob, None, None, None, 0,
                                      ctypes.byref(rk)))
        r = rk.value
        rows = self.rows(prob)
        U = torch.empty((max(r, 1), rows), dtype=torch.float64, device="cuda")
        V = torch.empty_like(U)
        S = torch.empty((max(r, 1),), dtype=torch.float64, device="cuda")
        _check(lib().pw_get_corrector(self._h, prob, _ptr(U), _ptr(S), _ptr(V),
                                      r, ctypes.byref(rk)))
        return U[:r], S[:r], V[:r]


def _traces_function():
    import torch

    class _PararealTraces(torch.autograd.Function):
        """traces = PararealTraces.apply(c, solver, receivers, K, prob):
        the receiver traces u^{K+1}_n(x_r) (N x n_rec, float64) of
        Algorithm 3 run on medium c (fine grid, float64 device tensor); the
        backward pass gives d/dc through the run with its correctors held
        fixed (pw_backward)."""

        @staticmethod
        def forward(ctx, c, solver, receivers, K, prob=0):
            solver.set_medium(c.detach(), prob)
            solver.run_taped(K, prob)
            ctx.solver, ctx.receivers, ctx.prob = solver, receivers, prob
            # the tape this graph's backward must read
            ctx.tape_id = solver.tape_id(prob)
            return solver.traces(receivers, prob)

        @staticmethod
        def backward(ctx, grad_traces):
            if ctx.solver.tape_id(ctx.prob) != ctx.tape_id:
                raise PwError(-5, "the solver ran another taped forward since "
                                  "this graph was recorded; its tape is gone "
                                  "(use one Solver per live graph)")
            g = ctx.solver.backward(ctx.receivers, grad_traces.contiguous(),
                                    wrt="c", prob=ctx.prob)
            return g, None, None, None, None

    return _PararealTraces


def _record_function():
    import torch

    class _PararealRecord(torch.autograd.Function):
        """record = PararealRecord.apply(c, solver, receivers, K, prob): the
        receiver record (N x m_fine x n_rec, float64) of one more F sweep
        from the iterate u^{K+1} of Algorithm 3 run on medium c (the
        trace_sweep of a taped run); the backward pass gives d/dc with the
        correctors and the absorbing layer held fixed
        (pw_backward_sweep)."""

        @staticmethod
        def forward(ctx, c, solver, receivers, K, prob=0):
            solver.set_medium(c.detach(), prob)
            solver.run_taped(K, prob)
            ctx.solver, ctx.receivers, ctx.prob = solver, receivers, prob
            ctx.tape_id = solver.tape_id(prob)
            return solver.trace_sweep(receivers, prob)

        @staticmethod
        def backward(ctx, grad_record):
            if ctx.solver.tape_id(ctx.prob) != ctx.tape_id:
                raise PwError(-5, "the solver ran another taped forward since "
                                  "this graph was recorded; its tape is gone "
                                  "(use one Solver per live graph)")
            g = ctx.solver.backward_sweep(ctx.receivers,
                                          grad_record.contiguous(), wrt="c",
                                          prob=ctx.prob)
            return g, None, None, None, None

    return _PararealRecord


class _Lazy:
    def __init__(self, make):
        self._make, self._obj = make, None

    def __getattr__(self, name):
        if self._obj is None:
            self._obj = self._make()
        return getattr(self._obj, name)


#: torch.autograd.Function over pw_run_taped / pw_traces / pw_backward
PararealTraces = _Lazy(_traces_function)
#: torch.autograd.Function over pw_run_taped / pw_trace_sweep /
#: pw_backward_sweep (a receiver record sampled every fine step)
PararealRecord = _Lazy(_record_function)
