"""Benchmark of the MI355X parareal-like wave solver (one GPU).

A step is one full solve of Algorithm 3 (coarse initialisation + K
iterations: batched fine propagation over all slices, Procrustes corrector,
corrected sweep, interpolation and update) on the disc2d workload: 2D
periodic 512^2 fine / 128^2 coarse grid, c = 1 with c = 2 inside a disc of
radius 0.2, Gaussian pulse (sigma 0.03) at (0.3, 0.5), T = 2, N = 64 slices,
m_F = 64, m_C = 16, K = 8, FP32 compensated state, FP64 corrector,
svd tol 1e-13.  Inputs are synthetic and already resident in HBM when the
timed region starts.

value = fine point-updates of the K batched fine sweeps (K * N * m_F *
512^2 per step) / wall time of the steps, in Gpoint-updates/s.

Also reported: the roofline of the fine stencil kernel (algorithmic 20 B
per FP32 point-update: read u, p, c^2, write u, p), the serial GPU fine
solve and the time to reach 1e-5 energy error against it, the comparator
iterations of Sec. 6 (Omega = I, no parareal-style correction, plain
parareal: error per iteration and time), the random subsampling of the
data matrices on the Sec. 6.5 waveguide (error per iteration and corrector
time per sample size, singular-value decay), the Sec. 6.4 gradient-order
table recomputed on the GPU beside the printed values, the comparisons of
Secs. 6.2 / 6.3 on the paper's 1D setup, the per-phase
split, and the FP64 oracle timed on the host on a bounded sample.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE_F32 = 20
# HBM bytes per launch of the fine stencil kernel, from the two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) of `bench.py --traffic-probe`, scaled
# by the same counters on a 512 MiB copy (profiles/disc2d_fine_stencil_
# traffic.md).  Valid only for the stencil revision it was measured on.
TRAFFIC = {"stencil-r6": 563.7e6}
# the same for the 3D stencil (layers3d) and the multi-problem 2D kernel
# (batch2d), per launch, keyed by the revision they were measured on
TRAFFIC3D = {}
TRAFFIC_BATCH = {}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s=8.0):
    """The oracle's fine propagator (numpy FP64) on a bounded sample of the
    workload's first fine sweep, timed two ways: one process, and a process
    pool over slices with one worker per host core (the parfor of Algorithm
    3).  The pool leg is the reported value."""
    import numpy as np

    import oracle as O
    from tests.gpu_helpers import oracle_pool
    c2 = w.c * w.c
    dx = 1.0 / w.shape[-1]
    h = w.T / w.N / w.m_fine
    u, p = w.u0.copy(), w.p0.copy()
    t0 = time.perf_counter()
    slices = 0
    while time.perf_counter() - t0 < budget_s and slices < w.N:
        u, p = O.propagate(u, p, c2, h, dx, w.m_fine)
        slices += 1
    dt1 = time.perf_counter() - t0
    one = slices * w.m_fine * w.npts / dt1 / 1e9
    cores = max(1, min(os.cpu_count() or 1, 64))
    # the pool propagates as many independent states as it has workers,
    # repeated while the budget lasts (the same state: the work per slice
    # does not depend on the data)
    states = [(w.u0, w.p0, c2, h, dx, w.m_fine)] * cores
    with oracle_pool(cores) as pm:
        list(pm(O.propagate, states[:1]))  # start the workers
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < budget_s or done == 0:
            list(pm(O.propagate, states))
            done += cores
        dtp = time.perf_counter() - t0
    pool = done * w.m_fine * w.npts / dtp / 1e9
    model = cpu_model()
    return {"value": round(pool, 5), "unit": "Gpoint-updates/s",
            "cores": cores, "kind": "oracle",
            "cpu_model": model,
            "single_process": {"value": round(one, 5), "cores": 1,
                               "sample": f"{slices} slices in {dt1:.1f} s"},
            "sample": f"oracle fine propagator F (numpy FP64) on "
                      f"{w.shape[0]}^{len(w.shape)} states of the "
                      f"{w.name} workload, {w.m_fine} steps per slice: "
                      f"{done} slice propagations on a pool of {cores} "
                      f"processes in {dtp:.1f} s ({model})"}


def batch_context(pw, W, K):
    ws = W.batch2d(K=K)
    probs = [pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine,
                             w.m_coarse, w.grad_order, w.tol, w.dtype,
                             w.compensated, K) for w in ws]
    sb = pw.Solver(probs)
    for i, w in enumerate(ws):
        sb.set_medium(w.c, prob=i)
        sb.set_initial(w.u0, w.p0, prob=i)
    return ws, sb


def batch_measurement(pw, W, torch):
    """32 independent 2D problems of uneven grids (batch2d recipe, FP32
    compensated): build the batch (autotune + hipGraph capture) with one
    batched iteration, time the batched fine sweep over all slices of all
    problems, then the full K = 6 batched solve."""
    K = 6
    ws, sb = batch_context(pw, W, K)
    log("batch context ready")
    t0 = time.perf_counter()
    sb.run_batch(1)
    t_iter = time.perf_counter() - t0
    info = sb.batch_info()
    ms = sb.batch_fine_sweeps(3)
    upd = sum(w.updates_per_sweep() for w in ws)
    gupd = upd / (ms * 1e-3) / 1e9
    log(f"batched fine sweep {ms:.2f} ms ({gupd:.1f} Gupd/s)")
    solve_ms = solve_time(sb, K, reps=2, run=lambda: sb.run_batch(K))
    info_k = sb.batch_info()
    log(f"batched K={K} solve {solve_ms:.1f} ms")
    depth = info["depth"]
    # one sweep = ceil(m_F / depth) launches per problem, all problems in one
    # launch sequence: the launch count of the longest problem
    launches = max(math.ceil(w.m_fine / depth) for w in ws)
    launch_ms = ms / launches
    bpl = BYTES_PER_UPDATE_F32 * upd / launches
    rev = pw.lib().pw_version().decode().split()[-1]
    grids = sorted({w.shape[0] for w in ws})
    out = {"workload": "batch2d: 32 problems, fine grids from "
                       f"{grids} (seed 0), N=32, K={K}, FP32 compensated",
           "updates_per_sweep": upd, "fine_sweep_ms": round(ms, 3),
           "gupd_s": round(gupd, 2),
           "hbm_frac_algorithmic": round(gupd * BYTES_PER_UPDATE_F32 / HBM_PEAK_GBS, 4),
           "roofline": roofline_stencil(
               f"k_prop_stream2d_multi<float, true, {depth}> (mean launch "
               f"of a sweep, {launches} launches)", launch_ms, int(bpl),
               TRAFFIC_BATCH.get(rev)),
           "depth": depth, "rows_per_stream": info["rows_per_stream"],
           "tune_ms": round(info["tune_ms"], 1),
           "first_batched_iteration_s": round(t_iter, 3),
           "solve_ms": round(solve_ms, 1),
           "solve_gupd_s": round(K * upd / (solve_ms * 1e-3) / 1e9, 2),
           "phases_ms": {k: round(info_k[k], 3) for k in
                         ("parallel", "corrector", "sweep", "total")}}
    sb.close()
    return out


def stream_time(fn, reps=3):
    """Mean time of fn() in ms from HIP events on torch's current stream (the
    library's context stream)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def solve_time(s, K, reps=3, run=None):
    """Best wall time (ms) of a K-iteration solve, synchronised."""
    import torch
    run = run or (lambda: s.run(K))
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        run()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - a)
    return min(ts) * 1e3


def errors_to_serial(s, w, uf, pf):
    """Energy error of slice N against the serial fine solution after
    k = 0..K iterations, from the iterate history of the last run."""
    errs = []
    for k in range(1, w.K + 2):
        uN, pN = s.iterate(k, w.N)
        nm = s.error_norms(uN, pN, uf, pf)
        errs.append(nm["energy"])
    return errs


def ttt_record(errs, serial_ms, par_ms_fn):
    kstar = next((k for k, e in enumerate(errs) if e <= 1e-5), None)
    par_ms = par_ms_fn(kstar) if kstar is not None else None
    return {"target": 1e-5, "reached_at_iteration": kstar,
            "parareal_ms": round(par_ms, 3) if par_ms else None,
            "serial_fine_ms": round(serial_ms, 3),
            "speedup_vs_serial": (round(serial_ms / par_ms, 4)
                                  if par_ms else None),
            "energy_error_per_iteration": [float(f"{e:.4e}") for e in errs],
            "plateau": float(f"{min(errs):.4e}")}


def roofline_stencil(name, launch_ms, bytes_per_launch, traffic):
    """Roofline object of a stencil kernel: achieved = algorithmic bytes per
    launch / launch time against the HBM peak; traffic = counter bytes per
    launch (profiles/), with the measured DRAM fraction beside it."""
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": traffic, "kernel": name,
           "launch_ms": round(launch_ms, 4),
           "algorithmic_bytes_per_launch": bytes_per_launch}
    if traffic:
        out["hbm_frac_measured"] = round(
            traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def layers3d_measurement(pw, W, torch):
    """The 3D layered workload at full size (256^3 / 64^3, N = 32, m_F =
    76, K = 6, FP32 compensated state): one batched fine sweep timed on its
    own (events), the full solve, the serial fine solve and the energy
    error of slice N after k iterations against it."""
    w = W.layers3d()
    K = w.K
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f32", True, K,
                        keep_history=True)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    log("layers3d context ready")
    s.run(0)
    u = torch.empty((w.N,) + w.shape, dtype=torch.float32, device="cuda")
    p = torch.empty_like(u)
    for n in range(w.N):
        u[n], p[n] = s.state(n)
    s.propagate(u, p)  # warm
    f_ms = stream_time(lambda: s.propagate(u, p), reps=2)
    del u, p
    torch.cuda.empty_cache()
    upd = w.N * w.m_fine * w.npts
    f_gupd = upd / (f_ms * 1e-3) / 1e9
    launches, spl = s.launch_plan(w.N)
    launch_ms = f_ms / launches
    bpl = BYTES_PER_UPDATE_F32 * w.N * w.npts * spl
    rev = pw.lib().pw_version().decode().split()[-1]
    roof = roofline_stencil(f"3D fine stencil ({spl} step(s) per launch)",
                            launch_ms, bpl, TRAFFIC3D.get(rev))
    log(f"layers3d F sweep {f_ms:.1f} ms ({f_gupd:.1f} Gupd/s)")
    solve_ms = solve_time(s, K, reps=1, run=lambda: s.run(K))
    phases = s.timings()
    uf, pf = s.serial_fine(w.N)
    serial_ms = stream_time(lambda: s.serial_fine(w.N), reps=1)
    errs = errors_to_serial(s, w, uf, pf)
    ttt = ttt_record(errs, serial_ms,
                     lambda k: solve_time(s, k, reps=1, run=lambda: s.run(k)))
    log(f"layers3d solve {solve_ms:.0f} ms, serial fine {serial_ms:.0f} ms, "
        "errors " + " ".join(f"{e:.2e}" for e in errs))
    rho, ranks = s.residuals()
    out = {"workload": "layers3d: 3D periodic 256^3 fine / 64^3 coarse, "
                       "layered c 1.0/1.5/2.2/3.0 x (1 + 0.05 U[-1,1]) (seed "
                       "0), Gaussian sigma 0.04 at the centre, T=1.5, N=32, "
                       f"m_F={w.m_fine}, m_C={w.m_coarse}, K={K}, FP32 "
                       "compensated state, FP64 corrector, tol 1e-13",
           "fine_sweep_ms": round(f_ms, 3), "gupd_s": round(f_gupd, 2),
           "hbm_frac_algorithmic": round(f_gupd * BYTES_PER_UPDATE_F32
                                         / HBM_PEAK_GBS, 4),
           "roofline": roof,
           "solve_ms": round(solve_ms, 1),
           "solve_gupd_s": round(K * upd / (solve_ms * 1e-3) / 1e9, 2),
           "phases_ms": {k: round(v, 2) for k, v in phases.items()},
           "rank": ranks, "rho": [float(f"{r:.4e}") for r in rho],
           "time_to_1e-5": ttt}
    s.close()
    torch.cuda.empty_cache()
    return out


def wave1d_measurement(pw, W, torch):
    """The 1D workload (256 / 64 points, N = 16, K = 6, FP64, tol 1e-14):
    time to reach an energy error of 1e-5 at T against the serial fine
    solve, both on the GPU."""
    w = W.wave1d()
    K = w.K
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f64", False, K,
                        keep_history=True)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    s.run(K)
    uf, pf = s.serial_fine(w.N)
    s.serial_fine(w.N)
    serial_ms = stream_time(lambda: s.serial_fine(w.N), reps=5)
    errs = errors_to_serial(s, w, uf, pf)
    ttt = ttt_record(errs, serial_ms,
                     lambda k: solve_time(s, k, reps=5, run=lambda: s.run(k)))
    s.run(K)
    ttt["phases_ms_K_iterations"] = {k: round(v, 3)
                                     for k, v in s.timings().items()}
    log(f"wave1d: serial {serial_ms:.3f} ms, parareal to 1e-5 "
        f"{ttt['parareal_ms']} ms at k={ttt['reached_at_iteration']}")
    s.close()
    return {"workload": "wave1d: 1D periodic 256 / 64 points, c = 1 + 0.2 "
                        "sin 2 pi x, N=16, m_F=32, m_C=8, K=6, FP64, tol "
                        "1e-14", "time_to_1e-5": ttt}


def serial_traces(pw, torch, w, c, receivers):
    """Receiver traces u_n(x_r), n = 1..N, of the serial fine solution on
    medium c (the synthetic data of the misfit workload)."""
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f64", False, 1)
    s = pw.Solver(P)
    s.set_medium(c)
    s.set_initial(w.u0, w.p0)
    u, p = s.state(0)
    u, p = u[None].contiguous(), p[None].contiguous()
    rec = torch.as_tensor(receivers, device="cuda")
    out = []
    for _ in range(w.N):
        u, p = s.propagate(u, p)
        out.append(u.reshape(-1)[rec])
    d = torch.stack(out).double().contiguous()
    s.close()
    return d


def adjoint_measurement(pw, W, torch, reps=3):
    """Gradient of the receiver misfit with respect to c^2 (misfit2d
    recipe): taped forward (Algorithm 3, FP32 compensated states) + traces
    + backward (FP64 adjoint, checkpoints every 64 fine steps)."""
    w, rec, target = W.misfit2d()
    data = serial_traces(pw, torch, w, target, rec)
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, w.dtype, w.compensated, w.K)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    recd = torch.as_tensor(rec, device="cuda")

    def once():
        s.run_taped(w.K)
        tr = s.traces(recd)
        seed = tr - data
        g = s.backward(recd, seed, wrt="c2", checkpoint_every=64)
        return 0.5 * float((seed * seed).sum()), g

    J, g = once()  # allocates the tape and the work buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        once()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    tm = s.timings()
    fwd_upd = w.K * w.N * w.m_fine * w.npts
    log(f"adjoint: gradient {ms:.1f} ms (taped forward {tm['taped']:.1f}, "
        f"backward {tm['backward']:.1f})")
    out = {"workload": "misfit2d: 2D periodic 512^2 / 128^2, c = 1 + 2 s "
                       "(GRF, seed 0), N=32, m_F=96, m_C=24, K=4, 128 "
                       "receivers, data from the serial fine solve on the "
                       "seed-1 medium",
           "forward_state": "f32 compensated", "adjoint": "f64",
           "checkpoint_every": 64,
           "gradient_ms": round(ms, 2),
           "taped_forward_ms": round(tm["taped"], 2),
           "backward_ms": round(tm["backward"], 2),
           "backward_over_forward": round(tm["backward"] / tm["taped"], 3),
           "fine_updates_forward": fwd_upd,
           "J": float(f"{J:.6e}"),
           "grad_norm": float(f"{float(g.norm()):.6e}")}
    s.close()
    return out


def variants_measurement(s, w, K, uf, pf, torch):
    """The comparator iterations of Sec. 6 on the same workload: energy
    error of the last slice after k = 0..K iterations and the time of a
    K-iteration run, for Omega = I, no parareal-style correction and plain
    parareal, beside Algorithm 3."""
    out = {}
    for name in ("omega_one", "no_correction", "plain"):
        s.set_variant(name)
        errs = []
        for k in range(0, K + 1):
            s.run(k)
            uN, pN = s.state(w.N)
            ed, er = s.energy(uN, pN, uf, pf)
            e = math.sqrt(ed / er) if er > 0 else math.sqrt(ed)
            errs.append(float(f"{e:.4e}") if math.isfinite(e) else None)
        torch.cuda.synchronize()
        a = time.perf_counter()
        s.run(K)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3
        rho, _ = s.residuals()
        out[name] = {"energy_error_per_iteration": errs,
                     "ms_K_iterations": round(ms, 3),
                     "rho": [float(f"{r:.4e}") if math.isfinite(r) else None
                             for r in rho]}
        log(f"variant {name}: {ms:.1f} ms, errors "
            + " ".join("nan" if e is None else f"{e:.2e}" for e in errs))
    s.set_variant("theta")
    return out


def sampling_measurement(pw, W, torch):
    """Random subsampling of the data matrices on the Sec. 6.5 waveguide
    (200^2 / 100^2, N = 200, FP64 state): energy error of the last slice
    after k = 0..K iterations, time of a K-iteration run and of its
    corrector phase, for N, N/2, N/4 and N/8 sampled columns per
    iteration; and the decay of the normalised singular values of the
    accumulated correlation matrix M after each iteration (all columns)."""
    w = W.waveguide2d()
    K = w.K
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f64", False, K)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    uf, pf = s.serial_fine(w.N)
    out = {"workload": "waveguide2d: 200^2 fine / 100^2 coarse, c = 1 - "
                       "0.3 cos(2 pi x), Gaussian plane pulse in y, T = 4, "
                       "N = 200, m_F = 250, m_C = 25, K = 6, FP64 state, "
                       "tol 1e-14", "by_sample_size": {}}
    idx = [0, 1, 3, 7, 15, 31, 63, 127, 255, 511, 1023]
    for n_s in (w.N, w.N // 2, w.N // 4, w.N // 8):
        s.set_sampling(None if n_s == w.N else
                       W.sample_columns(w.N, n_s, K, seed=0))
        errs, decay = [], []
        for k in range(0, K + 1):
            s.run(k)
            uN, pN = s.state(w.N)
            ed, er = s.energy(uN, pN, uf, pf)
            errs.append(float(f"{math.sqrt(ed / er):.4e}"))
            if n_s == w.N and k > 0:
                _, S, _ = s.corrector()
                S = S.cpu().numpy()
                decay.append([float(f"{S[i] / S[0]:.3e}") for i in idx
                              if i < len(S)])
        torch.cuda.synchronize()
        a = time.perf_counter()
        s.run(K)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3
        ph = s.timings()
        _, ranks = s.residuals()
        rec = {"energy_error_per_iteration": errs,
               "ms_K_iterations": round(ms, 2),
               "corrector_ms": round(ph["corrector"], 2),
               "rank": ranks}
        if decay:
            rec["sigma_over_sigma1"] = {"index": idx, "per_iteration": decay}
        out["by_sample_size"][str(n_s)] = rec
        log(f"sampling {n_s}/{w.N}: {ms:.1f} ms (corrector "
            f"{ph['corrector']:.1f}), errors "
            + " ".join(f"{e:.2e}" for e in errs))
    s.close()
    return out


def gradient_order_measurement(pw, torch):
    """The gradient-order table of Sec. 6.4 recomputed on the GPU: the
    mean of ||F - Omega^k G|| / ||F|| over the first three iterations for
    each nabla_h, beside the value the paper prints (1D, 100 points on
    [-0.5, 0.5), c = 1, one grid, dt/dx = 0.5, dt/dt_fine = 20, dt_com =
    0.05, T = 10: N = 200 slices; FP64 state, tol 1e-14)."""
    import numpy as np
    printed = {2: 3.8634e-3, 4: 3.8101e-3, 6: 3.8079e-3, 8: 3.8077e-3,
               "spectral": 3.8077e-3}
    n = 100
    x = -0.5 + np.arange(n) / n
    u0 = np.cos(10 * np.pi * x) * np.exp(-100 * x ** 2)
    out = {}
    for order, ref in printed.items():
        P = pw.Problem.make((n,), 1, 10.0, 200, 200, 10, order, 1e-14, "f64",
                            False, 3)
        s = pw.Solver(P)
        s.set_medium(np.ones(n))
        s.set_initial(u0, np.zeros(n))
        torch.cuda.synchronize()
        a = time.perf_counter()
        s.run(3)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3
        rho, _ = s.residuals()
        mean = float(np.mean(rho))
        out[str(order)] = {"mean_residual": float(f"{mean:.5e}"),
                           "printed": ref,
                           "rel_diff": float(f"{abs(mean - ref) / ref:.2e}"),
                           "ms_3_iterations": round(ms, 2)}
        s.close()
    log("Sec. 6.4 table: " + " ".join(f"{k}:{v['mean_residual']:.4e}"
                                      for k, v in out.items()))
    return out


def sec6_comparator_measurement(pw, torch, K=8):
    """The comparisons of Secs. 6.2 and 6.3 on the paper's own 1D setup
    (100 points on [-0.5, 0.5), c = 1, one grid, dt/dx = 0.5, dt/dt_fine =
    20, dt_com = 0.05, interpft, tol 1e-14, FP64): the energy error at T
    after k = 1..K iterations of Algorithm 3 against Omega = I with the
    second-order gradient for T = 2.5, 5, 10, 50 (Sec. 6.2; 1000 slices
    for T = 50), and against the
    iteration without the parareal-style correction with the fourth-order
    gradient for T = 10 (Sec. 6.3)."""
    import numpy as np
    n = 100
    x = -0.5 + np.arange(n) / n
    u0 = np.cos(10 * np.pi * x) * np.exp(-100 * x ** 2)

    def errors(T, order, variant):
        N = int(round(T / 0.05))
        P = pw.Problem.make((n,), 1, T, N, 200, 10, order, 1e-14, "f64",
                            False, K)
        s = pw.Solver(P)
        s.set_medium(np.ones(n))
        s.set_initial(u0, np.zeros(n))
        s.set_variant(variant)
        uf, pf = s.serial_fine(N)
        out = []
        for k in range(1, K + 1):
            s.run(k)
            uN, pN = s.state(N)
            ed, er = s.energy(uN, pN, uf, pf)
            e = math.sqrt(ed / er)
            out.append(float(f"{e:.3e}") if math.isfinite(e) else None)
        s.close()
        return out

    res = {"sec6_2_omega_one": {}, "sec6_3_no_correction": {}}
    for T in (2.5, 5.0, 10.0, 50.0):
        res["sec6_2_omega_one"][str(T)] = {
            "theta": errors(T, 2, "theta"),
            "omega_one": errors(T, 2, "omega_one")}
    res["sec6_3_no_correction"]["10.0"] = {
        "theta": errors(10.0, 4, "theta"),
        "no_correction": errors(10.0, 4, "no_correction")}
    for key, d in res.items():
        for T, v in d.items():
            log(f"{key} T={T}: " + "; ".join(
                f"{name} {v[name][-1]}" for name in v))
    return res


def traffic_probe(pw, W, torch, which):
    """One batched fine sweep of the batch2d or layers3d workload and one
    512 MiB device copy (the copy scales the rocprofv3 counters)."""
    if which == "batch":
        ws, sb = batch_context(pw, W, 1)
        sb.run_batch(1)
        torch.cuda.synchronize()
        sb.batch_fine_sweeps(1)
        sb.close()
    else:
        w = W.layers3d()
        P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                            w.grad_order, w.tol, "f32", True, 1)
        s = pw.Solver(P)
        s.set_medium(w.c)
        s.set_initial(w.u0, w.p0)
        s.run(0)
        u = torch.empty((w.N,) + w.shape, dtype=torch.float32, device="cuda")
        p = torch.empty_like(u)
        for n in range(w.N):
            u[n], p[n] = s.state(n)
        s.propagate(u, p)
        s.close()
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"traffic probe ({which}) done: one fine sweep, one 536870912-byte "
        "copy")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true",
                    help="skip the time-to-1e-5 study")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the comparator iterations of Sec. 6")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32-vs-FP64 comparison of the solve")
    ap.add_argument("--no-sec6", action="store_true",
                    help="skip the Secs. 6.2 / 6.3 comparisons")
    ap.add_argument("--no-table", action="store_true",
                    help="skip the Sec. 6.4 gradient-order table")
    ap.add_argument("--no-sampling", action="store_true",
                    help="skip the data-matrix subsampling study")
    ap.add_argument("--sampling-only", action="store_true",
                    help="only the data-matrix subsampling study")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 32-problem batched measurement")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the misfit-gradient measurement")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the misfit-gradient measurement (profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 32-problem batched measurement (profiling)")
    ap.add_argument("--layers-only", action="store_true",
                    help="only the 3D layered workload (profiling)")
    ap.add_argument("--no-layers", action="store_true",
                    help="skip the 3D layered workload")
    ap.add_argument("--no-wave1d", action="store_true",
                    help="skip the 1D time-to-1e-5 study")
    ap.add_argument("--traffic-probe", nargs="?", const="disc2d",
                    choices=["disc2d", "batch", "layers3d"],
                    help="only run one fine sweep of the workload and one "
                         "512 MiB device copy (for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); sharding the "
              "slices over several GPUs is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1905_00473_amd as pw
    import workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.adjoint_only:
        print(json.dumps(adjoint_measurement(pw, W, torch)), flush=True)
        return
    if args.sampling_only:
        print(json.dumps(sampling_measurement(pw, W, torch)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(batch_measurement(pw, W, torch)), flush=True)
        return
    if args.layers_only:
        print(json.dumps(layers3d_measurement(pw, W, torch)), flush=True)
        return
    if args.traffic_probe in ("batch", "layers3d"):
        traffic_probe(pw, W, torch, args.traffic_probe)
        return
    w = W.disc2d()
    K = w.K
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f32", True, K)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    torch.cuda.synchronize()
    log("context ready")
    if args.traffic_probe:
        u = torch.empty((w.N,) + w.shape, dtype=torch.float32, device="cuda")
        p = torch.empty_like(u)
        for n in range(w.N):
            u[n], p[n] = s.state(n)
        s.propagate(u, p)
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32,
                         device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)  # plain copy: 512 MiB read + 512 MiB written
        torch.cuda.synchronize()
        log("traffic probe done: 8 fine launches, one 536870912-byte copy")
        s.close()
        return

    # ---- timed region: full solves --------------------------------------
    for _ in range(args.warmup):
        s.run(K)
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.run(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    upd_step = K * w.N * w.m_fine * w.npts
    value = upd_step / (ms_step * 1e-3) / 1e9
    phases = s.timings()
    rho, ranks = s.residuals()
    log(f"solve {ms_step:.2f} ms/step")

    # ---- precision: the FP32 solve against the FP64 path ------------------
    # (the FP64 GPU path matches the FP64 oracle to 1e-12 in the parity
    # tests; at this size it stands in for the oracle, which takes minutes)
    precision = None
    if not args.no_precision:
        P64 = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine,
                              w.m_coarse, w.grad_order, w.tol, "f64", False,
                              K)
        s64 = pw.Solver(P64)
        s64.set_medium(w.c)
        s64.set_initial(w.u0.astype(np.float32).astype(np.float64),
                        w.p0.astype(np.float32).astype(np.float64))
        torch.cuda.synchronize()
        a = time.perf_counter()
        s64.run(K)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - a) * 1e3
        errs = {}
        for n in (1, w.N // 2, w.N):
            u32, p32 = s.state(n)
            u64, p64 = s64.state(n)
            ed, er = s64.energy(u32.double(), p32.double(), u64, p64)
            errs[str(n)] = float(f"{math.sqrt(ed / er):.3e}")
        precision = {"fp32_vs_fp64_energy_error_at_slice": errs,
                     "fp64_solve_ms": round(ms64, 2),
                     "note": "FP32 compensated solve against the FP64 path "
                             "from the same FP32-rounded initial data, "
                             "energy norm relative to the FP64 result"}
        log(f"FP32 vs FP64 energy error at slices 1, N/2, N: {errs}; "
            f"FP64 solve {ms64:.1f} ms")
        s64.close()
        torch.cuda.empty_cache()

    # ---- fine stencil kernel: the batched F sweep alone ------------------
    stencil_rev = pw.lib().pw_version().decode().split()[-1]
    dt = torch.float32
    u = torch.empty((w.N,) + w.shape, dtype=dt, device="cuda")
    p = torch.empty_like(u)
    for n in range(w.N):
        u[n], p[n] = s.state(n)
    uo, po = s.propagate(u, p)  # warm
    reps = 10
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        s.propagate(u, p)
    ev1.record()
    torch.cuda.synchronize()
    f_ms = ev0.elapsed_time(ev1) / reps
    launches, steps_per_launch = s.launch_plan(w.N)
    launch_ms = f_ms / launches
    bytes_per_launch = BYTES_PER_UPDATE_F32 * w.N * w.npts * steps_per_launch
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    f_gupd = w.N * w.m_fine * w.npts / (f_ms * 1e-3) / 1e9
    log(f"F sweep {f_ms:.3f} ms ({f_gupd:.1f} Gupd/s)")

    # ---- serial fine and time to 1e-5 -------------------------------------
    ttt = None
    serial_ms = None
    variants = None
    if not args.no_ttt:
        uf, pf = s.serial_fine(w.N)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            s.serial_fine(w.N)
        e1.record()
        torch.cuda.synchronize()
        serial_ms = e0.elapsed_time(e1) / 3
        errs = []
        for k in range(0, K + 1):
            s.run(k)
            uN, pN = s.state(w.N)
            ed, er = s.energy(uN, pN, uf, pf)
            errs.append(math.sqrt(ed / er) if er > 0 else math.sqrt(ed))
        log("errors per iteration: " + " ".join(f"{e:.2e}" for e in errs))
        kstar = next((k for k, e in enumerate(errs) if e <= 1e-5), None)
        if kstar is not None:
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                a = time.perf_counter()
                s.run(kstar)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - a)
            par_ms = min(ts) * 1e3
        else:
            par_ms = None
        ttt = {"target": 1e-5, "reached_at_iteration": kstar,
               "parareal_ms": par_ms, "serial_fine_ms": round(serial_ms, 3),
               "speedup_vs_serial": (round(serial_ms / par_ms, 4)
                                     if par_ms else None),
               "energy_error_per_iteration": [float(f"{e:.4e}")
                                              for e in errs],
               "plateau": float(f"{min(errs):.4e}"),
               "note": "energy error of the last slice against the serial "
                       "fine solution after k = 0..K iterations; the paper "
                       "reports that with different fine/coarse grids and a "
                       "discontinuous wave speed the iteration is stable but "
                       "stagnates instead of converging to the fine solution "
                       "(conclusions; 2D inclusion experiment), which is what "
                       "this workload shows"}
        if not args.no_variants:
            variants = variants_measurement(s, w, K, uf, pf, torch)
            variants["theta"] = {
                "energy_error_per_iteration": ttt[
                    "energy_error_per_iteration"],
                "ms_K_iterations": round(ms_step, 3),
                "rho": [float(f"{r:.4e}") for r in rho]}

    s.close()
    del u, p
    torch.cuda.empty_cache()
    batched = None if args.no_batch else batch_measurement(pw, W, torch)
    torch.cuda.empty_cache()
    adjoint = None if args.no_adjoint else adjoint_measurement(pw, W, torch)
    torch.cuda.empty_cache()
    sampling = None if args.no_sampling else sampling_measurement(pw, W,
                                                                  torch)
    layers = None if args.no_layers else layers3d_measurement(pw, W, torch)
    wave1d = None if args.no_wave1d else wave1d_measurement(pw, W, torch)
    table = None if args.no_table else gradient_order_measurement(pw, torch)
    sec6 = None if args.no_sec6 else sec6_comparator_measurement(pw, torch)

    cpu = None if args.no_cpu else cpu_baseline(w)

    out = {
        "metric": "batched fine-prop Gpoint-updates/s (%HBM roof) + "
                  "parareal time-to-1e-5 vs serial",
        "value": round(value, 3),
        "unit": "Gpoint-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "disc2d: 2D periodic 512^2 fine / 128^2 "
                               "coarse, disc c=2 in c=1, N=64 slices, "
                               "m_F=64, m_C=16, K=8, T=2, tol 1e-13",
                   "state": "f32 compensated", "corrector": "f64",
                   "step": "one full parareal solve (init + K iterations)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": TRAFFIC.get(stencil_rev),
                     "kernel": "k_prop_stream2d<float, true, 8, 0> (fine grid)",
                     "launch_ms": round(launch_ms, 4),
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "fine_sweep": {"ms": round(f_ms, 4), "gupd_s": round(f_gupd, 2),
                       "launches": launches},
        "phases_ms": {k: round(v, 3) for k, v in phases.items()},
        "precision": precision,
        "rho": [float(f"{r:.4e}") for r in rho],
        "rank": ranks,
        "time_to_1e-5": ttt,
        "variants": variants,
        "sampling": sampling,
        "gradient_order_table": table,
        "sec6_comparators": sec6,
        "batched": batched,
        "layers3d": layers,
        "wave1d": wave1d,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
