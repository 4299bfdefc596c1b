"""Benchmark of the MI355X parareal-like wave solver (one GPU).

A step is one full batched solve of Algorithm 3 on the batch2d workload: 32
independent 2D periodic problems whose fine grids are drawn from {256, 384,
512, 768, 1024}^2 (coarse = fine/4), smooth random media c = exp(0.3 g) (g a
Gaussian random field of correlation length 0.1), random Gaussian pulses,
N = 32 slices each, K = 6 iterations, T = 1, FP32 compensated state, FP64
corrector, svd tol 1e-13: the coarse initialisation, then per iteration the
fine sweep of every slice of every problem (one multi-problem launch per
time block, replayed from a hipGraph), the corrector (Algorithm 1) and the
corrected sweep of every problem (concurrently, one stream per problem),
interpolation and update.  Inputs are synthetic and resident in HBM when
the timed region starts.

value = fine point-updates of the K batched sweeps (K * sum_b N m_F,b n_b^2
per step) / wall time of the steps, in Gpoint-updates/s.

roofline: the dominant kernel, the multi-problem fine stencil
(algorithmic 20 B per FP32 point-update: read u, p, c^2, write u, p), timed
on its own with events on the context stream; `traffic` is the HBM bytes
per launch measured with rocprofv3 counters (profiles/).

Also reported: the disc2d workload (512^2, 64 slices: solve, fine-sweep
roofline, time to 1e-5 against the serial fine solve, comparator
iterations of Sec. 6), the 3D layered workload at full size (256^3, 32
slices), the 1D workload's time to 1e-5, the misfit gradient, random
subsampling and randomised sketching on the Sec. 6.5 waveguide, the Sec.
6.4 gradient-order table, the Secs. 6.2 / 6.3 comparisons, the FP32 error
against the FP64 oracle per result, and the oracle timed on the host (one
process and a pool over all cores) on a bounded sample.
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
FP32_VECTOR_PEAK_TFLOPS = 157.3
BYTES_PER_UPDATE_F32 = 20
# flops of one velocity-Verlet point-update in the merged (leapfrog) form,
# a fused multiply-add counted as 2: per axis a three-point second
# difference (one add, one multiply-add: 3), the axes summed (d - 1), the
# kick p += h (c^2/dx^2) lap (one multiply, one multiply-add: 3), the
# drift u += h p (2)
FLOPS_PER_UPDATE = {1: 8, 2: 12, 3: 16}
# HBM bytes per launch of the fine stencil kernel, from the two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) of `bench.py --traffic-probe`, scaled
# by the same counters on a 512 MiB copy (profiles/disc2d_fine_stencil_
# traffic.md).  Valid only for the stencil revision it was measured on.
TRAFFIC = {"stencil-r6": 563.7e6, "stencil-r7": 561.5e6, "stencil-r8": 563.3e6,
           "stencil-r9": 563.6e6, "stencil-r10": 563.5e6}
# the same for the 3D stencil (layers3d) and the multi-problem 2D kernel
# (batch2d), per launch (mean over one sweep), keyed by the revision they
# were measured on (profiles/batch2d_fine_stencil_counters.md,
# profiles/layers3d_fine_stencil_counters.md)
TRAFFIC3D = {"stencil-r7": 32386.9e6, "stencil-r8": 24877.7e6,
             "stencil-r9": 21802.8e6, "stencil-r10": 21796.3e6}
TRAFFIC_BATCH = {"stencil-r7": 13787.9e6, "stencil-r8": 13780.4e6,
                 "stencil-r9": 13787.3e6, "stencil-r10": 13792.9e6}
# VALU instructions issued / (SIMDs x 4 cycles x elapsed cycles) over the
# same launches, from SQ_INSTS_VALU and GRBM_GUI_ACTIVE (values above 1:
# some instructions dual-issued)
VALU_ISSUE = {"stencil-r7": {"multi": 1.095, "single2d": 0.935, "3d": 0.526},
              "stencil-r8": {"multi": 1.121, "single2d": 0.944, "3d": 0.544},
              "stencil-r9": {"multi": 1.097, "single2d": 0.933, "3d": 0.567},
              "stencil-r10": {"multi": 1.097, "single2d": 0.932, "3d": 0.567}}


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


def cpu_baseline(ws, budget_s=8.0):
    """The oracle's fine propagator (numpy FP64) on a bounded sample of the
    batched workload: slice propagations (m_F steps from a problem's initial
    state) of the batch's problems in order, timed two ways: one process,
    and a process pool over slices with one worker per host core (the parfor
    of Algorithm 3).  The pool leg is the reported value."""
    import oracle as O
    from tests.gpu_helpers import oracle_pool

    def task(w):
        return (w.u0, w.p0, w.c * w.c, w.T / w.N / w.m_fine,
                1.0 / w.shape[-1], w.m_fine)

    t0 = time.perf_counter()
    upd1, i = 0, 0
    while time.perf_counter() - t0 < budget_s:
        w = ws[i % len(ws)]
        O.propagate(*task(w))
        upd1 += w.m_fine * w.npts
        i += 1
    dt1 = time.perf_counter() - t0
    one = upd1 / dt1 / 1e9
    cores = max(1, min(os.cpu_count() or 1, 64))
    tasks = [task(w) for w in ws]
    with oracle_pool(cores) as pm:
        list(pm(O.propagate, tasks[:1]))  # start the workers
        t0 = time.perf_counter()
        upd, done, j = 0, 0, 0
        while time.perf_counter() - t0 < budget_s or done == 0:
            batch = [tasks[(j + q) % len(tasks)] for q in range(cores)]
            list(pm(O.propagate, batch))
            upd += sum(ws[(j + q) % len(ws)].m_fine * ws[(j + q) % len(ws)].npts
                       for q in range(cores))
            j += cores
            done += cores
        dtp = time.perf_counter() - t0
    pool = upd / dtp / 1e9
    model = cpu_model()
    return {"value": round(pool, 5), "unit": "Gpoint-updates/s",
            "cores": cores, "kind": "oracle",
            "cpu_model": model,
            "single_process": {"value": round(one, 5), "cores": 1,
                               "sample": f"{i} slice propagations in "
                                         f"{dt1:.1f} s"},
            "sample": f"oracle fine propagator F (numpy FP64): {done} slice "
                      f"propagations (m_F steps each) of the batch's problems "
                      f"in order on a pool of {cores} processes in "
                      f"{dtp:.1f} s ({model})"}


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
               f"of a sweep, {launches} launches)", launch_ms, upd / launches,
               TRAFFIC_BATCH.get(rev), 2, VALU_ISSUE.get(rev, {}).get("multi")),
           "depth": depth, "rows_per_stream": info["rows_per_stream"],
           "rows_per_stream_by_grid": info["rows_per_stream_by_size"],
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


def roofline_stencil(name, launch_ms, updates_per_launch, traffic, dim, valu):
    """Roofline object of a fine-stencil kernel.  The time-blocked kernels
    take several steps per launch from one read and one write of the state,
    so their algorithmic HBM rate exceeds the HBM peak; rocprofv3 counters
    (profiles/) give the real DRAM bytes and the VALU issue rate.  A kernel
    whose SIMDs issue a VALU instruction nearly every cycle is reported
    "alu": achieved = algorithmic flops per launch (FLOPS_PER_UPDATE of the
    scheme, compensation not counted) / launch time against the FP32 vector
    peak; otherwise "hbm": algorithmic bytes (20 B per point-update) / launch
    time against the HBM peak.  Both views are kept in the object."""
    t = launch_ms * 1e-3
    bytes_algo = BYTES_PER_UPDATE_F32 * updates_per_launch
    flops = FLOPS_PER_UPDATE[dim] * updates_per_launch
    hbm = {"achieved_algorithmic_GBs": round(bytes_algo / t / 1e9, 1),
           "frac_algorithmic": round(bytes_algo / t / 1e9 / HBM_PEAK_GBS, 4)}
    if traffic:
        hbm["measured_GBs"] = round(traffic / t / 1e9, 1)
        hbm["frac_measured"] = round(traffic / t / 1e9 / HBM_PEAK_GBS, 4)
    alu = {"achieved_TFLOPs": round(flops / t / 1e12, 3),
           "frac": round(flops / t / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4),
           "flops_per_update": FLOPS_PER_UPDATE[dim],
           "valu_issue_frac": valu}
    valu_bound = valu is not None and valu >= 0.8
    if valu_bound:
        out = {"bound": "alu", "achieved": alu["achieved_TFLOPs"],
               "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": alu["frac"]}
    else:
        out = {"bound": "hbm", "achieved": hbm["achieved_algorithmic_GBs"],
               "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": hbm["frac_algorithmic"]}
    out.update({"traffic": traffic, "kernel": name,
                "launch_ms": round(launch_ms, 4),
                "algorithmic_bytes_per_launch": int(bytes_algo),
                "algorithmic_flops_per_launch": int(flops),
                "hbm_view": hbm, "alu_view": alu})
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
    rev = pw.lib().pw_version().decode().split()[-1]
    roof = roofline_stencil(f"k_prop_stream3d<float, true, {spl}, 2, 16, false>",
                            launch_ms, w.N * w.npts * spl, TRAFFIC3D.get(rev),
                            3, VALU_ISSUE.get(rev, {}).get("3d"))
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


def forced_problem(pw, w, fd, dtype, compensated, max_iters):
    return pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                           w.grad_order, w.tol, dtype, compensated,
                           max_iters, sponge_width=fd["width"],
                           sponge_reflection=fd["reflection"],
                           sponge_cmax=fd["c_max"])


def serial_record(pw, torch, w, fd, c, receivers):
    """The receiver record, every fine step, of the serial fine solution on
    medium c (the synthetic data of the misfit workload): the serial chain
    u(t_n) taken as the iterate, then one more sweep (FP64)."""
    P = forced_problem(pw, w, fd, "f64", False, 1)
    s = pw.Solver(P)
    s.set_medium(c)
    s.set_source(fd["src_pos"], fd["freq"], fd["t0"])
    s.set_initial(w.u0, w.p0)
    s.run(0)
    us, ps = s.serial_fine_states()
    for n in range(1, w.N):
        s.set_iterate(n, us[n], ps[n])
    d = s.trace_sweep(torch.as_tensor(receivers, device="cuda"))
    s.close()
    return d


def adjoint_measurement(pw, W, torch, reps=3):
    """Gradient of the receiver misfit with respect to c^2 (misfit2d
    recipe: absorbing layer, point source, a record every fine step): taped
    forward (Algorithm 3, FP32 compensated states) + the record's sweep +
    backward (FP64 adjoint, checkpoints every 64 fine steps)."""
    w, rec, target, fd = W.misfit2d()
    data = serial_record(pw, torch, w, fd, target, rec)
    s = pw.Solver(forced_problem(pw, w, fd, w.dtype, w.compensated, w.K))
    s.set_medium(w.c)
    s.set_source(fd["src_pos"], fd["freq"], fd["t0"])
    s.set_initial(w.u0, w.p0)
    recd = torch.as_tensor(rec, device="cuda")
    dt = w.T / w.N / w.m_fine

    def once():
        s.run_taped(w.K)
        r = s.trace_sweep(recd)
        res = r - data
        g = s.backward_sweep(recd, dt * res, wrt="c2", checkpoint_every=64)
        return 0.5 * dt * float((res * res).sum()), g

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
    out = {"workload": "misfit2d: 2D 512^2 / 128^2, absorbing layer 0.05 "
                       "(round trip 1e-3), Ricker source f=10 at (0.5, 0.1), "
                       "c = 1 + 2 s (GRF, seed 0), N=32, m_F=96, m_C=24, K=4, "
                       "128 receivers at y=0.9 recorded every fine step, data "
                       "the record of the serial fine solve on the seed-1 "
                       "medium",
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
    s.set_sampling(None)
    # randomised sketching of the new data (range finder, one power
    # iteration) with as many directions per iteration as the samples above
    out["sketch"] = {}
    for l in (w.N // 4, w.N // 8):
        s.set_sketch(W.sketch_matrices(w.N, l, K, seed=0), power=1)
        errs = []
        for k in range(0, K + 1):
            s.run(k)
            uN, pN = s.state(w.N)
            ed, er = s.energy(uN, pN, uf, pf)
            errs.append(float(f"{math.sqrt(ed / er):.4e}"))
        torch.cuda.synchronize()
        a = time.perf_counter()
        s.run(K)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3
        ph = s.timings()
        _, ranks = s.residuals()
        out["sketch"][str(l)] = {"energy_error_per_iteration": errs,
                                 "ms_K_iterations": round(ms, 2),
                                 "corrector_ms": round(ph["corrector"], 2),
                                 "rank": ranks, "power_iterations": 1}
        log(f"sketch l={l}: {ms:.1f} ms (corrector {ph['corrector']:.1f}), "
            "errors " + " ".join(f"{e:.2e}" for e in errs))
    s.set_sketch(None)
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


def disc2d_traffic_probe(pw, W, torch):
    w = W.disc2d()
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f32", True, w.K)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    u = torch.empty((w.N,) + w.shape, dtype=torch.float32, device="cuda")
    p = torch.empty_like(u)
    for n in range(w.N):
        u[n], p[n] = s.state(n)
    s.propagate(u, p)
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)  # plain copy: 512 MiB read + 512 MiB written
    torch.cuda.synchronize()
    log("traffic probe (disc2d) done: one fine sweep, one 536870912-byte copy")
    s.close()


def disc2d_measurement(pw, W, torch, args):
    """The discontinuous-disc workload (512^2 / 128^2, N = 64, m_F = 64,
    K = 8, FP32 compensated state, tol 1e-13): the full solve, its phases,
    the batched fine sweep with its roofline, the serial fine solve and the
    energy error after k iterations against it, and the comparator
    iterations of Sec. 6."""
    w = W.disc2d()
    K = w.K
    P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                        w.grad_order, w.tol, "f32", True, K,
                        keep_history=True)
    s = pw.Solver(P)
    s.set_medium(w.c)
    s.set_initial(w.u0, w.p0)
    s.run(K)
    solve_ms = solve_time(s, K, reps=5)
    phases = s.timings()
    rho, ranks = s.residuals()
    diag = s.diagnostics()
    log(f"disc2d solve {solve_ms:.2f} ms")
    u = torch.empty((w.N,) + w.shape, dtype=torch.float32, device="cuda")
    p = torch.empty_like(u)
    for n in range(w.N):
        u[n], p[n] = s.state(n)
    s.propagate(u, p)  # warm
    f_ms = stream_time(lambda: s.propagate(u, p), reps=10)
    launches, spl = s.launch_plan(w.N)
    rev = pw.lib().pw_version().decode().split()[-1]
    roof = roofline_stencil(f"k_prop_stream2d<float, true, {spl}, 0>",
                            f_ms / launches, w.N * w.npts * spl,
                            TRAFFIC.get(rev), 2,
                            VALU_ISSUE.get(rev, {}).get("single2d"))
    f_gupd = w.N * w.m_fine * w.npts / (f_ms * 1e-3) / 1e9
    log(f"disc2d F sweep {f_ms:.3f} ms ({f_gupd:.1f} Gupd/s)")
    del u, p
    out = {"workload": "disc2d: 2D periodic 512^2 fine / 128^2 coarse, disc "
                       "c=2 in c=1, Gaussian sigma 0.03 at (0.3, 0.5), N=64 "
                       "slices, m_F=64, m_C=16, K=8, T=2, tol 1e-13, FP32 "
                       "compensated state, FP64 corrector",
           "solve_ms": round(solve_ms, 3),
           "solve_gupd_s": round(K * w.N * w.m_fine * w.npts
                                 / (solve_ms * 1e-3) / 1e9, 2),
           "phases_ms": {k: round(v, 3) for k, v in phases.items()},
           "fine_sweep": {"ms": round(f_ms, 4), "gupd_s": round(f_gupd, 2),
                          "launches": launches, "roofline": roof},
           "rho": [float(f"{r:.4e}") for r in rho], "rank": ranks,
           "trace_S": [float(f"{d['trace_S']:.6e}") for d in diag],
           "r2_min": [float(f"{d['r2_min']:.6e}") for d in diag]}
    if not args.no_ttt:
        uf, pf = s.serial_fine(w.N)
        serial_ms = stream_time(lambda: s.serial_fine(w.N), reps=3)
        s.run(K)
        errs = errors_to_serial(s, w, uf, pf)
        out["time_to_1e-5"] = ttt_record(
            errs, serial_ms, lambda k: solve_time(s, k, reps=3,
                                                  run=lambda: s.run(k)))
        out["time_to_1e-5"]["note"] = (
            "energy error of the last slice against the serial fine solution "
            "after k = 0..K iterations; with fine and coarse propagators on "
            "different grids and a discontinuous wave speed the iteration is "
            "stable but stagnates (the paper's conclusions and its 2D "
            "inclusion experiment), which is what this workload shows")
        log("disc2d errors per iteration: " + " ".join(f"{e:.2e}"
                                                        for e in errs))
        if not args.no_variants:
            out["variants"] = variants_measurement(s, w, K, uf, pf, torch)
    s.close()
    return out


def oracle_spread(O, Q, w, u0, p0, K, ref, pm, **kw):
    """How far the FP64 oracle itself moves when its initial state (the
    medium, when the initial state is zero and a source drives the run) is
    perturbed by FP32-sized rounding (relative 2^-24, seeded): the
    conditioning of the iteration at this tolerance, beside which an FP32
    result is to be read.  (energy, l2, max), max over slices."""
    import numpy as np

    from tests.gpu_helpers import state_errors
    rng = np.random.default_rng(11)
    c1 = w.c
    if np.any(u0):
        u1 = u0 * (1 + 2.0 ** -24 * rng.standard_normal(np.shape(u0)))
    else:
        u1 = u0
        c1 = w.c * (1 + 2.0 ** -24 * rng.standard_normal(np.shape(w.c)))
    r1 = O.theta_parareal(Q, c1, u1, p0, K, pmap=pm, **kw)
    e = np.max([state_errors(r1.u[n], r1.p[n], ref.u[n], ref.p[n], w.c,
                             Q.dx_fine) for n in range(1, Q.N + 1)], axis=0)
    return [float(f"{x:.3e}") for x in e]


def batch_precision(sb, ws, K, n_problems=2):
    """FP32 energy-norm error of the batched solve against the FP64 oracle,
    on the smallest problems of the batch (full configuration: grid, N,
    m_F, K); the oracle's fine propagations run on a process pool."""
    import numpy as np

    import oracle as O
    from tests.gpu_helpers import oracle_pool, state_errors
    order = sorted(range(len(ws)), key=lambda i: ws[i].npts)[:n_problems]
    res = {}
    t0 = time.perf_counter()
    with oracle_pool() as pm:
        for i in order:
            w = ws[i]
            Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                          w.grad_order, w.tol)
            u0 = w.u0.astype(np.float32).astype(np.float64)
            p0 = w.p0.astype(np.float32).astype(np.float64)
            ref = O.theta_parareal(Q, w.c, u0, p0, K, pmap=pm)
            worst = np.zeros(3)
            for n in range(1, w.N + 1):
                u, p = sb.state(n, prob=i)
                e = state_errors(u.double().cpu().numpy(),
                                 p.double().cpu().numpy(), ref.u[n], ref.p[n],
                                 w.c, Q.dx_fine)
                worst = np.maximum(worst, e)
            res[f"problem {i} ({w.shape[0]}^2)"] = {
                "gpu_fp32_vs_oracle": [float(f"{x:.3e}") for x in worst],
                "oracle_fp32_input_spread": oracle_spread(O, Q, w, u0, p0, K,
                                                          ref, pm)}
    log(f"batch precision {res} ({time.perf_counter() - t0:.0f} s)")
    return res


def precision_measurement(pw, W, torch, batch_res):
    """Energy-norm error of the FP32 compensated path against the FP64
    oracle per result: the batched problems (full configuration, smallest
    problems), layers3d at the reduced size 64^3 / 16^3 (N = 32, K = 6), the
    misfit forward (Algorithm 3, K = 4) at 128^2; max over all slices of
    (energy, l2, max) relative errors.  disc2d at full size is compared on
    every iterate by the GPU tests (tests/test_gpu_endtoend.py)."""
    import numpy as np

    import oracle as O
    from tests.gpu_helpers import oracle_pool, state_errors
    out = {"batch2d": batch_res,
           "norms": "(energy, l2, max) relative, max over slices, final "
                    "iterate; oracle_fp32_input_spread: the oracle's own "
                    "change when its initial state is perturbed by relative "
                    "2^-24 (the conditioning of the iteration)"}

    def solve_vs_oracle(w, K, fd=None):
        if fd is None:
            P = pw.Problem.make(w.shape, w.ratio, w.T, w.N, w.m_fine,
                                w.m_coarse, w.grad_order, w.tol, "f32", True, K)
        else:
            P = forced_problem(pw, w, fd, "f32", True, K)
        s = pw.Solver(P)
        u0 = w.u0.astype(np.float32).astype(np.float64)
        p0 = w.p0.astype(np.float32).astype(np.float64)
        s.set_medium(w.c)
        if fd is not None:
            s.set_source(fd["src_pos"], fd["freq"], fd["t0"])
        s.set_initial(u0, p0)
        s.run(K)
        Q = O.Problem(w.shape, w.ratio, w.T, w.N, w.m_fine, w.m_coarse,
                      w.grad_order, w.tol)
        kw = {} if fd is None else {"forcing": O.Forcing(**fd)}
        with oracle_pool() as pm:
            ref = O.theta_parareal(Q, w.c, u0, p0, K, pmap=pm, **kw)
            spread = oracle_spread(O, Q, w, u0, p0, K, ref, pm, **kw)
        worst = np.zeros(3)
        for n in range(1, w.N + 1):
            u, p = s.state(n)
            e = state_errors(u.double().cpu().numpy(),
                             p.double().cpu().numpy(), ref.u[n], ref.p[n],
                             w.c, Q.dx_fine)
            worst = np.maximum(worst, e)
        s.close()
        return {"gpu_fp32_vs_oracle": [float(f"{x:.3e}") for x in worst],
                "oracle_fp32_input_spread": spread}

    t0 = time.perf_counter()
    # the smallest batch problems again with the rank tolerance at the FP32
    # resolution of their data (2^-23): the corrector keeps only directions
    # FP32 data determine, and the iteration's sensitivity drops
    ws = W.batch2d()
    for i in sorted(range(len(ws)), key=lambda i: ws[i].npts)[:2]:
        w = ws[i]
        w.tol = 2.0 ** -23
        out[f"batch2d problem {i} ({w.shape[0]}^2), svd tol 2^-23"] = \
            solve_vs_oracle(w, 6)
    out["layers3d (64^3 / 16^3, N=32, K=6)"] = solve_vs_oracle(
        W.layers3d(n=64, ratio=4, N=32, K=6, T=1.5), 6)
    wm, _, _, fdm = W.misfit2d(n=128, N=32, K=4)
    out["misfit2d forward (128^2 / 32^2, N=32, K=4, layer and source)"] = \
        solve_vs_oracle(wm, 4, fdm)
    log(f"precision {out} ({time.perf_counter() - t0:.0f} s)")
    return out


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
    ap.add_argument("--headline-only", action="store_true",
                    help="only the batched headline solve (profiling)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the misfit-gradient measurement")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the misfit-gradient measurement (profiling)")
    ap.add_argument("--disc2d-only", action="store_true",
                    help="only the disc2d solve and its fine sweep "
                         "(profiling; with --no-ttt, no serial study)")
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
    if args.disc2d_only:
        print(json.dumps(disc2d_measurement(pw, W, torch, args)), flush=True)
        return
    if args.layers_only:
        print(json.dumps(layers3d_measurement(pw, W, torch)), flush=True)
        return
    if args.traffic_probe in ("batch", "layers3d"):
        traffic_probe(pw, W, torch, args.traffic_probe)
        return
    if args.traffic_probe == "disc2d":
        disc2d_traffic_probe(pw, W, torch)
        return

    # ---- headline: the 32-problem batched solve -----------------------------
    K = 6
    ws, sb = batch_context(pw, W, K)
    log("batch context ready")
    sb.run_batch(K)  # builds the batch (autotuner, graph capture)
    for _ in range(args.warmup):
        sb.run_batch(K)
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sb.run_batch(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    upd_sweep = sum(w.updates_per_sweep() for w in ws)
    value = K * upd_sweep / (ms_step * 1e-3) / 1e9
    info = sb.batch_info()
    log(f"batched K={K} solve {ms_step:.1f} ms/step ({value:.1f} Gupd/s)")
    # the dominant kernel: the multi-problem fine stencil, timed alone with
    # events on the context stream (one graph-free launch sequence per sweep)
    sweep_ms = sb.batch_fine_sweeps(5)
    depth = info["depth"]
    launches = max(math.ceil(w.m_fine / depth) for w in ws)
    rev = pw.lib().pw_version().decode().split()[-1]
    roof = roofline_stencil(
        f"k_prop_stream2d_multi<float, true, {depth}>", sweep_ms / launches,
        upd_sweep / launches, TRAFFIC_BATCH.get(rev), 2,
        VALU_ISSUE.get(rev, {}).get("multi"))
    roof["sweep_ms"] = round(sweep_ms, 3)
    roof["launches_per_sweep"] = launches
    roof["gupd_s_fine_sweep"] = round(upd_sweep / (sweep_ms * 1e-3) / 1e9, 2)
    log(f"batched fine sweep {sweep_ms:.2f} ms "
        f"({roof['gupd_s_fine_sweep']:.1f} Gupd/s)")
    grids = sorted({w.shape[0] for w in ws})
    headline_phases = {k: round(info[k], 3) for k in
                       ("parallel", "corrector", "sweep", "total")}
    batch_prec = None if (args.no_precision or args.headline_only) else \
        batch_precision(sb, ws, K)
    sb.close()
    del sb
    torch.cuda.empty_cache()

    extras = {}
    if args.headline_only:
        args.no_adjoint = args.no_layers = args.no_wave1d = True
        args.no_sampling = args.no_table = args.no_sec6 = True
        args.no_precision = args.no_cpu = True
    else:
        extras["disc2d"] = disc2d_measurement(pw, W, torch, args)
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        extras["adjoint"] = adjoint_measurement(pw, W, torch)
        torch.cuda.empty_cache()
    if not args.no_layers:
        extras["layers3d"] = layers3d_measurement(pw, W, torch)
        torch.cuda.empty_cache()
    if not args.no_wave1d:
        extras["wave1d"] = wave1d_measurement(pw, W, torch)
    if not args.no_sampling:
        extras["sampling"] = sampling_measurement(pw, W, torch)
    if not args.no_table:
        extras["gradient_order_table"] = gradient_order_measurement(pw, torch)
    if not args.no_sec6:
        extras["sec6_comparators"] = sec6_comparator_measurement(pw, torch)
    if not args.no_precision:
        extras["precision"] = precision_measurement(pw, W, torch, batch_prec)
    cpu = None if args.no_cpu else cpu_baseline(ws)

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
        "config": {"workload": f"batch2d: 32 independent 2D periodic problems, "
                               f"fine grids drawn from {grids} (seed 0), coarse "
                               "= fine/4, c = exp(0.3 GRF(corr 0.1)) (seed "
                               "1000+b), random Gaussian pulse (seed 2000+b), "
                               f"N=32 slices each, K={K}, T=1, tol 1e-13",
                   "state": "f32 compensated", "corrector": "f64",
                   "step": f"one batched solve of all 32 problems "
                           f"(initialisation + K={K} iterations)",
                   "updates_per_step": K * upd_sweep},
        "roofline": roof,
        "phases_ms": headline_phases,
        "batch": {"depth": depth, "rows_per_stream": info["rows_per_stream"],
                  "rows_per_stream_by_grid": info["rows_per_stream_by_size"],
                  "tune_ms": round(info["tune_ms"], 1),
                  "from_cache": info["from_cache"]},
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
