/*
 * pw.h -- C ABI of the MI355X (gfx950) implementation of the stabilised
 * parareal-like method for the second-order wave equation of
 * H. Nguyen and R. Tsai, "A stable parareal-like method for the second
 * order wave equation" (arXiv 1905.00473).
 *
 * Problem (eq. (1)): u_tt = c(x)^2 Lap u on the periodic box [0,1)^d,
 * d = 1, 2, 3, with u(.,0) = u0 and u_t(.,0) = p0.  The state of a wave
 * field is the pair [u, p] with p = u_t.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Grids (Sec. 3.1): the fine grid has n_fine[a] points on axis a
 *   (a = 0: x, 1: y, 2: z; unused axes are 1), spacing dx = 1 / n_fine[0]
 *   on every axis (cubic cells; n_fine[a] * dx is the box length along a).
 *   The coarse grid has n_fine[a] / ratio points; coarse node J is fine
 *   node ratio * J on every axis.
 * - A field is stored x-fastest: element (x, y, z) at x + nx (y + ny z).
 *   A "state" is a u field followed by a p field when it is stored in one
 *   block (coarse FP64 state columns); otherwise u and p are separate
 *   arrays of fields.  Batches of fields are contiguous (field stride =
 *   number of grid points).
 * - State dtype: PW_F64 (double) or PW_F32 (float), chosen per problem.
 *   Energy components, singular vectors, residuals and energies are always
 *   double.
 * - Energy-component column (eqs. matrixF / matrixG): rows
 *   [d_x U ; d_y U ; (d_z U) ; P / c] on the coarse grid, each block
 *   x-fastest, length (d+1) * n_coarse_points.  Columns are stored
 *   column-major (column j at offset j * rows).
 * - Pointers: arguments named *_dev are device pointers (hipMalloc'd or
 *   torch CUDA tensors) owned by the caller and must stay valid until the
 *   call's work on the context stream has finished; arguments named *_host
 *   are host pointers read or written synchronously.  The library never
 *   frees caller memory.  Device pointers must be 16-byte aligned.
 * - Streams: every call enqueues its kernels on the context's stream and
 *   returns without waiting unless stated otherwise.  Calls that return
 *   host data synchronise the stream first.
 * - Errors: every call returns a pw_status <= 0.  pw_last_error() gives a
 *   message for the last failing call on the calling thread.  No C++
 *   exception crosses the ABI.  A context is not thread-safe.
 */
#ifndef PW_H
#define PW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PW_OK = 0,
  PW_EINVAL = -1,      /* bad argument or size                                */
  PW_EUNSTABLE = -2,   /* c_max dt/dx >= 1/sqrt(d): velocity Verlet unstable  */
  PW_ENOMEM = -3,      /* device allocation failed                            */
  PW_EHIP = -4,        /* a HIP runtime call failed (message has the reason)  */
  PW_ESTATE = -5,      /* call order violated (e.g. run before set_initial)   */
  PW_ENUMERIC = -6     /* non-finite value or breakdown in the corrector      */
} pw_status;

typedef enum { PW_F32 = 0, PW_F64 = 1 } pw_dtype;

/* which propagator (Sec. 3.1) */
typedef enum { PW_FINE = 0, PW_COARSE = 1 } pw_grid;

/*
 * Discretisation of one problem (the parameter columns of the Sec. 6
 * tables).  dt_com = T / n_slices; the fine propagator F takes m_fine
 * velocity-Verlet steps of dt_com / m_fine on the fine grid, the coarse
 * propagator C takes m_coarse steps of dt_com / m_coarse on the coarse
 * grid with the pointwise coarse medium c(ratio J dx).
 */
typedef struct {
  int dim;             /* 1, 2 or 3                                           */
  int n_fine[3];       /* fine points per axis (x, y, z); unused axes = 1     */
  int ratio;           /* coarse spacing / fine spacing (>= 1, divides n)    */
  double T;            /* final time                                         */
  int n_slices;        /* N coupling intervals                               */
  int m_fine;          /* fine steps per interval                            */
  int m_coarse;        /* coarse steps per interval                          */
  int grad_order;      /* nabla_h: central difference of order 2, 4, 6 or 8,
                          or 0 for the Fourier (spectral) derivative         */
  double svd_tol;      /* relative rank tolerance of Algorithm 1 (> 0)       */
  int state_dtype;     /* pw_dtype of u, p                                   */
  int compensated;     /* FP32 only: compensated (Kahan) accumulation in F/C */
  int max_iters;       /* largest K that pw_run will be asked for (sizes the
                          corrector bases: rank <= max_iters * n_slices)     */
  int interp;          /* pw_interp: the interpolation I (0 = trigonometric) */
  int keep_history;    /* 1: keep every iterate u^k_n, k = 1..max_iters+1, on
                          the device for pw_get_iterate ((max_iters + 1) N
                          fine states); 0: only the current one         */
  int bc;              /* pw_bc: PW_PERIODIC, or PW_SPONGE (2D only)         */
  double sponge_width; /* PW_SPONGE: layer width, a fraction of the box in
                          (0, 0.5)                                         */
  double sponge_reflection; /* PW_SPONGE: amplitude left after a round trip
                          through the layer at c_max (0: 1e-3)             */
  double sponge_cmax;  /* PW_SPONGE: the c_max of sigma_max (0: the largest
                          c of the medium, taken at pw_set_medium)         */
} pw_problem;

/* Boundary of the box.  The paper's problem (eq. (1)) allows periodic,
 * absorbing or PML boundaries; the method itself is stated for the
 * periodic box, where the Fourier-based Lambda^dag of Sec. 4 holds.
 * PW_SPONGE keeps the periodic box and damps the waves in a layer of
 * width w along every face: u_tt = c^2 Lap u - sigma u_t, with
 * sigma = sigma_max (d / w)^2, d the largest penetration of a node into
 * the layer over the axes, sigma_max = (3 c_max / (2 w)) ln(1 / R).  Each
 * velocity-Verlet half kick first multiplies p by exp(-sigma h / 2) (the
 * exact decay over h / 2); the coarse propagator uses sigma at the coarse
 * nodes.  Every other step of Algorithm 3 is unchanged.  The layer is a
 * function of position only: the gradient of pw_backward holds it fixed.
 * 2D problems only (PW_EINVAL otherwise).                               */
typedef enum { PW_PERIODIC = 0, PW_SPONGE = 1 } pw_bc;

/* The interpolation I from the coarse to the fine grid: trigonometric
 * (the interpft of Sec. 6, the default), periodic piecewise linear, or
 * local cubic (4-point Lagrange through the coarse nodes J-1 .. J+2):
 * lower-order interpolants of the kind used in the numerical examples of
 * Sec. 7.  All satisfy R I = 1.  Taped runs (differentiation) support the
 * trigonometric one only.                                               */
typedef enum { PW_INTERP_TRIG = 0, PW_INTERP_LINEAR = 1, PW_INTERP_CUBIC = 2 } pw_interp;

typedef struct pw_ctx pw_ctx;

/* Create a context holding n_problems problems; all device buffers are
 * allocated here.  stream is a hipStream_t (NULL = default stream).
 * Returns PW_EINVAL for inconsistent sizes, PW_ENOMEM if allocation fails. */
pw_status pw_create(const pw_problem* probs, int n_problems, void* stream,
                    pw_ctx** out);

/* Release every device buffer of the context (synchronises first). */
pw_status pw_destroy(pw_ctx* ctx);

/* Message of the last failing call on this thread (valid until the next
 * failing call on the thread). */
const char* pw_last_error(void);

/* Number of problems / library version string. */
int pw_num_problems(const pw_ctx* ctx);
const char* pw_version(void);

/* Set the medium c(x) > 0 of problem `prob` from a double field on the
 * fine grid (eq. (1); the coarse propagator samples it pointwise, Sec.
 * 3.1).  Copies; returns PW_EUNSTABLE if c_max * dt / dx >= 1/sqrt(d) on
 * either grid.  on_device: 1 if c is a device pointer, 0 for host.       */
pw_status pw_set_medium(pw_ctx* ctx, int prob, const double* c,
                        int on_device);

/* Point source f(x, t) = r(t) delta_h(x - x_s) added to eq. (1)
 * (u_tt = c^2 Lap u + f): r is the Ricker wavelet (1 - 2a) exp(-a),
 * a = (pi freq (t - t0))^2, placed at the grid node nearest to pos (box
 * coordinates, x first, dim values; nearest fine node for F, nearest
 * coarse node for C) with weight 1 / dx^dim of that grid.  Slice n
 * propagates from t_{n-1} = (n - 1) T / N, so every kick of F and C adds
 * (its weight) * r(t) at the source node.  The correction of Algorithm 3
 * acts on differences of coarse propagations, in which the source
 * cancels: the sweep's coarse propagations of differences (and the
 * corrector-coordinate recurrence) use C without the source.  pos = NULL
 * removes the source.  freq > 0.  2D problems only; the comparator
 * PW_VARIANT_NO_CORRECTION, which propagates states rather than
 * differences, and batches (pw_run_batch) refuse a problem with a source
 * (PW_EINVAL).  Resets the iteration.                                   */
pw_status pw_set_source(pw_ctx* ctx, int prob, const double* pos, double freq,
                        double t0);

/* Set the initial state u0, p0 (double fields on the fine grid, eq. (1)),
 * converted to the state dtype.  Resets the iteration (k = 0).          */
pw_status pw_set_initial(pw_ctx* ctx, int prob, const double* u0,
                         const double* p0, int on_device);

/*
 * Algorithm 3 (eq. thetarelation): the coarse initialisation
 * u^1_n = I C R u^1_{n-1} followed by up to K iterations of: F on all
 * slices in one batched launch, the data matrices F^k = [Lambda R v_n],
 * G^k = [Lambda C R u^k_{n-1}], the incremental Procrustes SVD of
 * Algorithm 1, the corrected sweep over n and the update
 * u^{k+1}_n = v_n + I delta_n.  K <= max_iters.  Each call restarts from
 * u0 (the iteration count and corrector are reset).
 *
 * Stopping rule (the "while tolerance not met" of Algorithm 3, which the
 * paper leaves open): with stop_tol > 0 the run ends after the first
 * iteration k whose change max_n sqrt(E(u^{k+1}_n - u^k_n) / E(u^{k+1}_n))
 * (discrete energy on the fine grid, FP64) is <= stop_tol; that costs one
 * energy reduction per slice and one host synchronisation per iteration.
 * stop_tol = 0 runs exactly K iterations.  *k_done (may be NULL) receives
 * the number of iterations run; the current iterate is then u^{k_done+1}.
 * Runs on the context stream; synchronises once per iteration to read the
 * new rank of Algorithm 1 and once per Jacobi sweep of its core SVD.
 */
pw_status pw_run(pw_ctx* ctx, int prob, int K, double stop_tol, int* k_done);

/*
 * Resume Algorithm 3 from the current iterate and corrector (left by
 * pw_run, pw_run_batch, pw_continue, pw_load or overwritten with
 * pw_set_iterate / pw_set_corrector) for up to K more iterations,
 * numbered k_done + 1, ...; k_done + K <= max_iters.  update_corrector = 1:
 * each iteration updates the corrector with Algorithm 1 on its data, as
 * pw_run does; 0: the current corrector Omega = U~ V~^T is held fixed (no
 * data matrices, no SVD; the iteration's residual is reported as NaN).
 * stop_tol and *k_done as for pw_run.  PW_ESTATE without an iterate.
 */
pw_status pw_continue(pw_ctx* ctx, int prob, int K, int update_corrector, double stop_tol,
                      int* k_done);

/*
 * Comparator iterations of Sec. 6, run by pw_run in place of Algorithm 3
 * (the coarse initialisation and the batched fine step are the same):
 *   PW_VARIANT_THETA          Algorithm 3 as above (the default);
 *   PW_VARIANT_OMEGA_ONE      Omega = I in eq. thetarelation (Sec. 6.2):
 *                             u^{k+1}_n = v_n + I Lambda^dag Lambda
 *                             C (R u^{k+1}_{n-1} - R u^k_{n-1});
 *                             rho_k = ||F^k - G^k|| / ||F^k||, rank = rows;
 *   PW_VARIANT_NO_CORRECTION  the phase-corrected coarse propagation
 *                             without the parareal-style correction
 *                             (Sec. 6.3): u^{k+1}_n = I Lambda^dag Omega^k
 *                             Lambda C R u^{k+1}_{n-1}, with Omega^k from
 *                             Algorithm 1 on the same data as Algorithm 3;
 *   PW_VARIANT_PLAIN          plain parareal, eq. plainparareal with the
 *                             coarse propagator I C R; rho_k and rank as
 *                             for PW_VARIANT_OMEGA_ONE.
 * The Omega = I and plain sweeps are serial chains of N coarse
 * propagations (no reduced recurrence).  Applies to pw_run only:
 * pw_run_batch, pw_run_taped and pw_run_frozen return PW_EINVAL for a
 * problem whose variant is not PW_VARIANT_THETA.  Resets the iteration.
 * PW_EINVAL for an unknown variant.
 */
typedef enum {
  PW_VARIANT_THETA = 0,
  PW_VARIANT_OMEGA_ONE = 1,
  PW_VARIANT_NO_CORRECTION = 2,
  PW_VARIANT_PLAIN = 3
} pw_variant;
pw_status pw_set_variant(pw_ctx* ctx, int prob, int variant);

/*
 * Random subsampling of the data matrices (Sec. 6.5): in iteration k
 * (1-based) Algorithm 1 receives only the columns
 * cols[(k-1) * n_per_iter + j], j < n_per_iter, of F^k and G^k (column j
 * holds slice j + 1), so the truncated QR and the core SVD work on
 * n_per_iter instead of N columns.  The draw is the caller's: cols is a
 * host array of n_iters x n_per_iter int32, each row distinct indices in
 * [0, N); it is copied.  rho_k is still measured on all N columns.
 * n_per_iter = 0 switches sampling off (cols may be NULL).  Applies to
 * pw_run, pw_run_batch and pw_run_taped, which return PW_EINVAL when K
 * exceeds n_iters.  PW_EINVAL for sizes outside [0, N], a column outside
 * [0, N) or repeated within a row.  Resets the iteration.  Synchronises
 * the context stream.
 */
pw_status pw_set_sampling(pw_ctx* ctx, int prob, const int* cols,
                          int n_per_iter, int n_iters);

/*
 * Randomised sketching inside Algorithm 1 (Sec. 6.5 points to randomised
 * low-rank methods for the corrector): in iteration k the truncated QR of
 * the new data residuals F - U~ U~^T F (and likewise G) is replaced by the
 * randomised range finder of Halko, Martinsson and Tropp: Q_F = an
 * orthonormal basis of (A A^T)^power A Omega_k, A the residual, and R_F =
 * Q_F^T A, so that the core SVD is (r + l) square instead of (r + N).
 * omega is a host array of n_iters test matrices, each N x l column-major
 * (column j at offset j * N; the draw is the caller's, e.g. standard
 * normal), copied; 0 <= power <= 8.  Exact (to rounding) when the
 * residuals have rank <= l.  l = 0 switches sketching off.  Exclusive with
 * pw_set_sampling (PW_EINVAL).  Applies to pw_run, pw_continue,
 * pw_run_batch and pw_run_taped; PW_EINVAL when K exceeds n_iters.  Not
 * saved by pw_save.  Resets the iteration.  Synchronous.
 */
pw_status pw_set_sketch(pw_ctx* ctx, int prob, const double* omega, int l, int n_iters,
                        int power);

/*
 * Batching: Algorithm 3 for every problem of the context in lockstep (all
 * problems 2D, same state dtype and compensation, medium and initial state
 * set).  Per iteration, the parallel phase of all problems -- the fine
 * sweeps over all slices of every problem, the restrictions and the coarse
 * propagations -- is one launch sequence of the multi-problem streaming
 * kernel (one launch per time block), captured once in a hipGraph and
 * replayed; the corrector and the sweep then run per problem.  On the first
 * call an autotuner times the batched fine sweep for each candidate
 * (pipeline depth 4 or 8 steps, 64/128/256 rows per stream) and keeps the
 * fastest; with the environment variable PW_TUNE_CACHE naming a file the
 * choice is cached there across processes.  Results per problem are read
 * with pw_get_state / pw_get_residuals and equal those of pw_run bit for
 * bit.  Synchronises once per iteration.
 */
pw_status pw_run_batch(pw_ctx* ctx, int K);

/* Time `reps` batched fine sweeps (all slices of all problems, the launch
 * sequence of pw_run_batch) and return the mean time per sweep in *ms.
 * Needs a previous pw_run_batch.  Synchronises.                         */
pw_status pw_batch_fine_sweeps(pw_ctx* ctx, int reps, double* ms);

/* Configuration and timing of the batched runs: chosen pipeline depth and
 * rows per stream; ms[0..3] = parallel phase, corrector and sweep (run
 * concurrently over the problems: ms[1] is their wall time, ms[2] = 0),
 * total of the last pw_run_batch; ms[4] = autotuning time; ms[5] = fine
 * sweep time of the chosen configuration while tuning; ms[6] = 1 if the
 * choice came from the cache; ms[7] = number c of fine grid sizes whose
 * rows per stream the tuner set apart from the common value, followed by
 * c pairs (n_y, rows per stream) at ms[8 + 2i], ms[9 + 2i].  Host output,
 * cap = array length.                                                   */
pw_status pw_get_batch_info(pw_ctx* ctx, int* depth, int* rows_per_stream, double* ms,
                            int cap);

/* Wait for all work on the context stream. */
pw_status pw_sync(pw_ctx* ctx);

/* Copy the current iterate u^k_n, n = 0..N (after pw_run: k = K+1) into
 * caller buffers of n_points elements of the state dtype.  on_device
 * selects device or host destination; host copies are synchronous.     */
pw_status pw_get_state(pw_ctx* ctx, int prob, int n, void* u, void* p,
                       int on_device);

/* Iterate u^k_n of the last run (eq. (2) / Algorithm 3 notation: k = 1 is
 * the coarse initialisation, k = k_done + 1 the current iterate), n = 0..N
 * (u^k_0 = u0), into caller buffers of n_points elements of the state
 * dtype.  k < k_done + 1 needs keep_history = 1 (PW_EINVAL otherwise).
 * PW_ESTATE before the first run.  on_device as for pw_get_state.      */
pw_status pw_get_iterate(pw_ctx* ctx, int prob, int k, int n, void* u, void* p,
                         int on_device);

/* Overwrite slice n = 1..N of the current iterate u^{k_done+1}_n with the
 * double fields u, p (fine grid, rounded to the state dtype), e.g. to
 * resume from iterates computed elsewhere.  PW_ESTATE before the first
 * run.  Synchronous.                                                    */
pw_status pw_set_iterate(pw_ctx* ctx, int prob, int n, const double* u, const double* p,
                         int on_device);

/* Replace the corrector of Algorithm 1 by U~ (rows x rank), S~ (rank),
 * V~ (rows x rank), double, column-major, with orthonormal columns (the
 * caller's responsibility); Omega = U~ V~^T then acts in the sweep.  rank
 * <= min(max_iters * N, rows).  Synchronous.                           */
pw_status pw_set_corrector(pw_ctx* ctx, int prob, const double* U, const double* S,
                           const double* V, int rank, int on_device);

/* Per-iteration diagnostics of the last pw_run, k = 1..K: relative
 * Procrustes residual rho_k = ||F^k - Omega^k G^k||_F / ||F^k||_F
 * (Sec. 6.4) and the rank of Omega^k (Algorithm 1).  cap = array length;
 * returns the number of iterations in *count.  Host output, synchronous. */
pw_status pw_get_residuals(pw_ctx* ctx, int prob, double* rho_host,
                           int* rank_host, int cap, int* count);

/* Per-iteration record of the last run (FP64, host), PW_DIAG_STRIDE values
 * per iteration k = 1..k_done at out[(k-1) * PW_DIAG_STRIDE + i]:
 *   i = 0  rho_k = ||F^k - Omega^k G^k||_F / ||F^k||_F (Sec. 6.4)
 *   i = 1  rank of Omega^k (Algorithm 1)
 *   i = 2  ||F^k||_F^2 over all N columns
 *   i = 3  ||F^k_in||_F^2, i = 4  ||G^k_in||_F^2: the columns that entered
 *          Algorithm 1 (all N unless subsampled)
 *   i = 5  trace of S~^k (sum of the retained singular values)
 *   i = 6  r^2_min = sum_{j<=k} (||F^j_in||^2 + ||G^j_in||^2) - 2 tr S~^k,
 *          the minimum residual of the accumulated Procrustes problem of
 *          Sec. 3.3 (exact without truncation; reported as computed)
 *   i = 7  the stopping measure of pw_run (NaN unless stop_tol > 0)
 * Iterations without a fitted corrector (comparators, frozen corrector)
 * report 0 or NaN where a value does not exist.  cap = iterations the
 * array holds; *count = k_done.                                          */
#define PW_DIAG_STRIDE 8
pw_status pw_get_diagnostics(pw_ctx* ctx, int prob, double* out, int cap, int* count);

/* Serial fine reference u(t_n) = F^n [u0, p0] (Sec. 6: computed serially
 * with the fine propagator; with a source, step n of the chain propagates
 * slice n) written to caller device buffers u_dev, p_dev of n_points
 * elements of the state dtype.  0 <= n <= N.                            */
pw_status pw_serial_fine(pw_ctx* ctx, int prob, int n, void* u_dev,
                         void* p_dev);

/* The serial fine reference at every coupling time: u(t_n), p(t_n) for
 * n = 0..N written to u_dev + n * n_points, p_dev + n * n_points (N + 1
 * fields of the state dtype each), from one chain of N propagations.    */
pw_status pw_serial_fine_states(pw_ctx* ctx, int prob, void* u_dev, void* p_dev);

/* ------------------------------------------------------------------------
 * Building blocks of the path, exposed for parity checks.  All pointers
 * are device pointers; n_states fields are processed in one launch.
 * ------------------------------------------------------------------------ */

/* F (grid = PW_FINE) or C (PW_COARSE) of problem `prob` applied to
 * n_states states: u_out[s], p_out[s] = prop(u_in[s], p_in[s]) in the
 * state dtype (Sec. 3.1).  Inputs and outputs may not overlap.  With a
 * layer and source, state s propagates slice s + 1 (from t = s T / N), as
 * in the parallel step of Algorithm 3.                                   */
pw_status pw_propagate(pw_ctx* ctx, int prob, int grid, const void* u_in,
                       const void* p_in, void* u_out, void* p_out,
                       int n_states);

/* Energy components Lambda[U, P] (eqs. matrixF / matrixG) of n_states
 * states given on the fine grid (grid = PW_FINE: restricted first, i.e.
 * Lambda R) or on the coarse grid (PW_COARSE), in the state dtype, into
 * out (double, column-major, rows = (d+1) * n_coarse_points).           */
pw_status pw_energy_components(pw_ctx* ctx, int prob, int grid,
                               const void* u, const void* p,
                               double* out, int n_states);

/* Trigonometric interpolation and update (Algorithm 3, last line):
 * u_out[s] = v[s] + I(du[s]), p_out[s] = vp[s] + I(dp[s]), with du, dp
 * double coarse fields rounded to the state dtype before I.            */
pw_status pw_interp_add(pw_ctx* ctx, int prob, const double* du,
                        const double* dp, const void* v, const void* vp,
                        void* u_out, void* p_out, int n_states);

/* Lambda^dag displacement part (Algorithm 2, eq. gradient2coordinate):
 * w[s] = real(ifft(W)), W(xi) = -i xi.fft(q[s]) / |xi|^2, W(0) = sums[s];
 * q is n_states columns of d gradient blocks (double, d * n_coarse
 * rows each), w is n_states coarse double fields.                      */
pw_status pw_grad2func(pw_ctx* ctx, int prob, const double* q,
                       const double* sums, double* w, int n_states);

/* Algorithm 1 on the context's corrector of problem `prob`: given data
 * matrices F, G (double, rows x n_cols, column-major, device) update the
 * truncated SVD U S V^T of sum F G^T.  reset != 0 starts from an empty
 * SVD.  The new rank is returned in *rank (synchronises).               */
pw_status pw_update_svd(pw_ctx* ctx, int prob, const double* F,
                        const double* G, int n_cols, int reset, int* rank);

/* Copy the corrector of problem `prob` (U: rows x rank, S: rank,
 * V: rows x rank, double, column-major) to caller device buffers sized
 * for `cap` columns; PW_EINVAL if rank > cap.  With U, S and V all NULL
 * only the rank is returned.  Synchronises.                             */
pw_status pw_get_corrector(pw_ctx* ctx, int prob, double* U, double* S,
                           double* V, int cap, int* rank);

/* Discrete wave energy (eq. discrete-wave-energy) on the fine grid with
 * the fine medium and the context's gradient order (the fourth-order
 * central difference for a context with the spectral gradient), of the
 * difference [u - u_ref, p - p_ref] and of [u_ref, p_ref], in double
 * (synchronous; results to host).  u_ref may be NULL (then the energy of
 * [u, p]).                                                              */
pw_status pw_energy(pw_ctx* ctx, int prob, const void* u, const void* p,
                    const void* u_ref, const void* p_ref, double* e_diff,
                    double* e_ref);

/* Error measures of the Sec. 6 preamble on the fine grid, FP64 (host,
 * synchronous): out[0] = E([u - u_ref, p - p_ref]), out[1] = E([u_ref,
 * p_ref]) (as pw_energy), out[2] = sum (u - u_ref)^2, out[3] = sum u_ref^2
 * over the grid points (the l2 error of the displacement is
 * sqrt(out[2] / out[3])).  u_ref may be NULL (then out[0] = E([u, p]),
 * out[2] = sum u^2, out[1] = out[3] = 0).                              */
pw_status pw_error_norms(pw_ctx* ctx, int prob, const void* u, const void* p,
                         const void* u_ref, const void* p_ref, double* out);

/* Allocation-free form of pw_error_norms, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  No context: `desc` gives the fine
 * grid (dim, n_fine, 1 on unused axes), the gradient order (0 takes the
 * fourth-order difference, as pw_energy does for the spectral gradient) and
 * the state dtype; c is the fine-grid c^2 field (double, device, x fastest),
 * u, p, u_ref, p_ref device fields of the state dtype (u_ref, p_ref may both
 * be NULL), out a device buffer of 4 doubles that receives out[0..3] as
 * pw_error_norms (the same kernels, the same bits).  Runs asynchronously on
 * `stream` (NULL: the null stream) and allocates nothing: the reduction's
 * partial sums use a fixed 32 KiB device array of the library, one per GPU,
 * held until the process ends.  Grids of 2^31 points or more and bad
 * descriptions give PW_EINVAL before any device work.  All calls on one
 * GPU share that array: calls that overlap on one GPU (other streams or
 * host threads) race and must be serialised by the caller.            */
pw_status pw_energy_noalloc(const pw_problem* desc, const double* c,
                            const void* u, const void* p, const void* u_ref,
                            const void* p_ref, double* out, void* stream);

/* Checkpoint of the whole context: per problem the medium, u0, the current
 * iterate, kept history, corrector (U~, S~, V~, the sweep columns and
 * their coarse propagation C E), per-iteration records, comparator
 * variant, sampling table and source, written to the file `path` (host
 * byte order, format tag PWCKPT02; files written without C E still load,
 * and C E is then formed again at the next sweep).  pw_load restores
 * it into a context created with the same problem descriptions (PW_EINVAL
 * otherwise, or for a damaged file; the state is then unspecified until the
 * next set_* / run), after which pw_continue resumes the iteration exactly
 * where pw_save left it (bit for bit).  Tapes of taped runs are not saved.
 * Synchronous.                                                          */
pw_status pw_save(pw_ctx* ctx, const char* path);
pw_status pw_load(pw_ctx* ctx, const char* path);

/* Per-phase device time of the last pw_run in milliseconds, measured with
 * HIP events on the context stream: [0] parallel fine+coarse propagation,
 * [1] creating the corrector (data matrices + Algorithm 1), [2] corrected
 * sweep and update, [3] whole run; with cap >= 6 also [4] the last
 * pw_run_taped / pw_run_frozen and [5] the last pw_backward.  Host output,
 * synchronous.                                                          */
pw_status pw_get_timings(pw_ctx* ctx, int prob, double* ms_host, int cap);

/* ---- differentiation with respect to the medium ------------------------
 * Algorithm 3 is a composition of linear maps of the state whose only
 * dependence on the medium (besides the corrector) is through c^2 in the
 * propagators F and C of Sec. 3.1 (C sees the pointwise restriction of
 * c^2).  Holding the corrector theta^k = I Lambda^dag Omega^k Lambda of
 * eq. thetarelation fixed at the values a taped run produced (Omega^k from
 * Algorithm 1 and the c inside Lambda, Lambda^dag), the traces
 * u^{K+1}_n(x_r), n = 1..N, are differentiable in c^2 and their adjoint is
 * computed in FP64 by running every step in reverse: velocity Verlet
 * backwards (the forward trajectory recomputed from checkpoints), the
 * transposes of the interpolation I and restriction R, and the reduced
 * sweep recurrence transposed.                                           */

/* Algorithm 3 for K iterations as pw_run, recording a tape on the device:
 * the slice-start states of every iteration, the corrector pair of every
 * iteration and the coarse columns of the sweep (about
 * K*N*Nf*2*sizeof(state) + K*(4+2r)*Nc*8 bytes, owned by the context).
 * Asynchronous on the context stream except for the rank read-back of
 * Algorithm 1.                                                          */
pw_status pw_run_taped(pw_ctx* ctx, int prob, int K);

/* Algorithm 3 for K <= (K of the last pw_run_taped) iterations with the
 * recorded correctors instead of Algorithm 1 (no data matrices, no SVD),
 * using the current medium in F, C and R; re-records the states of the
 * tape.  Residuals are not formed (pw_get_residuals then reports 0
 * iterations).  PW_ESTATE without a prior taped run.                    */
pw_status pw_run_frozen(pw_ctx* ctx, int prob, int K);

/* Launch plan of one propagation F (grid = PW_FINE) or C (PW_COARSE) of
 * n_states states in one batch: the number of kernel launches and the time
 * steps each launch takes (the last one may take fewer).  Host only.     */
pw_status pw_launch_plan(pw_ctx* ctx, int prob, int grid, int n_states, int* launches,
                         int* steps_per_launch);

/* Serial number of the tape: bumped by every pw_run_taped and
 * pw_run_frozen, so a caller that keeps a gradient graph can tell whether
 * the tape pw_backward will read is still the one its forward recorded. */
pw_status pw_get_tape_id(pw_ctx* ctx, int prob, long long* id);

/* Traces of the current iterate: out[(n-1)*n_rec + r] = u_n(receivers[r])
 * for n = 1..N, receivers given as flat fine-grid indices (x fastest,
 * int64, all in [0, Nf) or PW_EINVAL).  on_device applies to receivers
 * and out (FP64, N x n_rec).  Synchronous.                               */
pw_status pw_traces(pw_ctx* ctx, int prob, const long long* receivers,
                    int n_rec, double* out, int on_device);

/* Gradient of J = sum_{n,r} seed[(n-1)*n_rec + r] u^{K+1}_n(receivers[r])
 * (the vector-Jacobian product of pw_traces) through the last taped or
 * frozen run, with its correctors held fixed.  grad: Nf doubles on the
 * fine grid, d J / d c^2 (wrt_velocity = 0) or d J / d c (= 2c dJ/dc^2,
 * wrt_velocity != 0).  For a misfit 1/2 sum (u - d)^2 pass seed = u - d.
 * The forward fine and coarse trajectories are recomputed from
 * checkpoints every `checkpoint_every` steps (<= 0: 64); results do not
 * depend on it.  on_device applies to receivers, seed and grad.
 * PW_ESTATE without a tape or after set_medium / set_initial since it was
 * recorded.  Work buffers (about (2*(N+1) + N*(4 + ckpt)) * Nf * 8 bytes
 * for ckpt <= m_F) are allocated on first use and kept.  Synchronous.   */
pw_status pw_backward(pw_ctx* ctx, int prob, const long long* receivers,
                      int n_rec, const double* seed, double* grad,
                      int on_device, int wrt_velocity, int checkpoint_every);

/* A receiver record of the current iterate sampled in time: one more
 * batched F sweep from the slice starts u_{n-1}, n = 1..N (with the layer
 * and source), recording u at the receivers after every fine step:
 * out[((n-1) * m_fine + i) * n_rec + r] = u of slice n after step i + 1 at
 * receiver r (FP64, N x m_fine x n_rec).  Receivers are distinct flat
 * fine-grid indices (x fastest, int64; PW_EINVAL for one outside [0, Nf)
 * or repeated).  2D problems only.  on_device applies to receivers and
 * out.  Synchronous.                                                     */
pw_status pw_trace_sweep(pw_ctx* ctx, int prob, const long long* receivers,
                         int n_rec, double* out, int on_device);

/* Gradient of J = sum seed[((n-1) * m_fine + i) * n_rec + r] * (the
 * record of pw_trace_sweep) through the last taped or frozen run, with its
 * correctors and the layer held fixed (the vector-Jacobian product of
 * pw_trace_sweep after that run).  For the misfit J = 1/2 dt sum (trace -
 * data)^2 of a record sampled every fine step pass seed = dt (trace -
 * data).  Arguments, checkpointing, work buffers and errors as
 * pw_backward (the record's sweep adds its N states to the fine adjoint).
 * Synchronous.                                                          */
pw_status pw_backward_sweep(pw_ctx* ctx, int prob, const long long* receivers,
                            int n_rec, const double* seed, double* grad,
                            int on_device, int wrt_velocity, int checkpoint_every);

#ifdef __cplusplus
}
#endif

#endif /* PW_H */
