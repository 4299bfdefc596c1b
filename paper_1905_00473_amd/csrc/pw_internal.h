// Internal declarations shared by the HIP translation units of libpwave.
// Not part of the public ABI (see include/pw.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pw.h"

namespace pw {

// ---------------------------------------------------------------------------
// error handling: internal functions throw pw::Error, the ABI layer turns it
// into a status code + thread-local message
// ---------------------------------------------------------------------------
struct Error {
  pw_status status;
  std::string msg;
};

[[noreturn]] void fail(pw_status st, const std::string& msg);
void check_hip(hipError_t e, const char* what, const char* file, int line);
#define PW_HIP(call) ::pw::check_hip((call), #call, __FILE__, __LINE__)
#define PW_LAUNCH_CHECK() ::pw::check_hip(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// grid geometry of one periodic grid (fine or coarse)
// ---------------------------------------------------------------------------
struct Grid {
  int dim = 1;
  int n[3] = {1, 1, 1};  // points per axis (x, y, z)
  double dx = 1.0;       // spacing (same on every axis)
  long long npts() const { return (long long)n[0] * n[1] * n[2]; }
};

// ---------------------------------------------------------------------------
// propagators (stencil.hip)
// ---------------------------------------------------------------------------
// Batched velocity-Verlet propagation of `nstates` states by `m` steps of
// size h on grid g.  State s is u[s*sstride ...], p[s*sstride ...].
// src and dst must not overlap.  work_* are scratch state sets used to
// ping-pong between time blocks (each nstates*sstride elements; the e*
// arrays are only used with compensation).  When m is done in a single
// launch the scratch sets are not touched.
// Absorbing layer, point source and receivers of a 2D propagation (the
// forcing of PW_SPONGE and pw_set_source, include/pw.h).  Every member is
// optional.  A kick of state s at level i first multiplies p by the
// layer's factor -- d at the first and last half kick of a slice, d^2
// where two half kicks meet, d = min(dmp_x[x], dmp_y[y]) = exp(-sigma h /
// 2) -- then adds its weight (h/2 or h/2 (1+d)) times c^2 Lap u + amp r(t)
// (the last term at the source node only; r(t) of state s at level i is
// src_tab[s src_stride + i], the wavelet at that state's slice time).
template <typename T>
struct Force {
  const T* dmp_x = nullptr;  // layer factor per column (null: no layer)
  const T* dmp_y = nullptr;  // per row
  int sx = -1, sy = -1;      // source node (sx < 0: no source)
  double amp = 0.0;          // weight 1 / dx^2
  const double* src_tab = nullptr;  // r(t) per state and level
  int src_stride = 0;
  // receivers: per row nonzero if the row holds one; per node its index or -1
  const int* rec_rows = nullptr;
  const int* rec_map = nullptr;
  // reverse pass (FP64) over many states: per-point fields of the layer,
  // wf = (1 + d) / 2, s2 = d^2, dd = d, c2e = c2 wf (null: from dmp_x/y)
  const double* wf = nullptr;
  const double* s2 = nullptr;
  const double* dd = nullptr;
  const double* c2e = nullptr;
  const long long* rec = nullptr;  // flat node of every receiver
  int n_rec = 0, m_tr = 0;         // receivers, steps per state of the record
  double* traces = nullptr;        // forward: u after step i of state s at [(s m_tr + i) n_rec + r]
  const double* seeds = nullptr;   // adjoint: added to the adjoint of that u, same layout
};

template <typename T>
struct StateSet {
  T* u = nullptr;
  T* p = nullptr;
  T* eu = nullptr;  // compensation terms (FP32 compensated mode only)
  T* ep = nullptr;
};

// `fine` only selects which (otherwise identical) kernel instantiation is
// launched, so that fine- and coarse-grid launches are told apart in traces.
// fo (2D grids only): the layer, source and receiver record of the
// propagation (null: none; see Force).
template <typename T>
void propagate(const Grid& g, const T* c2, const T* u_src, const T* p_src, T* u_dst, T* p_dst,
               long long sstride, int nstates, int m, T h, bool compensated, StateSet<T> work_a,
               StateSet<T> work_b, hipStream_t stream, bool fine = false,
               const Force<T>* fo = nullptr);

// largest number of steps one launch of the tiled kernel may take for this
// grid (the whole propagation when the grid is one periodic line in LDS)
int steps_per_launch(const Grid& g, bool is_double);
// launches and time steps per launch that propagate() takes for nstates
// states and m steps on grid g
void launch_plan(const Grid& g, bool is_double, int nstates, int m, int* launches, int* spl);

// Streams of one 2D problem in a launch of the streaming kernel: its
// in/out state sets, grid, and the first global wave index it owns.
template <typename T>
struct StreamDesc {
  const T* u_in;
  const T* p_in;
  const T* eu_in;
  const T* ep_in;
  T* u_out;
  T* p_out;
  T* eu_out;
  T* ep_out;
  const T* c2;
  long long sstride;
  int nx, ny;
  int ncb, nseg, Ly;  // column blocks, row segments, rows per segment
  int nstates;
  T h, idx2;
  int nsteps, first, last;
  long long wave_begin;
  // optional: u of every level produced by the launch, level j + 1 of the
  // launch at lv_out + j * lv_stride (state s at offset s * sstride)
  T* lv_out;
  long long lv_stride;
  // forced launches: layer, source, receivers and the level of the slice
  // at which this launch starts
  Force<T> f;
  int step0;
};

// one propagation of a batch: nstates states of one 2D problem by m steps
template <typename T>
struct PropJob {
  Grid g;
  const T* c2;
  const T* u_src;
  const T* p_src;
  T* u_dst;
  T* p_dst;
  long long sstride;
  int nstates;
  int m;
  T h;
  StateSet<T> wa, wb;
  int Ly = 0;  // target rows per stream of this job (0: the plan's Ly)
};

// Launch plan of a multi-problem batched propagation: launch l advances
// every job that still has steps by one time block of up to B steps.
// Tunables: B (pipeline depth, 4 or 8) and Ly (target rows per stream).
template <typename T>
struct MultiPlan {
  int B = 8;
  int Ly = 96;
  std::vector<int> first_desc;       // per launch: first descriptor index
  std::vector<int> ndesc;            // per launch: descriptor count
  std::vector<long long> nwaves;     // per launch
  std::vector<StreamDesc<T>> descs;  // all launches, host copy
};
template <typename T>
void plan_multi(const std::vector<PropJob<T>>& jobs, MultiPlan<T>& plan);
// descs_dev: device copy of plan.descs
template <typename T>
void run_multi(const MultiPlan<T>& plan, const StreamDesc<T>* descs_dev, bool comp,
               hipStream_t stream);

// ---------------------------------------------------------------------------
// grid transfer and energy components (transfer.hip)
// ---------------------------------------------------------------------------
// Scratch of the spectral (Fourier) gradient on the coarse grid, for up to
// `cols` fields: DFT tables per axis, complex work of 4 (d + 1) points
// x cols doubles, real work of d points x cols, restricted fields of
// points x cols.
struct SpecScratch {
  const double* const* dft = nullptr;
  double* ctmp = nullptr;
  double* rtmp = nullptr;
  double* ures = nullptr;
  int cols = 0;
};

// out[col * ldo + a * np + J] = D_a in_col (the Fourier derivative
// real(ifft(i xi_a fft(in)))) for a < d, columns of np points, ld ldi
void spectral_grad_cols(const Grid& grid, const SpecScratch& sp, const double* in,
                        long long ldi, int ncols, double* out, long long ldo,
                        hipStream_t stream);
// out[col * ldo + J] = -sum_a D_a q_a, q_a = in[col * ldi + a * np ..]
// (the transpose of the Fourier gradient, which is skew-symmetric)
void spectral_div_cols(const Grid& grid, const SpecScratch& sp, const double* in,
                       long long ldi, int ncols, double* out, long long ldo,
                       hipStream_t stream);

// out[:, s] = Lambda R [u_s, p_s] (double columns, rows = (d+1) * coarse
// points).  `ratio` = 1 when u, p already live on the coarse grid.  order
// 0 = spectral gradient (needs sp).
template <typename T>
void energy_columns(const Grid& fine_or_coarse, int ratio, const Grid& coarse, const T* u,
                    const T* p, long long sstride, const double* cc, int order, double* out,
                    long long ldo, int nstates, hipStream_t stream,
                    const SpecScratch* sp = nullptr);

// out[:, s] = [R(a_u - b_u) ; R(a_p - b_p)] as double coarse states
// (column length 2 * coarse points, leading dimension ldo).  Column s uses
// state s of a and b.
template <typename T>
void restrict_diff(const Grid& fine, int ratio, const Grid& coarse, const T* au, const T* ap,
                   const T* bu, const T* bp, long long sstride, double* out, long long ldo,
                   int nstates, hipStream_t stream);

// coarse T state from a double state column: u_T = (T) x (elementwise cast)
template <typename T>
void cast_from_double(const double* in, T* out, long long n, hipStream_t stream);
template <typename T>
void cast_to_double(const T* in, double* out, long long n, hipStream_t stream);
template <typename T>
void restrict_fields(const Grid& fine, int ratio, const Grid& coarse, const T* in,
                     long long sstride_in, T* out, long long sstride_out, int nfields,
                     hipStream_t stream);

// polyphase weights of trigonometric interpolation along one axis:
// table[s * nc + d], s in [0, ratio), d in [0, nc) (host-built)
std::vector<double> trig_interp_table(int nc, int ratio);
// the same layout for periodic piecewise-linear interpolation
std::vector<double> linear_interp_table(int nc, int ratio);
// and for local cubic (4-point Lagrange) interpolation
std::vector<double> cubic_interp_table(int nc, int ratio);

// u_out[s] = (v ? v[s] : 0) + I(in[s]) on the fine grid, fields of type T.
// tmp: double scratch of nfields * (fine points) * 2 elements.
template <typename T>
void interp_add(const Grid& fine, const Grid& coarse, int ratio, const double* const* tables,
                const T* in, long long sstride_in, const T* v, T* out, long long sstride_out,
                int nfields, double* tmp, hipStream_t stream);

// DFT tables e^{-2 pi i j / n}, j < n, for each axis of the coarse grid
std::vector<double> dft_table(int n);

// w[s] = grad2func(q[s], sums[s]) (Algorithm 2) for n columns; q columns
// hold d gradient blocks with leading dimension ldq; w columns have
// leading dimension ldw.  sums may be null (all zero).  ctmp: complex
// scratch (double2) of (d + 1) * coarse points * ncols elements.
void grad2func_cols(const Grid& coarse, const double* const* dft, const double* q, long long ldq,
                    const double* sums, double* w, long long ldw, int ncols, double* ctmp,
                    hipStream_t stream);

// Adjoint of Lambda on coarse energy-component columns:
// out_u = -sum_a grad_a(q_a) (gradient order `order`), out_p = p / cc.
// in: rows (d+1)*Nc, ld ldi; out: 2*Nc rows, ld ldo.
void lambda_adjoint_cols(const Grid& coarse, const double* in, long long ldi, const double* cc,
                         int order, double* out, long long ldo, int ncols, hipStream_t stream,
                         const SpecScratch* sp = nullptr);

// Lambda^dag of energy-component columns: out_u = grad2func(q, sums[col])
// (sums null: all zero), out_p = cc * p.
void lambda_dag_cols(const Grid& coarse, const double* const* dft, const double* in,
                     long long ldi, const double* cc, const double* sums, double* out,
                     long long ldo, int ncols, double* ctmp, hipStream_t stream);

// set column `col` of a 2*Nc-row matrix to [val_u * 1 ; 0]
void set_dc_column(double* mat, long long ld, int col, long long nc, double val,
                   hipStream_t stream);

// energy of fine-grid state differences (double partials on device, reduced
// on device in a fixed order).  result[0] = E(u - uref), result[1] = E(uref),
// result[2] = sum (u - uref)^2, result[3] = sum uref^2 (uref null: the
// energy and the sum of squares of [u, p]).  partials: kEnergyPartials
// doubles, every one written by each call.
template <typename T>
void energy_pair(const Grid& fine, const T* u, const T* p, const T* uref, const T* pref,
                 const double* cfine, int order, double* partials, double* result,
                 hipStream_t stream);
constexpr int kEnergyPartials = 4096;

// message of the last failing ABI call on this thread (pw_last_error)
void set_last_error(const std::string& msg);

// ---------------------------------------------------------------------------
// dense linear algebra (linalg.hip)
// ---------------------------------------------------------------------------
// C (a x b, ldc) = alpha * A^T B + beta * C with A (rows x a, lda),
// B (rows x b, ldb), column-major.  FP64 MFMA, split over rows, fixed-order
// reduction.  work: double scratch >= gemm_tn_work(rows, a, b).
// work needed by one call, and an upper bound over every a <= a_max,
// b <= b_max (the split count shrinks as the tile count grows, so the
// per-call need is not monotonic in a or b).  gemm_tn fails if work_elems
// is too small for the call.
size_t gemm_tn_work(long long rows, int a, int b);
size_t gemm_tn_work_bound(int a_max, int b_max);
void gemm_tn(long long rows, int a, int b, double alpha, const double* A, long long lda,
             const double* B, long long ldb, double beta, double* C, long long ldc, double* work,
             size_t work_elems, hipStream_t stream);

// C (rows x n, ldc) = alpha * A (rows x k, lda) B (k x n, ldb) + beta * C.
// FP64 MFMA.  C must not overlap A or B (it may be read when beta != 0).
void gemm_nn(long long rows, int n, int k, double alpha, const double* A, long long lda,
             const double* B, long long ldb, double beta, double* C, long long ldc,
             hipStream_t stream);

// small dense products: C (m x n) = alpha op(A) op(B) + beta C (column-major)
void gemm_small(int m, int n, int k, double alpha, const double* A, int lda, bool ta,
                const double* B, int ldb, bool tb, double beta, double* C, int ldc,
                hipStream_t stream);

// Orthonormalisation for the truncated QR of Algorithm 1 (two passes of
// pivoted Cholesky QR): A (rows x n, n <= 64) = Q R approximately; Q (rows x
// n, ldq), R (n x n).  Directions whose pivot is below 1e-15 times the
// largest diagonal of A^T A are dropped (zero Q column, zero R row).
struct OrthScratch {
  double* gram = nullptr;   // n*n (n <= 64)
  double* T = nullptr;      // n*n (n <= 64)
  double* info = nullptr;   // 2: pivoted Cholesky report
  // accept the Gram-based truncation at ~sqrt(eps) of the largest
  // direction whatever the conditioning (data from FP32 states, whose own
  // rounding is larger than that)
  bool gram_enough = false;
  double* R1 = nullptr;     // n*n
  double* R2 = nullptr;     // n*n
  double* Q1 = nullptr;     // rows*min(n, 64): reflectors of the first TSQR level
  double* hw = nullptr;     // TSQR stacked R factors (tsqr_work)
  double* htau = nullptr;   // TSQR reflector scalars (tsqr_work)
  double* W = nullptr;      // rows*64 (only for n > 64 columns)
  double* C = nullptr;      // n*64 (only for n > 64 columns)
  double* work = nullptr;   // gemm_tn work
  size_t work_elems = 0;
};
// workspace of the Householder TSQR of a rows x min(n, 64) block
void tsqr_work(long long rows, int n, size_t* stack_elems, size_t* tau_elems);
// A (rows x n) = Q R inside Algorithm 1 (Q with ld ldq, R n x n), in
// three steps so that two factorisations on two streams can be started
// before either stream is synchronised: orth_begin enqueues the Gram
// matrix and its pivoted Cholesky factor, orth_choose synchronises the
// stream and returns whether Cholesky QR is accurate enough, orth_finish
// enqueues the chosen method (Cholesky QR twice or Householder TSQR)
void orth_begin(long long rows, int n, const double* A, long long lda, const OrthScratch& s,
                hipStream_t stream);
bool orth_choose(long long rows, int n, const OrthScratch& s, hipStream_t stream);
void orth_finish(long long rows, int n, const double* A, long long lda, double* Q, long long ldq,
                 double* R, const OrthScratch& s, bool cholqr, hipStream_t stream);

// one-sided Jacobi SVD of the n x n matrix H (column-major, ld = n):
// on return X (n x n, ld n) holds left singular vectors, Y right singular
// vectors, sig singular values, sorted descending; *rank_dev the number
// with sig/sig_max > tol.  Scratch: Hw (2 n*n + 3n + 16), Vw (2 n*n),
// counters (40 ints); sig must hold max(n, 512) doubles.
void svd_jacobi(int n, const double* H, double* X, double* Y, double* sig, double tol,
                int* rank_dev, double* Hw, double* Vw, int* counters, hipStream_t stream);

// the arguments of one svd_jacobi call
struct SvdJob {
  int n;
  const double* H;
  double *X, *Y, *sig;
  double tol;
  int* rank_dev;
  double *Hw, *Vw;
  int* counters;
};
// svd_jacobi of every job, the block pairs of all of them in one launch per
// round (same results as separate calls).  jobs_dev: device scratch of
// 2 * jobs.size() * svd_multi_job_bytes() bytes; counts_dev: jobs.size()
// ints.  Synchronises the stream once per sweep.
size_t svd_multi_job_bytes();
void svd_jacobi_multi(const std::vector<SvdJob>& jobs, void* jobs_dev, int* counts_dev,
                      hipStream_t stream);

// linear recurrence t_1 = b_1, t_n = b_n + M t_{n-1} (t, b: dim x N
// column-major, M: dim x dim).  Scratch: two dim x dim matrices and two
// dim x N blocks.
struct RecScratch {
  double* P0 = nullptr;
  double* P1 = nullptr;
  double* ta = nullptr;
  double* tb = nullptr;
};
void recurrence(int dim, int N, const double* M, const double* b, double* t, RecScratch rs,
                hipStream_t stream);

// H = [Ua; Ra][Vb; Rb]^T + diag(S, 0): (r+N) x (r+N) helper pieces
void add_diag(int n, int r, const double* S, double* H, int ldh, hipStream_t stream);
void copy_block(int m, int n, const double* src, long long lds, double* dst, long long ldd,
                hipStream_t stream);
void fill(double* p, long long n, double v, hipStream_t stream);
// out[0] = x[0] + ... + x[n-1] (one workgroup, fixed order; n = 0 gives 0)
void vec_sum(const double* x, int n, double* out, hipStream_t stream);
void frob_norm2(const double* A, long long rows, int cols, long long lda, double* partials,
                double* out, hipStream_t stream);

// ---------------------------------------------------------------------------
// adjoint building blocks (adjoint.hip), FP64
// ---------------------------------------------------------------------------
// Scratch of vv_adjoint: one "time level" holds ns states of np points
// (state_elems >= ns * np).  ck_u / ck_p: max_ckpt levels (checkpoints);
// seg: max_seg levels (displacements of one recomputed segment);
// p_tmp, p_tmp2, a_tmp, lp_tmp: one level each.
struct AdjScratch {
  long long state_elems = 0;
  int max_ckpt = 0, max_seg = 0;
  double* ck_u = nullptr;
  double* ck_p = nullptr;
  double* seg = nullptr;
  double* p_tmp = nullptr;
  double* p_tmp2 = nullptr;
  double* a_tmp = nullptr;
  double* lp_tmp = nullptr;
};

// Leapfrog form of m velocity-Verlet steps of nstates 2D FP64 states
// (stride sstride), the state carried being (u_i, p_{i-1/2}): from
// (u_src, p_src) at level i0, every step kicks (weight h/2 if it is level 0
// of the trajectory, `level0`, else h) and drifts; u of levels i0+1..i0+m
// goes to lv + (k - 1) lv_stride, k = 1..m.  p ping-pongs between pa and pb
// (both distinct from p_src); the returned pointer holds p_{i0+m-1/2}.
// No closing half kick.  fo: the layer and source of the trajectory (its
// receiver members are ignored), i0 the level of the slice at u_src.
const double* leapfrog_levels2d(const Grid& g, const double* c2, const double* u_src,
                                const double* p_src, double* pa, double* pb, long long sstride,
                                int nstates, int m, double h, bool level0, double* lv,
                                long long lv_stride, hipStream_t stream,
                                const Force<double>* fo = nullptr, int i0 = 0);

// Reverse of m velocity-Verlet steps (size h, medium c2) of ns states whose
// inputs are (u0, p0) (state s at offset s * s0).  (lu, lp) hold the adjoint
// of the outputs on entry and of the inputs on return (stride sl);
// the ns fields gacc[s * sg + J] receive d J / d c2(J) of the ns states:
// only their sum over s is defined (states 8q .. 8q+7 add their
// contributions of a reverse step to field q).  The forward trajectory is
// recomputed from checkpoints taken every `ckpt` steps.  fo (2D only):
// the layer and source of the forward propagation (the adjoint applies the
// layer's factors; the source enters only the recomputed trajectory) and,
// with fo->seeds, the derivative of J with respect to u at the receivers
// after every step, added to the adjoint as the reverse pass reaches it.
void vv_adjoint(const Grid& g, const double* c2, const double* u0, const double* p0,
                long long s0, double* lu, double* lp, long long sl, double* gacc, long long sg,
                int ns, int m, double h, int ckpt, const AdjScratch& sc, hipStream_t stream,
                const Force<double>* fo = nullptr);

// the fields wf, s2, dd, c2e (see Force) of the layer with per-axis factor
// tables dmx, dmy on grid g and medium c2, into out (4 npts doubles, in
// that order)
void layer_fields(const Grid& g, const double* dmx, const double* dmy, const double* c2,
                  double* out, hipStream_t stream);

template <typename T>
void widen_fields(const T* in, long long si, double* out, long long so, long long np, int ns,
                  hipStream_t stream);
void copy_fields(const double* in, long long si, double* out, long long so, long long np, int ns,
                 hipStream_t stream);
// transpose of interp (without the added base field): fine fields -> coarse
void interp_transpose(const Grid& fine, const Grid& coarse, int ratio,
                      const double* const* tables, const double* in, long long sin, double* out,
                      long long sout, int nfields, double* tmp, hipStream_t stream);
// out[fine node ratio * J] += scale * in[J] (transpose of the restriction)
void restrict_transpose_add(const Grid& fine, int ratio, const Grid& coarse, const double* in,
                            long long sin, double* out, long long sout, double scale,
                            int nfields, hipStream_t stream);
// out[J] (+)= sum over ns fields in[s * si + J], summed in field order
void sum_fields(const double* in, long long si, int ns, double* out, long long np, bool acc,
                hipStream_t stream);
// res[n][r] = u_n(rec[r]) - data[n][r] (data may be null: zero)
template <typename T>
void receiver_values(const T* u, long long su, const long long* rec, int nrec, int nst,
                     double* out, hipStream_t stream);
// lam[n * sl + rec[r]] += seed[n][r], receivers handled in order (no atomics)
void receiver_scatter(const double* seed, const long long* rec, int nrec, int nst, double* lam,
                      long long sl, hipStream_t stream);
// dst column j = src column (n - 1 - j), m rows
void reverse_cols(int m, int n, const double* src, long long lds, double* dst, long long ldd,
                  hipStream_t stream);
// out[J] = scale * a[J] * b[J]
void mul_fields(const double* a, const double* b, double* out, long long n, double scale,
                hipStream_t stream);

// x neighbours through the DPP wavefront shifts (wave_shr:1 = 0x138 reads
// lane - 1, wave_shl:1 = 0x130 reads lane + 1): a modifier of a VALU move
// instead of an LDS-crossbar permute and its lane-index arithmetic.  Lanes
// 0 and 63 read 0 (the callers use them as halo lanes only); every lane of
// the wave must be active at the call.
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

}  // namespace pw
