// C ABI of libpwave: context, device memory plan and the driver of
// Algorithm 3 (eq. thetarelation) of Nguyen & Tsai.
//
// One iteration on the device:
//  1. parallel phase: v_n = F u^k_{n-1} for all n in one batched launch
//     sequence; U_n = C R u^k_{n-1} batched on the coarse grid;
//  2. corrector: data matrices F^k = [Lambda R v_n], G^k = [Lambda U_n],
//     Algorithm 1 (projections on the FP64 matrix cores, Gram-eigenvector
//     orthonormalisation, one-sided Jacobi SVD of the core, basis rotation);
//  3. corrected sweep.  By linearity of C, Lambda, Omega and Lambda^dag the
//     serial loop of Algorithm 3 is carried in the coordinates of the
//     corrector: with delta_n = u^{k+1}_n - v_n on the coarse grid,
//        Delta_n = C R u^{k+1}_{n-1} - C R u^k_{n-1} = a_n + C delta_{n-1},
//        a_n = C (R v_{n-1} - R u^k_{n-1}),
//        delta_n = Lambda^dag_u Omega Lambda Delta_n (+ the mean term)
//                = E t_n,  t_n = P^T Delta_n,
//     where E = [Lambda^dag_u U~ , 1/Nc ; c U~_p , 0] and
//     P = [Lambda^T V~ , 1_u] (Lambda^T = [-div_h ; 1/c]).  Hence
//        t_n = P^T a_n + (P^T C E) t_{n-1},
//     an (r+1)-dimensional recurrence; the a_n and C E are batched coarse
//     propagations and the products are matrix-core GEMMs.  Slices whose
//     inputs did not change get a_n = 0 and t_n = 0 exactly, so the
//     exactness of the first k slices after k iterations is kept.
//  4. u^{k+1}_n = v_n + I(delta_n) for all n (R I = 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pw_internal.h"

namespace pw {

void fail(pw_status st, const std::string& msg) { throw Error{st, msg}; }

void check_hip(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  char buf[512];
  snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  fail(e == hipErrorOutOfMemory ? PW_ENOMEM : PW_EHIP, buf);
}

namespace {

thread_local std::string g_last_error;

// per-iteration device record: [0] ||F - Omega G||_F^2, [1] ||F||_F^2 (all N
// columns), [2] ||F_in||_F^2, [3] ||G_in||_F^2 (the columns entering
// Algorithm 1), [4] trace of S~ after the update
constexpr int kRes = 5;
// host threads driving the per-problem corrector and sweep of a batch
constexpr int kBatchThreads = 8;
// values per iteration returned by pw_get_diagnostics
constexpr int kPwDiag = 8;

struct Buffers {
  std::vector<void*> ptrs;
  void* get(size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      char buf[160];
      snprintf(buf, sizeof(buf), "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      fail(PW_ENOMEM, buf);
    }
    ptrs.push_back(p);
    return p;
  }
  template <typename T>
  T* get_n(long long n) {
    return (T*)get(sizeof(T) * (size_t)std::max(1LL, n));
  }
  ~Buffers() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

// Record of a taped forward run, read by the backward pass: the slice-start
// states of every iteration, the coarse columns of the reduced sweep and the
// frozen corrector pair (E_k, P_k) of every iteration.
struct Tape {
  std::unique_ptr<Buffers> mem;
  int Kcap = 0;             // iterations the buffers hold
  int K = 0;                // iterations of the last taped / frozen run
  int Kc = 0;               // iterations with recorded correctors
  long long epoch = -1;     // medium/initial epoch of the recorded run
  void* us = nullptr;       // (Kcap + 1) x N fields, state dtype: u^k_n, n = 0..N-1
  void* ps = nullptr;
  double* W = nullptr;      // 2Nc x N: initialisation coarse states W_0..W_{N-1}
  double* Din = nullptr;    // Kcap x (2Nc x N)
  double* delta = nullptr;  // Kcap x (2Nc x N)
  double* E = nullptr;      // Kcap x (2Nc x (rmax + 1))
  double* P = nullptr;
  std::vector<int> dims;
  // backward work, allocated on first use
  std::unique_ptr<Buffers> bw;
  int bw_ckpt = 0;
  double *La = nullptr, *Lb = nullptr;   // (N + 1) slots of [u; p] fine adjoints
  double* Wf = nullptr;                  // N slots of [u; p] widened fine states
  double *GF = nullptr, *GC = nullptr;   // per-state gradient accumulators
  double *gc = nullptr, *grad = nullptr, *c2f = nullptr;
  double *Y = nullptr, *LA = nullptr, *X = nullptr;  // 2Nc x N
  double *Cn = nullptr, *Cr = nullptr, *Sr = nullptr, *Sn = nullptr, *MT = nullptr;
  double *layF = nullptr, *layC = nullptr;  // layer fields (wf, s2, dd, c2e) per grid
  AdjScratch as;
};

// growable device staging buffer
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void* ensure(size_t b) {
    if (b <= bytes) return p;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      fail(PW_ENOMEM, "hipMalloc of a staging buffer failed");
    }
    bytes = b;
    return p;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct Prob {
  pw_problem P{};
  Grid gf, gc;
  int ratio = 1, N = 1, mF = 1, mC = 1, order = 4;
  double hF = 0, hC = 0, tol = 1e-14;
  bool f64 = true, comp = false;
  long long Nf = 0, Nc = 0, rows = 0;
  int rmax = 0, cap = 0;
  size_t tsize = 8;

  Buffers mem;
  // medium
  double* cf = nullptr;   // fine c
  double* cc = nullptr;   // coarse c
  void* c2f = nullptr;    // fine c^2, state dtype
  void* c2c = nullptr;    // coarse c^2, state dtype
  double* c2c_d = nullptr;
  double* itab[3] = {nullptr, nullptr, nullptr};
  double* dtab[3] = {nullptr, nullptr, nullptr};
  // fine states (state dtype)
  void *u = nullptr, *p = nullptr;    // (N+1) fields: u^k_n
  void *v = nullptr, *vp = nullptr;   // N fields: v_n at index n-1
  void *fw[2][4] = {{nullptr}};       // fine work sets (u, p, eu, ep), N fields each
  void *sfa_u = nullptr, *sfa_p = nullptr, *sfb_u = nullptr, *sfb_p = nullptr;  // serial fine
  // coarse states (state dtype)
  void *Uc = nullptr, *Ucp = nullptr;  // U_n, N fields
  void *Rc = nullptr, *Rcp = nullptr;  // restricted inputs, N+1 fields
  void *cw[2][4] = {{nullptr}};       // coarse work sets, N+1 fields
  void *du_T = nullptr, *dp_T = nullptr;  // cast corrections, N fields
  // coarse FP64
  double* Din = nullptr;   // 2Nc x N
  double* Acol = nullptr;  // 2Nc x N
  double* E[2] = {nullptr, nullptr};   // 2Nc x cap
  double* Vp[2] = {nullptr, nullptr};  // 2Nc x cap
  double* CE = nullptr;                // 2Nc x (rmax+1), scratch
  // C E[cur] carried along with E: the new directions of an update are
  // propagated once and the rest rotates with E (C is linear)
  double* CEb[2] = {nullptr, nullptr};  // 2Nc x cap
  double* cdc = nullptr;                // C applied to the DC column, 2Nc
  bool ce_ok = false;                   // CEb[cur](:, 0:r+1) = C E[cur](:, 0:r+1)
  bool cdc_ok = false;
  double* dw[2] = {nullptr, nullptr};  // FP64 coarse work, 2Nc x max(rmax+1, N)
  double* delta = nullptr;             // 2Nc x N
  // corrector
  double *Fm = nullptr, *Gm = nullptr;        // rows x N
  double *Fp = nullptr, *Gp = nullptr;        // rows x N
  double* Ub[2] = {nullptr, nullptr};         // rows x cap
  double* Vb[2] = {nullptr, nullptr};
  double* S = nullptr;                        // cap
  double *UF = nullptr, *VG = nullptr, *UF2 = nullptr, *VG2 = nullptr;  // cap x N
  double *RF = nullptr, *RG = nullptr;        // N x N
  double *Af = nullptr, *Bg = nullptr;        // cap x N
  double *H = nullptr, *X = nullptr, *Y = nullptr, *sig = nullptr, *Hw = nullptr, *Vw = nullptr;
  int* counters = nullptr;
  int* rank_dev = nullptr;
  double *M = nullptr, *Bn = nullptr, *Tn = nullptr;
  RecScratch rs;
  double* ctmp = nullptr;   // complex DFT scratch
  double* itmp = nullptr;   // interpolation scratch
  double* gwork = nullptr;  // split-K partials
  double* gwork2 = nullptr; // split-K partials of the G branch of Algorithm 1
  size_t gwork_elems = 0;
  double* red = nullptr;    // reduction partials
  double* res = nullptr;    // per-iteration [||F - Omega G||^2, ||F||^2]
  OrthScratch os, os2;  // orthonormalisation scratch of the F and the G branch
  // Algorithm 1 treats the F-side and the G-side data independently up to
  // the core matrix: the G branch runs on a second stream, forked from and
  // joined to the caller's stream with events
  hipStream_t side = nullptr;
  // batched runs: this problem's corrector and sweep run on its own stream,
  // concurrently with the other problems' (joined with done_ev)
  hipStream_t own = nullptr;
  hipEvent_t done_ev = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  hipEvent_t pre_ev = nullptr;  // batch: this problem's core matrix is formed
  int variant = PW_VARIANT_THETA;  // iteration run by pw_run
  DevBuf samp;                     // sampled data columns, samp_iters x samp_n
  int samp_n = 0, samp_iters = 0;
  // randomised sketching in Algorithm 1: test matrices (sk_iters x N x sk_l),
  // range-finder scratch of the F and the G branch
  DevBuf sk, skYf, skYg, skZf, skZg;
  int sk_l = 0, sk_iters = 0, sk_power = 0;
  double* vsum = nullptr;          // column sum of the Omega = I chain
  SpecScratch spec;                // spectral gradient (grad_order 0)
  int cur = 0;    // which of the ping-pong corrector buffers is current
  int r = 0;      // current rank
  int k_done = 0;
  bool have_medium = false, have_initial = false;
  bool have_iterate = false;  // u^{k_done+1}_n exists (after a run, a continue or a load)
  std::vector<int> ranks;
  // iterate history (keep_history): level k-1 holds u^k_n, n = 1..N
  // ((max_iters + 1) levels of N fields; u^k_0 = u0 for every k)
  void *hist_u = nullptr, *hist_p = nullptr;
  DevBuf prev;                 // u^k_n, n = 1..N, for the stopping rule without history
  double* chg = nullptr;       // device: N x 4 energy sums of u^{k+1}_n - u^k_n
  std::vector<double> change;  // per iteration: max_n sqrt(E(u^{k+1}_n - u^k_n) / E(u^{k+1}_n))
  long long tape_serial = 0;   // bumped by every taped or frozen run
  double ms[4] = {0, 0, 0, 0};
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> pev;  // per-iteration phase events (4 per iteration)
  // absorbing layer (PW_SPONGE) and point source (pw_set_source), 2D:
  // per-axis layer factors exp(-sigma_a h / 2) of the fine and the coarse
  // grid ([x | y], nx + ny values), in the state dtype and in double
  bool sponge = false;
  double sponge_smax = 0.0;
  void *layF_t = nullptr, *layC_t = nullptr;
  double *layF_d = nullptr, *layC_d = nullptr;
  bool have_src = false;
  double src_pos[3] = {0, 0, 0}, src_freq = 0.0, src_t0 = 0.0;
  int srcF[2] = {-1, -1}, srcC[2] = {-1, -1};  // nearest fine / coarse node (x, y)
  // the wavelet at every level of every slice: [n - 1][i] = r((n - 1) T / N
  // + i h), n = 1..N, i = 0..m, for the fine and the coarse step
  DevBuf srcF_tab, srcC_tab;
  // receiver record (pw_trace_sweep, pw_backward_sweep): per-row flags,
  // per-node receiver index, the sweep's output states
  DevBuf rec_rows, rec_map, trace_u, trace_p;
  // adjoint
  long long epoch = 0;     // bumped by set_medium / set_initial / set_source
  std::unique_ptr<Tape> tape;
  DevBuf stage_rec, stage_seed, stage_out;
  double adj_ms[2] = {0, 0};  // last taped forward, last backward
  ~Prob() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : pev)
      if (e) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (pre_ev) (void)hipEventDestroy(pre_ev);
    if (side) (void)hipStreamDestroy(side);
    if (own) (void)hipStreamDestroy(own);
    if (done_ev) (void)hipEventDestroy(done_ev);
  }
};

}  // namespace
}  // namespace pw

namespace pw {
namespace {
// Lockstep execution of all problems of a context: the parallel phase of
// every problem (fine sweep over all slices, restriction, coarse U_n) is
// one launch sequence of the multi-problem streaming kernel, captured once
// in a hipGraph and replayed every iteration.
struct Batch {
  bool built = false;
  bool f64 = false, comp = false;
  MultiPlan<float> F32, C32;
  MultiPlan<double> F64, C64;
  void* dF = nullptr;  // device descriptor tables
  void* dC = nullptr;
  Buffers mem;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int B = 0, Ly = 0;
  std::vector<std::pair<int, int>> ly_by_size;  // (fine ny, rows per stream) overrides
  double tune_ms = 0.0;   // time spent tuning
  double best_ms = 0.0;   // fine sweep time of the chosen configuration
  bool from_cache = false;
  double ms[4] = {0, 0, 0, 0};
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork_ev = nullptr;  // end of the parallel phase (problem streams wait on it)
  hipEvent_t svd_ev = nullptr;   // the problems' SVDs are done
  void* svd_jobs = nullptr;      // device scratch of svd_jacobi_multi
  int* svd_counts = nullptr;
  ~Batch() {
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (svd_ev) (void)hipEventDestroy(svd_ev);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};
}  // namespace
}  // namespace pw

struct pw_ctx {
  hipStream_t stream = nullptr;
  std::vector<std::unique_ptr<pw::Prob>> probs;
  std::unique_ptr<pw::Batch> batch;
};

namespace pw {
namespace {

template <typename T>
T* tp(void* x) {
  return reinterpret_cast<T*>(x);
}

Prob& get_prob(pw_ctx* ctx, int i) {
  if (!ctx) fail(PW_EINVAL, "null context");
  if (i < 0 || i >= (int)ctx->probs.size()) fail(PW_EINVAL, "problem index out of range");
  return *ctx->probs[i];
}

void validate(const pw_problem& P) {
  if (P.dim < 1 || P.dim > 3) fail(PW_EINVAL, "dim must be 1, 2 or 3");
  for (int a = 0; a < 3; ++a) {
    if (a < P.dim && P.n_fine[a] < 1) fail(PW_EINVAL, "n_fine must be positive");
    if (a >= P.dim && P.n_fine[a] != 1) fail(PW_EINVAL, "unused axes must have n_fine = 1");
  }
  if (P.ratio < 1) fail(PW_EINVAL, "ratio must be >= 1");
  for (int a = 0; a < P.dim; ++a) {
    if (P.n_fine[a] % P.ratio) fail(PW_EINVAL, "ratio must divide every n_fine");
    if (P.n_fine[a] / P.ratio < 5) fail(PW_EINVAL, "coarse grid needs at least 5 points per axis");
  }
  if (!(P.T > 0)) fail(PW_EINVAL, "T must be positive");
  if (P.n_slices < 1 || P.m_fine < 1 || P.m_coarse < 1) fail(PW_EINVAL, "bad slice/step counts");
  if (P.grad_order != 0 && P.grad_order != 2 && P.grad_order != 4 && P.grad_order != 6 &&
      P.grad_order != 8)
    fail(PW_EINVAL, "grad_order must be 2, 4, 6, 8 or 0 (spectral)");
  if (!(P.svd_tol > 0)) fail(PW_EINVAL, "svd_tol must be positive");
  if (P.state_dtype != PW_F32 && P.state_dtype != PW_F64) fail(PW_EINVAL, "bad state dtype");
  if (P.compensated && P.state_dtype != PW_F32) fail(PW_EINVAL, "compensation is an FP32 mode");
  if (P.max_iters < 1) fail(PW_EINVAL, "max_iters must be >= 1");
  if (P.interp != PW_INTERP_TRIG && P.interp != PW_INTERP_LINEAR && P.interp != PW_INTERP_CUBIC)
    fail(PW_EINVAL, "interp must be PW_INTERP_TRIG, PW_INTERP_LINEAR or PW_INTERP_CUBIC");
  if (P.keep_history != 0 && P.keep_history != 1) fail(PW_EINVAL, "keep_history must be 0 or 1");
  if (P.bc != PW_PERIODIC && P.bc != PW_SPONGE) fail(PW_EINVAL, "bc must be PW_PERIODIC or PW_SPONGE");
  if (P.bc == PW_SPONGE) {
    if (P.dim != 2) fail(PW_EINVAL, "the absorbing layer is implemented for 2D problems only");
    if (!(P.sponge_width > 0 && P.sponge_width < 0.5))
      fail(PW_EINVAL, "sponge_width must be in (0, 0.5)");
    if (!(P.sponge_reflection >= 0 && P.sponge_reflection < 1))
      fail(PW_EINVAL, "sponge_reflection must be in [0, 1) (0: 1e-3)");
    if (!(P.sponge_cmax >= 0) || !std::isfinite(P.sponge_cmax))
      fail(PW_EINVAL, "sponge_cmax must be >= 0 (0: from the medium)");
  }
}

void setup(Prob& pr, const pw_problem& P) {
  validate(P);
  pr.P = P;
  pr.ratio = P.ratio;
  pr.N = P.n_slices;
  pr.mF = P.m_fine;
  pr.mC = P.m_coarse;
  pr.order = P.grad_order;
  pr.tol = P.svd_tol;
  pr.f64 = P.state_dtype == PW_F64;
  pr.comp = P.compensated != 0;
  pr.tsize = pr.f64 ? 8 : 4;
  pr.gf.dim = pr.gc.dim = P.dim;
  for (int a = 0; a < 3; ++a) {
    pr.gf.n[a] = P.n_fine[a];
    pr.gc.n[a] = a < P.dim ? P.n_fine[a] / P.ratio : 1;
  }
  pr.gf.dx = 1.0 / P.n_fine[0];
  pr.gc.dx = pr.gf.dx * P.ratio;
  const double dtc = P.T / P.n_slices;
  pr.hF = dtc / P.m_fine;
  pr.hC = dtc / P.m_coarse;
  pr.Nf = pr.gf.npts();
  pr.Nc = pr.gc.npts();
  pr.rows = (long long)(P.dim + 1) * pr.Nc;
  pr.rmax = (int)std::min<long long>((long long)P.max_iters * pr.N, pr.rows);
  pr.cap = pr.rmax + pr.N + 1;
  const int N = pr.N;
  const size_t ts = pr.tsize;
  Buffers& m = pr.mem;
  const long long Nf = pr.Nf, Nc = pr.Nc, rows = pr.rows, cap = pr.cap;
  pr.cf = m.get_n<double>(Nf);
  pr.cc = m.get_n<double>(Nc);
  pr.c2f = m.get(ts * Nf);
  pr.c2c = m.get(ts * Nc);
  pr.c2c_d = m.get_n<double>(Nc);
  for (int a = 0; a < P.dim; ++a) {
    std::vector<double> t = P.interp == PW_INTERP_LINEAR  ? linear_interp_table(pr.gc.n[a], P.ratio)
                            : P.interp == PW_INTERP_CUBIC ? cubic_interp_table(pr.gc.n[a], P.ratio)
                                                          : trig_interp_table(pr.gc.n[a], P.ratio);
    pr.itab[a] = m.get_n<double>((long long)t.size());
    PW_HIP(hipMemcpy(pr.itab[a], t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice));
    std::vector<double> d = dft_table(pr.gc.n[a]);
    pr.dtab[a] = m.get_n<double>((long long)d.size());
    PW_HIP(hipMemcpy(pr.dtab[a], d.data(), sizeof(double) * d.size(), hipMemcpyHostToDevice));
  }
  pr.u = m.get(ts * Nf * (N + 1));
  pr.p = m.get(ts * Nf * (N + 1));
  pr.v = m.get(ts * Nf * N);
  pr.vp = m.get(ts * Nf * N);
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 4; ++f)
      pr.fw[s][f] = (f < 2 || pr.comp) ? m.get(ts * Nf * N) : nullptr;
  pr.sfa_u = m.get(ts * Nf);
  pr.sfa_p = m.get(ts * Nf);
  pr.sfb_u = m.get(ts * Nf);
  pr.sfb_p = m.get(ts * Nf);
  pr.Uc = m.get(ts * Nc * N);
  pr.Ucp = m.get(ts * Nc * N);
  pr.Rc = m.get(ts * Nc * (N + 1));
  pr.Rcp = m.get(ts * Nc * (N + 1));
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < 4; ++f)
      pr.cw[s][f] = (f < 2 || pr.comp) ? m.get(ts * Nc * (N + 1)) : nullptr;
  pr.du_T = m.get(ts * Nc * N);
  pr.dp_T = m.get(ts * Nc * N);
  const long long dstates = std::max<long long>(pr.rmax + 1, N);
  pr.Din = m.get_n<double>(2 * Nc * N);
  pr.Acol = m.get_n<double>(2 * Nc * N);
  for (int s = 0; s < 2; ++s) {
    pr.E[s] = m.get_n<double>(2 * Nc * cap);
    pr.Vp[s] = m.get_n<double>(2 * Nc * cap);
    pr.dw[s] = m.get_n<double>(2 * Nc * dstates);
    pr.Ub[s] = m.get_n<double>(rows * cap);
    pr.Vb[s] = m.get_n<double>(rows * cap);
  }
  pr.CE = m.get_n<double>(2 * Nc * (pr.rmax + 1));
  pr.CEb[0] = m.get_n<double>(2 * Nc * cap);
  pr.CEb[1] = m.get_n<double>(2 * Nc * cap);
  pr.cdc = m.get_n<double>(2 * Nc);
  pr.delta = m.get_n<double>(2 * Nc * N);
  pr.Fm = m.get_n<double>(rows * N);
  pr.Gm = m.get_n<double>(rows * N);
  pr.Fp = m.get_n<double>(rows * N);
  pr.Gp = m.get_n<double>(rows * N);
  pr.S = m.get_n<double>(cap);
  pr.UF = m.get_n<double>(cap * N);
  pr.VG = m.get_n<double>(cap * N);
  pr.UF2 = m.get_n<double>(cap * N);
  pr.VG2 = m.get_n<double>(cap * N);
  pr.RF = m.get_n<double>((long long)N * N);
  pr.RG = m.get_n<double>((long long)N * N);
  pr.Af = m.get_n<double>(cap * N);
  pr.Bg = m.get_n<double>(cap * N);
  pr.H = m.get_n<double>(cap * cap);
  pr.X = m.get_n<double>(cap * cap);
  pr.Y = m.get_n<double>(cap * cap);
  pr.sig = m.get_n<double>(std::max<long long>(cap, 512));  // also reduction partials
  pr.Hw = m.get_n<double>(2 * cap * cap + 3 * cap + 32);
  pr.Vw = m.get_n<double>(2 * cap * cap);
  pr.counters = m.get_n<int>(64);
  pr.rank_dev = m.get_n<int>(4);
  pr.M = m.get_n<double>((long long)(pr.rmax + 1) * (pr.rmax + 1));
  pr.Bn = m.get_n<double>((long long)(pr.rmax + 1) * N);
  pr.Tn = m.get_n<double>((long long)(pr.rmax + 1) * N);
  pr.rs.P0 = m.get_n<double>((long long)(pr.rmax + 1) * (pr.rmax + 1));
  pr.rs.P1 = m.get_n<double>((long long)(pr.rmax + 1) * (pr.rmax + 1));
  pr.rs.ta = m.get_n<double>((long long)(pr.rmax + 1) * N);
  pr.rs.tb = m.get_n<double>((long long)(pr.rmax + 1) * N);
  const int gcols = std::max(N, 1);
  pr.ctmp = m.get_n<double>(4LL * P.dim * Nc * gcols);
  // interpolation scratch: the partially interpolated fields of one pass
  // pair (2D: (n_x fine) x (n_y coarse) per field; 3D: also fine x, y by
  // coarse z), and at least two fine fields for staging inputs
  long long interp_need = 0;
  if (P.dim == 2) interp_need = (long long)pr.gc.n[1] * pr.gf.n[0] * N;
  if (P.dim == 3)
    interp_need = ((long long)pr.gc.n[2] * pr.gc.n[1] * pr.gf.n[0] +
                   (long long)pr.gc.n[2] * pr.gf.n[1] * pr.gf.n[0]) * N;
  pr.itmp = m.get_n<double>(std::max(interp_need, 2 * Nf) + 16);
  // split-K partials: bound over every A^T B shape of the path
  // (a <= cap, b <= max(cap, N))
  pr.gwork_elems = gemm_tn_work_bound((int)cap, (int)std::max<long long>(cap, N));
  pr.gwork = m.get_n<double>((long long)pr.gwork_elems);
  pr.red = m.get_n<double>(kEnergyPartials + 16);
  pr.vsum = m.get_n<double>(16);
  if (pr.order == 0) {
    pr.spec.dft = pr.dtab;
    pr.spec.cols = N;
    pr.spec.ctmp = m.get_n<double>(4LL * (P.dim + 1) * Nc * N);
    pr.spec.rtmp = m.get_n<double>((long long)P.dim * Nc * N);
    pr.spec.ures = m.get_n<double>(Nc * N);
  }
  pr.sponge = P.bc == PW_SPONGE;
  if (pr.sponge) {
    const long long nf = pr.gf.n[0] + pr.gf.n[1], nc = pr.gc.n[0] + pr.gc.n[1];
    pr.layF_t = m.get(ts * nf);
    pr.layC_t = m.get(ts * nc);
    pr.layF_d = m.get_n<double>(nf);
    pr.layC_d = m.get_n<double>(nc);
  }
  pr.res = m.get_n<double>((long long)kRes * (P.max_iters + 1));
  pr.chg = m.get_n<double>(4LL * N);
  if (P.keep_history) {
    pr.hist_u = m.get(ts * Nf * N * (size_t)(P.max_iters + 1));
    pr.hist_p = m.get(ts * Nf * N * (size_t)(P.max_iters + 1));
  }
  size_t tsq_st = 0, tsq_tau = 0;
  tsqr_work(rows, N, &tsq_st, &tsq_tau);
  pr.os.gram = m.get_n<double>(64LL * 64);
  pr.os.T = m.get_n<double>(64LL * 64);
  pr.os.info = m.get_n<double>(16);
  pr.os.gram_enough = !pr.f64;
  pr.os.R1 = m.get_n<double>((long long)N * N);
  pr.os.R2 = m.get_n<double>((long long)N * N);
  pr.os.Q1 = m.get_n<double>(rows * N);
  pr.os.hw = m.get_n<double>((long long)tsq_st + 16);
  pr.os.htau = m.get_n<double>((long long)tsq_tau + 16);
  if (N > 64) {
    pr.os.W = m.get_n<double>(rows * 64);
    pr.os.C = m.get_n<double>((long long)N * 64);
  }
  pr.os.work = pr.gwork;
  pr.os.work_elems = pr.gwork_elems;
  pr.gwork2 = m.get_n<double>((long long)pr.gwork_elems);
  pr.os2.gram = m.get_n<double>(64LL * 64);
  pr.os2.T = m.get_n<double>(64LL * 64);
  pr.os2.info = m.get_n<double>(16);
  pr.os2.gram_enough = !pr.f64;
  pr.os2.R1 = m.get_n<double>((long long)N * N);
  pr.os2.R2 = m.get_n<double>((long long)N * N);
  pr.os2.Q1 = m.get_n<double>(rows * N);
  pr.os2.hw = m.get_n<double>((long long)tsq_st + 16);
  pr.os2.htau = m.get_n<double>((long long)tsq_tau + 16);
  if (N > 64) {
    pr.os2.W = m.get_n<double>(rows * 64);
    pr.os2.C = m.get_n<double>((long long)N * 64);
  }
  pr.os2.work = pr.gwork2;
  pr.os2.work_elems = pr.gwork_elems;
  for (int i = 0; i < 4; ++i) PW_HIP(hipEventCreate(&pr.ev[i]));
  PW_HIP(hipEventCreateWithFlags(&pr.done_ev, hipEventDisableTiming));
  PW_HIP(hipEventCreateWithFlags(&pr.fork_ev, hipEventDisableTiming));
  PW_HIP(hipEventCreateWithFlags(&pr.join_ev, hipEventDisableTiming));
  PW_HIP(hipEventCreateWithFlags(&pr.pre_ev, hipEventDisableTiming));
}

// ---------------------------------------------------------------------------
// typed helpers
// ---------------------------------------------------------------------------
template <typename T>
StateSet<T> fine_work(Prob& pr, int s) {
  return StateSet<T>{tp<T>(pr.fw[s][0]), tp<T>(pr.fw[s][1]), tp<T>(pr.fw[s][2]),
                     tp<T>(pr.fw[s][3])};
}
template <typename T>
StateSet<T> coarse_work(Prob& pr, int s) {
  return StateSet<T>{tp<T>(pr.cw[s][0]), tp<T>(pr.cw[s][1]), tp<T>(pr.cw[s][2]),
                     tp<T>(pr.cw[s][3])};
}

// ---- absorbing layer and point source (PW_SPONGE, pw_set_source) --------
// The layer: sigma = sigma_max (d / w)^2, d the largest penetration of a
// node into the layer over the axes, so sigma is the largest of the
// per-axis sigma_a and the factor exp(-sigma h / 2) the smallest of the
// per-axis factors: one table per axis, min taken in the kernels.  The
// coarse grid takes sigma at its nodes (fine node ratio * J).
std::vector<double> layer_axis(int n_fine, double dx, int ratio, double w, double smax, double h) {
  const double L = n_fine * dx;
  const int nc = n_fine / ratio;
  std::vector<double> d((size_t)nc);
  for (int J = 0; J < nc; ++J) {
    const double x = (double)(ratio * J) * dx;
    const double pen = std::max(0.0, w - std::min(x, L - x));
    const double q = pen / w;
    const double sig = smax * (q * q);
    d[(size_t)J] = std::exp(-0.5 * sig * h);
  }
  return d;
}

template <typename T>
void upload_cast(void* dst, const std::vector<double>& v) {
  std::vector<T> c(v.size());
  for (size_t i = 0; i < v.size(); ++i) c[i] = (T)v[i];
  PW_HIP(hipMemcpy(dst, c.data(), sizeof(T) * c.size(), hipMemcpyHostToDevice));
}

// tables of the layer for the medium's c_max (host copy of c given)
void setup_layer(Prob& pr, double cmax_medium) {
  if (!pr.sponge) return;
  const pw_problem& P = pr.P;
  const double w = P.sponge_width;
  const double R = P.sponge_reflection > 0 ? P.sponge_reflection : 1e-3;
  const double cmax = P.sponge_cmax > 0 ? P.sponge_cmax : cmax_medium;
  pr.sponge_smax = 3.0 * cmax / (2.0 * w) * std::log(1.0 / R);
  for (int g = 0; g < 2; ++g) {
    const int ratio = g == 0 ? 1 : pr.ratio;
    const double h = g == 0 ? pr.hF : pr.hC;
    std::vector<double> t = layer_axis(pr.gf.n[0], pr.gf.dx, ratio, w, pr.sponge_smax, h);
    std::vector<double> ty = layer_axis(pr.gf.n[1], pr.gf.dx, ratio, w, pr.sponge_smax, h);
    t.insert(t.end(), ty.begin(), ty.end());
    double* dd = g == 0 ? pr.layF_d : pr.layC_d;
    void* dt = g == 0 ? pr.layF_t : pr.layC_t;
    PW_HIP(hipMemcpy(dd, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice));
    if (pr.f64) upload_cast<double>(dt, t);
    else upload_cast<float>(dt, t);
  }
}

// Force of a propagation of problem pr on the fine or coarse grid, in
// precision T (tables: the state dtype's, or double); with the source when
// `source`: state s propagates slice first_slice + s (per_state) or
// first_slice (all states)
template <typename T>
Force<T> make_force(const Prob& pr, bool fine, bool source, int first_slice, bool per_state,
                    bool state_tables) {
  Force<T> f;
  const Grid& g = fine ? pr.gf : pr.gc;
  if (pr.sponge) {
    const T* base = state_tables ? tp<T>(fine ? pr.layF_t : pr.layC_t)
                                 : reinterpret_cast<const T*>(fine ? pr.layF_d : pr.layC_d);
    f.dmp_x = base;
    f.dmp_y = base + g.n[0];
  }
  if (source && pr.have_src) {
    const int* node = fine ? pr.srcF : pr.srcC;
    const int m = fine ? pr.mF : pr.mC;
    f.sx = node[0];
    f.sy = node[1];
    f.amp = std::pow(g.dx, -(double)g.dim);
    f.src_tab = (const double*)(fine ? pr.srcF_tab.p : pr.srcC_tab.p) +
                (long long)(first_slice - 1) * (m + 1);
    f.src_stride = per_state ? m + 1 : 0;
  }
  return f;
}

bool forced(const Prob& pr) { return pr.sponge || pr.have_src; }

// F of n states; state s propagates slice first_slice + s (from
// t = (first_slice + s - 1) T / N; only the source depends on it)
template <typename T>
void prop_fine(Prob& pr, const T* u, const T* p, T* uo, T* po, int n, hipStream_t st,
               int first_slice = 1) {
  if (n > pr.N) fail(PW_EINVAL, "too many fine states for one batched propagation");
  Force<T> fo;
  if (forced(pr)) fo = make_force<T>(pr, true, true, first_slice, true, true);
  propagate<T>(pr.gf, tp<T>(pr.c2f), u, p, uo, po, pr.Nf, n, pr.mF, (T)pr.hF, pr.comp,
               fine_work<T>(pr, 0), fine_work<T>(pr, 1), st, true, forced(pr) ? &fo : nullptr);
}

// C of n states (slices first_slice, first_slice + 1, ... as prop_fine)
template <typename T>
void prop_coarse(Prob& pr, const T* u, const T* p, T* uo, T* po, int n, hipStream_t st,
                 int first_slice = 1) {
  if (n > pr.N + 1) fail(PW_EINVAL, "too many coarse states for one batched propagation");
  Force<T> fo;
  if (forced(pr)) fo = make_force<T>(pr, false, true, first_slice, true, true);
  propagate<T>(pr.gc, tp<T>(pr.c2c), u, p, uo, po, pr.Nc, n, pr.mC, (T)pr.hC, pr.comp,
               coarse_work<T>(pr, 0), coarse_work<T>(pr, 1), st, false,
               forced(pr) ? &fo : nullptr);
}

// FP64 coarse propagation of state columns [u (Nc) ; p (Nc)] (linear C: the
// layer, never the source -- the columns are differences of states or
// corrector directions)
void prop_coarse_cols(Prob& pr, const double* in, double* out, int ncols, hipStream_t st) {
  const long long Nc = pr.Nc;
  if (ncols > std::max(pr.rmax + 1, pr.N)) fail(PW_EINVAL, "too many coarse columns");
  StateSet<double> a{pr.dw[0], pr.dw[0] + Nc, nullptr, nullptr};
  StateSet<double> b{pr.dw[1], pr.dw[1] + Nc, nullptr, nullptr};
  Force<double> fo;
  if (pr.sponge) fo = make_force<double>(pr, false, false, 1, false, false);
  propagate<double>(pr.gc, pr.c2c_d, in, in + Nc, out, out + Nc, 2 * Nc, ncols, pr.mC, pr.hC,
                    false, a, b, st, false, pr.sponge ? &fo : nullptr);
}

// ---------------------------------------------------------------------------
// Algorithm 1 on the device (see linalg.hip for the pieces)
// ---------------------------------------------------------------------------
void sync_rank(Prob& pr, hipStream_t st, int* out) {
  int h = 0;
  PW_HIP(hipMemcpyAsync(&h, pr.rank_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  PW_HIP(hipStreamSynchronize(st));
  *out = h;
}

__global__ void k_add_inplace(double* a, const double* b, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] += b[t];
}

void add_inplace(double* a, const double* b, long long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_add_inplace, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
  PW_LAUNCH_CHECK();
}

// remove the components along basis B (rows x r) from X (rows x n) twice,
// accumulating the coefficients in C (r x n): X <- X - B (B^T X)
void project_out(Prob& pr, long long rows, int r, int n, const double* B, double* X, double* C,
                 double* C2, double* work, hipStream_t st) {
  gemm_tn(rows, r, n, 1.0, B, rows, X, rows, 0.0, C, r, work, pr.gwork_elems, st);
  gemm_nn(rows, n, r, -1.0, B, rows, C, r, 1.0, X, rows, st);
  gemm_tn(rows, r, n, 1.0, B, rows, X, rows, 0.0, C2, r, work, pr.gwork_elems, st);
  gemm_nn(rows, n, r, -1.0, B, rows, C2, r, 1.0, X, rows, st);
  // C += C2 (both r x n, contiguous)
  add_inplace(C, C2, (long long)r * n, st);
}

// dst[:, j] = src[:, idx[j]] for j < ncols (rows x ncols, column-major)
__global__ void k_gather_cols(const double* src, long long rows, const int* idx, int ncols,
                              double* dst) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * ncols) return;
  const long long j = t / rows, i = t - j * rows;
  dst[t] = src[(long long)idx[j] * rows + i];
}

void gather_cols(const double* src, long long rows, const int* idx, int ncols, double* dst,
                 hipStream_t st) {
  const long long n = rows * ncols;
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src,
                     rows, idx, ncols, dst);
  PW_LAUNCH_CHECK();
}

// randomised range finder of Halko, Martinsson and Tropp on A (rows x nd):
// Q (l columns at q_out, ld rows) an orthonormal basis of the range of
// (A A^T)^power A Om, each power step re-orthonormalised, and R = Q^T A
// (l x nd, ld l, at R_out)
void range_basis(Prob& pr, const double* A, int nd, const double* Om, int l, double* Y,
                 double* Z, double* q_out, double* R_out, OrthScratch& os, double* work,
                 hipStream_t st) {
  const long long rows = pr.rows;
  gemm_nn(rows, l, nd, 1.0, A, rows, Om, nd, 0.0, Y, rows, st);
  for (int it = 0; it < pr.sk_power; ++it) {
    orth_begin(rows, l, Y, rows, os, st);
    const bool c = orth_choose(rows, l, os, st);
    orth_finish(rows, l, Y, rows, q_out, rows, R_out, os, c, st);
    gemm_tn(rows, nd, l, 1.0, A, rows, q_out, rows, 0.0, Z, nd, work, pr.gwork_elems, st);
    gemm_nn(rows, l, nd, 1.0, A, rows, Z, nd, 0.0, Y, rows, st);
  }
  orth_begin(rows, l, Y, rows, os, st);
  const bool c = orth_choose(rows, l, os, st);
  orth_finish(rows, l, Y, rows, q_out, rows, R_out, os, c, st);
  gemm_tn(rows, l, nd, 1.0, q_out, rows, A, rows, 0.0, R_out, l, work, pr.gwork_elems, st);
}

// Algorithm 1 on F, G (rows x ncols); with cols (device, ncols entries) it
// runs on the columns F[:, cols], G[:, cols] instead (random subsampling of
// the data matrices)
// Algorithm 1 in two halves around the SVD of its core matrix: the first
// forms H (n x n, pr.H) and returns n and the number of new basis columns;
// the second takes the SVD (pr.X, pr.Y, pr.sig, pr.rank_dev) and updates
// the corrector.  update_svd_dev runs both with the SVD in between; the
// batch runs the SVDs of all its problems together (svd_jacobi_multi).
struct SvdPending {
  int n = 0, nnew = 0;
};

SvdPending update_svd_begin(Prob& pr, const double* F, const double* G, int ncols,
                            hipStream_t st, const int* cols = nullptr, double* norms = nullptr,
                            const double* sketch = nullptr) {
  const long long rows = pr.rows;
  const int r = pr.r;
  const int cur = pr.cur, nxt = 1 - pr.cur;
  // new basis columns: the data columns, or the sketch width
  const int nnew = sketch ? pr.sk_l : ncols;
  if (r + ncols + 1 > pr.cap) fail(PW_EINVAL, "corrector capacity exceeded (raise max_iters)");
  double* U = pr.Ub[cur];
  double* V = pr.Vb[cur];
  int n;
  // the G branch (projection and orthonormalisation of the G-side data)
  // runs on the side stream between the fork and the join
  PW_HIP(hipEventRecord(pr.fork_ev, st));
  PW_HIP(hipStreamWaitEvent(pr.side, pr.fork_ev, 0));
  if (cols) {
    gather_cols(F, rows, cols, ncols, pr.Fp, st);
    gather_cols(G, rows, cols, ncols, pr.Gp, pr.side);
    F = pr.Fp;
    G = pr.Gp;
  }
  if (norms) {
    // ||F_in||^2 and ||G_in||^2 (own partial buffers on the two streams)
    frob_norm2(F, rows, ncols, rows, pr.red, norms, st);
    frob_norm2(G, rows, ncols, rows, pr.red + 1024, norms + 1, pr.side);
  }
  if (r == 0 && sketch) {
    range_basis(pr, F, ncols, sketch, nnew, (double*)pr.skYf.p, (double*)pr.skZf.p, U, pr.RF,
                pr.os, pr.gwork, st);
    range_basis(pr, G, ncols, sketch, nnew, (double*)pr.skYg.p, (double*)pr.skZg.p, V, pr.RG,
                pr.os2, pr.gwork2, pr.side);
    PW_HIP(hipEventRecord(pr.join_ev, pr.side));
    PW_HIP(hipStreamWaitEvent(st, pr.join_ev, 0));
    gemm_small(nnew, nnew, ncols, 1.0, pr.RF, nnew, false, pr.RG, nnew, true, 0.0, pr.H, nnew,
               st);
    n = nnew;
  } else if (r == 0) {
    orth_begin(rows, ncols, F, rows, pr.os, st);
    orth_begin(rows, ncols, G, rows, pr.os2, pr.side);
    const bool cf = orth_choose(rows, ncols, pr.os, st);
    const bool cg = orth_choose(rows, ncols, pr.os2, pr.side);
    orth_finish(rows, ncols, F, rows, U, rows, pr.RF, pr.os, cf, st);
    orth_finish(rows, ncols, G, rows, V, rows, pr.RG, pr.os2, cg, pr.side);
    PW_HIP(hipEventRecord(pr.join_ev, pr.side));
    PW_HIP(hipStreamWaitEvent(st, pr.join_ev, 0));
    gemm_small(ncols, ncols, ncols, 1.0, pr.RF, ncols, false, pr.RG, ncols, true, 0.0, pr.H,
               ncols, st);
    n = ncols;
  } else {
    if (F != pr.Fp)
      PW_HIP(hipMemcpyAsync(pr.Fp, F, sizeof(double) * rows * ncols, hipMemcpyDeviceToDevice,
                            st));
    if (G != pr.Gp)
      PW_HIP(hipMemcpyAsync(pr.Gp, G, sizeof(double) * rows * ncols, hipMemcpyDeviceToDevice,
                            pr.side));
    project_out(pr, rows, r, ncols, U, pr.Fp, pr.UF, pr.UF2, pr.gwork, st);
    project_out(pr, rows, r, ncols, V, pr.Gp, pr.VG, pr.VG2, pr.gwork2, pr.side);
    if (sketch) {
      range_basis(pr, pr.Fp, ncols, sketch, nnew, (double*)pr.skYf.p, (double*)pr.skZf.p,
                  U + rows * r, pr.RF, pr.os, pr.gwork, st);
      range_basis(pr, pr.Gp, ncols, sketch, nnew, (double*)pr.skYg.p, (double*)pr.skZg.p,
                  V + rows * r, pr.RG, pr.os2, pr.gwork2, pr.side);
    } else {
      orth_begin(rows, ncols, pr.Fp, rows, pr.os, st);
      orth_begin(rows, ncols, pr.Gp, rows, pr.os2, pr.side);
      const bool cf = orth_choose(rows, ncols, pr.os, st);
      const bool cg = orth_choose(rows, ncols, pr.os2, pr.side);
      orth_finish(rows, ncols, pr.Fp, rows, U + rows * r, rows, pr.RF, pr.os, cf, st);
      orth_finish(rows, ncols, pr.Gp, rows, V + rows * r, rows, pr.RG, pr.os2, cg, pr.side);
    }
    PW_HIP(hipEventRecord(pr.join_ev, pr.side));
    PW_HIP(hipStreamWaitEvent(st, pr.join_ev, 0));
    n = r + nnew;
    // Af = [UF; RF], Bg = [VG; RG] ((r + nnew) x ncols)
    copy_block(r, ncols, pr.UF, r, pr.Af, n, st);
    copy_block(nnew, ncols, pr.RF, nnew, pr.Af + r, n, st);
    copy_block(r, ncols, pr.VG, r, pr.Bg, n, st);
    copy_block(nnew, ncols, pr.RG, nnew, pr.Bg + r, n, st);
    gemm_small(n, n, ncols, 1.0, pr.Af, n, false, pr.Bg, n, true, 0.0, pr.H, n, st);
    add_diag(n, r, pr.S, pr.H, n, st);
  }
  return SvdPending{n, nnew};
}

SvdJob svd_job(Prob& pr, int n) {
  return SvdJob{n,        pr.H,  pr.X,  pr.Y,  pr.sig,     pr.tol,
                pr.rank_dev, pr.Hw, pr.Vw, pr.counters};
}

void update_svd_end(Prob& pr, const SvdPending& sp, hipStream_t st) {
  const long long rows = pr.rows;
  const int r = pr.r, n = sp.n, nnew = sp.nnew;
  const int cur = pr.cur, nxt = 1 - pr.cur;
  double* U = pr.Ub[cur];
  double* V = pr.Vb[cur];
  int rn = 0;
  sync_rank(pr, st, &rn);
  rn = std::min(rn, pr.rmax);
  // new columns of E and P for the sweep: Lambda^dag of Q_F, Lambda^T of Q_G
  const long long Nc = pr.Nc;
  lambda_dag_cols(pr.gc, pr.dtab, U + rows * r, rows, pr.cc, nullptr, pr.E[cur] + 2 * Nc * r,
                  2 * Nc, nnew, pr.ctmp, st);
  lambda_adjoint_cols(pr.gc, V + rows * r, rows, pr.cc, pr.order, pr.Vp[cur] + 2 * Nc * r, 2 * Nc,
                      nnew, st, &pr.spec);
  // C E: only the new directions go through C; the rest is in CEb[cur]
  const bool carry = pr.ce_ok || r == 0;
  if (carry)
    prop_coarse_cols(pr, pr.E[cur] + 2 * Nc * r, pr.CEb[cur] + 2 * Nc * r, nnew, st);
  // rotate: [U Q_F] X(:, 1:rn) etc.
  gemm_nn(rows, rn, n, 1.0, U, rows, pr.X, n, 0.0, pr.Ub[nxt], rows, st);
  gemm_nn(rows, rn, n, 1.0, V, rows, pr.Y, n, 0.0, pr.Vb[nxt], rows, st);
  gemm_nn(2 * Nc, rn, n, 1.0, pr.E[cur], 2 * Nc, pr.X, n, 0.0, pr.E[nxt], 2 * Nc, st);
  gemm_nn(2 * Nc, rn, n, 1.0, pr.Vp[cur], 2 * Nc, pr.Y, n, 0.0, pr.Vp[nxt], 2 * Nc, st);
  set_dc_column(pr.E[nxt], 2 * Nc, rn, Nc, 1.0 / (double)Nc, st);
  set_dc_column(pr.Vp[nxt], 2 * Nc, rn, Nc, 1.0, st);
  if (carry) {
    gemm_nn(2 * Nc, rn, n, 1.0, pr.CEb[cur], 2 * Nc, pr.X, n, 0.0, pr.CEb[nxt], 2 * Nc, st);
    if (!pr.cdc_ok) {
      prop_coarse_cols(pr, pr.E[nxt] + 2 * Nc * rn, pr.cdc, 1, st);
      pr.cdc_ok = true;
    }
    PW_HIP(hipMemcpyAsync(pr.CEb[nxt] + 2 * Nc * rn, pr.cdc, sizeof(double) * 2 * Nc,
                          hipMemcpyDeviceToDevice, st));
  }
  pr.ce_ok = carry;
  if (rn > 0)
    PW_HIP(hipMemcpyAsync(pr.S, pr.sig, sizeof(double) * rn, hipMemcpyDeviceToDevice, st));
  pr.cur = nxt;
  pr.r = rn;
}

void update_svd_dev(Prob& pr, const double* F, const double* G, int ncols, hipStream_t st,
                    const int* cols = nullptr, double* norms = nullptr,
                    const double* sketch = nullptr) {
  const SvdPending sp = update_svd_begin(pr, F, G, ncols, st, cols, norms, sketch);
  const SvdJob q = svd_job(pr, sp.n);
  svd_jacobi(q.n, q.H, q.X, q.Y, q.sig, q.tol, q.rank_dev, q.Hw, q.Vw, q.counters, st);
  update_svd_end(pr, sp, st);
}

void check_sampling(const Prob& pr, int K) {
  if (pr.samp_n > 0 && K > pr.samp_iters)
    fail(PW_EINVAL, "the sampled-column table covers fewer iterations than K");
  if (pr.sk_l > 0 && K > pr.sk_iters)
    fail(PW_EINVAL, "the sketch test matrices cover fewer iterations than K");
}

void reset_corrector(Prob& pr) {
  pr.r = 0;
  pr.cur = 0;
  pr.ce_ok = false;
  pr.ranks.clear();
}

// ---------------------------------------------------------------------------
// Algorithm 3
// ---------------------------------------------------------------------------
__global__ void k_split_cast_f(const double* delta, long long ld, long long nc, int ncols,
                               float* du, float* dp) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * ncols) return;
  const long long col = t / nc, J = t - col * nc;
  du[t] = (float)delta[col * ld + J];
  dp[t] = (float)delta[col * ld + nc + J];
}
__global__ void k_split_cast_d(const double* delta, long long ld, long long nc, int ncols,
                               double* du, double* dp) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * ncols) return;
  const long long col = t / nc, J = t - col * nc;
  du[t] = delta[col * ld + J];
  dp[t] = delta[col * ld + nc + J];
}

template <typename T>
void split_cast(const double* delta, long long ld, long long nc, int ncols, T* du, T* dp,
                hipStream_t st) {
  const long long n = nc * ncols;
  if (n == 0) return;
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL(k_split_cast_f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, delta,
                       ld, nc, ncols, du, dp);
  else
    hipLaunchKernelGGL(k_split_cast_d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, delta,
                       ld, nc, ncols, du, dp);
  PW_LAUNCH_CHECK();
}

// ---- phases of one iteration ---------------------------------------------
// initialisation: W_0 = R u0, W_n = C W_{n-1}; u^1_n = I W_n
template <typename T>
void init_phase(Prob& pr, hipStream_t st) {
  const int N = pr.N;
  const long long Nf = pr.Nf, Nc = pr.Nc;
  T* u = tp<T>(pr.u);
  T* p = tp<T>(pr.p);
  T* Uc = tp<T>(pr.Uc);
  T* Ucp = tp<T>(pr.Ucp);
  T* Rc = tp<T>(pr.Rc);
  T* Rcp = tp<T>(pr.Rcp);
  reset_corrector(pr);
  for (int i = 0; i < 4; ++i) pr.ms[i] = 0.0;
  pr.k_done = 0;
  pr.change.clear();
  restrict_fields<T>(pr.gf, pr.ratio, pr.gc, u, Nf, Rc, Nc, 1, st);
  restrict_fields<T>(pr.gf, pr.ratio, pr.gc, p, Nf, Rcp, Nc, 1, st);
  for (int n = 1; n <= N; ++n) {
    const T* su = n == 1 ? Rc : Uc + (n - 2) * Nc;
    const T* sp = n == 1 ? Rcp : Ucp + (n - 2) * Nc;
    prop_coarse<T>(pr, su, sp, Uc + (n - 1) * Nc, Ucp + (n - 1) * Nc, 1, st, n);
  }
  interp_add<T>(pr.gf, pr.gc, pr.ratio, pr.itab, Uc, Nc, (const T*)nullptr, u + Nf, Nf, N,
                pr.itmp, st);
  interp_add<T>(pr.gf, pr.gc, pr.ratio, pr.itab, Ucp, Nc, (const T*)nullptr, p + Nf, Nf, N,
                pr.itmp, st);
}

// restriction of the slice-start states for U_n = C R u^k_{n-1}
template <typename T>
void restrict_phase(Prob& pr, hipStream_t st) {
  restrict_fields<T>(pr.gf, pr.ratio, pr.gc, tp<T>(pr.u), pr.Nf, tp<T>(pr.Rc), pr.Nc, pr.N, st);
  restrict_fields<T>(pr.gf, pr.ratio, pr.gc, tp<T>(pr.p), pr.Nf, tp<T>(pr.Rcp), pr.Nc, pr.N, st);
}

// 2. data matrices, Algorithm 1 and the residual rho_k, in two halves
// around the SVD of Algorithm 1's core matrix (see update_svd_begin)
template <typename T>
SvdPending corrector_begin(Prob& pr, int k, hipStream_t st) {
  const int N = pr.N;
  const long long Nf = pr.Nf, Nc = pr.Nc, rows = pr.rows;
  energy_columns<T>(pr.gf, pr.ratio, pr.gc, tp<T>(pr.v), tp<T>(pr.vp), Nf, pr.cc, pr.order,
                    pr.Fm, rows, N, st, &pr.spec);
  energy_columns<T>(pr.gc, 1, pr.gc, tp<T>(pr.Uc), tp<T>(pr.Ucp), Nc, pr.cc, pr.order, pr.Gm,
                    rows, N, st, &pr.spec);
  double* rk = pr.res + (long long)kRes * (k - 1);
  if (pr.samp_n > 0) {
    if (k > pr.samp_iters) fail(PW_EINVAL, "no sampled columns for this iteration");
    return update_svd_begin(pr, pr.Fm, pr.Gm, pr.samp_n, st,
                            (const int*)pr.samp.p + (long long)(k - 1) * pr.samp_n, rk + 2);
  }
  if (pr.sk_l > 0) {
    if (k > pr.sk_iters) fail(PW_EINVAL, "no sketch test matrix for this iteration");
    return update_svd_begin(pr, pr.Fm, pr.Gm, N, st, nullptr, rk + 2,
                            (const double*)pr.sk.p + (long long)(k - 1) * N * pr.sk_l);
  }
  return update_svd_begin(pr, pr.Fm, pr.Gm, N, st, nullptr, rk + 2);
}

template <typename T>
void corrector_end(Prob& pr, int k, const SvdPending& sp, hipStream_t st) {
  const int N = pr.N;
  const long long rows = pr.rows;
  double* rk = pr.res + (long long)kRes * (k - 1);
  update_svd_end(pr, sp, st);
  pr.ranks.push_back(pr.r);
  // rho_k: || F - U (V^T G) ||_F / ||F||_F
  const int r = pr.r;
  gemm_tn(rows, r, N, 1.0, pr.Vb[pr.cur], rows, pr.Gm, rows, 0.0, pr.UF, std::max(r, 1),
          pr.gwork, pr.gwork_elems, st);
  PW_HIP(hipMemcpyAsync(pr.Fp, pr.Fm, sizeof(double) * rows * N, hipMemcpyDeviceToDevice, st));
  gemm_nn(rows, N, r, -1.0, pr.Ub[pr.cur], rows, pr.UF, std::max(r, 1), 1.0, pr.Fp, rows, st);
  frob_norm2(pr.Fp, rows, N, rows, pr.red, rk, st);
  frob_norm2(pr.Fm, rows, N, rows, pr.red, rk + 1, st);
  vec_sum(pr.S, r, rk + 4, st);
}

template <typename T>
void corrector_phase(Prob& pr, int k, hipStream_t st) {
  const SvdPending sp = corrector_begin<T>(pr, k, st);
  const SvdJob q = svd_job(pr, sp.n);
  svd_jacobi(q.n, q.H, q.X, q.Y, q.sig, q.tol, q.rank_dev, q.Hw, q.Vw, q.counters, st);
  corrector_end<T>(pr, k, sp, st);
}

// a_n = R v_{n-1} - R u^k_{n-1} (double coarse columns), v_0 = u0 -> column 0
// is zero
template <typename T>
void sweep_inputs(Prob& pr, hipStream_t st) {
  const long long Nf = pr.Nf, Nc = pr.Nc;
  fill(pr.Din, 2 * Nc, 0.0, st);
  if (pr.N > 1)
    restrict_diff<T>(pr.gf, pr.ratio, pr.gc, tp<T>(pr.v), tp<T>(pr.vp), tp<T>(pr.u) + Nf,
                     tp<T>(pr.p) + Nf, Nf, pr.Din + 2 * Nc, 2 * Nc, pr.N - 1, st);
}

// delta_n = E t_n with t_n = P^T Acol_n + (P^T C E) t_{n-1}, t_0 = 0: the
// serial sweep in corrector coordinates (Acol already formed).  With
// carry, E is the current corrector's E[cur] and C E comes from CEb[cur]
// (formed here when it is not carried yet); otherwise E (a taped copy) is
// propagated in full.
void corrector_chain(Prob& pr, const double* E, const double* P, int dim, hipStream_t st,
                     bool carry = false) {
  const int N = pr.N;
  const long long Nc = pr.Nc;
  double* CE = pr.CE;
  if (carry) {
    CE = pr.CEb[pr.cur];
    if (!pr.ce_ok) prop_coarse_cols(pr, E, CE, dim, st);
    pr.ce_ok = true;
  } else {
    prop_coarse_cols(pr, E, CE, dim, st);
  }
  gemm_tn(2 * Nc, dim, dim, 1.0, P, 2 * Nc, CE, 2 * Nc, 0.0, pr.M, dim, pr.gwork,
          pr.gwork_elems, st);
  gemm_tn(2 * Nc, dim, N, 1.0, P, 2 * Nc, pr.Acol, 2 * Nc, 0.0, pr.Bn, dim, pr.gwork,
          pr.gwork_elems, st);
  if (dim > pr.rmax + 1) fail(PW_EINVAL, "corrector rank exceeds its capacity");
  recurrence(dim, N, pr.M, pr.Bn, pr.Tn, pr.rs, st);
  gemm_nn(2 * Nc, N, dim, 1.0, E, 2 * Nc, pr.Tn, dim, 0.0, pr.delta, 2 * Nc, st);
}

// u^{k+1}_n = v_n + I(delta_n) (add_v) or I(delta_n), n = 1..N
template <typename T>
void sweep_update(Prob& pr, bool add_v, hipStream_t st) {
  const int N = pr.N;
  const long long Nf = pr.Nf, Nc = pr.Nc;
  const T* v = add_v ? tp<T>(pr.v) : nullptr;
  const T* vp = add_v ? tp<T>(pr.vp) : nullptr;
  split_cast<T>(pr.delta, 2 * Nc, Nc, N, tp<T>(pr.du_T), tp<T>(pr.dp_T), st);
  interp_add<T>(pr.gf, pr.gc, pr.ratio, pr.itab, tp<T>(pr.du_T), Nc, v, tp<T>(pr.u) + Nf, Nf, N,
                pr.itmp, st);
  interp_add<T>(pr.gf, pr.gc, pr.ratio, pr.itab, tp<T>(pr.dp_T), Nc, vp, tp<T>(pr.p) + Nf, Nf, N,
                pr.itmp, st);
}

// 3.-4. corrected sweep in corrector coordinates and the update:
// delta_n = Lambda^dag Omega Lambda C (a_n + delta_{n-1}) (R I = 1)
template <typename T>
void sweep_core(Prob& pr, const double* E, const double* P, int dim, hipStream_t st,
                bool carry) {
  sweep_inputs<T>(pr, st);
  prop_coarse_cols(pr, pr.Din, pr.Acol, pr.N, st);
  corrector_chain(pr, E, P, dim, st, carry);
  sweep_update<T>(pr, true, st);
}

// ---- comparator iterations of Sec. 6 -----------------------------------
__global__ void k_add_cols(const double* a, const double* b, double* out, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = b ? a[t] + b[t] : a[t];
}
__global__ void k_sub_cols(const double* a, const double* b, double* out, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = a[t] - b[t];
}
// out[0] = sum of x[0..n) (one workgroup, fixed summation order)
__global__ __launch_bounds__(256) void k_col_sum(const double* x, long long n, double* out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) acc += x[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

void add_cols(const double* a, const double* b, double* out, long long n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, out,
                     n);
  PW_LAUNCH_CHECK();
}

// rho_k = ||F^k - G^k|| / ||F^k|| for the iterations without a fitted
// corrector (Omega = I, plain); the rank reported is the row count
template <typename T>
void residual_identity_phase(Prob& pr, int k, hipStream_t st) {
  const int N = pr.N;
  const long long Nf = pr.Nf, Nc = pr.Nc, rows = pr.rows;
  energy_columns<T>(pr.gf, pr.ratio, pr.gc, tp<T>(pr.v), tp<T>(pr.vp), Nf, pr.cc, pr.order,
                    pr.Fm, rows, N, st, &pr.spec);
  energy_columns<T>(pr.gc, 1, pr.gc, tp<T>(pr.Uc), tp<T>(pr.Ucp), Nc, pr.cc, pr.order, pr.Gm,
                    rows, N, st, &pr.spec);
  pr.ranks.push_back((int)rows);
  const long long n = rows * N;
  hipLaunchKernelGGL(k_sub_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const double*)pr.Fm, (const double*)pr.Gm, pr.Fp, n);
  PW_LAUNCH_CHECK();
  double* rk = pr.res + (long long)kRes * (k - 1);
  frob_norm2(pr.Fp, rows, N, rows, pr.red, rk, st);
  frob_norm2(pr.Fm, rows, N, rows, pr.red, rk + 1, st);
  fill(rk + 2, 3, 0.0, st);
}

// Omega = I (project) or plain parareal: the serial chain
// delta_n = Pi C (a_n + delta_{n-1}), delta_1 = 0, with Pi = Lambda^dag
// Lambda (Omega = I) or the identity (plain); then u^{k+1}_n = v_n + I delta_n
template <typename T>
void sweep_serial_chain(Prob& pr, bool project, hipStream_t st) {
  const int N = pr.N;
  const long long Nc = pr.Nc, C2 = 2 * Nc, rows = pr.rows;
  sweep_inputs<T>(pr, st);
  for (int n = 1; n <= N; ++n) {
    double* x = pr.Acol + C2 * (n - 1);
    double* dn = pr.delta + C2 * (n - 1);
    add_cols(pr.Din + C2 * (n - 1), n > 1 ? pr.delta + C2 * (n - 2) : nullptr, x, C2, st);
    if (!project) {
      prop_coarse_cols(pr, x, dn, 1, st);
      continue;
    }
    prop_coarse_cols(pr, x, pr.CE, 1, st);
    energy_columns<double>(pr.gc, 1, pr.gc, pr.CE, pr.CE + Nc, C2, pr.cc, pr.order, pr.Fp, rows,
                           1, st, &pr.spec);
    hipLaunchKernelGGL(k_col_sum, dim3(1), dim3(256), 0, st, (const double*)pr.CE, Nc, pr.vsum);
    PW_LAUNCH_CHECK();
    lambda_dag_cols(pr.gc, pr.dtab, pr.Fp, rows, pr.cc, pr.vsum, dn, C2, 1, pr.ctmp, st);
  }
  sweep_update<T>(pr, true, st);
}

// Sec. 6.3: u^{k+1}_n = I Lambda^dag Omega Lambda C R u^{k+1}_{n-1}; with
// u^{k+1}_{n-1} = I delta_{n-1} (n >= 2) and R I = 1 this is the chain
// delta_n = Lambda^dag Omega Lambda C delta_{n-1}, delta_0 = R u0, i.e. the
// corrector-coordinate recurrence with Acol = [C R u0, 0, ..., 0]
template <typename T>
void sweep_no_correction(Prob& pr, hipStream_t st) {
  const long long Nc = pr.Nc, C2 = 2 * Nc;
  cast_to_double<T>(tp<T>(pr.Rc), pr.Din, Nc, st);
  cast_to_double<T>(tp<T>(pr.Rcp), pr.Din + Nc, Nc, st);
  if (pr.N > 1) fill(pr.Acol + C2, C2 * (pr.N - 1), 0.0, st);
  prop_coarse_cols(pr, pr.Din, pr.Acol, 1, st);
  corrector_chain(pr, pr.E[pr.cur], pr.Vp[pr.cur], pr.r + 1, st, true);
  sweep_update<T>(pr, false, st);
}

template <typename T>
void sweep_phase(Prob& pr, hipStream_t st) {
  switch (pr.variant) {
    case PW_VARIANT_OMEGA_ONE: sweep_serial_chain<T>(pr, true, st); break;
    case PW_VARIANT_PLAIN: sweep_serial_chain<T>(pr, false, st); break;
    case PW_VARIANT_NO_CORRECTION: sweep_no_correction<T>(pr, st); break;
    default: sweep_core<T>(pr, pr.E[pr.cur], pr.Vp[pr.cur], pr.r + 1, st, true);
  }
}

// u^k_n, n = 1..N, of the current iterate into history level k - 1
void store_history(Prob& pr, int k, hipStream_t st) {
  if (!pr.hist_u) return;
  const size_t fb = pr.tsize * pr.Nf;
  const size_t bytes = fb * pr.N;
  PW_HIP(hipMemcpyAsync((char*)pr.hist_u + bytes * (k - 1), (const char*)pr.u + fb, bytes,
                        hipMemcpyDeviceToDevice, st));
  PW_HIP(hipMemcpyAsync((char*)pr.hist_p + bytes * (k - 1), (const char*)pr.p + fb, bytes,
                        hipMemcpyDeviceToDevice, st));
}

// the previous iterate u^k_n, n = 1..N, for the stopping rule (the history
// level when kept, else a copy taken before the iteration)
const void* prev_iterate(Prob& pr, int k, bool p_field) {
  const size_t bytes = pr.tsize * pr.Nf * pr.N;
  if (pr.hist_u) return (const char*)(p_field ? pr.hist_p : pr.hist_u) + bytes * (k - 1);
  return (const char*)pr.prev.p + (p_field ? bytes : 0);
}

// stopping measure of iteration k (u^{k+1} current, u^k previous):
// max_n sqrt(E(u^{k+1}_n - u^k_n) / E(u^{k+1}_n)) on the fine grid, FP64
// reductions on the device, one read-back
template <typename T>
double change_measure(Prob& pr, int k, hipStream_t st) {
  const int N = pr.N;
  const long long Nf = pr.Nf;
  const T* ua = tp<T>((void*)prev_iterate(pr, k, false));
  const T* pa = tp<T>((void*)prev_iterate(pr, k, true));
  const T* ub = tp<T>(pr.u) + Nf;
  const T* pb = tp<T>(pr.p) + Nf;
  const int order = pr.order ? pr.order : 4;
  for (int n = 0; n < N; ++n)
    energy_pair<T>(pr.gf, ua + n * Nf, pa + n * Nf, ub + n * Nf, pb + n * Nf, pr.cf, order,
                   pr.red, pr.chg + 4 * n, st);
  std::vector<double> h(4 * (size_t)N);
  PW_HIP(hipMemcpyAsync(h.data(), pr.chg, sizeof(double) * 4 * N, hipMemcpyDeviceToHost, st));
  PW_HIP(hipStreamSynchronize(st));
  double worst = 0.0;
  for (int n = 0; n < N; ++n) {
    const double e = h[4 * n], e0 = h[4 * n + 1];
    const double c = e0 > 0 ? std::sqrt(e / e0) : std::sqrt(e);
    if (!(c <= worst)) worst = c;  // NaN propagates
  }
  return worst;
}

// phase events of one iteration (4 per iteration, created on first use);
// read once at the end of a run
hipEvent_t* phase_events(Prob& pr, int k) {
  const size_t need = 4 * (size_t)k;
  while (pr.pev.size() < need) {
    hipEvent_t e;
    PW_HIP(hipEventCreate(&e));
    pr.pev.push_back(e);
  }
  return pr.pev.data() + 4 * (size_t)(k - 1);
}

void accumulate_phase_times(Prob& pr, int k_first, int k_last) {
  if (k_last < k_first) return;
  PW_HIP(hipEventSynchronize(phase_events(pr, k_last)[3]));
  for (int k = k_first; k <= k_last; ++k) {
    hipEvent_t* ev = phase_events(pr, k);
    float a = 0, b = 0, c = 0;
    PW_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
    PW_HIP(hipEventElapsedTime(&b, ev[1], ev[2]));
    PW_HIP(hipEventElapsedTime(&c, ev[2], ev[3]));
    pr.ms[0] += a;
    pr.ms[1] += b;
    pr.ms[2] += c;
  }
}

// iteration k of the selected iteration: parallel phase, corrector (update:
// Algorithm 1 on the new data; otherwise the current corrector is kept and
// no data matrices are formed), sweep and update
template <typename T>
void iteration(Prob& pr, int k, bool update, hipStream_t st) {
  hipEvent_t* ev = phase_events(pr, k);
  PW_HIP(hipEventRecord(ev[0], st));
  prop_fine<T>(pr, tp<T>(pr.u), tp<T>(pr.p), tp<T>(pr.v), tp<T>(pr.vp), pr.N, st);
  restrict_phase<T>(pr, st);
  prop_coarse<T>(pr, tp<T>(pr.Rc), tp<T>(pr.Rcp), tp<T>(pr.Uc), tp<T>(pr.Ucp), pr.N, st);
  PW_HIP(hipEventRecord(ev[1], st));
  if (pr.variant == PW_VARIANT_OMEGA_ONE || pr.variant == PW_VARIANT_PLAIN) {
    residual_identity_phase<T>(pr, k, st);
  } else if (update) {
    corrector_phase<T>(pr, k, st);
  } else {
    pr.ranks.push_back(pr.r);
    fill(pr.res + (long long)kRes * (k - 1), kRes, std::nan(""), st);
  }
  PW_HIP(hipEventRecord(ev[2], st));
  sweep_phase<T>(pr, st);
  PW_HIP(hipEventRecord(ev[3], st));
}

// iterations k_done + 1 .. k_done + K; with stop_tol > 0 the run ends after
// the first iteration whose change measure is <= stop_tol
template <typename T>
void run_iterations(Prob& pr, int K, bool update, double stop_tol, hipStream_t st) {
  const int k0 = pr.k_done;
  const bool stop_rule = stop_tol > 0;
  const size_t fb = pr.tsize * pr.Nf;
  const size_t bytes = fb * pr.N;
  int k = k0;
  while (k < k0 + K) {
    ++k;
    if (stop_rule && !pr.hist_u) {
      char* d = (char*)pr.prev.ensure(2 * bytes);
      PW_HIP(hipMemcpyAsync(d, (const char*)pr.u + fb, bytes, hipMemcpyDeviceToDevice, st));
      PW_HIP(hipMemcpyAsync(d + bytes, (const char*)pr.p + fb, bytes, hipMemcpyDeviceToDevice,
                            st));
    }
    iteration<T>(pr, k, update, st);
    pr.k_done = k;
    store_history(pr, k + 1, st);
    const double chg = stop_rule ? change_measure<T>(pr, k, st) : std::nan("");
    pr.change.push_back(chg);
    if (stop_rule && chg <= stop_tol) break;
  }
  accumulate_phase_times(pr, k0 + 1, k);
}

template <typename T>
void run_typed(Prob& pr, int K, double stop_tol, hipStream_t st) {
  hipEvent_t e0, e1;
  PW_HIP(hipEventCreate(&e0));
  PW_HIP(hipEventCreate(&e1));
  PW_HIP(hipEventRecord(e0, st));
  init_phase<T>(pr, st);
  pr.have_iterate = true;
  store_history(pr, 1, st);
  run_iterations<T>(pr, K, true, stop_tol, st);
  PW_HIP(hipEventRecord(e1, st));
  PW_HIP(hipEventSynchronize(e1));
  float tot = 0;
  PW_HIP(hipEventElapsedTime(&tot, e0, e1));
  pr.ms[3] = tot;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename T>
void continue_typed(Prob& pr, int K, bool update, double stop_tol, hipStream_t st) {
  hipEvent_t e0, e1;
  PW_HIP(hipEventCreate(&e0));
  PW_HIP(hipEventCreate(&e1));
  for (int i = 0; i < 4; ++i) pr.ms[i] = 0.0;
  PW_HIP(hipEventRecord(e0, st));
  run_iterations<T>(pr, K, update, stop_tol, st);
  PW_HIP(hipEventRecord(e1, st));
  PW_HIP(hipEventSynchronize(e1));
  float tot = 0;
  PW_HIP(hipEventElapsedTime(&tot, e0, e1));
  pr.ms[3] = tot;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename T>
__global__ void k_from_double(const double* in, T* out, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = (T)in[t];
}
__global__ void k_square(const double* in, double* out, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = in[t] * in[t];
}

template <typename T>
void set_medium_typed(Prob& pr, hipStream_t st) {
  const long long Nf = pr.Nf, Nc = pr.Nc;
  pr.ce_ok = false;  // C changes
  pr.cdc_ok = false;
  restrict_fields<double>(pr.gf, pr.ratio, pr.gc, pr.cf, Nf, pr.cc, Nc, 1, st);
  double* tmp = pr.c2c_d;  // coarse c^2 in double
  hipLaunchKernelGGL(k_square, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, st,
                     (const double*)pr.cc, tmp, Nc);
  PW_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_from_double<T>), dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, st,
                     (const double*)tmp, tp<T>(pr.c2c), Nc);
  PW_LAUNCH_CHECK();
  // fine c^2: square in double then round once
  double* ftmp = (double*)pr.itmp;
  hipLaunchKernelGGL(k_square, dim3((unsigned)((Nf + 255) / 256)), dim3(256), 0, st,
                     (const double*)pr.cf, ftmp, Nf);
  PW_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_from_double<T>), dim3((unsigned)((Nf + 255) / 256)), dim3(256), 0, st,
                     (const double*)ftmp, tp<T>(pr.c2f), Nf);
  PW_LAUNCH_CHECK();
}

template <typename T>
void set_initial_typed(Prob& pr, const double* u0, const double* p0, hipStream_t st) {
  const long long Nf = pr.Nf;
  hipLaunchKernelGGL((k_from_double<T>), dim3((unsigned)((Nf + 255) / 256)), dim3(256), 0, st, u0,
                     tp<T>(pr.u), Nf);
  PW_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_from_double<T>), dim3((unsigned)((Nf + 255) / 256)), dim3(256), 0, st, p0,
                     tp<T>(pr.p), Nf);
  PW_LAUNCH_CHECK();
}

template <typename T>
void serial_fine_typed(Prob& pr, int n, T* uo, T* po, hipStream_t st) {
  const long long Nf = pr.Nf;
  const T* su = tp<T>(pr.u);
  const T* sp = tp<T>(pr.p);
  if (n == 0) {
    PW_HIP(hipMemcpyAsync(uo, su, sizeof(T) * Nf, hipMemcpyDeviceToDevice, st));
    PW_HIP(hipMemcpyAsync(po, sp, sizeof(T) * Nf, hipMemcpyDeviceToDevice, st));
    return;
  }
  T* bu[2] = {tp<T>(pr.sfa_u), tp<T>(pr.sfb_u)};
  T* bp[2] = {tp<T>(pr.sfa_p), tp<T>(pr.sfb_p)};
  for (int i = 0; i < n; ++i) {
    T* du = (i == n - 1) ? uo : bu[i % 2];
    T* dp = (i == n - 1) ? po : bp[i % 2];
    prop_fine<T>(pr, su, sp, du, dp, 1, st, i + 1);
    su = du;
    sp = dp;
  }
}

// ---------------------------------------------------------------------------
// taped forward, frozen-corrector replay and the backward pass
// ---------------------------------------------------------------------------
void ensure_tape(Prob& pr, int K) {
  if (!pr.tape) pr.tape = std::make_unique<Tape>();
  Tape& t = *pr.tape;
  const int Kc = std::max(K, 1);
  if (t.mem && t.Kcap >= Kc) return;
  // (re)allocate for Kc iterations; the backward work buffers are kept
  t.mem.reset();
  t.mem = std::make_unique<Buffers>();
  Buffers& m = *t.mem;
  t.dims.clear();
  t.K = t.Kc = 0;
  t.epoch = -1;
  const long long N = pr.N, Nf = pr.Nf, Nc = pr.Nc;
  t.Kcap = Kc;
  // levels 0..Kc-1: slice starts of the iterations; level K: those of the
  // final iterate u^{K+1} (the start of a receiver record's sweep)
  t.us = m.get(pr.tsize * Nf * N * (Kc + 1));
  t.ps = m.get(pr.tsize * Nf * N * (Kc + 1));
  t.W = m.get_n<double>(2 * Nc * N);
  t.Din = m.get_n<double>(2 * Nc * N * Kc);
  t.delta = m.get_n<double>(2 * Nc * N * Kc);
  t.E = m.get_n<double>(2 * Nc * (pr.rmax + 1) * Kc);
  t.P = m.get_n<double>(2 * Nc * (pr.rmax + 1) * Kc);
}

template <typename T>
void tape_init_states(Prob& pr, Tape& t, hipStream_t st) {
  const long long Nc = pr.Nc;
  const int N = pr.N;
  // W_0 = R u0 (restricted by the initialisation), W_n = U_n (n >= 1)
  widen_fields<T>(tp<T>(pr.Rc), Nc, t.W, 2 * Nc, Nc, 1, st);
  widen_fields<T>(tp<T>(pr.Rcp), Nc, t.W + Nc, 2 * Nc, Nc, 1, st);
  widen_fields<T>(tp<T>(pr.Uc), Nc, t.W + 2 * Nc, 2 * Nc, Nc, N - 1, st);
  widen_fields<T>(tp<T>(pr.Ucp), Nc, t.W + 3 * Nc, 2 * Nc, Nc, N - 1, st);
}

// Algorithm 3 recording the tape.  frozen = false: the corrector of every
// iteration comes from Algorithm 1 as in pw_run and is recorded; frozen =
// true: the recorded correctors are replayed (no data matrices, no SVD),
// with the current medium in F, C and R.
template <typename T>
void run_taped_typed(Prob& pr, int K, bool frozen, hipStream_t st) {
  Tape& t = *pr.tape;
  const int N = pr.N;
  const long long Nf = pr.Nf, Nc = pr.Nc;
  const size_t sbytes = pr.tsize * Nf * N;
  const long long ecols = 2 * Nc * (pr.rmax + 1);
  hipEvent_t e0, e1;
  PW_HIP(hipEventCreate(&e0));
  PW_HIP(hipEventCreate(&e1));
  PW_HIP(hipEventRecord(e0, st));
  init_phase<T>(pr, st);
  pr.have_iterate = true;
  ++pr.tape_serial;
  tape_init_states<T>(pr, t, st);
  if (!frozen) t.dims.assign(K, 0);
  for (int k = 1; k <= K; ++k) {
    const int kk = k - 1;
    PW_HIP(hipMemcpyAsync((char*)t.us + sbytes * kk, pr.u, sbytes, hipMemcpyDeviceToDevice, st));
    PW_HIP(hipMemcpyAsync((char*)t.ps + sbytes * kk, pr.p, sbytes, hipMemcpyDeviceToDevice, st));
    prop_fine<T>(pr, tp<T>(pr.u), tp<T>(pr.p), tp<T>(pr.v), tp<T>(pr.vp), N, st);
    const double* E;
    const double* P;
    int dim;
    if (!frozen) {
      restrict_phase<T>(pr, st);
      prop_coarse<T>(pr, tp<T>(pr.Rc), tp<T>(pr.Rcp), tp<T>(pr.Uc), tp<T>(pr.Ucp), N, st);
      corrector_phase<T>(pr, k, st);
      E = pr.E[pr.cur];
      P = pr.Vp[pr.cur];
      dim = pr.r + 1;
      PW_HIP(hipMemcpyAsync(t.E + ecols * kk, E, sizeof(double) * 2 * Nc * dim,
                            hipMemcpyDeviceToDevice, st));
      PW_HIP(hipMemcpyAsync(t.P + ecols * kk, P, sizeof(double) * 2 * Nc * dim,
                            hipMemcpyDeviceToDevice, st));
      t.dims[kk] = dim;
    } else {
      E = t.E + ecols * kk;
      P = t.P + ecols * kk;
      dim = t.dims[kk];
    }
    // C E in full, as the backward forms it from the taped E
    sweep_core<T>(pr, E, P, dim, st, false);
    PW_HIP(hipMemcpyAsync(t.Din + 2 * Nc * N * kk, pr.Din, sizeof(double) * 2 * Nc * N,
                          hipMemcpyDeviceToDevice, st));
    PW_HIP(hipMemcpyAsync(t.delta + 2 * Nc * N * kk, pr.delta, sizeof(double) * 2 * Nc * N,
                          hipMemcpyDeviceToDevice, st));
    if (!frozen) {
      pr.k_done = k;
      pr.change.push_back(std::nan(""));
    }
  }
  PW_HIP(hipMemcpyAsync((char*)t.us + sbytes * K, pr.u, sbytes, hipMemcpyDeviceToDevice, st));
  PW_HIP(hipMemcpyAsync((char*)t.ps + sbytes * K, pr.p, sbytes, hipMemcpyDeviceToDevice, st));
  PW_HIP(hipEventRecord(e1, st));
  PW_HIP(hipEventSynchronize(e1));
  float ms = 0;
  PW_HIP(hipEventElapsedTime(&ms, e0, e1));
  pr.adj_ms[0] = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  t.K = K;
  if (!frozen) t.Kc = K;
  t.epoch = pr.epoch;
  if (frozen) {
    pr.k_done = 0;  // no residuals: the data matrices were not formed
    pr.ranks.clear();
    pr.change.clear();
    pr.have_iterate = false;  // the state is a frozen replay, not an iterate to continue
  }
}

void ensure_backward(Prob& pr, int ckpt) {
  Tape& t = *pr.tape;
  if (t.bw && t.bw_ckpt == ckpt) return;
  t.bw.reset();
  t.bw = std::make_unique<Buffers>();
  Buffers& m = *t.bw;
  const long long N = pr.N, Nf = pr.Nf, Nc = pr.Nc;
  const long long d1 = pr.rmax + 1;
  t.La = m.get_n<double>((N + 1) * 2 * Nf);
  t.Lb = m.get_n<double>((N + 1) * 2 * Nf);
  t.Wf = m.get_n<double>(N * 2 * Nf);
  t.GF = m.get_n<double>(N * Nf);
  t.GC = m.get_n<double>(N * Nc);
  t.gc = m.get_n<double>(Nc);
  t.grad = m.get_n<double>(Nf);
  t.c2f = m.get_n<double>(Nf);
  t.Y = m.get_n<double>(2 * Nc * N);
  t.LA = m.get_n<double>(2 * Nc * N);
  t.X = m.get_n<double>(2 * Nc * N);
  t.Cn = m.get_n<double>(d1 * N);
  t.Cr = m.get_n<double>(d1 * N);
  t.Sr = m.get_n<double>(d1 * N);
  t.Sn = m.get_n<double>(d1 * N);
  t.MT = m.get_n<double>(d1 * d1);
  if (pr.sponge) {
    t.layF = m.get_n<double>(4 * Nf);
    t.layC = m.get_n<double>(4 * Nc);
  }
  // one time level holds N fine states (>= N coarse columns)
  const int msteps = std::max(pr.mF, pr.mC);
  AdjScratch& a = t.as;
  a.state_elems = N * Nf;
  a.max_ckpt = (msteps + ckpt - 1) / ckpt;
  a.max_seg = std::min(ckpt, msteps) + 1;
  a.ck_u = m.get_n<double>(a.state_elems * a.max_ckpt);
  a.ck_p = m.get_n<double>(a.state_elems * a.max_ckpt);
  a.seg = m.get_n<double>(a.state_elems * a.max_seg);
  a.p_tmp = m.get_n<double>(a.state_elems);
  a.p_tmp2 = m.get_n<double>(a.state_elems);
  a.a_tmp = m.get_n<double>(a.state_elems);
  a.lp_tmp = m.get_n<double>(a.state_elems);
  t.bw_ckpt = ckpt;
}

// d J / d c^2 of J = sum_{n, r} seed[n][r] u^{K+1}_{n+1}(x_r) through the
// recorded run (frozen correctors), written to t.grad (fine grid, FP64).
// rec_rows != null: J = sum seed[n][i][r] (u of slice n + 1 after step i + 1
// of the sweep from u^{K+1}_n) at x_r, the record of pw_trace_sweep (rec_rows,
// rec_map: its receiver tables on the device).
template <typename T>
void backward_typed(Prob& pr, const long long* rec, int nrec, const double* seed, int ckpt,
                    hipStream_t st, const int* rec_rows = nullptr,
                    const int* rec_map = nullptr) {
  Tape& t = *pr.tape;
  const int N = pr.N, K = t.K;
  const long long Nf = pr.Nf, Nc = pr.Nc;
  const long long F2 = 2 * Nf, C2 = 2 * Nc;
  const long long ecols = C2 * (pr.rmax + 1);
  const Grid& gf = pr.gf;
  const Grid& gc = pr.gc;
  hipEvent_t e0, e1;
  PW_HIP(hipEventCreate(&e0));
  PW_HIP(hipEventCreate(&e1));
  PW_HIP(hipEventRecord(e0, st));
  mul_fields(pr.cf, pr.cf, t.c2f, Nf, 1.0, st);
  fill(t.La, (N + 1) * F2, 0.0, st);
  fill(t.Lb, (N + 1) * F2, 0.0, st);
  fill(t.GF, (long long)N * Nf, 0.0, st);
  fill(t.GC, (long long)N * Nc, 0.0, st);
  // slot n of A holds the adjoint of the state u_n ([u; p], n = 0..N)
  double* A = t.La;
  double* B = t.Lb;
  // the layer and source of F, C (slice n from t_{n-1}) and the layer
  // alone for the coarse propagations of differences
  Force<double> fF, fCl;
  // the layer's per-point fields for the reverse streams
  auto with_fields = [&](Force<double> f, bool fine) {
    if (!pr.sponge) return f;
    const double* base = fine ? t.layF : t.layC;
    const long long np = fine ? Nf : Nc;
    f.wf = base;
    f.s2 = base + np;
    f.dd = base + 2 * np;
    f.c2e = base + 3 * np;
    return f;
  };
  if (pr.sponge) {
    layer_fields(gf, pr.layF_d, pr.layF_d + gf.n[0], t.c2f, t.layF, st);
    layer_fields(gc, pr.layC_d, pr.layC_d + gc.n[0], pr.c2c_d, t.layC, st);
  }
  if (forced(pr)) {
    fF = with_fields(make_force<double>(pr, true, true, 1, true, false), true);
    fCl = with_fields(make_force<double>(pr, false, false, 1, false, false), false);
  }
  const Force<double>* pF = forced(pr) ? &fF : nullptr;
  const Force<double>* pCl = pr.sponge ? &fCl : nullptr;
  if (rec_rows) {
    // the record's sweep from u^{K+1}_n, n = 0..N-1 (tape level K): its
    // adjoint, with the seeds entering after every step, lands in slots
    // 0..N-1
    widen_fields<T>(tp<T>(t.us) + Nf * N * K, Nf, t.Wf, F2, Nf, N, st);
    widen_fields<T>(tp<T>(t.ps) + Nf * N * K, Nf, t.Wf + Nf, F2, Nf, N, st);
    Force<double> fS = with_fields(make_force<double>(pr, true, true, 1, true, false), true);
    fS.rec = rec;
    fS.rec_rows = rec_rows;
    fS.rec_map = rec_map;
    fS.n_rec = nrec;
    fS.m_tr = pr.mF;
    fS.seeds = seed;
    vv_adjoint(gf, t.c2f, t.Wf, t.Wf + Nf, F2, A, A + Nf, F2, t.GF, Nf, N, pr.mF, pr.hF, ckpt,
               t.as, st, &fS);
  } else {
    receiver_scatter(seed, rec, nrec, N, A + F2, F2, st);
  }
  for (int k = K; k >= 1; --k) {
    const int kk = k - 1;
    const double* E = t.E + ecols * kk;
    const double* P = t.P + ecols * kk;
    const int dim = t.dims[kk];
    const double* Din = t.Din + C2 * N * kk;
    const double* dl = t.delta + C2 * N * kk;
    // adjoint of u^{k+1}_n = v_n + I E t_n: y_n = I^T L_n, c_n = E^T y_n
    interp_transpose(gf, gc, pr.ratio, pr.itab, A + F2, F2, t.Y, C2, N, pr.itmp, st);
    interp_transpose(gf, gc, pr.ratio, pr.itab, A + F2 + Nf, F2, t.Y + Nc, C2, N, pr.itmp, st);
    gemm_tn(C2, dim, N, 1.0, E, C2, t.Y, C2, 0.0, t.Cn, dim, pr.gwork, pr.gwork_elems, st);
    // t_n = P^T a_n + M t_{n-1}, M = P^T C E: s_n = c_n + M^T s_{n+1}
    prop_coarse_cols(pr, E, pr.CE, dim, st);
    gemm_tn(C2, dim, dim, 1.0, pr.CE, C2, P, C2, 0.0, t.MT, dim, pr.gwork, pr.gwork_elems, st);
    reverse_cols(dim, N, t.Cn, dim, t.Cr, dim, st);
    recurrence(dim, N, t.MT, t.Cr, t.Sr, pr.rs, st);
    reverse_cols(dim, N, t.Sr, dim, t.Sn, dim, st);
    // adjoint of a_n: P s_n
    gemm_nn(C2, N, dim, 1.0, P, C2, t.Sn, dim, 0.0, t.LA, C2, st);
    // C acts on x_n = Din_n + delta_{n-1} (a_n and the C E t_{n-1} of M)
    copy_fields(Din, C2 * N, t.X, C2 * N, C2 * N, 1, st);
    add_inplace(t.X + C2, dl, C2 * (N - 1), st);
    vv_adjoint(gc, pr.c2c_d, t.X, t.X + Nc, C2, t.LA, t.LA + Nc, C2, t.GC, Nc, N, pr.mC, pr.hC,
               ckpt, t.as, st, pCl);
    // LA column n now holds the adjoint of Din_{n+1} = R v_n - R u^k_n
    restrict_transpose_add(gf, pr.ratio, gc, t.LA + C2, C2, A + F2, F2, 1.0, N - 1, st);
    restrict_transpose_add(gf, pr.ratio, gc, t.LA + C2 + Nc, C2, A + F2 + Nf, F2, 1.0, N - 1,
                           st);
    // v_n = F u^k_{n-1}
    widen_fields<T>(tp<T>(t.us) + Nf * N * kk, Nf, t.Wf, F2, Nf, N, st);
    widen_fields<T>(tp<T>(t.ps) + Nf * N * kk, Nf, t.Wf + Nf, F2, Nf, N, st);
    vv_adjoint(gf, t.c2f, t.Wf, t.Wf + Nf, F2, A + F2, A + F2 + Nf, F2, t.GF, Nf, N, pr.mF, pr.hF,
               ckpt, t.as, st, pF);
    // slot n of A: adjoint of u^k_{n-1} through F; shift into B and add the
    // -R^T part of Din
    copy_fields(A + 2 * F2, F2, B + F2, F2, F2, N - 1, st);
    restrict_transpose_add(gf, pr.ratio, gc, t.LA + C2, C2, B + F2, F2, -1.0, N - 1, st);
    restrict_transpose_add(gf, pr.ratio, gc, t.LA + C2 + Nc, C2, B + F2 + Nf, F2, -1.0, N - 1,
                           st);
    fill(B + (long long)N * F2, F2, 0.0, st);
    std::swap(A, B);
  }
  // initialisation u^1_n = I W_n, W_n = C W_{n-1}
  interp_transpose(gf, gc, pr.ratio, pr.itab, A + F2, F2, t.Y, C2, N, pr.itmp, st);
  interp_transpose(gf, gc, pr.ratio, pr.itab, A + F2 + Nf, F2, t.Y + Nc, C2, N, pr.itmp, st);
  double* lam = t.LA;
  fill(lam, C2, 0.0, st);
  for (int n = N; n >= 1; --n) {
    add_inplace(lam, t.Y + C2 * (n - 1), C2, st);
    const double* Wn = t.W + C2 * (n - 1);
    Force<double> fCn;
    if (forced(pr)) fCn = with_fields(make_force<double>(pr, false, true, n, false, false), false);
    vv_adjoint(gc, pr.c2c_d, Wn, Wn + Nc, C2, lam, lam + Nc, C2, t.GC, Nc, 1, pr.mC, pr.hC, ckpt,
               t.as, st, forced(pr) ? &fCn : nullptr);
  }
  // the gradient: fine accumulators + R^T of the coarse ones
  sum_fields(t.GC, Nc, N, t.gc, Nc, false, st);
  sum_fields(t.GF, Nf, N, t.grad, Nf, false, st);
  restrict_transpose_add(gf, pr.ratio, gc, t.gc, Nc, t.grad, Nf, 1.0, 1, st);
  PW_HIP(hipEventRecord(e1, st));
  PW_HIP(hipEventSynchronize(e1));
  float ms = 0;
  PW_HIP(hipEventElapsedTime(&ms, e0, e1));
  pr.adj_ms[1] = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// ---------------------------------------------------------------------------
// batched lockstep driver, hipGraph capture and the autotuner
// ---------------------------------------------------------------------------
template <typename T>
MultiPlan<T>& planF(Batch& b);
template <>
MultiPlan<float>& planF<float>(Batch& b) { return b.F32; }
template <>
MultiPlan<double>& planF<double>(Batch& b) { return b.F64; }
template <typename T>
MultiPlan<T>& planC(Batch& b);
template <>
MultiPlan<float>& planC<float>(Batch& b) { return b.C32; }
template <>
MultiPlan<double>& planC<double>(Batch& b) { return b.C64; }

int ly_for(const std::vector<std::pair<int, int>>& by_size, int ny) {
  for (auto& e : by_size)
    if (e.first == ny) return e.second;
  return 0;
}

template <typename T>
std::vector<PropJob<T>> fine_jobs(pw_ctx* ctx,
                                  const std::vector<std::pair<int, int>>& by_size = {}) {
  std::vector<PropJob<T>> jobs;
  for (auto& up : ctx->probs) {
    Prob& pr = *up;
    PropJob<T> j;
    j.Ly = ly_for(by_size, pr.gf.n[1]);
    j.g = pr.gf;
    j.c2 = tp<T>(pr.c2f);
    j.u_src = tp<T>(pr.u);
    j.p_src = tp<T>(pr.p);
    j.u_dst = tp<T>(pr.v);
    j.p_dst = tp<T>(pr.vp);
    j.sstride = pr.Nf;
    j.nstates = pr.N;
    j.m = pr.mF;
    j.h = (T)pr.hF;
    j.wa = fine_work<T>(pr, 0);
    j.wb = fine_work<T>(pr, 1);
    jobs.push_back(j);
  }
  return jobs;
}

template <typename T>
std::vector<PropJob<T>> coarse_jobs(pw_ctx* ctx) {
  std::vector<PropJob<T>> jobs;
  for (auto& up : ctx->probs) {
    Prob& pr = *up;
    PropJob<T> j;
    j.g = pr.gc;
    j.c2 = tp<T>(pr.c2c);
    j.u_src = tp<T>(pr.Rc);
    j.p_src = tp<T>(pr.Rcp);
    j.u_dst = tp<T>(pr.Uc);
    j.p_dst = tp<T>(pr.Ucp);
    j.sstride = pr.Nc;
    j.nstates = pr.N;
    j.m = pr.mC;
    j.h = (T)pr.hC;
    j.wa = coarse_work<T>(pr, 0);
    j.wb = coarse_work<T>(pr, 1);
    jobs.push_back(j);
  }
  return jobs;
}

template <typename T>
void* upload_plan(Batch& b, const MultiPlan<T>& pl, hipStream_t st) {
  void* d = b.mem.get(sizeof(StreamDesc<T>) * std::max<size_t>(pl.descs.size(), 1));
  PW_HIP(hipMemcpyAsync(d, pl.descs.data(), sizeof(StreamDesc<T>) * pl.descs.size(),
                        hipMemcpyHostToDevice, st));
  PW_HIP(hipStreamSynchronize(st));
  return d;
}

std::string tune_key(pw_ctx* ctx, bool f64, bool comp) {
  hipDeviceProp_t prop;
  int dev = 0;
  PW_HIP(hipGetDevice(&dev));
  PW_HIP(hipGetDeviceProperties(&prop, dev));
  std::string k = std::string(prop.gcnArchName) + (f64 ? "|f64" : "|f32") + (comp ? "c" : "");
  std::vector<std::string> items;
  for (auto& up : ctx->probs) {
    char buf[96];
    snprintf(buf, sizeof(buf), "%dx%dN%dm%d", up->gf.n[0], up->gf.n[1], up->N, up->mF);
    items.push_back(buf);
  }
  std::sort(items.begin(), items.end());
  for (auto& i : items) k += "|" + i;
  for (auto& ch : k)
    if (ch == ' ' || ch == ':') ch = '_';
  return k;
}

// cache line: key B Ly count (ny Ly)*count
bool tune_lookup(const std::string& key, int* B, int* Ly,
                 std::vector<std::pair<int, int>>* by_size) {
  const char* path = getenv("PW_TUNE_CACHE");
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char kb[4096];
  int b = 0, l = 0, cnt = 0;
  bool found = false;
  while (fscanf(f, "%4095s %d %d %d", kb, &b, &l, &cnt) == 4) {
    if (cnt < 0 || cnt > 64) break;
    std::vector<std::pair<int, int>> v;
    bool ok = true;
    for (int i = 0; i < cnt; ++i) {
      int a = 0, c = 0;
      if (fscanf(f, "%d %d", &a, &c) != 2) {
        ok = false;
        break;
      }
      v.push_back({a, c});
    }
    if (!ok) break;
    if (key == kb && (b == 4 || b == 8) && l > 0) {
      *B = b;
      *Ly = l;
      *by_size = v;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void tune_store(const std::string& key, int B, int Ly,
                const std::vector<std::pair<int, int>>& by_size) {
  const char* path = getenv("PW_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d", key.c_str(), B, Ly, (int)by_size.size());
  for (auto& e : by_size) fprintf(f, " %d %d", e.first, e.second);
  fprintf(f, "\n");
  fclose(f);
}

// time the batched fine sweep of each candidate (pipeline depth, rows per
// stream) and keep the fastest
template <typename T>
void autotune(pw_ctx* ctx, Batch& b, hipStream_t st) {
  const std::string key = tune_key(ctx, b.f64, b.comp);
  int B = 0, Ly = 0;
  std::vector<std::pair<int, int>> by_size;
  if (tune_lookup(key, &B, &Ly, &by_size)) {
    b.B = B;
    b.Ly = Ly;
    b.ly_by_size = by_size;
    b.from_cache = true;
    return;
  }
  std::vector<std::pair<int, int>> cands;
  const int Bs_f[2] = {8, 4};
  const int Ls[3] = {64, 128, 256};
  for (int bb : Bs_f) {
    if (sizeof(T) == 8 && bb != 4) continue;
    for (int l : Ls) cands.push_back({bb, l});
  }
  hipEvent_t e0, e1, t0, t1;
  PW_HIP(hipEventCreate(&e0));
  PW_HIP(hipEventCreate(&e1));
  PW_HIP(hipEventCreate(&t0));
  PW_HIP(hipEventCreate(&t1));
  PW_HIP(hipEventRecord(t0, st));
  // time the fine sweep of one plan (a warm-up run, then the mean of two)
  auto time_plan = [&](int Bc, int Lc, const std::vector<std::pair<int, int>>& bs) -> double {
    MultiPlan<T> pl;
    pl.B = Bc;
    pl.Ly = Lc;
    plan_multi<T>(fine_jobs<T>(ctx, bs), pl);
    Buffers tmp;
    void* d = tmp.get(sizeof(StreamDesc<T>) * std::max<size_t>(pl.descs.size(), 1));
    PW_HIP(hipMemcpyAsync(d, pl.descs.data(), sizeof(StreamDesc<T>) * pl.descs.size(),
                          hipMemcpyHostToDevice, st));
    run_multi<T>(pl, (const StreamDesc<T>*)d, b.comp, st);  // warm
    PW_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 2; ++r) run_multi<T>(pl, (const StreamDesc<T>*)d, b.comp, st);
    PW_HIP(hipEventRecord(e1, st));
    PW_HIP(hipEventSynchronize(e1));
    float ms = 0;
    PW_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms / 2;
  };
  // 1. one (depth, rows per stream) for all problems
  double best = 1e30;
  for (auto c : cands) {
    const double ms = time_plan(c.first, c.second, {});
    if (ms < best) {
      best = ms;
      b.B = c.first;
      b.Ly = c.second;
    }
  }
  // 2. rows per stream refined per fine grid size, one size at a time with
  //    the others held (the depth is launch-wide: one kernel per time block)
  std::vector<int> sizes;
  for (auto& up : ctx->probs) sizes.push_back(up->gf.n[1]);
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  b.ly_by_size.clear();
  if (sizes.size() > 1) {
    for (int ny : sizes) {
      int keep = 0;
      for (int l : {b.Ly / 2, 2 * b.Ly}) {
        if (l == b.Ly) continue;
        auto trial = b.ly_by_size;
        trial.push_back({ny, l});
        const double ms = time_plan(b.B, b.Ly, trial);
        if (ms < best * 0.995) {
          best = ms;
          keep = l;
        }
      }
      if (keep > 0) b.ly_by_size.push_back({ny, keep});
    }
  }
  PW_HIP(hipEventRecord(t1, st));
  PW_HIP(hipEventSynchronize(t1));
  float tt = 0;
  PW_HIP(hipEventElapsedTime(&tt, t0, t1));
  b.tune_ms = tt;
  b.best_ms = best;
  for (hipEvent_t e : {e0, e1, t0, t1}) (void)hipEventDestroy(e);
  tune_store(key, b.B, b.Ly, b.ly_by_size);
}

// the parallel phase of every problem: fine sweeps, restrictions, coarse
// propagations (fixed buffers: graph-capturable)
template <typename T>
void batch_parallel_phase(pw_ctx* ctx, Batch& b, hipStream_t st) {
  run_multi<T>(planF<T>(b), (const StreamDesc<T>*)b.dF, b.comp, st);
  for (auto& up : ctx->probs) restrict_phase<T>(*up, st);
  run_multi<T>(planC<T>(b), (const StreamDesc<T>*)b.dC, b.comp, st);
}

template <typename T>
void build_batch(pw_ctx* ctx, Batch& b) {
  hipStream_t st = ctx->stream;
  autotune<T>(ctx, b, st);
  MultiPlan<T>& F = planF<T>(b);
  MultiPlan<T>& C = planC<T>(b);
  F.B = b.B;
  F.Ly = b.Ly;
  plan_multi<T>(fine_jobs<T>(ctx, b.ly_by_size), F);
  C.B = b.B;
  C.Ly = b.Ly;
  plan_multi<T>(coarse_jobs<T>(ctx), C);
  b.dF = upload_plan<T>(b, F, st);
  b.dC = upload_plan<T>(b, C, st);
  PW_HIP(hipStreamCreateWithFlags(&b.cap_stream, hipStreamNonBlocking));
  PW_HIP(hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    batch_parallel_phase<T>(ctx, b, b.cap_stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  PW_HIP(hipStreamEndCapture(b.cap_stream, &b.graph));
  PW_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
  for (auto& e : b.ev) PW_HIP(hipEventCreate(&e));
  PW_HIP(hipEventCreateWithFlags(&b.fork_ev, hipEventDisableTiming));
  b.built = true;
}

// run fn(problem index) for every problem on a pool of host threads; the
// first error is rethrown after every problem stream has drained
template <typename Fn>
void for_problems(pw_ctx* ctx, Fn fn) {
  const int np = (int)ctx->probs.size();
  std::atomic<int> next{0};
  std::vector<Error> errs;
  std::mutex mu;
  auto worker = [&] {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= np) return;
      try {
        fn(i);
      } catch (const Error& e) {
        std::lock_guard<std::mutex> lock(mu);
        errs.push_back(e);
        next.store(np);
      } catch (const std::exception& e) {
        std::lock_guard<std::mutex> lock(mu);
        errs.push_back(Error{PW_EINVAL, e.what()});
        next.store(np);
      }
    }
  };
  static const int threads = [] {
    const char* e = getenv("PW_BATCH_THREADS");  // override (1: one host thread)
    const int v = e ? atoi(e) : kBatchThreads;
    return v >= 1 && v <= 64 ? v : kBatchThreads;
  }();
  const int nt = std::max(1, std::min(np, threads));
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  if (!errs.empty()) {
    for (auto& up : ctx->probs) (void)hipStreamSynchronize(up->own);
    throw errs.front();
  }
}

// The corrector (data matrices, Algorithm 1) and the corrected sweep of
// every problem of a batch, after the batched parallel phase enqueued on
// `st`: each problem's Algorithm 1 up to its core matrix on its own stream
// (driven by one of a few host threads, so that the problems' chains of
// small launches and host synchronisations overlap), then the SVDs of all
// core matrices together on `st` (one launch per Jacobi round for all of
// them), then each problem's rest of Algorithm 1 and its sweep on its own
// stream again.  The context stream then waits for every problem.
template <typename T>
void concurrent_serial_phase(pw_ctx* ctx, int k, hipStream_t st) {
  const int np = (int)ctx->probs.size();
  Batch& b = *ctx->batch;
  hipEvent_t start = b.fork_ev;
  PW_HIP(hipEventRecord(start, st));
  std::vector<SvdPending> sp((size_t)np);
  for_problems(ctx, [&](int i) {
    Prob& pr = *ctx->probs[(size_t)i];
    PW_HIP(hipStreamWaitEvent(pr.own, start, 0));
    sp[(size_t)i] = corrector_begin<T>(pr, k, pr.own);
    PW_HIP(hipEventRecord(pr.pre_ev, pr.own));
  });
  std::vector<SvdJob> jobs;
  for (int i = 0; i < np; ++i) {
    Prob& pr = *ctx->probs[(size_t)i];
    PW_HIP(hipStreamWaitEvent(st, pr.pre_ev, 0));
    jobs.push_back(svd_job(pr, sp[(size_t)i].n));
  }
  if (!b.svd_jobs) {
    b.svd_jobs = b.mem.get(2 * (size_t)np * svd_multi_job_bytes());
    b.svd_counts = b.mem.get_n<int>(np);
    PW_HIP(hipEventCreateWithFlags(&b.svd_ev, hipEventDisableTiming));
  }
  svd_jacobi_multi(jobs, b.svd_jobs, b.svd_counts, st);
  PW_HIP(hipEventRecord(b.svd_ev, st));
  for_problems(ctx, [&](int i) {
    Prob& pr = *ctx->probs[(size_t)i];
    PW_HIP(hipStreamWaitEvent(pr.own, b.svd_ev, 0));
    corrector_end<T>(pr, k, sp[(size_t)i], pr.own);
    sweep_phase<T>(pr, pr.own);
    PW_HIP(hipEventRecord(pr.done_ev, pr.own));
  });
  for (auto& up : ctx->probs) PW_HIP(hipStreamWaitEvent(st, up->done_ev, 0));
}

template <typename T>
void run_batch_typed(pw_ctx* ctx, int K) {
  Batch& b = *ctx->batch;
  hipStream_t st = ctx->stream;
  if (!b.built) build_batch<T>(ctx, b);
  for (int i = 0; i < 4; ++i) b.ms[i] = 0.0;
  hipEvent_t e0, e1;
  PW_HIP(hipEventCreate(&e0));
  PW_HIP(hipEventCreate(&e1));
  PW_HIP(hipEventRecord(e0, st));
  for (auto& up : ctx->probs) {
    init_phase<T>(*up, st);
    up->have_iterate = true;
    store_history(*up, 1, st);
  }
  for (int k = 1; k <= K; ++k) {
    PW_HIP(hipEventRecord(b.ev[0], st));
    PW_HIP(hipGraphLaunch(b.exec, st));
    PW_HIP(hipEventRecord(b.ev[1], st));
    concurrent_serial_phase<T>(ctx, k, st);
    PW_HIP(hipEventRecord(b.ev[2], st));
    PW_HIP(hipEventRecord(b.ev[3], st));
    PW_HIP(hipEventSynchronize(b.ev[3]));
    float x = 0, y = 0, z = 0;
    PW_HIP(hipEventElapsedTime(&x, b.ev[0], b.ev[1]));
    PW_HIP(hipEventElapsedTime(&y, b.ev[1], b.ev[2]));
    PW_HIP(hipEventElapsedTime(&z, b.ev[2], b.ev[3]));
    b.ms[0] += x;
    b.ms[1] += y;
    b.ms[2] += z;
    for (auto& up : ctx->probs) {
      up->k_done = k;
      up->change.push_back(std::nan(""));
      store_history(*up, k + 1, st);
    }
  }
  PW_HIP(hipEventRecord(e1, st));
  PW_HIP(hipEventSynchronize(e1));
  float tot = 0;
  PW_HIP(hipEventElapsedTime(&tot, e0, e1));
  b.ms[3] = tot;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

pw_status report(const Error& e) {
  g_last_error = e.msg;
  return e.status;
}

template <typename F>
pw_status guarded(F&& f) {
  try {
    f();
    return PW_OK;
  } catch (const Error& e) {
    return report(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return PW_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PW_EINVAL;
  }
}

const void* stage_in(const double* src, long long n, int on_device, Prob& pr, double* scratch,
                     hipStream_t st) {
  (void)pr;
  if (on_device) return src;
  PW_HIP(hipMemcpyAsync(scratch, src, sizeof(double) * n, hipMemcpyHostToDevice, st));
  return scratch;
}

// E = [Lambda^dag_u U~ , DC] and P = [Lambda^T V~ , DC] of the current
// corrector, formed directly from U~ and V~ (in chunks of at most N columns,
// the capacity of the transform scratch)
void rebuild_sweep_columns(Prob& pr, hipStream_t st) {
  const long long rows = pr.rows, Nc = pr.Nc;
  const int r = pr.r, cur = pr.cur;
  pr.ce_ok = false;
  for (int j0 = 0; j0 < r; j0 += pr.N) {
    const int nc = std::min(pr.N, r - j0);
    lambda_dag_cols(pr.gc, pr.dtab, pr.Ub[cur] + rows * j0, rows, pr.cc, nullptr,
                    pr.E[cur] + 2 * Nc * j0, 2 * Nc, nc, pr.ctmp, st);
    lambda_adjoint_cols(pr.gc, pr.Vb[cur] + rows * j0, rows, pr.cc, pr.order,
                        pr.Vp[cur] + 2 * Nc * j0, 2 * Nc, nc, st, &pr.spec);
  }
  set_dc_column(pr.E[cur], 2 * Nc, r, Nc, 1.0 / (double)Nc, st);
  set_dc_column(pr.Vp[cur], 2 * Nc, r, Nc, 1.0, st);
}

// the point source of pw_set_source (pos = null: none)
void set_source(Prob& pr, const double* pos, double freq, double t0) {
  if (!pos) {
    pr.have_src = false;
    return;
  }
  if (pr.gf.dim != 2) fail(PW_EINVAL, "the point source is implemented for 2D problems only");
  if (!(freq > 0) || !std::isfinite(freq) || !std::isfinite(t0))
    fail(PW_EINVAL, "the source needs a positive finite frequency and a finite t0");
  for (int a = 0; a < pr.gf.dim; ++a)
    if (!std::isfinite(pos[a])) fail(PW_EINVAL, "source position must be finite");
  // nearest node (ties to even), periodic
  for (int g = 0; g < 2; ++g) {
    const Grid& gr = g == 0 ? pr.gf : pr.gc;
    int* node = g == 0 ? pr.srcF : pr.srcC;
    for (int a = 0; a < 2; ++a) {
      const double j = std::nearbyint(pos[a] / gr.dx);
      long long k = (long long)std::fmod(j, (double)gr.n[a]);
      if (k < 0) k += gr.n[a];
      node[a] = (int)k;
    }
  }
  for (int a = 0; a < 3; ++a) pr.src_pos[a] = a < pr.gf.dim ? pos[a] : 0.0;
  pr.src_freq = freq;
  pr.src_t0 = t0;
  // the Ricker wavelet (1 - 2a) exp(-a), a = (pi f (t - t0))^2, at the kick
  // times of every slice, t = (n - 1) T / N + i h
  const double dtc = pr.P.T / pr.N;
  for (int g = 0; g < 2; ++g) {
    const int m = g == 0 ? pr.mF : pr.mC;
    const double h = g == 0 ? pr.hF : pr.hC;
    std::vector<double> tab((size_t)pr.N * (m + 1));
    for (int n = 0; n < pr.N; ++n)
      for (int i = 0; i <= m; ++i) {
        const double b = M_PI * freq * ((n * dtc + i * h) - t0);
        const double a = b * b;
        tab[(size_t)n * (m + 1) + i] = (1.0 - 2.0 * a) * std::exp(-a);
      }
    DevBuf& dst = g == 0 ? pr.srcF_tab : pr.srcC_tab;
    PW_HIP(hipMemcpy(dst.ensure(sizeof(double) * tab.size()), tab.data(),
                     sizeof(double) * tab.size(), hipMemcpyHostToDevice));
  }
  pr.have_src = true;
}

// ---- checkpoint files ---------------------------------------------------
// Layout (host byte order): "PWCKPT02", int32 number of problems, then per
// problem: its pw_problem fields as 20 int64 / double slots, int32 flags
// [have_medium, have_initial, have_iterate, variant, k_done, r, cur,
// samp_n, samp_iters, n_ranks, n_change, history levels, have_source,
// have_CE, 0, 0], then the blocks that exist: c (Nf doubles); u0, p0 (state
// dtype); the current iterate n = 1..N; the history levels; ranks; change;
// the per-iteration record; U~, V~ (rows x r), S~ (r), E, P (2 Nc x (r + 1));
// the sampling table; the source (x, y, freq, t0); C E (2 Nc x (r + 1)).
// A file without C E (have_CE = 0) loads; C E is then formed in full at the
// next sweep.
constexpr char kCkptMagic[9] = "PWCKPT02";
constexpr int kSlots = 20;

void problem_slots(const pw_problem& P, double* d) {
  const double v[kSlots] = {(double)P.dim, (double)P.n_fine[0], (double)P.n_fine[1],
                            (double)P.n_fine[2], (double)P.ratio, P.T, (double)P.n_slices,
                            (double)P.m_fine, (double)P.m_coarse, (double)P.grad_order,
                            P.svd_tol, (double)P.state_dtype, (double)P.compensated,
                            (double)P.max_iters, (double)P.interp, (double)P.keep_history,
                            (double)P.bc, P.sponge_width, P.sponge_reflection, P.sponge_cmax};
  std::memcpy(d, v, sizeof(v));
}

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

void wr(FILE* f, const void* x, size_t bytes) {
  if (bytes && fwrite(x, 1, bytes, f) != bytes) fail(PW_EINVAL, "checkpoint write failed");
}
void rd(FILE* f, void* x, size_t bytes) {
  if (bytes && fread(x, 1, bytes, f) != bytes)
    fail(PW_EINVAL, "checkpoint file truncated or unreadable");
}
void wr_dev(FILE* f, const void* d, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  std::vector<char> h(bytes);
  PW_HIP(hipMemcpyAsync(h.data(), d, bytes, hipMemcpyDeviceToHost, st));
  PW_HIP(hipStreamSynchronize(st));
  wr(f, h.data(), bytes);
}
void rd_dev(FILE* f, void* d, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  std::vector<char> h(bytes);
  rd(f, h.data(), bytes);
  PW_HIP(hipMemcpyAsync(d, h.data(), bytes, hipMemcpyHostToDevice, st));
  PW_HIP(hipStreamSynchronize(st));
}

void save_problem(FILE* f, Prob& pr, hipStream_t st) {
  double slots[kSlots];
  problem_slots(pr.P, slots);
  wr(f, slots, sizeof(slots));
  const int levels = pr.hist_u && pr.have_iterate ? pr.k_done + 1 : 0;
  const int32_t fl[16] = {pr.have_medium, pr.have_initial, pr.have_iterate, pr.variant,
                          pr.k_done, pr.r, pr.cur, pr.samp_n, pr.samp_iters,
                          (int32_t)pr.ranks.size(), (int32_t)pr.change.size(), levels,
                          pr.have_src, pr.ce_ok && pr.have_medium, 0, 0};
  wr(f, fl, sizeof(fl));
  const size_t fb = pr.tsize * pr.Nf;
  const long long rows = pr.rows, Nc = pr.Nc;
  if (pr.have_medium) wr_dev(f, pr.cf, sizeof(double) * pr.Nf, st);
  if (pr.have_initial) {
    wr_dev(f, pr.u, fb, st);
    wr_dev(f, pr.p, fb, st);
  }
  if (pr.have_iterate) {
    wr_dev(f, (char*)pr.u + fb, fb * pr.N, st);
    wr_dev(f, (char*)pr.p + fb, fb * pr.N, st);
  }
  for (int l = 0; l < levels; ++l) {
    wr_dev(f, (char*)pr.hist_u + fb * pr.N * l, fb * pr.N, st);
    wr_dev(f, (char*)pr.hist_p + fb * pr.N * l, fb * pr.N, st);
  }
  wr(f, pr.ranks.data(), sizeof(int) * pr.ranks.size());
  wr(f, pr.change.data(), sizeof(double) * pr.change.size());
  wr_dev(f, pr.res, sizeof(double) * kRes * pr.k_done, st);
  if (pr.r > 0) {
    wr_dev(f, pr.Ub[pr.cur], sizeof(double) * rows * pr.r, st);
    wr_dev(f, pr.Vb[pr.cur], sizeof(double) * rows * pr.r, st);
    wr_dev(f, pr.S, sizeof(double) * pr.r, st);
  }
  wr_dev(f, pr.E[pr.cur], sizeof(double) * 2 * Nc * (pr.r + 1), st);
  wr_dev(f, pr.Vp[pr.cur], sizeof(double) * 2 * Nc * (pr.r + 1), st);
  if (pr.samp_n > 0) wr_dev(f, pr.samp.p, sizeof(int) * (size_t)pr.samp_n * pr.samp_iters, st);
  if (pr.have_src) {
    const double sb[4] = {pr.src_pos[0], pr.src_pos[1], pr.src_freq, pr.src_t0};
    wr(f, sb, sizeof(sb));
  }
  if (fl[13]) wr_dev(f, pr.CEb[pr.cur], sizeof(double) * 2 * Nc * (pr.r + 1), st);
}

template <typename T>
void load_medium_typed(Prob& pr, hipStream_t st) {
  set_medium_typed<T>(pr, st);
}

void load_problem(FILE* f, Prob& pr, hipStream_t st) {
  double slots[kSlots], mine[kSlots];
  rd(f, slots, sizeof(slots));
  problem_slots(pr.P, mine);
  if (std::memcmp(slots, mine, sizeof(slots)) != 0)
    fail(PW_EINVAL, "checkpoint was written for a different problem description");
  int32_t fl[16];
  rd(f, fl, sizeof(fl));
  const bool have_medium = fl[0], have_initial = fl[1], have_iterate = fl[2];
  const int k_done = fl[4], r = fl[5], cur = fl[6], samp_n = fl[7], samp_iters = fl[8];
  const int n_ranks = fl[9], n_change = fl[10], levels = fl[11];
  if (fl[3] < PW_VARIANT_THETA || fl[3] > PW_VARIANT_PLAIN || k_done < 0 ||
      k_done > pr.P.max_iters || r < 0 || r > pr.rmax || (cur != 0 && cur != 1) || samp_n < 0 ||
      samp_n > pr.N || samp_iters < 0 || n_ranks < 0 || n_ranks > pr.P.max_iters ||
      n_change < 0 || n_change > pr.P.max_iters || levels < 0 ||
      levels > (pr.hist_u ? k_done + 1 : 0) || (have_iterate && !have_initial) ||
      (!have_medium && (have_iterate || r > 0 || fl[13])) || fl[13] < 0 || fl[13] > 1)
    fail(PW_EINVAL, "inconsistent checkpoint header");
  const size_t fb = pr.tsize * pr.Nf;
  const long long rows = pr.rows, Nc = pr.Nc;
  if (have_medium) {
    std::vector<double> c((size_t)pr.Nf);
    rd(f, c.data(), sizeof(double) * c.size());
    double cmax = 0.0;
    for (double x : c) {
      if (!(x > 0.0) || !std::isfinite(x)) fail(PW_EINVAL, "checkpoint medium not positive");
      cmax = std::max(cmax, x);
    }
    PW_HIP(hipMemcpyAsync(pr.cf, c.data(), sizeof(double) * c.size(), hipMemcpyHostToDevice, st));
    if (pr.f64) load_medium_typed<double>(pr, st);
    else load_medium_typed<float>(pr, st);
    PW_HIP(hipStreamSynchronize(st));
    setup_layer(pr, cmax);
  }
  if (have_initial) {
    rd_dev(f, pr.u, fb, st);
    rd_dev(f, pr.p, fb, st);
  }
  if (have_iterate) {
    rd_dev(f, (char*)pr.u + fb, fb * pr.N, st);
    rd_dev(f, (char*)pr.p + fb, fb * pr.N, st);
  }
  for (int l = 0; l < levels; ++l) {
    rd_dev(f, (char*)pr.hist_u + fb * pr.N * l, fb * pr.N, st);
    rd_dev(f, (char*)pr.hist_p + fb * pr.N * l, fb * pr.N, st);
  }
  std::vector<int> ranks((size_t)n_ranks);
  rd(f, ranks.data(), sizeof(int) * ranks.size());
  std::vector<double> change((size_t)n_change);
  rd(f, change.data(), sizeof(double) * change.size());
  rd_dev(f, pr.res, sizeof(double) * kRes * k_done, st);
  if (r > 0) {
    rd_dev(f, pr.Ub[cur], sizeof(double) * rows * r, st);
    rd_dev(f, pr.Vb[cur], sizeof(double) * rows * r, st);
    rd_dev(f, pr.S, sizeof(double) * r, st);
  }
  rd_dev(f, pr.E[cur], sizeof(double) * 2 * Nc * (r + 1), st);
  rd_dev(f, pr.Vp[cur], sizeof(double) * 2 * Nc * (r + 1), st);
  if (samp_n > 0) {
    const size_t bytes = sizeof(int) * (size_t)samp_n * samp_iters;
    std::vector<int> tab((size_t)samp_n * samp_iters);
    rd(f, tab.data(), bytes);
    for (int x : tab)
      if (x < 0 || x >= pr.N) fail(PW_EINVAL, "checkpoint sampling table out of range");
    PW_HIP(hipMemcpy(pr.samp.ensure(bytes), tab.data(), bytes, hipMemcpyHostToDevice));
  }
  if (fl[12]) {
    double sb[4];
    rd(f, sb, sizeof(sb));
    set_source(pr, sb, sb[2], sb[3]);
  } else {
    set_source(pr, nullptr, 0.0, 0.0);
  }
  if (fl[13]) rd_dev(f, pr.CEb[cur], sizeof(double) * 2 * Nc * (r + 1), st);
  pr.ce_ok = fl[13] != 0;
  pr.have_medium = have_medium;
  pr.have_initial = have_initial;
  pr.have_iterate = have_iterate;
  pr.variant = fl[3];
  pr.k_done = k_done;
  pr.r = r;
  pr.cur = cur;
  pr.samp_n = samp_n;
  pr.samp_iters = samp_n > 0 ? samp_iters : 0;
  pr.ranks = ranks;
  pr.change = change;
  ++pr.epoch;  // a recorded tape no longer matches
}

}  // namespace
}  // namespace pw

using namespace pw;

extern "C" {

const char* pw_last_error(void) { return g_last_error.c_str(); }

// the last word names the revision of the fine stencil kernel (bench.py
// keys measured HBM traffic on it)
const char* pw_version(void) { return "pwave 0.4 (gfx950) stencil-r10"; }

int pw_num_problems(const pw_ctx* ctx) { return ctx ? (int)ctx->probs.size() : 0; }

pw_status pw_create(const pw_problem* probs, int n_problems, void* stream, pw_ctx** out) {
  return guarded([&] {
    if (!probs || n_problems < 1 || !out) fail(PW_EINVAL, "bad arguments to pw_create");
    auto ctx = std::make_unique<pw_ctx>();
    ctx->stream = (hipStream_t)stream;
    for (int i = 0; i < n_problems; ++i) {
      auto pr = std::make_unique<Prob>();
      setup(*pr, probs[i]);
      ctx->probs.push_back(std::move(pr));
    }
    // The runtime spreads streams over its hardware queues in creation
    // order (round robin).  Problem i's own stream (its corrector and
    // sweep in a batch, the F branch of Algorithm 1) is created i-th and
    // its side stream (the G branch) in a second pass rotated by two, so
    // that the own streams cover every queue and a problem's two branches
    // sit on different queues (created in pairs, the own streams of all
    // problems shared half of the queues).
    for (int i = 0; i < n_problems; ++i)
      PW_HIP(hipStreamCreateWithFlags(&ctx->probs[(size_t)i]->own, hipStreamNonBlocking));
    for (int i = 0; i < n_problems; ++i)
      PW_HIP(hipStreamCreateWithFlags(&ctx->probs[(size_t)((i + 2) % n_problems)]->side,
                                      hipStreamNonBlocking));
    PW_HIP(hipDeviceSynchronize());
    *out = ctx.release();
  });
}

pw_status pw_destroy(pw_ctx* ctx) {
  return guarded([&] {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& pr : ctx->probs)
      for (int i = 0; i < 4; ++i)
        if (pr->ev[i]) (void)hipEventDestroy(pr->ev[i]);
    delete ctx;
  });
}

pw_status pw_sync(pw_ctx* ctx) {
  return guarded([&] {
    if (!ctx) fail(PW_EINVAL, "null context");
    PW_HIP(hipStreamSynchronize(ctx->stream));
  });
}

pw_status pw_set_medium(pw_ctx* ctx, int prob, const double* c, int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!c) fail(PW_EINVAL, "null medium");
    hipStream_t st = ctx->stream;
    PW_HIP(hipMemcpyAsync(pr.cf, c, sizeof(double) * pr.Nf,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    // stability: c_max * dt / dx < 1 / sqrt(d) on both grids
    std::vector<double> h(pr.Nf);
    PW_HIP(hipMemcpyAsync(h.data(), pr.cf, sizeof(double) * pr.Nf, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    double cmax = 0.0;
    for (double x : h) {
      if (!(x > 0.0) || !std::isfinite(x)) fail(PW_EINVAL, "medium must be positive and finite");
      cmax = std::max(cmax, x);
    }
    const double lim = 1.0 / std::sqrt((double)pr.gf.dim);
    if (cmax * pr.hF / pr.gf.dx >= lim || cmax * pr.hC / pr.gc.dx >= lim) {
      char buf[200];
      snprintf(buf, sizeof(buf),
               "unstable: c_max dt/dx = %.4g (fine), %.4g (coarse) >= 1/sqrt(d) = %.4g",
               cmax * pr.hF / pr.gf.dx, cmax * pr.hC / pr.gc.dx, lim);
      fail(PW_EUNSTABLE, buf);
    }
    if (pr.f64) set_medium_typed<double>(pr, st);
    else set_medium_typed<float>(pr, st);
    PW_HIP(hipStreamSynchronize(st));
    setup_layer(pr, cmax);
    pr.have_medium = true;
    ++pr.epoch;
  });
}

pw_status pw_set_source(pw_ctx* ctx, int prob, const double* pos, double freq, double t0) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    set_source(pr, pos, freq, t0);
    ++pr.epoch;
    pr.k_done = 0;
    pr.have_iterate = false;
    pr.change.clear();
    reset_corrector(pr);
  });
}

pw_status pw_set_initial(pw_ctx* ctx, int prob, const double* u0, const double* p0,
                         int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!u0 || !p0) fail(PW_EINVAL, "null initial state");
    hipStream_t st = ctx->stream;
    double* s0 = pr.itmp;
    double* s1 = pr.itmp + pr.Nf;
    const double* du = (const double*)stage_in(u0, pr.Nf, on_device, pr, s0, st);
    const double* dp = (const double*)stage_in(p0, pr.Nf, on_device, pr, s1, st);
    if (pr.f64) set_initial_typed<double>(pr, du, dp, st);
    else set_initial_typed<float>(pr, du, dp, st);
    PW_HIP(hipStreamSynchronize(st));
    pr.have_initial = true;
    ++pr.epoch;
    pr.k_done = 0;
    pr.have_iterate = false;
    pr.change.clear();
    reset_corrector(pr);
  });
}

pw_status pw_run(pw_ctx* ctx, int prob, int K, double stop_tol, int* k_done) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium || !pr.have_initial) fail(PW_ESTATE, "set medium and initial state first");
    if (K < 0 || K > pr.P.max_iters) fail(PW_EINVAL, "K must be in [0, max_iters]");
    if (!(stop_tol >= 0)) fail(PW_EINVAL, "stop_tol must be >= 0");
    check_sampling(pr, K);
    if (pr.have_src && pr.variant == PW_VARIANT_NO_CORRECTION)
      fail(PW_EINVAL, "the comparator without correction propagates states, not differences: "
                      "it does not take a source");
    if (pr.f64) run_typed<double>(pr, K, stop_tol, ctx->stream);
    else run_typed<float>(pr, K, stop_tol, ctx->stream);
    if (k_done) *k_done = pr.k_done;
  });
}

pw_status pw_continue(pw_ctx* ctx, int prob, int K, int update_corrector, double stop_tol,
                      int* k_done) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium || !pr.have_iterate)
      fail(PW_ESTATE, "pw_continue needs an iterate (pw_run, pw_run_batch or pw_load first)");
    if (K < 0 || pr.k_done + K > pr.P.max_iters)
      fail(PW_EINVAL, "k_done + K must not exceed max_iters");
    if (!(stop_tol >= 0)) fail(PW_EINVAL, "stop_tol must be >= 0");
    if (update_corrector) check_sampling(pr, pr.k_done + K);
    if (pr.have_src && pr.variant == PW_VARIANT_NO_CORRECTION)
      fail(PW_EINVAL, "the comparator without correction does not take a source");
    if (pr.f64) continue_typed<double>(pr, K, update_corrector != 0, stop_tol, ctx->stream);
    else continue_typed<float>(pr, K, update_corrector != 0, stop_tol, ctx->stream);
    if (k_done) *k_done = pr.k_done;
  });
}

pw_status pw_set_sampling(pw_ctx* ctx, int prob, const int* cols, int n_per_iter,
                          int n_iters) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (n_per_iter < 0 || n_per_iter > pr.N || n_iters < 0)
      fail(PW_EINVAL, "sample size must be in [0, N] and the iteration count >= 0");
    if (n_per_iter > 0 && (n_iters == 0 || !cols)) fail(PW_EINVAL, "empty column table");
    if (n_per_iter > 0 && pr.sk_l > 0)
      fail(PW_EINVAL, "sketching and column sampling are exclusive");
    std::vector<char> seen((size_t)pr.N);
    for (int k = 0; k < (n_per_iter > 0 ? n_iters : 0); ++k) {
      std::fill(seen.begin(), seen.end(), 0);
      for (int j = 0; j < n_per_iter; ++j) {
        const int c = cols[(long long)k * n_per_iter + j];
        if (c < 0 || c >= pr.N) fail(PW_EINVAL, "sample column outside [0, N)");
        if (seen[(size_t)c]) fail(PW_EINVAL, "repeated sample column in one iteration");
        seen[(size_t)c] = 1;
      }
    }
    if (n_per_iter > 0) {
      const size_t bytes = sizeof(int) * (size_t)n_per_iter * (size_t)n_iters;
      PW_HIP(hipStreamSynchronize(ctx->stream));
      PW_HIP(hipMemcpy(pr.samp.ensure(bytes), cols, bytes, hipMemcpyHostToDevice));
    }
    pr.samp_n = n_per_iter;
    pr.samp_iters = n_per_iter > 0 ? n_iters : 0;
    pr.k_done = 0;
    pr.have_iterate = false;
    pr.change.clear();
    reset_corrector(pr);
  });
}

pw_status pw_set_sketch(pw_ctx* ctx, int prob, const double* omega, int l, int n_iters,
                        int power) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (l < 0 || l > pr.N || n_iters < 0 || power < 0 || power > 8)
      fail(PW_EINVAL, "sketch width must be in [0, N], power in [0, 8]");
    if (l > 0 && (n_iters == 0 || !omega)) fail(PW_EINVAL, "empty sketch table");
    if (l > 0 && pr.samp_n > 0) fail(PW_EINVAL, "sketching and column sampling are exclusive");
    if (l > 0) {
      const size_t n = (size_t)n_iters * pr.N * l;
      for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(omega[i])) fail(PW_EINVAL, "non-finite sketch entry");
      PW_HIP(hipStreamSynchronize(ctx->stream));
      PW_HIP(hipMemcpy(pr.sk.ensure(sizeof(double) * n), omega, sizeof(double) * n,
                       hipMemcpyHostToDevice));
      const size_t yb = sizeof(double) * (size_t)pr.rows * l;
      const size_t zb = sizeof(double) * (size_t)pr.N * l;
      pr.skYf.ensure(yb);
      pr.skYg.ensure(yb);
      pr.skZf.ensure(zb);
      pr.skZg.ensure(zb);
    }
    pr.sk_l = l;
    pr.sk_iters = l > 0 ? n_iters : 0;
    pr.sk_power = l > 0 ? power : 0;
    pr.k_done = 0;
    pr.have_iterate = false;
    pr.change.clear();
    reset_corrector(pr);
  });
}

pw_status pw_set_variant(pw_ctx* ctx, int prob, int variant) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (variant < PW_VARIANT_THETA || variant > PW_VARIANT_PLAIN)
      fail(PW_EINVAL, "unknown variant");
    pr.variant = variant;
    pr.k_done = 0;
    pr.have_iterate = false;
    pr.change.clear();
    reset_corrector(pr);
  });
}

pw_status pw_get_state(pw_ctx* ctx, int prob, int n, void* u, void* p, int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (n < 0 || n > pr.N) fail(PW_EINVAL, "slice index out of range");
    if (!u || !p) fail(PW_EINVAL, "null output");
    const size_t bytes = pr.tsize * pr.Nf;
    const char* su = (const char*)pr.u + bytes * n;
    const char* sp = (const char*)pr.p + bytes * n;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    PW_HIP(hipMemcpyAsync(u, su, bytes, kind, ctx->stream));
    PW_HIP(hipMemcpyAsync(p, sp, bytes, kind, ctx->stream));
    if (!on_device) PW_HIP(hipStreamSynchronize(ctx->stream));
  });
}

pw_status pw_get_iterate(pw_ctx* ctx, int prob, int k, int n, void* u, void* p, int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_iterate) fail(PW_ESTATE, "no iterate: run first");
    if (k < 1 || k > pr.k_done + 1) fail(PW_EINVAL, "k must be in [1, k_done + 1]");
    if (n < 0 || n > pr.N) fail(PW_EINVAL, "slice index out of range");
    if (!u || !p) fail(PW_EINVAL, "null output");
    const size_t fb = pr.tsize * pr.Nf;
    const char *su, *sp;
    if (n == 0 || k == pr.k_done + 1) {
      su = (const char*)pr.u + fb * n;
      sp = (const char*)pr.p + fb * n;
    } else {
      if (!pr.hist_u) fail(PW_EINVAL, "earlier iterates need keep_history = 1");
      const size_t lvl = fb * pr.N * (size_t)(k - 1);
      su = (const char*)pr.hist_u + lvl + fb * (n - 1);
      sp = (const char*)pr.hist_p + lvl + fb * (n - 1);
    }
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    PW_HIP(hipMemcpyAsync(u, su, fb, kind, ctx->stream));
    PW_HIP(hipMemcpyAsync(p, sp, fb, kind, ctx->stream));
    if (!on_device) PW_HIP(hipStreamSynchronize(ctx->stream));
  });
}

pw_status pw_set_iterate(pw_ctx* ctx, int prob, int n, const double* u, const double* p,
                         int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_iterate) fail(PW_ESTATE, "no iterate to overwrite: run first");
    if (n < 1 || n > pr.N) fail(PW_EINVAL, "n must be in [1, N] (slice 0 is u0)");
    if (!u || !p) fail(PW_EINVAL, "null input");
    hipStream_t st = ctx->stream;
    const long long Nf = pr.Nf;
    const double* du = (const double*)stage_in(u, Nf, on_device, pr, pr.itmp, st);
    const double* dp = (const double*)stage_in(p, Nf, on_device, pr, pr.itmp + Nf, st);
    const size_t fb = pr.tsize * Nf;
    if (pr.f64) {
      cast_from_double<double>(du, (double*)((char*)pr.u + fb * n), Nf, st);
      cast_from_double<double>(dp, (double*)((char*)pr.p + fb * n), Nf, st);
    } else {
      cast_from_double<float>(du, (float*)((char*)pr.u + fb * n), Nf, st);
      cast_from_double<float>(dp, (float*)((char*)pr.p + fb * n), Nf, st);
    }
    if (pr.hist_u) {
      // the current iterate's history level follows it
      const size_t lvl = fb * pr.N * (size_t)pr.k_done + fb * (n - 1);
      PW_HIP(hipMemcpyAsync((char*)pr.hist_u + lvl, (char*)pr.u + fb * n, fb,
                            hipMemcpyDeviceToDevice, st));
      PW_HIP(hipMemcpyAsync((char*)pr.hist_p + lvl, (char*)pr.p + fb * n, fb,
                            hipMemcpyDeviceToDevice, st));
    }
    PW_HIP(hipStreamSynchronize(st));
  });
}

pw_status pw_set_corrector(pw_ctx* ctx, int prob, const double* U, const double* S,
                           const double* V, int rank, int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium) fail(PW_ESTATE, "set the medium first");
    if (rank < 0 || rank > pr.rmax) fail(PW_EINVAL, "rank must be in [0, min(max_iters N, rows)]");
    if (rank > 0 && (!U || !S || !V)) fail(PW_EINVAL, "null corrector input");
    hipStream_t st = ctx->stream;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const size_t vb = sizeof(double) * (size_t)pr.rows * rank;
    if (rank > 0) {
      PW_HIP(hipMemcpyAsync(pr.Ub[pr.cur], U, vb, kind, st));
      PW_HIP(hipMemcpyAsync(pr.Vb[pr.cur], V, vb, kind, st));
      PW_HIP(hipMemcpyAsync(pr.S, S, sizeof(double) * rank, kind, st));
    }
    pr.r = rank;
    rebuild_sweep_columns(pr, st);
    PW_HIP(hipStreamSynchronize(st));
  });
}

pw_status pw_get_diagnostics(pw_ctx* ctx, int prob, double* out, int cap, int* count) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    const int K = pr.k_done;
    std::vector<double> h((size_t)kRes * std::max(K, 1));
    if (K > 0) {
      PW_HIP(hipMemcpyAsync(h.data(), pr.res, sizeof(double) * kRes * K, hipMemcpyDeviceToHost,
                            ctx->stream));
      PW_HIP(hipStreamSynchronize(ctx->stream));
    }
    double in2 = 0.0;  // sum over iterations of ||F_in||^2 + ||G_in||^2
    for (int k = 0; k < K; ++k) {
      const double* r = h.data() + (size_t)kRes * k;
      in2 += r[2] + r[3];
      if (k >= cap) continue;
      double* o = out + (size_t)kPwDiag * k;
      o[0] = r[1] > 0 ? std::sqrt(r[0] / r[1]) : (std::isnan(r[0]) ? r[0] : 0.0);
      o[1] = k < (int)pr.ranks.size() ? pr.ranks[(size_t)k] : 0;
      o[2] = r[1];
      o[3] = r[2];
      o[4] = r[3];
      o[5] = r[4];
      o[6] = in2 - 2.0 * r[4];
      o[7] = k < (int)pr.change.size() ? pr.change[(size_t)k] : std::nan("");
    }
    if (count) *count = K;
  });
}

pw_status pw_launch_plan(pw_ctx* ctx, int prob, int grid, int n_states, int* launches,
                         int* steps_per_launch) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (grid != PW_FINE && grid != PW_COARSE) fail(PW_EINVAL, "bad grid");
    if (n_states < 1) fail(PW_EINVAL, "n_states must be >= 1");
    int l = 0, b = 0;
    if (grid == PW_FINE) launch_plan(pr.gf, pr.f64, n_states, pr.mF, &l, &b);
    else launch_plan(pr.gc, pr.f64, n_states, pr.mC, &l, &b);
    if (launches) *launches = l;
    if (steps_per_launch) *steps_per_launch = b;
  });
}

pw_status pw_get_tape_id(pw_ctx* ctx, int prob, long long* id) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!id) fail(PW_EINVAL, "null output");
    *id = pr.tape_serial;
  });
}

pw_status pw_get_residuals(pw_ctx* ctx, int prob, double* rho, int* rank, int cap, int* count) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    const int K = pr.k_done;
    std::vector<double> h((size_t)kRes * std::max(K, 1));
    if (K > 0) {
      PW_HIP(hipMemcpyAsync(h.data(), pr.res, sizeof(double) * kRes * K, hipMemcpyDeviceToHost,
                            ctx->stream));
      PW_HIP(hipStreamSynchronize(ctx->stream));
    }
    for (int k = 0; k < K && k < cap; ++k) {
      const double* rr = h.data() + (size_t)kRes * k;
      if (rho) rho[k] = rr[1] > 0 ? std::sqrt(rr[0] / rr[1]) : (std::isnan(rr[0]) ? rr[0] : 0.0);
      if (rank) rank[k] = k < (int)pr.ranks.size() ? pr.ranks[k] : 0;
    }
    if (count) *count = K;
  });
}

pw_status pw_serial_fine(pw_ctx* ctx, int prob, int n, void* u, void* p) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium || !pr.have_initial) fail(PW_ESTATE, "set medium and initial state first");
    if (n < 0 || n > pr.N) fail(PW_EINVAL, "n out of range");
    if (!u || !p) fail(PW_EINVAL, "null output");
    if (pr.f64) serial_fine_typed<double>(pr, n, (double*)u, (double*)p, ctx->stream);
    else serial_fine_typed<float>(pr, n, (float*)u, (float*)p, ctx->stream);
  });
}

pw_status pw_serial_fine_states(pw_ctx* ctx, int prob, void* u, void* p) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium || !pr.have_initial) fail(PW_ESTATE, "set medium and initial state first");
    if (!u || !p) fail(PW_EINVAL, "null output");
    hipStream_t st = ctx->stream;
    const size_t fb = pr.tsize * pr.Nf;
    PW_HIP(hipMemcpyAsync(u, pr.u, fb, hipMemcpyDeviceToDevice, st));
    PW_HIP(hipMemcpyAsync(p, pr.p, fb, hipMemcpyDeviceToDevice, st));
    for (int n = 1; n <= pr.N; ++n) {
      char* uo = (char*)u + fb * n;
      char* po = (char*)p + fb * n;
      if (pr.f64)
        prop_fine<double>(pr, (const double*)(uo - fb), (const double*)(po - fb), (double*)uo,
                          (double*)po, 1, st, n);
      else
        prop_fine<float>(pr, (const float*)(uo - fb), (const float*)(po - fb), (float*)uo,
                         (float*)po, 1, st, n);
    }
  });
}

pw_status pw_propagate(pw_ctx* ctx, int prob, int grid, const void* u_in, const void* p_in,
                       void* u_out, void* p_out, int n_states) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium) fail(PW_ESTATE, "set the medium first");
    if (!u_in || !p_in || !u_out || !p_out || n_states < 0) fail(PW_EINVAL, "bad arguments");
    if (grid == PW_FINE) {
      if (pr.f64)
        prop_fine<double>(pr, (const double*)u_in, (const double*)p_in, (double*)u_out,
                          (double*)p_out, n_states, ctx->stream);
      else
        prop_fine<float>(pr, (const float*)u_in, (const float*)p_in, (float*)u_out,
                         (float*)p_out, n_states, ctx->stream);
    } else if (grid == PW_COARSE) {
      if (pr.f64)
        prop_coarse<double>(pr, (const double*)u_in, (const double*)p_in, (double*)u_out,
                            (double*)p_out, n_states, ctx->stream);
      else
        prop_coarse<float>(pr, (const float*)u_in, (const float*)p_in, (float*)u_out,
                           (float*)p_out, n_states, ctx->stream);
    } else {
      fail(PW_EINVAL, "grid must be PW_FINE or PW_COARSE");
    }
  });
}

pw_status pw_energy_components(pw_ctx* ctx, int prob, int grid, const void* u, const void* p,
                               double* out, int n_states) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium) fail(PW_ESTATE, "set the medium first");
    if (!u || !p || !out || n_states < 0) fail(PW_EINVAL, "bad arguments");
    if (grid != PW_FINE && grid != PW_COARSE) fail(PW_EINVAL, "bad grid");
    const Grid& src = grid == PW_FINE ? pr.gf : pr.gc;
    const int ratio = grid == PW_FINE ? pr.ratio : 1;
    const long long ss = src.npts();
    if (pr.f64)
      energy_columns<double>(src, ratio, pr.gc, (const double*)u, (const double*)p, ss, pr.cc,
                             pr.order, out, pr.rows, n_states, ctx->stream, &pr.spec);
    else
      energy_columns<float>(src, ratio, pr.gc, (const float*)u, (const float*)p, ss, pr.cc,
                            pr.order, out, pr.rows, n_states, ctx->stream, &pr.spec);
  });
}

pw_status pw_interp_add(pw_ctx* ctx, int prob, const double* du, const double* dp, const void* v,
                        const void* vp, void* u_out, void* p_out, int n_states) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!du || !dp || !u_out || !p_out || n_states < 0 || n_states > pr.N)
      fail(PW_EINVAL, "bad arguments (n_states must be <= n_slices)");
    hipStream_t st = ctx->stream;
    const long long Nc = pr.Nc, Nf = pr.Nf;
    if (pr.f64) {
      cast_from_double<double>(du, tp<double>(pr.du_T), Nc * n_states, st);
      cast_from_double<double>(dp, tp<double>(pr.dp_T), Nc * n_states, st);
      interp_add<double>(pr.gf, pr.gc, pr.ratio, pr.itab, tp<double>(pr.du_T), Nc,
                         (const double*)v, (double*)u_out, Nf, n_states, pr.itmp, st);
      interp_add<double>(pr.gf, pr.gc, pr.ratio, pr.itab, tp<double>(pr.dp_T), Nc,
                         (const double*)vp, (double*)p_out, Nf, n_states, pr.itmp, st);
    } else {
      cast_from_double<float>(du, tp<float>(pr.du_T), Nc * n_states, st);
      cast_from_double<float>(dp, tp<float>(pr.dp_T), Nc * n_states, st);
      interp_add<float>(pr.gf, pr.gc, pr.ratio, pr.itab, tp<float>(pr.du_T), Nc, (const float*)v,
                        (float*)u_out, Nf, n_states, pr.itmp, st);
      interp_add<float>(pr.gf, pr.gc, pr.ratio, pr.itab, tp<float>(pr.dp_T), Nc,
                        (const float*)vp, (float*)p_out, Nf, n_states, pr.itmp, st);
    }
  });
}

pw_status pw_grad2func(pw_ctx* ctx, int prob, const double* q, const double* sums, double* w,
                       int n_states) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!q || !w || n_states < 0 || n_states > pr.N)
      fail(PW_EINVAL, "bad arguments (n_states must be <= n_slices)");
    grad2func_cols(pr.gc, pr.dtab, q, (long long)pr.gc.dim * pr.Nc, sums, w, pr.Nc, n_states,
                   pr.ctmp, ctx->stream);
  });
}

pw_status pw_update_svd(pw_ctx* ctx, int prob, const double* F, const double* G, int n_cols,
                        int reset, int* rank) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!F || !G || n_cols < 1 || n_cols > pr.N) fail(PW_EINVAL, "bad arguments");
    if (!pr.have_medium) fail(PW_ESTATE, "set the medium first");
    if (reset) reset_corrector(pr);
    update_svd_dev(pr, F, G, n_cols, ctx->stream);
    if (rank) *rank = pr.r;
  });
}

pw_status pw_get_corrector(pw_ctx* ctx, int prob, double* U, double* S, double* V, int cap,
                           int* rank) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    const int r = pr.r;
    if (rank) *rank = r;
    if (!U && !S && !V) return;  // rank query
    if (r > cap) fail(PW_EINVAL, "output capacity smaller than the rank");
    hipStream_t st = ctx->stream;
    if (r > 0) {
      if (U)
        PW_HIP(hipMemcpyAsync(U, pr.Ub[pr.cur], sizeof(double) * pr.rows * r,
                              hipMemcpyDeviceToDevice, st));
      if (V)
        PW_HIP(hipMemcpyAsync(V, pr.Vb[pr.cur], sizeof(double) * pr.rows * r,
                              hipMemcpyDeviceToDevice, st));
      if (S) PW_HIP(hipMemcpyAsync(S, pr.S, sizeof(double) * r, hipMemcpyDeviceToDevice, st));
    }
    PW_HIP(hipStreamSynchronize(st));
  });
}

// energy and l2 sums of [u - u_ref, p - p_ref] and [u_ref, p_ref] on the
// fine grid (host output h[0..3], see energy_pair)
void energy_sums(pw_ctx* ctx, Prob& pr, const void* u, const void* p, const void* u_ref,
                 const void* p_ref, double* h) {
  if (!pr.have_medium) fail(PW_ESTATE, "set the medium first");
  if (!u || !p || (u_ref && !p_ref)) fail(PW_EINVAL, "bad arguments");
  hipStream_t st = ctx->stream;
  double* res = pr.red + kEnergyPartials;
  const int order = pr.order ? pr.order : 4;
  if (pr.f64)
    energy_pair<double>(pr.gf, (const double*)u, (const double*)p, (const double*)u_ref,
                        (const double*)p_ref, pr.cf, order, pr.red, res, st);
  else
    energy_pair<float>(pr.gf, (const float*)u, (const float*)p, (const float*)u_ref,
                       (const float*)p_ref, pr.cf, order, pr.red, res, st);
  PW_HIP(hipMemcpyAsync(h, res, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  PW_HIP(hipStreamSynchronize(st));
}

pw_status pw_energy(pw_ctx* ctx, int prob, const void* u, const void* p, const void* u_ref,
                    const void* p_ref, double* e_diff, double* e_ref) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    double h[4] = {0, 0, 0, 0};
    energy_sums(ctx, pr, u, p, u_ref, p_ref, h);
    if (e_diff) *e_diff = h[0];
    if (e_ref) *e_ref = h[1];
  });
}

pw_status pw_error_norms(pw_ctx* ctx, int prob, const void* u, const void* p, const void* u_ref,
                         const void* p_ref, double* out) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!out) fail(PW_EINVAL, "null output");
    energy_sums(ctx, pr, u, p, u_ref, p_ref, out);
  });
}

pw_status pw_save(pw_ctx* ctx, const char* path) {
  return guarded([&] {
    if (!ctx) fail(PW_EINVAL, "null context");
    if (!path) fail(PW_EINVAL, "null path");
    File fh;
    fh.f = fopen(path, "wb");
    if (!fh.f) fail(PW_EINVAL, std::string("cannot open checkpoint for writing: ") + path);
    wr(fh.f, kCkptMagic, 8);
    const int32_t np = (int32_t)ctx->probs.size();
    wr(fh.f, &np, sizeof(np));
    PW_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& up : ctx->probs) save_problem(fh.f, *up, ctx->stream);
    if (fclose(fh.f) != 0) {
      fh.f = nullptr;
      fail(PW_EINVAL, "checkpoint write failed");
    }
    fh.f = nullptr;
  });
}

pw_status pw_load(pw_ctx* ctx, const char* path) {
  return guarded([&] {
    if (!ctx) fail(PW_EINVAL, "null context");
    if (!path) fail(PW_EINVAL, "null path");
    File fh;
    fh.f = fopen(path, "rb");
    if (!fh.f) fail(PW_EINVAL, std::string("cannot open checkpoint: ") + path);
    char magic[8];
    rd(fh.f, magic, 8);
    if (std::memcmp(magic, kCkptMagic, 8) != 0) fail(PW_EINVAL, "not a pwave checkpoint");
    int32_t np = 0;
    rd(fh.f, &np, sizeof(np));
    if (np != (int32_t)ctx->probs.size())
      fail(PW_EINVAL, "checkpoint holds a different number of problems");
    PW_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& up : ctx->probs) load_problem(fh.f, *up, ctx->stream);
    char extra;
    if (fread(&extra, 1, 1, fh.f) != 0) fail(PW_EINVAL, "trailing bytes in checkpoint");
  });
}

pw_status pw_run_batch(pw_ctx* ctx, int K) {
  return guarded([&] {
    if (!ctx) fail(PW_EINVAL, "null context");
    const Prob& p0 = *ctx->probs[0];
    for (auto& up : ctx->probs) {
      const Prob& pr = *up;
      if (!pr.have_medium || !pr.have_initial)
        fail(PW_ESTATE, "set medium and initial state of every problem first");
      if (pr.gf.dim != 2) fail(PW_EINVAL, "batched runs need 2D problems");
      if (forced(pr)) fail(PW_EINVAL, "batched runs take periodic problems without a source");
      if (pr.variant != PW_VARIANT_THETA)
        fail(PW_EINVAL, "batched runs execute Algorithm 3 only (a problem has a variant set)");
      if (pr.f64 != p0.f64 || pr.comp != p0.comp)
        fail(PW_EINVAL, "all problems of a batch need the same state dtype and compensation");
      if (K < 0 || K > pr.P.max_iters) fail(PW_EINVAL, "K must be in [0, max_iters]");
      check_sampling(pr, K);
    }
    if (!ctx->batch) {
      ctx->batch = std::make_unique<Batch>();
      ctx->batch->f64 = p0.f64;
      ctx->batch->comp = p0.comp;
    }
    if (p0.f64) run_batch_typed<double>(ctx, K);
    else run_batch_typed<float>(ctx, K);
  });
}

pw_status pw_batch_fine_sweeps(pw_ctx* ctx, int reps, double* ms) {
  return guarded([&] {
    if (!ctx) fail(PW_EINVAL, "null context");
    if (!ctx->batch || !ctx->batch->built) fail(PW_ESTATE, "no batched run yet");
    if (reps < 1) fail(PW_EINVAL, "reps must be >= 1");
    Batch& b = *ctx->batch;
    hipStream_t st = ctx->stream;
    hipEvent_t e0, e1;
    PW_HIP(hipEventCreate(&e0));
    PW_HIP(hipEventCreate(&e1));
    PW_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) {
      if (b.f64) run_multi<double>(b.F64, (const StreamDesc<double>*)b.dF, b.comp, st);
      else run_multi<float>(b.F32, (const StreamDesc<float>*)b.dF, b.comp, st);
    }
    PW_HIP(hipEventRecord(e1, st));
    PW_HIP(hipEventSynchronize(e1));
    float t = 0;
    PW_HIP(hipEventElapsedTime(&t, e0, e1));
    if (ms) *ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

pw_status pw_get_batch_info(pw_ctx* ctx, int* depth, int* rows_per_stream, double* ms,
                            int cap) {
  return guarded([&] {
    if (!ctx) fail(PW_EINVAL, "null context");
    if (!ctx->batch || !ctx->batch->built) fail(PW_ESTATE, "no batched run yet");
    const Batch& b = *ctx->batch;
    if (depth) *depth = b.B;
    if (rows_per_stream) *rows_per_stream = b.Ly;
    std::vector<double> v = {b.ms[0], b.ms[1], b.ms[2], b.ms[3], b.tune_ms, b.best_ms,
                             b.from_cache ? 1.0 : 0.0, (double)b.ly_by_size.size()};
    for (auto& e : b.ly_by_size) {
      v.push_back((double)e.first);
      v.push_back((double)e.second);
    }
    for (int i = 0; i < (int)v.size() && i < cap; ++i) ms[i] = v[i];
  });
}

pw_status pw_get_timings(pw_ctx* ctx, int prob, double* ms, int cap) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    for (int i = 0; i < 4 && i < cap; ++i) ms[i] = pr.ms[i];
    for (int i = 0; i < 2 && i + 4 < cap; ++i) ms[i + 4] = pr.adj_ms[i];
  });
}

// ---- adjoint ---------------------------------------------------------------
pw_status pw_run_taped(pw_ctx* ctx, int prob, int K) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium || !pr.have_initial) fail(PW_ESTATE, "set medium and initial state first");
    if (pr.variant != PW_VARIANT_THETA)
      fail(PW_EINVAL, "taped runs differentiate Algorithm 3 only (a variant is set)");
    if (pr.P.interp != PW_INTERP_TRIG)
      fail(PW_EINVAL, "taped runs support the trigonometric interpolation only");
    if (K < 0 || K > pr.P.max_iters) fail(PW_EINVAL, "K must be in [0, max_iters]");
    check_sampling(pr, K);
    ensure_tape(pr, K);
    if (pr.f64) run_taped_typed<double>(pr, K, false, ctx->stream);
    else run_taped_typed<float>(pr, K, false, ctx->stream);
  });
}

pw_status pw_run_frozen(pw_ctx* ctx, int prob, int K) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    if (!pr.have_medium || !pr.have_initial) fail(PW_ESTATE, "set medium and initial state first");
    if (pr.variant != PW_VARIANT_THETA)
      fail(PW_EINVAL, "taped runs differentiate Algorithm 3 only (a variant is set)");
    if (!pr.tape || K < 0 || K > pr.tape->Kc)
      fail(PW_ESTATE, "run_frozen needs correctors recorded by pw_run_taped for K iterations");
    if (pr.f64) run_taped_typed<double>(pr, K, true, ctx->stream);
    else run_taped_typed<float>(pr, K, true, ctx->stream);
  });
}

// receivers: checked on the host (copied there first when on the device)
const long long* stage_receivers(Prob& pr, const long long* rec, int nrec, int on_device,
                                 hipStream_t st) {
  if (nrec < 0) fail(PW_EINVAL, "negative receiver count");
  if (nrec == 0) return nullptr;
  if (!rec) fail(PW_EINVAL, "null receivers");
  std::vector<long long> h((size_t)nrec);
  if (on_device) {
    PW_HIP(hipMemcpyAsync(h.data(), rec, sizeof(long long) * nrec, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
  } else {
    std::memcpy(h.data(), rec, sizeof(long long) * nrec);
  }
  for (long long x : h)
    if (x < 0 || x >= pr.Nf) fail(PW_EINVAL, "receiver index outside the fine grid");
  if (on_device) return rec;
  long long* d = (long long*)pr.stage_rec.ensure(sizeof(long long) * nrec);
  PW_HIP(hipMemcpyAsync(d, h.data(), sizeof(long long) * nrec, hipMemcpyHostToDevice, st));
  PW_HIP(hipStreamSynchronize(st));
  return d;
}

}  // extern "C"

namespace {

// receiver tables of a record (pw_trace_sweep, pw_backward_sweep): the
// receivers are checked on the host (inside the grid, distinct), the
// per-row flags and per-node indices uploaded; returns the device list
const long long* record_tables(Prob& pr, const long long* rec, int nrec, int on_device,
                               hipStream_t st) {
  if (pr.gf.dim != 2) fail(PW_EINVAL, "receiver records are implemented for 2D problems only");
  const long long* d = stage_receivers(pr, rec, nrec, on_device, st);
  if (nrec == 0) return d;
  std::vector<long long> h((size_t)nrec);
  if (on_device) {
    PW_HIP(hipMemcpyAsync(h.data(), rec, sizeof(long long) * nrec, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
  } else {
    std::memcpy(h.data(), rec, sizeof(long long) * nrec);
  }
  std::vector<int> map((size_t)pr.Nf, -1), rows((size_t)pr.gf.n[1], 0);
  for (int r = 0; r < nrec; ++r) {
    const long long x = h[(size_t)r];
    if (map[(size_t)x] >= 0) fail(PW_EINVAL, "receivers of a record must be distinct nodes");
    map[(size_t)x] = r;
    rows[(size_t)(x / pr.gf.n[0])] = 1;
  }
  PW_HIP(hipMemcpyAsync(pr.rec_map.ensure(sizeof(int) * map.size()), map.data(),
                        sizeof(int) * map.size(), hipMemcpyHostToDevice, st));
  PW_HIP(hipMemcpyAsync(pr.rec_rows.ensure(sizeof(int) * rows.size()), rows.data(),
                        sizeof(int) * rows.size(), hipMemcpyHostToDevice, st));
  PW_HIP(hipStreamSynchronize(st));
  return d;
}

template <typename T>
void trace_sweep_typed(Prob& pr, const long long* rec, int nrec, double* out, hipStream_t st) {
  Force<T> fo = make_force<T>(pr, true, true, 1, true, true);
  fo.rec = rec;
  fo.rec_rows = (const int*)pr.rec_rows.p;
  fo.rec_map = (const int*)pr.rec_map.p;
  fo.n_rec = nrec;
  fo.m_tr = pr.mF;
  fo.traces = out;
  const size_t bytes = pr.tsize * pr.Nf * pr.N;
  T* uo = (T*)pr.trace_u.ensure(bytes);
  T* po = (T*)pr.trace_p.ensure(bytes);
  propagate<T>(pr.gf, tp<T>(pr.c2f), tp<T>(pr.u), tp<T>(pr.p), uo, po, pr.Nf, pr.N, pr.mF,
               (T)pr.hF, pr.comp, fine_work<T>(pr, 0), fine_work<T>(pr, 1), st, true, &fo);
}

// shared by pw_backward (record at the coupling times) and
// pw_backward_sweep (record of every fine step)
void backward_common(pw_ctx* ctx, int prob, const long long* receivers, int n_rec,
                     const double* seed, double* grad, int on_device, int wrt_velocity,
                     int checkpoint_every, bool sweep) {
  Prob& pr = get_prob(ctx, prob);
  hipStream_t st = ctx->stream;
  if (!pr.tape || pr.tape->epoch < 0)
    fail(PW_ESTATE, "pw_backward needs a run by pw_run_taped or pw_run_frozen");
  if (pr.tape->epoch != pr.epoch)
    fail(PW_ESTATE, "medium or initial state changed since the taped run");
  if (!grad) fail(PW_EINVAL, "null gradient output");
  const int ckpt = checkpoint_every > 0 ? checkpoint_every : 64;
  const long long* rec = sweep ? record_tables(pr, receivers, n_rec, on_device, st)
                               : stage_receivers(pr, receivers, n_rec, on_device, st);
  const long long ns = (long long)pr.N * n_rec * (sweep ? pr.mF : 1);
  const double* sd = nullptr;
  if (n_rec > 0) {
    if (!seed) fail(PW_EINVAL, "null seed");
    sd = (const double*)stage_in(seed, ns, on_device, pr,
                                 (double*)pr.stage_seed.ensure(sizeof(double) * ns), st);
  }
  ensure_backward(pr, ckpt);
  const int* rows = sweep && n_rec > 0 ? (const int*)pr.rec_rows.p : nullptr;
  const int* map = sweep && n_rec > 0 ? (const int*)pr.rec_map.p : nullptr;
  if (sweep && n_rec == 0) rec = nullptr;
  if (pr.f64) backward_typed<double>(pr, rec, n_rec, sd, ckpt, st, rows, map);
  else backward_typed<float>(pr, rec, n_rec, sd, ckpt, st, rows, map);
  Tape& t = *pr.tape;
  double* g = t.grad;
  if (wrt_velocity) {
    // d J / d c = 2 c d J / d c^2
    mul_fields(pr.cf, t.grad, t.Wf, pr.Nf, 2.0, st);
    g = t.Wf;
  }
  PW_HIP(hipMemcpyAsync(grad, g, sizeof(double) * pr.Nf,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  PW_HIP(hipStreamSynchronize(st));
}

}  // namespace

extern "C" {

pw_status pw_trace_sweep(pw_ctx* ctx, int prob, const long long* receivers, int n_rec,
                         double* out, int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    hipStream_t st = ctx->stream;
    if (!pr.have_medium) fail(PW_ESTATE, "set the medium first");
    if (!pr.have_iterate && !(pr.tape && pr.tape->epoch == pr.epoch))
      fail(PW_ESTATE, "pw_trace_sweep needs an iterate (a run first)");
    const long long* rec = record_tables(pr, receivers, n_rec, on_device, st);
    if (n_rec == 0) return;
    if (!out) fail(PW_EINVAL, "null output");
    const long long n = (long long)pr.N * pr.mF * n_rec;
    double* dst = on_device ? out : (double*)pr.stage_out.ensure(sizeof(double) * n);
    if (pr.f64) trace_sweep_typed<double>(pr, rec, n_rec, dst, st);
    else trace_sweep_typed<float>(pr, rec, n_rec, dst, st);
    if (!on_device)
      PW_HIP(hipMemcpyAsync(out, dst, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
  });
}

pw_status pw_traces(pw_ctx* ctx, int prob, const long long* receivers, int n_rec, double* out,
                    int on_device) {
  return guarded([&] {
    Prob& pr = get_prob(ctx, prob);
    hipStream_t st = ctx->stream;
    const long long* rec = stage_receivers(pr, receivers, n_rec, on_device, st);
    if (n_rec == 0) return;
    if (!out) fail(PW_EINVAL, "null output");
    const long long n = (long long)pr.N * n_rec;
    double* dst = on_device ? out : (double*)pr.stage_out.ensure(sizeof(double) * n);
    const size_t off = pr.tsize * pr.Nf;  // fields n = 1..N
    if (pr.f64)
      receiver_values<double>((const double*)((const char*)pr.u + off), pr.Nf, rec, n_rec, pr.N,
                              dst, st);
    else
      receiver_values<float>((const float*)((const char*)pr.u + off), pr.Nf, rec, n_rec, pr.N,
                             dst, st);
    if (!on_device) {
      PW_HIP(hipMemcpyAsync(out, dst, sizeof(double) * n, hipMemcpyDeviceToHost, st));
      PW_HIP(hipStreamSynchronize(st));
    }
  });
}

pw_status pw_backward_sweep(pw_ctx* ctx, int prob, const long long* receivers, int n_rec,
                            const double* seed, double* grad, int on_device, int wrt_velocity,
                            int checkpoint_every) {
  return guarded([&] {
    backward_common(ctx, prob, receivers, n_rec, seed, grad, on_device, wrt_velocity,
                    checkpoint_every, true);
  });
}

pw_status pw_backward(pw_ctx* ctx, int prob, const long long* receivers, int n_rec,
                      const double* seed, double* grad, int on_device, int wrt_velocity,
                      int checkpoint_every) {
  return guarded([&] {
    backward_common(ctx, prob, receivers, n_rec, seed, grad, on_device, wrt_velocity,
                    checkpoint_every, false);
  });
}

}  // extern "C"
