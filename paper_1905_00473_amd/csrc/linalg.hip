// Dense FP64 linear algebra for the Procrustes corrector (Secs. 3.3,
// 3.3.1, Algorithm 1):
//  * tall-skinny A^T B products (the snapshot Gram / projection step) and
//    tall A B products (basis updates) on the FP64 matrix cores
//    (v_mfma_f64_16x16x4f64), the A^T B products split over rows with a
//    fixed-order second-stage sum so results do not depend on scheduling;
//  * cyclic two-sided Jacobi for small symmetric Gram matrices, used to
//    orthonormalise tall blocks (two passes of Gram eigen-orthonormalisation,
//    the "truncated QR" of Algorithm 1);
//  * one-sided (Hestenes) Jacobi SVD of the small core matrix H of
//    Algorithm 1 with round-robin pair ordering, singular values sorted and
//    the rank counted on the device;
//  * the (r+1)-dimensional linear recurrence of the corrected sweep, as a
//    doubling scan of matrix-core GEMMs.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pw_internal.h"

namespace pw {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kTB = 256;
inline unsigned nblocks(long long n, int tb = kTB) { return (unsigned)((n + tb - 1) / tb); }

// ---------------------------------------------------------------------------
// MFMA GEMMs.  Operand layout of v_mfma_f64_16x16x4f64 (64 lanes):
//   lane l supplies A[m = l%16][k = l/16] and B[k = l/16][n = l%16];
//   the 16x16 result lives in 4 doubles per lane: D[4*v + l/16][l%16]
//   (rows interleaved across the four lane groups).
// ---------------------------------------------------------------------------
// Tile sizes: 64 x 64 (4 waves of 32 x 32) for narrow results, 128 x 128
// (4 waves of 64 x 64) for wide ones; BK rows of the contraction per step.
constexpr int TBM = 64, TBN = 64;
constexpr int GBM = 128, GBN = 128;
constexpr int GBK = 16, GPAD = 4;

// Split-K partial of C = A^T B (A: rows x a, B: rows x b, column-major):
// TM x TN tiles of the a x b result, rows split over blockIdx.z; each
// partial goes to part[z] (a x b, column-major).  The matrix cores compute
// tiles of C^T (operand a from B, operand b from A), so that in the result
// layout D[4v + l/16][l%16] the lane index l%16 runs along the rows of C and
// each group of 16 lanes stores 128 contiguous bytes.  The next step's global
// loads are issued before the current step's MFMAs (two LDS buffers).
template <int TM, int TN, int BK>
__global__ __launch_bounds__(256, 2) void k_gemm_tn(long long rows, int a, int b, const double* A,
                                                  long long lda, const double* B, long long ldb,
                                                  double* part, long long rows_per_split) {
  constexpr int SJ = TM / 32, SI = TN / 32;  // 16 x 16 sub-tiles per wave along m, n
  constexpr int CS = 256 / BK;               // columns per loader pass
  constexpr int QA = TM / CS, QB = TN / CS;  // loads per thread per step
  __shared__ double As[2][BK][TM + GPAD];
  __shared__ double Bs[2][BK][TN + GPAD];
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const long long r0 = (long long)blockIdx.z * rows_per_split;
  const long long r1 = std::min(rows, r0 + rows_per_split);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * (TM / 2), wn = (wave >> 1) * (TN / 2);
  v4d acc[SI][SJ];
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  const int lk = tid % BK, lc = tid / BK;  // row lk of the step, columns lc + CS q
  double ra[QA], rb[QB];
  auto load = [&](long long k0) {
    const long long r = k0 + lk;
    const bool ok = r < r1;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int c = lc + CS * q;
      ra[q] = (ok && m0 + c < a) ? A[r + (long long)(m0 + c) * lda] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int c = lc + CS * q;
      rb[q] = (ok && n0 + c < b) ? B[r + (long long)(n0 + c) * ldb] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) As[buf][lk][lc + CS * q] = ra[q];
#pragma unroll
    for (int q = 0; q < QB; ++q) Bs[buf][lk][lc + CS * q] = rb[q];
  };
  load(r0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (long long k0 = r0; k0 < r1; k0 += BK) {
    const bool more = k0 + BK < r1;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[SI], bv[SJ];
#pragma unroll
      for (int i = 0; i < SI; ++i) av[i] = Bs[buf][kk + (lane >> 4)][wn + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < SJ; ++j) bv[j] = As[buf][kk + (lane >> 4)][wm + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* P = part + (long long)blockIdx.z * a * b;
  // acc[i][j][v] = C[m0 + wm + 16 j + l%16][n0 + wn + 16 i + 4 v + l/16]
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * j + (lane & 15);
        const int n = n0 + wn + 16 * i + 4 * v + (lane >> 4);
        if (m < a && n < b) P[m + (long long)n * a] = acc[i][j][v];
      }
}

__global__ void k_reduce_splits(const double* part, int nsplit, int a, int b, double alpha,
                                double beta, double* C, long long ldc) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ab = (long long)a * b;
  if (t >= ab) return;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[(long long)k * ab + t];
  const int m = (int)(t % a), n = (int)(t / a);
  double* c = C + m + (long long)n * ldc;
  *c = beta == 0.0 ? alpha * s : alpha * s + beta * (*c);
}

// many splits: one wave per output element; lane l adds partials l, l+64,
// ... and the wave sums its lanes in a fixed order
__global__ __launch_bounds__(256) void k_reduce_splits_wave(const double* part, int nsplit, int a,
                                                            int b, double alpha, double beta,
                                                            double* C, long long ldc) {
  const long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const long long ab = (long long)a * b;
  if (t >= ab) return;
  double s = 0.0;
  for (int k = lane; k < nsplit; k += 64) s += part[(long long)k * ab + t];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) {
    const int m = (int)(t % a), n = (int)(t / a);
    double* c = C + m + (long long)n * ldc;
    *c = beta == 0.0 ? alpha * s : alpha * s + beta * (*c);
  }
}

// C = alpha A B + beta C (A: rows x k, B: k x n, column-major): TM x TN
// tiles of C, 4 waves of TM/2 x TN/2, C^T tiles on the matrix cores for
// contiguous stores and the next k-step prefetched, as in k_gemm_tn.
template <int TM, int TN, int BK>
__global__ __launch_bounds__(256, 2) void k_gemm_nn(long long rows, int n, int k, double alpha,
                                                  const double* A, long long lda, const double* B,
                                                  long long ldb, double beta, double* C,
                                                  long long ldc) {
  constexpr int SJ = TM / 32, SI = TN / 32;
  constexpr int KA = 256 / TM, QA = BK / KA;  // A: row am, k = ak + KA q
  constexpr int NB = 256 / BK, QB = TN / NB;  // B: k = bk, column bn + NB q
  __shared__ double As[2][BK][TM + GPAD];
  __shared__ double Bs[2][BK][TN + GPAD];
  const long long m0 = (long long)blockIdx.x * TM;
  const int n0 = blockIdx.y * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * (TM / 2), wn = (wave >> 1) * (TN / 2);
  v4d acc[SI][SJ];  // [n sub-tile][m sub-tile]
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  const int am = tid % TM, ak = tid / TM;
  const int bk = tid % BK, bn = tid / BK;
  double ra[QA], rb[QB];
  auto load = [&](int k0) {
    const long long r = m0 + am;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int kk = k0 + ak + KA * q;
      ra[q] = (r < rows && kk < k) ? A[r + (long long)kk * lda] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int nn = n0 + bn + NB * q;
      rb[q] = (k0 + bk < k && nn < n) ? B[(k0 + bk) + (long long)nn * ldb] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) As[buf][ak + KA * q][am] = ra[q];
#pragma unroll
    for (int q = 0; q < QB; ++q) Bs[buf][bk][bn + NB * q] = rb[q];
  };
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < k; k0 += BK) {
    const bool more = k0 + BK < k;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[SI], bv[SJ];
#pragma unroll
      for (int i = 0; i < SI; ++i) av[i] = Bs[buf][kk + (lane >> 4)][wn + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < SJ; ++j) bv[j] = As[buf][kk + (lane >> 4)][wm + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < SI; ++i)
#pragma unroll
        for (int j = 0; j < SJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // acc[i][j][v] = C[m0 + wm + 16 j + l%16][n0 + wn + 16 i + 4 v + l/16]
#pragma unroll
  for (int i = 0; i < SI; ++i)
#pragma unroll
    for (int j = 0; j < SJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long m = m0 + wm + 16 * j + (lane & 15);
        const int nn = n0 + wn + 16 * i + 4 * v + (lane >> 4);
        if (m < rows && nn < n) {
          double* c = C + m + (long long)nn * ldc;
          *c = beta == 0.0 ? alpha * acc[i][j][v] : alpha * acc[i][j][v] + beta * (*c);
        }
      }
}

__global__ void k_gemm_small(int m, int n, int k, double alpha, const double* A, int lda, int ta,
                             const double* B, int ldb, int tb, double beta, double* C, int ldc) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m * n) return;
  const int i = (int)(t % m), j = (int)(t / m);
  double s = 0.0;
  for (int l = 0; l < k; ++l) {
    const double x = ta ? A[l + (long long)i * lda] : A[i + (long long)l * lda];
    const double y = tb ? B[j + (long long)l * ldb] : B[l + (long long)j * ldb];
    s += x * y;
  }
  double* c = C + i + (long long)j * ldc;
  *c = beta == 0.0 ? alpha * s : alpha * s + beta * (*c);
}

// ---------------------------------------------------------------------------
// round-robin ordering of the Jacobi sweeps: n/2 disjoint pairs per round
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rr_index(int j, int round, int np) {
  return j == 0 ? 0 : ((j - 1 + round) % (np - 1)) + 1;
}

constexpr int kCholMax = 64;

// Truncated pivoted Cholesky of the Gram matrix G = A^T A (n x n, n <= 64)
// in one workgroup, and the two factors of the orthonormalisation
// Q = A T, A ~ Q R:  with P G P^T = L L^T truncated at rank k (the pivot
// steps stop when the largest remaining diagonal entry is <= rel times the
// largest diagonal of G, or <= abs_thr), R = L^T P^T (rows k.. zero) and
// T = P [L_11^{-T}; 0] (columns k.. zero).  T and R are column-major n x n.
__global__ __launch_bounds__(1024) void k_pchol_factors(int n, const double* Gg, double rel,
                                                        double abs_thr, double* T, double* R,
                                                        double* info) {
  __shared__ double A[kCholMax][kCholMax + 1];   // trailing Gram matrix
  __shared__ double Rm[kCholMax][kCholMax + 1];  // rows of L^T, pivoted column order
  __shared__ double X[kCholMax][kCholMax + 1];   // inverse of the leading k x k block
  __shared__ int perm[kCholMax];
  __shared__ int piv_s, stop_s;
  __shared__ double d0_s;
  const int tid = threadIdx.x;
  const int lane = tid & 63, x = tid & 63, y = tid >> 6;
  for (int m = 0; m < 4; ++m) {
    const int k = y + 16 * m;
    A[x][k] = (x < n && k < n) ? Gg[x + (long long)k * n] : 0.0;
    Rm[x][k] = 0.0;
    X[x][k] = 0.0;
  }
  if (tid < kCholMax) perm[tid] = tid;
  __syncthreads();
  int rank = n;
  for (int j = 0; j < n; ++j) {
    if (tid < 64) {
      // pivot: largest remaining diagonal entry (lowest index on ties)
      double v = (lane >= j && lane < n) ? A[lane][lane] : -1.0;
      int idx = lane;
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
          v = ov;
          idx = oi;
        }
      }
      if (lane == 0) {
        if (j == 0) d0_s = v;
        const double d0 = j == 0 ? v : d0_s;
        piv_s = idx;
        stop_s = (!(v > rel * d0) || !(v > abs_thr)) ? 1 : 0;
      }
    }
    __syncthreads();
    if (stop_s) {
      rank = j;
      break;
    }
    const int pv = piv_s;
    if (pv != j) {
      if (tid < n) {
        const double t = A[j][tid];
        A[j][tid] = A[pv][tid];
        A[pv][tid] = t;
      }
      __syncthreads();
      if (tid < n) {
        const double t = A[tid][j];
        A[tid][j] = A[tid][pv];
        A[tid][pv] = t;
      }
      if (tid < j) {
        const double t = Rm[tid][j];
        Rm[tid][j] = Rm[tid][pv];
        Rm[tid][pv] = t;
      }
      if (tid == 0) {
        const int t = perm[j];
        perm[j] = perm[pv];
        perm[pv] = t;
      }
      __syncthreads();
    }
    const double r = sqrt(A[j][j]);
    if (tid >= j && tid < n) Rm[j][tid] = (tid == j) ? r : A[j][tid] / r;
    __syncthreads();
    for (int m = 0; m < 4; ++m) {
      const int k = y + 16 * m;
      if (x > j && x < n && k > j && k < n) A[x][k] -= Rm[j][x] * Rm[j][k];
    }
    __syncthreads();
  }
  // info: [kept rank, smallest kept pivot / largest diagonal]
  if (info && tid == 0) {
    info[0] = (double)rank;
    info[1] = rank > 0 && d0_s > 0.0 ? (Rm[rank - 1][rank - 1] * Rm[rank - 1][rank - 1]) / d0_s : 0.0;
  }
  // X = (leading rank x rank block of L^T)^{-1}, one column per thread
  if (tid < rank) {
    const int b = tid;
    X[b][b] = 1.0 / Rm[b][b];
    for (int a = b - 1; a >= 0; --a) {
      double s = 0.0;
      for (int c = a + 1; c <= b; ++c) s += Rm[a][c] * X[c][b];
      X[a][b] = -s / Rm[a][a];
    }
  }
  __syncthreads();
  for (int m = 0; m < 4; ++m) {
    const int b = y + 16 * m, a = x;
    if (a < n && b < n) {
      T[perm[a] + (long long)b * n] = (a < rank && b < rank) ? X[a][b] : 0.0;
      R[a + (long long)perm[b] * n] = (a < rank) ? Rm[a][b] : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// one-sided Jacobi SVD: one launch per round of disjoint column pairs
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_jacobi_round(int n, int np, int round, double* H,
                                                       double* V, int* counter,
                                                       const double* fro2) {
  const int lane = threadIdx.x & 63;
  const int pair = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pair >= np / 2) return;
  int p = rr_index(pair, round, np);
  int q = rr_index(np - 1 - pair, round, np);
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  if (q >= n) return;
  double* hp = H + (long long)p * n;
  double* hq = H + (long long)q * n;
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double x = hp[i], y = hq[i];
    al += x * x;
    be += y * y;
    ga += x * y;
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  // skip pairs already orthogonal to the rounding level of the dot
  // products (4 sqrt(n) eps, as one-sided Jacobi codes commonly use), and
  // pairs of two columns that are both rounding noise of H (norm below
  // eps ||H||_F: they carry singular values below any rank tolerance)
  const double noise2 = 4.9e-32 * (*fro2);
  if (ga == 0.0 || fabs(ga) <= 4.5e-16 * sqrt((double)n) * sqrt(al * be)) return;
  if (al < noise2 && be < noise2) return;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
  for (int i = lane; i < n; i += 64) {
    const double x = hp[i], y = hq[i];
    hp[i] = c * x - s * y;
    hq[i] = s * x + c * y;
  }
  double* vp = V + (long long)p * n;
  double* vq = V + (long long)q * n;
  for (int i = lane; i < n; i += 64) {
    const double x = vp[i], y = vq[i];
    vp[i] = c * x - s * y;
    vq[i] = s * x + c * y;
  }
  if (lane == 0) atomicAdd(counter, 1);
}

// Block one-sided Jacobi: columns are grouped in blocks of kJB; one launch
// is one round of the round-robin over blocks and one workgroup handles one
// block pair (16 columns).  The workgroup forms the 16 x 16 Gram matrix of
// its columns on the matrix cores, runs one cyclic sweep of two-sided
// rotations on it (the rotation of every pair from the current Gram
// entries, with the same relative threshold and noise rule as the column
// version), and applies the accumulated 16 x 16 rotation to the 16 columns
// of H and V.
constexpr int kJB = 8;
constexpr int kJC = 2 * kJB;

__device__ __forceinline__ void pair_rotation(const double* G, int i, int partner, bool valid,
                                              double thr, double noise2, double* a, double* b,
                                              bool* rot) {
  *a = 1.0;
  *b = 0.0;
  *rot = false;
  if (!valid) return;
  const int p = min(i, partner), q = max(i, partner);
  const double al = G[p * kJC + p], be = G[q * kJC + q], ga = G[p * kJC + q];
  if (ga == 0.0 || fabs(ga) <= thr * sqrt(al * be)) return;
  if (fmin(al, be) < noise2) return;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
  // column p <- c p - s q ; column q <- s p + c q
  *a = c;
  *b = (i == p) ? -s : s;
  *rot = true;
}

// rows of one staged block column (the block path takes n <= kJRows; a
// launch whose matrices all have n <= kJRowsSmall stages only that many,
// with a quarter of the LDS, so that several workgroups share a CU)
constexpr int kJRows = 1024;
constexpr int kJRowsSmall = 256;

// one block pair of one round (see k_jacobi_block); lb: the workgroup's
// index among the pairs of this matrix
// threads of a block-pair workgroup: 8 waves (the staging, the Gram matrix
// and the updates split over all of them; the 16 x 16 inner sweep on the
// first four)
constexpr int kJT = 512;
constexpr int kJW = kJT / 64;

template <int ROWS>
__device__ __forceinline__ void jacobi_block_pair(int n, int npb, int round, int lb, double* H,
                                                  double* V, int* counter, const double* fro2,
                                                  double* cnorm2) {
  constexpr int kJLd = ROWS + 1;  // odd stride: the 16 columns fall in distinct LDS banks
  constexpr int RPT = (ROWS + kJT - 1) / kJT;  // staged rows per thread and column
  constexpr int VT = 4;            // V tiles per wave prefetched at the start
  __shared__ double Hs[kJC * kJLd];
  __shared__ double Gp[kJW][kJC * kJC];
  __shared__ double G[2][kJC * kJC];
  __shared__ double W[2][kJC * kJC];
  __shared__ signed char part[kJC - 1][kJC];
  __shared__ int nrot;
  __shared__ int any_rot;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // blocks are dispatched round-robin over the 8 XCDs; pair indices are
  // given to them in contiguous chunks per XCD, so that a column block,
  // which moves to a neighbouring pair index from one round to the next,
  // mostly stays in the same XCD's L2
  const int np2 = npb / 2, per = (np2 + 7) / 8;
  const int pair = (lb % 8) * per + lb / 8;
  if (pair >= np2) return;
  int bp = rr_index(pair, round, npb);
  int bq = rr_index(npb - 1 - pair, round, npb);
  if (bp > bq) {
    const int t = bp;
    bp = bq;
    bq = t;
  }
  const int nb = (n + kJB - 1) / kJB;
  if (bq >= nb) return;  // paired with the padding block
  auto gcol = [&](int c) { return c < kJB ? bp * kJB + c : bq * kJB + (c - kJB); };
  // V operands of the first VT row tiles of this wave (see step 3), loaded
  // now so that their latency overlaps steps 1 and 2
  double va[VT][4];
#pragma unroll
  for (int u = 0; u < VT; ++u) {
    const int ra = 16 * (wave + kJW * u) + (lane & 15);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int gk = gcol(4 * t + (lane >> 4));
      va[u][t] = (ra < n && gk < n) ? V[(long long)gk * n + ra] : 0.0;
    }
  }
  // stage the 16 columns of H (all loads of a thread in flight together);
  // padding columns beyond n are zero
  {
    double v[kJC][RPT];
#pragma unroll
    for (int c = 0; c < kJC; ++c) {
      const int gc = gcol(c);
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int row = tid + kJT * r;
        v[c][r] = (gc < n && row < n) ? H[(long long)gc * n + row] : 0.0;
      }
    }
    const int n64 = (n + 63) & ~63;
#pragma unroll
    for (int c = 0; c < kJC; ++c)
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int row = tid + kJT * r;
        if (row < n64) Hs[c * kJLd + row] = v[c][r];
      }
  }
  // round-robin partners of the inner sweep
  if (tid < (kJC - 1) * (kJC / 2)) {
    const int r = tid / (kJC / 2), g = tid % (kJC / 2);
    const int a = rr_index(g, r, kJC), b = rr_index(kJC - 1 - g, r, kJC);
    part[r][a] = (signed char)b;
    part[r][b] = (signed char)a;
  }
  if (tid == 0) nrot = 0;
  __syncthreads();
  // 1. Gram matrix D = B^T B of the staged block B (n x 16) on the matrix
  //    cores, rows split over the 8 waves (wave w: rows 4 (w mod 4) + 16 s +
  //    {0..3}, s = 0..3, of the (w / 4)-th 64-row half of every 128 rows).
  //    Operand lane l: A[l%16][l/16] = B^T[l%16][k0 + l/16] = B[k0 +
  //    l/16][l%16], the same value for both.
  {
    // rows beyond n are zero in the staged block up to the next multiple
    // of 64 (cleared above), so full groups of four steps need no test
    v4d acc0 = v4d{0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    const double* col = Hs + (lane & 15) * kJLd + (lane >> 4);
    for (int k0 = 4 * (wave & 3) + 64 * (wave >> 2); k0 < n; k0 += 128) {
      const double x0 = col[k0], x1 = col[k0 + 16], x2 = col[k0 + 32], x3 = col[k0 + 48];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, x1, acc1, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x2, x2, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x3, x3, acc1, 0, 0, 0);
    }
    for (int v = 0; v < 4; ++v)
      Gp[wave][(4 * v + (lane >> 4)) * kJC + (lane & 15)] = acc0[v] + acc1[v];
  }
  __syncthreads();
  // the partial Gram matrices summed in a fixed order
  auto gram_sum = [&](int e) {
    double x = Gp[0][e];
#pragma unroll
    for (int w = 1; w < kJW; ++w) x += Gp[w][e];
    return x;
  };
  if (tid < kJC * kJC) {
    G[0][tid] = gram_sum(tid);
    W[0][tid] = (tid / kJC == tid % kJC) ? 1.0 : 0.0;
  }
  if (tid == 0) any_rot = 0;
  // squared norms of the block's columns, for the ordering of the next sweep
  // (the diagonal of G, summed in the same order)
  if (tid < kJC && gcol(tid) < n) cnorm2[gcol(tid)] = gram_sum(tid * (kJC + 1));
  __syncthreads();
  // a pair is rotated only if it is above the threshold in the current
  // Gram matrix; if no pair of the fresh one is, the sweep below would
  // leave everything unchanged: skip it
  const double noise2 = 4.9e-32 * (*fro2);
  const double thr2 = 4.5e-16 * 4.5e-16 * (double)n;
  if (tid < kJC * kJC) {
    const int pi_ = tid / kJC, pj_ = tid % kJC;
    if (pi_ < pj_ && gcol(pj_) < n) {
      const double al = G[0][pi_ * kJC + pi_], be = G[0][pj_ * kJC + pj_];
      const double ga = G[0][pi_ * kJC + pj_];
      if (ga != 0.0 && ga * ga > thr2 * (al * be) && fmin(al, be) >= noise2) any_rot = 1;
    }
  }
  __syncthreads();
  if (any_rot == 0) return;
  // 2. one cyclic sweep of rotations on the Gram matrix.  Thread (i, j)
  //    forms the rotation of column j's pair (the threads that share a pair
  //    compute it from the same entries, so they agree bit for bit) and takes
  //    the one of column i from lane (i mod 4, i) of its own wave, which formed
  //    it: no second barrier per round.  The partners of this thread's row
  //    and column index in the 15 rounds are packed four bits each into one
  //    register.
  // (threads 0..255, the first four waves; the others keep the barriers)
  const bool inner = tid < kJC * kJC;
  const int i = inner ? tid / kJC : 0, j = tid % kJC;  // this thread's Gram / rotation entry
  const int src_i = (lane & ~(kJC - 1)) | i;
  unsigned long long packi = 0, packj = 0;
  for (int r = 0; r < kJC - 1; ++r) {
    packi |= (unsigned long long)part[r][i] << (4 * r);
    packj |= (unsigned long long)part[r][j] << (4 * r);
  }
  int cur = 0, myrot = 0;
  for (int r = 0; r < kJC - 1; ++r) {
    if (!inner) {
      cur ^= 1;
      __syncthreads();
      continue;
    }
    const double* Gc = G[cur];
    const double* Wc = W[cur];
    const int pi = (int)((packi >> (4 * r)) & 15), pj = (int)((packj >> (4 * r)) & 15);
    const int lo = j < pj ? j : pj, hi = j < pj ? pj : j;
    const double g0 = Gc[i * kJC + j], g1 = Gc[i * kJC + pj], g2 = Gc[pi * kJC + j],
                 g3 = Gc[pi * kJC + pj], w0 = Wc[i * kJC + j], w1 = Wc[i * kJC + pj];
    const double al = Gc[lo * (kJC + 1)], be = Gc[hi * (kJC + 1)], ga = Gc[lo * kJC + hi];
    // the pair (lo, hi) is rotated only if it is above the threshold
    const bool rot = (gcol(hi) < n) & (ga != 0.0) & (ga * ga > thr2 * (al * be)) &
                     (al >= noise2) & (be >= noise2);
    // tan of the angle: t = sgn(d) g / (|d| + sqrt(d^2 + g^2)), d = be - al,
    // g = 2 ga (the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = d / g),
    // from the hardware reciprocal square root and reciprocal alone: an
    // angle off by a relative 1e-5 still reduces the pair's inner product by
    // that factor, and the sweep count does not change.  The rotation stays
    // orthogonal to rounding whatever t is: c = 1 / sqrt(1 + t^2) is refined
    // by two Newton steps to full double precision and s = c t.  Branch-free:
    // the values formed for a pair that is not rotated are discarded.
    const double d = be - al, g = 2.0 * ga;
    const double xx = fma(d, d, g * g);
    const double m = fma(xx, __builtin_amdgcn_rsq(xx), fabs(d));  // |d| + sqrt(d^2 + g^2)
    const double t = (d >= 0.0 ? g : -g) * __builtin_amdgcn_rcp(m);
    const double u = fma(t, t, 1.0), hu = 0.5 * u;
    double w = __builtin_amdgcn_rsq(u);
    w = fma(w, fma(-hu * w, w, 0.5), w);
    w = fma(w, fma(-hu * w, w, 0.5), w);
    const double cs = w, sn = w * t;
    // column x of the pair (p, q), p < q: x' = a x + b y with
    // column p <- c p - s q, column q <- s p + c q
    const double aj = rot ? cs : 1.0;
    const double bj = rot ? (j == lo ? -sn : sn) : 0.0;
    const double ai = __shfl(aj, src_i, 64), bi = __shfl(bj, src_i, 64);
    if (rot && i == j && j == lo) ++myrot;  // one counting thread per pair
    // G' = J^T G J entrywise, W' = W J
    G[cur ^ 1][tid] = ai * fma(bj, g1, aj * g0) + bi * fma(bj, g3, aj * g2);
    W[cur ^ 1][tid] = fma(bj, w1, aj * w0);
    cur ^= 1;
    __syncthreads();
  }
  if (myrot) atomicAdd(&nrot, myrot);
  __syncthreads();
  if (nrot == 0) return;
  // the rotated columns' squared norms: the diagonal of the rotated Gram
  if (tid < kJC && gcol(tid) < n) cnorm2[gcol(tid)] = G[cur][tid * (kJC + 1)];
  // 3. H(:, cols) <- B W (B staged), V(:, cols) <- V(:, cols) W, in 16-row
  //    tiles on the matrix cores, computed transposed, (X W)^T = W^T X^T:
  //    operand A[i][k] = W^T[i][4t + k] = W[4t + k][i] (lane l: i = l%16,
  //    k = l/16; held in four registers), operand B[k][j] = X[tile + j][4t + k],
  //    D[4v + l/16][l%16] = (X W)[tile + l%16][4v + l/16]: the 16 lanes of a
  //    group store 16 consecutive rows of one column (128 contiguous bytes).
  const double* Wf = W[cur];
  double bw[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) bw[t] = Wf[(4 * t + (lane >> 4)) * kJC + (lane & 15)];
  auto store = [&](double* X, int tile, const v4d& acc) {
    const int row = tile + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gc = gcol(4 * v + (lane >> 4));
      if (row < n && gc < n) X[(long long)gc * n + row] = acc[v];
    }
  };
  for (int tile = 16 * wave; tile < n; tile += 16 * kJW) {
    const int ra = tile + (lane & 15);
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 4 * t + (lane >> 4);
      const double a = (ra < n) ? Hs[k * kJLd + ra] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bw[t], a, acc, 0, 0, 0);
    }
    store(H, tile, acc);
  }
#pragma unroll
  for (int u = 0; u < VT; ++u) {
    const int tile = 16 * (wave + kJW * u);
    if (tile < n) {
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bw[t], va[u][t], acc, 0, 0, 0);
      store(V, tile, acc);
    }
  }
  for (int tile = 16 * (wave + kJW * VT); tile < n; tile += 16 * kJW) {
    const int ra = tile + (lane & 15);
    double a[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int gk = gcol(4 * t + (lane >> 4));
      a[t] = (ra < n && gk < n) ? V[(long long)gk * n + ra] : 0.0;
    }
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bw[t], a[t], acc, 0, 0, 0);
    store(V, tile, acc);
  }
  if (tid == 0) atomicAdd(counter, nrot);
}

template <int ROWS>
__global__ __launch_bounds__(kJT) void k_jacobi_block(int n, int npb, int round, double* H,
                                                      double* V, int* counter,
                                                      const double* fro2, double* cnorm2) {
  jacobi_block_pair<ROWS>(n, npb, round, (int)blockIdx.x, H, V, counter, fro2, cnorm2);
}

// column order of the next sweep: descending norm, ties by index (one
// workgroup; n <= kJRows).  perm[k] = the column that goes to position k.
__device__ __forceinline__ void norm_order(int n, const double* nrm, int* perm) {
  __shared__ double v[kJRows];
  // NaN sorts last, so that the ranks always form a permutation
  for (int c = threadIdx.x; c < n; c += 1024) v[c] = nrm[c] == nrm[c] ? nrm[c] : -1.0;
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += 1024) {
    const double x = v[c];
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += (v[k] > x) | ((v[k] == x) & (k < c));
    perm[rank] = c;
  }
}

__global__ __launch_bounds__(1024) void k_norm_order(int n, const double* nrm, int* perm) {
  norm_order(n, nrm, perm);
}

// ---- many Jacobi SVDs in lockstep (the correctors of a batch) ------------
// One launch per round covers the block pairs of every matrix still
// sweeping: workgroups [block_begin, block_begin + 8 ceil(npb / 16)) take
// one matrix's pairs, which are computed exactly as in its own launch.
struct JacobiJob {
  int n, npb, block_begin;
  double *Hc, *Hn, *Vc, *Vn;  // current columns and the gather target
  int* pos;                   // this sweep's column order
  double* cnorm2;
  const double* fro2;
  int* counter;               // this sweep's rotation count
};

__device__ __forceinline__ int job_of(const JacobiJob* jobs, int nj, int blk) {
  int lo = 0, hi = nj - 1;  // last job with block_begin <= blk
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_begin <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int ROWS>
__global__ __launch_bounds__(kJT) void k_jacobi_block_multi(const JacobiJob* jobs, int nj,
                                                            int round) {
  const JacobiJob& j = jobs[job_of(jobs, nj, (int)blockIdx.x)];
  if (round >= j.npb - 1) return;  // this matrix has fewer rounds per sweep
  jacobi_block_pair<ROWS>(j.n, j.npb, round, (int)blockIdx.x - j.block_begin, j.Hc, j.Vc,
                          j.counter, j.fro2, j.cnorm2);
}

__global__ __launch_bounds__(1024) void k_norm_order_multi(const JacobiJob* jobs) {
  const JacobiJob& j = jobs[blockIdx.x];
  norm_order(j.n, j.cnorm2, j.pos);
}

// Hn(:, k) = Hc(:, pos[k]), Vn likewise, for job blockIdx.y
__global__ void k_gather_cols2_multi(const JacobiJob* jobs) {
  const JacobiJob& j = jobs[blockIdx.y];
  const int n = j.n;
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / n), i = (int)(e % n);
    const int pk = j.pos[k];
    const bool ok = (unsigned)pk < (unsigned)n;
    const long long src = (long long)(ok ? pk : 0) * n + i;
    j.Hn[e] = ok ? j.Hc[src] : 0.0;
    j.Vn[e] = ok ? j.Vc[src] : 0.0;
  }
}

__global__ void k_collect_counters(const JacobiJob* jobs, int nj, int* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nj) out[t] = *jobs[t].counter;
}

// Hd(:, k) = Hs(:, perm[k]) and Vd(:, k) = Vs(:, perm[k]) (n x n, column-major)
__global__ void k_gather_cols2(int n, const int* perm, const double* Hs, double* Hd,
                               const double* Vs, double* Vd) {
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / n), i = (int)(e % n);
    const int pk = perm[k];
    const bool ok = (unsigned)pk < (unsigned)n;
    const long long src = (long long)(ok ? pk : 0) * n + i;
    Hd[e] = ok ? Hs[src] : 0.0;
    Vd[e] = ok ? Vs[src] : 0.0;
  }
}

__global__ void k_col_norms(int n, const double* H, double* sig) {
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= n) return;
  double s = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double x = H[(long long)col * n + i];
    s += x * x;
  }
  s = wave_sum(s);
  if (lane == 0) sig[col] = sqrt(s);
}

// position of every column in descending order of its norm (ties by index)
// and the rank count
__global__ void k_sort_rank(int n, const double* sig_unsorted, int* pos, double tol,
                            int* rank_dev, double* sig_sorted) {
  __shared__ double smax;
  __shared__ int cnt;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, sig_unsorted[i]);
    smax = m;
    cnt = 0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double sj = sig_unsorted[j];
    int r = 0;
    for (int i = 0; i < n; ++i) {
      const double si = sig_unsorted[i];
      r += (si > sj || (si == sj && i < j)) ? 1 : 0;
    }
    pos[j] = r;
    sig_sorted[r] = sj;
    if (smax > 0.0 && sj / smax > tol) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *rank_dev = cnt;
}

__global__ void k_scatter_svd(int n, const double* Hw, const double* Vw, const int* pos,
                              const double* sig_unsorted, double* X, double* Y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int i = (int)(t % n), j = (int)(t / n);
  const int dst = pos[j];
  const double s = sig_unsorted[j];
  X[i + (long long)dst * n] = s > 0.0 ? Hw[i + (long long)j * n] / s : 0.0;
  Y[i + (long long)dst * n] = Vw[i + (long long)j * n];
}

__global__ void k_identity(int n, double* V) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  V[t] = (t % n == t / n) ? 1.0 : 0.0;
}

__global__ void k_add_diag(int r, const double* S, double* H, int ldh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < r) H[i + (long long)i * ldh] += S[i];
}

__global__ void k_copy_block(int m, int n, const double* src, long long lds, double* dst,
                             long long ldd) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m * n) return;
  const long long i = t % m, j = t / m;
  dst[i + j * ldd] = src[i + j * lds];
}

__global__ void k_fill(double* p, long long n, double v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_sumsq_cols(const double* A, long long rows, int cols, long long lda,
                             double* partials) {
  __shared__ double s[kTB];
  const long long total = rows * cols;
  double acc = 0.0;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long i = t % rows, j = t / rows;
    const double x = A[i + j * lda];
    acc += x * x;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kTB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

__global__ void k_sum(const double* partials, int nb, double* out) {
  __shared__ double s[kTB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partials[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kTB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

constexpr int kSplitTarget = 512;

// large results use the 128 x 128 tile kernel with about kBigTarget
// workgroups (the scratch bound below covers both schemes)
constexpr int kBigTarget = 256;
bool small_tiles_forced() {
  static const bool on = getenv("PW_GEMM_SMALL_TILES") != nullptr;
  return on;
}

bool tn_big(long long rows, int a, int b) {
  return a > TBM && b > TBN && rows >= GBM && !small_tiles_forced();
}

int tn_splits(long long rows, int a, int b) {
  const bool big = tn_big(rows, a, b);
  const int bm = big ? GBM : TBM, bn = big ? GBN : TBN, bk = GBK;
  const long long tiles = (long long)((a + bm - 1) / bm) * ((b + bn - 1) / bn);
  const long long target = big ? kBigTarget : kSplitTarget;
  long long s = (target + tiles - 1) / tiles;
  const long long maxs = (rows + bk - 1) / bk;
  s = std::max(1LL, std::min(s, maxs));
  return (int)s;
}

}  // namespace

size_t gemm_tn_work(long long rows, int a, int b) {
  return (size_t)tn_splits(rows, a, b) * a * b;
}

size_t gemm_tn_work_bound(int a_max, int b_max) {
  // splits <= ceil(target / tiles) <= target / tiles + 1 and
  // a * b <= tiles * BM * BN, so splits * a * b <= target * BM * BN + a * b
  // for either tile scheme
  return std::max((size_t)kSplitTarget * TBM * TBN, (size_t)kBigTarget * GBM * GBN) +
         (size_t)a_max * b_max;
}

void gemm_tn(long long rows, int a, int b, double alpha, const double* A, long long lda,
             const double* B, long long ldb, double beta, double* C, long long ldc, double* work,
             size_t work_elems, hipStream_t st) {
  if (a <= 0 || b <= 0) return;
  if (rows > 0 && gemm_tn_work(rows, a, b) > work_elems)
    fail(PW_EINVAL, "gemm_tn: split-K scratch too small");
  if (rows <= 0) {
    // empty contraction: C = beta C
    for (int j = 0; j < b; ++j) {
      if (beta == 0.0) {
        hipLaunchKernelGGL(k_fill, dim3(nblocks(a)), dim3(kTB), 0, st, C + (long long)j * ldc,
                           (long long)a, 0.0);
        PW_LAUNCH_CHECK();
      }
    }
    return;
  }
  const bool big = tn_big(rows, a, b);
  const int splits = tn_splits(rows, a, b);
  long long rps = (rows + splits - 1) / splits;
  rps = (rps + GBK - 1) / GBK * GBK;
  const int ns = (int)((rows + rps - 1) / rps);
  if (big) {
    dim3 grid((a + GBM - 1) / GBM, (b + GBN - 1) / GBN, ns);
    hipLaunchKernelGGL((k_gemm_tn<GBM, GBN, GBK>), grid, dim3(256), 0, st, rows, a, b, A, lda, B,
                       ldb, work, rps);
  } else {
    dim3 grid((a + TBM - 1) / TBM, (b + TBN - 1) / TBN, ns);
    hipLaunchKernelGGL((k_gemm_tn<TBM, TBN, GBK>), grid, dim3(256), 0, st, rows, a, b, A, lda, B,
                       ldb, work, rps);
  }
  PW_LAUNCH_CHECK();
  const long long ab = (long long)a * b;
  if (ns >= 32)
    hipLaunchKernelGGL(k_reduce_splits_wave, dim3((unsigned)((ab + 3) / 4)), dim3(256), 0, st,
                       (const double*)work, ns, a, b, alpha, beta, C, ldc);
  else
    hipLaunchKernelGGL(k_reduce_splits, dim3(nblocks(ab)), dim3(kTB), 0, st, (const double*)work,
                       ns, a, b, alpha, beta, C, ldc);
  PW_LAUNCH_CHECK();
}

void gemm_nn(long long rows, int n, int k, double alpha, const double* A, long long lda,
             const double* B, long long ldb, double beta, double* C, long long ldc,
             hipStream_t st) {
  if (rows <= 0 || n <= 0) return;
  if (k <= 0) {
    if (beta != 1.0) {
      // C = beta C (only used with beta 0 by the library)
      for (int j = 0; j < n; ++j) {
        hipLaunchKernelGGL(k_fill, dim3(nblocks(rows)), dim3(kTB), 0, st, C + (long long)j * ldc,
                           rows, 0.0);
        PW_LAUNCH_CHECK();
      }
    }
    return;
  }
  if (n > TBN && rows >= GBM && !small_tiles_forced()) {
    dim3 grid((unsigned)((rows + GBM - 1) / GBM), (n + GBN - 1) / GBN);
    hipLaunchKernelGGL((k_gemm_nn<GBM, GBN, GBK>), grid, dim3(256), 0, st, rows, n, k, alpha, A,
                       lda, B, ldb, beta, C, ldc);
    PW_LAUNCH_CHECK();
    return;
  }
  dim3 grid((unsigned)((rows + TBM - 1) / TBM), (n + TBN - 1) / TBN);
  hipLaunchKernelGGL((k_gemm_nn<TBM, TBN, GBK>), grid, dim3(256), 0, st, rows, n, k, alpha, A,
                     lda, B, ldb, beta, C, ldc);
  PW_LAUNCH_CHECK();
}

void gemm_small(int m, int n, int k, double alpha, const double* A, int lda, bool ta,
                const double* B, int ldb, bool tb, double beta, double* C, int ldc,
                hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  const long long mn = (long long)m * n;
  hipLaunchKernelGGL(k_gemm_small, dim3(nblocks(mn)), dim3(kTB), 0, st, m, n, k, alpha, A, lda,
                     (int)ta, B, ldb, (int)tb, beta, C, ldc);
  PW_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Householder QR of a tall matrix with at most 64 columns (TSQR): the rows
// are cut into chunks of at most 256 rows, each chunk is factored by
// Householder reflections in the LDS of one workgroup, the stacked n x n
// R factors of all chunks form the next, shorter matrix, until one chunk
// is left.  Q is then formed from the top down by applying each chunk's
// reflectors to its n-row block of the level above ([I; 0] at the top).
// Backward stable: Q is orthonormal to rounding whatever the conditioning
// of A (directions far below sqrt(eps) of the largest are resolved, which
// a Gram-based QR cannot do).
// ---------------------------------------------------------------------------
constexpr int kQrRows = 256;          // rows per chunk (at most)
constexpr int kQrRPT = kQrRows / 4;  // rows per thread (4 threads per column)
constexpr int kQrCols = 64;           // columns per factorisation

// rows [off, off + m) of chunk c when M rows are cut into nch near-equal
// chunks
__device__ __forceinline__ void qr_chunk(long long M, int nch, int c, long long& off, int& m) {
  const long long base = M / nch, rem = M % nch;
  off = (long long)c * base + (c < rem ? c : rem);
  m = (int)(base + (c < rem ? 1 : 0));
}

// Householder QR of chunk blockIdx.x of A (M x n, n <= 64): reflector j is
// I - tau_j v v^T with v_j = 1 and v_i (i > j) stored in V below the
// diagonal (LAPACK's convention; V is zero elsewhere); tau to
// tau[c * n + j]; the n x n R factor (rows >= min(m, n) zero) to rows
// [c n, c n + n) of Rout.  V may alias A (the chunk is read completely
// before anything is written).  Thread (k, s) = (t mod 64, t / 64) holds
// column k of the rows i = s + 4 q in registers; wave 0 finishes each
// reflector in LDS (kept there until the end), so a step costs 2 x 64
// register FMAs per thread and no global memory access.
__global__ __launch_bounds__(256) void k_hqr_chunk(long long M, int n, int nch, const double* A,
                                                   long long lda, double* V, long long ldv,
                                                   double* tau, double* Rout, long long ldr) {
  __shared__ double vs[kQrCols * kQrRows];  // reflector j in vs[j * kQrRows + i]
  __shared__ double part[4 * kQrCols];
  __shared__ double w[kQrCols];
  __shared__ double taus[kQrCols];
  __shared__ double betas[kQrCols];
  long long off;
  int m;
  qr_chunk(M, nch, blockIdx.x, off, m);
  const int t = threadIdx.x, k = t & 63, seg = t >> 6;
  double reg[kQrRPT];
#pragma unroll
  for (int q = 0; q < kQrRPT; ++q) {
    const int i = seg + 4 * q;
    reg[q] = (k < n && i < m) ? A[(off + i) + (long long)k * lda] : 0.0;
  }
  const int r = m < n ? m : n;
  for (int j = 0; j < r; ++j) {
    double* vcol = vs + j * kQrRows;
    if (k == j) {
#pragma unroll
      for (int q = 0; q < kQrRPT; ++q) {
        const int i = seg + 4 * q;
        vcol[i] = i >= j ? reg[q] : 0.0;
      }
    }
    __syncthreads();
    if (seg == 0) {
      // every lane of wave 0 forms the reflector (beta, tau, 1 / (alpha -
      // beta)) from the butterfly sum, then finishes its four entries of v
      double s = 0.0;
      for (int i = j + 1 + k; i < m; i += 64) s = fma(vcol[i], vcol[i], s);
      s = wave_sum(s);
      const double alpha = vcol[j];
      double beta = alpha, tj = 0.0, sc = 0.0;
      if (s != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        tj = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
      }
      for (int i = k; i < kQrRows; i += 64) vcol[i] = i == j ? 1.0 : (i > j ? vcol[i] * sc : 0.0);
      if (k == 0) {
        taus[j] = tj;
        betas[j] = beta;
      }
    }
    __syncthreads();
    const double tj = taus[j];
    if (tj != 0.0) {
      // w_k = tau sum_{i >= j} v_i a_ik, k > j
      double acc[4] = {0.0, 0.0, 0.0, 0.0};  // four independent FMA chains
      if (k > j && k < n) {
#pragma unroll
        for (int q = 0; q < kQrRPT; ++q) acc[q & 3] = fma(vcol[seg + 4 * q], reg[q], acc[q & 3]);
      }
      part[seg * kQrCols + k] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
      __syncthreads();
      if (t > j && t < n)
        w[t] = tj * ((part[t] + part[kQrCols + t]) + (part[2 * kQrCols + t] + part[3 * kQrCols + t]));
      __syncthreads();
      if (k > j && k < n) {
        const double wk = w[k];
#pragma unroll
        for (int q = 0; q < kQrRPT; ++q) reg[q] = fma(-wk, vcol[seg + 4 * q], reg[q]);
      }
      __syncthreads();  // part is rewritten by the next step
    }
  }
  for (int k2 = 0; k2 < n; ++k2)
    if (t < m) V[(off + t) + (long long)k2 * ldv] = (k2 < r && t > k2) ? vs[k2 * kQrRows + t] : 0.0;
  if (t < n) tau[(long long)blockIdx.x * n + t] = t < r ? taus[t] : 0.0;
#pragma unroll
  for (int q = 0; q < kQrRPT; ++q) {
    const int i = seg + 4 * q;
    if (k < n && i < n) {
      double val = 0.0;
      if (i < r && i < k) val = reg[q];
      else if (i < r && i == k) val = betas[i];
      Rout[((long long)blockIdx.x * n + i) + (long long)k * ldr] = val;
    }
  }
}

// Q rows of chunk blockIdx.x: the chunk's reflectors applied, last first,
// to [Qup rows c n .. c n + n - 1; 0] (Qup null: [I; 0]).  Q may alias V
// (the reflectors are staged in LDS first).  Same register layout as
// k_hqr_chunk.
__global__ __launch_bounds__(256) void k_hqr_formq(long long M, int n, int nch, const double* V,
                                                   long long ldv, const double* tau,
                                                   const double* Qup, long long ldu, double* Q,
                                                   long long ldq) {
  __shared__ double vs[kQrCols * kQrRows];
  __shared__ double part[4 * kQrCols];
  __shared__ double w[kQrCols];
  long long off;
  int m;
  qr_chunk(M, nch, blockIdx.x, off, m);
  const int t = threadIdx.x, k = t & 63, seg = t >> 6;
  const int r = m < n ? m : n;
  for (int j = 0; j < r; ++j)
    vs[j * kQrRows + t] = t == j ? 1.0 : ((t > j && t < m) ? V[(off + t) + (long long)j * ldv] : 0.0);
  double reg[kQrRPT];
#pragma unroll
  for (int q = 0; q < kQrRPT; ++q) {
    const int i = seg + 4 * q;
    double val = 0.0;
    if (k < n && i < m && i < n)
      val = Qup ? Qup[((long long)blockIdx.x * n + i) + (long long)k * ldu] : (i == k ? 1.0 : 0.0);
    reg[q] = val;
  }
  __syncthreads();
  for (int j = r - 1; j >= 0; --j) {
    const double tj = tau[(long long)blockIdx.x * n + j];
    if (tj == 0.0) continue;  // the same for every thread of the block
    const double* vcol = vs + j * kQrRows;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // four independent FMA chains
    if (k < n) {
#pragma unroll
      for (int q = 0; q < kQrRPT; ++q) acc[q & 3] = fma(vcol[seg + 4 * q], reg[q], acc[q & 3]);
    }
    part[seg * kQrCols + k] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (t < n)
      w[t] = tj * ((part[t] + part[kQrCols + t]) + (part[2 * kQrCols + t] + part[3 * kQrCols + t]));
    __syncthreads();
    if (k < n) {
      const double wk = w[k];
#pragma unroll
      for (int q = 0; q < kQrRPT; ++q) reg[q] = fma(-wk, vcol[seg + 4 * q], reg[q]);
    }
    __syncthreads();  // part is rewritten by the next step
  }
#pragma unroll
  for (int q = 0; q < kQrRPT; ++q) {
    const int i = seg + 4 * q;
    if (k < n && i < m) Q[(off + i) + (long long)k * ldq] = reg[q];
  }
}

// chunk count of one TSQR level of M rows
static int qr_nchunks(long long M) { return (int)((M + kQrRows - 1) / kQrRows); }

void tsqr_work(long long rows, int n, size_t* stack_elems, size_t* tau_elems) {
  n = std::min(n, kQrCols);
  size_t st = 0, ta = 0;
  long long M = rows;
  for (;;) {
    const int nch = qr_nchunks(M);
    ta += (size_t)nch * n;
    if (nch == 1) break;
    M = (long long)nch * n;
    st += (size_t)M * n;
  }
  *stack_elems = st;
  *tau_elems = ta;
}

// A (rows x n, n <= 64) = Q R, Q with ld ldq, R n x n (ld n, rows >=
// min(rows, n) zero).  A and Q must not alias.
static void tsqr(long long rows, int n, const double* A, long long lda, double* Q, long long ldq,
                 double* R, const OrthScratch& s, hipStream_t st) {
  struct Level {
    long long M;
    int nch;
    double* V;
    long long ldv;
    double* tau;
  };
  Level lv[40];
  int L = 0;
  long long M = rows;
  const double* in = A;
  long long ldin = lda;
  double* V = s.Q1;  // level 0 reflectors (rows x n)
  long long ldv = rows;
  double* stack = s.hw;
  double* tp = s.htau;
  for (;;) {
    const int nch = qr_nchunks(M);
    const bool top = nch == 1;
    double* Rout = top ? R : stack;
    const long long ldr = top ? n : (long long)nch * n;
    hipLaunchKernelGGL(k_hqr_chunk, dim3((unsigned)nch), dim3(256), 0, st, M, n, nch, in, ldin, V,
                       ldv, tp, Rout, ldr);
    PW_LAUNCH_CHECK();
    if (L >= 40) fail(PW_EINVAL, "TSQR level count exceeded");
    lv[L++] = Level{M, nch, V, ldv, tp};
    if (top) break;
    tp += (size_t)nch * n;
    M = (long long)nch * n;
    in = stack;
    ldin = M;
    V = stack;  // the next level factors its input in place
    ldv = M;
    stack += (size_t)M * n;
  }
  const double* Qup = nullptr;
  long long ldu = 0;
  for (int l = L - 1; l >= 0; --l) {
    double* out = l == 0 ? Q : lv[l].V;
    const long long ldo = l == 0 ? ldq : lv[l].ldv;
    hipLaunchKernelGGL(k_hqr_formq, dim3((unsigned)lv[l].nch), dim3(256), 0, st, lv[l].M, n,
                       lv[l].nch, (const double*)lv[l].V, lv[l].ldv, (const double*)lv[l].tau, Qup,
                       ldu, out, ldo);
    PW_LAUNCH_CHECK();
    Qup = out;
    ldu = ldo;
  }
}

void pchol_factors(int n, const double* G, double rel, double abs_thr, double* T, double* R,
                   double* info, hipStream_t st) {
  if (n > kCholMax) fail(PW_EINVAL, "a Cholesky QR block holds at most 64 columns");
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pchol_factors, dim3(1), dim3(1024), 0, st, n, G, rel, abs_thr, T, R, info);
  PW_LAUNCH_CHECK();
}

// Two ways to factor A = Q R inside Algorithm 1.  Cholesky QR twice
// (Gram matrix, pivoted Cholesky, Q = A T, repeated on Q) costs a few
// GEMMs and is as accurate as Householder QR when A is well conditioned
// (kappa(A) below about 1 / sqrt(11 (rows n + n^2) eps)); beyond that its
// Gram matrix loses the small directions, and the Householder TSQR above
// is used.  orth_begin forms the Gram matrix and its pivoted Cholesky
// factor (with a report of the smallest pivot), orth_choose reads the
// report (synchronising the stream), orth_finish completes either method.
// With FP32 states the data carry rounding of ~6e-8 of their size, so
// the truncation of Cholesky QR at ~3e-8 loses nothing and it is always
// used (gram_enough).
void orth_begin(long long rows, int n, const double* A, long long lda, const OrthScratch& s,
                hipStream_t st) {
  if (n <= 0 || n > kCholMax) return;
  gemm_tn(rows, n, n, 1.0, A, lda, A, lda, 0.0, s.gram, n, s.work, s.work_elems, st);
  pchol_factors(n, s.gram, 1e-15, 1e-290, s.T, s.R1, s.info, st);
}

bool orth_choose(long long rows, int n, const OrthScratch& s, hipStream_t st) {
  if (n <= 0 || n > kCholMax) return false;
  if (s.gram_enough) return true;
  double h[2] = {0.0, 0.0};
  PW_HIP(hipMemcpyAsync(h, s.info, sizeof(h), hipMemcpyDeviceToHost, st));
  PW_HIP(hipStreamSynchronize(st));
  const double thr = 11.0 * ((double)rows * n + (double)n * n) * 2.220446049250313e-16;
  // kept rank n and sigma_min^2 / sigma_max^2 (the smallest pivot ratio)
  // at least 100 thr: Cholesky QR twice is backward stable there
  return (int)h[0] == n && h[1] > 100.0 * thr;
}

void orth_finish(long long rows, int n, const double* A, long long lda, double* Q, long long ldq,
                 double* R, const OrthScratch& s, bool cholqr, hipStream_t st) {
  if (n <= 0) return;
  if (cholqr) {
    gemm_nn(rows, n, n, 1.0, A, lda, s.T, n, 0.0, s.Q1, rows, st);
    gemm_tn(rows, n, n, 1.0, s.Q1, rows, s.Q1, rows, 0.0, s.gram, n, s.work, s.work_elems, st);
    pchol_factors(n, s.gram, 0.0, 0.25, s.T, s.R2, nullptr, st);
    gemm_nn(rows, n, n, 1.0, s.Q1, rows, s.T, n, 0.0, Q, ldq, st);
    gemm_small(n, n, n, 1.0, s.R2, n, false, s.R1, n, false, 0.0, R, n, st);
    return;
  }
  if (n <= kQrCols) {
    tsqr(rows, n, A, lda, Q, ldq, R, s, st);
    return;
  }
  // More than 64 columns: column blocks of 64 by block classical
  // Gram-Schmidt, projection passes each followed by a Householder QR of
  // the block:
  //   W = A_b - Qp C1 = Q1 R1;  Q1 - Qp C2 = Q2 R2;  Q2 - Qp C3 = Q_b R3
  //   => A_b = Qp (C1 + C2 R1 + C3 R2 R1) + Q_b (R3 R2 R1)
  // Two passes are not enough when A_b is numerically rank deficient
  // against Qp: then Q1 - Qp C2 is ill conditioned, its QR amplifies the
  // rounding left along Qp (orthogonality lost to ~1e-9 on such data), and
  // the third pass, applied to a block already orthogonal to Qp but for
  // that amplified rounding, restores it to rounding level.
  // With fewer rows than columns only the first m = rows columns are
  // factored that way (their Q, noise directions included, is a complete
  // orthonormal basis); the remaining columns get R = Q^T A and zero Q
  // columns, as an economy Householder QR of a wide matrix gives.
  const int m = (int)std::min<long long>(rows, n);
  if (m < n && ldq != rows) fail(PW_EINVAL, "wide orthonormalisation needs ldq = rows");
  fill(R, (long long)n * n, 0.0, st);
  for (int b0 = 0; b0 < m; b0 += kQrCols) {
    const int nb = std::min(kQrCols, m - b0);
    double* Qb = Q + (long long)b0 * ldq;
    double* Rtop = R + (long long)b0 * n;      // rows 0..b0 of the block's columns
    double* Rbb = R + b0 + (long long)b0 * n;  // diagonal block
    PW_HIP(hipMemcpy2DAsync(s.W, sizeof(double) * rows, A + (long long)b0 * lda,
                            sizeof(double) * lda, sizeof(double) * rows, nb,
                            hipMemcpyDeviceToDevice, st));
    if (b0 > 0) {
      gemm_tn(rows, b0, nb, 1.0, Q, ldq, s.W, rows, 0.0, Rtop, n, s.work, s.work_elems, st);
      gemm_nn(rows, nb, b0, -1.0, Q, ldq, Rtop, n, 1.0, s.W, rows, st);
    }
    tsqr(rows, nb, s.W, rows, Qb, ldq, s.R1, s, st);
    if (b0 > 0) {
      gemm_tn(rows, b0, nb, 1.0, Q, ldq, Qb, ldq, 0.0, s.C, b0, s.work, s.work_elems, st);
      gemm_nn(rows, nb, b0, -1.0, Q, ldq, s.C, b0, 1.0, Qb, ldq, st);
      gemm_small(b0, nb, nb, 1.0, s.C, b0, false, s.R1, nb, false, 1.0, Rtop, n, st);
      PW_HIP(hipMemcpy2DAsync(s.W, sizeof(double) * rows, Qb, sizeof(double) * ldq,
                              sizeof(double) * rows, nb, hipMemcpyDeviceToDevice, st));
      tsqr(rows, nb, s.W, rows, Qb, ldq, s.R2, s, st);
      gemm_small(nb, nb, nb, 1.0, s.R2, nb, false, s.R1, nb, false, 0.0, Rbb, n, st);
      // third pass: Rtop += C3 (R2 R1), Rbb = R3 (R2 R1)
      gemm_tn(rows, b0, nb, 1.0, Q, ldq, Qb, ldq, 0.0, s.C, b0, s.work, s.work_elems, st);
      gemm_nn(rows, nb, b0, -1.0, Q, ldq, s.C, b0, 1.0, Qb, ldq, st);
      gemm_small(b0, nb, nb, 1.0, s.C, b0, false, Rbb, (int)n, false, 1.0, Rtop, n, st);
      copy_block(nb, nb, Rbb, n, s.R1, nb, st);
      PW_HIP(hipMemcpy2DAsync(s.W, sizeof(double) * rows, Qb, sizeof(double) * ldq,
                              sizeof(double) * rows, nb, hipMemcpyDeviceToDevice, st));
      tsqr(rows, nb, s.W, rows, Qb, ldq, s.R2, s, st);
      gemm_small(nb, nb, nb, 1.0, s.R2, nb, false, s.R1, nb, false, 0.0, Rbb, n, st);
    } else {
      copy_block(nb, nb, s.R1, nb, Rbb, n, st);
    }
  }
  if (m < n) {
    gemm_tn(rows, m, n - m, 1.0, Q, ldq, A + (long long)m * lda, lda, 0.0, R + (long long)m * n,
            n, s.work, s.work_elems, st);
    fill(Q + (long long)m * ldq, (long long)(n - m) * ldq, 0.0, st);
  }
}


void svd_jacobi(int n, const double* H, double* X, double* Y, double* sig, double tol,
                int* rank_dev, double* Hw, double* Vw, int* counters, hipStream_t st) {
  if (n <= 0) {
    PW_HIP(hipMemsetAsync(rank_dev, 0, sizeof(int), st));
    return;
  }
  const long long nn = (long long)n * n;
  // workspace: Hw = two n x n buffers, then n + n (sort) + 8 + 8 (norm of H)
  // + n (column norms) doubles; Vw = two n x n buffers.  The block version
  // gathers the columns of H and V into the other buffer before each sweep.
  double* Hc = Hw;
  double* Hn = Hw + nn;
  double* Vc = Vw;
  double* Vn = Vw + nn;
  double* ws = Hw + 2 * nn;
  double* sig_u = ws;
  int* pos = (int*)(sig_u + n);
  double* fro2 = ws + 2 * n + 8;
  double* cnorm2 = ws + 2 * n + 16;
  PW_HIP(hipMemcpyAsync(Hc, H, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_identity, dim3(nblocks(nn)), dim3(kTB), 0, st, n, Vc);
  PW_LAUNCH_CHECK();
  const int np = (n + 1) & ~1;
  const int maxsweeps = 40;
  PW_HIP(hipMemsetAsync(counters, 0, sizeof(int) * maxsweeps, st));
  const unsigned blocks = (unsigned)((np / 2 + 3) / 4);
  frob_norm2(Hc, n, n, n, sig, fro2, st);  // sig used as partials (>= 512 doubles)
  // block version from two block pairs up (columns in blocks of kJB)
  const int nb = (n + kJB - 1) / kJB;
  const int npb = nb + (nb & 1);
  const bool blocked = n >= 2 * kJC && n <= kJRows && !getenv("PW_JACOBI_COLUMNS");
  if (blocked) {
    hipLaunchKernelGGL(k_col_norms, dim3((n + 3) / 4), dim3(256), 0, st, n, (const double*)Hc,
                       cnorm2);
    PW_LAUNCH_CHECK();
  }
  for (int sw = 0; sw < maxsweeps; ++sw) {
    if (blocked) {
      // each sweep visits the columns in descending order of their norms
      // (blocks of similar norms), which saves sweeps; the same permutation
      // of the columns of H and V keeps H0 V = H
      hipLaunchKernelGGL(k_norm_order, dim3(1), dim3(1024), 0, st, n, (const double*)cnorm2, pos);
      PW_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_gather_cols2, dim3(std::min(nblocks(nn), 2048u)), dim3(kTB), 0, st, n,
                         (const int*)pos, (const double*)Hc, Hn, (const double*)Vc, Vn);
      PW_LAUNCH_CHECK();
      std::swap(Hc, Hn);
      std::swap(Vc, Vn);
      for (int round = 0; round < npb - 1; ++round) {
        hipLaunchKernelGGL(k_jacobi_block<kJRows>, dim3(8 * ((npb / 2 + 7) / 8)), dim3(kJT), 0,
                           st, n, npb, round, Hc, Vc, counters + sw, (const double*)fro2, cnorm2);
        PW_LAUNCH_CHECK();
      }
    } else {
      for (int round = 0; round < np - 1; ++round) {
        hipLaunchKernelGGL(k_jacobi_round, dim3(blocks), dim3(256), 0, st, n, np, round, Hc, Vc,
                           counters + sw, (const double*)fro2);
        PW_LAUNCH_CHECK();
      }
    }
    int h = 0;
    PW_HIP(hipMemcpyAsync(&h, counters + sw, sizeof(int), hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    if (h == 0) break;
  }
  hipLaunchKernelGGL(k_col_norms, dim3((n + 3) / 4), dim3(256), 0, st, n, (const double*)Hc, sig_u);
  PW_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sort_rank, dim3(1), dim3(1024), 0, st, n, (const double*)sig_u, pos, tol,
                     rank_dev, sig);
  PW_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scatter_svd, dim3(nblocks(nn)), dim3(kTB), 0, st, n, (const double*)Hc,
                     (const double*)Vc, (const int*)pos, (const double*)sig_u, X, Y);
  PW_LAUNCH_CHECK();
}

// Many matrices at once: each is set up, swept and finished as by
// svd_jacobi (same kernels per block pair, same column order, same stopping
// rule per matrix), but every round is one launch over the block pairs of
// all matrices still sweeping, and one read-back per sweep serves all.
// Matrices outside the block path's sizes are handled by svd_jacobi.
void svd_jacobi_multi(const std::vector<SvdJob>& jobs, void* jobs_dev, int* counts_dev,
                      hipStream_t st) {
  constexpr int maxsweeps = 40;
  struct State {
    JacobiJob j;
    int* counters;
    double* sig_u;
    size_t qi;  // index of the job
  };
  std::vector<State> act, done;
  const bool force_columns = getenv("PW_JACOBI_COLUMNS") != nullptr;
  for (size_t qi = 0; qi < jobs.size(); ++qi) {
    const SvdJob& q = jobs[qi];
    const int n = q.n;
    if (n < 2 * kJC || n > kJRows || force_columns) {
      svd_jacobi(n, q.H, q.X, q.Y, q.sig, q.tol, q.rank_dev, q.Hw, q.Vw, q.counters, st);
      continue;
    }
    const long long nn = (long long)n * n;
    State a;
    a.j.n = n;
    const int nb = (n + kJB - 1) / kJB;
    a.j.npb = nb + (nb & 1);
    a.j.block_begin = 0;
    a.j.Hc = q.Hw;
    a.j.Hn = q.Hw + nn;
    a.j.Vc = q.Vw;
    a.j.Vn = q.Vw + nn;
    double* ws = q.Hw + 2 * nn;
    a.sig_u = ws;
    a.j.pos = (int*)(ws + n);
    double* fro2 = ws + 2 * n + 8;
    a.j.fro2 = fro2;
    a.j.cnorm2 = ws + 2 * n + 16;
    a.j.counter = nullptr;
    a.counters = q.counters;
    a.qi = qi;
    PW_HIP(hipMemcpyAsync(a.j.Hc, q.H, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_identity, dim3(nblocks(nn)), dim3(kTB), 0, st, n, a.j.Vc);
    PW_LAUNCH_CHECK();
    PW_HIP(hipMemsetAsync(q.counters, 0, sizeof(int) * maxsweeps, st));
    frob_norm2(a.j.Hc, n, n, n, q.sig, fro2, st);
    hipLaunchKernelGGL(k_col_norms, dim3((n + 3) / 4), dim3(256), 0, st, n,
                       (const double*)a.j.Hc, a.j.cnorm2);
    PW_LAUNCH_CHECK();
    act.push_back(a);
  }
  std::vector<JacobiJob> ga, ro;  // host copies of the uploaded records (alive until the sync)
  JacobiJob* dga = (JacobiJob*)jobs_dev;
  JacobiJob* dro = dga + jobs.size();
  std::vector<int> cnt;
  for (int sw = 0; sw < maxsweeps && !act.empty(); ++sw) {
    const int na = (int)act.size();
    ga.clear();
    long long nnmax = 0;
    for (State& a : act) {
      a.j.counter = a.counters + sw;
      ga.push_back(a.j);
      nnmax = std::max(nnmax, (long long)a.j.n * a.j.n);
    }
    PW_HIP(hipMemcpyAsync(dga, ga.data(), sizeof(JacobiJob) * na, hipMemcpyHostToDevice, st));
    // this sweep's column order and the gathered columns
    hipLaunchKernelGGL(k_norm_order_multi, dim3((unsigned)na), dim3(1024), 0, st,
                       (const JacobiJob*)dga);
    PW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gather_cols2_multi, dim3(std::min(nblocks(nnmax), 2048u), (unsigned)na),
                       dim3(kTB), 0, st, (const JacobiJob*)dga);
    PW_LAUNCH_CHECK();
    ro.clear();
    int blocks = 0, maxr = 0, nmax = 0;
    for (State& a : act) {
      std::swap(a.j.Hc, a.j.Hn);
      std::swap(a.j.Vc, a.j.Vn);
      a.j.block_begin = blocks;
      blocks += 8 * ((a.j.npb / 2 + 7) / 8);
      maxr = std::max(maxr, a.j.npb - 1);
      nmax = std::max(nmax, a.j.n);
      ro.push_back(a.j);
    }
    PW_HIP(hipMemcpyAsync(dro, ro.data(), sizeof(JacobiJob) * na, hipMemcpyHostToDevice, st));
    for (int round = 0; round < maxr; ++round) {
      if (nmax <= kJRowsSmall)
        hipLaunchKernelGGL(k_jacobi_block_multi<kJRowsSmall>, dim3((unsigned)blocks), dim3(kJT), 0,
                           st, (const JacobiJob*)dro, na, round);
      else
        hipLaunchKernelGGL(k_jacobi_block_multi<kJRows>, dim3((unsigned)blocks), dim3(kJT), 0, st,
                           (const JacobiJob*)dro, na, round);
      PW_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_collect_counters, dim3(nblocks(na)), dim3(kTB), 0, st,
                       (const JacobiJob*)dro, na, counts_dev);
    PW_LAUNCH_CHECK();
    cnt.assign((size_t)na, 0);
    PW_HIP(hipMemcpyAsync(cnt.data(), counts_dev, sizeof(int) * na, hipMemcpyDeviceToHost, st));
    PW_HIP(hipStreamSynchronize(st));
    std::vector<State> keep;
    for (int i = 0; i < na; ++i) (cnt[(size_t)i] == 0 ? done : keep).push_back(act[(size_t)i]);
    act.swap(keep);
  }
  for (const State& a : act) done.push_back(a);  // the sweep limit reached
  // singular values, order and rank of every matrix, as svd_jacobi
  for (const State& a : done) {
    const SvdJob& q = jobs[a.qi];
    const int n = a.j.n;
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(k_col_norms, dim3((n + 3) / 4), dim3(256), 0, st, n, (const double*)a.j.Hc,
                       a.sig_u);
    PW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sort_rank, dim3(1), dim3(1024), 0, st, n, (const double*)a.sig_u,
                       a.j.pos, q.tol, q.rank_dev, q.sig);
    PW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scatter_svd, dim3(nblocks(nn)), dim3(kTB), 0, st, n,
                       (const double*)a.j.Hc, (const double*)a.j.Vc, (const int*)a.j.pos,
                       (const double*)a.sig_u, q.X, q.Y);
    PW_LAUNCH_CHECK();
  }
}

size_t svd_multi_job_bytes() { return sizeof(JacobiJob); }

// one step of the serial recurrence: t_n = b_n + M t_{n-1} (M: dim x dim,
// column-major).  A workgroup owns 64 rows (lane = row); its 16 waves sum
// interleaved column groups with four independent accumulators each, and
// the partial sums are combined in a fixed order through LDS.
constexpr int kRecWaves = 16;
__global__ __launch_bounds__(64 * kRecWaves) void k_rec_step(int dim, const double* M,
                                                              const double* tprev,
                                                              const double* b, double* t) {
  __shared__ double part[kRecWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + lane;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (row < dim) {
    int j = wave;
    for (; j + 3 * kRecWaves < dim; j += 4 * kRecWaves) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int jj = j + k * kRecWaves;
        acc[k] = fma(M[row + (long long)jj * dim], tprev[jj], acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {  // at most three columns remain
      const int jj = j + k * kRecWaves;
      if (jj < dim) acc[k] = fma(M[row + (long long)jj * dim], tprev[jj], acc[k]);
    }
  }
  part[wave][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (wave == 0 && row < dim) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kRecWaves; ++w) s += part[w][lane];
    t[row] = b[row] + s;
  }
}

void recurrence(int dim, int N, const double* M, const double* b, double* t, RecScratch rs,
                hipStream_t st) {
  if (dim > 64 && N > 1) {
    // large dim: N - 1 matrix-vector steps cost less than the doubling
    // scan's log2(N) dim x dim products
    PW_HIP(hipMemcpyAsync(t, b, sizeof(double) * dim, hipMemcpyDeviceToDevice, st));
    for (int n = 1; n < N; ++n) {
      hipLaunchKernelGGL(k_rec_step, dim3((dim + 63) / 64), dim3(64 * kRecWaves), 0, st, dim, M,
                         (const double*)(t + (long long)(n - 1) * dim),
                         b + (long long)n * dim, t + (long long)n * dim);
      PW_LAUNCH_CHECK();
    }
    return;
  }
  // Hillis-Steele doubling: with t^(0)_n = b_n and P = M,
  //   t^(l+1)_n = t^(l)_n + P^(2^l) t^(l)_{n - 2^l}   (n >= 2^l)
  // gives t_n = sum_{j <= n} M^(n-j) b_j after ceil(log2 N) levels; each
  // level is one matrix-core GEMM (and one squaring of P).
  if (dim <= 0 || N <= 0) return;
  const long long dn = (long long)dim * N;
  double* ta = rs.ta;
  double* tb = rs.tb;
  double* P = rs.P0;
  double* Pn = rs.P1;
  PW_HIP(hipMemcpyAsync(ta, b, sizeof(double) * dn, hipMemcpyDeviceToDevice, st));
  PW_HIP(hipMemcpyAsync(P, M, sizeof(double) * dim * dim, hipMemcpyDeviceToDevice, st));
  for (int s = 1; s < N; s *= 2) {
    PW_HIP(hipMemcpyAsync(tb, ta, sizeof(double) * dn, hipMemcpyDeviceToDevice, st));
    gemm_nn(dim, N - s, dim, 1.0, P, dim, ta, dim, 1.0, tb + (long long)s * dim, dim, st);
    std::swap(ta, tb);
    if (2 * s < N) {
      gemm_nn(dim, dim, dim, 1.0, P, dim, P, dim, 0.0, Pn, dim, st);
      std::swap(P, Pn);
    }
  }
  PW_HIP(hipMemcpyAsync(t, ta, sizeof(double) * dn, hipMemcpyDeviceToDevice, st));
}

void add_diag(int n, int r, const double* S, double* H, int ldh, hipStream_t st) {
  (void)n;
  if (r <= 0) return;
  hipLaunchKernelGGL(k_add_diag, dim3(nblocks(r)), dim3(kTB), 0, st, r, S, H, ldh);
  PW_LAUNCH_CHECK();
}

void copy_block(int m, int n, const double* src, long long lds, double* dst, long long ldd,
                hipStream_t st) {
  const long long mn = (long long)m * n;
  if (mn <= 0) return;
  hipLaunchKernelGGL(k_copy_block, dim3(nblocks(mn)), dim3(kTB), 0, st, m, n, src, lds, dst, ldd);
  PW_LAUNCH_CHECK();
}

void fill(double* p, long long n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kTB), 0, st, p, n, v);
  PW_LAUNCH_CHECK();
}

void vec_sum(const double* x, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kTB), 0, st, x, n, out);
  PW_LAUNCH_CHECK();
}

void frob_norm2(const double* A, long long rows, int cols, long long lda, double* partials,
                double* out, hipStream_t st) {
  const int nb = 512;
  hipLaunchKernelGGL(k_sumsq_cols, dim3(nb), dim3(kTB), 0, st, A, rows, cols, lda, partials);
  PW_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kTB), 0, st, (const double*)partials, nb, out);
  PW_LAUNCH_CHECK();
}

}  // namespace pw
