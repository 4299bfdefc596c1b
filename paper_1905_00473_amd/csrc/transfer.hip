// Grid transfer and energy components:
//  * restriction R (pointwise, coarse node J = fine node ratio*J, Sec. 3.1)
//  * energy components Lambda[U, P] = [nabla_h U ; P / c] (eqs. matrixF /
//    matrixG) with the central gradient of order 2, 4, 6 or 8
//  * trigonometric interpolation I (the Fourier interpolation of Sec. 6)
//    evaluated as a separable polyphase convolution with the periodic
//    Dirichlet-type kernel of the zero-padded spectrum, the Nyquist
//    coefficient split between +n/2 and -n/2
//  * Lambda^dag (Algorithm 2, eq. gradient2coordinate) through separable
//    discrete Fourier transforms on the coarse grid
//  * the adjoint of Lambda and the discrete wave energy reduction
#include <cmath>

#include "pw_internal.h"

namespace pw {
namespace {

constexpr int kTB = 256;

inline unsigned nblocks(long long n, int tb = kTB) {
  return (unsigned)((n + tb - 1) / tb);
}

__device__ __forceinline__ int wrapi(int g, int n) {
  g %= n;
  return g < 0 ? g + n : g;
}

struct GridArg {
  int dim, nx, ny, nz;
  double dx;
};

inline GridArg garg(const Grid& g) { return GridArg{g.dim, g.n[0], g.n[1], g.n[2], g.dx}; }

// weight b_j of f(x + j h) - f(x - j h) in the central first difference of
// order 2m = order (j = 1..m): b_j = 2 (-1)^(j+1) (m!)^2 / (j (m-j)! (m+j)!),
// the coefficients of the Taylor-matched antisymmetric stencil
__device__ __forceinline__ double fd_weight(int order, int j) {
  switch (order) {
    case 2: return 0.5;
    case 4: return j == 1 ? 2.0 / 3.0 : -1.0 / 12.0;
    case 6: return j == 1 ? 3.0 / 4.0 : (j == 2 ? -3.0 / 20.0 : 1.0 / 60.0);
    default:  // 8
      return j == 1 ? 4.0 / 5.0 : (j == 2 ? -1.0 / 5.0 : (j == 3 ? 4.0 / 105.0 : -1.0 / 280.0));
  }
}

// central first difference of order 2, 4, 6 or 8 along axis `ax` at coarse
// point (X, Y, Z) of a field sampled at fine index ratio * coarse index
template <typename T>
__device__ __forceinline__ double grad_at(const T* f, int ax, int X, int Y, int Z, const GridArg& c,
                                          int ratio, int fnx, int fny, int order) {
  auto val = [&](int dxo) -> double {
    int x = X, y = Y, z = Z;
    if (ax == 0) x = wrapi(X + dxo, c.nx);
    if (ax == 1) y = wrapi(Y + dxo, c.ny);
    if (ax == 2) z = wrapi(Z + dxo, c.nz);
    const long long gi =
        (long long)x * ratio + (long long)fnx * ((long long)y * ratio + (long long)fny * z * ratio);
    return (double)f[gi];
  };
  double d = 0.0;
  for (int j = 1; j <= order / 2; ++j) d += fd_weight(order, j) * (val(j) - val(-j));
  return d / c.dx;
}

// order 0 (spectral gradient): the gradient rows are left to the caller
// and the restricted u goes to ures (nstates x coarse points) instead
template <typename T>
__global__ void k_energy_columns(const T* u, const T* p, long long sstride, GridArg c, int ratio,
                                 int fnx, int fny, const double* cc, int order, double* out,
                                 long long ldo, int nstates, double* ures) {
  const long long nc = (long long)c.nx * c.ny * c.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nstates) return;
  const int s = (int)(t / nc);
  const long long J = t - (long long)s * nc;
  const int X = (int)(J % c.nx);
  const int Y = (int)((J / c.nx) % c.ny);
  const int Z = (int)(J / ((long long)c.nx * c.ny));
  const T* us = u + (long long)s * sstride;
  const T* ps = p + (long long)s * sstride;
  double* o = out + (long long)s * ldo;
  const long long gi =
      (long long)X * ratio + (long long)fnx * ((long long)Y * ratio + (long long)fny * Z * ratio);
  if (order > 0) {
    for (int a = 0; a < c.dim; ++a)
      o[a * nc + J] = grad_at(us, a, X, Y, Z, c, ratio, fnx, fny, order);
  } else {
    ures[(long long)s * nc + J] = (double)us[gi];
  }
  o[c.dim * nc + J] = (double)ps[gi] / cc[J];
}

template <typename T>
__global__ void k_restrict_diff(const T* au, const T* ap, const T* bu, const T* bp,
                                long long sstride, GridArg c, int ratio, int fnx, int fny,
                                double* out, long long ldo, int nstates) {
  const long long nc = (long long)c.nx * c.ny * c.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nstates) return;
  const int s = (int)(t / nc);
  const long long J = t - (long long)s * nc;
  const int X = (int)(J % c.nx);
  const int Y = (int)((J / c.nx) % c.ny);
  const int Z = (int)(J / ((long long)c.nx * c.ny));
  const long long gi = (long long)s * sstride + (long long)X * ratio +
                       (long long)fnx * ((long long)Y * ratio + (long long)fny * Z * ratio);
  double* o = out + (long long)s * ldo;
  o[J] = (double)au[gi] - (double)bu[gi];
  o[nc + J] = (double)ap[gi] - (double)bp[gi];
}

template <typename T>
__global__ void k_restrict_fields(const T* in, long long sin, GridArg c, int ratio, int fnx,
                                  int fny, T* out, long long sout, int nfields) {
  const long long nc = (long long)c.nx * c.ny * c.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nfields) return;
  const int s = (int)(t / nc);
  const long long J = t - (long long)s * nc;
  const int X = (int)(J % c.nx);
  const int Y = (int)((J / c.nx) % c.ny);
  const int Z = (int)(J / ((long long)c.nx * c.ny));
  const long long gi = (long long)s * sin + (long long)X * ratio +
                       (long long)fnx * ((long long)Y * ratio + (long long)fny * Z * ratio);
  out[(long long)s * sout + J] = in[gi];
}

template <typename Tin, typename Tout>
__global__ void k_cast(const Tin* in, Tout* out, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = (Tout)in[t];
}

// one axis of the polyphase trigonometric interpolation:
// in (outer, nc, inner) -> out (outer, nc*ratio, inner) per field.
// Fine index j = ratio*J + s takes sum_m tab[s*nc + (J-m) mod nc] in[m];
// s = 0 copies in[J] (R I = 1 exactly).  FINAL: out = (T)(v + acc).
template <typename Tin, typename Tout, bool FINAL>
__global__ void k_interp_axis(const Tin* in, long long sin, Tout* out, long long sout,
                              const Tout* v, const double* tab, int outer, int nc, int ratio,
                              int inner, int nfields) {
  const int nf = nc * ratio;
  const long long per = (long long)outer * nf * inner;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nfields) return;
  const int f = (int)(t / per);
  long long r = t - (long long)f * per;
  const int i = (int)(r % inner);
  r /= inner;
  const int j = (int)(r % nf);
  const int o = (int)(r / nf);
  const int J = j / ratio;
  const int s = j - J * ratio;
  const Tin* src = in + (long long)f * sin + (long long)o * nc * inner + i;
  double acc;
  if (s == 0) {
    acc = (double)src[(long long)J * inner];
  } else {
    const double* w = tab + (long long)s * nc;
    acc = 0.0;
    for (int m = 0; m < nc; ++m) {
      int dd = J - m;
      if (dd < 0) dd += nc;
      acc += w[dd] * (double)src[(long long)m * inner];
    }
  }
  const long long oi = (long long)f * sout + ((long long)o * nf + j) * inner + i;
  if (FINAL) {
    const double base = v ? (double)v[oi] : 0.0;
    out[oi] = (Tout)(base + acc);
  } else {
    out[oi] = (Tout)acc;
  }
}

// Register-blocked variant for a compile-time ratio R: a thread produces
// the R phases of RJ consecutive coarse intervals J, so every input value
// loaded feeds R*RJ accumulators; the polyphase table sits in LDS.
template <typename Tin, typename Tout, bool FINAL, int R, int RJ>
__global__ __launch_bounds__(256) void k_interp_axis_rb(const Tin* in, long long sin, Tout* out,
                                                         long long sout, const Tout* v,
                                                         const double* tab, int outer, int nc,
                                                         int inner, int nfields) {
  extern __shared__ double wt[];
  for (int t = threadIdx.x; t < R * nc; t += blockDim.x) wt[t] = tab[t];
  __syncthreads();
  const int njb = (nc + RJ - 1) / RJ;
  const long long per = (long long)outer * njb * inner;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nfields) return;
  const int f = (int)(t / per);
  long long rr = t - (long long)f * per;
  const int i = (int)(rr % inner);
  rr /= inner;
  const int jb = (int)(rr % njb);
  const int o = (int)(rr / njb);
  const int J0 = jb * RJ;
  const Tin* src = in + (long long)f * sin + (long long)o * nc * inner + i;
  double acc[RJ][R];
#pragma unroll
  for (int a = 0; a < RJ; ++a)
#pragma unroll
    for (int s = 0; s < R; ++s) acc[a][s] = 0.0;
  // acc[a][s] += w_s[(J0 + a - m) mod nc] x_m.  Over RJ consecutive m the
  // index J0 + a - m takes 2 RJ - 1 values, so a block of RJ inputs needs
  // 2 RJ - 1 weights per phase from LDS instead of RJ^2.
  int m = 0;
  for (; m + RJ <= nc; m += RJ) {
    double x[RJ];
#pragma unroll
    for (int u = 0; u < RJ; ++u) x[u] = (double)src[(long long)(m + u) * inner];
#pragma unroll
    for (int s = 1; s < R; ++s) {
      double w[2 * RJ - 1];  // w[k] = w_s[(J0 - m + k - (RJ - 1)) mod nc]
#pragma unroll
      for (int k = 0; k < 2 * RJ - 1; ++k) {
        int dd = J0 - m + k - (RJ - 1);
        dd += dd < 0 ? nc : 0;
        dd -= dd >= nc ? nc : 0;
        w[k] = wt[s * nc + dd];
      }
#pragma unroll
      for (int u = 0; u < RJ; ++u)
#pragma unroll
        for (int a = 0; a < RJ; ++a) acc[a][s] += w[a - u + RJ - 1] * x[u];
    }
  }
  for (; m < nc; ++m) {
    const double x = (double)src[(long long)m * inner];
#pragma unroll
    for (int a = 0; a < RJ; ++a) {
      int dd = (J0 + a - m) % nc;  // J0 + a may pass nc (discarded outputs)
      if (dd < 0) dd += nc;
#pragma unroll
      for (int s = 1; s < R; ++s) acc[a][s] += wt[s * nc + dd] * x;
    }
  }
  const int nf = nc * R;
#pragma unroll
  for (int a = 0; a < RJ; ++a) {
    const int J = J0 + a;
    if (J >= nc) break;
    acc[a][0] = (double)src[(long long)J * inner];  // R I = 1 exactly
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const long long oi = (long long)f * sout + ((long long)o * nf + (long long)J * R + s) * inner + i;
      if (FINAL) {
        const double base = v ? (double)v[oi] : 0.0;
        out[oi] = (Tout)(base + acc[a][s]);
      } else {
        out[oi] = (Tout)acc[a][s];
      }
    }
  }
}

template <typename Tin, typename Tout, bool FINAL>
void interp_pass(const Tin* in, long long sin, Tout* out, long long sout, const Tout* v,
                 const double* tab, int outer, int nc, int ratio, int inner, int nfields,
                 hipStream_t st) {
  constexpr int RJ = 8;
  if (ratio == 4 || ratio == 2) {
    const long long n = (long long)outer * ((nc + RJ - 1) / RJ) * inner * nfields;
    const size_t smem = sizeof(double) * (size_t)ratio * nc;
    if (ratio == 4)
      hipLaunchKernelGGL((k_interp_axis_rb<Tin, Tout, FINAL, 4, RJ>), dim3(nblocks(n)), dim3(kTB),
                         smem, st, in, sin, out, sout, v, tab, outer, nc, inner, nfields);
    else
      hipLaunchKernelGGL((k_interp_axis_rb<Tin, Tout, FINAL, 2, RJ>), dim3(nblocks(n)), dim3(kTB),
                         smem, st, in, sin, out, sout, v, tab, outer, nc, inner, nfields);
  } else {
    const long long n = (long long)outer * nc * ratio * inner * nfields;
    hipLaunchKernelGGL((k_interp_axis<Tin, Tout, FINAL>), dim3(nblocks(n)), dim3(kTB), 0, st, in,
                       sin, out, sout, v, tab, outer, nc, ratio, inner, nfields);
  }
  PW_LAUNCH_CHECK();
}

// DFT along one axis of length n with stride `inner`:
// out[b][o][k][i] = sum_j in[b][o][j][i] * tw[(j*k) mod n] (conj if INV).
// IN_REAL: input is real, batch b at offset (b/sub)*s_hi + (b%sub)*s_lo.
// OUT_REAL: output real part * scale, batch b at offset b*s_out.
template <bool IN_REAL, bool OUT_REAL, bool INV>
__global__ void k_dft_axis(const void* inp, long long s_hi, long long s_lo, int sub,
                           long long s_in_c, void* outp, long long s_out, const double2* tw,
                           int outer, int n, int inner, int nbatch, double scale) {
  const long long per = (long long)outer * n * inner;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nbatch) return;
  const int b = (int)(t / per);
  long long r = t - (long long)b * per;
  const int i = (int)(r % inner);
  r /= inner;
  const int k = (int)(r % n);
  const int o = (int)(r / n);
  double re = 0.0, im = 0.0;
  const long long off = (long long)o * n * inner + i;
  if (IN_REAL) {
    const double* in = (const double*)inp + (long long)(b / sub) * s_hi + (long long)(b % sub) * s_lo + off;
    int idx = 0;
    for (int j = 0; j < n; ++j) {
      const double2 w = tw[idx];
      const double x = in[(long long)j * inner];
      re += x * w.x;
      im += x * (INV ? -w.y : w.y);
      idx += k;
      if (idx >= n) idx -= n;
    }
  } else {
    const double2* in = (const double2*)inp + (long long)b * s_in_c + off;
    int idx = 0;
    for (int j = 0; j < n; ++j) {
      const double2 w = tw[idx];
      const double2 x = in[(long long)j * inner];
      const double wy = INV ? -w.y : w.y;
      re += x.x * w.x - x.y * wy;
      im += x.x * wy + x.y * w.x;
      idx += k;
      if (idx >= n) idx -= n;
    }
  }
  const long long oi = off + (long long)k * inner;
  if (OUT_REAL) {
    ((double*)outp)[(long long)b * s_out + oi] = re * scale;
  } else {
    ((double2*)outp)[(long long)b * s_out + oi] = make_double2(re, im);
  }
}

// The same transform for a power-of-two length n <= kFftTile by the
// radix-2 Stockham algorithm (self-sorting, out of place between two LDS
// buffers): a workgroup takes kFftTile / n consecutive lines, loads them
// with consecutive lanes on consecutive addresses (along the line when it
// is contiguous, across lines otherwise), runs the log2(n) butterfly stages
// in LDS and writes the lines back the same way.  Stage s combines
// transforms of length ns = 2^s: for butterfly j < n/2, k = j mod ns,
// v0 = a[j], v1 = a[j + n/2] w^(k n / (2 ns)), and b[2 ns (j / ns) + k] =
// v0 + v1, b[... + ns] = v0 - v1 (w the n-th root of unity of the table,
// conjugated for the inverse).  O(n log n) operations per line instead of
// O(n^2); the result is in natural order.
constexpr int kFftTile = 2048;  // complex values per workgroup

template <bool IN_REAL, bool OUT_REAL, bool INV>
__global__ __launch_bounds__(256) void k_fft_axis(const void* inp, long long s_hi, long long s_lo,
                                                  int sub, long long s_in_c, void* outp,
                                                  long long s_out, const double2* tw, int outer,
                                                  int n, int log2n, int inner, int nbatch,
                                                  double scale) {
  __shared__ double2 buf[2][kFftTile];
  const int L = kFftTile / n;  // lines of this workgroup
  const int nlines = nbatch * outer * inner;
  const int l0 = blockIdx.x * L;
  const int tid = threadIdx.x;
  // element e of the tile: (line, j); lanes run along j for contiguous lines
  auto coords = [&](int e, int& line, int& j) {
    if (inner == 1) {
      line = e >> log2n;
      j = e & (n - 1);
    } else {
      line = e % L;
      j = e / L;
    }
  };
  auto offset = [&](int gl, int& b) -> long long {
    const int i = gl % inner;
    const int bo = gl / inner;
    const int o = bo % outer;
    b = bo / outer;
    return (long long)o * n * inner + i;
  };
  for (int e = tid; e < kFftTile; e += 256) {
    int line, j;
    coords(e, line, j);
    const int gl = l0 + line;
    double2 v = make_double2(0.0, 0.0);
    if (gl < nlines) {
      int b;
      const long long off = offset(gl, b) + (long long)j * inner;
      if (IN_REAL) {
        v.x = ((const double*)inp)[(long long)(b / sub) * s_hi + (long long)(b % sub) * s_lo + off];
      } else {
        v = ((const double2*)inp)[(long long)b * s_in_c + off];
      }
    }
    buf[0][line * n + j] = v;
  }
  __syncthreads();
  const int half = n >> 1;
  int cur = 0;
  for (int s = 0; s < log2n; ++s) {
    const int ns = 1 << s;
    const double2* a = buf[cur];
    double2* o = buf[cur ^ 1];
    for (int e = tid; e < kFftTile / 2; e += 256) {
      const int line = e / half, j = e - line * half;
      const int k = j & (ns - 1);
      const double2 w = tw[k << (log2n - 1 - s)];
      const double wy = INV ? -w.y : w.y;
      const double2 v0 = a[line * n + j], x1 = a[line * n + j + half];
      const double2 v1 = make_double2(x1.x * w.x - x1.y * wy, x1.x * wy + x1.y * w.x);
      const int d = line * n + ((j - k) << 1) + k;
      o[d] = make_double2(v0.x + v1.x, v0.y + v1.y);
      o[d + ns] = make_double2(v0.x - v1.x, v0.y - v1.y);
    }
    cur ^= 1;
    __syncthreads();
  }
  for (int e = tid; e < kFftTile; e += 256) {
    int line, j;
    coords(e, line, j);
    const int gl = l0 + line;
    if (gl >= nlines) continue;
    int b;
    const long long oi = offset(gl, b) + (long long)j * inner;
    const double2 v = buf[cur][line * n + j];
    if (OUT_REAL)
      ((double*)outp)[(long long)b * s_out + oi] = v.x * scale;
    else
      ((double2*)outp)[(long long)b * s_out + oi] = v;
  }
}

__device__ __forceinline__ double wavenumber(int k, int n, double len) {
  const int f = (k < (n + 1) / 2) ? k : k - n;
  return 2.0 * 3.14159265358979323846 * (double)f / len;
}

// W(xi) = -i sum_a xi_a Q_a(xi) / |xi|^2, W(0) = sums[col]
__global__ void k_g2f_combine(const double2* Q, int d, GridArg c, const double* sums, double2* W,
                              int ncols) {
  const long long nc = (long long)c.nx * c.ny * c.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * ncols) return;
  const int col = (int)(t / nc);
  const long long J = t - (long long)col * nc;
  const int X = (int)(J % c.nx);
  const int Y = (int)((J / c.nx) % c.ny);
  const int Z = (int)(J / ((long long)c.nx * c.ny));
  double2 w;
  if (J == 0) {
    w = make_double2(sums ? sums[col] : 0.0, 0.0);
  } else {
    const double xi[3] = {wavenumber(X, c.nx, c.nx * c.dx), wavenumber(Y, c.ny, c.ny * c.dx),
                          wavenumber(Z, c.nz, c.nz * c.dx)};
    double sr = 0.0, si = 0.0, x2 = 0.0;
    for (int a = 0; a < d; ++a) {
      const double2 q = Q[((long long)col * d + a) * nc + J];
      sr += xi[a] * q.x;
      si += xi[a] * q.y;
      x2 += xi[a] * xi[a];
    }
    // -i (sr + i si) = si - i sr
    w = make_double2(si / x2, -sr / x2);
  }
  W[(long long)col * nc + J] = w;
}

// out_u = -sum_a grad_a q_a, out_p = p / cc   (adjoint of Lambda)
__global__ void k_lambda_adjoint(const double* in, long long ldi, GridArg c, const double* cc,
                                 int order, double* out, long long ldo, int ncols) {
  const long long nc = (long long)c.nx * c.ny * c.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * ncols) return;
  const int col = (int)(t / nc);
  const long long J = t - (long long)col * nc;
  const int X = (int)(J % c.nx);
  const int Y = (int)((J / c.nx) % c.ny);
  const int Z = (int)(J / ((long long)c.nx * c.ny));
  const double* q = in + (long long)col * ldi;
  double acc = 0.0;
  for (int a = 0; a < c.dim; ++a)
    acc += grad_at(q + a * nc, a, X, Y, Z, c, 1, c.nx, c.ny, order);
  double* o = out + (long long)col * ldo;
  o[J] = -acc;
  o[nc + J] = q[c.dim * nc + J] / cc[J];
}

__global__ void k_scale_p(const double* in, long long ldi, int d, const double* cc, double* out,
                          long long ldo, long long nc, int ncols) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * ncols) return;
  const int col = (int)(t / nc);
  const long long J = t - (long long)col * nc;
  out[(long long)col * ldo + nc + J] = cc[J] * in[(long long)col * ldi + d * nc + J];
}

__global__ void k_set_dc(double* mat, long long ld, int col, long long nc, double val) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nc) return;
  mat[(long long)col * ld + t] = t < nc ? val : 0.0;
}

// per-block partial sums of |grad_h(u-uref)|^2 + (p-pref)^2 / c^2, of the
// same for (uref, pref), and of (u-uref)^2 and uref^2 (the l2 error of the
// displacement); the final sums are taken by k_finish_pair
template <typename T>
__global__ void k_energy_pair(const T* u, const T* p, const T* ur, const T* pr, const double* cf,
                              GridArg g, int order, double* partials) {
  __shared__ double s0[kTB], s1[kTB], s2[kTB], s3[kTB];
  const long long np = (long long)g.nx * g.ny * g.nz;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (long long J = (long long)blockIdx.x * blockDim.x + threadIdx.x; J < np;
       J += (long long)gridDim.x * blockDim.x) {
    const int X = (int)(J % g.nx);
    const int Y = (int)((J / g.nx) % g.ny);
    const int Z = (int)(J / ((long long)g.nx * g.ny));
    for (int a = 0; a < g.dim; ++a) {
      if (ur) {
        // gradient of the difference, built from differences of values
        auto val = [&](int dxo) -> double {
          int x = X, y = Y, z = Z;
          if (a == 0) x = wrapi(X + dxo, g.nx);
          if (a == 1) y = wrapi(Y + dxo, g.ny);
          if (a == 2) z = wrapi(Z + dxo, g.nz);
          const long long gi = (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
          return (double)u[gi] - (double)ur[gi];
        };
        double d = 0.0;
        for (int j = 1; j <= order / 2; ++j) d += fd_weight(order, j) * (val(j) - val(-j));
        d /= g.dx;
        a0 += d * d;
        const double e = grad_at(ur, a, X, Y, Z, g, 1, g.nx, g.ny, order);
        a1 += e * e;
      } else {
        const double d = grad_at(u, a, X, Y, Z, g, 1, g.nx, g.ny, order);
        a0 += d * d;
      }
    }
    const double c2 = cf[J] * cf[J];
    if (ur) {
      const double dp = (double)p[J] - (double)pr[J];
      a0 += dp * dp / c2;
      a1 += (double)pr[J] * (double)pr[J] / c2;
      const double du = (double)u[J] - (double)ur[J];
      a2 += du * du;
      a3 += (double)ur[J] * (double)ur[J];
    } else {
      a0 += (double)p[J] * (double)p[J] / c2;
      a2 += (double)u[J] * (double)u[J];
    }
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  s3[threadIdx.x] = a3;
  __syncthreads();
  for (int w = kTB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
      s3[threadIdx.x] += s3[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[4 * blockIdx.x] = s0[0];
    partials[4 * blockIdx.x + 1] = s1[0];
    partials[4 * blockIdx.x + 2] = s2[0];
    partials[4 * blockIdx.x + 3] = s3[0];
  }
}

// result = [E(u - uref), E(uref), sum (u - uref)^2, sum uref^2]: the
// energies carry the factor 1/2 dx^d of the discrete energy, the l2 sums
// are plain sums over the grid points
__global__ void k_finish_pair(const double* partials, int nb, double scale, double* result) {
  __shared__ double s[4][kTB];
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    for (int q = 0; q < 4; ++q) a[q] += partials[4 * i + q];
  for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int w = kTB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    result[0] = 0.5 * scale * s[0][0];
    result[1] = 0.5 * scale * s[1][0];
    result[2] = s[2][0];
    result[3] = s[3][0];
  }
}

constexpr int kEnergyBlocks = 1024;

}  // namespace

template <typename T>
void energy_columns(const Grid& src, int ratio, const Grid& c, const T* u, const T* p,
                    long long sstride, const double* cc, int order, double* out, long long ldo,
                    int nstates, hipStream_t st, const SpecScratch* sp) {
  const long long n = c.npts() * nstates;
  if (n == 0) return;
  if (order == 0 && !sp) fail(PW_EINVAL, "spectral gradient without its scratch");
  hipLaunchKernelGGL((k_energy_columns<T>), dim3(nblocks(n)), dim3(kTB), 0, st, u, p, sstride,
                     garg(c), ratio, src.n[0], src.n[1], cc, order, out, ldo, nstates,
                     order == 0 ? sp->ures : (double*)nullptr);
  PW_LAUNCH_CHECK();
  if (order == 0) spectral_grad_cols(c, *sp, sp->ures, c.npts(), nstates, out, ldo, st);
}

template <typename T>
void restrict_diff(const Grid& f, int ratio, const Grid& c, const T* au, const T* ap, const T* bu,
                   const T* bp, long long sstride, double* out, long long ldo, int nstates,
                   hipStream_t st) {
  const long long n = c.npts() * nstates;
  if (n == 0) return;
  hipLaunchKernelGGL((k_restrict_diff<T>), dim3(nblocks(n)), dim3(kTB), 0, st, au, ap, bu, bp,
                     sstride, garg(c), ratio, f.n[0], f.n[1], out, ldo, nstates);
  PW_LAUNCH_CHECK();
}

template <typename T>
void restrict_fields(const Grid& f, int ratio, const Grid& c, const T* in, long long sin, T* out,
                     long long sout, int nfields, hipStream_t st) {
  const long long n = c.npts() * nfields;
  if (n == 0) return;
  hipLaunchKernelGGL((k_restrict_fields<T>), dim3(nblocks(n)), dim3(kTB), 0, st, in, sin, garg(c),
                     ratio, f.n[0], f.n[1], out, sout, nfields);
  PW_LAUNCH_CHECK();
}

template <typename T>
void cast_from_double(const double* in, T* out, long long n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_cast<double, T>), dim3(nblocks(n)), dim3(kTB), 0, st, in, out, n);
  PW_LAUNCH_CHECK();
}

template <typename T>
void cast_to_double(const T* in, double* out, long long n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_cast<T, double>), dim3(nblocks(n)), dim3(kTB), 0, st, in, out, n);
  PW_LAUNCH_CHECK();
}

std::vector<double> trig_interp_table(int nc, int ratio) {
  std::vector<double> tab((size_t)nc * ratio, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int s = 0; s < ratio; ++s) {
    for (int d = 0; d < nc; ++d) {
      if (s == 0) {
        tab[(size_t)s * nc + d] = (d == 0) ? 1.0 : 0.0;
        continue;
      }
      const long double x = ((long double)d + (long double)s / ratio) / nc;
      long double acc = 1.0L;
      if (nc % 2 == 0) {
        for (int k = 1; k < nc / 2; ++k) acc += 2.0L * cosl(2.0L * pi * k * x);
        acc += cosl(pi * nc * x);
      } else {
        for (int k = 1; k <= (nc - 1) / 2; ++k) acc += 2.0L * cosl(2.0L * pi * k * x);
      }
      tab[(size_t)s * nc + d] = (double)(acc / nc);
    }
  }
  return tab;
}

// polyphase weights of periodic piecewise-linear interpolation in the same
// layout: fine node ratio J + s takes 1 - s/ratio of coarse node J (d = 0)
// and s/ratio of coarse node J + 1 (d = nc - 1)
std::vector<double> linear_interp_table(int nc, int ratio) {
  std::vector<double> tab((size_t)nc * ratio, 0.0);
  for (int s = 0; s < ratio; ++s) {
    const double t = (double)s / ratio;
    tab[(size_t)s * nc] += 1.0 - t;
    tab[(size_t)s * nc + (size_t)(nc - 1)] += t;
  }
  return tab;
}

// the same layout for local cubic interpolation: fine node ratio J + s
// (t = s / ratio) takes the 4-point Lagrange weights of coarse nodes
// J - 1, J, J + 1, J + 2, i.e. d = 1, 0, nc - 1, nc - 2 (nc >= 4)
std::vector<double> cubic_interp_table(int nc, int ratio) {
  std::vector<double> tab((size_t)nc * ratio, 0.0);
  for (int s = 0; s < ratio; ++s) {
    const double t = (double)s / ratio;
    const double w[4] = {-t * (t - 1.0) * (t - 2.0) / 6.0, (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
                         -(t + 1.0) * t * (t - 2.0) / 2.0, (t + 1.0) * t * (t - 1.0) / 6.0};
    const int dd[4] = {1, 0, nc - 1, nc - 2};
    for (int k = 0; k < 4; ++k) tab[(size_t)s * nc + (size_t)dd[k]] += w[k];
  }
  return tab;
}

template <typename T>
void interp_add(const Grid& f, const Grid& c, int ratio, const double* const* tables, const T* in,
                long long sin, const T* v, T* out, long long sout, int nfields, double* tmp,
                hipStream_t st) {
  if (nfields == 0) return;
  const int d = f.dim;
  const int fx = f.n[0], fy = f.n[1];
  const int cx = c.n[0], cy = c.n[1], cz = c.n[2];
  if (d == 1) {
    interp_pass<T, T, true>(in, sin, out, sout, v, tables[0], 1, cx, ratio, 1, nfields, st);
    return;
  }
  // pass x: (cz*cy, cx, 1) -> tA (cz*cy, fx, 1)
  double* tA = tmp;
  const long long sA = (long long)cz * cy * fx;
  double* tB = tmp + sA * nfields;
  interp_pass<T, double, false>(in, sin, tA, sA, (const double*)nullptr, tables[0], cz * cy, cx,
                                ratio, 1, nfields, st);
  if (d == 2) {
    interp_pass<double, T, true>(tA, sA, out, sout, v, tables[1], 1, cy, ratio, fx, nfields, st);
    return;
  }
  // 3D: pass y: (cz, cy, fx) -> tB (cz, fy, fx); pass z: (1, cz, fy*fx) -> out
  const long long sB = (long long)cz * fy * fx;
  interp_pass<double, double, false>(tA, sA, tB, sB, (const double*)nullptr, tables[1], cz, cy,
                                     ratio, fx, nfields, st);
  interp_pass<double, T, true>(tB, sB, out, sout, v, tables[2], 1, cz, ratio, fy * fx, nfields,
                               st);
}

std::vector<double> dft_table(int n) {
  std::vector<double> tw(2 * (size_t)n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < n; ++j) {
    const long double a = 2.0L * pi * j / n;
    tw[2 * j] = (double)cosl(a);
    tw[2 * j + 1] = (double)(-sinl(a));
  }
  return tw;
}

// one transform pass along an axis of length n: the FFT for powers of two
// up to kFftTile, the direct sum otherwise
template <bool IN_REAL, bool OUT_REAL, bool INV>
void dft_pass(const void* in, long long s_hi, long long s_lo, int sub, long long s_in_c,
              void* out, long long s_out, const double* tw, int outer, int n, int inner,
              int nbatch, double scale, hipStream_t st) {
  int log2n = 0;
  while ((1 << log2n) < n) ++log2n;
  if (n >= 2 && (1 << log2n) == n && n <= kFftTile) {
    const long long lines = (long long)nbatch * outer * inner;
    const int L = kFftTile / n;
    hipLaunchKernelGGL((k_fft_axis<IN_REAL, OUT_REAL, INV>), dim3((unsigned)((lines + L - 1) / L)),
                       dim3(256), 0, st, in, s_hi, s_lo, sub, s_in_c, out, s_out,
                       (const double2*)tw, outer, n, log2n, inner, nbatch, scale);
  } else {
    const long long total = (long long)outer * n * inner * nbatch;
    hipLaunchKernelGGL((k_dft_axis<IN_REAL, OUT_REAL, INV>), dim3(nblocks(total)), dim3(kTB), 0,
                       st, in, s_hi, s_lo, sub, s_in_c, out, s_out, (const double2*)tw, outer, n,
                       inner, nbatch, scale);
  }
  PW_LAUNCH_CHECK();
}

// G[(col d + a) np + J] = i xi_a S[col np + J]
__global__ void k_spec_grad_mul(const double2* S, GridArg c, double2* G, int ncols) {
  const long long nc = (long long)c.nx * c.ny * c.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * ncols) return;
  const int col = (int)(t / nc);
  const long long J = t - (long long)col * nc;
  const int X = (int)(J % c.nx);
  const int Y = (int)((J / c.nx) % c.ny);
  const int Z = (int)(J / ((long long)c.nx * c.ny));
  const double xi[3] = {wavenumber(X, c.nx, c.nx * c.dx), wavenumber(Y, c.ny, c.ny * c.dx),
                        wavenumber(Z, c.nz, c.nz * c.dx)};
  const double2 s = S[t];
  for (int a = 0; a < c.dim; ++a)
    G[((long long)col * c.dim + a) * nc + J] = make_double2(-xi[a] * s.y, xi[a] * s.x);
}

// S[col np + J] = -i sum_a xi_a Q[(col d + a) np + J]
__global__ void k_spec_div_mul(const double2* Q, GridArg c, double2* S, int ncols) {
  const long long nc = (long long)c.nx * c.ny * c.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * ncols) return;
  const int col = (int)(t / nc);
  const long long J = t - (long long)col * nc;
  const int X = (int)(J % c.nx);
  const int Y = (int)((J / c.nx) % c.ny);
  const int Z = (int)(J / ((long long)c.nx * c.ny));
  const double xi[3] = {wavenumber(X, c.nx, c.nx * c.dx), wavenumber(Y, c.ny, c.ny * c.dx),
                        wavenumber(Z, c.nz, c.nz * c.dx)};
  double sr = 0.0, si = 0.0;
  for (int a = 0; a < c.dim; ++a) {
    const double2 q = Q[((long long)col * c.dim + a) * nc + J];
    sr += xi[a] * q.x;
    si += xi[a] * q.y;
  }
  S[t] = make_double2(si, -sr);  // -i (sr + i si)
}

// out[col * ldo + a * np + J] = r[(col d + a) np + J]
__global__ void k_spec_scatter(const double* r, int d, long long nc, int ncols, double* out,
                               long long ldo) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * d * ncols) return;
  const long long b = t / nc, J = t - b * nc;
  const int col = (int)(b / d), a = (int)(b % d);
  out[(long long)col * ldo + (long long)a * nc + J] = r[t];
}

// forward transform of nb real fields (batch b at (b / sub) s_hi + (b % sub)
// s_lo) into the complex spectrum; returns the buffer holding it
static double2* spec_forward(const Grid& c, const double* const* dft, const void* in,
                             long long s_hi, long long s_lo, int sub, int nb, double2* A,
                             double2* B, hipStream_t st) {
  const long long nc = c.npts();
  const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
  dft_pass<true, false, false>(in, s_hi, s_lo, sub, 0LL, A, nc, dft[0], ny * nz, nx, 1, nb, 1.0, st);
  double2* cur = A;
  double2* oth = B;
  if (c.dim >= 2) {
    dft_pass<false, false, false>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[1], nz, ny, nx, nb, 1.0, st);
    std::swap(cur, oth);
  }
  if (c.dim >= 3) {
    dft_pass<false, false, false>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[2], 1, nz, nx * ny, nb, 1.0,
                                  st);
    std::swap(cur, oth);
  }
  return cur;
}

// inverse transform of nb spectra in `cur` (work buffer `oth`), real part
// / np written to out, batch b at b * s_out
static void spec_inverse_real(const Grid& c, const double* const* dft, double2* cur,
                              double2* oth, int nb, double* out, long long s_out,
                              hipStream_t st) {
  const long long nc = c.npts();
  const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
  const double scale = 1.0 / (double)nc;
  if (c.dim == 1) {
    dft_pass<false, true, true>(cur, 0LL, 0LL, 1, nc, out, s_out, dft[0], 1, nx, 1, nb, scale, st);
    return;
  }
  dft_pass<false, false, true>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[0], ny * nz, nx, 1, nb, 1.0, st);
  std::swap(cur, oth);
  if (c.dim == 2) {
    dft_pass<false, true, true>(cur, 0LL, 0LL, 1, nc, out, s_out, dft[1], nz, ny, nx, nb, scale,
                                st);
    return;
  }
  dft_pass<false, false, true>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[1], nz, ny, nx, nb, 1.0, st);
  std::swap(cur, oth);
  dft_pass<false, true, true>(cur, 0LL, 0LL, 1, nc, out, s_out, dft[2], 1, nz, nx * ny, nb, scale,
                              st);
}

void spectral_grad_cols(const Grid& c, const SpecScratch& sp, const double* in, long long ldi,
                        int ncols, double* out, long long ldo, hipStream_t st) {
  if (ncols == 0) return;
  if (ncols > sp.cols) fail(PW_EINVAL, "too many columns for the spectral gradient scratch");
  const int d = c.dim;
  const long long nc = c.npts();
  double2* A = (double2*)sp.ctmp;          // ncols spectra
  double2* B = A + nc * ncols;             // ncols
  double2* G = B + nc * ncols;             // ncols * d
  double2* G2 = G + nc * ncols * d;        // ncols * d
  double2* S = spec_forward(c, sp.dft, in, ldi, 0LL, 1, ncols, A, B, st);
  hipLaunchKernelGGL(k_spec_grad_mul, dim3(nblocks(nc * ncols)), dim3(kTB), 0, st,
                     (const double2*)S, garg(c), G, ncols);
  PW_LAUNCH_CHECK();
  spec_inverse_real(c, sp.dft, G, G2, ncols * d, sp.rtmp, nc, st);
  hipLaunchKernelGGL(k_spec_scatter, dim3(nblocks(nc * d * ncols)), dim3(kTB), 0, st,
                     (const double*)sp.rtmp, d, nc, ncols, out, ldo);
  PW_LAUNCH_CHECK();
}

void spectral_div_cols(const Grid& c, const SpecScratch& sp, const double* in, long long ldi,
                       int ncols, double* out, long long ldo, hipStream_t st) {
  if (ncols == 0) return;
  if (ncols > sp.cols) fail(PW_EINVAL, "too many columns for the spectral gradient scratch");
  const int d = c.dim;
  const long long nc = c.npts();
  double2* A = (double2*)sp.ctmp;          // ncols * d spectra
  double2* B = A + nc * ncols * d;         // ncols * d
  double2* S = B + nc * ncols * d;         // ncols
  double2* S2 = S + nc * ncols;            // ncols
  double2* Q = spec_forward(c, sp.dft, in, ldi, nc, d, ncols * d, A, B, st);
  hipLaunchKernelGGL(k_spec_div_mul, dim3(nblocks(nc * ncols)), dim3(kTB), 0, st,
                     (const double2*)Q, garg(c), S, ncols);
  PW_LAUNCH_CHECK();
  spec_inverse_real(c, sp.dft, S, S2, ncols, out, ldo, st);
}

void grad2func_cols(const Grid& c, const double* const* dft, const double* q, long long ldq,
                    const double* sums, double* w, long long ldw, int ncols, double* ctmp,
                    hipStream_t st) {
  if (ncols == 0) return;
  const int d = c.dim;
  const long long nc = c.npts();
  const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
  double2* A = (double2*)ctmp;
  double2* B = A + nc * d * ncols;
  const int nb = d * ncols;
  // forward x (real in): batch b = col*d + a
  dft_pass<true, false, false>(q, ldq, nc, d, 0LL, A, nc, dft[0], ny * nz, nx, 1, nb, 1.0, st);
  double2* cur = A;
  double2* oth = B;
  if (d >= 2) {
    dft_pass<false, false, false>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[1], nz, ny, nx, nb, 1.0, st);
    std::swap(cur, oth);
  }
  if (d >= 3) {
    dft_pass<false, false, false>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[2], 1, nz, nx * ny, nb, 1.0,
                                  st);
    std::swap(cur, oth);
  }
  {
    const long long n = nc * ncols;
    hipLaunchKernelGGL(k_g2f_combine, dim3(nblocks(n)), dim3(kTB), 0, st, (const double2*)cur, d,
                       garg(c), sums, oth, ncols);
    PW_LAUNCH_CHECK();
    std::swap(cur, oth);
  }
  // inverse passes; the last one writes the real part / nc into w
  const double scale = 1.0 / (double)nc;
  if (d == 1) {
    dft_pass<false, true, true>(cur, 0LL, 0LL, 1, nc, w, ldw, dft[0], 1, nx, 1, ncols, scale, st);
    return;
  }
  dft_pass<false, false, true>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[0], ny * nz, nx, 1, ncols, 1.0,
                               st);
  std::swap(cur, oth);
  if (d == 2) {
    dft_pass<false, true, true>(cur, 0LL, 0LL, 1, nc, w, ldw, dft[1], nz, ny, nx, ncols, scale, st);
    return;
  }
  dft_pass<false, false, true>(cur, 0LL, 0LL, 1, nc, oth, nc, dft[1], nz, ny, nx, ncols, 1.0, st);
  std::swap(cur, oth);
  dft_pass<false, true, true>(cur, 0LL, 0LL, 1, nc, w, ldw, dft[2], 1, nz, nx * ny, ncols, scale,
                              st);
}

void lambda_adjoint_cols(const Grid& c, const double* in, long long ldi, const double* cc,
                         int order, double* out, long long ldo, int ncols, hipStream_t st,
                         const SpecScratch* sp) {
  const long long n = c.npts() * ncols;
  if (n == 0) return;
  if (order == 0 && !sp) fail(PW_EINVAL, "spectral gradient without its scratch");
  hipLaunchKernelGGL(k_lambda_adjoint, dim3(nblocks(n)), dim3(kTB), 0, st, in, ldi, garg(c), cc,
                     order, out, ldo, ncols);
  PW_LAUNCH_CHECK();
  if (order == 0) spectral_div_cols(c, *sp, in, ldi, ncols, out, ldo, st);
}

void lambda_dag_cols(const Grid& c, const double* const* dft, const double* in, long long ldi,
                     const double* cc, const double* sums, double* out, long long ldo, int ncols,
                     double* ctmp, hipStream_t st) {
  if (ncols == 0) return;
  grad2func_cols(c, dft, in, ldi, sums, out, ldo, ncols, ctmp, st);
  const long long n = c.npts() * ncols;
  hipLaunchKernelGGL(k_scale_p, dim3(nblocks(n)), dim3(kTB), 0, st, in, ldi, c.dim, cc, out, ldo,
                     c.npts(), ncols);
  PW_LAUNCH_CHECK();
}

void set_dc_column(double* mat, long long ld, int col, long long nc, double val, hipStream_t st) {
  hipLaunchKernelGGL(k_set_dc, dim3(nblocks(2 * nc)), dim3(kTB), 0, st, mat, ld, col, nc, val);
  PW_LAUNCH_CHECK();
}

template <typename T>
void energy_pair(const Grid& f, const T* u, const T* p, const T* ur, const T* pr,
                 const double* cf, int order, double* partials, double* result, hipStream_t st) {
  hipLaunchKernelGGL((k_energy_pair<T>), dim3(kEnergyBlocks), dim3(kTB), 0, st, u, p, ur, pr, cf,
                     garg(f), order, partials);
  PW_LAUNCH_CHECK();
  double scale = 1.0;
  for (int a = 0; a < f.dim; ++a) scale *= f.dx;
  hipLaunchKernelGGL(k_finish_pair, dim3(1), dim3(kTB), 0, st, (const double*)partials,
                     kEnergyBlocks, scale, result);
  PW_LAUNCH_CHECK();
}

static_assert(4 * kEnergyBlocks == kEnergyPartials, "energy partial layout");

#define PW_INST(T)                                                                              \
  template void energy_columns<T>(const Grid&, int, const Grid&, const T*, const T*, long long, \
                                  const double*, int, double*, long long, int, hipStream_t,    \
                                  const SpecScratch*);                                         \
  template void restrict_diff<T>(const Grid&, int, const Grid&, const T*, const T*, const T*,   \
                                 const T*, long long, double*, long long, int, hipStream_t);   \
  template void restrict_fields<T>(const Grid&, int, const Grid&, const T*, long long, T*,      \
                                   long long, int, hipStream_t);                                \
  template void cast_from_double<T>(const double*, T*, long long, hipStream_t);                 \
  template void cast_to_double<T>(const T*, double*, long long, hipStream_t);                   \
  template void interp_add<T>(const Grid&, const Grid&, int, const double* const*, const T*,    \
                              long long, const T*, T*, long long, int, double*, hipStream_t);   \
  template void energy_pair<T>(const Grid&, const T*, const T*, const T*, const T*,             \
                               const double*, int, double*, double*, hipStream_t);
PW_INST(float)
PW_INST(double)
#undef PW_INST

}  // namespace pw
