// Adjoint building blocks for d J / d c^2 through Algorithm 3 with the
// phase corrector held fixed:
//  * reverse velocity Verlet (Sec. 3.1 scheme run backwards) with the c^2
//    gradient accumulated per state, the forward displacements recomputed
//    from checkpoints taken every `ckpt` steps;
//  * transposes of the trigonometric interpolation and of the pointwise
//    restriction;
//  * the receiver misfit and its seed.
// All adjoint arithmetic is FP64; forward states of the FP32 path are
// widened when read.
#include <algorithm>
#include <cmath>

#include "pw_internal.h"

namespace pw {
namespace {

constexpr int kTB = 256;
inline unsigned nblocks(long long n, int tb = kTB) { return (unsigned)((n + tb - 1) / tb); }

struct G3 {
  int dim, nx, ny, nz;
  double idx2;
};
inline G3 g3(const Grid& g) { return G3{g.dim, g.n[0], g.n[1], g.n[2], 1.0 / (g.dx * g.dx)}; }

__device__ __forceinline__ int wrapi(int g, int n) {
  g %= n;
  return g < 0 ? g + n : g;
}

// periodic CD2 Laplacian of f at point J (f: one field)
__device__ __forceinline__ double lap_at(const double* f, long long J, const G3& g) {
  const int x = (int)(J % g.nx);
  const int y = (int)((J / g.nx) % g.ny);
  const int z = (int)(J / ((long long)g.nx * g.ny));
  const double c = f[J];
  auto at = [&](int xx, int yy, int zz) {
    return f[(long long)xx + (long long)g.nx * ((long long)yy + (long long)g.ny * zz)];
  };
  double s = at(wrapi(x + 1, g.nx), y, z) - 2.0 * c + at(wrapi(x - 1, g.nx), y, z);
  if (g.dim >= 2) s += at(x, wrapi(y + 1, g.ny), z) - 2.0 * c + at(x, wrapi(y - 1, g.ny), z);
  if (g.dim >= 3) s += at(x, y, wrapi(z + 1, g.nz)) - 2.0 * c + at(x, y, wrapi(z - 1, g.nz));
  return s * g.idx2;
}

// c^2 * lambda of a field, staged for the adjoint Laplacian
__global__ void k_mul_c2(const double* c2, const double* l, long long sl, double* out,
                         long long so, long long np, int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * ns) return;
  const int s = (int)(t / np);
  const long long J = t - (long long)s * np;
  out[(long long)s * so + J] = c2[J] * l[(long long)s * sl + J];
}

// forward half kick + drift: ph = p + h/2 c2 Lap u ; u_next = u + h ph
__global__ void k_fwd_kick_drift(const double* u, long long su, double* p, long long sp,
                                 double* un, long long sun, const double* c2, double h, G3 g,
                                 long long np, int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * ns) return;
  const int s = (int)(t / np);
  const long long J = t - (long long)s * np;
  const double* us = u + (long long)s * su;
  double pv = p[(long long)s * sp + J] + 0.5 * h * (c2[J] * lap_at(us, J, g));
  p[(long long)s * sp + J] = pv;
  un[(long long)s * sun + J] = us[J] + h * pv;
}

// forward closing half kick: p += h/2 c2 Lap u
__global__ void k_fwd_kick(const double* u, long long su, double* p, long long sp,
                           const double* c2, double h, G3 g, long long np, int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * ns) return;
  const int s = (int)(t / np);
  const long long J = t - (long long)s * np;
  p[(long long)s * sp + J] += 0.5 * h * (c2[J] * lap_at(u + (long long)s * su, J, g));
}

// reverse of the second half kick and the drift of a step:
//   lu += h/2 Lap(c2 lp);  g += h/2 lp Lap(u_next);  lp_new = lp + h lu
// a = c2 lp (staged); u1 = displacement after the drift
__global__ void k_adj_kick2_drift(const double* a, long long sa, double* lu, long long slu,
                                  const double* lp, long long slp, double* lpn, long long slpn,
                                  const double* u1, long long su1, double* gacc, long long sg,
                                  double h, G3 g, long long np, int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * ns) return;
  const int s = (int)(t / np);
  const long long J = t - (long long)s * np;
  const double lpv = lp[(long long)s * slp + J];
  const double luv = lu[(long long)s * slu + J] + 0.5 * h * lap_at(a + (long long)s * sa, J, g);
  lu[(long long)s * slu + J] = luv;
  gacc[(long long)s * sg + J] += 0.5 * h * lpv * lap_at(u1 + (long long)s * su1, J, g);
  lpn[(long long)s * slpn + J] = lpv + h * luv;
}

// reverse of the first half kick: lu += h/2 Lap(c2 lp); g += h/2 lp Lap(u0)
__global__ void k_adj_kick1(const double* a, long long sa, double* lu, long long slu,
                            const double* lp, long long slp, const double* u0, long long su0,
                            double* gacc, long long sg, double h, G3 g, long long np, int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * ns) return;
  const int s = (int)(t / np);
  const long long J = t - (long long)s * np;
  lu[(long long)s * slu + J] += 0.5 * h * lap_at(a + (long long)s * sa, J, g);
  gacc[(long long)s * sg + J] +=
      0.5 * h * lp[(long long)s * slp + J] * lap_at(u0 + (long long)s * su0, J, g);
}

template <typename T>
__global__ void k_widen(const T* in, long long si, double* out, long long so, long long np,
                        int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * ns) return;
  const int s = (int)(t / np);
  const long long J = t - (long long)s * np;
  out[(long long)s * so + J] = (double)in[(long long)s * si + J];
}

__global__ void k_copy_fields(const double* in, long long si, double* out, long long so,
                              long long np, int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np * ns) return;
  const int s = (int)(t / np);
  const long long J = t - (long long)s * np;
  out[(long long)s * so + J] = in[(long long)s * si + J];
}

// transpose of one axis pass of the polyphase interpolation:
// fine (outer, nc*ratio, inner) -> coarse (outer, nc, inner),
// out[m] = fine[ratio m] + sum_{J, s>=1} tab[s nc + (J-m) mod nc] fine[ratio J + s]
__global__ void k_interp_T_axis(const double* in, long long sin, double* out, long long sout,
                                const double* tab, int outer, int nc, int ratio, int inner,
                                int nfields) {
  const long long per = (long long)outer * nc * inner;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nfields) return;
  const int f = (int)(t / per);
  long long r = t - (long long)f * per;
  const int i = (int)(r % inner);
  r /= inner;
  const int m = (int)(r % nc);
  const int o = (int)(r / nc);
  const int nf = nc * ratio;
  const double* src = in + (long long)f * sin + (long long)o * nf * inner + i;
  double acc = src[(long long)ratio * m * inner];
  for (int J = 0; J < nc; ++J) {
    int d = J - m;
    if (d < 0) d += nc;
    for (int s = 1; s < ratio; ++s)
      acc += tab[(long long)s * nc + d] * src[((long long)ratio * J + s) * inner];
  }
  out[(long long)f * sout + ((long long)o * nc + m) * inner + i] = acc;
}

// fine[ratio J] += scale * coarse[J] (transpose of the restriction)
__global__ void k_restrict_T_add(const double* c, long long sc, double* f, long long sf, G3 cg,
                                 int ratio, int fnx, int fny, double scale, int nfields) {
  const long long nc = (long long)cg.nx * cg.ny * cg.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc * nfields) return;
  const int s = (int)(t / nc);
  const long long J = t - (long long)s * nc;
  const int X = (int)(J % cg.nx);
  const int Y = (int)((J / cg.nx) % cg.ny);
  const int Z = (int)(J / ((long long)cg.nx * cg.ny));
  const long long gi = (long long)X * ratio + (long long)fnx * ((long long)Y * ratio +
                                                                  (long long)fny * Z * ratio);
  f[(long long)s * sf + gi] += scale * c[(long long)s * sc + J];
}

// sum of nstates fields in a fixed order: out[J] (+)= sum_s in[s][J]
__global__ void k_sum_fields(const double* in, long long si, int ns, double* out, long long np,
                             int accumulate) {
  const long long J = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= np) return;
  double a = 0.0;
  for (int s = 0; s < ns; ++s) a += in[(long long)s * si + J];
  out[J] = accumulate ? out[J] + a : a;
}

// values at the receivers: out[n][r] = u_n(x_r)
template <typename T>
__global__ void k_receiver_values(const T* u, long long su, const long long* rec, int nrec,
                                  int nst, double* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nst * nrec) return;
  const int n = (int)(t / nrec), r = (int)(t % nrec);
  out[t] = (double)u[(long long)n * su + rec[r]];
}

// one thread per state: lam_n(x_r) += seed[n][r] for r in order, so that
// repeated receivers accumulate deterministically
__global__ void k_receiver_scatter(const double* seed, const long long* rec, int nrec, int nst,
                                   double* lam, long long sl) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nst) return;
  double* l = lam + (long long)n * sl;
  for (int r = 0; r < nrec; ++r) l[rec[r]] += seed[(long long)n * nrec + r];
}

__global__ void k_reverse_cols(int m, int n, const double* src, long long lds, double* dst,
                               long long ldd) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)m * n) return;
  const int j = (int)(t / m), i = (int)(t % m);
  dst[(long long)j * ldd + i] = src[(long long)(n - 1 - j) * lds + i];
}

__global__ void k_mul_fields(const double* a, const double* b, double* out, long long n,
                             double scale) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = scale * a[t] * b[t];
}

}  // namespace

template <typename T>
void widen_fields(const T* in, long long si, double* out, long long so, long long np, int ns,
                  hipStream_t st) {
  if (np * ns == 0) return;
  hipLaunchKernelGGL((k_widen<T>), dim3(nblocks(np * ns)), dim3(kTB), 0, st, in, si, out, so,
                     np, ns);
  PW_LAUNCH_CHECK();
}

void copy_fields(const double* in, long long si, double* out, long long so, long long np, int ns,
                 hipStream_t st) {
  if (np * ns == 0) return;
  hipLaunchKernelGGL(k_copy_fields, dim3(nblocks(np * ns)), dim3(kTB), 0, st, in, si, out, so,
                     np, ns);
  PW_LAUNCH_CHECK();
}

void vv_adjoint(const Grid& grid, const double* c2, const double* u0, const double* p0,
                long long s0, double* lu, double* lp, long long sl, double* gacc, long long sg,
                int ns, int m, double h, int ckpt, const AdjScratch& sc, hipStream_t st) {
  if (ns == 0 || m == 0) return;
  if (ckpt < 1) fail(PW_EINVAL, "checkpoint interval must be >= 1");
  const long long np = grid.npts();
  const G3 g = g3(grid);
  const unsigned nb = nblocks(np * ns);
  const int nseg = (m + ckpt - 1) / ckpt;
  if ((long long)ns * np > sc.state_elems) fail(PW_EINVAL, "adjoint scratch too small");
  if (nseg > sc.max_ckpt) fail(PW_EINVAL, "too many checkpoints for the adjoint scratch");
  if (std::min(m, ckpt) + 1 > sc.max_seg) fail(PW_EINVAL, "checkpoint segment too long");
  const long long S = sc.state_elems;  // stride of one stored time level
  // forward pass: checkpoints (u, p) at the start of every segment
  copy_fields(u0, s0, sc.ck_u, np, np, ns, st);
  copy_fields(p0, s0, sc.ck_p, np, np, ns, st);
  double* cu = sc.ck_u;
  double* cp = sc.ck_p;
  for (int seg = 0; seg + 1 < nseg; ++seg) {
    double* nu = sc.ck_u + (seg + 1) * S;
    double* npp = sc.ck_p + (seg + 1) * S;
    copy_fields(cp, np, npp, np, np, ns, st);
    // ckpt steps from (cu, cp) into (nu, npp), ping-ponging u in the
    // segment store
    const double* src = cu;
    for (int i = 0; i < ckpt; ++i) {
      double* dst = (i == ckpt - 1) ? nu : sc.seg + (long long)(i % 2) * S;
      hipLaunchKernelGGL(k_fwd_kick_drift, dim3(nb), dim3(kTB), 0, st, src, np, npp, np, dst, np,
                         c2, h, g, np, ns);
      hipLaunchKernelGGL(k_fwd_kick, dim3(nb), dim3(kTB), 0, st, (const double*)dst, np, npp, np,
                         c2, h, g, np, ns);
      PW_LAUNCH_CHECK();
      src = dst;
    }
    cu = nu;
    cp = npp;
  }
  // reverse over the segments: recompute the displacements, step back.
  // The adjoint momentum ping-pongs between lp (stride sl) and lp_tmp
  // (stride np).
  double* lpa = lp;
  long long sa = sl;
  double* lpb = sc.lp_tmp;
  long long sb = np;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int i0 = seg * ckpt;
    const int len = std::min(ckpt, m - i0);
    // displacements u_{i0} .. u_{i0+len} in the segment store
    copy_fields(sc.ck_u + seg * S, np, sc.seg, np, np, ns, st);
    copy_fields(sc.ck_p + seg * S, np, sc.p_tmp, np, np, ns, st);
    for (int i = 0; i < len; ++i) {
      const double* src = sc.seg + (long long)i * S;
      double* dst = sc.seg + (long long)(i + 1) * S;
      hipLaunchKernelGGL(k_fwd_kick_drift, dim3(nb), dim3(kTB), 0, st, src, np, sc.p_tmp, np, dst,
                         np, c2, h, g, np, ns);
      hipLaunchKernelGGL(k_fwd_kick, dim3(nb), dim3(kTB), 0, st, (const double*)dst, np,
                         sc.p_tmp, np, c2, h, g, np, ns);
      PW_LAUNCH_CHECK();
    }
    for (int i = len - 1; i >= 0; --i) {
      const double* ui = sc.seg + (long long)i * S;
      const double* ui1 = sc.seg + (long long)(i + 1) * S;
      // second half kick + drift
      hipLaunchKernelGGL(k_mul_c2, dim3(nb), dim3(kTB), 0, st, c2, (const double*)lpa, sa,
                         sc.a_tmp, np, np, ns);
      hipLaunchKernelGGL(k_adj_kick2_drift, dim3(nb), dim3(kTB), 0, st, (const double*)sc.a_tmp,
                         np, lu, sl, (const double*)lpa, sa, lpb, sb, ui1, np, gacc, sg, h, g, np,
                         ns);
      // first half kick
      hipLaunchKernelGGL(k_mul_c2, dim3(nb), dim3(kTB), 0, st, c2, (const double*)lpb, sb,
                         sc.a_tmp, np, np, ns);
      hipLaunchKernelGGL(k_adj_kick1, dim3(nb), dim3(kTB), 0, st, (const double*)sc.a_tmp, np, lu,
                         sl, (const double*)lpb, sb, ui, np, gacc, sg, h, g, np, ns);
      PW_LAUNCH_CHECK();
      std::swap(lpa, lpb);
      std::swap(sa, sb);
    }
  }
  if (lpa != lp) copy_fields(lpa, sa, lp, sl, np, ns, st);
}

void interp_transpose(const Grid& f, const Grid& c, int ratio, const double* const* tables,
                      const double* in, long long sin, double* out, long long sout, int nfields,
                      double* tmp, hipStream_t st) {
  if (nfields == 0) return;
  const int d = f.dim;
  const int fx = f.n[0], fy = f.n[1], fz = f.n[2];
  const int cx = c.n[0], cy = c.n[1], cz = c.n[2];
  if (d == 1) {
    const long long n = (long long)cx * nfields;
    hipLaunchKernelGGL(k_interp_T_axis, dim3(nblocks(n)), dim3(kTB), 0, st, in, sin, out, sout,
                       tables[0], 1, cx, ratio, 1, nfields);
    PW_LAUNCH_CHECK();
    return;
  }
  if (d == 2) {
    // y transpose: (1, fy, fx) -> tmp (1, cy, fx); x transpose: (cy, fx, 1) -> out
    const long long sA = (long long)cy * fx;
    hipLaunchKernelGGL(k_interp_T_axis, dim3(nblocks(sA * nfields)), dim3(kTB), 0, st, in, sin,
                       tmp, sA, tables[1], 1, cy, ratio, fx, nfields);
    hipLaunchKernelGGL(k_interp_T_axis, dim3(nblocks((long long)cy * cx * nfields)), dim3(kTB), 0,
                       st, (const double*)tmp, sA, out, sout, tables[0], cy, cx, ratio, 1,
                       nfields);
    PW_LAUNCH_CHECK();
    return;
  }
  // 3D: z: (1, fz, fy*fx) -> A (1, cz, fy*fx); y: (cz, fy, fx) -> B (cz, cy, fx);
  // x: (cz*cy, fx, 1) -> out
  (void)fz;
  const long long sA = (long long)cz * fy * fx;
  const long long sB = (long long)cz * cy * fx;
  double* A = tmp;
  double* B = tmp + sA * nfields;
  hipLaunchKernelGGL(k_interp_T_axis, dim3(nblocks(sA * nfields)), dim3(kTB), 0, st, in, sin, A,
                     sA, tables[2], 1, cz, ratio, fy * fx, nfields);
  hipLaunchKernelGGL(k_interp_T_axis, dim3(nblocks(sB * nfields)), dim3(kTB), 0, st,
                     (const double*)A, sA, B, sB, tables[1], cz, cy, ratio, fx, nfields);
  hipLaunchKernelGGL(k_interp_T_axis, dim3(nblocks((long long)cz * cy * cx * nfields)),
                     dim3(kTB), 0, st, (const double*)B, sB, out, sout, tables[0], cz * cy, cx,
                     ratio, 1, nfields);
  PW_LAUNCH_CHECK();
}

void restrict_transpose_add(const Grid& f, int ratio, const Grid& c, const double* in,
                            long long sin, double* out, long long sout, double scale,
                            int nfields, hipStream_t st) {
  const long long n = c.npts() * nfields;
  if (n == 0) return;
  hipLaunchKernelGGL(k_restrict_T_add, dim3(nblocks(n)), dim3(kTB), 0, st, in, sin, out, sout,
                     g3(c), ratio, f.n[0], f.n[1], scale, nfields);
  PW_LAUNCH_CHECK();
}

void sum_fields(const double* in, long long si, int ns, double* out, long long np, bool acc,
                hipStream_t st) {
  if (np == 0) return;
  hipLaunchKernelGGL(k_sum_fields, dim3(nblocks(np)), dim3(kTB), 0, st, in, si, ns, out, np,
                     (int)acc);
  PW_LAUNCH_CHECK();
}

template <typename T>
void receiver_values(const T* u, long long su, const long long* rec, int nrec, int nst,
                     double* out, hipStream_t st) {
  const long long n = (long long)nst * nrec;
  if (n == 0) return;
  hipLaunchKernelGGL((k_receiver_values<T>), dim3(nblocks(n)), dim3(kTB), 0, st, u, su, rec, nrec,
                     nst, out);
  PW_LAUNCH_CHECK();
}

void receiver_scatter(const double* seed, const long long* rec, int nrec, int nst, double* lam,
                      long long sl, hipStream_t st) {
  if (nst == 0 || nrec == 0) return;
  hipLaunchKernelGGL(k_receiver_scatter, dim3(nblocks(nst, 64)), dim3(64), 0, st, seed, rec, nrec,
                     nst, lam, sl);
  PW_LAUNCH_CHECK();
}

void reverse_cols(int m, int n, const double* src, long long lds, double* dst, long long ldd,
                  hipStream_t st) {
  const long long mn = (long long)m * n;
  if (mn == 0) return;
  hipLaunchKernelGGL(k_reverse_cols, dim3(nblocks(mn)), dim3(kTB), 0, st, m, n, src, lds, dst,
                     ldd);
  PW_LAUNCH_CHECK();
}

void mul_fields(const double* a, const double* b, double* out, long long n, double scale,
                hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_mul_fields, dim3(nblocks(n)), dim3(kTB), 0, st, a, b, out, n, scale);
  PW_LAUNCH_CHECK();
}

template void widen_fields<float>(const float*, long long, double*, long long, long long, int,
                                  hipStream_t);
template void widen_fields<double>(const double*, long long, double*, long long, long long, int,
                                   hipStream_t);
template void receiver_values<float>(const float*, long long, const long long*, int, int, double*,
                                     hipStream_t);
template void receiver_values<double>(const double*, long long, const long long*, int, int,
                                      double*, hipStream_t);

}  // namespace pw
