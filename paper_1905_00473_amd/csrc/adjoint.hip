// Adjoint building blocks for d J / d c^2 through Algorithm 3 with the
// phase corrector held fixed:
//  * reverse velocity Verlet (Sec. 3.1 scheme run backwards, in leapfrog
//    form: the two half kicks that meet at a level are one kick) with the
//    c^2 gradient accumulated per state, the forward displacements
//    recomputed from checkpoints taken every `ckpt` steps;
//  * transposes of the trigonometric interpolation and of the pointwise
//    restriction;
//  * the receiver misfit and its seed.
// All adjoint arithmetic is FP64; forward states of the FP32 path are
// widened when read.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "pw_internal.h"

namespace pw {
namespace {

constexpr int kTB = 256;
inline unsigned nblocks(long long n, int tb = kTB) { return (unsigned)((n + tb - 1) / tb); }

__device__ __forceinline__ double lane_dn(double v) { return lane_shift<0x130>(v); }   // lane + 1
__device__ __forceinline__ double lane_upv(double v) { return lane_shift<0x138>(v); }  // lane - 1

struct G3 {
  int dim, nx, ny, nz;
  double idx2;
};
inline G3 g3(const Grid& g) { return G3{g.dim, g.n[0], g.n[1], g.n[2], 1.0 / (g.dx * g.dx)}; }

// Launch geometry of the per-point kernels: a 1D grid of blocks of kTB
// points along x.  Blocks are dispatched round-robin over the 8 XCDs, each
// with its own L2; block L is given the logical block (L % 8) * per + L / 8
// so that every XCD sweeps a contiguous range of rows and finds the
// neighbouring rows of its stencils in its own L2.  Logical blocks run
// x-block fastest, then y, z and the state; coordinates need one division
// chain per block, none per thread.
constexpr int kXcd = 8;
struct Pt {
  int x, y, z, s;
  long long J;  // index within the state
  bool ok;
};
// (logical block counts stay below 2^31: 32-bit decoding)
__device__ __forceinline__ Pt point(const G3& g, int nxb, int nblk) {
  Pt p;
  const int per = (nblk + kXcd - 1) / kXcd;
  const int L = (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
  p.ok = L < nblk;
  int r = L;
  const int xb = r % nxb;
  r /= nxb;
  p.y = r % g.ny;
  r /= g.ny;
  p.z = r % g.nz;
  p.s = r / g.nz;
  p.x = xb * kTB + (int)threadIdx.x;
  p.ok = p.ok && p.x < g.nx;
  p.J = (long long)p.x + (long long)g.nx * ((long long)p.y + (long long)g.ny * p.z);
  return p;
}
struct PtLaunch {
  dim3 grid;
  int nxb;
  int nblk;
};
PtLaunch pt_launch(const G3& g, int ns) {
  PtLaunch l;
  l.nxb = (g.nx + kTB - 1) / kTB;
  const long long nblk = (long long)l.nxb * g.ny * g.nz * ns;
  if (nblk >= (1LL << 31) - kXcd) fail(PW_EINVAL, "adjoint launch too large");
  l.nblk = (int)nblk;
  const int per = (l.nblk + kXcd - 1) / kXcd;
  l.grid = dim3((unsigned)per * kXcd);
  return l;
}

// periodic neighbour offsets of a point (2 D of them), relative to it
template <int D>
struct Nbr {
  long long off[2 * D];
};
template <int D>
__device__ __forceinline__ Nbr<D> neighbours(const Pt& p, const G3& g) {
  Nbr<D> nb;
  nb.off[0] = p.x + 1 < g.nx ? 1 : 1 - g.nx;
  nb.off[1] = p.x > 0 ? -1 : g.nx - 1;
  if (D >= 2) {
    const long long sy = g.nx;
    nb.off[2] = p.y + 1 < g.ny ? sy : sy - (long long)g.ny * sy;
    nb.off[3] = p.y > 0 ? -sy : (long long)g.ny * sy - sy;
  }
  if (D >= 3) {
    const long long sz = (long long)g.nx * g.ny;
    nb.off[4] = p.z + 1 < g.nz ? sz : sz - (long long)g.nz * sz;
    nb.off[5] = p.z > 0 ? -sz : (long long)g.nz * sz - sz;
  }
  return nb;
}

// CD2 Laplacian of field f at J (f points at J's field)
template <int D>
__device__ __forceinline__ double lap_nb(const double* f, long long J, const Nbr<D>& nb,
                                         double idx2) {
  double s = -2.0 * D * f[J];
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) s += f[J + nb.off[k]];
  return s * idx2;
}

// Forward recomputation, leapfrog form of velocity Verlet: the state
// carried between steps is (u_i, p_{i-1/2}); one step is the kick at level
// i with weight w (h/2 at level 0, h after) and the drift:
//   p <- p + w c2 Lap u_i,  u_{i+1} = u_i + h p.
template <int D>
__global__ void k_fwd_step(const double* u, long long su, double* p, long long sp, double* un,
                           long long sun, const double* c2, double w, double h, G3 g, int nxb,
                           int nblk) {
  const Pt q = point(g, nxb, nblk);
  if (!q.ok) return;
  const Nbr<D> nb = neighbours<D>(q, g);
  const long long J = q.J;
  const double* us = u + (long long)q.s * su;
  double* ps = p + (long long)q.s * sp;
  const double pv = ps[J] + w * (c2[J] * lap_nb<D>(us, J, nb, g.idx2));
  ps[J] = pv;
  un[(long long)q.s * sun + J] = us[J] + h * pv;
}

// Reverse of the closing half kick at level m (p_m = p_{m-1/2} + h/2 c2 Lap u_m):
//   lu += w Lap(c2 lp),  g += w lp Lap u_m   (w = h/2)
template <int D>
__global__ void k_adj_kick(double* lu, const double* lp, long long sl, const double* u,
                           long long su, double* gacc, long long sg, const double* c2, double w,
                           G3 g, int nxb, int nblk) {
  const Pt q = point(g, nxb, nblk);
  if (!q.ok) return;
  const Nbr<D> nb = neighbours<D>(q, g);
  const long long J = q.J;
  const double* l = lp + (long long)q.s * sl;
  double a = -2.0 * D * c2[J] * l[J];
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) a += c2[J + nb.off[k]] * l[J + nb.off[k]];
  lu[(long long)q.s * sl + J] += w * a * g.idx2;
  gacc[(long long)q.s * sg + J] += w * l[J] * lap_nb<D>(u + (long long)q.s * su, J, nb, g.idx2);
}

// One reverse leapfrog step, from level i+1 to level i, for all ns states
// of a point in one thread: the reverse drift lp' = lp + h lu (pointwise,
// formed at J and its neighbours), then the reverse kick at level i with
// weight w:
//   lu' = lu + w Lap(c2 lp'),  g += w lp' Lap u_i.
// (lu, lp) and (lu', lp') are distinct buffers.  A thread takes the
// states kAdjGroup q .. kAdjGroup q + kAdjGroup - 1 of a point: their c^2
// gradient contributions are summed in a register and added once to field
// q of gacc (the caller sums the fields of gacc).  Per point and state this
// moves 40 B (read lu, lp, u; write lu', lp') plus 16 B per group, instead
// of the 64 B of one thread per state, whose gradient accumulator is read
// and written per state.
constexpr int kAdjGroup = 8;

// Layer (2D): the kick at level i multiplies p by s(x) and weighs the
// acceleration by W(x): s = d, W = h/2 at level 0 (first half kick of the
// slice), s = d^2, W = h/2 (1 + d) where two half kicks meet, with
// d = min(dmx[x], dmy[y]).  Its reverse: lu' = lu + Lap(W c2 lp'),
// lp_out = s lp', g += W lp' Lap u_i.
__device__ __forceinline__ double layer_d(const double* dmx, const double* dmy, int x, int y) {
  return fmin(dmx[x], dmy[y]);
}

template <int D, bool FORCED = false>
__global__ void k_adj_step_grp(const double* lu, const double* lp, long long sl, double* lu2,
                               double* lp2, long long sl2, const double* u, long long su,
                               double* gacc, long long sg, const double* c2, double w, double h,
                               G3 g, int nxb, int nblk, int ns, const double* dmx,
                               const double* dmy, int lev0) {
  const Pt q = point(g, nxb, nblk);  // q.s: state group
  if (!q.ok) return;
  const Nbr<D> nb = neighbours<D>(q, g);
  const long long J = q.J;
  const double cc = c2[J];
  double cn[2 * D];
#pragma unroll
  for (int k = 0; k < 2 * D; ++k) cn[k] = c2[J + nb.off[k]];
  // FORCED (2D): the weights W at J and its neighbours, the factor at J
  double WJ = w, sJ = 1.0;
  if constexpr (FORCED) {
    if (dmx) {
      const int xp = q.x + 1 < g.nx ? q.x + 1 : 0, xm = q.x > 0 ? q.x - 1 : g.nx - 1;
      const int yp = q.y + 1 < g.ny ? q.y + 1 : 0, ym = q.y > 0 ? q.y - 1 : g.ny - 1;
      const double dJ = layer_d(dmx, dmy, q.x, q.y);
      const double dn[4] = {layer_d(dmx, dmy, xp, q.y), layer_d(dmx, dmy, xm, q.y),
                            layer_d(dmx, dmy, q.x, yp), layer_d(dmx, dmy, q.x, ym)};
      WJ = lev0 ? 0.5 * h : 0.5 * h * (1.0 + dJ);
      sJ = lev0 ? dJ : dJ * dJ;
#pragma unroll
      for (int k = 0; k < 2 * D; ++k) cn[k] *= lev0 ? 0.5 * h : 0.5 * h * (1.0 + dn[k]);
    } else {
#pragma unroll
      for (int k = 0; k < 2 * D; ++k) cn[k] *= w;
    }
  }
  const double ccw = FORCED ? cc * WJ : cc;
  double gsum = 0.0;
  const int s1 = min(ns, (q.s + 1) * kAdjGroup);
#pragma unroll 2
  for (int s = q.s * kAdjGroup; s < s1; ++s) {
    const double* lus = lu + (long long)s * sl;
    const double* lps = lp + (long long)s * sl;
    const double lpc = fma(h, lus[J], lps[J]);
    double a = -2.0 * D * ccw * lpc;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
      const long long o = J + nb.off[k];
      a += cn[k] * fma(h, lus[o], lps[o]);
    }
    if constexpr (FORCED) {
      lu2[(long long)s * sl2 + J] = lus[J] + a * g.idx2;
      lp2[(long long)s * sl2 + J] = sJ * lpc;
      gsum += WJ * lpc * lap_nb<D>(u + (long long)s * su, J, nb, g.idx2);
    } else {
      lu2[(long long)s * sl2 + J] = lus[J] + w * a * g.idx2;
      lp2[(long long)s * sl2 + J] = lpc;
      gsum += w * lpc * lap_nb<D>(u + (long long)s * su, J, nb, g.idx2);
    }
  }
  gacc[(long long)q.s * sg + J] += gsum;
}

// per-point fields of the layer for the reverse streams (2D): d =
// min(dmx[x], dmy[y]); wf = (1 + d) / 2, s2 = d^2, dd = d, c2e = c2 wf
__global__ void k_layer_fields(int nx, int ny, const double* dmx, const double* dmy,
                               const double* c2, double* wf, double* s2, double* dd,
                               double* c2e) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nx * ny) return;
  const int x = (int)(t % nx), y = (int)(t / nx);
  const double d = fmin(dmx[x], dmy[y]);
  const double w = 0.5 * (1.0 + d);
  wf[t] = w;
  s2[t] = d * d;
  dd[t] = d;
  c2e[t] = c2[t] * w;
}

// lp <- d lp (the layer's factor of a closing half kick, 2D)
__global__ void k_damp_fields(double* lp, long long sl, const double* dmx, const double* dmy,
                              G3 g, int nxb, int nblk) {
  const Pt q = point(g, nxb, nblk);
  if (!q.ok) return;
  lp[(long long)q.s * sl + q.J] *= layer_d(dmx, dmy, q.x, q.y);
}

// lu[s sl + rec[r]] += seeds[(s m_tr + step) n_rec + r] (distinct receivers)
__global__ void k_inject_seeds(double* lu, long long sl, const long long* rec, int nrec,
                               const double* seeds, int m_tr, int step, int ns) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nrec * ns) return;
  const int s = (int)(t / nrec), r = (int)(t - (long long)s * nrec);
  lu[(long long)s * sl + rec[r]] += seeds[((long long)s * m_tr + step) * nrec + r];
}

// Reverse leapfrog steps in 2D as a row stream, RB steps per launch
// (pipeline stages held in registers, as in the forward streaming
// propagator): one wavefront owns 64 - 2 RB output columns of one state
// (RB halo lanes on each side, the x neighbours from the adjacent lanes) and
// walks down a segment of rows.  Stage j performs reverse step top - j on
// the row r = t - 2j of stream step t: from (lu, lp) at level top - j + 1,
//   lp' = lp + h lu,  lu' = lu + w Lap(c2 lp'),  g += w lp' Lap u_{top-j},
// reading u of its level from the segment store and its input rows from the
// stage before (stage 0 from memory).  g is read at stage 0, carried through
// the stages and written after the last, so the contributions are added in
// the order of one launch per step.  Per point and step: 8 B of u, plus
// 48 B per launch (lu, lp in and out, g in and out).
constexpr int kAdjRB = 4;

struct AdjStreamDesc {
  const double* lu_in;
  const double* lp_in;
  long long s_in;
  double* lu_out;
  double* lp_out;
  long long s_out;
  const double* useg;  // level 0 of the segment store
  long long s_lev, s_u;  // stride of a level, of a state within a level
  double* gacc;
  long long sg;
  const double* c2;
  double h, idx2;
  double w[kAdjRB];
  int top, nsteps;
  int nx, ny, ncb, nseg, Ly, nstates;
  // forced launches: the layer as per-point fields (null: none; see
  // Force), the level of the slice at segment level 0, and the receiver
  // seeds (null: none)
  const double* wf;
  const double* s2;
  const double* dd;
  const double* c2e;
  int lev_base;
  const int* rec_rows;
  const int* rec_map;
  const double* seeds;
  int n_rec, m_tr;
};

// FORCED: the layer (and the level-0 half kick); SEEDS: also the receiver
// seeds (a separate instantiation, as for the forward record)
template <bool FORCED, bool SEEDS = false>
__global__ __launch_bounds__(256) void k_adj_stream2d(AdjStreamDesc a) {
  constexpr int B = kAdjRB;
  constexpr int H = B;
  constexpr int XV = 64 - 2 * H;
  const long long nwaves = (long long)a.nstates * a.ncb * a.nseg;
  // blocks of one XCD take consecutive waves (neighbouring segments share
  // halo rows in that XCD's L2)
  const long long nblk = (nwaves + 3) / 4;
  long long blk = blockIdx.x;
  if ((nblk & 7) == 0) blk = (blk & 7) * (nblk >> 3) + (blk >> 3);
  const long long wid = blk * 4 + (threadIdx.x >> 6);
  if (wid >= nwaves) return;
  const int lane = threadIdx.x & 63;
  const int cb = (int)(wid % a.ncb);
  const int seg = (int)((wid / a.ncb) % a.nseg);
  const int st = (int)(wid / ((long long)a.ncb * a.nseg));
  const int nx = a.nx, ny = a.ny;
  int gx = (cb * XV - H + lane) % nx;
  if (gx < 0) gx += nx;
  const bool out_lane = lane >= H && lane < 64 - H && (cb * XV + lane - H) < nx;
  const int Y0 = seg * a.Ly;
  const int Y1 = min(Y0 + a.Ly, ny);
  auto rowidx = [&](int y) -> long long {
    int r = y % ny;
    if (r < 0) r += ny;
    return (long long)r * nx + gx;
  };
  const double* lui = a.lu_in + (long long)st * a.s_in;
  const double* lpi = a.lp_in + (long long)st * a.s_in;
  double* gs = a.gacc + (long long)st * a.sg;
  // the layer: a kick at level 0 of the slice is a half kick (weight h/2,
  // factor d); elsewhere two half kicks meet (weight h/2 (1 + d) = h wf,
  // factor d^2), so that W c2 = h c2e: the unforced formulas with c2e in
  // place of c2, the gradient weight wf and the factor applied to lp'
  const bool damp = FORCED && a.c2e != nullptr;
  // row of a logical index within one period of the grid (the general
  // modulo only for grids smaller than the stream's reach)
  auto near_row = [&](int y) {
    const int w = y < 0 ? y + ny : (y >= ny ? y - ny : y);
    if ((unsigned)w < (unsigned)ny) return w;
    int r = y % ny;
    return r < 0 ? r + ny : r;
  };
  const double* ul[B];
#pragma unroll
  for (int j = 0; j < B; ++j)
    ul[j] = a.useg + (long long)(j < a.nsteps ? a.top - j : a.top) * a.s_lev +
            (long long)st * a.s_u;
  // stage j: windows of its input level, rows (r-1, r, r+1) of q = c2 lp'
  // and of u (its own level); rows (r, r+1) of lu, lp' and the carried g;
  // pending row r+2 (from stage j-1, or loaded for j = 0)
  double wq[B][3], wu[B][3], wl[B][2], wp[B][2], wg[B][2];
  double pl[B], pp[B], pg[B];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    wq[j][0] = wq[j][1] = wq[j][2] = 0.0;
    wu[j][0] = wu[j][1] = wu[j][2] = 0.0;
    wl[j][0] = wl[j][1] = wp[j][0] = wp[j][1] = wg[j][0] = wg[j][1] = 0.0;
    pl[j] = pp[j] = pg[j] = 0.0;
  }
  const int tbeg = Y0 - H - 2;
  const int tend = Y1 - 1 + 2 * (B - 1);
  for (int t = tbeg; t <= tend; ++t) {
    // input level, row t+2 -> pending slot of stage 0
    if (t + 2 < Y1 + H) {
      const long long gi = rowidx(t + 2);
      pl[0] = lui[gi];
      pp[0] = lpi[gi];
      pg[0] = (t + 2 >= Y0 && t + 2 < Y1) ? gs[gi] : 0.0;
    }
    // the layer factor of every stage's centre row, loaded together ahead
    // of the stages (the row index is wave-uniform)
    double ddv[B];
    if constexpr (FORCED) {
      const int tu = __builtin_amdgcn_readfirstlane(t);
#pragma unroll
      for (int j = 0; j < B; ++j)
        ddv[j] = (damp && j < a.nsteps) ? a.dd[(long long)near_row(tu - 2 * j) * nx + gx] : 1.0;
    }
    // every stage takes its pending row into its windows (lp', q) and
    // loads the same row of its u level; then processes its centre row
    double ol[B], op[B], og[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int r = t - 2 * j;
      const double lc = wl[j][0], pc = wp[j][0], gc = wg[j][0];
      double lo = lc, po = pc, go = gc;
      if (j < a.nsteps) {
        const double uc = wu[j][1];
        const double qc = wq[j][1];
        // neighbours in the order x+1, x-1, y+1, y-1
        double aa = -2.0 * 2 * qc;
        aa += lane_dn(qc);
        aa += lane_upv(qc);
        aa += wq[j][2];
        aa += wq[j][0];
        double lu_ = -2.0 * 2 * uc;
        lu_ += lane_dn(uc);
        lu_ += lane_upv(uc);
        lu_ += wu[j][2];
        lu_ += wu[j][0];
        lo = lc + a.w[j] * aa * a.idx2;
        if constexpr (FORCED) {
          if (damp) {
            const bool lev0 = a.lev_base + a.top - j == 0;
            const double dc = ddv[j];
            go = gc + a.w[j] * (lev0 ? 1.0 : 0.5 * (1.0 + dc)) * pc * (lu_ * a.idx2);
            po = (lev0 ? dc : dc * dc) * pc;
          } else {
            go = gc + a.w[j] * pc * (lu_ * a.idx2);
          }
        } else {
          go = gc + a.w[j] * pc * (lu_ * a.idx2);
        }
      }
      (void)r;
      ol[j] = lo;
      op[j] = po;
      og[j] = go;
    }
    // outputs: stage j's row goes to stage j+1 (the last stage writes)
#pragma unroll
    for (int j = 0; j + 1 < B; ++j) {
      pl[j + 1] = ol[j];
      pp[j + 1] = op[j];
      pg[j + 1] = og[j];
    }
    {
      const int orow = t - 2 * (B - 1);
      if (out_lane && orow >= Y0 && orow < Y1) {
        const long long gi = (long long)orow * nx + gx;
        a.lu_out[(long long)st * a.s_out + gi] = ol[B - 1];
        a.lp_out[(long long)st * a.s_out + gi] = op[B - 1];
        gs[gi] = og[B - 1];
      }
    }
    // advance every window by one row, taking in the pending row: lp' and
    // q = c2 lp' of the incoming row (pointwise), and the same row of u
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int rin = t + 2 - 2 * j;  // row of the pending slot of stage j
      const long long gi = rowidx(rin);
      const double* cq = a.c2;
      if constexpr (FORCED) {
        if (j < a.nsteps) {
          const int lev = a.lev_base + a.top - j;
          if (damp && lev != 0) cq = a.c2e;
          // receiver seed of u at level lev + 1 (record index lev)
          if (SEEDS) {
            const int ry = near_row(rin);
            if (a.rec_rows[ry]) {
              const int rid = a.rec_map[gi];
              if (rid >= 0) pl[j] += a.seeds[((long long)st * a.m_tr + lev) * a.n_rec + rid];
            }
          }
        }
      }
      const double lpn = (j < a.nsteps) ? fma(a.h, pl[j], pp[j]) : pp[j];
      wq[j][0] = wq[j][1];
      wq[j][1] = wq[j][2];
      wq[j][2] = cq[gi] * lpn;
      wu[j][0] = wu[j][1];
      wu[j][1] = wu[j][2];
      wu[j][2] = ul[j][gi];
      wl[j][0] = wl[j][1];
      wl[j][1] = pl[j];
      wp[j][0] = wp[j][1];
      wp[j][1] = lpn;
      wg[j][0] = wg[j][1];
      wg[j][1] = pg[j];
    }
  }
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

// Register-blocked variant for a compile-time ratio R: a thread produces RM
// consecutive coarse outputs m, so every fine value loaded feeds RM
// accumulators; over RM consecutive J the weight index J - m takes 2 RM - 1
// values per phase, read from LDS once per block.  The terms of each output
// are added in the order of k_interp_T_axis (J ascending, s ascending).
template <int R, int RM>
__global__ __launch_bounds__(256) void k_interp_T_axis_rb(const double* in, long long sin,
                                                          double* out, long long sout,
                                                          const double* tab, int outer, int nc,
                                                          int inner, int nfields) {
  extern __shared__ double wt[];
  for (int t = threadIdx.x; t < R * nc; t += blockDim.x) wt[t] = tab[t];
  __syncthreads();
  const int nmb = (nc + RM - 1) / RM;
  const long long per = (long long)outer * nmb * inner;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nfields) return;
  const int f = (int)(t / per);
  long long rr = t - (long long)f * per;
  const int i = (int)(rr % inner);
  rr /= inner;
  const int mb = (int)(rr % nmb);
  const int o = (int)(rr / nmb);
  const int m0 = mb * RM;
  const double* src = in + (long long)f * sin + (long long)o * nc * R * inner + i;
  double acc[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a)
    acc[a] = (m0 + a < nc) ? src[(long long)R * (m0 + a) * inner] : 0.0;
  int J = 0;
  for (; J + RM <= nc; J += RM) {
    double x[RM][R];
#pragma unroll
    for (int u = 0; u < RM; ++u)
#pragma unroll
      for (int s = 1; s < R; ++s) x[u][s] = src[((long long)R * (J + u) + s) * inner];
    double w[R][2 * RM - 1];  // w[s][k] = w_s[(J - m0 + k - (RM - 1)) mod nc]
#pragma unroll
    for (int s = 1; s < R; ++s)
#pragma unroll
      for (int k = 0; k < 2 * RM - 1; ++k) {
        // J - m0 + k - (RM - 1) lies in (-nc - RM, nc): at most two wraps
        int d = J - m0 + k - (RM - 1);
        d += d < 0 ? nc : 0;
        d += d < 0 ? nc : 0;
        w[s][k] = wt[s * nc + d];
      }
#pragma unroll
    for (int u = 0; u < RM; ++u)
#pragma unroll
      for (int s = 1; s < R; ++s)
#pragma unroll
        for (int a = 0; a < RM; ++a) acc[a] += w[s][u - a + RM - 1] * x[u][s];
  }
  for (; J < nc; ++J) {
#pragma unroll
    for (int s = 1; s < R; ++s) {
      const double x = src[((long long)R * J + s) * inner];
#pragma unroll
      for (int a = 0; a < RM; ++a) {
        int d = (J - m0 - a) % nc;
        d += d < 0 ? nc : 0;
        acc[a] += wt[s * nc + d] * x;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < RM; ++a)
    if (m0 + a < nc) out[(long long)f * sout + ((long long)o * nc + m0 + a) * inner + i] = acc[a];
}

// one transposed interpolation pass: fine (outer, nc*ratio, inner) ->
// coarse (outer, nc, inner)
void interp_T_pass(const double* in, long long sin, double* out, long long sout,
                   const double* tab, int outer, int nc, int ratio, int inner, int nfields,
                   hipStream_t st) {
  constexpr int RM = 4;
  if (ratio == 4 || ratio == 2) {
    const long long n = (long long)outer * ((nc + RM - 1) / RM) * inner * nfields;
    const size_t smem = sizeof(double) * (size_t)ratio * nc;
    if (ratio == 4)
      hipLaunchKernelGGL((k_interp_T_axis_rb<4, RM>), dim3(nblocks(n)), dim3(kTB), smem, st, in,
                         sin, out, sout, tab, outer, nc, inner, nfields);
    else
      hipLaunchKernelGGL((k_interp_T_axis_rb<2, RM>), dim3(nblocks(n)), dim3(kTB), smem, st, in,
                         sin, out, sout, tab, outer, nc, inner, nfields);
  } else {
    const long long n = (long long)outer * nc * inner * nfields;
    hipLaunchKernelGGL(k_interp_T_axis, dim3(nblocks(n)), dim3(kTB), 0, st, in, sin, out, sout,
                       tab, outer, nc, ratio, inner, nfields);
  }
  PW_LAUNCH_CHECK();
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

template <int D>
void vv_adjoint_d(const Grid& grid, const double* c2, const double* u0, const double* p0,
                long long s0, double* lu, double* lp, long long sl, double* gacc, long long sg,
                int ns, int m, double h, int ckpt, const AdjScratch& sc, hipStream_t st,
                const Force<double>* fo) {
  if (ns == 0 || m == 0) return;
  if (ckpt < 1) fail(PW_EINVAL, "checkpoint interval must be >= 1");
  if (fo && D != 2) fail(PW_EINVAL, "the absorbing layer and source are 2D only");
  if (fo && fo->seeds && (!fo->rec || !fo->rec_rows || !fo->rec_map || fo->m_tr < m))
    fail(PW_EINVAL, "receiver seeds need the receiver tables and m steps per state");
  const double* dmx = fo ? fo->dmp_x : nullptr;
  const double* dmy = fo ? fo->dmp_y : nullptr;
  const long long np = grid.npts();
  const G3 g = g3(grid);
  const PtLaunch pl = pt_launch(g, ns);
  const PtLaunch pg = pt_launch(g, (ns + kAdjGroup - 1) / kAdjGroup);  // per state group
  const dim3 gr = pl.grid;
  const int nseg = (m + ckpt - 1) / ckpt;
  if ((long long)ns * np > sc.state_elems) fail(PW_EINVAL, "adjoint scratch too small");
  if (nseg > sc.max_ckpt) fail(PW_EINVAL, "too many checkpoints for the adjoint scratch");
  if (std::min(m, ckpt) + 1 > sc.max_seg) fail(PW_EINVAL, "checkpoint segment too long");
  const long long S = sc.state_elems;  // stride of one stored time level
  auto wk = [&](int level) { return level == 0 ? 0.5 * h : h; };
  // forward pass: checkpoints (u_i, p_{i-1/2}) at the start of every
  // segment (p_{-1/2} = p_0, with the half kick at level 0)
  copy_fields(u0, s0, sc.ck_u, np, np, ns, st);
  copy_fields(p0, s0, sc.ck_p, np, np, ns, st);
  for (int seg = 0; seg + 1 < nseg; ++seg) {
    if (D == 2) {
      // the streaming propagator, levels into the segment store
      const double* pf = leapfrog_levels2d(grid, c2, sc.ck_u + seg * S, sc.ck_p + seg * S,
                                           sc.p_tmp, sc.p_tmp2, np, ns, ckpt, h, seg == 0, sc.seg,
                                           S, st, fo, seg * ckpt);
      copy_fields(sc.seg + (long long)(ckpt - 1) * S, np, sc.ck_u + (seg + 1) * S, np, np, ns,
                  st);
      copy_fields(pf, np, sc.ck_p + (seg + 1) * S, np, np, ns, st);
      continue;
    }
    const double* cu = sc.ck_u + seg * S;
    double* nu = sc.ck_u + (seg + 1) * S;
    double* npp = sc.ck_p + (seg + 1) * S;
    copy_fields(sc.ck_p + seg * S, np, npp, np, np, ns, st);
    const double* src = cu;
    for (int i = 0; i < ckpt; ++i) {
      double* dst = (i == ckpt - 1) ? nu : sc.seg + (long long)(i % 2) * S;
      hipLaunchKernelGGL(k_fwd_step<D>, gr, dim3(kTB), 0, st, src, np, npp, np, dst, np, c2,
                         wk(seg * ckpt + i), h, g, pl.nxb, pl.nblk);
      PW_LAUNCH_CHECK();
      src = dst;
    }
  }
  // reverse over the segments.  (lu, lp) ping-pong between the caller's
  // arrays (stride sl) and scratch (stride np).
  double* lua = lu;
  double* lpa = lp;
  long long sa = sl;
  double* lub = sc.a_tmp;
  double* lpb = sc.lp_tmp;
  long long sb = np;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int i0 = seg * ckpt;
    const int len = std::min(ckpt, m - i0);
    // displacements u_{i0} .. u_{i0+len} in the segment store
    copy_fields(sc.ck_u + seg * S, np, sc.seg, np, np, ns, st);
    if (D == 2) {
      leapfrog_levels2d(grid, c2, sc.ck_u + seg * S, sc.ck_p + seg * S, sc.p_tmp, sc.p_tmp2, np,
                        ns, len, h, i0 == 0, sc.seg + S, S, st, fo, i0);
    } else {
      copy_fields(sc.ck_p + seg * S, np, sc.p_tmp, np, np, ns, st);
      for (int i = 0; i < len; ++i) {
        hipLaunchKernelGGL(k_fwd_step<D>, gr, dim3(kTB), 0, st,
                           (const double*)(sc.seg + (long long)i * S), np, sc.p_tmp, np,
                           sc.seg + (long long)(i + 1) * S, np, c2, wk(i0 + i), h, g, pl.nxb,
                           pl.nblk);
        PW_LAUNCH_CHECK();
      }
    }
    if (seg == nseg - 1) {
      // closing half kick at level m
      hipLaunchKernelGGL(k_adj_kick<D>, gr, dim3(kTB), 0, st, lua, (const double*)lpa, sa,
                         (const double*)(sc.seg + (long long)len * S), np, gacc, sg, c2, 0.5 * h,
                         g, pl.nxb, pl.nblk);
      PW_LAUNCH_CHECK();
      if (dmx) {  // the closing half kick's factor d
        hipLaunchKernelGGL(k_damp_fields, gr, dim3(kTB), 0, st, lpa, sa, dmx, dmy, g, pl.nxb,
                           pl.nblk);
        PW_LAUNCH_CHECK();
      }
    }
    if (D == 2 && (long long)ns * np >= (1LL << 18)) {
      // kAdjRB reverse steps per launch (launches too small to fill the
      // chip, such as one coarse state, keep one step per launch: a stream
      // is a serial chain of row steps)
      AdjStreamDesc d{};
      if (fo) {
        if (dmx && !fo->c2e) fail(PW_EINVAL, "the layer's reverse streams need its fields");
        d.wf = fo->wf;
        d.s2 = fo->s2;
        d.dd = fo->dd;
        d.c2e = fo->c2e;
        d.lev_base = i0;
        d.rec_rows = fo->rec_rows;
        d.rec_map = fo->rec_map;
        d.seeds = fo->seeds;
        d.n_rec = fo->n_rec;
        d.m_tr = fo->m_tr;
      }
      d.useg = sc.seg;
      d.s_lev = S;
      d.s_u = np;
      d.gacc = gacc;
      d.sg = sg;
      d.c2 = c2;
      d.h = h;
      d.idx2 = g.idx2;
      d.nx = g.nx;
      d.ny = g.ny;
      d.nstates = ns;
      d.ncb = (g.nx + (64 - 2 * kAdjRB) - 1) / (64 - 2 * kAdjRB);
      {
        // about 1920 streams (measured best on 32 states of 512^2: longer
        // segments repeat fewer halo rows), segments of at least 16 rows
        static const long long want_env = [] {
          const char* e = getenv("PW_ADJ_STREAMS");  // tuning override
          return e ? atoll(e) : 0LL;
        }();
        const long long want = want_env > 0 ? want_env : 1920;
        const long long lanes = (long long)ns * d.ncb;
        long long nsg = (want + lanes - 1) / lanes;
        nsg = std::max(1LL, std::min(nsg, (long long)((g.ny + 15) / 16)));
        d.Ly = (int)((g.ny + nsg - 1) / nsg);
        d.nseg = (g.ny + d.Ly - 1) / d.Ly;
      }
      const long long nw = (long long)ns * d.ncb * d.nseg;
      if ((nw + 3) / 4 >= (1LL << 31)) fail(PW_EINVAL, "adjoint launch too large");
      for (int i = len - 1; i >= 0;) {
        d.top = i;
        d.nsteps = std::min(kAdjRB, i + 1);
        for (int j = 0; j < kAdjRB; ++j) d.w[j] = j < d.nsteps ? wk(i0 + i - j) : 0.0;
        d.lu_in = lua;
        d.lp_in = lpa;
        d.s_in = sa;
        d.lu_out = lub;
        d.lp_out = lpb;
        d.s_out = sb;
        if (fo && fo->seeds)
          hipLaunchKernelGGL((k_adj_stream2d<true, true>), dim3((unsigned)((nw + 3) / 4)),
                             dim3(256), 0, st, d);
        else if (fo)
          hipLaunchKernelGGL(k_adj_stream2d<true>, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0,
                             st, d);
        else
          hipLaunchKernelGGL(k_adj_stream2d<false>, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0,
                             st, d);
        PW_LAUNCH_CHECK();
        std::swap(lua, lub);
        std::swap(lpa, lpb);
        std::swap(sa, sb);
        i -= d.nsteps;
      }
    } else {
      for (int i = len - 1; i >= 0; --i) {
        if (fo && fo->seeds) {  // receiver seeds of u at level i0 + i + 1
          const long long nt = (long long)fo->n_rec * ns;
          hipLaunchKernelGGL(k_inject_seeds, dim3(nblocks(nt)), dim3(kTB), 0, st, lua, sa, fo->rec,
                             fo->n_rec, fo->seeds, fo->m_tr, i0 + i, ns);
          PW_LAUNCH_CHECK();
        }
        if constexpr (D == 2) {
          if (fo) {
            hipLaunchKernelGGL((k_adj_step_grp<D, true>), pg.grid, dim3(kTB), 0, st,
                               (const double*)lua, (const double*)lpa, sa, lub, lpb, sb,
                               (const double*)(sc.seg + (long long)i * S), np, gacc, sg, c2,
                               wk(i0 + i), h, g, pg.nxb, pg.nblk, ns, dmx, dmy,
                               (int)(i0 + i == 0));
            PW_LAUNCH_CHECK();
            std::swap(lua, lub);
            std::swap(lpa, lpb);
            std::swap(sa, sb);
            continue;
          }
        }
        hipLaunchKernelGGL((k_adj_step_grp<D, false>), pg.grid, dim3(kTB), 0, st,
                           (const double*)lua, (const double*)lpa, sa, lub, lpb, sb,
                           (const double*)(sc.seg + (long long)i * S), np, gacc, sg, c2,
                           wk(i0 + i), h, g, pg.nxb, pg.nblk, ns, (const double*)nullptr,
                           (const double*)nullptr, 0);
        PW_LAUNCH_CHECK();
        std::swap(lua, lub);
        std::swap(lpa, lpb);
        std::swap(sa, sb);
      }
    }
  }
  if (lua != lu) {
    copy_fields(lua, sa, lu, sl, np, ns, st);
    copy_fields(lpa, sa, lp, sl, np, ns, st);
  }
}

void vv_adjoint(const Grid& grid, const double* c2, const double* u0, const double* p0,
                long long s0, double* lu, double* lp, long long sl, double* gacc, long long sg,
                int ns, int m, double h, int ckpt, const AdjScratch& sc, hipStream_t st,
                const Force<double>* fo) {
  if (grid.dim == 1)
    vv_adjoint_d<1>(grid, c2, u0, p0, s0, lu, lp, sl, gacc, sg, ns, m, h, ckpt, sc, st, fo);
  else if (grid.dim == 2)
    vv_adjoint_d<2>(grid, c2, u0, p0, s0, lu, lp, sl, gacc, sg, ns, m, h, ckpt, sc, st, fo);
  else
    vv_adjoint_d<3>(grid, c2, u0, p0, s0, lu, lp, sl, gacc, sg, ns, m, h, ckpt, sc, st, fo);
}

void layer_fields(const Grid& g, const double* dmx, const double* dmy, const double* c2,
                  double* out, hipStream_t st) {
  if (g.dim != 2) fail(PW_EINVAL, "the absorbing layer is 2D only");
  const long long np = g.npts();
  hipLaunchKernelGGL(k_layer_fields, dim3(nblocks(np)), dim3(kTB), 0, st, g.n[0], g.n[1], dmx,
                     dmy, c2, out, out + np, out + 2 * np, out + 3 * np);
  PW_LAUNCH_CHECK();
}

void interp_transpose(const Grid& f, const Grid& c, int ratio, const double* const* tables,
                      const double* in, long long sin, double* out, long long sout, int nfields,
                      double* tmp, hipStream_t st) {
  if (nfields == 0) return;
  const int d = f.dim;
  const int fx = f.n[0], fy = f.n[1];
  const int cx = c.n[0], cy = c.n[1], cz = c.n[2];
  if (d == 1) {
    interp_T_pass(in, sin, out, sout, tables[0], 1, cx, ratio, 1, nfields, st);
    return;
  }
  if (d == 2) {
    // y transpose: (1, fy, fx) -> tmp (1, cy, fx); x transpose: (cy, fx, 1) -> out
    const long long sA = (long long)cy * fx;
    interp_T_pass(in, sin, tmp, sA, tables[1], 1, cy, ratio, fx, nfields, st);
    interp_T_pass(tmp, sA, out, sout, tables[0], cy, cx, ratio, 1, nfields, st);
    return;
  }
  // 3D: z: (1, fz, fy*fx) -> A (1, cz, fy*fx); y: (cz, fy, fx) -> B (cz, cy, fx);
  // x: (cz*cy, fx, 1) -> out
  const long long sA = (long long)cz * fy * fx;
  const long long sB = (long long)cz * cy * fx;
  double* A = tmp;
  double* B = tmp + sA * nfields;
  interp_T_pass(in, sin, A, sA, tables[2], 1, cz, ratio, fy * fx, nfields, st);
  interp_T_pass(A, sA, B, sB, tables[1], cz, cy, ratio, fx, nfields, st);
  interp_T_pass(B, sB, out, sout, tables[0], cz * cy, cx, ratio, 1, nfields, st);
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
