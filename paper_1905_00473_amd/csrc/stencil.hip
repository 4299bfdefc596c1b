// Fine and coarse propagators (Sec. 3.1): periodic second-order central
// difference Laplacian + velocity Verlet, batched over states.
//
// Inside one launch the velocity-Verlet half kicks of consecutive steps are
// merged into one full kick (the leapfrog form): starting from the true
// state (u_i, p_i) at a slice start the first kick is a half kick, the last
// launch of a slice closes with a half kick.  Between launches of the same
// slice the carried momentum is the half-step one.
//
// Three kernels:
//  * k_prop_line: a 1D periodic line lives entirely in LDS; all steps of a
//    propagation run in one launch (no halo).
//  * k_prop_stream2d: 2D grids; each wavefront streams down its columns with
//    the time steps of a launch pipelined in registers (see below).
//  * k_prop_tile: 3D (and long 1D) grids are cut into tiles; a tile plus
//    a halo of H = (steps in this launch) + (closing kick) points is loaded,
//    every thread keeps u, p, c^2 (and the compensation terms) of its points
//    in registers, u is mirrored in LDS for the neighbour reads, and the
//    valid region shrinks by one point per Laplacian evaluation, so after
//    H evaluations the tile interior is exact.
//
// FP32 compensated mode: every increment of p and u is added with Kahan's
// compensated summation; the compensation is carried across launches of a
// slice and folded into the state at the slice end.
#include <algorithm>

#include <cstdlib>

#include "pw_internal.h"

namespace pw {
namespace {

template <typename T>
struct PropArgs {
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
  int nx, ny, nz;
  int tx, ty, tz;     // tile interior
  int ntx, nty, ntz;  // tiles per axis
  int H;              // halo
  int rx, ry, rz;     // region = tile + 2H per used axis
  int nstates;
  T h, idx2;
  int nsteps, first, last;
};

__device__ __forceinline__ int wrap_idx(int g, int n) {
  g %= n;
  return g < 0 ? g + n : g;
}

// the same for an index within one period of the range (one add or
// subtract); the general form only where it is not (tiny grids)
__device__ __forceinline__ int wrap_near(int g, int n) {
  const int w = g < 0 ? g + n : (g >= n ? g - n : g);
  return (unsigned)w < (unsigned)n ? w : wrap_idx(g, n);
}

// s += x, with Kahan compensation e when COMP
template <typename T, bool COMP>
__device__ __forceinline__ void kadd(T& s, T& e, T x) {
  if constexpr (COMP) {
    const T y = x - e;
    const T t = s + y;
    e = (t - s) - y;
    s = t;
  } else {
    s += x;
  }
}

// ---------------------------------------------------------------------------
// whole periodic line in LDS
// ---------------------------------------------------------------------------
template <typename T, bool COMP, int NT, int PPT>
__global__ __launch_bounds__(NT) void k_prop_line(PropArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T* su = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  const int n = a.nx;
  T* se = su + n;  // COMP: the displacement's compensation term
  const long long base = (long long)blockIdx.x * a.sstride;
  T ru[PPT], rp[PPT], rc[PPT], reu[PPT], rep[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * NT;
    ru[k] = rp[k] = rc[k] = reu[k] = rep[k] = T(0);
    if (i < n) {
      ru[k] = a.u_in[base + i];
      rp[k] = a.p_in[base + i];
      rc[k] = a.c2[i];
      if (COMP && !a.first) {
        reu[k] = a.eu_in[base + i];
        rep[k] = a.ep_in[base + i];
      }
      su[i] = ru[k];
      if (COMP) se[i] = reu[k];
    }
  }
  __syncthreads();
  for (int j = 0; j < a.nsteps; ++j) {
    const T w = (a.first && j == 0) ? a.h * T(0.5) : a.h;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int i = tid + k * NT;
      if (i < n) {
        const int im = i == 0 ? n - 1 : i - 1;
        const int ip = i == n - 1 ? 0 : i + 1;
        T lap = su[ip] - T(2) * ru[k] + su[im];
        if (COMP) lap -= se[ip] - T(2) * reu[k] + se[im];  // second difference of u - e
        kadd<T, COMP>(rp[k], rep[k], w * (rc[k] * (lap * a.idx2)));
        kadd<T, COMP>(ru[k], reu[k], a.h * rp[k]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int i = tid + k * NT;
      if (i < n) {
        su[i] = ru[k];
        if (COMP) se[i] = reu[k];
      }
    }
    __syncthreads();
  }
  if (a.last) {
    const T w = a.h * T(0.5);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int i = tid + k * NT;
      if (i < n) {
        const int im = i == 0 ? n - 1 : i - 1;
        const int ip = i == n - 1 ? 0 : i + 1;
        T lap = su[ip] - T(2) * ru[k] + su[im];
        if (COMP) lap -= se[ip] - T(2) * reu[k] + se[im];
        kadd<T, COMP>(rp[k], rep[k], w * (rc[k] * (lap * a.idx2)));
      }
    }
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * NT;
    if (i < n) {
      if (COMP && a.last) {
        a.u_out[base + i] = ru[k] - reu[k];
        a.p_out[base + i] = rp[k] - rep[k];
      } else {
        a.u_out[base + i] = ru[k];
        a.p_out[base + i] = rp[k];
        if (COMP) {
          a.eu_out[base + i] = reu[k];
          a.ep_out[base + i] = rep[k];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// tiled, time-blocked kernel for D = 1, 2, 3
// ---------------------------------------------------------------------------
template <typename T, int D, bool COMP, int NT, int PPT>
__global__ __launch_bounds__(NT) void k_prop_tile(PropArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T* su = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  const int ntiles = a.ntx * a.nty * a.ntz;
  const long long total = (long long)ntiles * a.nstates;
  long long b = blockIdx.x;
  // consecutive block ids go to different XCDs; remap so that the blocks
  // of one XCD cover consecutive tiles (shared halos stay in one L2)
  if ((total & 7) == 0) b = (b & 7) * (total >> 3) + (b >> 3);
  const int state = (int)(b / ntiles);
  const int tile = (int)(b - (long long)state * ntiles);
  const int tix = tile % a.ntx;
  const int tiy = (tile / a.ntx) % a.nty;
  const int tiz = tile / (a.ntx * a.nty);
  const int H = a.H;
  const int ox = tix * a.tx - H;
  const int oy = (D >= 2) ? tiy * a.ty - H : 0;
  const int oz = (D >= 3) ? tiz * a.tz - H : 0;
  const int rx = a.rx, ry = a.ry, rz = a.rz;
  const int RN = rx * ry * rz;
  const int sy = rx, sz = rx * ry;
  T* se = su + RN;  // COMP: the displacement's compensation term
  const long long base = (long long)state * a.sstride;

  T ru[PPT], rp[PPT], rc[PPT], reu[PPT], rep[PPT];
  unsigned inner = 0u;  // bit k: point k has all neighbours inside the region
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * NT;
    ru[k] = rp[k] = rc[k] = reu[k] = rep[k] = T(0);
    if (i < RN) {
      const int x = i % rx;
      const int y = (i / rx) % ry;
      const int z = i / sz;
      bool ring = (x == 0 || x == rx - 1);
      if (D >= 2) ring = ring || (y == 0 || y == ry - 1);
      if (D >= 3) ring = ring || (z == 0 || z == rz - 1);
      if (!ring) inner |= (1u << k);
      const int gx = wrap_idx(ox + x, a.nx);
      const int gy = (D >= 2) ? wrap_idx(oy + y, a.ny) : 0;
      const int gz = (D >= 3) ? wrap_idx(oz + z, a.nz) : 0;
      const long long gi = (long long)gx + (long long)a.nx * (gy + (long long)a.ny * gz);
      ru[k] = a.u_in[base + gi];
      rp[k] = a.p_in[base + gi];
      rc[k] = a.c2[gi];
      if (COMP && !a.first) {
        reu[k] = a.eu_in[base + gi];
        rep[k] = a.ep_in[base + gi];
      }
      su[i] = ru[k];
      if (COMP) se[i] = reu[k];
    }
  }
  __syncthreads();

  auto kick = [&](T w) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (inner & (1u << k)) {
        const int i = tid + k * NT;
        const T uc = ru[k];
        T lap = su[i + 1] - T(2) * uc + su[i - 1];
        if (D >= 2) lap += su[i + sy] - T(2) * uc + su[i - sy];
        if (D >= 3) lap += su[i + sz] - T(2) * uc + su[i - sz];
        if (COMP) {  // second difference of u - e
          const T ec = reu[k];
          T le = se[i + 1] - T(2) * ec + se[i - 1];
          if (D >= 2) le += se[i + sy] - T(2) * ec + se[i - sy];
          if (D >= 3) le += se[i + sz] - T(2) * ec + se[i - sz];
          lap -= le;
        }
        kadd<T, COMP>(rp[k], rep[k], w * (rc[k] * (lap * a.idx2)));
      }
    }
  };

  for (int j = 0; j < a.nsteps; ++j) {
    kick((a.first && j == 0) ? a.h * T(0.5) : a.h);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (tid + k * NT < RN) kadd<T, COMP>(ru[k], reu[k], a.h * rp[k]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int i = tid + k * NT;
      if (i < RN) {
        su[i] = ru[k];
        if (COMP) se[i] = reu[k];
      }
    }
    __syncthreads();
  }
  if (a.last) kick(a.h * T(0.5));

#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int i = tid + k * NT;
    if (i < RN) {
      const int x = i % rx;
      const int y = (i / rx) % ry;
      const int z = i / sz;
      bool in = (x >= H && x < H + a.tx);
      if (D >= 2) in = in && (y >= H && y < H + a.ty);
      if (D >= 3) in = in && (z >= H && z < H + a.tz);
      const int gx = ox + x, gy = oy + y, gz = oz + z;
      in = in && gx < a.nx && gy < a.ny && gz < a.nz;
      if (in) {
        const long long gi = (long long)gx + (long long)a.nx * (gy + (long long)a.ny * gz);
        if (COMP && a.last) {
          a.u_out[base + gi] = ru[k] - reu[k];
          a.p_out[base + gi] = rp[k] - rep[k];
        } else {
          a.u_out[base + gi] = ru[k];
          a.p_out[base + gi] = rp[k];
          if (COMP) {
            a.eu_out[base + gi] = reu[k];
            a.ep_out[base + gi] = rep[k];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 2D streaming kernel with register-pipelined time steps.
//
// One wavefront owns 64 consecutive columns x (periodic) and streams down a
// segment of rows.  The B time steps of a launch are B pipeline stages held
// in registers: at stream step t stage j turns level-j row t-2j into level
// j+1 row t-2j.  With this lag of two rows per stage every stage reads only
// rows produced in the previous stream step, so the B stages of one step
// are independent of each other.  A row enters at level 0 (read from
// memory) and leaves at level B (written).  Each stage keeps a three-row
// window of its input level plus one pending row; the x neighbours come
// from the adjacent lanes, so the valid lanes shrink by one per stage and
// the halo is H = B + 1 columns on each side (the +1 for the closing half
// kick).  No LDS and no barriers.
// ---------------------------------------------------------------------------
}  // namespace

// descriptor of one problem's streams in a (possibly multi-problem) launch;
// declared in pw_internal.h as StreamDesc<T>
namespace {

template <typename T>
__device__ __forceinline__ T lane_up(T v) {  // value of lane - 1
  return lane_shift<0x138>(v);
}
template <typename T>
__device__ __forceinline__ T lane_down(T v) {  // value of lane + 1
  return lane_shift<0x130>(v);
}

// p <- f p with the compensation term carried along: the exact product
// f s is s' + r (r from one fused multiply-add), so the compensated value
// s - e becomes s' - (f e - r)
template <typename T, bool COMP>
__device__ __forceinline__ void kscale(T& s, T& e, T f) {
  if constexpr (COMP) {
    const T sf = s * f;
    const T r = fma(f, s, -sf);
    e = fma(f, e, -r);
    s = sf;
  } else {
    s *= f;
  }
}

// one stream (wavefront) of problem descriptor `a`; wid = local wave index.
// FORCED: the layer and source of a.f (see Force); REC: also its receiver
// record (a separate instantiation: the recording code holds registers
// that would cost the other forced launches a wave per SIMD)
template <typename T, bool COMP, int B, bool LV = false, bool FORCED = false, bool REC = false>
__device__ __forceinline__ void stream2d_body(const StreamDesc<T>& a, long long wid, int lane) {
  constexpr int H = B + 1;
  constexpr int XV = 64 - 2 * H;  // output columns per wave
  const int cb = (int)(wid % a.ncb);
  const int seg = (int)((wid / a.ncb) % a.nseg);
  const int state = (int)(wid / ((long long)a.ncb * a.nseg));
  const int nx = a.nx, ny = a.ny;
  const int xl = cb * XV - H + lane;  // logical column of this lane
  const int gx = wrap_idx(xl, nx);
  const bool out_lane = lane >= H && lane < 64 - H && (cb * XV + lane - H) < nx;
  const int Y0 = seg * a.Ly;
  const int Y1 = min(Y0 + a.Ly, ny);
  const long long base = (long long)state * a.sstride;
  const T h = a.h;
  const int ns = a.nsteps;
  const bool first = a.first, last = a.last;
  // stage j window: level-j rows (r-1, r, r+1), r = t - 2j; pending: row
  // r+2, produced during step t by stage j-1 (or loaded, for j = 0)
  // weu holds rows (r-1, r, r+1) like wu: with COMP the second difference
  // is taken of u - e, the compensated displacement
  T wu[B + 1][3], wp[B + 1][2], weu[B + 1][3], wep[B + 1][2], wk[B + 1][2];
  T qu[B + 1], qp[B + 1], qeu[B + 1], qep[B + 1], qk[B + 1];
#pragma unroll
  for (int j = 0; j <= B; ++j) {
    wu[j][0] = wu[j][1] = wu[j][2] = T(0);
    wp[j][0] = wp[j][1] = weu[j][0] = weu[j][1] = weu[j][2] = T(0);
    wep[j][0] = wep[j][1] = wk[j][0] = wk[j][1] = T(0);
    qu[j] = qp[j] = qeu[j] = qep[j] = qk[j] = T(0);
  }
  const int tout = last ? 2 * B : 2 * (B - 1);  // lag of the written level
  const int tbeg = Y0 - H - 2;
  const int tend = Y1 - 1 + tout;  // inclusive
  // forced launches: this lane's column factor of the layer, the slice
  // start time of this state
  const bool damp = FORCED && a.f.dmp_x != nullptr;
  const T dcol = damp ? a.f.dmp_x[gx] : T(1);
  // the source's table, for a stream whose stages visit the source row
  // (rows tbeg - 2B .. tend, wrapped); the others skip the source
  const double* srow = nullptr;
  if (FORCED && a.f.sx >= 0) {
    const int lo = tbeg - 2 * B, span = tend - lo;
    const int d = wrap_idx(a.f.sy - lo, ny);
    if (span + 1 >= ny || d <= span) srow = a.f.src_tab + (long long)state * a.f.src_stride;
  }
  // kick on a stage's row: damp p by the row's layer factor drow, then
  // add w (c^2 Lap u + source), the source value sv being that of the
  // row (zero off the source row)
  auto forced_kick = [&](T& pn, T& ep, T kl, T drow, double sv, bool half) {
    const T d = damp ? min(dcol, drow) : T(1);
    if (damp) kscale<T, COMP>(pn, ep, half ? d : d * d);
    const T w = half ? h * T(0.5) : h * T(0.5) * (T(1) + d);
    T acc = kl;
    if (sv != 0.0 && gx == a.f.sx) acc += T(sv);
    kadd<T, COMP>(pn, ep, w * acc);
  };
  for (int t = tbeg; t <= tend; ++t) {
    // forced launches: the row factors of every stage's row for this step,
    // from the wave-uniform row index, loaded together ahead of the stages
    T drow[B + 1];
    double srcv[B + 1];
    if constexpr (FORCED) {
      // rows t, t - 2, ..., t - 2B wrapped into [0, ny), each on its own
      // (a chain of wraps from row to row measured 8 % slower)
      const int tu = __builtin_amdgcn_readfirstlane(t);
#pragma unroll
      for (int j = 0; j <= B; ++j) {
        const int ry = wrap_near(tu - 2 * j, ny);
        drow[j] = damp ? a.f.dmp_y[ry] : T(1);
        // stage j kicks level step0 + j when j < nsteps; stage B closes the
        // slice at level step0 + nsteps
        const bool act = j < B ? j < ns : (bool)last;
        const int lev = a.step0 + (j < B ? j : ns);
        srcv[j] = (srow && act && ry == a.f.sy) ? a.f.amp * srow[lev] : 0.0;
      }
    }
    // level 0, row t+2 -> pending slot of stage 0
    if (t + 2 < Y1 + H) {
      const int gy = wrap_idx(t + 2, ny);
      const long long gi = base + (long long)gy * nx + gx;
      qu[0] = a.u_in[gi];
      qp[0] = a.p_in[gi];
      qk[0] = a.c2[(long long)gy * nx + gx] * a.idx2;
      if (COMP) {
        qeu[0] = first ? T(0) : a.eu_in[gi];
        qep[0] = first ? T(0) : a.ep_in[gi];
      }
    }
    // stages 0..B-1: kick + drift (stages past nsteps pass the row through)
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const T uc = wu[j][1];
      T un = uc, pn = wp[j][0], eu = weu[j][1], ep = wep[j][0];
      const T kj = wk[j][0];
      if (j < ns) {
        T lap =
            (lane_up(uc) - T(2) * uc + lane_down(uc)) + (wu[j][0] - T(2) * uc + wu[j][2]);
        if (COMP)
          lap -= (lane_up(eu) - T(2) * eu + lane_down(eu)) +
                 (weu[j][0] - T(2) * eu + weu[j][2]);
        if constexpr (FORCED) {
          forced_kick(pn, ep, kj * lap, drow[j], srcv[j], j == 0 && first);
        } else {
          const T w = (j == 0 && first) ? h * T(0.5) : h;
          kadd<T, COMP>(pn, ep, w * (kj * lap));
        }
        kadd<T, COMP>(un, eu, h * pn);
        if constexpr (REC) {
          // receiver record: u after step step0 + j + 1 of the slice
          const int orow = t - 2 * j;
          if (a.f.rec_rows && orow >= Y0 && orow < Y1 && a.f.rec_rows[orow]) {
            const int rid = a.f.rec_map[(long long)orow * nx + gx];
            if (out_lane && rid >= 0)
              a.f.traces[((long long)state * a.f.m_tr + a.step0 + j) * a.f.n_rec + rid] =
                  COMP ? (double)un - (double)eu : (double)un;
          }
        }
      }
      qu[j + 1] = un;
      qp[j + 1] = pn;
      qeu[j + 1] = eu;
      qep[j + 1] = ep;
      qk[j + 1] = kj;
      if (LV && j < ns) {
        const int orow = t - 2 * j;
        if (out_lane && orow >= Y0 && orow < Y1)
          a.lv_out[(long long)j * a.lv_stride + base + (long long)orow * nx + gx] = un;
      }
      if (j == B - 1 && !last) {
        const int orow = t - 2 * j;
        if (out_lane && orow >= Y0 && orow < Y1) {
          const long long gi = base + (long long)orow * nx + gx;
          a.u_out[gi] = un;
          a.p_out[gi] = pn;
          if (COMP) {
            a.eu_out[gi] = eu;
            a.ep_out[gi] = ep;
          }
        }
      }
    }
    // stage B: closing half kick of the slice, then fold and write
    if (last) {
      const T uc = wu[B][1];
      const T ec = weu[B][1];
      T lap = (lane_up(uc) - T(2) * uc + lane_down(uc)) + (wu[B][0] - T(2) * uc + wu[B][2]);
      if (COMP)
        lap -= (lane_up(ec) - T(2) * ec + lane_down(ec)) + (weu[B][0] - T(2) * ec + weu[B][2]);
      T pn = wp[B][0], ep = wep[B][0];
      if constexpr (FORCED)
        forced_kick(pn, ep, wk[B][0] * lap, drow[B], srcv[B], true);
      else
        kadd<T, COMP>(pn, ep, h * T(0.5) * (wk[B][0] * lap));
      const int orow = t - 2 * B;
      if (out_lane && orow >= Y0 && orow < Y1) {
        const long long gi = base + (long long)orow * nx + gx;
        if (COMP) {
          a.u_out[gi] = uc - ec;
          a.p_out[gi] = pn - ep;
        } else {
          a.u_out[gi] = uc;
          a.p_out[gi] = pn;
        }
      }
    }
    // advance every window by one row, taking in the pending row
#pragma unroll
    for (int j = 0; j <= B; ++j) {
      wu[j][0] = wu[j][1];
      wu[j][1] = wu[j][2];
      wu[j][2] = qu[j];
      wp[j][0] = wp[j][1];
      wp[j][1] = qp[j];
      weu[j][0] = weu[j][1];
      weu[j][1] = weu[j][2];
      weu[j][2] = qeu[j];
      wep[j][0] = wep[j][1];
      wep[j][1] = qep[j];
      wk[j][0] = wk[j][1];
      wk[j][1] = qk[j];
    }
  }
}

// waves of a launch, remapped so that consecutive blocks of one XCD hold
// consecutive waves (neighbouring streams share halo rows in one L2)
__device__ __forceinline__ long long launch_wave(long long nwaves) {
  const long long nblk = (nwaves + 3) / 4;
  long long blk = blockIdx.x;
  if ((nblk & 7) == 0) blk = (blk & 7) * (nblk >> 3) + (blk >> 3);
  return blk * 4 + (threadIdx.x >> 6);
}

// single problem; TAG separates the fine-grid (0) and coarse-grid (1)
// instantiations in profiles, the code is the same
template <typename T, bool COMP, int B, int TAG>
__global__ __launch_bounds__(256) void k_prop_stream2d(StreamDesc<T> a) {
  const long long nwaves = (long long)a.nstates * a.ncb * a.nseg;
  const long long wid = launch_wave(nwaves);
  if (wid >= nwaves) return;
  stream2d_body<T, COMP, B>(a, wid, threadIdx.x & 63);
}

// the same with the layer and source of a.f (REC: and its receivers)
template <typename T, bool COMP, int B, bool REC>
__global__ __launch_bounds__(256) void k_prop_stream2d_forced(StreamDesc<T> a) {
  const long long nwaves = (long long)a.nstates * a.ncb * a.nseg;
  const long long wid = launch_wave(nwaves);
  if (wid >= nwaves) return;
  stream2d_body<T, COMP, B, false, true, REC>(a, wid, threadIdx.x & 63);
}

// the same with every produced level of u written to a.lv_out (the forward
// recomputation of the adjoint)
template <typename T, int B, bool FORCED>
__global__ __launch_bounds__(256) void k_prop_stream2d_levels(StreamDesc<T> a) {
  const long long nwaves = (long long)a.nstates * a.ncb * a.nseg;
  const long long wid = launch_wave(nwaves);
  if (wid >= nwaves) return;
  stream2d_body<T, false, B, true, FORCED>(a, wid, threadIdx.x & 63);
}

// many problems of different grids in one launch: wave -> problem through
// the prefix sums wave_begin of the descriptor table
template <typename T, bool COMP, int B>
__global__ __launch_bounds__(256) void k_prop_stream2d_multi(const StreamDesc<T>* descs, int nd,
                                                             long long nwaves) {
  const long long wid = launch_wave(nwaves);
  if (wid >= nwaves) return;
  int lo = 0, hi = nd - 1;  // last descriptor with wave_begin <= wid
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].wave_begin <= wid) lo = mid;
    else hi = mid - 1;
  }
  const StreamDesc<T> a = descs[lo];
  stream2d_body<T, COMP, B>(a, wid - a.wave_begin, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// 3D streaming kernel with register-pipelined time steps.
//
// A workgroup of WY waves owns a 64 (x) by WY*R (y) block of columns and
// streams it along z through a segment of planes.  Wave w holds rows
// w*R .. w*R+R-1 of the block, lane l column l, one value per row in
// registers.  As in the 2D kernel the B time steps of a launch are B
// pipeline stages: at stream step t stage j turns level-j plane t-2j into
// level j+1 plane t-2j from its window of three level-j planes (the z
// neighbours), so the stages of one step are independent.  The x neighbours
// come from the adjacent lanes (DPP wavefront shifts), the y neighbours from
// the wave's own rows or, for its first and last row, from the waves above
// and below through LDS: every step each wave publishes the first and last
// row of every stage's centre plane, one barrier, and reads its
// neighbours' (two LDS buffers alternate, so one barrier per step
// suffices).  The valid region shrinks by one lane / row per stage on each
// side, so the halo is H = B + 1 lanes and rows (the +1 for the closing
// half kick) and a block writes 64 - 2H columns of WY*R - 2H rows.  Row and
// column indices are wrapped once per thread, the plane index by one
// conditional add per loaded plane.  Registers go to the u and p windows
// only: each stage reads c^2 of its centre plane from memory, the stages
// run last to first so that a stage's result lands directly in the next
// stage's window, and only the last launch of a slice (LAST) carries the
// window of the closing half kick.
// ---------------------------------------------------------------------------
template <typename T>
struct Stream3Desc {
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
  int nx, ny, nz;
  int ncb, nyb, nseg, Lz;  // column blocks, row blocks, z segments, planes per segment
  int nstates;
  T h, idx2;
  int nsteps, first, last;
};

template <typename T, bool COMP, int B, int R, int WY, bool LAST>
__global__ __launch_bounds__(64 * WY) void k_prop_stream3d(Stream3Desc<T> a) {
  constexpr int H = B + 1;
  // stages that hold a window: stage B (the closing half kick) only in the
  // last launch of a slice; the other launches keep no registers for it
  constexpr int NW = LAST ? B + 1 : B;
  constexpr int XV = 64 - 2 * H;  // output columns of a block
  constexpr int YR = WY * R;      // rows of a block
  constexpr int YV = YR - 2 * H;  // output rows of a block
  constexpr int NX = COMP ? 2 : 1;
  // [buffer][field u / e][stage][first / last row][wave][lane]
  __shared__ T xch[2][NX][NW][2][WY][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  // blocks of one XCD (block ids congruent mod 8) take consecutive streams,
  // so that neighbouring blocks, which share halo columns and rows, share
  // an L2
  const long long nblk = (long long)a.nstates * a.nseg * a.nyb * a.ncb;
  long long blk = blockIdx.x;
  if ((nblk & 7) == 0) blk = (blk & 7) * (nblk >> 3) + (blk >> 3);
  const int cb = (int)(blk % a.ncb);
  const int yb = (int)((blk / a.ncb) % a.nyb);
  const int seg = (int)((blk / ((long long)a.ncb * a.nyb)) % a.nseg);
  const int state = (int)(blk / ((long long)a.ncb * a.nyb * a.nseg));
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int gx = wrap_idx(cb * XV - H + lane, nx);
  const bool out_lane = lane >= H && lane < 64 - H && (cb * XV + lane - H) < nx;
  // byte offset of this thread's row r inside a plane (a plane of one state
  // holds fewer than 2^31 bytes): every access is a wave-uniform plane
  // address plus this 32-bit offset
  unsigned rowb[R];
  bool out_row[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int yr = w * R + r;  // row within the block
    const int gy = wrap_idx(yb * YV - H + yr, ny);
    rowb[r] = (unsigned)(gy * nx + gx) * (unsigned)sizeof(T);
    out_row[r] = out_lane && yr >= H && yr < YR - H && (yb * YV + yr - H) < ny;
  }
  auto ld = [&](const T* pl, int r) -> T {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(pl) + rowb[r]);
  };
  auto st = [&](T* pl, int r, T v) { *reinterpret_cast<T*>(reinterpret_cast<char*>(pl) + rowb[r]) = v; };
  const long long plane = (long long)nx * ny;
  const int Z0 = seg * a.Lz;
  const int Z1 = min(Z0 + a.Lz, nz);
  const long long base = (long long)state * a.sstride;
  const T h = a.h;
  const int ns = a.nsteps;
  const bool first = a.first;
  constexpr bool last = LAST;
  // stage j window: level-j planes (z-1, z, z+1), z = t - 2j; the pending
  // plane z+2 comes from stage j-1 (or memory, for j = 0) in step t
  T wu[B + 1][3][R], weu[B + 1][3][R], wp[B + 1][2][R], wep[B + 1][2][R];
  T qu[R], qp[R], qeu[R], qep[R];
#pragma unroll
  for (int j = 0; j <= B; ++j)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      wu[j][0][r] = wu[j][1][r] = wu[j][2][r] = T(0);
      weu[j][0][r] = weu[j][1][r] = weu[j][2][r] = T(0);
      wp[j][0][r] = wp[j][1][r] = wep[j][0][r] = wep[j][1][r] = T(0);
    }
#pragma unroll
  for (int r = 0; r < R; ++r) qu[r] = qp[r] = qeu[r] = qep[r] = T(0);
  const int tout = last ? 2 * B : 2 * (B - 1);  // lag of the written level
  const int tbeg = Z0 - H - 2;
  const int tend = Z1 - 1 + tout;  // inclusive
  int zl = tbeg + 2;               // plane loaded this step, wrapped below
  zl = zl < 0 ? zl + nz : zl;
  // centre plane of stage j (t - 2j, wrapped): c^2 is read there by each
  // stage from memory (an L2 hit: stage 0 read the plane's u and p two
  // steps per stage earlier) instead of riding the register pipeline
  int zs[B + 1];
#pragma unroll
  for (int j = 0; j <= B; ++j) zs[j] = ((tbeg - 2 * j) % nz + nz) % nz;
  for (int t = tbeg; t <= tend; ++t) {
    // level 0, plane t+2 -> pending slot of stage 0
    if (t + 2 < Z1 + H) {
      const long long po = base + (long long)zl * plane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        qu[r] = ld(a.u_in + po, r);
        qp[r] = ld(a.p_in + po, r);
        if (COMP) {
          qeu[r] = first ? T(0) : ld(a.eu_in + po, r);
          qep[r] = first ? T(0) : ld(a.ep_in + po, r);
        }
      }
    }
    zl = zl + 1 == nz ? 0 : zl + 1;
    // publish the first and last row of every stage's centre plane
    const int buf = t & 1;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      xch[buf][0][j][0][w][lane] = wu[j][1][0];
      xch[buf][0][j][1][w][lane] = wu[j][1][R - 1];
      if (COMP) {
        xch[buf][NX - 1][j][0][w][lane] = weu[j][1][0];
        xch[buf][NX - 1][j][1][w][lane] = weu[j][1][R - 1];
      }
    }
    __syncthreads();
    // y neighbours of the first and last row (zero outside the block: those
    // rows are in the halo)
    T au[B + 1], bu[B + 1], ae[B + 1], be[B + 1];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      au[j] = w > 0 ? xch[buf][0][j][1][w - 1][lane] : T(0);
      bu[j] = w < WY - 1 ? xch[buf][0][j][0][w + 1][lane] : T(0);
      ae[j] = (COMP && w > 0) ? xch[buf][NX - 1][j][1][w - 1][lane] : T(0);
      be[j] = (COMP && w < WY - 1) ? xch[buf][NX - 1][j][0][w + 1][lane] : T(0);
    }
    // second difference of x on the centre plane of stage j, row r
    auto lap_of = [&](const T (&win)[3][R], T above, T below, int r) -> T {
      const T c = win[1][r];
      const T ym = r > 0 ? win[1][r - 1] : above;
      const T yp = r < R - 1 ? win[1][r + 1] : below;
      return (lane_up(c) - T(2) * c + lane_down(c)) + (ym - T(2) * c + yp) +
             (win[0][r] - T(2) * c + win[2][r]);
    };
    // stages last to first: once stage j + 1 has used its window and moved
    // it on by one plane, stage j writes its result straight into that
    // window's top slot, so no pending plane stays live across the step
#pragma unroll
    for (int j = B; j >= 0; --j) {
      if (j == B) {
        // closing half kick of the slice, then fold and write
        if constexpr (LAST) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const T uc = wu[B][1][r];
            const T ec = weu[B][1][r];
            T lap = lap_of(wu[B], au[B], bu[B], r);
            if (COMP) lap -= lap_of(weu[B], ae[B], be[B], r);
            T pn = wp[B][0][r], ep = wep[B][0][r];
            const T kb = ld(a.c2 + (long long)zs[B] * plane, r) * a.idx2;
            kadd<T, COMP>(pn, ep, h * T(0.5) * (kb * lap));
            const int oz = t - 2 * B;
            if (out_row[r] && oz >= Z0 && oz < Z1) {
              const long long go = base + (long long)oz * plane;
              if (COMP) {
                st(a.u_out + go, r, uc - ec);
                st(a.p_out + go, r, pn - ep);
              } else {
                st(a.u_out + go, r, uc);
                st(a.p_out + go, r, pn);
              }
            }
          }
        }
      } else {
        // kick + drift (stages past nsteps pass the plane through)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T uc = wu[j][1][r];
          T un = uc, pn = wp[j][0][r], eu = weu[j][1][r], ep = wep[j][0][r];
          if (j < ns) {
            const T kj = ld(a.c2 + (long long)zs[j] * plane, r) * a.idx2;
            T lap = lap_of(wu[j], au[j], bu[j], r);
            if (COMP) lap -= lap_of(weu[j], ae[j], be[j], r);
            const T wgt = (j == 0 && first) ? h * T(0.5) : h;
            kadd<T, COMP>(pn, ep, wgt * (kj * lap));
            kadd<T, COMP>(un, eu, h * pn);
          }
          if (j == B - 1 && !last) {
            const int oz = t - 2 * j;
            if (out_row[r] && oz >= Z0 && oz < Z1) {
              const long long go = base + (long long)oz * plane;
              st(a.u_out + go, r, un);
              st(a.p_out + go, r, pn);
              if (COMP) {
                st(a.eu_out + go, r, eu);
                st(a.ep_out + go, r, ep);
              }
            }
          }
          if (j + 1 < NW) {
            wu[j + 1][2][r] = un;
            wp[j + 1][1][r] = pn;
            weu[j + 1][2][r] = eu;
            wep[j + 1][1][r] = ep;
          }
        }
      }
      // stage j's window moves on by one plane; its top slot is written by
      // stage j - 1 next (for stage 0, from the plane loaded above)
#pragma unroll
      for (int r = 0; r < R && j < NW; ++r) {
        wu[j][0][r] = wu[j][1][r];
        wu[j][1][r] = wu[j][2][r];
        wp[j][0][r] = wp[j][1][r];
        weu[j][0][r] = weu[j][1][r];
        weu[j][1][r] = weu[j][2][r];
        wep[j][0][r] = wep[j][1][r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      wu[0][2][r] = qu[r];
      wp[0][1][r] = qp[r];
      weu[0][2][r] = qeu[r];
      wep[0][1][r] = qep[r];
    }
#pragma unroll
    for (int j = 0; j <= B; ++j) zs[j] = zs[j] + 1 == nz ? 0 : zs[j] + 1;
  }
}

// tile geometry per dimension: interior and the largest halo of one launch
struct TileCfg {
  int tx, ty, tz, hmax;
};
constexpr TileCfg kTile1 = {1024, 1, 1, 9};
constexpr TileCfg kTile2 = {64, 32, 1, 9};
constexpr TileCfg kTile3 = {32, 8, 8, 2};
constexpr int kNT = 256;

constexpr int region_max(TileCfg c, int D) {
  return (c.tx + 2 * c.hmax) * (D >= 2 ? c.ty + 2 * c.hmax : 1) *
         (D >= 3 ? c.tz + 2 * c.hmax : 1);
}
constexpr int ppt_for(TileCfg c, int D) { return (region_max(c, D) + kNT - 1) / kNT; }

template <typename T, bool COMP, int PPT>
void launch_line(const PropArgs<T>& a, int nt, hipStream_t st) {
  const size_t smem = sizeof(T) * (size_t)a.nx * (COMP ? 2 : 1);
  switch (nt) {
    case 64:
      hipLaunchKernelGGL((k_prop_line<T, COMP, 64, PPT>), dim3(a.nstates), dim3(64), smem, st, a);
      break;
    case 128:
      hipLaunchKernelGGL((k_prop_line<T, COMP, 128, PPT>), dim3(a.nstates), dim3(128), smem, st,
                         a);
      break;
    default:
      hipLaunchKernelGGL((k_prop_line<T, COMP, 256, PPT>), dim3(a.nstates), dim3(256), smem, st,
                         a);
      break;
  }
  PW_LAUNCH_CHECK();
}

template <typename T, bool COMP>
void dispatch_line(const PropArgs<T>& a, hipStream_t st) {
  const int n = a.nx;
  const int nt = n <= 64 ? 64 : (n <= 128 ? 128 : 256);
  const int ppt = (n + nt - 1) / nt;
  if (ppt <= 1)
    launch_line<T, COMP, 1>(a, nt, st);
  else if (ppt <= 2)
    launch_line<T, COMP, 2>(a, nt, st);
  else if (ppt <= 4)
    launch_line<T, COMP, 4>(a, nt, st);
  else if (ppt <= 8)
    launch_line<T, COMP, 8>(a, nt, st);
  else if (ppt <= 16)
    launch_line<T, COMP, 16>(a, nt, st);
  else
    fail(PW_EINVAL, "1D line longer than 4096 points");
}

template <typename T, int D, bool COMP>
void dispatch_tile(PropArgs<T> a, hipStream_t st) {
  constexpr TileCfg c = D == 1 ? kTile1 : (D == 2 ? kTile2 : kTile3);
  constexpr int PPT = ppt_for(c, D);
  const long long blocks = (long long)a.ntx * a.nty * a.ntz * a.nstates;
  const size_t smem = sizeof(T) * (size_t)a.rx * a.ry * a.rz * (COMP ? 2 : 1);
  hipLaunchKernelGGL((k_prop_tile<T, D, COMP, kNT, PPT>), dim3((unsigned)blocks), dim3(kNT), smem,
                     st, a);
  PW_LAUNCH_CHECK();
}

template <typename T>
constexpr int stream_depth() {
  return sizeof(T) == 4 ? 8 : 4;
}

template <typename T, bool COMP, int B = stream_depth<T>()>
void dispatch_stream2d(const StreamDesc<T>& a, bool fine, bool forced, hipStream_t st) {
  const long long nwaves = (long long)a.nstates * a.ncb * a.nseg;
  const long long nblk = (nwaves + 3) / 4;
  if (nblk >= (1LL << 31)) fail(PW_EINVAL, "too many streams for one launch");
  if (forced && a.f.traces)
    hipLaunchKernelGGL((k_prop_stream2d_forced<T, COMP, B, true>), dim3((unsigned)nblk),
                       dim3(256), 0, st, a);
  else if (forced)
    hipLaunchKernelGGL((k_prop_stream2d_forced<T, COMP, B, false>), dim3((unsigned)nblk),
                       dim3(256), 0, st, a);
  else if (fine)
    hipLaunchKernelGGL((k_prop_stream2d<T, COMP, B, 0>), dim3((unsigned)nblk), dim3(256), 0, st,
                       a);
  else
    hipLaunchKernelGGL((k_prop_stream2d<T, COMP, B, 1>), dim3((unsigned)nblk), dim3(256), 0, st,
                       a);
  PW_LAUNCH_CHECK();
}

// streams of a 2D launch: column blocks of XV output columns, row segments
// sized so that about 4096 streams fill the chip
template <typename T, int B = stream_depth<T>()>
void stream_geometry(StreamDesc<T>& a, int nstates, long long want_default = 0) {
  constexpr int XV = 64 - 2 * (B + 1);
  a.ncb = (a.nx + XV - 1) / XV;
  // enough independent streams to fill the chip once at the kernel's
  // occupancy (256 CUs x 4 SIMDs x 3 waves for the 8-step FP32 kernel, 4
  // waves otherwise): a whole number of workgroups per CU, no tail;
  // segments of >= 32 rows, or of >= B rows when even that leaves fewer
  // than 256 streams (one small state: each stream is a serial chain of row
  // steps, so shorter segments finish sooner although they repeat more halo
  // rows)
  static const long long want_env = [] {
    const char* e = getenv("PW_STREAM_TARGET");  // tuning override
    return e ? atoll(e) : 0LL;
  }();
  const long long want =
      want_env > 0 ? want_env
                   : (want_default > 0 ? want_default : (sizeof(T) == 4 && B == 8 ? 3072 : 4096));
  const long long lanes = (long long)nstates * a.ncb;
  long long nseg = (want + lanes - 1) / lanes;
  const long long minrows = lanes * ((a.ny + 31) / 32) < 256 ? B : 32;
  nseg = std::max(1LL, std::min(nseg, (long long)((a.ny + minrows - 1) / minrows)));
  a.Ly = (int)((a.ny + nseg - 1) / nseg);
  a.nseg = (a.ny + a.Ly - 1) / a.Ly;
}

template <typename T, int B>
void propagate_stream2d_b(const Grid& g, const T* c2, const T* u_src, const T* p_src, T* u_dst,
                          T* p_dst, long long sstride, int nstates, int m, T h, bool comp,
                          StateSet<T> wa, StateSet<T> wb, bool fine, hipStream_t st,
                          const Force<T>* fo) {
  StreamDesc<T> a{};
  if (fo) a.f = *fo;
  a.c2 = c2;
  a.sstride = sstride;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nstates = nstates;
  a.h = h;
  a.idx2 = T(1.0 / (g.dx * g.dx));
  stream_geometry<T, B>(a, nstates);
  const int nl = (m + B - 1) / B;
  if (nl > 1 && (wa.u == nullptr || wb.u == nullptr || (comp && (wa.eu == nullptr || wb.eu == nullptr))))
    fail(PW_EINVAL, "propagation needs scratch state sets");
  const T* cu = u_src;
  const T* cp = p_src;
  const T* ceu = nullptr;
  const T* cep = nullptr;
  for (int l = 0; l < nl; ++l) {
    a.first = (l == 0);
    a.last = (l == nl - 1);
    a.nsteps = std::min(B, m - l * B);
    a.u_in = cu;
    a.p_in = cp;
    a.eu_in = ceu;
    a.ep_in = cep;
    StateSet<T> out;
    if (a.last) {
      out.u = u_dst;
      out.p = p_dst;
    } else {
      out = ((nl - 1 - l) % 2 == 1) ? wa : wb;
    }
    a.u_out = out.u;
    a.p_out = out.p;
    a.eu_out = out.eu;
    a.ep_out = out.ep;
    a.step0 = l * B;
    if (comp) {
      if constexpr (sizeof(T) == 4) dispatch_stream2d<T, true, B>(a, fine, fo != nullptr, st);
      else fail(PW_EINVAL, "compensation is an FP32 mode");
    } else {
      dispatch_stream2d<T, false, B>(a, fine, fo != nullptr, st);
    }
    cu = out.u;
    cp = out.p;
    ceu = out.eu;
    cep = out.ep;
  }
}

// FP32 states of a launch too small to fill the chip (a few small states,
// as in the serial chain of coarse propagations) take 4 time steps per
// launch instead of 8: each stream is then a chain of about half as many
// row steps (half the stages, half the halo rows, shorter segments)
template <typename T>
void propagate_stream2d(const Grid& g, const T* c2, const T* u_src, const T* p_src, T* u_dst,
                        T* p_dst, long long sstride, int nstates, int m, T h, bool comp,
                        StateSet<T> wa, StateSet<T> wb, bool fine, hipStream_t st,
                        const Force<T>* fo) {
  if constexpr (sizeof(T) == 4) {
    constexpr int XV = 64 - 2 * (stream_depth<T>() + 1);
    const long long lanes = (long long)nstates * ((g.n[0] + XV - 1) / XV);
    if (lanes * ((g.n[1] + 31) / 32) < 256) {
      propagate_stream2d_b<T, 4>(g, c2, u_src, p_src, u_dst, p_dst, sstride, nstates, m, h, comp,
                                 wa, wb, fine, st, fo);
      return;
    }
  }
  propagate_stream2d_b<T, stream_depth<T>()>(g, c2, u_src, p_src, u_dst, p_dst, sstride, nstates,
                                             m, h, comp, wa, wb, fine, st, fo);
}

// launch shape of the 3D streaming kernel per state type: time steps per
// launch, rows per wave, waves per workgroup.  FP32 (compensated): 4 steps
// of 64 x 32 blocks, one workgroup of 16 waves per CU (119 VGPRs); the
// last launch of a slice, which also holds the closing half kick, runs 12
// waves on 64 x 24 blocks (148 VGPRs; at 16 waves it spills).  Measured on the layers3d sweep (256^3, 32 states, 76
// steps), all shapes bit-identical: the last launch at 12 waves 173 ms,
// at 8 waves 183 and at 16 (spilling) 184; with the last launch also at
// 16 waves, (B, R, WY) = (4, 2, 16) 183 ms against
// (3, 2, 16) 185, (4, 2, 12) 198, (3, 2, 12) 209, (3, 3, 12) 235, (2, 3,
// 16) 261 and (3, 3, 8) 252; the kernel that carried c^2 in registers and
// every stage window in every launch ran (3, 3, 8) in 206 ms.  FP64
// (uncompensated): 3 steps of 64 x 32 blocks of 16 waves (98 VGPRs), the
// last launch 8 waves (126 VGPRs); the FP64 layers3d sweep (256^3, 32
// states) takes 178 ms against (B, R, WY, last) = (3, 2, 16, 12) 185,
// (4, 2, 16, 12) 182, (2, 1, 16, 16) 211, (2, 2, 16, 12) 225, (2, 2, 8, 8)
// 234, (4, 1, 16, 16) 275 and the earlier (2, 1, 8, 8) 368, all
// bit-identical.  Build-time overrides PW_S3_B / PW_S3_R / PW_S3_WY /
// PW_S3_WYL (FP32) and PW_S3D_B / PW_S3D_R / PW_S3D_WY / PW_S3D_WYL (FP64)
// for such sweeps.
#ifndef PW_S3_B
#define PW_S3_B 4
#endif
#ifndef PW_S3_R
#define PW_S3_R 2
#endif
#ifndef PW_S3_WY
#define PW_S3_WY 16
#endif
#ifndef PW_S3_WYL
#define PW_S3_WYL 12
#endif
#ifndef PW_S3D_B
#define PW_S3D_B 3
#endif
#ifndef PW_S3D_R
#define PW_S3D_R 2
#endif
#ifndef PW_S3D_WY
#define PW_S3D_WY 16
#endif
#ifndef PW_S3D_WYL
#define PW_S3D_WYL 8
#endif
template <typename T>
struct Stream3Cfg {
  static constexpr int B = sizeof(T) == 4 ? PW_S3_B : PW_S3D_B;
  static constexpr int R = sizeof(T) == 4 ? PW_S3_R : PW_S3D_R;
  static constexpr int WY = sizeof(T) == 4 ? PW_S3_WY : PW_S3D_WY;
  // waves of the last launch of a slice, whose closing half kick holds one
  // more stage window (at 16 waves it would spill)
  static constexpr int WYL = sizeof(T) == 4 ? PW_S3_WYL : PW_S3D_WYL;
  static_assert(WY * R > 2 * (B + 1) && WYL * R > 2 * (B + 1), "3D blocks need output rows");
};

template <typename T, bool COMP>
void dispatch_stream3d(const Stream3Desc<T>& a, hipStream_t st) {
  using C = Stream3Cfg<T>;
  const long long nblk = (long long)a.nstates * a.nseg * a.nyb * a.ncb;
  if (nblk >= (1LL << 31)) fail(PW_EINVAL, "too many streams for one launch");
  if (a.last)
    hipLaunchKernelGGL((k_prop_stream3d<T, COMP, C::B, C::R, C::WYL, true>), dim3((unsigned)nblk),
                       dim3(64 * C::WYL), 0, st, a);
  else
    hipLaunchKernelGGL((k_prop_stream3d<T, COMP, C::B, C::R, C::WY, false>), dim3((unsigned)nblk),
                       dim3(64 * C::WY), 0, st, a);
  PW_LAUNCH_CHECK();
}

// 3D streams: blocks of (64 - 2H) columns by (WY R - 2H) rows, z segments
// sized so that about kStream3Target workgroups fill the chip (segments of
// at least 16 planes, or of 2 B planes when even that leaves few blocks)
constexpr long long kStream3Target = 1024;

template <typename T>
void propagate_stream3d(const Grid& g, const T* c2, const T* u_src, const T* p_src, T* u_dst,
                        T* p_dst, long long sstride, int nstates, int m, T h, bool comp,
                        StateSet<T> wa, StateSet<T> wb, hipStream_t st) {
  using C = Stream3Cfg<T>;
  constexpr int B = C::B, H = B + 1;
  constexpr int XV = 64 - 2 * H;
  Stream3Desc<T> a{};
  a.c2 = c2;
  a.sstride = sstride;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  if (a.nx < H || a.ny < H || a.nz < H) fail(PW_EINVAL, "3D grid smaller than the stencil halo");
  if ((long long)a.nx * a.ny * (long long)sizeof(T) >= (1LL << 31))
    fail(PW_EINVAL, "3D plane of 2^31 bytes or more");
  a.nstates = nstates;
  a.h = h;
  a.idx2 = T(1.0 / (g.dx * g.dx));
  // block geometry for a workgroup of wy waves
  auto geometry = [&](int wy) {
    const int YV = wy * C::R - 2 * H;
    a.ncb = (a.nx + XV - 1) / XV;
    a.nyb = (a.ny + YV - 1) / YV;
    const long long blocks = (long long)nstates * a.ncb * a.nyb;
    const int minz = blocks < 256 ? 2 * B : 16;
    long long nseg = (kStream3Target + blocks - 1) / blocks;
    nseg = std::max(1LL, std::min(nseg, (long long)((a.nz + minz - 1) / minz)));
    a.Lz = (int)((a.nz + nseg - 1) / nseg);
    a.nseg = (a.nz + a.Lz - 1) / a.Lz;
  };
  const int nl = (m + B - 1) / B;
  if (nl > 1 && (wa.u == nullptr || wb.u == nullptr || (comp && (wa.eu == nullptr || wb.eu == nullptr))))
    fail(PW_EINVAL, "propagation needs scratch state sets");
  const T* cu = u_src;
  const T* cp = p_src;
  const T* ceu = nullptr;
  const T* cep = nullptr;
  for (int l = 0; l < nl; ++l) {
    a.first = (l == 0);
    a.last = (l == nl - 1);
    a.nsteps = std::min(B, m - l * B);
    geometry(a.last ? C::WYL : C::WY);
    a.u_in = cu;
    a.p_in = cp;
    a.eu_in = ceu;
    a.ep_in = cep;
    StateSet<T> out;
    if (a.last) {
      out.u = u_dst;
      out.p = p_dst;
    } else {
      out = ((nl - 1 - l) % 2 == 1) ? wa : wb;
    }
    a.u_out = out.u;
    a.p_out = out.p;
    a.eu_out = out.eu;
    a.ep_out = out.ep;
    if (comp) {
      if constexpr (sizeof(T) == 4) dispatch_stream3d<T, true>(a, st);
      else fail(PW_EINVAL, "compensation is an FP32 mode");
    } else {
      dispatch_stream3d<T, false>(a, st);
    }
    cu = out.u;
    cp = out.p;
    ceu = out.eu;
    cep = out.ep;
  }
}

TileCfg tile_cfg(int dim) { return dim == 1 ? kTile1 : (dim == 2 ? kTile2 : kTile3); }

bool use_line(const Grid& g) { return g.dim == 1 && g.n[0] <= 4096; }

}  // namespace

const double* leapfrog_levels2d(const Grid& g, const double* c2, const double* u_src,
                                const double* p_src, double* pa, double* pb, long long sstride,
                                int nstates, int m, double h, bool level0, double* lv,
                                long long lv_stride, hipStream_t st, const Force<double>* fo,
                                int i0) {
  if (g.dim != 2) fail(PW_EINVAL, "leapfrog_levels2d: 2D grids only");
  if (nstates <= 0 || m <= 0) return p_src;
  if (pa == p_src || pb == p_src || pa == pb) fail(PW_EINVAL, "leapfrog_levels2d: p buffers alias");
  constexpr int B = stream_depth<double>();
  StreamDesc<double> a{};
  a.c2 = c2;
  a.sstride = sstride;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nstates = nstates;
  a.h = h;
  a.idx2 = 1.0 / (g.dx * g.dx);
  stream_geometry(a, nstates, 3072);  // measured best for the level-writing kernel
  a.lv_stride = lv_stride;
  a.last = 0;  // leapfrog form: no closing half kick
  if (fo) {
    a.f = *fo;
    a.f.rec_rows = nullptr;  // the recomputation records nothing
    a.f.traces = nullptr;
  }
  const int nl = (m + B - 1) / B;
  const double* cp = p_src;
  for (int l = 0; l < nl; ++l) {
    a.first = (level0 && l == 0) ? 1 : 0;
    a.nsteps = std::min(B, m - l * B);
    a.u_in = l == 0 ? u_src : lv + (long long)(l * B - 1) * lv_stride;
    a.p_in = cp;
    double* po = (l % 2 == 0) ? pa : pb;
    a.u_out = lv + (long long)(l * B + a.nsteps - 1) * lv_stride;
    a.p_out = po;
    a.lv_out = lv + (long long)(l * B) * lv_stride;
    a.step0 = i0 + l * B;
    const long long nwaves = (long long)a.nstates * a.ncb * a.nseg;
    if ((nwaves + 3) / 4 >= (1LL << 31)) fail(PW_EINVAL, "too many streams for one launch");
    if (fo)
      hipLaunchKernelGGL((k_prop_stream2d_levels<double, B, true>),
                         dim3((unsigned)((nwaves + 3) / 4)), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_prop_stream2d_levels<double, B, false>),
                         dim3((unsigned)((nwaves + 3) / 4)), dim3(256), 0, st, a);
    PW_LAUNCH_CHECK();
    cp = po;
  }
  return cp;
}

void launch_plan(const Grid& g, bool is_double, int nstates, int m, int* launches, int* spl) {
  int b;
  if (use_line(g)) {
    b = std::max(m, 1);
  } else if (g.dim == 2) {
    b = is_double ? stream_depth<double>() : stream_depth<float>();
    if (!is_double) {
      constexpr int XV = 64 - 2 * (stream_depth<float>() + 1);
      const long long lanes = (long long)nstates * ((g.n[0] + XV - 1) / XV);
      if (lanes * ((g.n[1] + 31) / 32) < 256) b = 4;
    }
  } else if (g.dim == 3) {
    b = is_double ? Stream3Cfg<double>::B : Stream3Cfg<float>::B;
  } else {
    b = tile_cfg(g.dim).hmax - 1;
  }
  *spl = b;
  *launches = m <= 0 ? 0 : (m + b - 1) / b;
}

int steps_per_launch(const Grid& g, bool is_double) {
  if (use_line(g)) return 1 << 30;
  if (g.dim == 2) return is_double ? stream_depth<double>() : stream_depth<float>();
  if (g.dim == 3) return is_double ? Stream3Cfg<double>::B : Stream3Cfg<float>::B;
  return tile_cfg(g.dim).hmax - 1;
}

template <typename T>
void propagate(const Grid& g, const T* c2, const T* u_src, const T* p_src, T* u_dst, T* p_dst,
               long long sstride, int nstates, int m, T h, bool compensated, StateSet<T> wa,
               StateSet<T> wb, hipStream_t st, bool fine, const Force<T>* fo) {
  if (nstates <= 0) return;
  if (fo && g.dim != 2) fail(PW_EINVAL, "the absorbing layer and source are 2D only");
  if (fo && fo->traces && m <= 0) fail(PW_EINVAL, "a receiver record needs time steps");
  if (m <= 0) {
    for (int s = 0; s < nstates; ++s) {
      PW_HIP(hipMemcpyAsync(u_dst + (long long)s * sstride, u_src + (long long)s * sstride,
                            sizeof(T) * g.npts(), hipMemcpyDeviceToDevice, st));
      PW_HIP(hipMemcpyAsync(p_dst + (long long)s * sstride, p_src + (long long)s * sstride,
                            sizeof(T) * g.npts(), hipMemcpyDeviceToDevice, st));
    }
    return;
  }
  PropArgs<T> a{};
  a.c2 = c2;
  a.sstride = sstride;
  a.nx = g.n[0];
  a.ny = g.n[1];
  a.nz = g.n[2];
  a.nstates = nstates;
  a.h = h;
  a.idx2 = T(1.0 / (g.dx * g.dx));
  const bool comp = compensated;
  if (use_line(g)) {
    a.u_in = u_src;
    a.p_in = p_src;
    a.u_out = u_dst;
    a.p_out = p_dst;
    a.nsteps = m;
    a.first = 1;
    a.last = 1;
    if (comp) {
      if constexpr (sizeof(T) == 4) dispatch_line<T, true>(a, st);
      else fail(PW_EINVAL, "compensation is an FP32 mode");
    } else {
      dispatch_line<T, false>(a, st);
    }
    return;
  }
  if (g.dim == 2) {
    propagate_stream2d<T>(g, c2, u_src, p_src, u_dst, p_dst, sstride, nstates, m, h, comp, wa, wb,
                          fine, st, fo);
    return;
  }
  if (g.dim == 3) {
    propagate_stream3d<T>(g, c2, u_src, p_src, u_dst, p_dst, sstride, nstates, m, h, comp, wa, wb,
                          st);
    return;
  }
  const TileCfg c = tile_cfg(g.dim);
  const int b = c.hmax - 1;
  const int nl = (m + b - 1) / b;
  a.tx = std::min(c.tx, a.nx);
  a.ty = g.dim >= 2 ? std::min(c.ty, a.ny) : 1;
  a.tz = g.dim >= 3 ? std::min(c.tz, a.nz) : 1;
  a.ntx = (a.nx + a.tx - 1) / a.tx;
  a.nty = (a.ny + a.ty - 1) / a.ty;
  a.ntz = (a.nz + a.tz - 1) / a.tz;
  if ((long long)a.ntx * a.nty * a.ntz * nstates >= (1LL << 31))
    fail(PW_EINVAL, "too many tiles for one launch");
  if (nl > 1 && (wa.u == nullptr || wb.u == nullptr || (comp && (wa.eu == nullptr || wb.eu == nullptr))))
    fail(PW_EINVAL, "propagation needs scratch state sets");
  const T* cu = u_src;
  const T* cp = p_src;
  const T* ceu = nullptr;
  const T* cep = nullptr;
  for (int l = 0; l < nl; ++l) {
    const int steps = std::min(b, m - l * b);
    a.first = (l == 0);
    a.last = (l == nl - 1);
    a.nsteps = steps;
    a.H = steps + a.last;
    a.rx = a.tx + 2 * a.H;
    a.ry = g.dim >= 2 ? a.ty + 2 * a.H : 1;
    a.rz = g.dim >= 3 ? a.tz + 2 * a.H : 1;
    a.u_in = cu;
    a.p_in = cp;
    a.eu_in = ceu;
    a.ep_in = cep;
    StateSet<T> out;
    if (a.last) {
      out.u = u_dst;
      out.p = p_dst;
    } else {
      out = ((nl - 1 - l) % 2 == 1) ? wa : wb;
    }
    a.u_out = out.u;
    a.p_out = out.p;
    a.eu_out = out.eu;
    a.ep_out = out.ep;
    if (comp) {
      if constexpr (sizeof(T) == 4) {
        if (g.dim == 1) dispatch_tile<T, 1, true>(a, st);
        else if (g.dim == 2) dispatch_tile<T, 2, true>(a, st);
        else dispatch_tile<T, 3, true>(a, st);
      } else {
        fail(PW_EINVAL, "compensation is an FP32 mode");
      }
    } else {
      if (g.dim == 1) dispatch_tile<T, 1, false>(a, st);
      else if (g.dim == 2) dispatch_tile<T, 2, false>(a, st);
      else dispatch_tile<T, 3, false>(a, st);
    }
    cu = out.u;
    cp = out.p;
    ceu = out.eu;
    cep = out.ep;
  }
}

template <typename T>
void plan_multi(const std::vector<PropJob<T>>& jobs, MultiPlan<T>& plan) {
  const int B = plan.B;
  if (B != 4 && B != 8) fail(PW_EINVAL, "pipeline depth must be 4 or 8");
  if (sizeof(T) == 8 && B != 4) fail(PW_EINVAL, "FP64 streams use depth 4");
  const int XV = 64 - 2 * (B + 1);
  plan.first_desc.clear();
  plan.ndesc.clear();
  plan.nwaves.clear();
  plan.descs.clear();
  int nl = 0;
  for (const auto& j : jobs) {
    if (j.g.dim != 2) fail(PW_EINVAL, "batched streams need 2D problems");
    if (j.m < 1 || j.nstates < 1) fail(PW_EINVAL, "empty job in a batch");
    nl = std::max(nl, (j.m + B - 1) / B);
  }
  for (int l = 0; l < nl; ++l) {
    plan.first_desc.push_back((int)plan.descs.size());
    long long waves = 0;
    for (const auto& j : jobs) {
      const int njl = (j.m + B - 1) / B;
      if (l >= njl) continue;
      if (njl > 1 && (j.wa.u == nullptr || j.wb.u == nullptr))
        fail(PW_EINVAL, "propagation needs scratch state sets");
      StreamDesc<T> d{};
      d.c2 = j.c2;
      d.sstride = j.sstride;
      d.nx = j.g.n[0];
      d.ny = j.g.n[1];
      d.nstates = j.nstates;
      d.h = j.h;
      d.idx2 = T(1.0 / (j.g.dx * j.g.dx));
      d.ncb = (d.nx + XV - 1) / XV;
      const int ly = j.Ly > 0 ? j.Ly : plan.Ly;
      d.nseg = std::max(1, (d.ny + ly - 1) / ly);
      d.Ly = (d.ny + d.nseg - 1) / d.nseg;
      d.nseg = (d.ny + d.Ly - 1) / d.Ly;
      d.first = (l == 0);
      d.last = (l == njl - 1);
      d.nsteps = std::min(B, j.m - l * B);
      // ping-pong: launch l of this job reads what launch l-1 wrote
      auto set_of = [&](int ll) -> StateSet<T> {
        StateSet<T> o;
        if (ll == njl - 1) {
          o.u = j.u_dst;
          o.p = j.p_dst;
        } else {
          o = ((njl - 1 - ll) % 2 == 1) ? j.wa : j.wb;
        }
        return o;
      };
      if (l == 0) {
        d.u_in = j.u_src;
        d.p_in = j.p_src;
        d.eu_in = nullptr;
        d.ep_in = nullptr;
      } else {
        const StateSet<T> in = set_of(l - 1);
        d.u_in = in.u;
        d.p_in = in.p;
        d.eu_in = in.eu;
        d.ep_in = in.ep;
      }
      const StateSet<T> out = set_of(l);
      d.u_out = out.u;
      d.p_out = out.p;
      d.eu_out = out.eu;
      d.ep_out = out.ep;
      d.wave_begin = waves;
      waves += (long long)d.nstates * d.ncb * d.nseg;
      plan.descs.push_back(d);
    }
    plan.ndesc.push_back((int)plan.descs.size() - plan.first_desc.back());
    plan.nwaves.push_back(waves);
  }
}

template <typename T>
void run_multi(const MultiPlan<T>& plan, const StreamDesc<T>* dev, bool comp, hipStream_t st) {
  for (size_t l = 0; l < plan.nwaves.size(); ++l) {
    const long long nw = plan.nwaves[l];
    const long long nblk = (nw + 3) / 4;
    if (nblk >= (1LL << 31)) fail(PW_EINVAL, "too many streams for one launch");
    const StreamDesc<T>* d = dev + plan.first_desc[l];
    const int nd = plan.ndesc[l];
    if constexpr (sizeof(T) == 4) {
      if (comp) {
        if (plan.B == 8)
          hipLaunchKernelGGL((k_prop_stream2d_multi<T, true, 8>), dim3((unsigned)nblk), dim3(256),
                             0, st, d, nd, nw);
        else
          hipLaunchKernelGGL((k_prop_stream2d_multi<T, true, 4>), dim3((unsigned)nblk), dim3(256),
                             0, st, d, nd, nw);
      } else {
        if (plan.B == 8)
          hipLaunchKernelGGL((k_prop_stream2d_multi<T, false, 8>), dim3((unsigned)nblk),
                             dim3(256), 0, st, d, nd, nw);
        else
          hipLaunchKernelGGL((k_prop_stream2d_multi<T, false, 4>), dim3((unsigned)nblk),
                             dim3(256), 0, st, d, nd, nw);
      }
    } else {
      if (comp) fail(PW_EINVAL, "compensation is an FP32 mode");
      hipLaunchKernelGGL((k_prop_stream2d_multi<T, false, 4>), dim3((unsigned)nblk), dim3(256), 0,
                         st, d, nd, nw);
    }
    PW_LAUNCH_CHECK();
  }
}

template void plan_multi<float>(const std::vector<PropJob<float>>&, MultiPlan<float>&);
template void plan_multi<double>(const std::vector<PropJob<double>>&, MultiPlan<double>&);
template void run_multi<float>(const MultiPlan<float>&, const StreamDesc<float>*, bool,
                               hipStream_t);
template void run_multi<double>(const MultiPlan<double>&, const StreamDesc<double>*, bool,
                                hipStream_t);

template void propagate<float>(const Grid&, const float*, const float*, const float*, float*,
                               float*, long long, int, int, float, bool, StateSet<float>,
                               StateSet<float>, hipStream_t, bool, const Force<float>*);
template void propagate<double>(const Grid&, const double*, const double*, const double*,
                                double*, double*, long long, int, int, double, bool,
                                StateSet<double>, StateSet<double>, hipStream_t, bool,
                                const Force<double>*);

}  // namespace pw
