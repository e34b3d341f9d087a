// Interpolation G and its adjoint (Sec. 2; Sec. 5: 8x8 Kaiser-Bessel
// kernels), with the data-block dual update of Algorithm 3 fused in.
//
// Work item: up to chunk_max visibilities whose first tap lies in one
// T x T grid tile, as per-block segments (at most 64), flattened into one
// range and taken in batches of 64.  The workgroup works on the tile plus
// its 7-cell halo, (T+7)^2 complex cells, in LDS:
//   degrid: the forward spectrum region is copied in, each thread then
//           interpolates its visibilities from LDS (64 taps each);
//   grid:   8 x 8 tiles (the default): the region is one 16 x 16 matrix
//           tile and gridding a product of the separable weights, done on
//           the matrix cores (k_grid_mfma).  Larger tiles: each wave owns
//           private copies of the region; a batch of 64 visibilities is
//           prepared one per lane (weights to LDS), then applied one
//           visibility at a time with lane (a, b) owning tap (a, b), so a
//           wave's 64 read-modify-writes never collide and no atomics are
//           needed (k_grid).  Either way the item's region is stored to a
//           per-item scratch slot; a fold pass then sums, for every grid
//           cell, the slots of the owning tile and the halos of its left /
//           upper / upper-left neighbours.  No global atomics, no zeroing
//           pass, and a fixed summation order across items.
// The 8 per-axis weights are evaluated on the fly from the even and odd
// parts of four degree-9 polynomials (the kernel is even), so only the two
// float32 frequencies are read per visibility.
// Items are launched in spatial order through an XCD-aware remap.
#include "ppd_internal.h"

namespace ppd {
namespace {

struct Taps {
  int ou, ov;         // first tap relative to the staged region
  float wx[KB_TAPS];  // u-axis weights
  float wy[KB_TAPS];  // v-axis weights
};

template <int T>
__device__ __forceinline__ void taps_for(float omu, float omv, double su, double sv, int Kx, int Ky,
                                         int c0, int r0, const float* coef, Taps& t) {
  const double tu = double(omu) * su, tv = double(omv) * sv;
  const double fu = floor(tu), fv = floor(tv);
  const int cu0 = (int(fu) - 3) & (Kx - 1);
  const int cv0 = (int(fv) - 3) & (Ky - 1);
  t.ou = min(max(cu0 - c0, 0), T - 1);
  t.ov = min(max(cv0 - r0, 0), T - 1);
  kb_weights(float(tu - fu), coef, t.wx);
  kb_weights(float(tv - fv), coef, t.wy);
}

// The coefficients kb_weights reads (taps 0..3), loaded with uniform
// addresses so that they stay in scalar registers (an LDS copy would be
// re-read by every lane for every batch).
struct KbCoef {
  float c[KB_TAPS / 2 * KB_NC];
};
__device__ __forceinline__ void load_kb(const float* __restrict__ kbc, KbCoef& k) {
#pragma unroll
  for (int i = 0; i < KB_TAPS / 2 * KB_NC; ++i) k.c[i] = kbc[i];
}

#ifndef PPD_DEGRID_WAVES
#define PPD_DEGRID_WAVES 4
#endif
#ifndef PPD_DEGRID_WAVES8
#define PPD_DEGRID_WAVES8 1
#endif
// Waves per degridding workgroup: 8 x 8 tiles hold ~100 visibilities, one
// wave's worth, so there each item is one single-wave workgroup.
template <int T>
struct DegridCfg {
  static constexpr int NW = T == 8 ? PPD_DEGRID_WAVES8 : PPD_DEGRID_WAVES;
};

// Degridding: one workgroup per item, the region staged in LDS; the item's
// visibilities (all its segments, flattened) are taken in batches of 64, a
// batch per wave in turn, one visibility per lane.  In the dual mode the
// per-segment partials of ||q - y||^2 and ||G a - y||^2 are wave sums over
// the lanes of each segment, added per wave in batch order and summed over
// the waves in a fixed order at the end: deterministic.
// 8 x 8 tiles: the 15 x 15 region is staged twice in LDS with a row stride
// of G8_RS float2 (16-byte aligned rows), copy E holding cell (r, c) at
// r G8_RS + c and copy O holding cell (r, c + 1) there, so that a lane's 8
// consecutive cells of a tap row start at an even float2 of one copy and
// are read as four 16-byte loads (half the LDS instructions of 8-byte
// loads).  The weighted sums run in the same order as the 8-byte form.
#ifndef PPD_DEGRID_B128
#define PPD_DEGRID_B128 1
#endif
constexpr int G8_RS = 18;
constexpr int G8_COPY = 15 * G8_RS;   // float2 per copy

__device__ __forceinline__ void stage8(float2* reg2, int e, float2 g) {
  const int a = e / 15, b = e - a * 15;
  reg2[a * G8_RS + b] = g;
  if (b > 0) reg2[G8_COPY + a * G8_RS + b - 1] = g;
}

__device__ __forceinline__ float2 gather8(const float2* reg2, const Taps& t) {
  const float2* base = (t.ou & 1) ? reg2 + G8_COPY + t.ov * G8_RS + (t.ou - 1) : reg2 + t.ov * G8_RS + t.ou;
  float ax = 0.f, ay = 0.f;
#pragma unroll
  for (int a = 0; a < KB_TAPS; ++a) {
    const float4* row = reinterpret_cast<const float4*>(base + a * G8_RS);
    const float4 q0 = row[0], q1 = row[1], q2 = row[2], q3 = row[3];
    float sx = 0.f, sy = 0.f;
    sx = fmaf(t.wx[0], q0.x, sx);
    sy = fmaf(t.wx[0], q0.y, sy);
    sx = fmaf(t.wx[1], q0.z, sx);
    sy = fmaf(t.wx[1], q0.w, sy);
    sx = fmaf(t.wx[2], q1.x, sx);
    sy = fmaf(t.wx[2], q1.y, sy);
    sx = fmaf(t.wx[3], q1.z, sx);
    sy = fmaf(t.wx[3], q1.w, sy);
    sx = fmaf(t.wx[4], q2.x, sx);
    sy = fmaf(t.wx[4], q2.y, sy);
    sx = fmaf(t.wx[5], q2.z, sx);
    sy = fmaf(t.wx[5], q2.w, sy);
    sx = fmaf(t.wx[6], q3.x, sx);
    sy = fmaf(t.wx[6], q3.y, sy);
    sx = fmaf(t.wx[7], q3.z, sx);
    sy = fmaf(t.wx[7], q3.w, sy);
    const float wya = a == 0 ? t.wy[0] : a == 1 ? t.wy[1] : a == 2 ? t.wy[2] : a == 3 ? t.wy[3]
                    : a == 4 ? t.wy[4] : a == 5 ? t.wy[5] : a == 6 ? t.wy[6] : t.wy[7];
    ax = fmaf(wya, sx, ax);
    ay = fmaf(wya, sy, ay);
  }
  return make_float2(ax, ay);
}

template <int T, bool DUAL>
__global__ __launch_bounds__(64 * DegridCfg<T>::NW) void k_degrid(
    const float2* __restrict__ grid, int Kx, int Ky, const Item* __restrict__ items, int n_items,
    const Seg* __restrict__ segs, const float* __restrict__ wu, const float* __restrict__ wv,
    const float* __restrict__ theta, double su, double sv, const float* __restrict__ kbc,
    float2* __restrict__ out, const float2* __restrict__ y, const double* __restrict__ U,
    const float2* __restrict__ v, const double2* __restrict__ z, float2* __restrict__ gout, double mu,
    double* __restrict__ part, double* __restrict__ rpart, XcdSplit xs) {
  constexpr int R = T + 7;
  constexpr int NW = DegridCfg<T>::NW;
  constexpr bool B128 = PPD_DEGRID_B128 && T == 8;
  __shared__ __align__(16) float2 reg[B128 ? 2 * G8_COPY : R * R];
  __shared__ ItemTab tab;
  __shared__ double s_q[NW][MAX_ITEM_SEGS], s_r[NW][MAX_ITEM_SEGS];
  const int ii = xcd_unit(blockIdx.x, xs);
  if (ii < 0 || ii >= n_items) return;
  const Item it = items[ii];
  const int r0 = it.ty * T, c0 = it.tx * T;
  const int lane = threadIdx.x & 63;
  const int uwid = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  // staging: all of the thread's loads are issued before its LDS stores
  constexpr int RPT = (R * R + 64 * NW - 1) / (64 * NW);
  float2 gv[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = threadIdx.x + k * 64 * NW;
    if (i < R * R) {
      const int a = i / R, b = i - a * R;
      gv[k] = grid[size_t((r0 + a) & (Ky - 1)) * Kx + ((c0 + b) & (Kx - 1))];
    }
  }
  load_item_tab(it, segs, tab);
  KbCoef kbw;
  load_kb(kbc, kbw);
  if (DUAL)
    for (int i = threadIdx.x; i < NW * MAX_ITEM_SEGS; i += blockDim.x) {
      (&s_q[0][0])[i] = 0.0;
      (&s_r[0][0])[i] = 0.0;
    }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = threadIdx.x + k * 64 * NW;
    if (i < R * R) {
      if constexpr (B128) stage8(reg, i, gv[k]);
      else reg[i] = gv[k];
    }
  }
  __syncthreads();
  const int nseg = it.seg1 - it.seg0;
  const int total = tab.pre[nseg];
  // Batch k of 64 flattened visibilities goes to wave k mod NW; a wave
  // loads its next batch's operands before working on the current one.
  struct Batch {
    float ou, ov, th;
    float2 v, y;
    double2 z;
    double U;
    int pi, sg, sb;
  };
  auto load = [&](int bt, int& sb, Batch& b) {
    while (bt * 64 >= tab.pre[sb + 1]) ++sb;
    b.sb = sb;
    const int li = bt * 64 + lane;
    b.sg = sb;
    if (li < total) {
      b.sg = seg_of(li, sb, tab.pre);
      b.pi = tab.start[b.sg] + (li - tab.pre[b.sg]);
      b.ou = wu[b.pi];
      b.ov = wv[b.pi];
      b.th = theta ? theta[b.pi] : 1.0f;
      if (DUAL) {
        b.v = v[b.pi];
        b.U = U[b.pi];
        b.z = z[b.pi];
        b.y = y[b.pi];
      }
    }
  };
  int sbl = 0;
  Batch bn{};
  if (uwid * 64 < total) load(uwid, sbl, bn);
  for (int bt = uwid; bt * 64 < total; bt += NW) {
    const Batch cb = bn;
    if ((bt + NW) * 64 < total) load(bt + NW, sbl, bn);
    const int li = bt * 64 + lane;
    const bool act = li < total;
    const int sb = __builtin_amdgcn_readfirstlane(cb.sb), sg = cb.sg, pi = cb.pi;
    double qn = 0.0, rn = 0.0;
    if (act) {
      const float omu = cb.ou, omv = cb.ov, th = cb.th;
      const float2 ve = cb.v, ye = cb.y;
      const double Ue = DUAL ? cb.U : 1.0;
      const double2 ze = cb.z;
      Taps t;
      taps_for<T>(omu, omv, su, sv, Kx, Ky, c0, r0, kbw.c, t);
      float ax = 0.f, ay = 0.f;
      if constexpr (B128) {
        const float2 s2 = gather8(reg, t);
        ax = s2.x;
        ay = s2.y;
      } else {
#pragma unroll
        for (int a = 0; a < KB_TAPS; ++a) {
          const float2* row = reg + (t.ov + a) * R + t.ou;
          float sx = 0.f, sy = 0.f;
#pragma unroll
          for (int b = 0; b < KB_TAPS; ++b) {
            const float2 g = row[b];
            sx = fmaf(t.wx[b], g.x, sx);
            sy = fmaf(t.wx[b], g.y, sy);
          }
          const float wya = a == 0 ? t.wy[0] : a == 1 ? t.wy[1] : a == 2 ? t.wy[2] : a == 3 ? t.wy[3]
                          : a == 4 ? t.wy[4] : a == 5 ? t.wy[5] : a == 6 ? t.wy[6] : t.wy[7];
          ax = fmaf(wya, sx, ax);
          ay = fmaf(wya, sy, ay);
        }
      }
      const float2 g = make_float2(ax * th, ay * th);
      if (!DUAL) {
        out[pi] = g;
      } else {
        // argument of the data-dual update of Algorithm 3: w = U^-1 v + Theta G a (Theta G a kept for the
        // gridding pass, which rebuilds w); first Algorithm 2 step
        gout[pi] = g;
        const double2 we = dual_arg(ve, Ue, g);
        const double wx = we.x, wy = we.y;
        const double mU = mu * Ue;
        const double dx = (ze.x - mU * (ze.x - wx)) - double(ye.x);
        const double dy = (ze.y - mU * (ze.y - wy)) - double(ye.y);
        qn = dx * dx + dy * dy;
        const double ex = double(g.x) - double(ye.x), ey = double(g.y) - double(ye.y);
        rn = ex * ex + ey * ey;
      }
    }
    if (DUAL) {
      const int slast = __builtin_amdgcn_readlane(sg, min(63, total - 1 - bt * 64));
      for (int ss = sb; ss <= slast; ++ss) {
        const double a = part ? wave_sum(act && sg == ss ? qn : 0.0) : 0.0;
        const double r = rpart ? wave_sum(act && sg == ss ? rn : 0.0) : 0.0;
        if (lane == 0) {
          s_q[uwid][ss] += a;
          s_r[uwid][ss] += r;
        }
      }
    }
  }
  if (DUAL) {
    __syncthreads();
    for (int k = threadIdx.x; k < nseg; k += blockDim.x) {
      double q = 0.0, r = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        q += s_q[w][k];
        r += s_r[w][k];
      }
      if (part) part[it.seg0 + k] = q;
      if (rpart) rpart[it.seg0 + k] = r;
    }
  }
}

// Operands of one gridding batch (one visibility per lane), loaded a batch
// ahead of use.
struct GridBatch {
  float ou, ov, th;
  float2 vin, y, v, ga;
  double2 z, bf;
  double U;
  int pi;
  bool act;
};

struct GridSrc {
  const float* wu; const float* wv; const float* theta;
  const float2* vin; const float2* y; const double* U; const float2* v; const double2* z;
  const float2* ga; const double2* bfac; const uint8_t* active;
};

// Loads batch bt (64 flattened visibilities of the item) for this lane;
// sb tracks the segment of the batch's first visibility.
template <bool DUAL>
__device__ __forceinline__ void grid_load(const GridSrc& g, const ItemTab& tab, int total, int lane, int bt,
                                          int& sb, GridBatch& b) {
  while (bt * 64 >= tab.pre[sb + 1]) ++sb;
  const int li = bt * 64 + lane;
  if (li < total) {
    const int sg = seg_of(li, sb, tab.pre);
    const int pi = tab.start[sg] + (li - tab.pre[sg]);
    b.pi = pi;
    b.ou = g.wu[pi];
    b.ov = g.wv[pi];
    b.th = g.theta ? g.theta[pi] : 1.0f;
    if (!DUAL) {
      b.vin = g.vin[pi];
    } else {
      b.ga = g.ga[pi];
      b.z = g.z[pi];
      b.U = g.U[pi];
      b.y = g.y[pi];
      b.v = g.v[pi];
      b.bf = g.bfac[tab.block[sg]];
      b.act = !g.active || g.active[tab.block[sg]];
    }
  }
}

// The value a visibility spreads onto the grid (before Theta).  In the dual
// mode: the last Algorithm 2 projection z = P_B(q) with the block's factor
// (or the exact prox with the block's nu), then the dual finish and relaxation; an inactive
// block (randomised updates of Algorithm 3) keeps v and z and spreads its v.
template <bool DUAL>
__device__ __forceinline__ float2 grid_value(const GridBatch& bt, double mu, double lambda, int exact,
                                             double2& znew, float2& vnew) {
  if (!DUAL) return bt.vin;
  if (!bt.act) return bt.v;
  const double2 bw = dual_arg(bt.v, bt.U, bt.ga);   // w of the data-dual update
  double zx, zy;
  if (exact) {
    // exact prox: (U w + nu y) / (U + nu) with the block's nu, w if nu = 0
    const double nu = bt.bf.x, inv = 1.0 / (bt.U + nu);
    zx = nu == 0.0 ? bw.x : (bt.U * bw.x + nu * double(bt.y.x)) * inv;
    zy = nu == 0.0 ? bw.y : (bt.U * bw.y + nu * double(bt.y.y)) * inv;
  } else {
    const double fac = bt.bf.x;
    const bool inside = bt.bf.y != 0.0;
    const double mU = mu * bt.U;
    const double qx = bt.z.x - mU * (bt.z.x - bw.x), qy = bt.z.y - mU * (bt.z.y - bw.y);
    zx = inside ? qx : double(bt.y.x) + (qx - double(bt.y.x)) * fac;
    zy = inside ? qy : double(bt.y.y) + (qy - double(bt.y.y)) * fac;
  }
  znew = make_double2(zx, zy);
  const double vbx = bt.U * (bw.x - zx), vby = bt.U * (bw.y - zy);
  vnew = make_float2(float(double(bt.v.x) + lambda * (vbx - double(bt.v.x))),
                     float(double(bt.v.y) + lambda * (vby - double(bt.v.y))));
  return vnew;
}

// Gridding workgroup shape: NW waves, each owning C private copies of the
// (T+7)^2 region in LDS (rows padded to T+8 cells, so the 8 tap rows of a
// footprint fall in distinct LDS banks).  Visibility k of a batch goes to
// copy k mod C: C independent read-modify-write chains per wave that the
// compiler interleaves (distinct LDS arrays cannot alias).
#ifndef PPD_GRID_CHAINS
#define PPD_GRID_CHAINS 2
#endif
#ifndef PPD_GRID_WAVES16
#define PPD_GRID_WAVES16 2
#endif
template <int T>
struct GridCfg {
  static constexpr int R = T + 7;
  static constexpr int RS = T + 8;
  static constexpr int C = (T <= 32) ? PPD_GRID_CHAINS : 2;
  static constexpr int NW = (T <= 16) ? PPD_GRID_WAVES16 : (T <= 32 ? 2 : 1);
  static constexpr int THREADS = NW * 64;
};

template <int T, bool DUAL>
__global__ __launch_bounds__(GridCfg<T>::THREADS) void k_grid(
    float2* __restrict__ scratch, int Kx, int Ky, const Item* __restrict__ items, int n_items,
    const Seg* __restrict__ segs, const float* __restrict__ wu, const float* __restrict__ wv,
    const float* __restrict__ theta, double su, double sv, const float* __restrict__ kbc,
    const float2* __restrict__ vin, const float2* __restrict__ y, const double* __restrict__ U,
    float2* __restrict__ v, double2* __restrict__ z, const float2* __restrict__ ga, double mu,
    double lambda, const double2* __restrict__ bfac, int exact, const uint8_t* __restrict__ active,
    XcdSplit xs) {
  constexpr int R = GridCfg<T>::R;
  constexpr int RS = GridCfg<T>::RS;
  constexpr int C = GridCfg<T>::C;
  constexpr int NW = GridCfg<T>::NW;
  __shared__ float2 acc[NW][C][R * RS];
  constexpr int WXS = KB_TAPS + 1;             // staging stride per visibility (bank spread)
  __shared__ float2 wxv[NW][64 * WXS];         // wx[b] * value, per visibility of the batch
  __shared__ float wyb[NW][64 * WXS];          // wy[a]
  __shared__ ItemTab tab;
  const int ii = xcd_unit(blockIdx.x, xs);
  if (ii < 0 || ii >= n_items) return;
  const Item it = items[ii];
  const int r0 = it.ty * T, c0 = it.tx * T;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int uwid = __builtin_amdgcn_readfirstlane(wid);   // wave-uniform
  load_item_tab(it, segs, tab);
  for (int i = threadIdx.x; i < NW * C * R * RS; i += blockDim.x) (&acc[0][0][0])[i] = make_float2(0.f, 0.f);
  KbCoef kbw;
  load_kb(kbc, kbw);
  __syncthreads();
  float2 (*myacc)[R * RS] = acc[wid];
  float2* mywxv = wxv[wid];
  float* mywy = wyb[wid];
  const int ta = lane >> 3, tb = lane & 7;   // tap of this lane in the apply phase
  const int lofs = ta * RS + tb;
  // The item's visibilities (all segments, flattened) are taken in batches
  // of 64, batch k by wave k mod NW.  The global operands of a wave's next
  // batch are loaded before its current batch is prepared and applied, so
  // their latency overlaps the LDS work.
  const GridSrc src{wu, wv, theta, vin, y, U, v, z, ga, bfac, active};
  const int nseg = it.seg1 - it.seg0;
  const int total = tab.pre[nseg];
  int sb = 0;
  GridBatch bn{};
  if (uwid * 64 < total) grid_load<DUAL>(src, tab, total, lane, uwid, sb, bn);
  for (int k = uwid; k * 64 < total; k += NW) {
    const GridBatch bt = bn;
    if ((k + NW) * 64 < total) grid_load<DUAL>(src, tab, total, lane, k + NW, sb, bn);
    const int nb = min(64, total - k * 64);
    // prepare: one visibility per lane (lanes past nb carry zero weight).
    // The new z and v are stored after the apply loop, so that no store is
    // in flight (and waited for) while the loop runs.
    double2 znew{};
    float2 vnew{};
    int pos = 0;
    float vx = 0.f, vy = 0.f;
    Taps t;
    if (lane < nb) {
      taps_for<T>(bt.ou, bt.ov, su, sv, Kx, Ky, c0, r0, kbw.c, t);
      const float2 val = grid_value<DUAL>(bt, mu, lambda, exact, znew, vnew);
      vx = val.x * bt.th;
      vy = val.y * bt.th;
      pos = t.ov * RS + t.ou;
    } else {
#pragma unroll
      for (int m = 0; m < KB_TAPS; ++m) {
        t.wx[m] = 0.f;
        t.wy[m] = 0.f;
      }
    }
#pragma unroll
    for (int m = 0; m < KB_TAPS; ++m) {
      mywxv[lane * WXS + m] = make_float2(t.wx[m] * vx, t.wx[m] * vy);
      mywy[lane * WXS + m] = t.wy[m];
    }
    __builtin_amdgcn_wave_barrier();
    // apply: lane (a, b) owns tap (a, b) of one visibility at a time, so
    // the wave's 64 read-modify-writes touch distinct cells (LDS float
    // atomics are far slower on this part, collisions or not).
    // C visibilities per step, visibility k into copy k mod C: C independent
    // read-modify-write chains.  (Summing runs of visibilities that share a
    // first-tap cell in registers before one read-modify-write per run was
    // measured slower: the data-dependent loop costs more than it saves.)
    const int nbc = (nb + C - 1) / C * C;
    for (int k = 0; k < nbc; k += C) {
      int pc[C];
      float2 xc[C], cc[C];
      float gc[C];
#pragma unroll
      for (int j = 0; j < C; ++j) {
        pc[j] = __builtin_amdgcn_readlane(pos, k + j) + lofs;
        xc[j] = mywxv[(k + j) * WXS + tb];
        gc[j] = mywy[(k + j) * WXS + ta];
        cc[j] = myacc[j][pc[j]];
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
        cc[j].x = fmaf(gc[j], xc[j].x, cc[j].x);
        cc[j].y = fmaf(gc[j], xc[j].y, cc[j].y);
        myacc[j][pc[j]] = cc[j];
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (DUAL && lane < nb && bt.act) {
      z[bt.pi] = znew;
      v[bt.pi] = vnew;
    }
  }
  __syncthreads();
  float2* dst = scratch + size_t(ii) * (R * R);
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
    const int ra = i / R, li = ra * RS + (i - ra * R);
    float sx = 0.f, sy = 0.f;
#pragma unroll
    for (int q2 = 0; q2 < NW; ++q2)
#pragma unroll
      for (int j = 0; j < C; ++j) {
        sx += acc[q2][j][li].x;
        sy += acc[q2][j][li].y;
      }
    dst[i] = make_float2(sx, sy);
  }
}

// Gridding of 8 x 8 tiles as a matrix product on the matrix cores.  The
// item's region (15 x 15 cells, padded to 16 x 16) receives
//     G[i][j] = sum_k wy_k(i) * (wx_k(j) * theta_k * val_k),
// wy_k(i) the v-axis weight of visibility k at region row i (zero outside
// its 8 taps), wx_k(j) likewise along u: a 16 x 16 x K product of the
// separable weights, accumulated over the item's visibilities 4 at a time by
// v_mfma_f32_16x16x4_f32 (real and imaginary parts), in FP32 registers.  A
// batch of 64 visibilities is prepared one per lane, as in k_grid, and its
// taps are written into 16-entry LDS rows that are zero elsewhere: weight
// rows (the A operand) and value-scaled weight rows (B), 32 rows at a time;
// lane l of a product step then reads row 4 g + l / 16, entry l mod 16, of
// each.  No read-modify-write of LDS.
//
// An 8 x 8 tile holds about one batch, so a single-wave workgroup takes a
// run of consecutive items, and the wave's (item, batch) steps form one
// software pipeline: the operands of the next step, which may be the next
// item's first batch, are loaded before the current step is prepared and
// applied, and the next item's segment list is fetched into registers when
// the current item starts.  Only the first step of a run waits for memory.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int GM_T = 8;
constexpr int GM_AS = 17;   // A row stride (floats): spreads the prepare writes over banks
constexpr int GM_BS = 17;   // B row stride (float2)
static_assert(PPD_GRIDM_RUN >= 1 && PPD_GRIDM_RUN <= 64, "a run's items are held one per lane");

// The segment list of one item as a lane's register (lane s: segment s).
__device__ __forceinline__ Seg item_seg(const Seg* __restrict__ segs, int seg0, int seg1, int lane) {
  Seg sg{0, 0, 0, 0};
  if (lane < seg1 - seg0) sg = segs[seg0 + lane];
  return sg;
}

// Segment table of an item from its lanes' segments (exclusive prefix sum
// of the counts); wave-local.
__device__ __forceinline__ void tab_from_seg(const Seg& sg, int lane, ItemTab& tab) {
  tab.start[lane] = sg.start;
  tab.block[lane] = sg.block;
  int inc = sg.count;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  tab.pre[lane + 1] = inc;
  if (lane == 0) tab.pre[0] = 0;
}

// Degridding of 8 x 8 tiles with the dual update by single-wave workgroups
// that each take a run of PPD_DEGRID_RUN consecutive items (0: one item per
// workgroup, k_degrid, which also serves plain Phi).
// The next item's region and segment list are loaded into registers while
// the current item is worked on; per-segment sums are kept by the lane of
// the segment (same order as k_degrid's).
__global__ __launch_bounds__(64) void k_degrid8(
    const float2* __restrict__ grid, int Kx, int Ky, const Item* __restrict__ items, int n_items,
    const Seg* __restrict__ segs, const float* __restrict__ wu, const float* __restrict__ wv,
    const float* __restrict__ theta, double su, double sv, const float* __restrict__ kbc,
    const float2* __restrict__ y, const double* __restrict__ U,
    const float2* __restrict__ v, const double2* __restrict__ z, float2* __restrict__ gout, double mu,
    double* __restrict__ part, double* __restrict__ rpart, XcdSplit xs) {
  constexpr int T = 8, R = T + 7, RUN = PPD_DEGRID_RUN > 0 ? PPD_DEGRID_RUN : 1;
  constexpr int RPT = (R * R + 63) / 64;
  static_assert(RUN <= 64, "a run's items are held one per lane");
  __shared__ float2 reg[R * R];
  __shared__ ItemTab tab;
  const int unit = xcd_unit(blockIdx.x, xs);
  if (unit < 0) return;
  const int i0 = unit * RUN;
  if (i0 >= n_items) return;
  const int i1 = min(i0 + RUN, n_items);
  const int lane = threadIdx.x;
  Item itl{0, 0, 0, 0};
  if (i0 + lane < i1) itl = items[i0 + lane];
  auto field = [&](int f, int i) { return __builtin_amdgcn_readlane(f, i - i0); };
  float2 gv[RPT];
  auto region = [&](int i) {
    const int r0 = field(itl.ty, i) * T, c0 = field(itl.tx, i) * T;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int e = lane + k * 64;
      if (e < R * R) {
        const int a = e / R, b = e - a * R;
        gv[k] = grid[size_t((r0 + a) & (Ky - 1)) * Kx + ((c0 + b) & (Kx - 1))];
      }
    }
  };
  region(i0);
  Seg sgn = item_seg(segs, field(itl.seg0, i0), field(itl.seg1, i0), lane);
  KbCoef kbw;
  load_kb(kbc, kbw);
  struct Batch {
    float ou, ov, th;
    float2 v, y;
    double2 z;
    double U;
    int pi, sg, sb;
  };
  for (int cur = i0; cur < i1; ++cur) {
    // the previous item's LDS reads are done (program order within the wave)
    tab_from_seg(sgn, lane, tab);
#pragma unroll
    for (int k = 0; k < RPT; ++k)
      if (lane + k * 64 < R * R) reg[lane + k * 64] = gv[k];
    __builtin_amdgcn_wave_barrier();
    const int r0 = field(itl.ty, cur) * T, c0 = field(itl.tx, cur) * T;
    const int seg0 = field(itl.seg0, cur), nseg = field(itl.seg1, cur) - seg0;
    const int total = __builtin_amdgcn_readfirstlane(tab.pre[nseg]);
    auto load = [&](int bt, int& sb, Batch& b) {
      while (bt * 64 >= tab.pre[sb + 1]) ++sb;
      b.sb = sb;
      const int li = bt * 64 + lane;
      b.sg = sb;
      if (li < total) {
        b.sg = seg_of(li, sb, tab.pre);
        b.pi = tab.start[b.sg] + (li - tab.pre[b.sg]);
        b.ou = wu[b.pi];
        b.ov = wv[b.pi];
        b.th = theta ? theta[b.pi] : 1.0f;
        b.v = v[b.pi];
        b.U = U[b.pi];
        b.z = z[b.pi];
        b.y = y[b.pi];
      }
    };
    int sbl = 0;
    Batch bn{};
    if (total > 0) load(0, sbl, bn);
    // the next item's region and segments, behind this item's first batch
    if (cur + 1 < i1) {
      region(cur + 1);
      sgn = item_seg(segs, field(itl.seg0, cur + 1), field(itl.seg1, cur + 1), lane);
    }
    double q_acc = 0.0, r_acc = 0.0;   // lane s: segment s of the item
    for (int bt = 0; bt * 64 < total; ++bt) {
      const Batch cb = bn;
      if ((bt + 1) * 64 < total) load(bt + 1, sbl, bn);
      const int li = bt * 64 + lane;
      const bool act = li < total;
      const int sb = __builtin_amdgcn_readfirstlane(cb.sb), sg = cb.sg, pi = cb.pi;
      double qn = 0.0, rn = 0.0;
      if (act) {
        Taps t;
        taps_for<T>(cb.ou, cb.ov, su, sv, Kx, Ky, c0, r0, kbw.c, t);
        // 8-byte gathers: the 16-byte form of k_degrid took this kernel to
        // 158 VGPRs (3 waves per SIMD) and was not faster here
        float ax = 0.f, ay = 0.f;
#pragma unroll
        for (int a = 0; a < KB_TAPS; ++a) {
          const float2* row = reg + (t.ov + a) * R + t.ou;
          float sx = 0.f, sy = 0.f;
#pragma unroll
          for (int b = 0; b < KB_TAPS; ++b) {
            const float2 g = row[b];
            sx = fmaf(t.wx[b], g.x, sx);
            sy = fmaf(t.wx[b], g.y, sy);
          }
          const float wya = a == 0 ? t.wy[0] : a == 1 ? t.wy[1] : a == 2 ? t.wy[2] : a == 3 ? t.wy[3]
                          : a == 4 ? t.wy[4] : a == 5 ? t.wy[5] : a == 6 ? t.wy[6] : t.wy[7];
          ax = fmaf(wya, sx, ax);
          ay = fmaf(wya, sy, ay);
        }
        // the data-dual argument of Algorithm 3 and the first Algorithm 2 step, as in
        // k_degrid
        const float2 g = make_float2(ax * cb.th, ay * cb.th);
        gout[pi] = g;
        const double Ue = cb.U;
        const double2 we = dual_arg(cb.v, Ue, g), ze = cb.z;
        const double mU = mu * Ue;
        const double dx = (ze.x - mU * (ze.x - we.x)) - double(cb.y.x);
        const double dy = (ze.y - mU * (ze.y - we.y)) - double(cb.y.y);
        qn = dx * dx + dy * dy;
        const double ex = double(g.x) - double(cb.y.x), ey = double(g.y) - double(cb.y.y);
        rn = ex * ex + ey * ey;
      }
      const int slast = __builtin_amdgcn_readlane(sg, min(63, total - 1 - bt * 64));
      for (int ss = sb; ss <= slast; ++ss) {
        const double a = part ? wave_sum(act && sg == ss ? qn : 0.0) : 0.0;   // Algorithm 2 only
        const double r = rpart ? wave_sum(act && sg == ss ? rn : 0.0) : 0.0;   // statistics only
        if (lane == ss) {
          q_acc += a;
          r_acc += r;
        }
      }
    }
    if (lane < nseg) {
      if (part) part[seg0 + lane] = q_acc;
      if (rpart) rpart[seg0 + lane] = r_acc;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <bool DUAL>
__global__ __launch_bounds__(64 * PPD_GRIDM_WPG) void k_grid_mfma(
    float2* __restrict__ scratch, int Kx, int Ky, const Item* __restrict__ items, int n_items,
    const Seg* __restrict__ segs, const float* __restrict__ wu, const float* __restrict__ wv,
    const float* __restrict__ theta, double su, double sv, const float* __restrict__ kbc,
    const float2* __restrict__ vin, const float2* __restrict__ y, const double* __restrict__ U,
    float2* __restrict__ v, double2* __restrict__ z, const float2* __restrict__ ga, double mu,
    double lambda, const double2* __restrict__ bfac, int exact, const uint8_t* __restrict__ active,
    XcdSplit xs) {
  constexpr int T = GM_T, R = T + 7, WPG = PPD_GRIDM_WPG;
  static_assert(R <= 16, "the region must fit one 16 x 16 product tile");
  __shared__ float sAw[WPG][32 * GM_AS];
  __shared__ float2 sBw[WPG][32 * GM_BS];
  __shared__ ItemTab tabsw[WPG][2];   // per wave: current and next item
  KbCoef kbw;
  load_kb(kbc, kbw);
  __syncthreads();
  // each wave of the workgroup works alone from here on
  const int wid = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int unit = xcd_unit(blockIdx.x, xs);
  if (unit < 0) return;
  const int i0 = (unit * WPG + wid) * PPD_GRIDM_RUN;
  if (i0 >= n_items) return;
  const int i1 = min(i0 + PPD_GRIDM_RUN, n_items);
  const int lane = threadIdx.x & 63;
  float* sA = sAw[wid];
  float2* sB = sBw[wid];
  ItemTab* tabs = tabsw[wid];
  const int gq = lane >> 4, gc = lane & 15;   // row-in-group and entry read in a product step
  // the run's items, one per lane; item i's fields come from lane i - i0
  Item itl{0, 0, 0, 0};
  if (i0 + lane < i1) itl = items[i0 + lane];
  const GridSrc src{wu, wv, theta, vin, y, U, v, z, ga, bfac, active};
  auto field = [&](int v, int i) { return __builtin_amdgcn_readlane(v, i - i0); };
  tab_from_seg(item_seg(segs, field(itl.seg0, i0), field(itl.seg1, i0), lane), lane, tabs[0]);
  Seg sgn{0, 0, 0, 0};   // next item's segments, fetched when an item starts
  if (i0 + 1 < i1) sgn = item_seg(segs, field(itl.seg0, i0 + 1), field(itl.seg1, i0 + 1), lane);
  __builtin_amdgcn_wave_barrier();
  f32x4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
  f32x4 accr2 = {0.f, 0.f, 0.f, 0.f}, acci2 = {0.f, 0.f, 0.f, 0.f};
  int cur = i0, kb = 0, sb = 0;
  int total = __builtin_amdgcn_readfirstlane(tabs[0].pre[field(itl.seg1, i0) - field(itl.seg0, i0)]);
  GridBatch bn{};
  grid_load<DUAL>(src, tabs[0], total, lane, 0, sb, bn);
  float* arow = sA + (lane & 31) * GM_AS;
  float2* brow = sB + (lane & 31) * GM_BS;
  const float* aq = sA + gq * GM_AS + gc;    // entry read by this lane in product step 0
  const float2* bq = sB + gq * GM_BS + gc;
  // the staging rows start zero; each batch writes its taps and clears them
  for (int e = lane; e < 32 * GM_AS; e += 64) sA[e] = 0.f;
  for (int e = lane; e < 32 * GM_BS; e += 64) sB[e] = make_float2(0.f, 0.f);
  __builtin_amdgcn_wave_barrier();
  while (true) {
    const int nb = min(64, total - kb * 64);
    const int c0 = field(itl.tx, cur) * T, r0 = field(itl.ty, cur) * T;
    // this step's taps and values, from the operands loaded during the
    // previous step; bn is free again afterwards
    double2 znew{};
    float2 vnew{};
    float vx = 0.f, vy = 0.f;
    Taps t;
    t.ou = 0;
    t.ov = 0;
    const bool has = lane < nb;
    const int pi = bn.pi;
    const bool zst = DUAL && has && bn.act;
    if (has) {
      taps_for<T>(bn.ou, bn.ov, su, sv, Kx, Ky, c0, r0, kbw.c, t);
      const float2 val = grid_value<DUAL>(bn, mu, lambda, exact, znew, vnew);
      vx = val.x * bn.th;
      vy = val.y * bn.th;
    }
    // stores before the next step's loads: vector memory operations
    // complete in issue order, so the wait for those loads does not add a
    // wait for stores issued after them
    if (zst) {
      z[pi] = znew;
      v[pi] = vnew;
    }
    // the next step: the next batch of this item, else the next item's first
    const bool last = (kb + 1) * 64 >= total;
    const int nxt = last ? cur + 1 : cur;
    int ntotal = total;
    if (nxt < i1) {
      ItemTab& tn = tabs[(nxt - i0) & 1];
      if (last) {
        tab_from_seg(sgn, lane, tn);
        __builtin_amdgcn_wave_barrier();
        ntotal = __builtin_amdgcn_readfirstlane(tn.pre[field(itl.seg1, nxt) - field(itl.seg0, nxt)]);
        sb = 0;
        if (nxt + 1 < i1) sgn = item_seg(segs, field(itl.seg0, nxt + 1), field(itl.seg1, nxt + 1), lane);
      }
      grid_load<DUAL>(src, tn, ntotal, lane, last ? 0 : kb + 1, sb, bn);
    }
    // The batch goes through LDS in two halves of 32 rows (half the staging
    // memory: more waves per CU): lanes 0-31 write their 8 taps into rows
    // that are otherwise zero and the first 8 product steps read them, the
    // lanes put the zeros back, then the same for lanes 32-63.  Rows of
    // lanes past the batch end are never written.  The tap stores go to a
    // per-lane base with constant offsets; LDS operations of one wave take
    // effect in program order, so the zeros land after the product reads.
    float* pa = arow + t.ov;
    float2* pb = brow + t.ou;
    for (int h = 0; h * 32 < nb; ++h) {
      const bool mine = has && (lane >> 5) == h;
      if (mine) {
#pragma unroll
        for (int m = 0; m < KB_TAPS; ++m) {
          pa[m] = t.wy[m];
          pb[m] = make_float2(t.wx[m] * vx, t.wx[m] * vy);
        }
      }
      __builtin_amdgcn_wave_barrier();
      // the operands of PPD_GRIDM_READ_AHEAD product steps are read before
      // their first product (rows past the batch end read as zero); two
      // accumulator pairs (even / odd steps) make independent chains
      constexpr int RA = PPD_GRIDM_READ_AHEAD;
      static_assert(RA == 2 || RA == 4 || RA == 8, "read-ahead of 2, 4 or 8 product steps");
      const int ng = (min(32, nb - 32 * h) + 3) >> 2;
#pragma unroll
      for (int g0 = 0; g0 < 8; g0 += RA) {
        float a8[RA];
        float2 b8[RA];
#pragma unroll
        for (int g = 0; g < RA; ++g) {
          a8[g] = aq[4 * (g0 + g) * GM_AS];
          b8[g] = bq[4 * (g0 + g) * GM_BS];
        }
#pragma unroll
        for (int g = 0; g < RA; g += 2) {
          if (g0 + g < ng) {
            accr = __builtin_amdgcn_mfma_f32_16x16x4f32(a8[g], b8[g].x, accr, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_16x16x4f32(a8[g], b8[g].y, acci, 0, 0, 0);
          }
          if (g0 + g + 1 < ng) {
            accr2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a8[g + 1], b8[g + 1].x, accr2, 0, 0, 0);
            acci2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a8[g + 1], b8[g + 1].y, acci2, 0, 0, 0);
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (mine) {
#pragma unroll
        for (int m = 0; m < KB_TAPS; ++m) {
          pa[m] = 0.f;
          pb[m] = make_float2(0.f, 0.f);
        }
      }
    }
    if (last) {
      // Lane l holds rows 4 (l / 16) + e, e = 0..3, of column l mod 16 (row
      // 15 and column 15 stay zero: no footprint reaches them).
      const f32x4 sr = accr + accr2, si = acci + acci2;
      float2* dst = scratch + size_t(cur) * (R * R);
      if (gc < R)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (4 * gq + e < R) dst[(4 * gq + e) * R + gc] = make_float2(sr[e], si[e]);
      accr = accr2 = acci = acci2 = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    if (nxt >= i1) break;
    cur = nxt;
    kb = last ? 0 : kb + 1;
    total = ntotal;
  }
}

// One thread per grid cell (FOLD_CELLS cells per workgroup, T*T/FOLD_CELLS
// workgroups per tile); the item loops are unrolled so their independent
// loads overlap.
constexpr int FOLD_CELLS = 256;

__device__ __forceinline__ void fold_items(const float2* __restrict__ scratch, int R2, int off, int i0,
                                           int i1, float& sx, float& sy) {
  int i = i0;
  for (; i + 4 <= i1; i += 4) {
    const float2 g0 = scratch[size_t(i) * R2 + off];
    const float2 g1 = scratch[size_t(i + 1) * R2 + off];
    const float2 g2 = scratch[size_t(i + 2) * R2 + off];
    const float2 g3 = scratch[size_t(i + 3) * R2 + off];
    sx += (g0.x + g1.x) + (g2.x + g3.x);
    sy += (g0.y + g1.y) + (g2.y + g3.y);
  }
  for (; i < i1; ++i) {
    const float2 g = scratch[size_t(i) * R2 + off];
    sx += g.x;
    sy += g.y;
  }
}

template <int T>
__global__ __launch_bounds__(FOLD_CELLS) void k_fold(const float2* __restrict__ scratch,
                                                     const int32_t* __restrict__ tio, int tiles_x,
                                                     int tiles_y, int Kx, float2* __restrict__ grid) {
  constexpr int R = T + 7;
  constexpr int PARTS = (T * T) / FOLD_CELLS;
  static_assert(PARTS >= 1 && T > 7, "whole workgroups per tile; a cell lies in at most 4 tile regions");
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  if (wg >= tiles_x * tiles_y * PARTS) return;
  const int t = wg / PARTS, part = wg - t * PARTS;
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int lx = (tx + tiles_x - 1) % tiles_x, uy = (ty + tiles_y - 1) % tiles_y;
  const int tl = ty * tiles_x + lx, tu = uy * tiles_x + tx, tul = uy * tiles_x + lx;
  const int c = part * FOLD_CELLS + threadIdx.x;
  const int a = c / T, b = c - a * T;
  float sx = 0.f, sy = 0.f;
  fold_items(scratch, R * R, a * R + b, tio[t], tio[t + 1], sx, sy);
  if (b < 7) fold_items(scratch, R * R, a * R + T + b, tio[tl], tio[tl + 1], sx, sy);
  if (a < 7) {
    fold_items(scratch, R * R, (T + a) * R + b, tio[tu], tio[tu + 1], sx, sy);
    if (b < 7) fold_items(scratch, R * R, (T + a) * R + T + b, tio[tul], tio[tul + 1], sx, sy);
  }
  grid[size_t(ty * T + a) * Kx + (tx * T + b)] = make_float2(sx, sy);
}

// 8 x 8 tiles, 4-wave workgroups in the plan's fold order (tile rows spread
// over the XCDs, on each XCD the tiles with the most item regions first).
// Entry {t0, t1, t2, t3} folds up to four light tiles, one per wave, one
// thread per cell; entry {t, -2, -2, -2} folds one heavy tile (more than
// FOLD_HEAVY regions to sum: the dense centre of the coverage), wave w
// summing every fourth item region of each source tile from the w-th, the
// four partial sums then added in wave order.
__device__ __forceinline__ void fold_items4(const float2* __restrict__ scratch, int R2, int off, int i0, int i1,
                                            float& sx, float& sy) {
  int i = i0;
  for (; i + 12 < i1; i += 16) {
    const float2 g0 = scratch[size_t(i) * R2 + off];
    const float2 g1 = scratch[size_t(i + 4) * R2 + off];
    const float2 g2 = scratch[size_t(i + 8) * R2 + off];
    const float2 g3 = scratch[size_t(i + 12) * R2 + off];
    sx += (g0.x + g1.x) + (g2.x + g3.x);
    sy += (g0.y + g1.y) + (g2.y + g3.y);
  }
  for (; i < i1; i += 4) {
    const float2 g = scratch[size_t(i) * R2 + off];
    sx += g.x;
    sy += g.y;
  }
}

__global__ __launch_bounds__(256) void k_fold8(const float2* __restrict__ scratch, const int32_t* __restrict__ tio,
                                                const int4* __restrict__ wgs, int tiles_x, int tiles_y, int Kx,
                                                float2* __restrict__ grid) {
  constexpr int T = 8, R = T + 7;
  __shared__ float2 part[4][64];
  const int4 e = wgs[xcd_remap(blockIdx.x, gridDim.x)];
  const int w = threadIdx.x >> 6, c = threadIdx.x & 63;
  const int a = c / T, b = c - a * T;
  const bool heavy = e.y == -2;   // uniform over the workgroup
  const int t = heavy ? e.x : (w == 0 ? e.x : w == 1 ? e.y : w == 2 ? e.z : e.w);
  if (t < 0) return;              // never taken by a heavy workgroup
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int lx = (tx + tiles_x - 1) % tiles_x, uy = (ty + tiles_y - 1) % tiles_y;
  const int tl = ty * tiles_x + lx, tu = uy * tiles_x + tx, tul = uy * tiles_x + lx;
  float sx = 0.f, sy = 0.f;
  if (!heavy) {
    fold_items(scratch, R * R, a * R + b, tio[t], tio[t + 1], sx, sy);
    if (b < 7) fold_items(scratch, R * R, a * R + T + b, tio[tl], tio[tl + 1], sx, sy);
    if (a < 7) {
      fold_items(scratch, R * R, (T + a) * R + b, tio[tu], tio[tu + 1], sx, sy);
      if (b < 7) fold_items(scratch, R * R, (T + a) * R + T + b, tio[tul], tio[tul + 1], sx, sy);
    }
    grid[size_t(ty * T + a) * Kx + (tx * T + b)] = make_float2(sx, sy);
    return;
  }
  fold_items4(scratch, R * R, a * R + b, tio[t] + w, tio[t + 1], sx, sy);
  if (b < 7) fold_items4(scratch, R * R, a * R + T + b, tio[tl] + w, tio[tl + 1], sx, sy);
  if (a < 7) {
    fold_items4(scratch, R * R, (T + a) * R + b, tio[tu] + w, tio[tu + 1], sx, sy);
    if (b < 7) fold_items4(scratch, R * R, (T + a) * R + T + b, tio[tul] + w, tio[tul + 1], sx, sy);
  }
  part[w][c] = make_float2(sx, sy);
  __syncthreads();
  if (w == 0) {
    const float2 p0 = part[0][c], p1 = part[1][c], p2 = part[2][c], p3 = part[3][c];
    grid[size_t(ty * T + a) * Kx + (tx * T + b)] =
        make_float2(((p0.x + p1.x) + p2.x) + p3.x, ((p0.y + p1.y) + p2.y) + p3.y);
  }
}

template <typename E>
__global__ void k_permute(const int32_t* __restrict__ perm, int64_t M, int to_user,
                          const E* __restrict__ in, E* __restrict__ out) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    if (to_user) out[perm[i]] = in[i];
    else out[i] = in[perm[i]];
  }
}


template <int T>
int launch_degrid(ppd_plan* p, bool dual, float2* out, const DualArgs* a, double* part_out) {
  // runs for the fused dual pass only: plain Phi is faster one item per
  // workgroup (27.4 against 29.7 us at 512^2, M = 1.3M)
  if (T == 8 && PPD_DEGRID_RUN > 0 && dual) {
    hipLaunchKernelGGL(k_degrid8, dim3(p->split_degrid.launch), dim3(64), 0, p->stream, p->grid_f, p->Kx, p->Ky,
                       p->items, p->n_items, p->segs, p->wu, p->wv, p->theta, p->su_scale, p->sv_scale, p->kbc,
                       a->y, a->U, a->v, a->z, p->gabuf, a->mu, part_out, a->rpart, p->split_degrid);
    PPD_HIP(hipGetLastError());
    return PPD_OK;
  }
  if (!dual) {
    hipLaunchKernelGGL((k_degrid<T, false>), dim3(p->split1.launch), dim3(64 * DegridCfg<T>::NW), 0, p->stream,
                       p->grid_f, p->Kx, p->Ky, p->items, p->n_items, p->segs, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, out, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0,
                       nullptr, nullptr, p->split1);
  } else {
    hipLaunchKernelGGL((k_degrid<T, true>), dim3(p->split1.launch), dim3(64 * DegridCfg<T>::NW), 0, p->stream,
                       p->grid_f, p->Kx, p->Ky, p->items, p->n_items, p->segs, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, nullptr, a->y, a->U, a->v, a->z, p->gabuf, a->mu,
                       part_out, a->rpart, p->split1);
  }
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

int launch_grid_mfma(ppd_plan* p, bool dual, const float2* vin, const DualArgs* a, int exact) {
  if (!dual) {
    hipLaunchKernelGGL((k_grid_mfma<false>), dim3(p->split_grid.launch), dim3(64 * PPD_GRIDM_WPG), 0, p->stream,
                       p->gscratch, p->Kx, p->Ky, p->items, p->n_items, p->segs, p->wu, p->wv, p->theta,
                       p->su_scale, p->sv_scale, p->kbc, vin, nullptr, nullptr, nullptr, nullptr, nullptr,
                       0.0, 0.0, nullptr, 0, nullptr, p->split_grid);
  } else {
    hipLaunchKernelGGL((k_grid_mfma<true>), dim3(p->split_grid.launch), dim3(64 * PPD_GRIDM_WPG), 0, p->stream,
                       p->gscratch, p->Kx, p->Ky, p->items, p->n_items, p->segs, p->wu, p->wv, p->theta,
                       p->su_scale, p->sv_scale, p->kbc, nullptr, a->y, a->U, a->v, a->z, p->gabuf, a->mu,
                       a->lambda, p->bfac, exact, a->active, p->split_grid);
  }
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

template <int T>
int launch_grid(ppd_plan* p, bool dual, const float2* vin, const DualArgs* a, int exact) {
  if (!dual) {
    hipLaunchKernelGGL((k_grid<T, false>), dim3(p->split1.launch), dim3(GridCfg<T>::THREADS), 0, p->stream,
                       p->gscratch, p->Kx, p->Ky, p->items, p->n_items, p->segs, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, vin, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0,
                       0.0, nullptr, 0, nullptr, p->split1);
  } else {
    hipLaunchKernelGGL((k_grid<T, true>), dim3(p->split1.launch), dim3(GridCfg<T>::THREADS), 0, p->stream,
                       p->gscratch, p->Kx, p->Ky, p->items, p->n_items, p->segs, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, nullptr, a->y, a->U, a->v, a->z, p->gabuf, a->mu,
                       a->lambda, p->bfac, exact, a->active, p->split1);
  }
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

template <int T>
int launch_fold(ppd_plan* p) {
  const int n = p->n_tiles * ((T * T) / FOLD_CELLS);
  const int nl = ((n + MAX_XCD - 1) / MAX_XCD) * MAX_XCD;
  hipLaunchKernelGGL(k_fold<T>, dim3(nl), dim3(FOLD_CELLS), 0, p->stream, p->gscratch,
                     p->tile_item_off, p->tiles_x, p->tiles_y, p->Kx, p->grid_a);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

int launch_fold8(ppd_plan* p) {
  hipLaunchKernelGGL(k_fold8, dim3(p->n_fold_wg), dim3(256), 0, p->stream, p->gscratch, p->tile_item_off,
                     reinterpret_cast<const int4*>(p->fold_wg), p->tiles_x, p->tiles_y, p->Kx, p->grid_a);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

int dispatch_degrid(ppd_plan* p, bool dual, float2* out, const DualArgs* a, double* part_out) {
  int slot;
  PPD_TRY(timer_begin(p, KK_DEGRID, &slot));
  int st;
  switch (p->T) {
    case 8: st = launch_degrid<8>(p, dual, out, a, part_out); break;
    case 16: st = launch_degrid<16>(p, dual, out, a, part_out); break;
    case 32: st = launch_degrid<32>(p, dual, out, a, part_out); break;
    default: st = launch_degrid<64>(p, dual, out, a, part_out); break;
  }
  PPD_TRY(st);
  return timer_end(p, slot);
}

int dispatch_grid(ppd_plan* p, bool dual, const float2* vin, const DualArgs* a, int exact) {
  int slot;
  PPD_TRY(timer_begin(p, KK_GRID, &slot));
  int st;
  switch (p->T) {
    case 8: st = launch_grid_mfma(p, dual, vin, a, exact); break;
    case 16: st = launch_grid<16>(p, dual, vin, a, exact); break;
    case 32: st = launch_grid<32>(p, dual, vin, a, exact); break;
    default: st = launch_grid<64>(p, dual, vin, a, exact); break;
  }
  PPD_TRY(st);
  return timer_end(p, slot);
}

}  // namespace

int degrid_plain(ppd_plan* p, float2* out) { return dispatch_degrid(p, false, out, nullptr, nullptr); }
int degrid_dual(ppd_plan* p, const DualArgs& a, double* part_out) {
  return dispatch_degrid(p, true, nullptr, &a, part_out);
}

int grid_plain(ppd_plan* p, const float2* v) {
  PPD_TRY(dispatch_grid(p, false, v, nullptr, 0));
  return fold_grid(p);
}

int grid_dual(ppd_plan* p, const DualArgs& a, const double* part_in) {
  PPD_TRY(block_factors(p, part_in));
  PPD_TRY(dispatch_grid(p, true, nullptr, &a, 0));
  return fold_grid(p);
}

int grid_dual_factored(ppd_plan* p, const DualArgs& a) {
  PPD_TRY(dispatch_grid(p, true, nullptr, &a, 0));
  return fold_grid(p);
}

int grid_dual_exact(ppd_plan* p, const DualArgs& a) {
  PPD_TRY(dispatch_grid(p, true, nullptr, &a, 1));
  return fold_grid(p);
}

int fold_grid(ppd_plan* p) {
  int slot;
  PPD_TRY(timer_begin(p, KK_FOLD, &slot));
  int st;
  switch (p->T) {
    case 8: st = launch_fold8(p); break;
    case 16: st = launch_fold<16>(p); break;
    case 32: st = launch_fold<32>(p); break;
    default: st = launch_fold<64>(p); break;
  }
  PPD_TRY(st);
  return timer_end(p, slot);
}

int permute(ppd_plan* p, int direction, const void* in, void* out, int elem_bytes) {
  int slot;
  PPD_TRY(timer_begin(p, KK_PERMUTE, &slot));
  const int to_user = direction == PPD_PLAN_TO_USER;
  const int blocks = int(std::min<int64_t>((p->M + 255) / 256, 4096));
  switch (elem_bytes) {
    case 4:
      hipLaunchKernelGGL(k_permute<float>, dim3(blocks), dim3(256), 0, p->stream, p->perm, p->M,
                         to_user, static_cast<const float*>(in), static_cast<float*>(out));
      break;
    case 8:
      hipLaunchKernelGGL(k_permute<float2>, dim3(blocks), dim3(256), 0, p->stream, p->perm, p->M,
                         to_user, static_cast<const float2*>(in), static_cast<float2*>(out));
      break;
    default:
      hipLaunchKernelGGL(k_permute<double2>, dim3(blocks), dim3(256), 0, p->stream, p->perm, p->M,
                         to_user, static_cast<const double2*>(in), static_cast<double2*>(out));
      break;
  }
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

}  // namespace ppd

using namespace ppd;

extern "C" int ppd_phi(ppd_plan* p, const float* x, float* y, int order) {
  if (!p || !x || !y) return fail(PPD_EINVAL, "ppd_phi: NULL argument");
  if (order != PPD_ORDER_PLAN && order != PPD_ORDER_USER) return fail(PPD_EINVAL, "ppd_phi: bad order");
  PPD_TRY(fft_forward(p, x));
  if (order == PPD_ORDER_PLAN) return degrid_plain(p, reinterpret_cast<float2*>(y));
  PPD_TRY(degrid_plain(p, p->ybuf));
  return permute(p, PPD_PLAN_TO_USER, p->ybuf, y, 8);
}

extern "C" int ppd_phit(ppd_plan* p, const float* y, float* x, int order) {
  if (!p || !x || !y) return fail(PPD_EINVAL, "ppd_phit: NULL argument");
  if (order != PPD_ORDER_PLAN && order != PPD_ORDER_USER) return fail(PPD_EINVAL, "ppd_phit: bad order");
  const float2* v = reinterpret_cast<const float2*>(y);
  if (order == PPD_ORDER_USER) {
    PPD_TRY(permute(p, PPD_USER_TO_PLAN, y, p->ybuf, 8));
    v = p->ybuf;
  }
  PPD_TRY(grid_plain(p, v));
  return fft_adjoint(p, x);
}
