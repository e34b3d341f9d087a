// SARA sparsity operator (Sec. 5.1): Psi = (1/3)[I, W_1, .., W_8], W_p the
// orthonormal periodised 2D Daubechies-p wavelet transform, coefficients in
// the Mallat layout of the image.  Float32.
//
// Analysis runs one launch per level for the 8 wavelet bases at once
// (one grid dimension per basis; the Dirac basis rides in the first launch): a
// workgroup stages the periodic input region of its output tile in LDS,
// filters the columns, then the rows, and writes the four sub-bands.  In
// the dual mode (the sparsity dual update of Algorithm 3) every final coefficient c is
// consumed in place: u <- u + lambda (clip(u + c, +-alpha) - u).
// Synthesis is the transpose, one launch per level; the last level sums the
// 8 reconstructions and the Dirac part in registers (no atomics) and applies
// the 1/3.
#include <cmath>

#include "ppd_internal.h"

namespace ppd {
namespace {

constexpr int AT = 16;   // analysis output tile per sub-band
constexpr int ST = 32;   // synthesis output tile (inner levels)
constexpr int STF = 16;  // synthesis output tile of the last level (8 bases summed)
constexpr int SIN = 2 * AT + 2 * FILT_STRIDE - 2;   // staged analysis input extent (db8)
constexpr int SK = ST / 2 + FILT_STRIDE / 2;         // staged synthesis coefficient extent

struct SaraGeom {
  int nx, ny, L;
  size_t N;
  size_t off[8];   // per-level temporaries: off[l] for level l (1 <= l < L)
};

__device__ __host__ inline size_t lvl_size(const SaraGeom& g, int l) { return g.N >> (2 * l); }

enum { A_PLAIN = 0, A_DUAL = 1 };

// The tile (x, y) and basis (z) of this workgroup.  Consecutive workgroups
// go round-robin to the XCDs; the tiles are handed out so that each XCD
// takes a contiguous band of them instead, and neighbouring tiles, whose
// staged windows overlap, meet in one L2.
struct TileId {
  int x, y, z;
};
__device__ inline TileId sara_tile() {
  const int gx = gridDim.x, gy = gridDim.y, total = gx * gy * int(gridDim.z);
  int lin = int(blockIdx.x) + gx * (int(blockIdx.y) + gy * int(blockIdx.z));
  if (total % MAX_XCD == 0) lin = xcd_remap(lin, total);
  return TileId{lin % gx, (lin / gx) % gy, lin / (gx * gy)};
}

// Filters of db-Q: 2Q taps each, low-pass h and high-pass g, in registers
// (the addresses are wave-uniform, so the compiler uses scalar loads).
template <int Q>
__device__ __forceinline__ void load_filt(const float* __restrict__ filt, float (&h)[2 * Q], float (&g)[2 * Q]) {
  const float* b = filt + (Q - 1) * 2 * FILT_STRIDE;
#pragma unroll
  for (int n = 0; n < 2 * Q; ++n) {
    h[n] = b[n];
    g[n] = b[FILT_STRIDE + n];
  }
}

// One analysis level of basis db-Q on one output tile: stage the periodic
// input region, filter the columns (axis 0), then the rows (axis 1).
// a[k] = sum_n h[n] s[(2k + n) mod L], d[k] likewise with g.
template <int Q, int MODE>
__device__ void dwt_tile(const float* __restrict__ src, int sstride, float scale, int hh, int ww, int k0y,
                         int k0x, int toy, int tox, const float* __restrict__ filt, float* s_in, float* s_lo,
                         float* s_hi, float* __restrict__ ub, const float* __restrict__ wb, int nx, int oh,
                         int ow, float* __restrict__ llout, float alpha, float lambda) {
  constexpr int TAPS = 2 * Q;
  float h[TAPS], g[TAPS];
  load_filt<Q>(filt, h, g);
  // This thread's output position (tiles hold at most blockDim.x outputs):
  // its weights and, in the dual mode, its u values are loaded before the
  // input is staged, so both loads are in flight together.
  const bool mine = int(threadIdx.x) < toy * tox;
  const int k = mine ? int(threadIdx.x) / tox : 0, m = mine ? int(threadIdx.x) - k * tox : 0;
  const int r = k0y + k, c = k0x + m;
  const size_t pos[4] = {size_t(r) * nx + (ow + c), size_t(oh + r) * nx + c, size_t(oh + r) * nx + (ow + c),
                         size_t(r) * nx + c};
  const int nout = llout ? 3 : 4;
  float wv[4] = {1.f, 1.f, 1.f, 1.f}, uo[4] = {0.f, 0.f, 0.f, 0.f};
  if (mine) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s < nout) {
        if (wb) wv[s] = wb[pos[s]];
        if (MODE == A_DUAL) uo[s] = ub[pos[s]];
      }
    }
  }
  const int IR = 2 * toy + TAPS - 2, IC = 2 * tox + TAPS - 2;
  const int ty = threadIdx.x >> 6, tx = threadIdx.x & 63, nty = blockDim.x >> 6;
  // staging: all of the thread's loads are issued before its LDS stores
  constexpr int SPT = (SIN + 3) / 4;   // rows per thread with 4 row groups
  float sv[SPT];
  const int cx = (2 * k0x + tx) & (ww - 1);
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int a = ty + k * nty;
    if (a < IR && tx < IC) sv[k] = src[size_t((2 * k0y + a) & (hh - 1)) * sstride + cx];
  }
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int a = ty + k * nty;
    if (a < IR && tx < IC) s_in[a * SIN + tx] = sv[k] * scale;
  }
  __syncthreads();
  for (int kk = ty; kk < toy; kk += nty) {   // columns
    if (tx < IC) {
      const float* col = s_in + 2 * kk * SIN + tx;
      float lo = 0.f, hi = 0.f;
#pragma unroll
      for (int n = 0; n < TAPS; ++n) {
        const float v = col[n * SIN];
        lo = fmaf(h[n], v, lo);
        hi = fmaf(g[n], v, hi);
      }
      s_lo[kk * SIN + tx] = lo;
      s_hi[kk * SIN + tx] = hi;
    }
  }
  __syncthreads();
  if (!mine) return;
  const float* lrow = s_lo + k * SIN + 2 * m;   // rows
  const float* hrow = s_hi + k * SIN + 2 * m;
  float ll = 0.f, lh = 0.f, hl = 0.f, hhv = 0.f;
#pragma unroll
  for (int n = 0; n < TAPS; ++n) {
    const float a = lrow[n], d = hrow[n];
    ll = fmaf(h[n], a, ll);
    lh = fmaf(g[n], a, lh);
    hl = fmaf(h[n], d, hl);
    hhv = fmaf(g[n], d, hhv);
  }
  const float cv[4] = {lh, hl, hhv, ll};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (s >= nout) break;
    const float cs = cv[s] * wv[s];
    if (MODE == A_PLAIN) {
      ub[pos[s]] = cs;
    } else {
      // the sparsity dual update of Algorithm 3 on the coefficient of Psi^H x~
      const float cl = fminf(fmaxf(uo[s] + cs, -alpha), alpha);
      ub[pos[s]] = uo[s] + lambda * (cl - uo[s]);
    }
  }
  if (llout) llout[size_t(r) * ow + c] = ll;
}

static_assert(AT * AT <= 256, "an analysis tile must fit one output per thread of 256");

// Level l of the 8 wavelet bases (tile z = basis - 1); at level 1 the
// Dirac basis is z = 8.  `active` (dual mode, may be NULL) masks
// the bases updated this iteration.  Level 1 reads the image scaled by 1/3,
// deeper levels the low-pass band of the previous level.
template <int MODE>
__global__ __launch_bounds__(256) void k_dwt(const float* __restrict__ x, float* __restrict__ tmp,
                                             float* __restrict__ out, const float* __restrict__ filt,
                                             const float* __restrict__ W, SaraGeom g, int l, float alpha,
                                             float lambda, const uint8_t* __restrict__ active) {
  __shared__ float s_in[SIN * SIN];
  __shared__ float s_lo[AT * SIN];
  __shared__ float s_hi[AT * SIN];
  const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
  const int oh = hh >> 1, ow = ww >> 1;
  const int toy = min(AT, oh), tox = min(AT, ow);
  const TileId tl = sara_tile();
  const int k0y = tl.y * toy, k0x = tl.x * tox;
  const int q = tl.z + 1;   // 1..8 wavelets, 9 = Dirac (level 1 only)
  const float third = 1.0f / 3.0f;
  // randomised updates (Algorithm 3 with a random set of bases): an inactive basis keeps
  // its u_i (basis index 0 is the Dirac basis)
  if (active && !active[q == 9 ? 0 : q]) return;
  if (q == 9) {
    // Dirac basis: coefficient x / 3 at every pixel of this tile's footprint
    // (at most 4 pixels per thread; all loads issued first)
    constexpr int DPT = 4 * AT * AT / 256;
    float xv[DPT], wv[DPT], uo[DPT];
    size_t Pv[DPT];
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int i = threadIdx.x + k * 256;
      Pv[k] = 0;
      if (i < 4 * toy * tox) {
        const int a = i / (2 * tox), b = i - a * (2 * tox);
        Pv[k] = size_t(2 * k0y + a) * g.nx + (2 * k0x + b);
        xv[k] = x[Pv[k]];
        wv[k] = W ? W[Pv[k]] : 1.0f;
        uo[k] = MODE == A_DUAL ? out[Pv[k]] : 0.f;
      }
    }
#pragma unroll
    for (int k = 0; k < DPT; ++k) {
      const int i = threadIdx.x + k * 256;
      if (i < 4 * toy * tox) {
        const float c = xv[k] * third * wv[k];
        if (MODE == A_PLAIN) {
          out[Pv[k]] = c;
        } else {
          const float cl = fminf(fmaxf(uo[k] + c, -alpha), alpha);
          out[Pv[k]] = uo[k] + lambda * (cl - uo[k]);
        }
      }
    }
    return;
  }
  const float* src = l == 1 ? x : tmp + g.off[l - 1] + size_t(q - 1) * lvl_size(g, l - 1);
  const int sstride = l == 1 ? g.nx : ww;
  const float scale = l == 1 ? third : 1.0f;
  float* ub = out + size_t(q) * g.N;
  const float* wb = W ? W + size_t(q) * g.N : nullptr;
  float* llout = l == g.L ? nullptr : tmp + g.off[l] + size_t(q - 1) * lvl_size(g, l);
#define PPD_DWT_CASE(Q)                                                                                     \
  case Q:                                                                                                   \
    dwt_tile<Q, MODE>(src, sstride, scale, hh, ww, k0y, k0x, toy, tox, filt, s_in, s_lo, s_hi, ub, wb, g.nx, \
                      oh, ow, llout, alpha, lambda);                                                        \
    break;
  switch (q) {
    PPD_DWT_CASE(1) PPD_DWT_CASE(2) PPD_DWT_CASE(3) PPD_DWT_CASE(4)
    PPD_DWT_CASE(5) PPD_DWT_CASE(6) PPD_DWT_CASE(7) PPD_DWT_CASE(8)
  }
#undef PPD_DWT_CASE
}

// Inverse of one level for basis db-Q: sub-bands (oh x ow) -> (hh x ww) on
// the output tile (y0, x0, tsy x tsx).  Transposing the analysis gives
// s[2j + e] = sum_t h[2t + e] a[j - t] + g[2t + e] d[j - t], e in {0, 1}, so
// each thread makes an even / odd output pair from the same Q coefficients.
// Rows (axis 1) first, then columns (axis 0).  sink(slot, r, c, v) receives
// the outputs; slot counts the thread's outputs in a fixed order.
// The low-pass band of a coefficient window taken from LDS instead of
// memory: window entry (a, b) of the tile is p[(a + offy) * stride + b + offx].
struct LLWin {
  const float* p = nullptr;
  int stride = 0, offy = 0, offx = 0;
};

template <int Q, typename Sink>
__device__ void idwt_tile(const float* __restrict__ llsrc, int llstride, const float* __restrict__ ucoef,
                          const float* __restrict__ wcoef, const float* __restrict__ llw, int nx, int hh,
                          int ww, int y0, int x0, int tsy, int tsx, const float* __restrict__ filt,
                          float* s_ll, float* s_lh, float* s_hl, float* s_hh, float* s_a, float* s_d,
                          Sink sink, const LLWin win = LLWin{}) {
  float h[2 * Q], g[2 * Q];
  load_filt<Q>(filt, h, g);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int oh = hh >> 1, ow = ww >> 1;
  const int hx = tsx >> 1, hy = tsy >> 1;
  const int KR = hy + Q, KC = hx + Q;
  const int krb = (y0 >> 1) - Q, kcb = (x0 >> 1) - Q;
  // staging: all of the thread's loads are issued before its LDS stores
  constexpr int IPT = (SK * SK + 255) / 256;
  float v4[IPT][4];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const int i = tid + k * nth;
    if (i < KR * KC) {
      const int a = i / KC, b = i - a * KC;
      const int r = (krb + a) & (oh - 1), c = (kcb + b) & (ow - 1);
      const size_t pll = size_t(r) * llstride + c;
      const size_t plh = size_t(r) * nx + (ow + c), phl = size_t(oh + r) * nx + c;
      const size_t phh = size_t(oh + r) * nx + (ow + c);
      v4[k][0] = win.p ? win.p[(a + win.offy) * win.stride + (b + win.offx)]
                       : llsrc[pll] * (llw ? llw[pll] : 1.0f);
      v4[k][1] = ucoef[plh] * (wcoef ? wcoef[plh] : 1.0f);
      v4[k][2] = ucoef[phl] * (wcoef ? wcoef[phl] : 1.0f);
      v4[k][3] = ucoef[phh] * (wcoef ? wcoef[phh] : 1.0f);
    }
  }
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const int i = tid + k * nth;
    if (i < KR * KC) {
      const int a = i / KC, b = i - a * KC;
      const int li = a * SK + b;
      s_ll[li] = v4[k][0];
      s_lh[li] = v4[k][1];
      s_hl[li] = v4[k][2];
      s_hh[li] = v4[k][3];
    }
  }
  __syncthreads();
  for (int i = tid; i < KR * hx; i += nth) {   // rows: A from (LL, LH), D from (HL, HH)
    const int kr = i / hx, j = i - kr * hx;
    const int base = kr * SK + j + Q;
    float a0 = 0.f, a1 = 0.f, d0 = 0.f, d1 = 0.f;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const float ll = s_ll[base - t], lh = s_lh[base - t], hl = s_hl[base - t], hv = s_hh[base - t];
      a0 = fmaf(h[2 * t], ll, fmaf(g[2 * t], lh, a0));
      a1 = fmaf(h[2 * t + 1], ll, fmaf(g[2 * t + 1], lh, a1));
      d0 = fmaf(h[2 * t], hl, fmaf(g[2 * t], hv, d0));
      d1 = fmaf(h[2 * t + 1], hl, fmaf(g[2 * t + 1], hv, d1));
    }
    s_a[kr * ST + 2 * j] = a0;
    s_a[kr * ST + 2 * j + 1] = a1;
    s_d[kr * ST + 2 * j] = d0;
    s_d[kr * ST + 2 * j + 1] = d1;
  }
  __syncthreads();
  int slot = 0;
  for (int i = tid; i < hy * tsx; i += nth, slot += 2) {   // columns: S from (A, D)
    const int j = i / tsx, m = i - j * tsx;
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const int lr = (j + Q - t) * ST + m;
      const float av = s_a[lr], dv = s_d[lr];
      s0 = fmaf(h[2 * t], av, fmaf(g[2 * t], dv, s0));
      s1 = fmaf(h[2 * t + 1], av, fmaf(g[2 * t + 1], dv, s1));
    }
    sink(slot, 2 * j, m, s0);
    sink(slot + 1, 2 * j + 1, m, s1);
  }
  __syncthreads();
}

#define PPD_IDWT_SWITCH(q, ...)                       \
  switch (q) {                                        \
    case 1: idwt_tile<1>(__VA_ARGS__); break;         \
    case 2: idwt_tile<2>(__VA_ARGS__); break;         \
    case 3: idwt_tile<3>(__VA_ARGS__); break;         \
    case 4: idwt_tile<4>(__VA_ARGS__); break;         \
    case 5: idwt_tile<5>(__VA_ARGS__); break;         \
    case 6: idwt_tile<6>(__VA_ARGS__); break;         \
    case 7: idwt_tile<7>(__VA_ARGS__); break;         \
    default: idwt_tile<8>(__VA_ARGS__); break;        \
  }

// Intermediate synthesis level l >= 2 (output = low-pass band of level l-1).
__global__ __launch_bounds__(256) void k_idwt(const float* __restrict__ u, float* __restrict__ rec,
                                              const float* __restrict__ filt, const float* __restrict__ W,
                                              SaraGeom g, int l) {
  __shared__ float s_ll[SK * SK], s_lh[SK * SK], s_hl[SK * SK], s_hh[SK * SK];
  __shared__ float s_a[SK * ST], s_d[SK * ST];
  const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
  const int tsy = min(ST, hh), tsx = min(ST, ww);
  const TileId tl = sara_tile();
  const int y0 = tl.y * tsy, x0 = tl.x * tsx;
  const int q = tl.z + 1;
  const float* ucoef = u + size_t(q) * g.N;
  const float* wcoef = W ? W + size_t(q) * g.N : nullptr;
  const float* llsrc;
  const float* llw = nullptr;
  int llstride = ww >> 1;
  if (l == g.L) {
    llsrc = ucoef;
    llw = wcoef;
    llstride = g.nx;
  } else {
    llsrc = rec + g.off[l] + size_t(q - 1) * lvl_size(g, l);
  }
  float* dst = rec + g.off[l - 1] + size_t(q - 1) * lvl_size(g, l - 1);
  auto sink = [&](int, int r, int c, float v) { dst[size_t(y0 + r) * ww + (x0 + c)] = v; };
  PPD_IDWT_SWITCH(q, llsrc, llstride, ucoef, wcoef, llw, g.nx, hh, ww, y0, x0, tsy, tsx, filt, s_ll, s_lh,
                  s_hl, s_hh, s_a, s_d, sink)
}

// The two coarsest synthesis levels L and L-1 (L >= 3) in one launch: a
// workgroup first rebuilds, from the level-L coefficients, the window of
// the level-(L-1) low-pass band its level-(L-1) tile reads (periodic, even
// aligned; neighbouring workgroups recompute the overlap), keeps it in LDS,
// then synthesises its tile of the level-(L-2) low-pass band.  One launch
// fewer on SARA's chain of dependent launches.
constexpr int WIN = ST / 2 + FILT_STRIDE / 2 + 2;   // LL window edge (outer window + alignment, even)

template <int Q>
__device__ void idwt2_body(const float* __restrict__ ucoef, const float* __restrict__ wcoef, float* dst,
                           const float* __restrict__ filt, int nx, int hh, int ww, int y0, int x0, int tsy,
                           int tsx, float* s_ll, float* s_lh, float* s_hl, float* s_hh, float* s_a, float* s_d,
                           float* s_win) {
  const int oh = hh >> 1, ow = ww >> 1;                      // level-(L-1) band = inner output
  const int wy0 = (y0 >> 1) - Q, wx0 = (x0 >> 1) - Q;        // outer coefficient window origin
  const int ya = wy0 - (wy0 & 1), xa = wx0 - (wx0 & 1);      // even-aligned inner tile origin
  const int offy = wy0 - ya, offx = wx0 - xa;
  const int ti_y = ((tsy >> 1) + Q + offy + 1) & ~1, ti_x = ((tsx >> 1) + Q + offx + 1) & ~1;
  auto sink_win = [&](int, int r, int c, float v) { s_win[r * WIN + c] = v; };
  // level L: its low-pass band and details are coefficients (in u, weighted)
  idwt_tile<Q>(ucoef, nx, ucoef, wcoef, wcoef, nx, oh, ow, ya, xa, ti_y, ti_x, filt, s_ll, s_lh, s_hl, s_hh,
               s_a, s_d, sink_win);
  auto sink = [&](int, int r, int c, float v) { dst[size_t(y0 + r) * ww + (x0 + c)] = v; };
  LLWin win;
  win.p = s_win;
  win.stride = WIN;
  win.offy = offy;
  win.offx = offx;
  idwt_tile<Q>(nullptr, 0, ucoef, wcoef, nullptr, nx, hh, ww, y0, x0, tsy, tsx, filt, s_ll, s_lh, s_hl, s_hh,
               s_a, s_d, sink, win);
}

__global__ __launch_bounds__(256) void k_idwt2(const float* __restrict__ u, float* __restrict__ rec,
                                               const float* __restrict__ filt, const float* __restrict__ W,
                                               SaraGeom g) {
  __shared__ float s_ll[SK * SK], s_lh[SK * SK], s_hl[SK * SK], s_hh[SK * SK];
  __shared__ float s_a[SK * ST], s_d[SK * ST];
  __shared__ float s_win[WIN * WIN];
  const int l = g.L - 1;                                      // outer level
  const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
  const int tsy = min(ST, hh), tsx = min(ST, ww);
  const TileId tl = sara_tile();
  const int y0 = tl.y * tsy, x0 = tl.x * tsx;
  const int q = tl.z + 1;
  const float* ucoef = u + size_t(q) * g.N;
  const float* wcoef = W ? W + size_t(q) * g.N : nullptr;
  float* dst = rec + g.off[l - 1] + size_t(q - 1) * lvl_size(g, l - 1);
  switch (q) {
    case 1: idwt2_body<1>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
    case 2: idwt2_body<2>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
    case 3: idwt2_body<3>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
    case 4: idwt2_body<4>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
    case 5: idwt2_body<5>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
    case 6: idwt2_body<6>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
    case 7: idwt2_body<7>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
    default: idwt2_body<8>(ucoef, wcoef, dst, filt, g.nx, hh, ww, y0, x0, tsy, tsx, s_ll, s_lh, s_hl, s_hh, s_a, s_d, s_win); break;
  }
}
static_assert(ST / 2 + FILT_STRIDE / 2 + 1 <= WIN && WIN <= ST, "the LL window fits an inner tile");
static_assert(WIN / 2 + FILT_STRIDE / 2 <= SK, "the inner coefficient window fits the staging");

// Level 1 for all 8 wavelet bases, plus the Dirac part, times 1/3, on a
// STF x STF output tile.  The coefficient windows of all 8 bases are loaded
// in one pass (one round of global loads, into registers), then staged in
// LDS FPARTS bases at a time: the row passes of a part, then its column
// passes, which each thread sums over the bases in registers in basis
// order.  Parts keep the workgroup's LDS small, which leaves room on each
// compute unit for the concurrent data-path launches.
#ifndef PPD_FINAL_PARTS
#define PPD_FINAL_PARTS 2
#endif
constexpr int FPARTS = PPD_FINAL_PARTS;
constexpr int FB = 8 / FPARTS;                       // bases per part
static_assert(FB * FPARTS == 8, "the parts split the 8 bases evenly");
constexpr int FINAL_THREADS = 128;
constexpr int FH = STF / 2;                          // coefficients per tile side and band
constexpr int FKS = FH + FILT_STRIDE / 2;            // staged row stride (FH + max Q)
constexpr int FELEM = 8 * FH * FH + 2 * FH * 36 + 204;   // sum over Q of (FH + Q)^2
constexpr int FEPT = (FELEM + FINAL_THREADS - 1) / FINAL_THREADS;
constexpr int FROWS = FB * FH + FB * (17 - FB) / 2;  // rows of the last (largest) part: sum of FH + Q over it
constexpr int FPART = FROWS * FKS;                   // staging index offset of one part
static_assert(FH * STF == FINAL_THREADS, "one column pair per thread");

// first staged row of basis q within its part (each part from row 0)
__device__ __forceinline__ int final_row0(int q) {
  const int q0 = (q - 1) / FB * FB + 1;
  return (q - q0) * FH + ((q - 1) * q - (q0 - 1) * q0) / 2;
}
__device__ __forceinline__ int final_elem0(int q) {
  int e = 0;
  for (int p = 1; p < q; ++p) e += (FH + p) * (FH + p);
  return e;
}

template <int Q>
__device__ __forceinline__ void final_rows(const float* __restrict__ filt, const float* s_c, float* s_a,
                                           float* s_d) {
  float h[2 * Q], g[2 * Q];
  load_filt<Q>(filt, h, g);
  constexpr int KR = FH + Q;
  const int r0 = final_row0(Q);
  const float* s_ll = s_c;
  const float* s_lh = s_c + FROWS * FKS;
  const float* s_hl = s_c + 2 * FROWS * FKS;
  const float* s_hh = s_c + 3 * FROWS * FKS;
  for (int i = threadIdx.x; i < KR * FH; i += blockDim.x) {
    const int kr = i / FH, j = i - kr * FH;
    const int base = (r0 + kr) * FKS + j + Q;
    float a0 = 0.f, a1 = 0.f, d0 = 0.f, d1 = 0.f;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const float ll = s_ll[base - t], lh = s_lh[base - t], hl = s_hl[base - t], hv = s_hh[base - t];
      a0 = fmaf(h[2 * t], ll, fmaf(g[2 * t], lh, a0));
      a1 = fmaf(h[2 * t + 1], ll, fmaf(g[2 * t + 1], lh, a1));
      d0 = fmaf(h[2 * t], hl, fmaf(g[2 * t], hv, d0));
      d1 = fmaf(h[2 * t + 1], hl, fmaf(g[2 * t + 1], hv, d1));
    }
    s_a[(r0 + kr) * STF + 2 * j] = a0;
    s_a[(r0 + kr) * STF + 2 * j + 1] = a1;
    s_d[(r0 + kr) * STF + 2 * j] = d0;
    s_d[(r0 + kr) * STF + 2 * j + 1] = d1;
  }
}

template <int Q>
__device__ __forceinline__ void final_cols(const float* __restrict__ filt, const float* s_a, const float* s_d,
                                           int j, int m, float& o0, float& o1) {
  float h[2 * Q], g[2 * Q];
  load_filt<Q>(filt, h, g);
  const int r0 = final_row0(Q);
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    const int lr = (r0 + j + Q - t) * STF + m;
    const float av = s_a[lr], dv = s_d[lr];
    o0 = fmaf(h[2 * t], av, fmaf(g[2 * t], dv, o0));
    o1 = fmaf(h[2 * t + 1], av, fmaf(g[2 * t + 1], dv, o1));
  }
}

template <int Q, int QE>
__device__ __forceinline__ void final_rows_range(const float* __restrict__ filt, const float* s_c, float* s_a,
                                                 float* s_d) {
  final_rows<Q>(filt, s_c, s_a, s_d);
  if constexpr (Q < QE) final_rows_range<Q + 1, QE>(filt, s_c, s_a, s_d);
}

template <int Q, int QE>
__device__ __forceinline__ void final_cols_range(const float* __restrict__ filt, const float* s_a,
                                                 const float* s_d, int j, int m, float& o0, float& o1) {
  final_cols<Q>(filt, s_a, s_d, j, m, o0, o1);
  if constexpr (Q < QE) final_cols_range<Q + 1, QE>(filt, s_a, s_d, j, m, o0, o1);
}

// Part PART of the bases: stage its windows (s_c was last read by the
// previous part's row passes, before the barrier ahead of its column
// passes), then its row and column passes.
template <int PART>
__device__ __forceinline__ void final_part(const float* __restrict__ filt, float* s_c, float* s_a, float* s_d,
                                           const float (&vals)[FEPT][4], const int (&at)[FEPT], int j, int m,
                                           float& o0, float& o1) {
#pragma unroll
  for (int k = 0; k < FEPT; ++k) {
    if (at[k] >= PART * FPART && at[k] < (PART + 1) * FPART) {
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) s_c[c4 * FPART + at[k] - PART * FPART] = vals[k][c4];
    }
  }
  __syncthreads();
  final_rows_range<PART * FB + 1, PART * FB + FB>(filt, s_c, s_a, s_d);
  __syncthreads();
  final_cols_range<PART * FB + 1, PART * FB + FB>(filt, s_a, s_d, j, m, o0, o1);
  if constexpr (PART + 1 < FPARTS) final_part<PART + 1>(filt, s_c, s_a, s_d, vals, at, j, m, o0, o1);
}

__global__ __launch_bounds__(FINAL_THREADS) void k_idwt_final(const float* __restrict__ u,
                                                              const float* __restrict__ rec,
                                                              const float* __restrict__ filt,
                                                              const float* __restrict__ W, SaraGeom g,
                                                              float* __restrict__ out) {
  __shared__ float s_c[4 * FPART];   // one part's LL, LH, HL, HH windows
  __shared__ float s_a[FROWS * STF], s_d[FROWS * STF];
  const int nx = g.nx, ww = g.nx, hh = g.ny;
  const int oh = hh >> 1, ow = ww >> 1;
  const TileId tl = sara_tile();
  const int y0 = tl.y * STF, x0 = tl.x * STF;
  const int tid = threadIdx.x;
  // stage: element e of the flattened (basis, row, column) windows
  float vals[FEPT][4];
  int at[FEPT];
#pragma unroll
  for (int k = 0; k < FEPT; ++k) {
    const int e = tid + k * FINAL_THREADS;
    at[k] = -1;
    if (e < FELEM) {
      int q = 1;
#pragma unroll
      for (int p = 2; p <= 8; ++p)
        if (e >= final_elem0(p)) q = p;
      const int KC = FH + q;
      const int le = e - final_elem0(q);
      const int a = le / KC, b = le - a * KC;
      const int r = ((y0 >> 1) - q + a) & (oh - 1), c = ((x0 >> 1) - q + b) & (ow - 1);
      const float* ucoef = u + size_t(q) * g.N;
      const float* wcoef = W ? W + size_t(q) * g.N : nullptr;
      const size_t plh = size_t(r) * nx + (ow + c), phl = size_t(oh + r) * nx + c;
      const size_t phh = size_t(oh + r) * nx + (ow + c);
      if (g.L == 1) {
        const size_t pll = size_t(r) * nx + c;
        vals[k][0] = ucoef[pll] * (wcoef ? wcoef[pll] : 1.0f);
      } else {
        vals[k][0] = rec[g.off[1] + size_t(q - 1) * lvl_size(g, 1) + size_t(r) * ow + c];
      }
      vals[k][1] = ucoef[plh] * (wcoef ? wcoef[plh] : 1.0f);
      vals[k][2] = ucoef[phl] * (wcoef ? wcoef[phl] : 1.0f);
      vals[k][3] = ucoef[phh] * (wcoef ? wcoef[phh] : 1.0f);
      at[k] = (final_row0(q) + a) * FKS + b + (q - 1) / FB * FPART;
    }
  }
  const int j = tid / STF, m = tid - j * STF;
  const size_t P0 = size_t(y0 + 2 * j) * nx + (x0 + m), P1 = P0 + nx;
  const float dirac0 = u[P0] * (W ? W[P0] : 1.0f), dirac1 = u[P1] * (W ? W[P1] : 1.0f);
  float o0 = 0.f, o1 = 0.f;
  final_part<0>(filt, s_c, s_a, s_d, vals, at, j, m, o0, o1);
  const float third = 1.0f / 3.0f;
  out[P0] = (o0 + dirac0) * third;
  out[P1] = (o1 + dirac1) * third;
}
#undef PPD_IDWT_SWITCH

// Algorithm 1 weights (eq. reweighting): W = omega / (omega + |c|), in
// place over the analysis coefficients c.
__global__ void k_reweight(float* __restrict__ w, size_t n, float omega) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    w[i] = omega / (omega + fabsf(w[i]));
}

SaraGeom geom(const ppd_plan* p) {
  SaraGeom g{};
  g.nx = p->nx;
  g.ny = p->ny;
  g.L = p->levels;
  g.N = size_t(p->nx) * p->ny;
  size_t o = 0;
  for (int l = 1; l < g.L; ++l) {
    g.off[l] = o;
    o += 8 * (g.N >> (2 * l));
  }
  return g;
}

int analysis_launch(ppd_plan* p, const float* x, float* out, const float* W, bool dual, float alpha,
                    float lambda, const uint8_t* active) {
  const SaraGeom g = geom(p);
  for (int l = 1; l <= g.L; ++l) {
    const int oh = (g.ny >> l), ow = (g.nx >> l);
    const int toy = std::min(AT, oh), tox = std::min(AT, ow);
    dim3 grid(ow / tox, oh / toy, l == 1 ? 9 : 8);
    int slot;
    PPD_TRY(timer_begin(p, KK_DWT, &slot));
    if (dual)
      hipLaunchKernelGGL(k_dwt<A_DUAL>, grid, dim3(256), 0, p->stream, x, p->sara_ll, out, p->filt, W, g, l,
                         alpha, lambda, active);
    else
      hipLaunchKernelGGL(k_dwt<A_PLAIN>, grid, dim3(256), 0, p->stream, x, p->sara_ll, out, p->filt, W, g, l,
                         alpha, lambda, nullptr);
    PPD_HIP(hipGetLastError());
    PPD_TRY(timer_end(p, slot));
  }
  return PPD_OK;
}

}  // namespace

int sara_analysis(ppd_plan* p, const float* x, float* coef, const float* W) {
  return analysis_launch(p, x, coef, W, false, 0.f, 0.f, nullptr);
}

int sara_dual(ppd_plan* p, const float* x, float* u, float alpha, float lambda, const float* W,
              const uint8_t* active) {
  return analysis_launch(p, x, u, W, true, alpha, lambda, active);
}

int sara_synthesis(ppd_plan* p, const float* u, float* out, const float* W) {
  const SaraGeom g = geom(p);
  int top = g.L;
  if (g.L >= 3) {
    // levels L and L-1 in one launch
    const int l = g.L - 1;
    const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
    const int tsy = std::min(ST, hh), tsx = std::min(ST, ww);
    int slot;
    PPD_TRY(timer_begin(p, KK_IDWT, &slot));
    hipLaunchKernelGGL(k_idwt2, dim3(ww / tsx, hh / tsy, 8), dim3(256), 0, p->stream, u, p->sara_rec, p->filt,
                       W, g);
    PPD_HIP(hipGetLastError());
    PPD_TRY(timer_end(p, slot));
    top = g.L - 2;
  }
  for (int l = top; l >= 2; --l) {
    const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
    const int tsy = std::min(ST, hh), tsx = std::min(ST, ww);
    int slot;
    PPD_TRY(timer_begin(p, KK_IDWT, &slot));
    hipLaunchKernelGGL(k_idwt, dim3(ww / tsx, hh / tsy, 8), dim3(256), 0, p->stream, u, p->sara_rec, p->filt,
                       W, g, l);
    PPD_HIP(hipGetLastError());
    PPD_TRY(timer_end(p, slot));
  }
  int slot;
  PPD_TRY(timer_begin(p, KK_IDWT, &slot));
  hipLaunchKernelGGL(k_idwt_final, dim3(g.nx / STF, g.ny / STF), dim3(FINAL_THREADS), 0, p->stream, u, p->sara_rec,
                     p->filt, W, g, out);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

}  // namespace ppd

using namespace ppd;

extern "C" int ppd_sara_w(ppd_plan* p, int op, const float* in, float* out, float* u, const float* W,
                          float alpha, float lambda) {
  if (!p || !in || !out) return fail(PPD_EINVAL, "ppd_sara: NULL argument");
  switch (op) {
    case PPD_SARA_ANALYSIS:
      return sara_analysis(p, in, out, W);
    case PPD_SARA_SYNTHESIS:
      return sara_synthesis(p, in, out, W);
    case PPD_SARA_DUAL:
      if (!u) return fail(PPD_EINVAL, "ppd_sara: dual mode needs u_inout");
      if (!(alpha >= 0.0f)) return fail(PPD_EINVAL, "ppd_sara: alpha must be >= 0");
      PPD_TRY(sara_dual(p, in, u, alpha, lambda, W));
      return sara_synthesis(p, u, out, W);
    default:
      return fail(PPD_EINVAL, "ppd_sara: unknown op");
  }
}

extern "C" int ppd_sara(ppd_plan* p, int op, const float* in, float* out, float* u, float alpha,
                        float lambda) {
  return ppd_sara_w(p, op, in, out, u, nullptr, alpha, lambda);
}

extern "C" int ppd_reweight(ppd_plan* p, const float* x, float omega, float* W) {
  if (!p || !x || !W) return fail(PPD_EINVAL, "ppd_reweight: NULL argument");
  if (!(omega > 0.0f) || !std::isfinite(omega)) return fail(PPD_EINVAL, "ppd_reweight: omega must be > 0");
  PPD_TRY(sara_analysis(p, x, W, nullptr));
  const size_t n = size_t(N_BASES) * p->nx * p->ny;
  int slot;
  PPD_TRY(timer_begin(p, KK_MISC, &slot));
  hipLaunchKernelGGL(k_reweight, dim3(int(std::min<size_t>((n + 255) / 256, 4096))), dim3(256), 0, p->stream, W,
                     n, omega);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}
