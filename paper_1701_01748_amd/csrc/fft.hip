// Oversampled 2D FFT of the measurement operator (Sec. 2: F Z and
// Z^H F^H), complex float32, entirely in LDS.
//
// Forward: each image row is deapodised and zero-padded into its wrapped
// position of a length-Kx sequence and transformed (rows that are all zero
// in the 2x oversampled grid are never touched), then every grid column is
// transformed from its ny non-zero entries.  Adjoint: full column inverse
// transforms keep only the ny rows the image needs, then row inverse
// transforms keep the nx wanted entries, undo the deapodisation and keep the
// real part -- optionally fused with the primal update of Algorithm 3.
//
// In-LDS transform: iterative decimation in time on bit-reversed input,
// two radix-2 stages per LDS round trip (a radix-4 butterfly), one leading
// radix-2 stage when log2 L is odd.  LDS index i is padded by i/32 (+1 per
// sequence) against bank conflicts.  Twiddles exp(-2 pi i k / L), k < L/2,
// are computed in float64 on the host and staged in LDS.
#include "ppd_internal.h"

namespace ppd {
namespace {

// Elements per thread of a staging pass: every launch below has at most
// 4 * blockDim.x of them (checked on the host).
constexpr int FFT_PER = 4;
// Columns per workgroup of the column passes (at most 4096 / L).
#ifndef PPD_FFT_COLS
#define PPD_FFT_COLS 16
#endif

__device__ __forceinline__ int padi(int i) { return i + (i >> 5); }
__host__ __device__ inline int padded_len(int L) { return L + (L >> 5) + 1; }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ int bitrev(int n, int log2L) { return int(__brev(unsigned(n)) >> (32 - log2L)); }

template <bool INV>
__device__ void lds_fft(float2* s, int log2L, int nseq, int sstride, const float2* tw) {
  const int L = 1 << log2L;
  const int tid = threadIdx.x, nth = blockDim.x;
  int log2h = 0;
  if (log2L & 1) {
    const int half = L >> 1;
    for (int g = tid; g < nseq * half; g += nth) {
      const int sq = g >> (log2L - 1), k = g & (half - 1);
      float2* b = s + sq * sstride;
      const int i0 = padi(2 * k), i1 = padi(2 * k + 1);
      const float2 a = b[i0], c = b[i1];
      b[i0] = cadd(a, c);
      b[i1] = csub(a, c);
    }
    log2h = 1;
    __syncthreads();
  }
  for (; log2h < log2L; log2h += 2) {
    const int h = 1 << log2h;
    const int quarter = L >> 2;
    for (int g = tid; g < nseq * quarter; g += nth) {
      const int sq = g >> (log2L - 2), r = g & (quarter - 1);
      const int j = r & (h - 1), blk = r >> log2h;
      const int base = (blk << (log2h + 2)) + j;
      float2* b = s + sq * sstride;
      const int i0 = padi(base), i1 = padi(base + h), i2 = padi(base + 2 * h), i3 = padi(base + 3 * h);
      const float2 a0 = b[i0], a1 = b[i1], a2 = b[i2], a3 = b[i3];
      float2 w1 = tw[j << (log2L - log2h - 1)];   // W_{2h}^j
      float2 w2 = tw[j << (log2L - log2h - 2)];   // W_{4h}^j
      if (INV) {
        w1.y = -w1.y;
        w2.y = -w2.y;
      }
      const float2 t1 = cmul(w1, a1), t3 = cmul(w1, a3);
      const float2 b0 = cadd(a0, t1), b1 = csub(a0, t1), b2 = cadd(a2, t3), b3 = csub(a2, t3);
      const float2 u2 = cmul(w2, b2);
      float2 u3 = cmul(w2, b3);   // times W_{4h}^h = -i (forward) or +i (inverse)
      u3 = INV ? make_float2(-u3.y, u3.x) : make_float2(u3.y, -u3.x);
      b[i0] = cadd(b0, u2);
      b[i2] = csub(b0, u2);
      b[i1] = cadd(b1, u3);
      b[i3] = csub(b1, u3);
    }
    __syncthreads();
  }
}

// Forward rows: image rows r0 .. r0+rpb-1 -> half rows (length Kx).
__global__ void k_fft_rows_fwd(const float* __restrict__ x, const float* __restrict__ dpx,
                               const float* __restrict__ dpy, const float2* __restrict__ tw,
                               int nx, int log2L, int rpb, float2* __restrict__ half) {
  extern __shared__ float2 sm[];
  const int L = 1 << log2L, Lp = padded_len(L);
  float2* tws = sm + rpb * Lp;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int r0 = blockIdx.x * rpb;
  // all global loads of the thread are issued before the first LDS store
  float2 twv[FFT_PER];
  float xv[FFT_PER];
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) twv[k] = tw[i];
    if (i < rpb * nx) {
      const int q = i / nx, c = i - q * nx, r = r0 + q;
      xv[k] = x[size_t(r) * nx + c] * dpx[c] * dpy[r];
    }
  }
  for (int i = tid; i < rpb * Lp; i += nth) sm[i] = make_float2(0.f, 0.f);
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) tws[i] = twv[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < rpb * nx) {
      const int q = i / nx, c = i - q * nx;
      const int n = (c - (nx >> 1)) & (L - 1);
      sm[q * Lp + padi(bitrev(n, log2L))] = make_float2(xv[k], 0.f);
    }
  }
  __syncthreads();
  lds_fft<false>(sm, log2L, rpb, Lp, tws);
  for (int i = tid; i < rpb * L; i += nth) {
    const int q = i >> log2L, k = i & (L - 1);
    half[size_t(r0 + q) * L + k] = sm[q * Lp + padi(k)];
  }
}

// Forward columns: C grid columns from their ny non-zero rows -> grid.
__global__ void k_fft_cols_fwd(const float2* __restrict__ half, const float2* __restrict__ tw,
                               int ny, int Kx, int log2L, int C, int ngroups,
                               float2* __restrict__ grid) {
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  if (grp >= ngroups) return;
  extern __shared__ float2 sm[];
  const int L = 1 << log2L, Lp = padded_len(L);
  float2* tws = sm + C * Lp;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int c0 = grp * C;
  float2 twv[FFT_PER], hv[FFT_PER];
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) twv[k] = tw[i];
    if (i < ny * C) {
      const int r = i / C, cc = i - r * C;
      hv[k] = half[size_t(r) * Kx + c0 + cc];
    }
  }
  for (int i = tid; i < C * Lp; i += nth) sm[i] = make_float2(0.f, 0.f);
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) tws[i] = twv[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < ny * C) {
      const int r = i / C, cc = i - r * C;
      const int g = (r - (ny >> 1)) & (L - 1);
      sm[cc * Lp + padi(bitrev(g, log2L))] = hv[k];
    }
  }
  __syncthreads();
  lds_fft<false>(sm, log2L, C, Lp, tws);
  for (int i = tid; i < L * C; i += nth) {
    const int g = i / C, cc = i - g * C;
    grid[size_t(g) * Kx + c0 + cc] = sm[cc * Lp + padi(g)];
  }
}

// Inverse columns: full column transforms of the accumulated grid, keeping
// only the ny rows that map to image rows.
__global__ void k_fft_cols_inv(const float2* __restrict__ grid, const float2* __restrict__ tw,
                               int ny, int Kx, int log2L, int C, int ngroups,
                               float2* __restrict__ half) {
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  if (grp >= ngroups) return;
  extern __shared__ float2 sm[];
  const int L = 1 << log2L, Lp = padded_len(L);
  float2* tws = sm + C * Lp;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int c0 = grp * C;
  float2 twv[FFT_PER], gv[FFT_PER];
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) twv[k] = tw[i];
    if (i < L * C) {
      const int g = i / C, cc = i - g * C;
      gv[k] = grid[size_t(g) * Kx + c0 + cc];
    }
  }
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) tws[i] = twv[k];
    if (i < L * C) {
      const int g = i / C, cc = i - g * C;
      sm[cc * Lp + padi(bitrev(g, log2L))] = gv[k];
    }
  }
  __syncthreads();
  lds_fft<true>(sm, log2L, C, Lp, tws);
  for (int i = tid; i < ny * C; i += nth) {
    const int r = i / C, cc = i - r * C;
    const int g = (r - (ny >> 1)) & (L - 1);
    half[size_t(r) * Kx + c0 + cc] = sm[cc * Lp + padi(g)];
  }
}

__device__ inline double block_sum(double v, double* red) {
  // wave reduction then across waves through LDS (red: >= 16 doubles)
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// Inverse rows: half rows -> image rows.  PRIMAL fuses the primal update of
// Algorithm 3 (gradient step, projection onto the positive orthant,
// relaxation and the extrapolated iterate) and the FP64 statistics partials
// of the new iterate; NEXT also runs
// the forward row pass of the new x~ (the first transform of the next
// iteration's F Z x~) on the rows just updated, into half_next.
template <bool PRIMAL, bool NEXT>
__global__ void k_fft_rows_inv(const float2* __restrict__ half, const float2* __restrict__ tw,
                               const float* __restrict__ dpx, const float* __restrict__ dpy,
                               int nx, int log2L, int rpb, float* __restrict__ x,
                               float* __restrict__ xt, const float* __restrict__ ut,
                               const float* __restrict__ x_true, double tau, double eta,
                               double zeta, double lambda, double* __restrict__ part,
                               float2* __restrict__ half_next) {
  static_assert(PRIMAL || !NEXT, "the next forward pass needs the primal update");
  extern __shared__ float2 sm[];
  __shared__ double red[16];
  const int L = 1 << log2L, Lp = padded_len(L);
  float2* tws = sm + rpb * Lp;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int r0 = blockIdx.x * rpb;
  float2 twv[FFT_PER], hv[FFT_PER];
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) twv[k] = tw[i];
    if (i < rpb * L) hv[k] = half[size_t(r0 + (i >> log2L)) * L + (i & (L - 1))];
  }
#pragma unroll
  for (int k = 0; k < FFT_PER; ++k) {
    const int i = tid + k * nth;
    if (i < (L >> 1)) tws[i] = twv[k];
    if (i < rpb * L) sm[(i >> log2L) * Lp + padi(bitrev(i & (L - 1), log2L))] = hv[k];
  }
  __syncthreads();
  lds_fft<true>(sm, log2L, rpb, Lp, tws);
  double dx2 = 0.0, xx = 0.0, ee = 0.0, tt = 0.0;
  // rpb * nx <= 2 * nth (the staging capacity check on the host)
  float xtn[FFT_PER / 2];
#pragma unroll
  for (int k = 0; k < FFT_PER / 2; ++k) {
    const int i = tid + k * nth;
    if (i >= rpb * nx) break;
    const int q = i / nx, c = i - q * nx, r = r0 + q;
    const int n = (c - (nx >> 1)) & (L - 1);
    const float val = sm[q * Lp + padi(n)].x * dpx[c] * dpy[r];
    const size_t idx = size_t(r) * nx + c;
    if (!PRIMAL) {
      x[idx] = val;
    } else {
      const double xo = x[idx];
      double xb = xo - tau * (eta * double(val) + zeta * double(ut[idx]));   // primal step, then P_C
      xb = xb > 0.0 ? xb : 0.0;
      const double xn = xo + lambda * (xb - xo);                              // relaxation
      const float xnf = float(xn);
      x[idx] = xnf;
      const float xtf = float(2.0 * xb - xo);                                 // x~ = 2 xbar - x
      xt[idx] = xtf;
      if (NEXT) xtn[k] = xtf;
      const double dn = double(xnf) - xo;
      dx2 += dn * dn;
      xx += double(xnf) * double(xnf);
      if (part && x_true) {
        const double tv = x_true[idx];
        ee += (tv - double(xnf)) * (tv - double(xnf));
        tt += tv * tv;
      }
    }
  }
  if (PRIMAL && part) {   // statistics partials only when the call reads them (uniform branch)
    dx2 = block_sum(dx2, red);
    xx = block_sum(xx, red);
    ee = block_sum(ee, red);
    tt = block_sum(tt, red);
    if (tid == 0) {
      part[4 * blockIdx.x + 0] = dx2;
      part[4 * blockIdx.x + 1] = xx;
      part[4 * blockIdx.x + 2] = ee;
      part[4 * blockIdx.x + 3] = tt;
    }
  }
  if (NEXT) {
    // the same deapodisation, zero padding and wrapped placement as
    // k_fft_rows_fwd, from the x~ values just stored
    __syncthreads();
    for (int i = tid; i < rpb * Lp; i += nth) sm[i] = make_float2(0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < FFT_PER / 2; ++k) {
      const int i = tid + k * nth;
      if (i >= rpb * nx) break;
      const int q = i / nx, c = i - q * nx, r = r0 + q;
      const int n = (c - (nx >> 1)) & (L - 1);
      sm[q * Lp + padi(bitrev(n, log2L))] = make_float2(xtn[k] * dpx[c] * dpy[r], 0.f);
    }
    __syncthreads();
    lds_fft<false>(sm, log2L, rpb, Lp, tws);
    for (int i = tid; i < rpb * L; i += nth) {
      const int q = i >> log2L, k = i & (L - 1);
      half_next[size_t(r0 + q) * L + k] = sm[q * Lp + padi(k)];
    }
  }
}

struct RowCfg { int rpb, threads, blocks; size_t lds; bool ok; };
struct ColCfg { int C, threads, ngroups, blocks; size_t lds; bool ok; };

RowCfg row_cfg(int L, int rows) {
  RowCfg c;
  c.rpb = 1;
  while (c.rpb * L < 1024 && c.rpb * 2 <= rows) c.rpb *= 2;
  c.threads = std::min(1024, std::max(64, c.rpb * L / 4));
  c.blocks = rows / c.rpb;
  c.lds = (size_t(c.rpb) * padded_len(L) + L / 2) * sizeof(float2);
  c.ok = c.rpb * L <= FFT_PER * c.threads && L / 2 <= FFT_PER * c.threads;
  return c;
}

ColCfg col_cfg(int L, int Kx) {
  ColCfg c;
  c.C = std::max(1, std::min(PPD_FFT_COLS, 4096 / L));
  c.C = std::min(c.C, Kx);
  c.threads = std::min(1024, std::max(64, c.C * L / 4));
  c.ngroups = Kx / c.C;
  c.blocks = ((c.ngroups + MAX_XCD - 1) / MAX_XCD) * MAX_XCD;
  c.lds = (size_t(c.C) * padded_len(L) + L / 2) * sizeof(float2);
  c.ok = c.C * L <= FFT_PER * c.threads && L / 2 <= FFT_PER * c.threads;
  return c;
}

}  // namespace

int fft_rows_forward(ppd_plan* p, const float* x, float2* dst) {
  int slot;
  const RowCfg rc = row_cfg(p->Kx, p->ny);
  if (!rc.ok) return fail(PPD_EUNSUPPORTED, "fft: row launch shape exceeds the staging capacity");
  PPD_TRY(timer_begin(p, KK_FFT_ROWS_FWD, &slot));
  hipLaunchKernelGGL(k_fft_rows_fwd, dim3(rc.blocks), dim3(rc.threads), rc.lds, p->stream, x, p->dpx,
                     p->dpy, p->twx, p->nx, p->log2Kx, rc.rpb, dst);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

int fft_cols_forward(ppd_plan* p, const float2* src) {
  int slot;
  const ColCfg cc = col_cfg(p->Ky, p->Kx);
  if (!cc.ok) return fail(PPD_EUNSUPPORTED, "fft: column launch shape exceeds the staging capacity");
  PPD_TRY(timer_begin(p, KK_FFT_COLS_FWD, &slot));
  hipLaunchKernelGGL(k_fft_cols_fwd, dim3(cc.blocks), dim3(cc.threads), cc.lds, p->stream, src,
                     p->twy, p->ny, p->Kx, p->log2Ky, cc.C, cc.ngroups, p->grid_f);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

int fft_forward(ppd_plan* p, const float* x) {
  PPD_TRY(fft_rows_forward(p, x, p->half));
  return fft_cols_forward(p, p->half);
}

int fft_cols_inverse(ppd_plan* p) {
  int slot;
  const ColCfg cc = col_cfg(p->Ky, p->Kx);
  if (!cc.ok) return fail(PPD_EUNSUPPORTED, "fft: column launch shape exceeds the staging capacity");
  PPD_TRY(timer_begin(p, KK_FFT_COLS_INV, &slot));
  hipLaunchKernelGGL(k_fft_cols_inv, dim3(cc.blocks), dim3(cc.threads), cc.lds, p->stream, p->grid_a,
                     p->twy, p->ny, p->Kx, p->log2Ky, cc.C, cc.ngroups, p->half);
  PPD_HIP(hipGetLastError());
  PPD_TRY(timer_end(p, slot));
  return PPD_OK;
}

int fft_adjoint(ppd_plan* p, float* x) {
  PPD_TRY(fft_cols_inverse(p));
  int slot;
  const RowCfg rc = row_cfg(p->Kx, p->ny);
  if (!rc.ok) return fail(PPD_EUNSUPPORTED, "fft: row launch shape exceeds the staging capacity");
  PPD_TRY(timer_begin(p, KK_FFT_ROWS_INV, &slot));
  hipLaunchKernelGGL((k_fft_rows_inv<false, false>), dim3(rc.blocks), dim3(rc.threads), rc.lds, p->stream,
                     p->half, p->twx, p->dpx, p->dpy, p->nx, p->log2Kx, rc.rpb, x, nullptr, nullptr,
                     nullptr, 0.0, 0.0, 0.0, 0.0, nullptr, nullptr);
  PPD_HIP(hipGetLastError());
  PPD_TRY(timer_end(p, slot));
  return PPD_OK;
}

int fft_rows_inverse_primal(ppd_plan* p, const PrimalArgs& a, float2* next) {
  int slot;
  const RowCfg rc = row_cfg(p->Kx, p->ny);
  if (!rc.ok) return fail(PPD_EUNSUPPORTED, "fft: row launch shape exceeds the staging capacity");
  PPD_TRY(timer_begin(p, KK_FFT_ROWS_INV, &slot));
  if (next)
    hipLaunchKernelGGL((k_fft_rows_inv<true, true>), dim3(rc.blocks), dim3(rc.threads), rc.lds, p->stream,
                       p->half, p->twx, p->dpx, p->dpy, p->nx, p->log2Kx, rc.rpb, a.x, a.xt, a.ut,
                       a.x_true, a.tau, a.eta, a.zeta, a.lambda, a.part, next);
  else
    hipLaunchKernelGGL((k_fft_rows_inv<true, false>), dim3(rc.blocks), dim3(rc.threads), rc.lds, p->stream,
                       p->half, p->twx, p->dpx, p->dpy, p->nx, p->log2Kx, rc.rpb, a.x, a.xt, a.ut,
                       a.x_true, a.tau, a.eta, a.zeta, a.lambda, a.part, nullptr);
  PPD_HIP(hipGetLastError());
  PPD_TRY(timer_end(p, slot));
  return PPD_OK;
}

int primal_partial_count(ppd_plan* p) { return row_cfg(p->Kx, p->ny).blocks; }

}  // namespace ppd
