// SARA sparsity operator (Sec. 5.1): Psi = (1/3)[I, W_1, .., W_8], W_p the
// orthonormal periodised 2D Daubechies-p wavelet transform, coefficients in
// the Mallat layout of the image.  Float32.
//
// Analysis runs one launch per level for the 8 wavelet bases at once
// (blockIdx.z = basis; the Dirac basis rides in the first launch): a
// workgroup stages the periodic input region of its output tile in LDS,
// filters the columns, then the rows, and writes the four sub-bands.  In
// the dual mode (Algorithm 3 steps 19-20) every final coefficient c is
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
constexpr int MAXR = 2 * AT + 2 * FILT_STRIDE;   // staged input extent

struct SaraGeom {
  int nx, ny, L;
  size_t N;
  size_t off[8];   // per-level temporaries: off[l] for level l (1 <= l < L)
};

__device__ __host__ inline size_t lvl_size(const SaraGeom& g, int l) { return g.N >> (2 * l); }

enum { A_PLAIN = 0, A_DUAL = 1 };

template <int MODE>
__global__ __launch_bounds__(256) void k_dwt(const float* __restrict__ x, float* __restrict__ tmp,
                                             float* __restrict__ out, const float* __restrict__ filt,
                                             const float* __restrict__ W, SaraGeom g, int l, float alpha,
                                             float lambda) {
  __shared__ float sin_[MAXR * MAXR];
  __shared__ float slo[AT * MAXR];
  __shared__ float shi[AT * MAXR];
  const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
  const int oh = hh >> 1, ow = ww >> 1;
  const int toy = min(AT, oh), tox = min(AT, ow);
  const int k0y = blockIdx.y * toy, k0x = blockIdx.x * tox;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int q = blockIdx.z + 1;   // 1..8 wavelets, 9 = Dirac (level 1 only)
  const float third = 1.0f / 3.0f;
  if (q == 9) {
    // Dirac basis: coefficient x / 3 at every pixel of this tile's footprint
    for (int i = tid; i < 4 * toy * tox; i += nth) {
      const int a = i / (2 * tox), b = i - a * (2 * tox);
      const size_t P = size_t(2 * k0y + a) * g.nx + (2 * k0x + b);
      const float c = x[P] * third * (W ? W[P] : 1.0f);
      if (MODE == A_PLAIN) {
        out[P] = c;
      } else {
        const float uo = out[P];
        const float ub = fminf(fmaxf(uo + c, -alpha), alpha);
        out[P] = uo + lambda * (ub - uo);
      }
    }
    return;
  }
  const float* h = filt + (q - 1) * 2 * FILT_STRIDE;
  const float* gh = h + FILT_STRIDE;
  const int taps = 2 * q;
  const int IR = 2 * toy + taps - 2, IC = 2 * tox + taps - 2;
  // input: level 1 reads the image (scaled by 1/3), deeper levels the
  // low-pass band of the previous level
  const float* src;
  int sstride;
  float scale;
  if (l == 1) {
    src = x;
    sstride = g.nx;
    scale = third;
  } else {
    src = tmp + g.off[l - 1] + size_t(q - 1) * lvl_size(g, l - 1);
    sstride = ww;
    scale = 1.0f;
  }
  for (int i = tid; i < IR * IC; i += nth) {
    const int a = i / IC, b = i - a * IC;
    const int r = (2 * k0y + a) & (hh - 1), c = (2 * k0x + b) & (ww - 1);
    sin_[a * IC + b] = src[size_t(r) * sstride + c] * scale;
  }
  __syncthreads();
  for (int i = tid; i < toy * IC; i += nth) {   // columns (axis 0)
    const int k = i / IC, c = i - k * IC;
    float lo = 0.f, hi = 0.f;
    for (int n = 0; n < taps; ++n) {
      const float s = sin_[(2 * k + n) * IC + c];
      lo = fmaf(h[n], s, lo);
      hi = fmaf(gh[n], s, hi);
    }
    slo[k * IC + c] = lo;
    shi[k * IC + c] = hi;
  }
  __syncthreads();
  float* ub = out + size_t(q) * g.N;
  const float* wb = W ? W + size_t(q) * g.N : nullptr;
  for (int i = tid; i < toy * tox; i += nth) {  // rows (axis 1)
    const int k = i / tox, m = i - k * tox;
    float ll = 0.f, lh = 0.f, hl = 0.f, hh_ = 0.f;
    for (int n = 0; n < taps; ++n) {
      const float a = slo[k * IC + 2 * m + n], d = shi[k * IC + 2 * m + n];
      ll = fmaf(h[n], a, ll);
      lh = fmaf(gh[n], a, lh);
      hl = fmaf(h[n], d, hl);
      hh_ = fmaf(gh[n], d, hh_);
    }
    const int r = k0y + k, c = k0x + m;
    const size_t pLH = size_t(r) * g.nx + (ow + c);
    const size_t pHL = size_t(oh + r) * g.nx + c;
    const size_t pHH = size_t(oh + r) * g.nx + (ow + c);
    const size_t pos[3] = {pLH, pHL, pHH};
    const float vals[3] = {lh * (wb ? wb[pLH] : 1.0f), hl * (wb ? wb[pHL] : 1.0f), hh_ * (wb ? wb[pHH] : 1.0f)};
    for (int s = 0; s < 3; ++s) {
      if (MODE == A_PLAIN) {
        ub[pos[s]] = vals[s];
      } else {
        const float uo = ub[pos[s]];
        const float cl = fminf(fmaxf(uo + vals[s], -alpha), alpha);
        ub[pos[s]] = uo + lambda * (cl - uo);
      }
    }
    if (l == g.L) {
      const size_t pLL = size_t(r) * g.nx + c;
      if (wb) ll *= wb[pLL];
      if (MODE == A_PLAIN) {
        ub[pLL] = ll;
      } else {
        const float uo = ub[pLL];
        const float cl = fminf(fmaxf(uo + ll, -alpha), alpha);
        ub[pLL] = uo + lambda * (cl - uo);
      }
    } else {
      tmp[g.off[l] + size_t(q - 1) * lvl_size(g, l) + size_t(r) * ow + c] = ll;
    }
  }
}

// Inverse of one level for basis q: sub-bands (oh x ow) -> (hh x ww).
// Writes the tile into `acc` (registers of the caller, indexed by the
// thread's loop position) through the functor.
template <typename Sink>
__device__ void idwt_tile(const float* __restrict__ llsrc, int llstride, const float* __restrict__ ucoef,
                          const float* __restrict__ wcoef, const float* __restrict__ llw,
                          int nx, int hh, int ww, int y0, int x0, int tsy, int tsx,
                          const float* __restrict__ h, const float* __restrict__ gh, int taps,
                          float* s_ll, float* s_lh, float* s_hl, float* s_hh, float* s_a, float* s_d,
                          Sink sink) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int oh = hh >> 1, ow = ww >> 1;
  const int q = taps >> 1;
  const int KR = (tsy >> 1) + q, KC = (tsx >> 1) + q;
  const int krb = (y0 >> 1) - q, kcb = (x0 >> 1) - q;
  for (int i = tid; i < KR * KC; i += nth) {
    const int a = i / KC, b = i - a * KC;
    const int r = (krb + a) & (oh - 1), c = (kcb + b) & (ow - 1);
    const size_t pll = size_t(r) * llstride + c;
    const size_t plh = size_t(r) * nx + (ow + c), phl = size_t(oh + r) * nx + c;
    const size_t phh = size_t(oh + r) * nx + (ow + c);
    s_ll[i] = llsrc[pll] * (llw ? llw[pll] : 1.0f);
    s_lh[i] = ucoef[plh] * (wcoef ? wcoef[plh] : 1.0f);
    s_hl[i] = ucoef[phl] * (wcoef ? wcoef[phl] : 1.0f);
    s_hh[i] = ucoef[phh] * (wcoef ? wcoef[phh] : 1.0f);
  }
  __syncthreads();
  // rows: A = synth(LL, LH), D = synth(HL, HH) along axis 1
  for (int i = tid; i < KR * tsx; i += nth) {
    const int kr = i / tsx, m = i - kr * tsx;
    const int mp = x0 + m;
    float av = 0.f, dv = 0.f;
    for (int n = (mp & 1); n < taps; n += 2) {
      const int kk = ((mp - n) & (ww - 1)) >> 1;
      const int lc = (kk - kcb) & (ow - 1);
      const int li = kr * KC + lc;
      av = fmaf(h[n], s_ll[li], fmaf(gh[n], s_lh[li], av));
      dv = fmaf(h[n], s_hl[li], fmaf(gh[n], s_hh[li], dv));
    }
    s_a[kr * tsx + m] = av;
    s_d[kr * tsx + m] = dv;
  }
  __syncthreads();
  // columns: S = synth(A, D) along axis 0
  int slot = 0;
  for (int i = tid; i < tsy * tsx; i += nth, ++slot) {
    const int m2 = i / tsx, m = i - m2 * tsx;
    const int mp = y0 + m2;
    float sv = 0.f;
    for (int n = (mp & 1); n < taps; n += 2) {
      const int kk = ((mp - n) & (hh - 1)) >> 1;
      const int lr = (kk - krb) & (oh - 1);
      sv = fmaf(h[n], s_a[lr * tsx + m], fmaf(gh[n], s_d[lr * tsx + m], sv));
    }
    sink(slot, m2, m, sv);
  }
  __syncthreads();
}

constexpr int SK = ST / 2 + FILT_STRIDE / 2;   // max staged coefficient extent

// Intermediate synthesis level l >= 2 (output = low-pass band of level l-1).
__global__ __launch_bounds__(256) void k_idwt(const float* __restrict__ u, float* __restrict__ rec,
                                              const float* __restrict__ filt, const float* __restrict__ W,
                                              SaraGeom g, int l) {
  __shared__ float s_ll[SK * SK], s_lh[SK * SK], s_hl[SK * SK], s_hh[SK * SK];
  __shared__ float s_a[SK * ST], s_d[SK * ST];
  const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
  const int tsy = min(ST, hh), tsx = min(ST, ww);
  const int y0 = blockIdx.y * tsy, x0 = blockIdx.x * tsx;
  const int q = blockIdx.z + 1;
  const float* h = filt + (q - 1) * 2 * FILT_STRIDE;
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
  idwt_tile(llsrc, llstride, ucoef, wcoef, llw, g.nx, hh, ww, y0, x0, tsy, tsx, h, h + FILT_STRIDE, 2 * q,
            s_ll, s_lh, s_hl, s_hh, s_a, s_d,
            [&](int, int r, int c, float v) { dst[size_t(y0 + r) * ww + (x0 + c)] = v; });
}

// Level 1 for all 8 wavelet bases, plus the Dirac part, times 1/3.
__global__ __launch_bounds__(256) void k_idwt_final(const float* __restrict__ u, const float* __restrict__ rec,
                                                    const float* __restrict__ filt,
                                                    const float* __restrict__ W, SaraGeom g,
                                                    float* __restrict__ out) {
  __shared__ float s_ll[SK * SK], s_lh[SK * SK], s_hl[SK * SK], s_hh[SK * SK];
  __shared__ float s_a[SK * ST], s_d[SK * ST];
  const int hh = g.ny, ww = g.nx;
  const int tsy = min(STF, hh), tsx = min(STF, ww);
  const int y0 = blockIdx.y * tsy, x0 = blockIdx.x * tsx;
  float acc[(STF * STF + 255) / 256];
  for (int s = 0; s < (STF * STF + 255) / 256; ++s) acc[s] = 0.f;
  for (int q = 1; q <= 8; ++q) {
    const float* h = filt + (q - 1) * 2 * FILT_STRIDE;
    const float* ucoef = u + size_t(q) * g.N;
    const float* wcoef = W ? W + size_t(q) * g.N : nullptr;
    const float* llsrc = g.L == 1 ? ucoef : rec + g.off[1] + size_t(q - 1) * lvl_size(g, 1);
    const float* llw = g.L == 1 ? wcoef : nullptr;
    const int llstride = g.L == 1 ? g.nx : (ww >> 1);
    idwt_tile(llsrc, llstride, ucoef, wcoef, llw, g.nx, hh, ww, y0, x0, tsy, tsx, h, h + FILT_STRIDE, 2 * q,
              s_ll, s_lh, s_hl, s_hh, s_a, s_d,
              [&](int slot, int, int, float v) { acc[slot] += v; });
  }
  const float third = 1.0f / 3.0f;
  int slot = 0;
  for (int i = threadIdx.x; i < tsy * tsx; i += blockDim.x, ++slot) {
    const int r = i / tsx, c = i - r * tsx;
    const size_t P = size_t(y0 + r) * g.nx + (x0 + c);
    out[P] = (acc[slot] + u[P] * (W ? W[P] : 1.0f)) * third;
  }
}

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
                    float lambda) {
  const SaraGeom g = geom(p);
  for (int l = 1; l <= g.L; ++l) {
    const int oh = (g.ny >> l), ow = (g.nx >> l);
    const int toy = std::min(AT, oh), tox = std::min(AT, ow);
    dim3 grid(ow / tox, oh / toy, l == 1 ? 9 : 8);
    int slot;
    PPD_TRY(timer_begin(p, KK_DWT, &slot));
    if (dual)
      hipLaunchKernelGGL(k_dwt<A_DUAL>, grid, dim3(256), 0, p->stream, x, p->sara_ll, out, p->filt, W, g, l,
                         alpha, lambda);
    else
      hipLaunchKernelGGL(k_dwt<A_PLAIN>, grid, dim3(256), 0, p->stream, x, p->sara_ll, out, p->filt, W, g, l,
                         alpha, lambda);
    PPD_HIP(hipGetLastError());
    PPD_TRY(timer_end(p, slot));
  }
  return PPD_OK;
}

}  // namespace

int sara_analysis(ppd_plan* p, const float* x, float* coef, const float* W) {
  return analysis_launch(p, x, coef, W, false, 0.f, 0.f);
}

int sara_dual(ppd_plan* p, const float* x, float* u, float alpha, float lambda, const float* W) {
  return analysis_launch(p, x, u, W, true, alpha, lambda);
}

int sara_synthesis(ppd_plan* p, const float* u, float* out, const float* W) {
  const SaraGeom g = geom(p);
  for (int l = g.L; l >= 2; --l) {
    const int hh = g.ny >> (l - 1), ww = g.nx >> (l - 1);
    const int tsy = std::min(ST, hh), tsx = std::min(ST, ww);
    int slot;
    PPD_TRY(timer_begin(p, KK_IDWT, &slot));
    hipLaunchKernelGGL(k_idwt, dim3(ww / tsx, hh / tsy, 8), dim3(256), 0, p->stream, u, p->sara_rec, p->filt,
                       W, g, l);
    PPD_HIP(hipGetLastError());
    PPD_TRY(timer_end(p, slot));
  }
  const int tsy = std::min(STF, g.ny), tsx = std::min(STF, g.nx);
  int slot;
  PPD_TRY(timer_begin(p, KK_IDWT, &slot));
  hipLaunchKernelGGL(k_idwt_final, dim3(g.nx / tsx, g.ny / tsy), dim3(256), 0, p->stream, u, p->sara_rec,
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
