// Interpolation G and its adjoint (Sec. 2; Sec. 5: 8x8 Kaiser-Bessel
// kernels), with the data-block dual update of Algorithm 3 fused in.
//
// Work unit: a chunk of <= chunk_max visibilities of one data block whose
// first tap lies in one T x T grid tile.  The workgroup stages the tile
// plus its 7-cell halo ((T+7)^2 complex cells) in LDS:
//   degrid: the forward spectrum region is copied in, every thread then
//           interpolates its visibilities from LDS (64 taps each);
//   grid:   contributions accumulate in LDS with ds_add_f32 and the region
//           is added to the global grid once per chunk (no global atomics
//           in the per-visibility loop).
// The 8 per-axis weights are evaluated on the fly from degree-9
// polynomials; only the two float32 frequencies are read per visibility.
// Chunks are launched in spatial order with an XCD-aware remap.
#include "ppd_internal.h"

namespace ppd {
namespace {

__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

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

// Norm of one data block's residual from its chunk partials (wave 0,
// fixed order, so every workgroup of the block gets the same value).
__device__ inline double block_norm2(int j, const double* __restrict__ part,
                                     const int32_t* __restrict__ bids, const int32_t* __restrict__ boff) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int c = boff[j] + lane; c < boff[j + 1]; c += 64) s += part[bids[c]];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

template <int T, bool DUAL>
__global__ __launch_bounds__(256) void k_degrid(
    const float2* __restrict__ grid, int Kx, int Ky, const Chunk* __restrict__ chunks, int n_chunks,
    const float* __restrict__ wu, const float* __restrict__ wv, const float* __restrict__ theta,
    double su, double sv, const float* __restrict__ kbc, float2* __restrict__ out,
    const float2* __restrict__ y, const double* __restrict__ U, const float2* __restrict__ v,
    const double2* __restrict__ z, double2* __restrict__ wout, double mu,
    double* __restrict__ part, double* __restrict__ rpart) {
  constexpr int R = T + 7;
  __shared__ float2 reg[R * R];
  __shared__ float coef[KB_TAPS * KB_NC];
  __shared__ double red[16];
  const int ci = xcd_remap(blockIdx.x, gridDim.x);
  if (ci >= n_chunks) return;
  const Chunk ch = chunks[ci];
  const int r0 = ch.ty * T, c0 = ch.tx * T;
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
    const int a = i / R, b = i - a * R;
    reg[i] = grid[size_t((r0 + a) & (Ky - 1)) * Kx + ((c0 + b) & (Kx - 1))];
  }
  if (threadIdx.x < KB_TAPS * KB_NC) coef[threadIdx.x] = kbc[threadIdx.x];
  __syncthreads();
  double qn = 0.0, rn = 0.0;
  for (int k = threadIdx.x; k < ch.count; k += blockDim.x) {
    const int pi = ch.start + k;
    Taps t;
    taps_for<T>(wu[pi], wv[pi], su, sv, Kx, Ky, c0, r0, coef, t);
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
      ax = fmaf(t.wy[a], sx, ax);
      ay = fmaf(t.wy[a], sy, ay);
    }
    const float th = theta ? theta[pi] : 1.0f;
    const float2 g = make_float2(ax * th, ay * th);
    if (!DUAL) {
      out[pi] = g;
    } else {
      // Algorithm 3 step 10: w = U^-1 v + Theta G a; first Algorithm 2 step
      const float2 ve = v[pi];
      const double Ue = U[pi];
      const double2 ze = z[pi];
      const float2 ye = y[pi];
      const double wx = double(ve.x) / Ue + double(g.x);
      const double wy = double(ve.y) / Ue + double(g.y);
      wout[pi] = make_double2(wx, wy);
      const double mU = mu * Ue;
      const double dx = (ze.x - mU * (ze.x - wx)) - double(ye.x);
      const double dy = (ze.y - mU * (ze.y - wy)) - double(ye.y);
      qn += dx * dx + dy * dy;
      const double ex = double(g.x) - double(ye.x), ey = double(g.y) - double(ye.y);
      rn += ex * ex + ey * ey;
    }
  }
  if (DUAL) {
    qn = block_sum(qn, red);
    rn = block_sum(rn, red);
    if (threadIdx.x == 0) {
      part[ci] = qn;
      rpart[ci] = rn;
    }
  }
}

// Alg. 2 projection: z' = P_B(q) with the block's scale factor.
__device__ __forceinline__ void project(double qx, double qy, float2 ye, bool inside, double f,
                                        double& zx, double& zy) {
  if (inside) {
    zx = qx;
    zy = qy;
  } else {
    zx = double(ye.x) + (qx - double(ye.x)) * f;
    zy = double(ye.y) + (qy - double(ye.y)) * f;
  }
}

template <int T, bool DUAL>
__global__ __launch_bounds__(256) void k_grid(
    float2* __restrict__ grid, int Kx, int Ky, const Chunk* __restrict__ chunks, int n_chunks,
    const float* __restrict__ wu, const float* __restrict__ wv, const float* __restrict__ theta,
    double su, double sv, const float* __restrict__ kbc, const float2* __restrict__ vin,
    const float2* __restrict__ y, const double* __restrict__ U, float2* __restrict__ v,
    double2* __restrict__ z, const double2* __restrict__ w, double mu, double lambda,
    const double* __restrict__ part, const int32_t* __restrict__ bids,
    const int32_t* __restrict__ boff, const double* __restrict__ eps) {
  constexpr int R = T + 7;
  __shared__ float acc[2 * R * R];
  __shared__ float coef[KB_TAPS * KB_NC];
  __shared__ double s_fac;
  __shared__ int s_inside;
  const int ci = xcd_remap(blockIdx.x, gridDim.x);
  if (ci >= n_chunks) return;
  const Chunk ch = chunks[ci];
  const int r0 = ch.ty * T, c0 = ch.tx * T;
  for (int i = threadIdx.x; i < 2 * R * R; i += blockDim.x) acc[i] = 0.f;
  if (threadIdx.x < KB_TAPS * KB_NC) coef[threadIdx.x] = kbc[threadIdx.x];
  if (DUAL && threadIdx.x < 64) {
    const double r = sqrt(block_norm2(ch.block, part, bids, boff));
    if (threadIdx.x == 0) {
      const double e = eps[ch.block];
      s_inside = r <= e;
      s_fac = r > e ? e / r : 1.0;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ch.count; k += blockDim.x) {
    const int pi = ch.start + k;
    Taps t;
    taps_for<T>(wu[pi], wv[pi], su, sv, Kx, Ky, c0, r0, coef, t);
    float2 val;
    if (!DUAL) {
      val = vin[pi];
    } else {
      // last Algorithm 2 projection, then steps 10-11
      const double2 we = w[pi], ze = z[pi];
      const double Ue = U[pi];
      const float2 ye = y[pi], vo = v[pi];
      const double mU = mu * Ue;
      double zx, zy;
      project(ze.x - mU * (ze.x - we.x), ze.y - mU * (ze.y - we.y), ye, s_inside, s_fac, zx, zy);
      z[pi] = make_double2(zx, zy);
      const double vbx = Ue * (we.x - zx), vby = Ue * (we.y - zy);
      const float2 vn = make_float2(float(double(vo.x) + lambda * (vbx - double(vo.x))),
                                    float(double(vo.y) + lambda * (vby - double(vo.y))));
      v[pi] = vn;
      val = vn;
    }
    const float th = theta ? theta[pi] : 1.0f;
    val.x *= th;
    val.y *= th;
#pragma unroll
    for (int a = 0; a < KB_TAPS; ++a) {
      const float ra = t.wy[a] * val.x, ia = t.wy[a] * val.y;
      float* rowp = acc + 2 * ((t.ov + a) * R + t.ou);
#pragma unroll
      for (int b = 0; b < KB_TAPS; ++b) {
        atomicAdd(rowp + 2 * b, t.wx[b] * ra);
        atomicAdd(rowp + 2 * b + 1, t.wx[b] * ia);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) {
    const float re = acc[2 * i], im = acc[2 * i + 1];
    if (re != 0.f || im != 0.f) {
      const int a = i / R, b = i - a * R;
      float* gp = reinterpret_cast<float*>(grid + size_t((r0 + a) & (Ky - 1)) * Kx + ((c0 + b) & (Kx - 1)));
      atomicAdd(gp, re);
      atomicAdd(gp + 1, im);
    }
  }
}

template <int ELEM>
struct Elem;
template <> struct Elem<4> { using type = float; };
template <> struct Elem<8> { using type = float2; };
template <> struct Elem<16> { using type = double2; };

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
  if (!dual) {
    hipLaunchKernelGGL((k_degrid<T, false>), dim3(p->n_launch), dim3(256), 0, p->stream, p->grid_f,
                       p->Kx, p->Ky, p->chunks, p->n_chunks, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, out, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0,
                       nullptr, nullptr);
  } else {
    hipLaunchKernelGGL((k_degrid<T, true>), dim3(p->n_launch), dim3(256), 0, p->stream, p->grid_f,
                       p->Kx, p->Ky, p->chunks, p->n_chunks, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, nullptr, a->y, a->U, a->v, a->z, p->wbuf, a->mu,
                       part_out, p->rpart);
  }
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

template <int T>
int launch_grid(ppd_plan* p, bool dual, const float2* vin, const DualArgs* a, const double* part_in) {
  if (!dual) {
    hipLaunchKernelGGL((k_grid<T, false>), dim3(p->n_launch), dim3(256), 0, p->stream, p->grid_a,
                       p->Kx, p->Ky, p->chunks, p->n_chunks, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, vin, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0,
                       0.0, nullptr, nullptr, nullptr, nullptr);
  } else {
    hipLaunchKernelGGL((k_grid<T, true>), dim3(p->n_launch), dim3(256), 0, p->stream, p->grid_a,
                       p->Kx, p->Ky, p->chunks, p->n_chunks, p->wu, p->wv, p->theta, p->su_scale,
                       p->sv_scale, p->kbc, nullptr, a->y, a->U, a->v, a->z, p->wbuf, a->mu,
                       a->lambda, part_in, p->bchunk_ids, p->bchunk_off_d, p->eps_d);
  }
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

int dispatch_degrid(ppd_plan* p, bool dual, float2* out, const DualArgs* a, double* part_out) {
  int slot;
  PPD_TRY(timer_begin(p, KK_DEGRID, &slot));
  int st;
  switch (p->T) {
    case 16: st = launch_degrid<16>(p, dual, out, a, part_out); break;
    case 32: st = launch_degrid<32>(p, dual, out, a, part_out); break;
    default: st = launch_degrid<64>(p, dual, out, a, part_out); break;
  }
  PPD_TRY(st);
  return timer_end(p, slot);
}

int dispatch_grid(ppd_plan* p, bool dual, const float2* vin, const DualArgs* a, const double* part_in) {
  int slot;
  PPD_TRY(timer_begin(p, KK_GRID, &slot));
  int st;
  switch (p->T) {
    case 16: st = launch_grid<16>(p, dual, vin, a, part_in); break;
    case 32: st = launch_grid<32>(p, dual, vin, a, part_in); break;
    default: st = launch_grid<64>(p, dual, vin, a, part_in); break;
  }
  PPD_TRY(st);
  return timer_end(p, slot);
}

}  // namespace

int degrid_plain(ppd_plan* p, float2* out) { return dispatch_degrid(p, false, out, nullptr, nullptr); }
int degrid_dual(ppd_plan* p, const DualArgs& a, double* part_out) {
  return dispatch_degrid(p, true, nullptr, &a, part_out);
}
int grid_plain(ppd_plan* p, const float2* v) { return dispatch_grid(p, false, v, nullptr, nullptr); }
int grid_dual(ppd_plan* p, const DualArgs& a, const double* part_in) {
  return dispatch_grid(p, true, nullptr, &a, part_in);
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
  PPD_TRY(zero_grid(p, p->grid_a));
  PPD_TRY(grid_plain(p, v));
  return fft_adjoint(p, x);
}
