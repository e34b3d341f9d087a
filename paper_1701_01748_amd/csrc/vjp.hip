// Differentiable pieces of Algorithm 3 for unrolled iterations: the
// data-dual update (Algorithm 2 inside the generalised Moreau step), the
// sparsity dual update (the clip (I - S_alpha) and relaxation) and the
// primal update (P_C, relaxation and x~), each as a forward kernel and a
// vector-Jacobian product (VJP) kernel.  Gradients follow torch's
// convention for complex tensors (dL/dRe + i dL/dIm of a real loss L).
//
// The data-dual update works on plan-order vectors, block by block, in
// chunks of SEC_CHUNK consecutive points of one block (the chunk table of
// the exact prox); every block norm or block inner product is a sum of
// chunk partials in chunk order (deterministic).
#include <cmath>

#include "ppd_internal.h"

namespace ppd {
namespace {

constexpr int DU_THREADS = 256;

__device__ __forceinline__ double du_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < DU_THREADS / 64; ++k) s += red[k];
  __syncthreads();
  return s;
}

struct DuIn {
  const float2* g; const float2* y; const double* U; const float2* v;
  double mu;
};

// w = U^-1 v + g in FP64 (the argument of the generalised Moreau step)
__device__ __forceinline__ double2 du_w(const DuIn& a, int64_t i, double Ue) {
  const float2 ve = a.v[i], ge = a.g[i];
  return dual_arg(ve, Ue, ge);
}

// Chunk partials of ||q - y||^2 (and, with gz, of Re <q - y, gz>) for
// q = z - mu U (z - w), z = zprev.
__global__ __launch_bounds__(DU_THREADS) void k_du_partials(DuIn a, const int32_t* __restrict__ cstart,
                                                            const double2* __restrict__ zprev,
                                                            const double2* __restrict__ gz,
                                                            double* __restrict__ p2, double* __restrict__ pd) {
  __shared__ double red[DU_THREADS / 64];
  const int c = blockIdx.x;
  double s2 = 0.0, sd = 0.0;
  for (int64_t i = cstart[c] + threadIdx.x; i < cstart[c + 1]; i += DU_THREADS) {
    const double Ue = a.U[i], mU = a.mu * Ue;
    const double2 we = du_w(a, i, Ue), ze = zprev[i];
    const float2 ye = a.y[i];
    const double dx = (ze.x - mU * (ze.x - we.x)) - double(ye.x);
    const double dy = (ze.y - mU * (ze.y - we.y)) - double(ye.y);
    s2 += dx * dx + dy * dy;
    if (gz) {
      const double2 ge = gz[i];
      sd += dx * ge.x + dy * ge.y;
    }
  }
  s2 = du_block_sum(s2, red);
  if (gz) sd = du_block_sum(sd, red);
  if (threadIdx.x == 0) {
    p2[c] = s2;
    if (gz) pd[c] = sd;
  }
}

// Per block j: r = ||q - y||, and (forward) the P_B factor, or (VJP) the
// coefficients of the P_B Jacobian's transpose applied to gz:
// outside the ball gq = (eps / r) gz - (eps <d, gz> / r^3) d.
// blk[j] = (factor or eps / r, eps <d, gz> / r^3, inside, r).
__global__ __launch_bounds__(DU_THREADS) void k_du_blocks(const int32_t* __restrict__ coff,
                                                          const double* __restrict__ eps,
                                                          const double* __restrict__ p2,
                                                          const double* __restrict__ pd,
                                                          double4* __restrict__ blk) {
  __shared__ double red[DU_THREADS / 64];
  const int j = blockIdx.x;
  double s2 = 0.0, sd = 0.0;
  for (int c = coff[j] + int(threadIdx.x); c < coff[j + 1]; c += DU_THREADS) {
    s2 += p2[c];
    if (pd) sd += pd[c];
  }
  s2 = du_block_sum(s2, red);
  if (pd) sd = du_block_sum(sd, red);
  if (threadIdx.x == 0) {
    const double r = sqrt(s2), e = eps[j];
    const bool inside = r <= e;
    blk[j] = inside ? make_double4(1.0, 0.0, 1.0, r) : make_double4(e / r, e * sd / (r * r * r), 0.0, r);
  }
}

// Forward step s: z_s = P_B(q_s), q_s from zprev.
__global__ void k_du_apply(DuIn a, int64_t M, const int32_t* __restrict__ vblk, const double4* __restrict__ blk,
                           const double2* __restrict__ zprev, double2* __restrict__ znext) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const double Ue = a.U[i], mU = a.mu * Ue;
    const double2 we = du_w(a, i, Ue), ze = zprev[i];
    const float2 ye = a.y[i];
    const double4 b = blk[vblk[i]];
    const double qx = ze.x - mU * (ze.x - we.x), qy = ze.y - mU * (ze.y - we.y);
    znext[i] = b.z != 0.0 ? make_double2(qx, qy)
                          : make_double2(double(ye.x) + (qx - double(ye.x)) * b.x,
                                         double(ye.y) + (qy - double(ye.y)) * b.x);
  }
}

// v' = v + lambda (U (w - z_n) - v), z' = z_n.
__global__ void k_du_finish(DuIn a, int64_t M, double lambda, const double2* __restrict__ zn,
                            float2* __restrict__ v_out, double2* __restrict__ z_out) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const double Ue = a.U[i];
    const double2 we = du_w(a, i, Ue), ze = zn[i];
    const float2 ve = a.v[i];
    const double vbx = Ue * (we.x - ze.x), vby = Ue * (we.y - ze.y);
    v_out[i] = make_float2(float(double(ve.x) + lambda * (vbx - double(ve.x))),
                           float(double(ve.y) + lambda * (vby - double(ve.y))));
    if (z_out != zn) z_out[i] = ze;
  }
}

// VJP start: gz_n = gz' - lambda U gv', gw = lambda U gv', gy = 0.
__global__ void k_du_vjp_init(int64_t M, const double* __restrict__ U, double lambda,
                              const float2* __restrict__ gv, const double2* __restrict__ gz,
                              double2* __restrict__ gzc, double2* __restrict__ gw, double2* __restrict__ gy) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const double lU = lambda * U[i];
    const float2 g = gv ? gv[i] : make_float2(0.f, 0.f);
    const double2 z = gz ? gz[i] : make_double2(0.0, 0.0);
    gzc[i] = make_double2(z.x - lU * double(g.x), z.y - lU * double(g.y));
    gw[i] = make_double2(lU * double(g.x), lU * double(g.y));
    gy[i] = make_double2(0.0, 0.0);
  }
}

// VJP of step s: gq = P_B Jacobian^T gz_s; gy += gz_s - gq;
// gz_{s-1} = (1 - mu U) gq; gw += mu U gq.  (In place on gzc.)
__global__ void k_du_vjp_step(DuIn a, int64_t M, const int32_t* __restrict__ vblk, const double4* __restrict__ blk,
                              const double2* __restrict__ zprev, double2* __restrict__ gzc,
                              double2* __restrict__ gw, double2* __restrict__ gy) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const double Ue = a.U[i], mU = a.mu * Ue;
    const double4 b = blk[vblk[i]];
    const double2 g = gzc[i];
    double2 gq;
    if (b.z != 0.0) {
      gq = g;
    } else {
      const double2 we = du_w(a, i, Ue), ze = zprev[i];
      const float2 ye = a.y[i];
      const double dx = (ze.x - mU * (ze.x - we.x)) - double(ye.x);
      const double dy = (ze.y - mU * (ze.y - we.y)) - double(ye.y);
      gq = make_double2(b.x * g.x - b.y * dx, b.x * g.y - b.y * dy);
    }
    const double2 yo = gy[i];
    gy[i] = make_double2(yo.x + (g.x - gq.x), yo.y + (g.y - gq.y));
    gzc[i] = make_double2((1.0 - mU) * gq.x, (1.0 - mU) * gq.y);
    const double2 wo = gw[i];
    gw[i] = make_double2(wo.x + mU * gq.x, wo.y + mU * gq.y);
  }
}

// VJP end: gg = gw, gv = (1 - lambda) gv' + gw / U, gy to complex64.
__global__ void k_du_vjp_finish(int64_t M, const double* __restrict__ U, double lambda,
                                const float2* __restrict__ gv_out, const double2* __restrict__ gw,
                                const double2* __restrict__ gy, float2* __restrict__ g_g, float2* __restrict__ g_v,
                                float2* __restrict__ g_y) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const double2 w = gw[i];
    const float2 g = gv_out ? gv_out[i] : make_float2(0.f, 0.f);
    const double Ue = U[i];
    if (g_g) g_g[i] = make_float2(float(w.x), float(w.y));
    if (g_v)
      g_v[i] = make_float2(float((1.0 - lambda) * double(g.x) + w.x / Ue), float((1.0 - lambda) * double(g.y) + w.y / Ue));
    if (g_y) {
      const double2 yy = gy[i];
      g_y[i] = make_float2(float(yy.x), float(yy.y));
    }
  }
}

// Sparsity dual update, per coefficient: u' = u + lambda (clip(u + c) - u);
// VJP: g_u = (1 - lambda) g + lambda m g, g_c = lambda m g, m = [|u + c| < alpha].
__global__ void k_su(int64_t n, const float* __restrict__ u, const float* __restrict__ c, float alpha, float lambda,
                     float* __restrict__ u_out) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float s = u[i] + c[i];
    const float ub = fminf(fmaxf(s, -alpha), alpha);
    u_out[i] = u[i] + lambda * (ub - u[i]);
  }
}

__global__ void k_su_vjp(int64_t n, const float* __restrict__ u, const float* __restrict__ c, float alpha,
                         float lambda, const float* __restrict__ g, float* __restrict__ g_u, float* __restrict__ g_c) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float s = u[i] + c[i];
    const float m = fabsf(s) < alpha ? 1.0f : 0.0f;
    if (g_u) g_u[i] = (1.0f - lambda) * g[i] + lambda * m * g[i];
    if (g_c) g_c[i] = lambda * m * g[i];
  }
}

// Primal update, per pixel (FP64 as in the fused kernel):
// xbar = P_C(x - tau (eta a + zeta b)), x' = x + lambda (xbar - x), x~' = 2 xbar - x.
// VJP: gxbar = lambda gx' + 2 gx~', m = [x - tau (eta a + zeta b) > 0],
// g_x = (1 - lambda) gx' - gx~' + m gxbar, g_a = -tau eta m gxbar, g_b = -tau zeta m gxbar.
__global__ void k_pu(int64_t n, const float* __restrict__ x, const float* __restrict__ a, const float* __restrict__ b,
                     double tau, double eta, double zeta, double lambda, float* __restrict__ x_out,
                     float* __restrict__ xt_out) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double xo = x[i];
    double xb = xo - tau * (eta * double(a[i]) + zeta * double(b[i]));
    xb = xb > 0.0 ? xb : 0.0;
    x_out[i] = float(xo + lambda * (xb - xo));
    xt_out[i] = float(2.0 * xb - xo);
  }
}

__global__ void k_pu_vjp(int64_t n, const float* __restrict__ x, const float* __restrict__ a,
                         const float* __restrict__ b, double tau, double eta, double zeta, double lambda,
                         const float* __restrict__ gx, const float* __restrict__ gxt, float* __restrict__ g_x,
                         float* __restrict__ g_a, float* __restrict__ g_b) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double arg = double(x[i]) - tau * (eta * double(a[i]) + zeta * double(b[i]));
    const double g1 = gx ? double(gx[i]) : 0.0, g2 = gxt ? double(gxt[i]) : 0.0;
    const double gb = arg > 0.0 ? lambda * g1 + 2.0 * g2 : 0.0;
    if (g_x) g_x[i] = float((1.0 - lambda) * g1 - g2 + gb);
    if (g_a) g_a[i] = float(-tau * eta * gb);
    if (g_b) g_b[i] = float(-tau * zeta * gb);
  }
}

int ew_blocks(int64_t n) { return int(std::min<int64_t>((n + 255) / 256, 4096)); }

// q partials, block coefficients (r and, with gz, the Jacobian terms)
int du_blocks(ppd_plan* p, const DuIn& in, const double2* zprev, const double2* gz) {
  double* p2 = p->sec_part;
  double* pd = p->sec_part + p->n_sec_chunks;
  hipLaunchKernelGGL(k_du_partials, dim3(p->n_sec_chunks), dim3(DU_THREADS), 0, p->stream, in, p->sec_cstart, zprev,
                     gz, p2, pd);
  hipLaunchKernelGGL(k_du_blocks, dim3(p->d), dim3(DU_THREADS), 0, p->stream, p->sec_coff, p->eps_d, p2,
                     gz ? pd : nullptr, p->du_blk);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

}  // namespace
}  // namespace ppd

using namespace ppd;

extern "C" int ppd_dual_update(ppd_plan* p, const float* g, const float* y, const double* U, const double* eps,
                               const float* v, const double* z, int n_itr, double mu, double lambda, float* v_out,
                               double* z_out, double* zs) {
  if (!p || !g || !y || !U || !eps || !v || !z || !v_out || !z_out)
    return fail(PPD_EINVAL, "ppd_dual_update: NULL argument");
  if (n_itr < 1) return fail(PPD_EINVAL, "ppd_dual_update: n_itr must be >= 1");
  if (!(mu > 0.0) || !std::isfinite(mu) || !(lambda > 0.0 && lambda <= 1.0))
    return fail(PPD_EINVAL, "ppd_dual_update: need mu > 0 and 0 < lambda <= 1");
  if (z_out == z) return fail(PPD_EINVAL, "ppd_dual_update: z_out must not alias z");
  PPD_TRY(upload_eps(p, eps));
  const DuIn in{reinterpret_cast<const float2*>(g), reinterpret_cast<const float2*>(y), U,
                reinterpret_cast<const float2*>(v), mu};
  double2* zo = reinterpret_cast<double2*>(z_out);
  double2* hist = reinterpret_cast<double2*>(zs);
  const double2* zprev = reinterpret_cast<const double2*>(z);
  for (int s = 1; s <= n_itr; ++s) {
    // z_s goes to zs[s - 1] when a history is kept, else to z_out
    double2* znext = hist ? hist + size_t(s - 1) * p->M : zo;
    PPD_TRY(du_blocks(p, in, zprev, nullptr));
    hipLaunchKernelGGL(k_du_apply, dim3(ew_blocks(p->M)), dim3(256), 0, p->stream, in, p->M, p->vis_block, p->du_blk,
                       zprev, znext);
    zprev = znext;
  }
  hipLaunchKernelGGL(k_du_finish, dim3(ew_blocks(p->M)), dim3(256), 0, p->stream, in, p->M, lambda, zprev,
                     reinterpret_cast<float2*>(v_out), zo);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

extern "C" int ppd_dual_update_vjp(ppd_plan* p, const float* g, const float* y, const double* U, const double* eps,
                                   const float* v, const double* z, int n_itr, double mu, double lambda,
                                   const double* zs, const float* gv_out, const double* gz_out, float* g_g,
                                   float* g_v, double* g_z, float* g_y) {
  if (!p || !g || !y || !U || !eps || !v || !z || !zs || !g_z)
    return fail(PPD_EINVAL, "ppd_dual_update_vjp: NULL argument");
  if (n_itr < 1) return fail(PPD_EINVAL, "ppd_dual_update_vjp: n_itr must be >= 1");
  if (!(mu > 0.0) || !std::isfinite(mu) || !(lambda > 0.0 && lambda <= 1.0))
    return fail(PPD_EINVAL, "ppd_dual_update_vjp: need mu > 0 and 0 < lambda <= 1");
  if (static_cast<const void*>(gz_out) == static_cast<const void*>(g_z))
    return fail(PPD_EINVAL, "ppd_dual_update_vjp: g_z must not alias gz_out");
  PPD_TRY(upload_eps(p, eps));
  const DuIn in{reinterpret_cast<const float2*>(g), reinterpret_cast<const float2*>(y), U,
                reinterpret_cast<const float2*>(v), mu};
  double2* gzc = reinterpret_cast<double2*>(g_z);   // the running gradient of z_s
  double2* gw = p->wbuf;
  double2* gy = p->qbuf;
  const double2* hist = reinterpret_cast<const double2*>(zs);
  hipLaunchKernelGGL(k_du_vjp_init, dim3(ew_blocks(p->M)), dim3(256), 0, p->stream, p->M, U, lambda,
                     reinterpret_cast<const float2*>(gv_out), reinterpret_cast<const double2*>(gz_out), gzc, gw, gy);
  for (int s = n_itr; s >= 1; --s) {
    const double2* zprev = s == 1 ? reinterpret_cast<const double2*>(z) : hist + size_t(s - 2) * p->M;
    PPD_TRY(du_blocks(p, in, zprev, gzc));
    hipLaunchKernelGGL(k_du_vjp_step, dim3(ew_blocks(p->M)), dim3(256), 0, p->stream, in, p->M, p->vis_block,
                       p->du_blk, zprev, gzc, gw, gy);
  }
  hipLaunchKernelGGL(k_du_vjp_finish, dim3(ew_blocks(p->M)), dim3(256), 0, p->stream, p->M, U, lambda,
                     reinterpret_cast<const float2*>(gv_out), gw, gy, reinterpret_cast<float2*>(g_g),
                     reinterpret_cast<float2*>(g_v), reinterpret_cast<float2*>(g_y));
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

extern "C" int ppd_sparsity_update(ppd_plan* p, const float* u, const float* c, float alpha, float lambda,
                                   float* u_out) {
  if (!p || !u || !c || !u_out) return fail(PPD_EINVAL, "ppd_sparsity_update: NULL argument");
  if (!(alpha >= 0.0f) || !(lambda > 0.0f && lambda <= 1.0f))
    return fail(PPD_EINVAL, "ppd_sparsity_update: need alpha >= 0 and 0 < lambda <= 1");
  const int64_t n = int64_t(N_BASES) * p->nx * p->ny;
  hipLaunchKernelGGL(k_su, dim3(ew_blocks(n)), dim3(256), 0, p->stream, n, u, c, alpha, lambda, u_out);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

extern "C" int ppd_sparsity_update_vjp(ppd_plan* p, const float* u, const float* c, float alpha, float lambda,
                                       const float* g_out, float* g_u, float* g_c) {
  if (!p || !u || !c || !g_out) return fail(PPD_EINVAL, "ppd_sparsity_update_vjp: NULL argument");
  if (!(alpha >= 0.0f) || !(lambda > 0.0f && lambda <= 1.0f))
    return fail(PPD_EINVAL, "ppd_sparsity_update_vjp: need alpha >= 0 and 0 < lambda <= 1");
  const int64_t n = int64_t(N_BASES) * p->nx * p->ny;
  hipLaunchKernelGGL(k_su_vjp, dim3(ew_blocks(n)), dim3(256), 0, p->stream, n, u, c, alpha, lambda, g_out, g_u, g_c);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

extern "C" int ppd_primal_update(ppd_plan* p, const float* x, const float* a, const float* b, double tau, double eta,
                                 double zeta, double lambda, float* x_out, float* xt_out) {
  if (!p || !x || !a || !b || !x_out || !xt_out) return fail(PPD_EINVAL, "ppd_primal_update: NULL argument");
  if (!std::isfinite(tau) || !std::isfinite(eta) || !std::isfinite(zeta) || !(lambda > 0.0 && lambda <= 1.0))
    return fail(PPD_EINVAL, "ppd_primal_update: non-finite step or lambda outside (0, 1]");
  const int64_t n = int64_t(p->nx) * p->ny;
  hipLaunchKernelGGL(k_pu, dim3(ew_blocks(n)), dim3(256), 0, p->stream, n, x, a, b, tau, eta, zeta, lambda, x_out,
                     xt_out);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

extern "C" int ppd_primal_update_vjp(ppd_plan* p, const float* x, const float* a, const float* b, double tau,
                                     double eta, double zeta, double lambda, const float* gx_out,
                                     const float* gxt_out, float* g_x, float* g_a, float* g_b) {
  if (!p || !x || !a || !b) return fail(PPD_EINVAL, "ppd_primal_update_vjp: NULL argument");
  if (!std::isfinite(tau) || !std::isfinite(eta) || !std::isfinite(zeta) || !(lambda > 0.0 && lambda <= 1.0))
    return fail(PPD_EINVAL, "ppd_primal_update_vjp: non-finite step or lambda outside (0, 1]");
  const int64_t n = int64_t(p->nx) * p->ny;
  hipLaunchKernelGGL(k_pu_vjp, dim3(ew_blocks(n)), dim3(256), 0, p->stream, n, x, a, b, tau, eta, zeta, lambda,
                     gx_out, gxt_out, g_x, g_a, g_b);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}
