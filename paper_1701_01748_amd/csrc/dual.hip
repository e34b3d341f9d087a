// Data-fidelity dual update of Algorithm 3 and Algorithm 2,
// FP64: the standalone ellipsoid projection entry point, the unfused
// per-block ("plain") form of the dual update, and the uniform-weighting
// preconditioner (inverse local sampling density, Sec. 4.3).
#include <cmath>

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

// One Algorithm 2 iteration over every block, item by item (the item's
// segments flattened into batches of 64, as in the degridding).
//   mode 0: partials of ||q - y||^2, q = z - mu U (z - w)   (z unchanged)
//   mode 1: z <- P_B(q) with the block factors, then partials of the next q
//   mode 2: z <- P_B(q) only
// NW waves per workgroup: 1 for items of at most two batches (the 8 x 8
// default, 128 points: 4 waves left half of them idle, 296 against 242 us
// per iteration with n_itr = 5 at 512^2, 1.3M), else 4.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_alg2(
    int mode, const Item* __restrict__ items, int n_items, const Seg* __restrict__ segs,
    const double2* __restrict__ w, const float2* __restrict__ v, const float2* __restrict__ ga,
    const float2* __restrict__ y, const double* __restrict__ U,
    double2* __restrict__ z, double mu, const double2* __restrict__ bfac, const uint8_t* __restrict__ active,
    double* __restrict__ part_out, XcdSplit xs) {
  __shared__ ItemTab tab;
  __shared__ double s_q[NW][MAX_ITEM_SEGS];
  const int ii = xcd_unit(blockIdx.x, xs);
  if (ii < 0 || ii >= n_items) return;
  const Item it = items[ii];
  const int lane = threadIdx.x & 63;
  const int uwid = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  load_item_tab(it, segs, tab);
  for (int i = threadIdx.x; i < NW * MAX_ITEM_SEGS; i += blockDim.x) (&s_q[0][0])[i] = 0.0;
  __syncthreads();
  const int nseg = it.seg1 - it.seg0;
  const int total = tab.pre[nseg];
  int sb = 0;
  for (int bt = uwid; bt * 64 < total; bt += NW) {
    while (bt * 64 >= tab.pre[sb + 1]) ++sb;
    const int li = bt * 64 + lane;
    const bool act = li < total;
    const int sg = act ? seg_of(li, sb, tab.pre) : sb;
    double qn = 0.0;
    if (act) {
      const int pi = tab.start[sg] + (li - tab.pre[sg]);
      const double Ue = U[pi];
      const double2 we = w ? w[pi] : dual_arg(v[pi], Ue, ga[pi]);
      double2 ze = z[pi];
      const double mU = mu * Ue;
      const float2 ye = y[pi];
      // randomised updates of Algorithm 3: an inactive block keeps z
      if (mode != 0 && (!active || active[tab.block[sg]])) {
        const double2 bf = bfac[tab.block[sg]];
        const double qx = ze.x - mU * (ze.x - we.x), qy = ze.y - mU * (ze.y - we.y);
        ze.x = bf.y != 0.0 ? qx : double(ye.x) + (qx - double(ye.x)) * bf.x;
        ze.y = bf.y != 0.0 ? qy : double(ye.y) + (qy - double(ye.y)) * bf.x;
        z[pi] = ze;
      }
      if (mode != 2) {
        const double dx = (ze.x - mU * (ze.x - we.x)) - double(ye.x);
        const double dy = (ze.y - mU * (ze.y - we.y)) - double(ye.y);
        qn = dx * dx + dy * dy;
      }
    }
    if (mode != 2) {
      const int slast = __builtin_amdgcn_readlane(sg, min(63, total - 1 - bt * 64));
      for (int ss = sb; ss <= slast; ++ss) {
        const double a = wave_sum(act && sg == ss ? qn : 0.0);
        if (lane == 0) s_q[uwid][ss] += a;
      }
    }
  }
  if (mode != 2) {
    __syncthreads();
    for (int k = threadIdx.x; k < nseg; k += blockDim.x) {
      double q = 0.0;
#pragma unroll
      for (int wv = 0; wv < NW; ++wv) q += s_q[wv][k];
      part_out[it.seg0 + k] = q;
    }
  }
}

// Projection factor of every data block for P_B (Sec. 3.3, eq. proj-L2):
// workgroup j sums the segment partials of ||q - y_j||^2 in a fixed order
// and stores (eps_j / r, 0) if r > eps_j, else (1, 1).
constexpr int BF_PER = 8;
// One pass of 1024 threads covers up to 8192 segments (the largest block of
// the 512^2, 1.3M workload has ~3k); 256 threads took two passes there.
constexpr int BF_THREADS = 1024;
__global__ __launch_bounds__(BF_THREADS) void k_block_factors(const double* __restrict__ part,
                                                              const int32_t* __restrict__ bids,
                                                              const int32_t* __restrict__ boff,
                                                              const double* __restrict__ eps,
                                                              double2* __restrict__ bfac) {
  __shared__ double red[BF_THREADS / 64];
  const int j = blockIdx.x;
  const int c0 = boff[j], c1 = boff[j + 1];
  double s = 0.0;
  for (int base = c0; base < c1; base += BF_THREADS * BF_PER) {
    int id[BF_PER];
#pragma unroll
    for (int k = 0; k < BF_PER; ++k) {
      const int c = base + int(threadIdx.x) + k * BF_THREADS;
      id[k] = c < c1 ? bids[c] : -1;
    }
    double v[BF_PER];
#pragma unroll
    for (int k = 0; k < BF_PER; ++k) v[k] = id[k] >= 0 ? part[id[k]] : 0.0;
#pragma unroll
    for (int k = 0; k < BF_PER; ++k) s += v[k];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < BF_THREADS / 64; ++q) t += red[q];
    const double r = sqrt(t), e = eps[j];
    bfac[j] = r > e ? make_double2(e / r, 0.0) : make_double2(1.0, 1.0);
  }
}

// ---- persistent middle steps of Algorithm 2 ---------------------------------
// One launch runs the n_itr - 1 middle forward-backward steps of every block
// with the per-point state (w, z, U, y) held in registers: workgroup g owns
// the PA_CHUNK plan-order points from g PA_CHUNK (blocks are contiguous in
// plan order, so these span at most PA_MAXB blocks; the plan checks it).  A
// step applies z <- P_B(q) with the block factors and forms the workgroup's
// partial ||q - y_j||^2 of the next q per block it touches; every workgroup
// of block j then sums the block's workgroup partials in the same fixed
// order, so all of them get the same factor.  The grid is launched only when
// all its workgroups fit the device at once.
//
// There is no grid-wide barrier: a step of block j waits only for the
// partials of block j's workgroups.  Each partial is published in a slot of
// its own with one device-scope atomic exchange and carries its step in the
// sign bit (the partials are sums of squares, so the sign is free): slot
// s mod 2 of step s holds +p when bit 1 of s is clear and -p when it is set.
// A reader of step s finds in that slot either step s's partial (ready),
// step s - 2's (the writer is behind; it can never be ahead, because its
// step s + 1 needs the reader's own step s + 1 partial) or a NaN left by the
// previous launch's reset (step 0 and 1), so the sign tells them apart.  The
// wait is bounded: a thread that has polled spin_limit times sets a give-up
// flag that every other waiter checks, all workgroups run to the end, and
// the host reports the flag.  The last workgroup out puts NaN back into
// every slot for the next launch (the plan starts them at NaN).
#ifndef PPD_PA_SLEEP
#define PPD_PA_SLEEP 1   // s_sleep argument between polls (units of 64 clocks)
#endif
struct PaArgs {
  int steps, G, d, spin_limit;
  int64_t M;
  double mu;
  const float2* v; const float2* ga; const float2* y; const double* U;
  double2* z;
  const uint8_t* active;
  const int32_t* voff; const int32_t* wgb0; const int32_t* gfirst; const int32_t* glast;
  const double* eps;
  double2* bfac;
  uint64_t* part;   // [2][G][PA_MAXB] tagged partials
  uint32_t* sync;   // [1] exits, [2] give-up flag
};

// Waits for the tagged partial in *slot; returns its value, or -1 after a
// give-up (polls exceeded here, or the flag raised elsewhere).
__device__ double pa_wait(uint64_t* slot, uint64_t tag, uint32_t* sync, int spin_limit) {
  int polls = 0;
  while (true) {
    const uint64_t b = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (b != PA_EMPTY && (b & PA_SIGN) == tag) return __longlong_as_double(int64_t(b & ~PA_SIGN));
    if ((polls & 31) == 31 && __hip_atomic_load(&sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return -1.0;
    if (++polls > spin_limit) {
      __hip_atomic_store(&sync[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return -1.0;
    }
#if PPD_PA_SLEEP > 0
    __builtin_amdgcn_s_sleep(PPD_PA_SLEEP);
#endif
  }
}

__global__ __launch_bounds__(PA_THREADS) void k_alg2_persistent(PaArgs a) {
  static_assert(PA_THREADS == 256, "partials are summed over exactly 4 waves");
  __shared__ double red[PA_THREADS / 64][PA_MAXB];
  __shared__ double2 fac[PA_MAXB];
  __shared__ int act[PA_MAXB];
  __shared__ int quit;
  const int g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = int64_t(g) * PA_CHUNK;
  const int64_t i1 = min(i0 + PA_CHUNK, a.M);
  const int b0 = a.wgb0[g];
  int nb = 1;
  while (nb < PA_MAXB && b0 + nb < a.d && a.voff[b0 + nb] < i1) ++nb;
  double2 w[PA_PER], z[PA_PER];
  double U[PA_PER];
  float2 y[PA_PER];
  int sl[PA_PER];
#pragma unroll
  for (int k = 0; k < PA_PER; ++k) {
    const int64_t i = i0 + int64_t(k) * PA_THREADS + tid;
    sl[k] = -1;
    if (i < i1) {
      U[k] = a.U[i];
      w[k] = dual_arg(a.v[i], U[k], a.ga[i]);
      z[k] = a.z[i];
      y[k] = a.y[i];
      int b = 0;
      while (b + 1 < nb && i >= a.voff[b0 + b + 1]) ++b;
      sl[k] = b;
    }
  }
  // factors of the first middle step (from the degridding's partials)
  if (tid < nb) {
    fac[tid] = a.bfac[b0 + tid];
    act[tid] = !a.active || a.active[b0 + tid];
  }
  if (tid == 0) quit = 0;
  __syncthreads();
  for (int s = 0; s < a.steps; ++s) {
    double acc[PA_MAXB];
#pragma unroll
    for (int b = 0; b < PA_MAXB; ++b) acc[b] = 0.0;
#pragma unroll
    for (int k = 0; k < PA_PER; ++k) {
      if (sl[k] < 0) continue;
      const int b = sl[k];
      const double mU = a.mu * U[k];
      if (act[b]) {
        const double2 f = fac[b];
        const double qx = z[k].x - mU * (z[k].x - w[k].x), qy = z[k].y - mU * (z[k].y - w[k].y);
        z[k].x = f.y != 0.0 ? qx : double(y[k].x) + (qx - double(y[k].x)) * f.x;
        z[k].y = f.y != 0.0 ? qy : double(y[k].y) + (qy - double(y[k].y)) * f.x;
      }
      const double dx = (z[k].x - mU * (z[k].x - w[k].x)) - double(y[k].x);
      const double dy = (z[k].y - mU * (z[k].y - w[k].y)) - double(y[k].y);
      const double q2 = dx * dx + dy * dy;
#pragma unroll
      for (int bb = 0; bb < PA_MAXB; ++bb) acc[bb] += bb == b ? q2 : 0.0;
    }
    // the workgroup's partial per block, summed in a fixed order
#pragma unroll
    for (int b = 0; b < PA_MAXB; ++b) {
      const double t = wave_sum(acc[b]);
      if (lane == 0) red[wid][b] = t;
    }
    __syncthreads();
    uint64_t* part = a.part + size_t(s & 1) * size_t(a.G) * PA_MAXB;
    const uint64_t tag = (s & 2) ? PA_SIGN : 0ull;
    if (wid == 0) {
      // this wave's earlier exchanges (steps s - 1, s - 2) are acknowledged
      // before the slot of step s - 2 is overwritten
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    if (tid < nb) {
      const double p = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      // a NaN partial (diverged data) must not read as an empty slot
      uint64_t bits = uint64_t(__double_as_longlong(p)) & ~PA_SIGN;
      if (bits == PA_EMPTY) bits |= 1ull;
      (void)__hip_atomic_exchange(&part[size_t(g) * PA_MAXB + tid], bits | tag, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }
    // the factors of this workgroup's blocks from all their workgroups' partials
    for (int b = 0; b < nb; ++b) {
      const int j = b0 + b;
      double t = 0.0;
      int bad = 0;
      for (int gg = a.gfirst[j] + tid; gg <= a.glast[j]; gg += PA_THREADS) {
        const double v = pa_wait(&part[size_t(gg) * PA_MAXB + (j - a.wgb0[gg])], tag, a.sync, a.spin_limit);
        if (v < 0.0) bad = 1;
        else t += v;
      }
      t = wave_sum(t);
      __syncthreads();   // red is free again
      if (lane == 0) red[wid][0] = t;
      if (bad) quit = 1;
      __syncthreads();
      if (tid == 0) {
        const double r = sqrt(((red[0][0] + red[1][0]) + red[2][0]) + red[3][0]), e = a.eps[j];
        fac[b] = r > e ? make_double2(e / r, 0.0) : make_double2(1.0, 1.0);
      }
    }
    __syncthreads();
    if (quit) break;   // uniform: read after the barrier
  }
#pragma unroll
  for (int k = 0; k < PA_PER; ++k) {
    const int64_t i = i0 + int64_t(k) * PA_THREADS + tid;
    if (sl[k] >= 0 && act[sl[k]]) a.z[i] = z[k];
  }
  // the last step's factors, for the final projection in the gridding:
  // stored by the first workgroup of each block (all others hold the same)
  if (tid < nb && a.gfirst[b0 + tid] == g) a.bfac[b0 + tid] = fac[tid];
  // the last workgroup out empties every slot for the next launch and clears
  // the exit count
  __shared__ int last_out;
  if (tid == 0) {
    // the partials this wave published are acknowledged before the exit
    // is counted, so that the reset cannot be overtaken by one of them
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const uint32_t out = __hip_atomic_fetch_add(&a.sync[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last_out = out == uint32_t(a.G) - 1u;
  }
  __syncthreads();
  if (last_out) {
    for (size_t e = tid; e < 2 * size_t(a.G) * PA_MAXB; e += PA_THREADS)
      __hip_atomic_store(&a.part[e], PA_EMPTY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) __hip_atomic_store(&a.sync[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- exact prox of eq. elip-proj-1: Newton on the secular equation ------
// With a = U |w - y| and r(nu)^2 = sum a^2 / (U + nu)^2 per block, the prox
// is (U w + nu y) / (U + nu) at the root of g(nu) = 1 / r(nu) - 1 / eps
// (nu = 0 when r(0) <= eps).  g is concave and increasing, so Newton from
// nu = 0 climbs to the root without overshooting; g'(nu) = S3 / r^3 with
// S3 = sum a^2 / (U + nu)^3.  bfac[j].x carries nu between the passes.

// A pass runs over chunks of SEC_CHUNK consecutive plan-order points inside
// one block (blocks are contiguous in plan order).  The first pass forms
// a^2 = U^2 |w - y|^2 and keeps (a^2, U) per point, the later ones read only
// that (16 bytes per point); each workgroup writes its chunk's S2, S3 at the
// block's current nu, summed in a fixed order (deterministic).  A later
// pass first takes the Newton step from the previous pass's partials
// itself (every workgroup of a block computes the same value in the same
// order), so one launch per step remains; partials and nu alternate
// between two buffers, and a last k_sec_update takes the final step.
constexpr int SEC_THREADS = 256;

// Newton step of block j from its chunk partials [c0, c1): nu = max(0, nu0
// - g / g'), g = 1 / r - 1 / eps.  All SEC_THREADS threads take part; the
// result is returned to every thread.
__device__ double newton_nu(const double* __restrict__ p2, const double* __restrict__ p3, int c0, int c1,
                            double eps, double nu0, double* red2, double* red3, double* out) {
  double a = 0.0, b = 0.0;
  for (int c = c0 + int(threadIdx.x); c < c1; c += SEC_THREADS) {
    a += p2[c];
    b += p3[c];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    red2[threadIdx.x >> 6] = a;
    red3[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double S2 = 0.0, S3 = 0.0;
#pragma unroll
    for (int k = 0; k < SEC_THREADS / 64; ++k) {
      S2 += red2[k];
      S3 += red3[k];
    }
    double nu = 0.0;
    if (S2 > 0.0 && S3 > 0.0) {
      const double r = sqrt(S2);
      const double g = 1.0 / r - 1.0 / eps, gp = S3 / (r * r * r);
      nu = fmax(0.0, nu0 - g / gp);
    }
    *out = nu;
  }
  __syncthreads();
  return *out;
}

// FIRST: nu = 0.  Else the step from the previous partials (pp2, pp3) and
// the previous nu (pnu, NULL after the first pass); the chunk that starts
// its block stores the new nu to nnu.
template <bool FIRST>
__global__ __launch_bounds__(SEC_THREADS) void k_sec_chunk(
    const int32_t* __restrict__ cstart, const int32_t* __restrict__ cblock, const int32_t* __restrict__ coff,
    const double* __restrict__ eps, const double2* __restrict__ w, const float2* __restrict__ v,
    const float2* __restrict__ ga, const float2* __restrict__ y, const double* __restrict__ U,
    double2* __restrict__ aq, const double* __restrict__ pp2, const double* __restrict__ pp3,
    const double* __restrict__ pnu, double* __restrict__ nnu, double* __restrict__ p2, double* __restrict__ p3) {
  __shared__ double red2[SEC_THREADS / 64], red3[SEC_THREADS / 64], s_nu;
  const int c = blockIdx.x;
  const int i0 = cstart[c], i1 = cstart[c + 1];
  double nu = 0.0;
  if (!FIRST) {
    const int j = cblock[c];
    nu = newton_nu(pp2, pp3, coff[j], coff[j + 1], eps[j], pnu ? pnu[j] : 0.0, red2, red3, &s_nu);
    if (c == coff[j] && threadIdx.x == 0) nnu[j] = nu;
  }
  double t2 = 0.0, t3 = 0.0;
#pragma unroll 4
  for (int i = i0 + int(threadIdx.x); i < i1; i += SEC_THREADS) {
    double a2, Ue;
    if (FIRST) {
      Ue = U[i];
      const double2 we = w ? w[i] : dual_arg(v[i], Ue, ga[i]);
      const float2 ye = y[i];
      const double dx = we.x - double(ye.x), dy = we.y - double(ye.y);
      a2 = Ue * Ue * (dx * dx + dy * dy);
      aq[i] = make_double2(a2, Ue);
    } else {
      const double2 q = aq[i];
      a2 = q.x;
      Ue = q.y;
    }
    const double inv = 1.0 / (Ue + nu);
    const double s2 = a2 * inv * inv;
    t2 += s2;
    t3 += s2 * inv;
  }
  t2 = wave_sum(t2);
  t3 = wave_sum(t3);
  __syncthreads();   // red2 / red3 reused after newton_nu
  if ((threadIdx.x & 63) == 0) {
    red2[threadIdx.x >> 6] = t2;
    red3[threadIdx.x >> 6] = t3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int k = 0; k < SEC_THREADS / 64; ++k) {
      a += red2[k];
      b += red3[k];
    }
    p2[c] = a;
    p3[c] = b;
  }
}

// The last Newton step: workgroup j takes it from the last pass's partials
// and stores nu_j to the block factors.
__global__ __launch_bounds__(SEC_THREADS) void k_sec_update(const double* __restrict__ p2,
                                                            const double* __restrict__ p3,
                                                            const int32_t* __restrict__ coff,
                                                            const double* __restrict__ eps,
                                                            const double* __restrict__ pnu,
                                                            double2* __restrict__ bfac) {
  __shared__ double red2[SEC_THREADS / 64], red3[SEC_THREADS / 64], s_nu;
  const int j = blockIdx.x;
  const double nu = newton_nu(p2, p3, coff[j], coff[j + 1], eps[j], pnu ? pnu[j] : 0.0, red2, red3, &s_nu);
  if (threadIdx.x == 0) bfac[j] = make_double2(nu, 0.0);
}

// z = (U w + nu y) / (U + nu) with the block's nu (z = w when nu = 0).
__global__ void k_prox_apply(int64_t M, const int32_t* __restrict__ vblk, const double2* __restrict__ w,
                             const float2* __restrict__ y, const double* __restrict__ U,
                             const double2* __restrict__ bfac, double2* __restrict__ z) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const double nu = bfac[vblk[i]].x, Ue = U[i];
    const double2 we = w[i];
    const float2 ye = y[i];
    const double inv = 1.0 / (Ue + nu);
    z[i] = nu == 0.0 ? we   // inside the ellipsoid: the prox is w itself
                     : make_double2((Ue * we.x + nu * double(ye.x)) * inv, (Ue * we.y + nu * double(ye.y)) * inv);
  }
}

// ---- plain form: one block at a time, each step its own launch ---------
constexpr int PL_THREADS = 256;
constexpr int PL_MAX_BLOCKS = 512;

// w = U^-1 v + yhat, and partials of ||yhat - y||^2 (residual statistics)
__global__ void k_pl_w(int64_t b0, int64_t b1, const float2* __restrict__ v, const double* __restrict__ U,
                       const float2* __restrict__ yhat, const float2* __restrict__ y,
                       double2* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[16];
  double rn = 0.0;
  for (int64_t i = b0 + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < b1; i += int64_t(gridDim.x) * blockDim.x) {
    const float2 ve = v[i], g = yhat[i], ye = y[i];
    const double Ue = U[i];
    w[i] = dual_arg(ve, Ue, g);
    const double ex = double(g.x) - double(ye.x), ey = double(g.y) - double(ye.y);
    rn += ex * ex + ey * ey;
  }
  rn = block_sum(rn, red);
  if (threadIdx.x == 0) part[blockIdx.x] = rn;
}

// q = z - mu U (z - w) and partials of ||q - y||^2
__global__ void k_pl_q(int64_t b0, int64_t b1, const double2* __restrict__ w, const double2* __restrict__ z,
                       const double* __restrict__ U, const float2* __restrict__ y, double mu,
                       double2* __restrict__ q, double* __restrict__ part) {
  __shared__ double red[16];
  double qn = 0.0;
  for (int64_t i = b0 + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < b1; i += int64_t(gridDim.x) * blockDim.x) {
    const double2 we = w[i], ze = z[i];
    const double mU = mu * U[i];
    const double qx = ze.x - mU * (ze.x - we.x), qy = ze.y - mU * (ze.y - we.y);
    q[i] = make_double2(qx, qy);
    const float2 ye = y[i];
    const double dx = qx - double(ye.x), dy = qy - double(ye.y);
    qn += dx * dx + dy * dy;
  }
  qn = block_sum(qn, red);
  if (threadIdx.x == 0) part[blockIdx.x] = qn;
}

// out[slot] = sum of n partials (one wave, fixed order)
__global__ void k_pl_reduce(const double* __restrict__ part, int n, double* __restrict__ out, int slot) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += part[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (threadIdx.x == 0) out[slot] = s;
}

// z = P_B(q) (Sec. 3.3, eq. proj-L2) with ||q - y||^2 in *norm2
__global__ void k_pl_proj(int64_t b0, int64_t b1, const double2* __restrict__ q, const float2* __restrict__ y,
                          const double* __restrict__ norm2, const double* __restrict__ eps, int j,
                          double2* __restrict__ z) {
  const double r = sqrt(*norm2), e = eps[j];
  const bool inside = r <= e;
  const double f = inside ? 1.0 : e / r;
  for (int64_t i = b0 + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < b1; i += int64_t(gridDim.x) * blockDim.x) {
    const double2 qe = q[i];
    if (inside) {
      z[i] = qe;
    } else {
      const float2 ye = y[i];
      z[i] = make_double2(double(ye.x) + (qe.x - double(ye.x)) * f, double(ye.y) + (qe.y - double(ye.y)) * f);
    }
  }
}

// vbar = U (w - z); v <- v + lambda (vbar - v)
__global__ void k_pl_finish(int64_t b0, int64_t b1, const double2* __restrict__ w, const double2* __restrict__ z,
                            const double* __restrict__ U, double lambda, float2* __restrict__ v) {
  for (int64_t i = b0 + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < b1; i += int64_t(gridDim.x) * blockDim.x) {
    const double2 we = w[i], ze = z[i];
    const double Ue = U[i];
    const float2 vo = v[i];
    const double vbx = Ue * (we.x - ze.x), vby = Ue * (we.y - ze.y);
    v[i] = make_float2(float(double(vo.x) + lambda * (vbx - double(vo.x))),
                       float(double(vo.y) + lambda * (vby - double(vo.y))));
  }
}

// ---- uniform-weighting preconditioner ----------------------------------
__device__ __forceinline__ int density_cell(float w, int n) {
  // floor((w + pi) n / (2 pi)), evaluated exactly in this order, clamped
  const double a = __dadd_rn(double(w), M_PI);
  const double b = __dmul_rn(a, double(n));
  const double c = __ddiv_rn(b, 2.0 * M_PI);
  int i = int(floor(c));
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

__global__ void k_hist(const float* __restrict__ wu, const float* __restrict__ wv, int64_t M, int nx, int ny,
                       int32_t* __restrict__ counts) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const int cu = density_cell(wu[i], nx), cv = density_cell(wv[i], ny);
    atomicAdd(&counts[cv * nx + cu], 1);
  }
}

__global__ void k_hist_min(const float* __restrict__ wu, const float* __restrict__ wv, int64_t M, int nx, int ny,
                           const int32_t* __restrict__ counts, int32_t* __restrict__ cmin) {
  int m = 0x7fffffff;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const int cu = density_cell(wu[i], nx), cv = density_cell(wv[i], ny);
    m = min(m, counts[cv * nx + cu]);
  }
  for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMin(cmin, m);
}

__global__ void k_hist_u(const float* __restrict__ wu, const float* __restrict__ wv, int64_t M, int nx, int ny,
                         const int32_t* __restrict__ counts, const int32_t* __restrict__ cmin,
                         double* __restrict__ U) {
  const double c0 = double(*cmin);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const int cu = density_cell(wu[i], nx), cv = density_cell(wv[i], ny);
    U[i] = c0 / double(counts[cv * nx + cu]);
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) a[i] = v;
}

int grid_blocks(int64_t n) { return int(std::min<int64_t>((n + PL_THREADS - 1) / PL_THREADS, PL_MAX_BLOCKS)); }

}  // namespace

int alg2_launch(ppd_plan* p, int mode, const double2* w, const float2* v, const float2* ga, const float2* y,
                const double* U, double2* z, double mu, const double* part_in, double* part_out,
                const uint8_t* active) {
  if (mode != 0) PPD_TRY(block_factors(p, part_in));
  int slot;
  PPD_TRY(timer_begin(p, KK_SUBITER, &slot));
  if (p->chunk_max <= 128)
    hipLaunchKernelGGL(k_alg2<1>, dim3(p->split1.launch), dim3(64), 0, p->stream, mode, p->items, p->n_items,
                       p->segs, w, v, ga, y, U, z, mu, p->bfac, active, part_out, p->split1);
  else
    hipLaunchKernelGGL(k_alg2<4>, dim3(p->split1.launch), dim3(256), 0, p->stream, mode, p->items, p->n_items,
                       p->segs, w, v, ga, y, U, z, mu, p->bfac, active, part_out, p->split1);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

int secular_solve(ppd_plan* p, const double2* w, const float2* v, const float2* ga, const float2* y,
                  const double* U, int n_newton) {
  // pass s writes its partials to buffer s & 1 and (s >= 1) its nu to
  // nu buffer s & 1
  const int nc = p->n_sec_chunks;
  double* part[2] = {p->sec_part, p->sec_part + 2 * nc};
  double* nub[2] = {p->sec_nu, p->sec_nu + p->d};
  for (int s = 0; s < n_newton; ++s) {
    double* p2 = part[s & 1];
    double* p3 = part[s & 1] + nc;
    const double* q2 = part[(s + 1) & 1];
    const double* q3 = part[(s + 1) & 1] + nc;
    const double* pnu = s >= 2 ? nub[(s + 1) & 1] : nullptr;
    int slot;
    PPD_TRY(timer_begin(p, KK_SUBITER, &slot));
    if (s == 0)
      hipLaunchKernelGGL(k_sec_chunk<true>, dim3(nc), dim3(SEC_THREADS), 0, p->stream, p->sec_cstart, p->sec_cblock,
                         p->sec_coff, p->eps_d, w, v, ga, y, U, p->qbuf, nullptr, nullptr, nullptr, nullptr, p2, p3);
    else
      hipLaunchKernelGGL(k_sec_chunk<false>, dim3(nc), dim3(SEC_THREADS), 0, p->stream, p->sec_cstart,
                         p->sec_cblock, p->sec_coff, p->eps_d, w, v, ga, y, U, p->qbuf, q2, q3, pnu, nub[s & 1], p2,
                         p3);
    PPD_HIP(hipGetLastError());
    PPD_TRY(timer_end(p, slot));
  }
  const int last = n_newton - 1;
  int slot;
  PPD_TRY(timer_begin(p, KK_MISC, &slot));
  hipLaunchKernelGGL(k_sec_update, dim3(p->d), dim3(SEC_THREADS), 0, p->stream, part[last & 1],
                     part[last & 1] + nc, p->sec_coff, p->eps_d, last >= 1 ? nub[last & 1] : nullptr, p->bfac);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

int alg2_persistent_capacity() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_alg2_persistent),
                                                   PA_THREADS, 0) != hipSuccess)
    return 0;
  return cus * per;
}

int alg2_persistent(ppd_plan* p, const DualArgs& a, int spin_limit) {
  if (!p->pa_ok) return fail(PPD_EUNSUPPORTED, "persistent Algorithm 2 is not available for this plan");
  PaArgs pa;
  pa.steps = a.n_itr - 1;
  pa.G = p->pa_groups;
  pa.d = p->d;
  pa.spin_limit = spin_limit > 0 ? spin_limit : (1 << 20);
  pa.M = p->M;
  pa.mu = a.mu;
  pa.v = a.v;
  pa.ga = p->gabuf;
  pa.y = a.y;
  pa.U = a.U;
  pa.z = a.z;
  pa.active = a.active;
  pa.voff = p->voff_d;
  pa.wgb0 = p->pa_wgb0;
  pa.gfirst = p->pa_gfirst;
  pa.glast = p->pa_glast;
  pa.eps = p->eps_d;
  pa.bfac = p->bfac;
  pa.part = p->pa_part;
  pa.sync = p->pa_sync;
  int slot;
  PPD_TRY(timer_begin(p, KK_SUBITER, &slot));
  hipLaunchKernelGGL(k_alg2_persistent, dim3(pa.G), dim3(PA_THREADS), 0, p->stream, pa);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

int block_factors(ppd_plan* p, const double* part) {
  int slot;
  PPD_TRY(timer_begin(p, KK_MISC, &slot));
  hipLaunchKernelGGL(k_block_factors, dim3(p->d), dim3(BF_THREADS), 0, p->stream, part, p->bseg_ids, p->bseg_off_d,
                     p->eps_d, p->bfac);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

// Unfused reference form of the data-dual update: per block, per sub-iteration,
// separate FP64 launches.  Expects Theta G F Z x~ in p->ybuf (plan order).
int plain_dual(ppd_plan* p, const DualArgs& a) {
  for (int j = 0; j < p->d; ++j) {
    const int64_t b0 = p->block_off[j], b1 = p->block_off[j + 1];
    const int G = grid_blocks(b1 - b0);
    int slot;
    PPD_TRY(timer_begin(p, KK_PLAIN_DUAL, &slot));
    hipLaunchKernelGGL(k_pl_w, dim3(G), dim3(PL_THREADS), 0, p->stream, b0, b1, a.v, a.U, p->ybuf, a.y,
                       p->wbuf, p->pl_part);
    hipLaunchKernelGGL(k_pl_reduce, dim3(1), dim3(64), 0, p->stream, p->pl_part, G, p->res_sq, j);
    for (int s = 0; s < a.n_itr; ++s) {
      hipLaunchKernelGGL(k_pl_q, dim3(G), dim3(PL_THREADS), 0, p->stream, b0, b1, p->wbuf, a.z, a.U, a.y,
                         a.mu, p->qbuf, p->pl_part);
      hipLaunchKernelGGL(k_pl_reduce, dim3(1), dim3(64), 0, p->stream, p->pl_part, G, p->pl_scalar, 0);
      hipLaunchKernelGGL(k_pl_proj, dim3(G), dim3(PL_THREADS), 0, p->stream, b0, b1, p->qbuf, a.y,
                         p->pl_scalar, p->eps_d, j, a.z);
    }
    hipLaunchKernelGGL(k_pl_finish, dim3(G), dim3(PL_THREADS), 0, p->stream, b0, b1, p->wbuf, a.z, a.U,
                       a.lambda, a.v);
    PPD_HIP(hipGetLastError());
    PPD_TRY(timer_end(p, slot));
  }
  return PPD_OK;
}

}  // namespace ppd

using namespace ppd;

extern "C" int ppd_ellipsoid_proj(ppd_plan* p, const double* w, const float* y, const double* U,
                                  const double* eps, int n_itr, double mu, double* zbar) {
  if (!p || !w || !y || !U || !eps || !zbar) return fail(PPD_EINVAL, "ppd_ellipsoid_proj: NULL argument");
  if (n_itr < 1) return fail(PPD_EINVAL, "ppd_ellipsoid_proj: n_itr must be >= 1");
  if (!(mu > 0.0) || !std::isfinite(mu)) return fail(PPD_EINVAL, "ppd_ellipsoid_proj: mu must be > 0");
  PPD_TRY(upload_eps(p, eps));
  const double2* w2 = reinterpret_cast<const double2*>(w);
  const float2* y2 = reinterpret_cast<const float2*>(y);
  double2* z2 = reinterpret_cast<double2*>(zbar);
  double* pa = p->part;
  double* pb = p->part + p->n_segs;
  PPD_TRY(alg2_launch(p, 0, w2, nullptr, nullptr, y2, U, z2, mu, nullptr, pa, nullptr));
  for (int s = 1; s < n_itr; ++s) {
    PPD_TRY(alg2_launch(p, 1, w2, nullptr, nullptr, y2, U, z2, mu, pa, pb, nullptr));
    std::swap(pa, pb);
  }
  return alg2_launch(p, 2, w2, nullptr, nullptr, y2, U, z2, mu, pa, nullptr, nullptr);
}

extern "C" int ppd_prox_metric(ppd_plan* p, const double* w, const float* y, const double* U, const double* eps,
                               int n_newton, double* z, double* nu) {
  if (!p || !w || !y || !U || !eps || !z) return fail(PPD_EINVAL, "ppd_prox_metric: NULL argument");
  if (n_newton < 1 || n_newton > 64) return fail(PPD_EINVAL, "ppd_prox_metric: n_newton must be in [1, 64]");
  PPD_TRY(upload_eps(p, eps));
  const double2* w2 = reinterpret_cast<const double2*>(w);
  const float2* y2 = reinterpret_cast<const float2*>(y);
  PPD_TRY(secular_solve(p, w2, nullptr, nullptr, y2, U, n_newton));
  int slot;
  PPD_TRY(timer_begin(p, KK_MISC, &slot));
  hipLaunchKernelGGL(k_prox_apply, dim3(int(std::min<int64_t>((p->M + 255) / 256, 4096))), dim3(256), 0, p->stream,
                     p->M, p->vis_block, w2, y2, U, p->bfac, reinterpret_cast<double2*>(z));
  PPD_HIP(hipGetLastError());
  PPD_TRY(timer_end(p, slot));
  if (nu) {
    PPD_HIP(hipMemcpy2DAsync(nu, sizeof(double), p->bfac, sizeof(double2), sizeof(double), p->d,
                             hipMemcpyDeviceToDevice, p->stream));
  }
  return PPD_OK;
}

extern "C" int ppd_uniform_weights(ppd_plan* p, double* U) {
  if (!p || !U) return fail(PPD_EINVAL, "ppd_uniform_weights: NULL argument");
  int slot;
  PPD_TRY(timer_begin(p, KK_HIST, &slot));
  const int64_t N = int64_t(p->nx) * p->ny;
  const int gb = int(std::min<int64_t>((p->M + 255) / 256, 2048));
  hipLaunchKernelGGL(k_fill_i32, dim3(int(std::min<int64_t>((N + 255) / 256, 2048))), dim3(256), 0,
                     p->stream, p->icount, N, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, p->stream, p->imin, int64_t(1), 0x7fffffff);
  hipLaunchKernelGGL(k_hist, dim3(gb), dim3(256), 0, p->stream, p->wu, p->wv, p->M, p->nx, p->ny, p->icount);
  hipLaunchKernelGGL(k_hist_min, dim3(gb), dim3(256), 0, p->stream, p->wu, p->wv, p->M, p->nx, p->ny,
                     p->icount, p->imin);
  hipLaunchKernelGGL(k_hist_u, dim3(gb), dim3(256), 0, p->stream, p->wu, p->wv, p->M, p->nx, p->ny,
                     p->icount, p->imin, U);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}
