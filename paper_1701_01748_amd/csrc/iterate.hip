// Algorithm 3 driver (PPD; PD when U = 1), FP64 statistics, the operator
// norm of U^1/2 Phi by power iteration, and HIP-graph replay of one
// iteration.
#include <cmath>
#include <cstdio>
#include <string>

#include "ppd_internal.h"

namespace ppd {

int primal_partial_count(ppd_plan* p);
int alg2_launch(ppd_plan* p, int mode, const double2* w, const float2* v, const float2* ga, const float2* y,
                const double* U, double2* z, double mu, const double* part_in, double* part_out,
                const uint8_t* active);

namespace {

// One workgroup of 64 threads: statistics of the last iteration.
// Block residuals r_j = ||Theta_j G_j F Z x~ - y_j|| of the statistics:
// workgroup j sums block j's segment partials (one pass of 1024 threads
// over up to 8192 segments, fixed order), or takes the plain form's sum.
constexpr int STAT_THREADS = 1024, STAT_PER = 8;
// The statistics of a call go to out, or with a cursor to row *cursor of a
// history with rows of `stride` doubles (k_stats advances the cursor), so
// that a captured graph can write a new row at every replay.
__global__ __launch_bounds__(STAT_THREADS) void k_stats_resid(const double* __restrict__ rpart,
                                                              const int32_t* __restrict__ bids,
                                                              const int32_t* __restrict__ boff,
                                                              const double* __restrict__ res_sq, int use_res_sq,
                                                              double* __restrict__ out_base,
                                                              const int32_t* __restrict__ cursor, int stride,
                                                              double* __restrict__ rj) {
  __shared__ double red[STAT_THREADS / 64];
  double* out = out_base + (cursor ? size_t(*cursor) * stride : 0);
  const int j = blockIdx.x;
  double r2 = 0.0;
  if (use_res_sq) {
    r2 = res_sq[j];
  } else {
    const int c0 = boff[j], c1 = boff[j + 1];
    for (int base = c0; base < c1; base += STAT_THREADS * STAT_PER) {
      int id[STAT_PER];
#pragma unroll
      for (int k = 0; k < STAT_PER; ++k) {
        const int c = base + int(threadIdx.x) + k * STAT_THREADS;
        id[k] = c < c1 ? bids[c] : -1;
      }
#pragma unroll
      for (int k = 0; k < STAT_PER; ++k) r2 += id[k] >= 0 ? rpart[id[k]] : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) r2 += __shfl_xor(r2, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2;
    __syncthreads();
    r2 = 0.0;
    for (int q = 0; q < STAT_THREADS / 64; ++q) r2 += red[q];
  }
  if (threadIdx.x == 0) {
    out[8 + j] = sqrt(r2);
    rj[j] = sqrt(r2);   // a device copy for k_stats (out may be host memory)
  }
}

// out: [0] rel change, [1] ||x||, [2] SNR dB, [3] max_j r_j / eps_j,
//      [4..7] raw sums, [8 + j] r_j (from k_stats_resid).
__global__ __launch_bounds__(256) void k_stats(const double* __restrict__ ppart, int nparts,
                                               const double* __restrict__ eps, int d, int has_truth,
                                               double* __restrict__ out_base, int32_t* __restrict__ cursor,
                                               int stride, const uint32_t* __restrict__ flag,
                                               const double* __restrict__ rj) {
  __shared__ double red[4][4];
  double* out = out_base + (cursor ? size_t(*cursor) * stride : 0);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nparts; i += 256)
    for (int k = 0; k < 4; ++k) s[k] += ppart[4 * i + k];
  for (int k = 0; k < 4; ++k)
    for (int o = 32; o > 0; o >>= 1) s[k] += __shfl_xor(s[k], o);
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) red[threadIdx.x >> 6][k] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) s[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    double rmax = 0.0;
    for (int j = 0; j < d; ++j) rmax = fmax(rmax, rj[j] / eps[j]);
    // ||x_t - x_{t-1}|| / ||x_t||, 0 when both vanish (an all-zero iterate)
    out[0] = sqrt(s[0]) / fmax(sqrt(s[1]), 1e-300);
    out[1] = sqrt(s[1]);
    out[2] = has_truth ? 20.0 * log10(sqrt(s[3] / s[2])) : __builtin_nan("");
    out[3] = rmax;
    out[4] = s[0];
    out[5] = s[1];
    out[6] = s[2];
    out[7] = s[3];
    if (cursor) *cursor += 1;
    if (flag) out[8 + d] = double(*flag);   // the persistent launch's give-up flag, read back with them
  }
}

__global__ void k_set_i32(int32_t* __restrict__ a, int32_t v) { *a = v; }

__global__ void k_img_norm2(const float* __restrict__ a, int64_t n, double* __restrict__ part) {
  double s = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double v = a[i];
    s += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += part[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_img_scale(const float* __restrict__ a, int64_t n, double s, float* __restrict__ b) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = float(double(a[i]) * s);
}

__global__ void k_vis_mul_U(float2* __restrict__ y, const double* __restrict__ U, int64_t M) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < M; i += int64_t(gridDim.x) * blockDim.x) {
    const float2 v = y[i];
    const double u = U[i];
    y[i] = make_float2(float(double(v.x) * u), float(double(v.y) * u));
  }
}

int img_norm(ppd_plan* p, const float* a, double* out_host) {
  const int64_t n = int64_t(p->nx) * p->ny;
  const int G = int(std::min<int64_t>((n + 255) / 256, 512));
  hipLaunchKernelGGL(k_img_norm2, dim3(G), dim3(256), 0, p->stream, a, n, p->pl_part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, p->stream, p->pl_part, G, p->pl_scalar);
  PPD_HIP(hipGetLastError());
  double v = 0.0;
  PPD_HIP(hipMemcpyAsync(&v, p->pl_scalar, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  PPD_HIP(hipStreamSynchronize(p->stream));
  *out_host = std::sqrt(v);
  return PPD_OK;
}

int img_scale(ppd_plan* p, const float* a, double s, float* b) {
  const int64_t n = int64_t(p->nx) * p->ny;
  hipLaunchKernelGGL(k_img_scale, dim3(int(std::min<int64_t>((n + 255) / 256, 2048))), dim3(256), 0,
                     p->stream, a, n, s, b);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}

struct IterCtx {
  DualArgs dual;
  PrimalArgs primal;
  float* u;
  const float* W;
  float alpha, lambda;
  int form;
  int prox, n_newton;
  const uint8_t* basis_active;
  bool sara_forked;   // SARA on the second stream (eager), else the data path (graph)
  bool persistent;    // Algorithm 2 middle steps in one persistent launch
  int spin_limit;     // polls per wait of the persistent launch (0: default)
  // statistics reduced right after the iteration (captured graphs): into
  // stats_out, at the plan's history cursor if stats_cursor
  double* stats_out = nullptr;
  bool stats_cursor = false;
  int has_truth = 0, use_res_sq = 0;
};

// Runs the plan's launches on another stream for the lifetime of the object.
struct OnStream {
  ppd_plan* p;
  hipStream_t saved;
  OnStream(ppd_plan* pl, hipStream_t s) : p(pl), saved(pl->stream) { p->stream = s; }
  ~OnStream() { p->stream = saved; }
};

// The data-fidelity path of one iteration (F Z x~, the data-dual update
// of every block and the gridding, then the inverse column FFT of the
// primal step) on the plan's current stream.
int data_path(ppd_plan* p, const IterCtx& c) {
  PPD_TRY(fft_cols_forward(p, p->half_f));                  // a = F Z x~ (rows done)
  if (c.form == PPD_FORM_FUSED && c.prox == PPD_PROX_EXACT) {
    PPD_TRY(degrid_dual(p, c.dual, nullptr));               // dual argument w (no Algorithm 2 partials)
    PPD_TRY(secular_solve(p, nullptr, c.dual.v, p->gabuf, c.dual.y, c.dual.U, c.n_newton));  // prox^U_h(w)
    PPD_TRY(grid_dual_exact(p, c.dual));                    // dual finish, relaxation, gridding
  } else if (c.form == PPD_FORM_FUSED) {
    double* pa = p->part;
    double* pb = p->part + p->n_segs;
    PPD_TRY(degrid_dual(p, c.dual, pa));                    // dual argument, first Alg. 2 step
    if (c.dual.n_itr > 1 && c.persistent) {
      // the middle steps in one launch, state in registers; it leaves the
      // last step's factors for the gridding.  It runs beside the SARA
      // branch: workgroups of it that the SARA launches keep from being
      // resident at first get room as those finish (they never wait on
      // this launch), while the resident ones wait for their partials.
      PPD_TRY(block_factors(p, pa));
      PPD_TRY(alg2_persistent(p, c.dual, c.spin_limit));
      PPD_TRY(grid_dual_factored(p, c.dual));               // last projection, dual finish, gridding
    } else {
      for (int s = 1; s < c.dual.n_itr; ++s) {
        PPD_TRY(alg2_launch(p, 1, nullptr, c.dual.v, p->gabuf, c.dual.y, c.dual.U, c.dual.z, c.dual.mu, pa, pb,
                            c.dual.active));
        std::swap(pa, pb);
      }
      PPD_TRY(grid_dual(p, c.dual, pa));                    // last projection, dual finish, gridding
    }
  } else {
    PPD_TRY(degrid_plain(p, p->ybuf));
    PPD_TRY(plain_dual(p, c.dual));                         // data-dual update, block by block
    PPD_TRY(grid_plain(p, c.dual.v));                       // G^H Theta^H v
  }
  return fft_cols_inverse(p);
}

// The sparsity dual update and synthesis (SARA) on the plan's current stream.
int sara_path(ppd_plan* p, const IterCtx& c) {
  PPD_TRY(sara_dual(p, c.primal.xt, c.u, c.alpha, c.lambda, c.W, c.basis_active));   // clip and relaxation
  return sara_synthesis(p, c.u, p->ut, c.W);                // Psi u, summed over the bases
}

// One iteration of Algorithm 3 on the plan's stream.  SARA needs only x~
// and u, so it runs concurrently with the data-fidelity path, one of the two
// forked to the plan's second stream; the primal update waits
// for both on the plan's stream.  Eager, SARA is forked and the data path
// stays on the plan's stream (no queue hand-off at its start); captured
// into a graph, the data path is forked: replayed graphs put a forked SARA
// branch's join, and with it the primal update, on the other hardware queue
// (measured 142.5 against 132.7 us per iteration at 512^2).
int one_iteration(ppd_plan* p, const IterCtx& c) {
  PPD_HIP(hipEventRecord(p->ev_fork, p->stream));
  PPD_HIP(hipStreamWaitEvent(p->aux, p->ev_fork, 0));
  if (c.sara_forked) {
    {
      OnStream on(p, p->aux);
      PPD_TRY(sara_path(p, c));
      PPD_HIP(hipEventRecord(p->ev_join, p->aux));
    }
    PPD_TRY(data_path(p, c));
  } else {
    {
      OnStream on(p, p->aux);
      PPD_TRY(data_path(p, c));
      PPD_HIP(hipEventRecord(p->ev_join, p->aux));
    }
    PPD_TRY(sara_path(p, c));
  }
  PPD_HIP(hipStreamWaitEvent(p->stream, p->ev_join, 0));
  // the primal update, and the forward row pass of the new x~ for the next iteration
  return fft_rows_inverse_primal(p, c.primal, p->half_f);
}

std::string graph_key(const IterCtx& c) {
  char buf[700];
  std::snprintf(buf, sizeof(buf), "%p %p %p %p %p %p %p %p %p %p %p %p %p %p %a %a %a %a %a %a %a %d %d %d %d %d %d %p %d %d %d",
                (void*)c.dual.y, (void*)c.dual.U, (void*)c.dual.v, (void*)c.dual.z, (void*)c.primal.x,
                (void*)c.primal.xt, (void*)c.primal.x_true, (void*)c.u, (void*)c.primal.ut, (void*)c.W,
                (const void*)c.dual.active, (const void*)c.basis_active, (const void*)c.primal.part, (const void*)c.dual.rpart,
                c.dual.mu,
                c.dual.lambda, c.primal.tau, c.primal.eta, c.primal.zeta, double(c.alpha),
                double(c.lambda), c.dual.n_itr, c.form, c.prox, c.n_newton, int(c.persistent), c.spin_limit,
                (void*)c.stats_out, int(c.stats_cursor), c.has_truth, c.use_res_sq);
  return std::string(buf);
}

// The instantiated graph of a run of iterations in graph slot `slot`: `n`
// iterations with context `plain`, then, if `tail` is non-NULL, one more
// with context *tail (and its statistics reduction when it has a target).
// Captured on first use, re-captured when a pointer or scalar changes.
int iteration_graph(ppd_plan* p, const IterCtx& plain, int n, const IterCtx* tail, int slot,
                    hipGraphExec_t* out) {
  const std::string key = std::to_string(n) + " x " + graph_key(plain) + " | " + (tail ? graph_key(*tail) : "-");
  if (!p->graph_exec[slot] || key != p->graph_key[slot]) {
    if (p->graph_exec[slot]) (void)hipGraphExecDestroy(p->graph_exec[slot]);
    if (p->graph[slot]) (void)hipGraphDestroy(p->graph[slot]);
    p->graph_exec[slot] = nullptr;
    p->graph[slot] = nullptr;
    p->graph_key[slot].clear();
    PPD_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    int cst = PPD_OK;
    for (int r = 0; r < n && cst == PPD_OK; ++r) cst = one_iteration(p, plain);
    if (cst == PPD_OK && tail) {
      cst = one_iteration(p, *tail);
      if (cst == PPD_OK && tail->stats_out)
        cst = stats_finalize(p, tail->has_truth, tail->use_res_sq, tail->stats_out,
                             tail->stats_cursor ? p->hist_cursor : nullptr, 8 + p->d);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->stream, &g);
    if (cst != PPD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return cst;
    }
    if (e != hipSuccess) return fail(PPD_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p->graph[slot] = g;
    PPD_HIP(hipGraphInstantiate(&p->graph_exec[slot], g, nullptr, nullptr, 0));
    p->graph_key[slot] = key;
  }
  *out = p->graph_exec[slot];
  return PPD_OK;
}

}  // namespace

int stats_finalize(ppd_plan* p, int has_truth, int use_res_sq, double* out, int32_t* cursor, int stride) {
  int slot;
  PPD_TRY(timer_begin(p, KK_STATS, &slot));
  hipLaunchKernelGGL(k_stats_resid, dim3(p->d), dim3(STAT_THREADS), 0, p->stream, p->rpart, p->bseg_ids,
                     p->bseg_off_d, p->res_sq, use_res_sq, out, cursor, stride, p->rj_d);
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(256), 0, p->stream, p->ppart, primal_partial_count(p), p->eps_d, p->d,
                     has_truth, out, cursor, stride, out == p->host_stats_dev ? p->pa_sync + 2 : nullptr, p->rj_d);
  PPD_HIP(hipGetLastError());
  return timer_end(p, slot);
}

}  // namespace ppd

using namespace ppd;

extern "C" int ppd_iterate(ppd_plan* p, ppd_state* st, const ppd_params* prm, int n_iter, ppd_stats* stats,
                           double* residual) {
  if (!p || !st || !prm) return fail(PPD_EINVAL, "ppd_iterate: NULL argument");
  if (!st->x || !st->xt || !st->v || !st->u || !st->z || !prm->y || !prm->U || !prm->eps)
    return fail(PPD_EINVAL, "ppd_iterate: state and params need x, xt, v, u, z, y, U, eps");
  if (n_iter < 0) return fail(PPD_EINVAL, "ppd_iterate: n_iter must be >= 0");
  if (prm->n_itr < 1) return fail(PPD_EINVAL, "ppd_iterate: n_itr must be >= 1");
  if (prm->form != PPD_FORM_FUSED && prm->form != PPD_FORM_PLAIN)
    return fail(PPD_EINVAL, "ppd_iterate: unknown form");
  if (prm->prox != PPD_PROX_FB && prm->prox != PPD_PROX_EXACT)
    return fail(PPD_EINVAL, "ppd_iterate: unknown prox");
  if (prm->prox == PPD_PROX_EXACT && prm->form != PPD_FORM_FUSED)
    return fail(PPD_EUNSUPPORTED, "ppd_iterate: the exact prox is implemented in the fused form only");
  if (prm->n_newton < 0 || prm->n_newton > 64) return fail(PPD_EINVAL, "ppd_iterate: n_newton must be in [0, 64]");
  if (prm->block_active && prm->form != PPD_FORM_FUSED)
    return fail(PPD_EUNSUPPORTED, "ppd_iterate: randomised block updates are implemented in the fused form only");
  const double vals[6] = {prm->tau, prm->eta, prm->zeta, prm->lambda, prm->alpha, prm->mu};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(PPD_EINVAL, "ppd_iterate: non-finite parameter");
  if (!(prm->tau > 0 && prm->eta > 0 && prm->zeta >= 0 && prm->lambda > 0 && prm->lambda <= 1 &&
        prm->alpha >= 0 && prm->mu > 0))
    return fail(PPD_EINVAL, "ppd_iterate: need tau, eta, mu > 0, zeta, alpha >= 0, 0 < lambda <= 1");
  if (prm->use_graph && p->stream == nullptr)
    return fail(PPD_EINVAL, "ppd_iterate: graph replay needs a non-default stream");
  PPD_TRY(upload_eps(p, prm->eps));

  IterCtx c{};
  c.dual.y = reinterpret_cast<const float2*>(prm->y);
  c.dual.U = prm->U;
  c.dual.v = reinterpret_cast<float2*>(st->v);
  c.dual.z = reinterpret_cast<double2*>(st->z);
  c.dual.mu = prm->mu;
  c.dual.lambda = prm->lambda;
  c.dual.n_itr = prm->n_itr;
  c.primal.x = st->x;
  c.primal.xt = st->xt;
  c.primal.ut = p->ut;
  c.primal.x_true = prm->x_true;
  c.primal.tau = prm->tau;
  c.primal.eta = prm->eta;
  c.primal.zeta = prm->zeta;
  c.primal.lambda = prm->lambda;
  // statistics partials of the new iterate only when this call reduces them
  const int every = prm->stats_every;
  if (every < 0) return fail(PPD_EINVAL, "ppd_iterate: stats_every must be >= 0");
  const bool want = stats || residual || every > 0;
  c.primal.part = want ? p->ppart : nullptr;
  c.dual.rpart = want ? p->rpart : nullptr;
  // the periodic reduction: row k of the history, else the plan's buffer
  auto periodic = [&](int done) -> int {
    if (every <= 0 || done % every) return PPD_OK;
    double* out = prm->stats_history ? prm->stats_history + size_t(done / every - 1) * (8 + p->d) : p->stats_d;
    return stats_finalize(p, prm->x_true != nullptr, prm->form == PPD_FORM_PLAIN, out, nullptr, 0);
  };
  c.u = st->u;
  c.W = prm->W;
  c.alpha = float(prm->alpha);
  c.lambda = float(prm->lambda);
  c.form = prm->form;
  c.prox = prm->prox;
  c.dual.active = prm->block_active;
  c.basis_active = prm->basis_active;
  c.n_newton = prm->n_newton == 0 ? 12 : prm->n_newton;
#ifndef PPD_GRAPH_FORK_SARA
#define PPD_GRAPH_FORK_SARA 0
#endif
  c.sara_forked = PPD_GRAPH_FORK_SARA || !prm->use_graph;
  if (prm->persistent != PPD_PERSIST_AUTO && prm->persistent != PPD_PERSIST_OFF)
    return fail(PPD_EINVAL, "ppd_iterate: unknown persistent mode");
  if (prm->spin_limit < 0) return fail(PPD_EINVAL, "ppd_iterate: spin_limit must be >= 0");
  c.persistent = prm->persistent == PPD_PERSIST_AUTO && p->pa_ok && prm->form == PPD_FORM_FUSED &&
                 prm->prox == PPD_PROX_FB && prm->n_itr > 1;
  c.spin_limit = prm->spin_limit;

  if (n_iter > 0) {
    // the first iteration's forward row pass; each iteration then leaves
    // the next one's
    PPD_TRY(fft_rows_forward(p, st->xt, p->half_f));
    if (prm->use_graph) {
      // captured iterations: slot 0 without statistics partials, slot 1
      // with them and the periodic reduction (into the next history row at
      // the plan's cursor, or the plan's buffer), slot 2 with the partials
      // only (the call's last iteration, reduced after the loop), slot 3 a
      // captured run
      IterCtx c0 = c, c1 = c;
      c0.primal.part = nullptr;
      c0.dual.rpart = nullptr;
      c1.has_truth = prm->x_true != nullptr;
      c1.use_res_sq = prm->form == PPD_FORM_PLAIN;
      c1.stats_cursor = prm->stats_history != nullptr;
      c1.stats_out = prm->stats_history ? prm->stats_history : p->stats_d;
      if (every > 0 && prm->stats_history) {
        hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, p->stream, p->hist_cursor, 0);
        PPD_HIP(hipGetLastError());
      }
      // Each graph launch costs a few microseconds of the device's time, so
      // iterations are replayed in captured runs: with periodic statistics,
      // a period of `every` iterations whose last one reduces them (slot 3);
      // otherwise runs of GRAPH_RUN iterations without partials (slot 3);
      // the rest one at a time (slots 0-2).  Measured at 512^2: 143.9 us per
      // iteration replayed one at a time, 137.9 in periods of 10, 137.0
      // eager.
      int t = 0;
      while (t < n_iter) {
        hipGraphExec_t ex = nullptr;
        if (every > 1 && t % every == 0 && t + every <= n_iter) {
          PPD_TRY(iteration_graph(p, c0, every - 1, &c1, 3, &ex));
          PPD_HIP(hipGraphLaunch(ex, p->stream));
          t += every;
          continue;
        }
        // iterations [t, plain_end) need neither the periodic reduction nor
        // the final read-back
        const int next_periodic = every > 0 ? (t / every + 1) * every - 1 : n_iter;
        const int plain_end = std::min(next_periodic, n_iter - ((stats || residual) ? 1 : 0));
        if (GRAPH_RUN > 1 && t + GRAPH_RUN <= plain_end) {
          PPD_TRY(iteration_graph(p, c0, GRAPH_RUN, nullptr, 3, &ex));
          PPD_HIP(hipGraphLaunch(ex, p->stream));
          t += GRAPH_RUN;
          continue;
        }
        const bool periodic_t = every > 0 && (t + 1) % every == 0;
        const bool last_read = t + 1 == n_iter && (stats || residual);
        if (periodic_t) PPD_TRY(iteration_graph(p, c0, 0, &c1, 1, &ex));
        else if (last_read) PPD_TRY(iteration_graph(p, c0, 0, &c, 2, &ex));
        else PPD_TRY(iteration_graph(p, c0, 1, nullptr, 0, &ex));
        PPD_HIP(hipGraphLaunch(ex, p->stream));
        ++t;
      }
    } else {
      for (int t = 0; t < n_iter; ++t) {
        IterCtx ct = c;
        const bool read = (t + 1 == n_iter && (stats || residual)) || (every > 0 && (t + 1) % every == 0);
        if (!read) {   // partials nobody reduces are not formed
          ct.primal.part = nullptr;
          ct.dual.rpart = nullptr;
        }
        PPD_TRY(one_iteration(p, ct));
        PPD_TRY(periodic(t + 1));
      }
    }
    st->iter += n_iter;
  }
  if (stats || residual) {
    if (n_iter == 0) return fail(PPD_EINVAL, "ppd_iterate: statistics need n_iter >= 1");
    // the reduction writes the statistics and the give-up flag straight into
    // mapped pinned host memory: one synchronisation, no copy
    PPD_TRY(stats_finalize(p, prm->x_true != nullptr, prm->form == PPD_FORM_PLAIN, p->host_stats_dev, nullptr, 0));
    PPD_HIP(hipStreamSynchronize(p->stream));
    const double* h = p->host_stats;
    const bool gave_up = h[8 + p->d] != 0.0;
    if (gave_up) {
      // a wait of the persistent launch gave up (this call or an earlier
      // one without statistics): its results are not valid
      PPD_HIP(hipMemsetAsync(p->pa_sync + 2, 0, sizeof(uint32_t), p->stream));
      PPD_HIP(hipStreamSynchronize(p->stream));
      return fail(PPD_EDEVICE, "ppd_iterate: a wait of the persistent Algorithm 2 launch gave up; "
                               "the iterates of this call are not valid");
    }
    if (stats) {
      stats->iter = st->iter;
      stats->rel_change = h[0];
      stats->x_norm = h[1];
      stats->snr_db = h[2];
      stats->residual_max = h[3];
    }
    if (residual)
      for (int j = 0; j < p->d; ++j) residual[j] = h[8 + j];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || !std::isfinite(h[3]) || (prm->x_true && std::isnan(h[2])))
      return fail(PPD_ENONFINITE, "ppd_iterate: non-finite statistics");
  }
  return PPD_OK;
}

extern "C" int ppd_op_norm(ppd_plan* p, const double* U, const float* x0, int max_iter, double tol,
                           double* norm2, int* iters) {
  if (!p || !x0 || !norm2) return fail(PPD_EINVAL, "ppd_op_norm: NULL argument");
  if (max_iter < 1 || !(tol >= 0.0)) return fail(PPD_EINVAL, "ppd_op_norm: bad max_iter / tol");
  double n0 = 0.0;
  PPD_TRY(img_norm(p, x0, &n0));
  if (!(n0 > 0.0) || !std::isfinite(n0)) return fail(PPD_EINVAL, "ppd_op_norm: start image must be non-zero");
  PPD_TRY(img_scale(p, x0, 1.0 / n0, p->vec_tmp));
  double lam = 0.0, lam_prev = 0.0;
  int k = 0;
  for (; k < max_iter; ++k) {
    PPD_TRY(fft_forward(p, p->vec_tmp));
    PPD_TRY(degrid_plain(p, p->ybuf));
    if (U) {
      hipLaunchKernelGGL(k_vis_mul_U, dim3(int(std::min<int64_t>((p->M + 255) / 256, 4096))), dim3(256), 0,
                         p->stream, p->ybuf, U, p->M);
      PPD_HIP(hipGetLastError());
    }
    PPD_TRY(grid_plain(p, p->ybuf));
    PPD_TRY(fft_adjoint(p, p->img_tmp));
    PPD_TRY(img_norm(p, p->img_tmp, &lam));
    if (!(lam > 0.0) || !std::isfinite(lam)) return fail(PPD_ENONFINITE, "ppd_op_norm: degenerate iterate");
    PPD_TRY(img_scale(p, p->img_tmp, 1.0 / lam, p->vec_tmp));
    if (k > 0 && std::fabs(lam - lam_prev) <= tol * lam) {
      ++k;
      break;
    }
    lam_prev = lam;
  }
  PPD_HIP(hipStreamSynchronize(p->stream));
  *norm2 = lam;
  if (iters) *iters = k;
  return PPD_OK;
}

extern "C" int ppd_reweighted(ppd_plan* p, ppd_state* st, const ppd_params* prm, int n_reweights,
                              int iters_per_solve, double omega0, double decay, float* W_work, ppd_stats* stats) {
  if (!p || !st || !prm) return fail(PPD_EINVAL, "ppd_reweighted: NULL argument");
  if (n_reweights < 0 || iters_per_solve < 1)
    return fail(PPD_EINVAL, "ppd_reweighted: n_reweights >= 0 and iters_per_solve >= 1 needed");
  if (!(omega0 > 0.0) || !std::isfinite(omega0) || !(decay > 0.0) || !std::isfinite(decay))
    return fail(PPD_EINVAL, "ppd_reweighted: omega0 > 0 and decay > 0 needed");
  if (n_reweights > 0 && (!W_work || W_work == prm->W))
    return fail(PPD_EINVAL, "ppd_reweighted: W_work is required and must not alias params->W");
  ppd_params solve = *prm;
  double omega = omega0;
  for (int k = 0; k <= n_reweights; ++k) {
    PPD_TRY(ppd_iterate(p, st, &solve, iters_per_solve, stats ? &stats[k] : nullptr, nullptr));
    if (k == n_reweights) break;
    omega *= decay;
    PPD_TRY(ppd_reweight(p, st->x, float(omega), W_work));
    solve.W = W_work;
  }
  return PPD_OK;
}
