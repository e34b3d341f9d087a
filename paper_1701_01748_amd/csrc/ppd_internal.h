// Internal declarations of libppd (gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ppd.h"

namespace ppd {

// ---- errors -------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

#define PPD_HIP(expr)                                                           \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess)                                                       \
      return ::ppd::fail(PPD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define PPD_TRY(expr)                 \
  do {                                \
    int s_ = (expr);                  \
    if (s_ != PPD_OK) return s_;      \
  } while (0)

// ---- constants ----------------------------------------------------------
constexpr int KB_TAPS = 8;        // kernel width per axis
constexpr int KB_DEG = 9;         // polynomial degree per tap
constexpr int KB_NC = KB_DEG + 1; // coefficients per tap
constexpr int N_BASES = 9;        // Dirac + db1..db8
constexpr int FILT_STRIDE = 16;   // max Daubechies taps (db8)
constexpr int SEC_CHUNK = 2048;   // points per workgroup of an exact-prox Newton pass
constexpr int MAX_ITEM_SEGS = 64; // per-block segments of one work item (one wave scans them)
constexpr int MAX_XCD = 8;
constexpr int PA_THREADS = 256;   // persistent Algorithm 2: threads per workgroup
#ifndef PPD_PA_PER
#define PPD_PA_PER 12
#endif
// points per thread held in registers: 12 (230 VGPRs, 2 waves per SIMD)
// leaves fewer workgroups to wait for at each step than 8 and still fits
// the co-residency limit at 1.3M points
constexpr int PA_PER = PPD_PA_PER;
constexpr int PA_CHUNK = PA_THREADS * PA_PER;
constexpr int PA_MAXB = 4;        // data blocks one workgroup's points may span
constexpr int PA_SYNC_WORDS = 32;   // [1] exit count, [2] give-up flag
// tagged partial slots of the persistent launch (see k_alg2_persistent)
constexpr uint64_t PA_SIGN = 0x8000000000000000ull;
constexpr uint64_t PA_EMPTY = 0x7ff8000000000000ull;   // quiet NaN: no partial yet
#ifndef PPD_FOLD_HEAVY
#define PPD_FOLD_HEAVY 16
#endif
constexpr int FOLD_HEAVY = PPD_FOLD_HEAVY;   // item regions above which a tile's fold takes a whole workgroup
// Work items per workgroup of the 8 x 8 degridding with the dual update:
// 0 takes one item per single-wave workgroup in k_degrid<8, DUAL> (88
// VGPRs, 5 waves per SIMD), n > 0 runs of n items in k_degrid8 (107 VGPRs,
// 4 waves per SIMD), which the lighter SARA branch no longer repays.
#ifndef PPD_DEGRID_RUN
#define PPD_DEGRID_RUN 0
#endif
#ifndef PPD_GRIDM_RUN
#define PPD_GRIDM_RUN 2
#endif
#ifndef PPD_GRIDM_WPG
#define PPD_GRIDM_WPG 1
#endif
// Captured-iteration graphs per plan: one iteration without statistics
// partials, one with them and the periodic reduction, one with the partials
// only, and a captured run (a statistics period, or GRAPH_RUN iterations
// without partials).
constexpr int GRAPH_SLOTS = 4;
#ifndef PPD_GRAPH_RUN
#define PPD_GRAPH_RUN 8
#endif
constexpr int GRAPH_RUN = PPD_GRAPH_RUN;
// Product steps of the matrix-core gridding whose LDS operands are read
// before the first of their products (2, 4 or 8).
#ifndef PPD_GRIDM_READ_AHEAD
#define PPD_GRIDM_READ_AHEAD 2
#endif

// Launch order of the work items over the XCDs: the items, in spatial
// order, are cut into 8 contiguous bands of near-equal work (64-point
// batches plus one per item for its region), XCD k taking the units
// (workgroups of `unit` consecutive items) [off[k], off[k+1]).  Workgroup
// ids go round-robin over the XCDs, so workgroup b runs unit
// off[b mod 8] + b / 8 of band b mod 8, if that band has it.
struct XcdSplit {
  int32_t off[MAX_XCD + 1];
  int32_t unit;     // items per workgroup
  int32_t launch;   // workgroups to launch: 8 x the longest band
};

// A segment: plan-order visibilities [start, start+count) of one data
// block whose first tap lies in one grid tile.
struct Seg {
  int32_t start, count, block, item;
};
// A work item (one workgroup): the segments [seg0, seg1) of tile (tx, ty),
// at most chunk_max visibilities.  Items are ordered tile by tile in
// row-major tile order.
struct Item {
  int32_t tx, ty, seg0, seg1;
};

// Kernel kinds for the optional per-launch event timer.
enum KernelKind {
  KK_FFT_ROWS_FWD, KK_FFT_COLS_FWD, KK_DEGRID, KK_GRID, KK_FFT_COLS_INV, KK_FFT_ROWS_INV,
  KK_FOLD, KK_PERMUTE, KK_SUBITER, KK_DWT, KK_IDWT, KK_STATS, KK_PLAIN_DUAL, KK_HIST,
  KK_NORM, KK_MISC, KK_COUNT
};
const char* kernel_kind_name(int k);

}  // namespace ppd

struct ppd_plan {
  // geometry
  int nx = 0, ny = 0, Kx = 0, Ky = 0, log2Kx = 0, log2Ky = 0;
  int64_t M = 0;
  int d = 0, levels = 3, T = 32, chunk_max = 1024;
  int tiles_x = 0, tiles_y = 0;
  double beta = 0.0;
  double su_scale = 0.0, sv_scale = 0.0;   // K / (2 pi) per axis
  bool has_theta = false;
  hipStream_t stream = nullptr;
  int device = 0;
  // second stream of an iteration (the SARA dual step runs there, forked
  // from and joined back to `stream` through the two events)
  hipStream_t aux = nullptr;
  double2* bfac = nullptr;                 // [d] (factor, inside) of the last block_factors call
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // host copies
  std::vector<int64_t> block_off;          // [d+1]
  std::vector<int32_t> perm_host;          // plan -> user
  std::vector<ppd::Item> items_host;       // launch order
  std::vector<ppd::Seg> segs_host;
  std::vector<int32_t> bseg_off;           // [d+1] into bseg_ids
  int n_items = 0, n_segs = 0;
  ppd::XcdSplit split1{}, split_degrid{}, split_grid{};   // 1, PPD_DEGRID_RUN, PPD_GRIDM_RUN x WPG items per workgroup
  int n_tiles = 0, n_tile_launch = 0;

  // device: coverage and plan tables
  float* wu = nullptr;
  float* wv = nullptr;
  float* theta = nullptr;
  int32_t* perm = nullptr;
  ppd::Item* items = nullptr;
  ppd::Seg* segs = nullptr;
  int32_t* tile_item_off = nullptr;        // [n_tiles+1] items of each tile
  int32_t* fold_wg = nullptr;              // [n_fold_wg][4] tiles per 4-wave fold workgroup
  int n_fold_wg = 0;                       // multiple of MAX_XCD
  int32_t* bseg_ids = nullptr;             // segment ids grouped by block
  int32_t* bseg_off_d = nullptr;           // [d+1]
  float2* gscratch = nullptr;              // [n_items][(T+7)^2] gridding partials
  int32_t* vis_block = nullptr;            // plan index -> block (plain form)
  float* kbc = nullptr;                    // [8][10] tap polynomials
  float* dpx = nullptr;                    // [nx] 1/phi_hat(n_c / Kx)
  float* dpy = nullptr;                    // [ny] 1/phi_hat(n_r / Ky)
  float2* twx = nullptr;                   // [Kx/2] exp(-2 pi i k / Kx)
  float2* twy = nullptr;                   // [Ky/2]
  float* filt = nullptr;                   // [8][2][16] lo / hi Daubechies filters

  // device: work buffers
  float2* grid_f = nullptr;                // forward spectrum  Ky x Kx
  float2* grid_a = nullptr;                // adjoint accumulation Ky x Kx
  float2* half = nullptr;                  // ny x Kx intermediate
  float2* half_f = nullptr;                // ny x Kx forward row pass of x~ (iterations)
  float2* ybuf = nullptr;                  // [M] complex64 scratch
  double2* wbuf = nullptr;                 // [M] complex128 w (plain form)
  float2* gabuf = nullptr;                 // [M] complex64 Theta G a (fused form; w is rebuilt from it)
  double2* qbuf = nullptr;                 // [M] complex128 (plain form; (a^2, U) of the Newton passes)
  // Newton passes of the exact prox: chunks of consecutive plan-order
  // visibilities inside one block
  int n_sec_chunks = 0;
  int32_t* sec_cstart = nullptr;           // [n_sec_chunks + 1] first visibility of each chunk
  int32_t* sec_cblock = nullptr;           // [n_sec_chunks] block of each chunk
  int32_t* sec_coff = nullptr;             // [d + 1] chunks of block j: [sec_coff[j], sec_coff[j+1])
  double* sec_part = nullptr;              // [2][2][n_sec_chunks] S2, S3 partials, two passes
  double* sec_nu = nullptr;                // [2][d] nu of the last two Newton passes
  double4* du_blk = nullptr;               // [d] block terms of the differentiable dual update
  // persistent Algorithm 2 middle steps (one launch, state in registers):
  // workgroup g holds plan-order points [g PA_CHUNK, (g+1) PA_CHUNK)
  int pa_groups = 0;                       // workgroups of the persistent launch
  bool pa_ok = false;                      // every workgroup co-resident and within PA_MAXB blocks
  int32_t* voff_d = nullptr;               // [d+1] block offsets (plan order)
  int32_t* pa_wgb0 = nullptr;              // [pa_groups] first block of each workgroup
  int32_t* pa_gfirst = nullptr;            // [d] first workgroup of each block
  int32_t* pa_glast = nullptr;             // [d] last workgroup of each block
  uint64_t* pa_part = nullptr;             // [2][pa_groups][PA_MAXB] tagged per-workgroup block partials
  uint32_t* pa_sync = nullptr;             // [PA_SYNC_WORDS] exit count, give-up flag
  double* part = nullptr;                  // [2][n_segs] block-norm partials
  double* rpart = nullptr;                 // [n_segs] residual partials
  double* eps_d = nullptr;                 // [d]
  std::vector<double> eps_cache;
  double* ppart = nullptr;                 // [ny][4] primal statistics partials
  double* stats_d = nullptr;               // [8 + d]
  int32_t* hist_cursor = nullptr;          // [1] next statistics history row of a graph replay
  double* rj_d = nullptr;                  // [d] block residuals of the last statistics reduction
  double* host_stats = nullptr;            // pinned host [8 + d + 1]: a call's statistics and give-up flag
  double* host_stats_dev = nullptr;        // its device-side address
  float* sara_ll = nullptr;                // LL temporaries, analysis
  float* sara_rec = nullptr;               // reconstruction temporaries
  float* ut = nullptr;                     // [ny][nx] Psi u
  float* img_tmp = nullptr;                // [ny][nx]
  float* vec_tmp = nullptr;                // [ny][nx] power iteration
  double* pl_part = nullptr;               // [1024] plain-form / image partials
  double* res_sq = nullptr;                // [d] plain-form residual norms^2
  double* pl_scalar = nullptr;             // [4]
  int32_t* icount = nullptr;               // [ny][nx] sampling-density counts
  int32_t* imin = nullptr;                 // [1]
  size_t sara_ll_floats = 0;
  size_t device_bytes = 0;
  std::vector<void*> allocations;          // hipMalloc'd buffers (plans without a workspace)
  // caller-owned workspace the buffers are carved from (256-byte aligned
  // offsets), or a sizing pass that only adds up the bytes
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_used = 0;
  bool ws_measure = false;

  // graph replay of one iteration: slot 0 without the statistics partials,
  // slot 1 with them and the periodic reduction, slot 2 with them only
  hipGraphExec_t graph_exec[ppd::GRAPH_SLOTS] = {};
  hipGraph_t graph[ppd::GRAPH_SLOTS] = {};
  std::string graph_key[ppd::GRAPH_SLOTS];

  // optional per-launch timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pending;   // (kind, event pair index)
  int64_t t_counts[ppd::KK_COUNT] = {};
  double t_ms[ppd::KK_COUNT] = {};
};

namespace ppd {

// launch bracketing for the per-kernel timer
int timer_begin(ppd_plan* p, int kind, int* slot);
int timer_end(ppd_plan* p, int slot);

// ---- component launchers (each returns a PPD_* status) -------------------
int fft_forward(ppd_plan* p, const float* x);                  // x -> grid_f (via half)
int fft_rows_forward(ppd_plan* p, const float* x, float2* dst);  // x -> dst (ny x Kx)
int fft_cols_forward(ppd_plan* p, const float2* src);           // src (ny x Kx) -> grid_f
int fft_adjoint(ppd_plan* p, float* x);                        // grid_a -> x (plain)
int fft_cols_inverse(ppd_plan* p);                             // grid_a -> half
struct PrimalArgs {
  float* x; float* xt; const float* ut; const float* x_true;
  double tau, eta, zeta, lambda;
  double* part;                    // [ny][4] statistics partials, or NULL to skip them
};
// half -> primal update; with next != NULL also the forward row pass of the
// new x~ into next (ny x Kx)
int fft_rows_inverse_primal(ppd_plan* p, const PrimalArgs& a, float2* next);
int fold_grid(ppd_plan* p);                                    // gscratch -> grid_a

int degrid_plain(ppd_plan* p, float2* out);                    // grid_f -> out (plan order)
struct DualArgs {
  const float2* y; const double* U; float2* v; double2* z;
  double mu, lambda;
  int n_itr;
  const uint8_t* active;   // DEVICE [d] block mask of this iteration, NULL = all
  double* rpart = nullptr; // DEVICE [n_segs] residual partials for the statistics, NULL = skip them
};
int degrid_dual(ppd_plan* p, const DualArgs& a, double* part_out);   // grid_f -> gabuf; part_out NULL: no Algorithm 2 partials
int grid_plain(ppd_plan* p, const float2* v);                 // v -> grid_a (accumulate)
int grid_dual(ppd_plan* p, const DualArgs& a, const double* part_in);  // dual finish + grid
int grid_dual_factored(ppd_plan* p, const DualArgs& a);   // the same with the block factors already in bfac

int plain_dual(ppd_plan* p, const DualArgs& a);               // per-block unfused dual update
// Per-block projection factors of P_B from per-segment partials of
// ||q - y||^2: bfac[j] = (min(1, eps_j / r_j), r_j <= eps_j), r_j the block norm.
int block_factors(ppd_plan* p, const double* part);
// The n_itr - 1 middle Algorithm 2 steps of the fused form in one persistent
// launch (needs p->pa_ok and the first step's factors in bfac; leaves the
// last step's factors in bfac).  spin_limit bounds each wait
// (0: default).
int alg2_persistent(ppd_plan* p, const DualArgs& a, int spin_limit);
// Maximum co-resident workgroups of the persistent launch on the current
// device (0 if it cannot be determined).
int alg2_persistent_capacity();
// n_newton Newton steps of the exact prox per block; nu_j in bfac[j].x.
// The prox argument is w if non-NULL, else U^-1 v + ga (see dual_arg).
int secular_solve(ppd_plan* p, const double2* w, const float2* v, const float2* ga, const float2* y,
                  const double* U, int n_newton);
int grid_dual_exact(ppd_plan* p, const DualArgs& a);   // dual finish with the exact prox + grid
int permute(ppd_plan* p, int direction, const void* in, void* out, int elem_bytes);

int sara_analysis(ppd_plan* p, const float* x, float* coef, const float* W);
int sara_dual(ppd_plan* p, const float* x, float* u, float alpha, float lambda, const float* W,
              const uint8_t* active = nullptr);   // active: DEVICE [9] basis mask, NULL = all
int sara_synthesis(ppd_plan* p, const float* u, float* out, const float* W);

// out: [8 + d], or with a cursor row *cursor of rows of `stride` doubles (advanced)
int stats_finalize(ppd_plan* p, int has_truth, int use_res_sq, double* out, int32_t* cursor, int stride);
int upload_eps(ppd_plan* p, const double* eps_host);

// host-side setup helpers
void kb_tap_polynomials(double beta, float* coef /* [8][KB_NC] */);
double kb_ft(double xi, double beta);
void daubechies(int p, double* h);

}  // namespace ppd

// ---- device helpers --------------------------------------------------------
namespace ppd {

// The 8 tap weights at fractional offset s in [0, 1), x = 2s - 1.  The
// kernel is even, so tap 7-m at x equals tap m at -x: with the even and odd
// parts of tap m's polynomial, P(+-x) = E(x^2) +- x O(x^2), four polynomial
// pairs give all eight weights (half the multiply-adds of eight Horner
// evaluations).  c holds the coefficients of taps 0..3 (of 8) in powers of x.
__host__ __device__ inline void kb_weights(float s, const float* __restrict__ c, float* w) {
  const float x = 2.0f * s - 1.0f;
  const float y = x * x;
#pragma unroll
  for (int m = 0; m < KB_TAPS / 2; ++m) {
    const float* cm = c + m * KB_NC;
    float e = cm[KB_DEG - 1], o = cm[KB_DEG];   // KB_DEG is odd
#pragma unroll
    for (int k = KB_DEG - 3; k >= 0; k -= 2) {
      e = fmaf(e, y, cm[k]);
      o = fmaf(o, y, cm[k + 1]);
    }
    const float xo = x * o;
    w[m] = e + xo;
    w[KB_TAPS - 1 - m] = e - xo;
  }
}
static_assert(KB_DEG % 2 == 1, "even / odd split assumes an odd degree");

// argument of the data-dual update of Algorithm 3, w = U^-1 v + Theta G a, in FP64; the fused form
// stores Theta G a (complex64) and rebuilds w where it is needed, bitwise
// the same each time.
__device__ __forceinline__ double2 dual_arg(float2 v, double U, float2 ga) {
  const double r = 1.0 / U;   // one division per visibility, shared by both parts
  return make_double2(double(v.x) * r + double(ga.x), double(v.y) * r + double(ga.y));
}

// Segment table of a work item in LDS: the offsets of its segments in the
// item's flattened visibility range (pre[n] = total), their first visibility
// in plan order and their data block.
struct ItemTab {
  int pre[MAX_ITEM_SEGS + 1];
  int start[MAX_ITEM_SEGS];
  int block[MAX_ITEM_SEGS];
};

// Wave 0 loads the item's segments (one per lane) and scans their counts;
// the caller synchronises before use.
__device__ inline void load_item_tab(const Item& it, const Seg* __restrict__ segs, ItemTab& tab) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int cnt = 0;
    if (lane < it.seg1 - it.seg0) {
      const Seg sg = segs[it.seg0 + lane];
      cnt = sg.count;
      tab.start[lane] = sg.start;
      tab.block[lane] = sg.block;
    }
    int inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(inc, o);
      if (lane >= o) inc += t;
    }
    tab.pre[lane + 1] = inc;
    if (lane == 0) tab.pre[0] = 0;
  }
}

// Segment of flattened index li, searching forward from segment s.
__device__ __forceinline__ int seg_of(int li, int s, const int* pre) {
  while (li >= pre[s + 1]) ++s;
  return s;
}

// Sum over the 64 lanes of a wave by a fixed butterfly (lanes may differ in
// the last bit; callers use lane 0's value).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The unit (first item / unit) a workgroup takes in a work-balanced XCD
// split, or -1 when its XCD's band has no unit left for it.
__device__ __forceinline__ int xcd_unit(int bid, const XcdSplit& s) {
  const int k = bid % MAX_XCD;
  const int u = s.off[k] + bid / MAX_XCD;
  return u < s.off[k + 1] ? u : -1;
}

// XCD-aware remap: consecutive workgroup ids go round-robin over the XCDs;
// give each XCD a contiguous range of the (spatially ordered) work list so
// its L2 holds one band of the grid.
__device__ inline int xcd_remap(int bid, int nlaunch) {
  const int per = nlaunch / MAX_XCD;     // nlaunch is a multiple of MAX_XCD
  return (bid % MAX_XCD) * per + bid / MAX_XCD;
}

}  // namespace ppd
