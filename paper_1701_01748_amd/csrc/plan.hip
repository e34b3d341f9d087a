// Plan creation: argument validation, (block, tile) binning of the
// visibilities, host-computed tables (Kaiser-Bessel tap polynomials,
// deapodisation, FFT twiddles, Daubechies filters) and work buffers.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>

#include "ppd_internal.h"

namespace ppd {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

const char* kernel_kind_name(int k) {
  static const char* names[KK_COUNT] = {
      "fft_rows_fwd", "fft_cols_fwd", "degrid", "grid", "fft_cols_inv", "fft_rows_inv",
      "fold", "permute", "subiter", "dwt", "idwt", "stats", "plain_dual", "hist", "norm", "misc"};
  return (k >= 0 && k < KK_COUNT) ? names[k] : "?";
}

// ---- Kaiser-Bessel kernel (Sec. 5: 8x8 kernels after Fessler & Sutton) ---
// I0 by its power series sum_k (x^2/4)^k / (k!)^2 (all terms positive).
static double bessel_i0(double x) {
  const double y = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= y / (double(k) * double(k));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

static double kb_phi(double dist, double beta) {
  const double a = 1.0 - (2.0 * dist / KB_TAPS) * (2.0 * dist / KB_TAPS);
  return a < 0.0 ? 0.0 : bessel_i0(beta * std::sqrt(a));
}

// Continuous Fourier transform of the kernel: J sinh(z)/z,
// z = sqrt(beta^2 - (pi J xi)^2) (Jackson et al. 1991).
double kb_ft(double xi, double beta) {
  const double t = M_PI * KB_TAPS * xi;
  const double z = std::sqrt(beta * beta - t * t);
  return KB_TAPS * std::sinh(z) / z;
}

// Tap m of a visibility with fractional grid offset s in [0, 1) sits at
// distance s + 3 - m from the kernel centre.  Each tap is interpolated by a
// degree-9 polynomial in x = 2s - 1 through 10 Chebyshev nodes (solved in
// float64 by Gaussian elimination with partial pivoting).  The nodes are
// symmetric in x, so tap 7-m's polynomial is tap m's at -x; the device
// evaluation reads taps 0..3 only.
void kb_tap_polynomials(double beta, float* coef) {
  const int n = KB_NC;
  for (int m = 0; m < KB_TAPS; ++m) {
    double A[KB_NC][KB_NC + 1];
    for (int i = 0; i < n; ++i) {
      const double node = 0.5 * (1.0 - std::cos(M_PI * (i + 0.5) / n));
      const double x = 2.0 * node - 1.0;
      double pw = 1.0;
      for (int k = 0; k < n; ++k) {
        A[i][k] = pw;
        pw *= x;
      }
      A[i][n] = kb_phi(node + 3.0 - m, beta);
    }
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
      for (int k = 0; k <= n; ++k) std::swap(A[c][k], A[piv][k]);
      for (int r = c + 1; r < n; ++r) {
        const double f = A[r][c] / A[c][c];
        for (int k = c; k <= n; ++k) A[r][k] -= f * A[c][k];
      }
    }
    double sol[KB_NC];
    for (int c = n - 1; c >= 0; --c) {
      double s = A[c][n];
      for (int k = c + 1; k < n; ++k) s -= A[c][k] * sol[k];
      sol[c] = s / A[c][c];
    }
    for (int k = 0; k < n; ++k) coef[m * KB_NC + k] = float(sol[k]);
  }
}

// ---- Daubechies filters (Sec. 5.1: SARA = Dirac + db1..db8) --------------
// Spectral factorisation: |m0(w)|^2 = cos^{2p}(w/2) P(sin^2(w/2)),
// P(y) = sum_{k<p} C(p-1+k, k) y^k.  The p-1 roots of P are found by
// Durand-Kerner iteration and Newton polishing; each maps through
// z + 1/z = 2 - 4y to the root inside the unit circle (minimum phase);
// h is then (1 + z^-1)^p prod (1 - r z^-1), scaled to sum sqrt(2).
void daubechies(int p, double* h) {
  using cd = std::complex<double>;
  std::vector<double> P(p);
  for (int k = 0; k < p; ++k) {
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * double(p - 1 + i) / double(i);
    P[k] = c;
  }
  const int deg = p - 1;
  std::vector<cd> roots(deg);
  auto evalP = [&](cd y) {
    cd acc = P[deg];
    for (int k = deg - 1; k >= 0; --k) acc = acc * y + P[k];
    return acc;
  };
  auto evaldP = [&](cd y) {
    cd acc = double(deg) * P[deg];
    for (int k = deg - 1; k >= 1; --k) acc = acc * y + double(k) * P[k];
    return acc;
  };
  if (deg > 0) {
    const cd seed(0.4, 0.9);
    cd pw(1.0, 0.0);
    for (int i = 0; i < deg; ++i) {
      roots[i] = pw;
      pw *= seed;
    }
    for (int it = 0; it < 2000; ++it) {
      double delta = 0.0;
      for (int i = 0; i < deg; ++i) {
        cd den = P[deg];
        for (int j = 0; j < deg; ++j)
          if (j != i) den *= (roots[i] - roots[j]);
        const cd step = evalP(roots[i]) / den;
        roots[i] -= step;
        delta = std::max(delta, std::abs(step));
      }
      if (delta < 1e-15) break;
    }
    for (int it = 0; it < 5; ++it)
      for (int i = 0; i < deg; ++i) roots[i] -= evalP(roots[i]) / evaldP(roots[i]);
  }
  std::vector<cd> poly(1, cd(1.0, 0.0));
  auto mul = [&](cd a0, cd a1) {   // poly *= (a0 + a1 z^-1)
    std::vector<cd> out(poly.size() + 1, cd(0.0, 0.0));
    for (size_t i = 0; i < poly.size(); ++i) {
      out[i] += a0 * poly[i];
      out[i + 1] += a1 * poly[i];
    }
    poly.swap(out);
  };
  for (int i = 0; i < p; ++i) mul(1.0, 1.0);
  for (int i = 0; i < deg; ++i) {
    const cd b = 1.0 - 2.0 * roots[i];
    const cd sq = std::sqrt(b * b - 1.0);
    const cd z = std::abs(b + sq) < 1.0 ? b + sq : b - sq;
    mul(1.0, -z);
  }
  double s = 0.0;
  for (int i = 0; i < 2 * p; ++i) s += poly[i].real();
  for (int i = 0; i < 2 * p; ++i) h[i] = poly[i].real() * (std::sqrt(2.0) / s);
}

int upload_eps(ppd_plan* p, const double* eps_host) {
  for (int j = 0; j < p->d; ++j)
    if (!(eps_host[j] > 0.0) || !std::isfinite(eps_host[j]))
      return fail(PPD_EINVAL, "eps must be finite and > 0 for every block");
  if (p->eps_cache.size() == size_t(p->d) &&
      std::equal(p->eps_cache.begin(), p->eps_cache.end(), eps_host))
    return PPD_OK;
  p->eps_cache.assign(eps_host, eps_host + p->d);
  PPD_HIP(hipMemcpyAsync(p->eps_d, p->eps_cache.data(), sizeof(double) * p->d,
                         hipMemcpyHostToDevice, p->stream));
  PPD_HIP(hipStreamSynchronize(p->stream));
  return PPD_OK;
}

}  // namespace ppd

using namespace ppd;

static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
static int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

constexpr size_t WS_ALIGN = 256;

template <typename T>
static int dalloc(ppd_plan* p, T** ptr, size_t count) {
  if (count == 0) count = 1;
  if (p->ws || p->ws_measure) {
    const size_t off = (p->ws_used + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN;
    p->ws_used = off + sizeof(T) * count;
    p->device_bytes += sizeof(T) * count;
    *ptr = nullptr;
    if (p->ws_measure) return PPD_OK;
    if (p->ws_used > p->ws_bytes)
      return fail(PPD_EINVAL, "workspace of " + std::to_string(p->ws_bytes) + " bytes is too small");
    *ptr = reinterpret_cast<T*>(p->ws + off);
    return PPD_OK;
  }
  void* q = nullptr;
  if (hipMalloc(&q, sizeof(T) * count) != hipSuccess)
    return fail(PPD_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed");
  p->allocations.push_back(q);
  p->device_bytes += sizeof(T) * count;
  *ptr = static_cast<T*>(q);
  return PPD_OK;
}

static void destroy_plan(ppd_plan* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (int k = 0; k < ppd::GRAPH_SLOTS; ++k) {
    if (p->graph_exec[k]) (void)hipGraphExecDestroy(p->graph_exec[k]);
    if (p->graph[k]) (void)hipGraphDestroy(p->graph[k]);
  }
  if (p->host_stats) (void)hipHostFree(p->host_stats);
  if (p->aux) (void)hipStreamSynchronize(p->aux);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  for (void* q : p->allocations) (void)hipFree(q);
  delete p;
}

extern "C" {

const char* ppd_strerror(int status) {
  switch (status) {
    case PPD_OK: return "ok";
    case PPD_EINVAL: return "invalid argument";
    case PPD_ENOMEM: return "out of device memory";
    case PPD_EDEVICE: return "HIP runtime error";
    case PPD_ENONFINITE: return "non-finite iteration statistics";
    case PPD_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* ppd_last_error(void) { return g_last_error.c_str(); }

int ppd_kb_weights_host(double kb_beta, int64_t n, const float* s, float* w) {
  if (n < 0 || (n > 0 && (!s || !w))) return fail(PPD_EINVAL, "ppd_kb_weights_host: bad pointers");
  if (kb_beta <= 0.0) kb_beta = M_PI * std::sqrt(35.2);
  float coef[KB_TAPS * KB_NC];
  kb_tap_polynomials(kb_beta, coef);
  for (int64_t i = 0; i < n; ++i) kb_weights(s[i], coef, w + KB_TAPS * i);
  return PPD_OK;
}

int ppd_daubechies_host(int p, double* h) {
  if (p < 1 || p > 8 || !h) return fail(PPD_EINVAL, "ppd_daubechies_host: p must be 1..8");
  daubechies(p, h);
  return PPD_OK;
}

}  // extern "C"

// Plan creation.  With `measure` set, only the host work runs and the device
// bytes the plan needs are returned there (no HIP call); with a workspace the
// device buffers are carved from it, else they are allocated.
static int create_plan(ppd_plan** out, const ppd_plan_desc* desc, void* stream, void* workspace,
                       size_t ws_bytes, size_t* measure) {
  if (!out || !desc) return fail(PPD_EINVAL, "ppd_plan_create: NULL argument");
  *out = nullptr;
  const ppd_plan_desc& D = *desc;
  if (!is_pow2(D.nx) || !is_pow2(D.ny) || D.nx < 16 || D.ny < 16 || D.nx > 2048 || D.ny > 2048)
    return fail(PPD_EUNSUPPORTED, "image sides must be powers of two in [16, 2048]");
  const int levels = D.levels == 0 ? 3 : D.levels;
  if (levels < 1 || levels > 6 || (D.nx >> levels) < 1 || (D.ny >> levels) < 1 ||
      (D.nx % (1 << levels)) || (D.ny % (1 << levels)))
    return fail(PPD_EINVAL, "levels must be in 1..6 with both sides divisible by 2^levels");
  if (D.M < 1 || D.M >= (int64_t(1) << 31)) return fail(PPD_EINVAL, "M must be in [1, 2^31)");
  if (D.d < 1 || !D.block_off) return fail(PPD_EINVAL, "d >= 1 and block_off required");
  if (D.block_off[0] != 0 || D.block_off[D.d] != D.M)
    return fail(PPD_EINVAL, "block_off must start at 0 and end at M");
  for (int j = 0; j < D.d; ++j)
    if (D.block_off[j + 1] <= D.block_off[j])
      return fail(PPD_EINVAL, "block_off must be strictly increasing (no empty block)");
  if (!D.omega_u || !D.omega_v) return fail(PPD_EINVAL, "omega_u / omega_v required");
  int T = D.tile == 0 ? 8 : D.tile;
  if (T != 8 && T != 16 && T != 32 && T != 64) return fail(PPD_EINVAL, "tile must be 8, 16, 32 or 64");
  const int chunk_max = D.chunk != 0 ? D.chunk : (T == 8 ? 128 : 512);
  if (chunk_max < 64 || chunk_max > 65536) return fail(PPD_EINVAL, "chunk must be in [64, 65536]");
  const float lim = 3.14159274f;   // float32(pi) rounds above pi
  for (int64_t i = 0; i < D.M; ++i) {
    const float a = D.omega_u[i], b = D.omega_v[i];
    if (!(a > -lim && a < lim && b > -lim && b < lim))
      return fail(PPD_EINVAL, "omega must be finite and inside [-pi, pi) (index " + std::to_string(i) + ")");
    if (D.theta && !(D.theta[i] > 0.0f && std::isfinite(D.theta[i])))
      return fail(PPD_EINVAL, "theta must be finite and > 0");
  }

  ppd_plan* p = new ppd_plan();
  p->nx = D.nx;
  p->ny = D.ny;
  p->Kx = 2 * D.nx;
  p->Ky = 2 * D.ny;
  p->log2Kx = ilog2(p->Kx);
  p->log2Ky = ilog2(p->Ky);
  p->M = D.M;
  p->d = D.d;
  p->levels = levels;
  p->T = std::min(T, std::min(p->Kx, p->Ky));
  p->chunk_max = chunk_max;
  p->tiles_x = p->Kx / p->T;
  p->tiles_y = p->Ky / p->T;
  p->beta = D.kb_beta > 0.0 ? D.kb_beta : M_PI * std::sqrt(35.2);
  p->su_scale = double(p->Kx) / (2.0 * M_PI);
  p->sv_scale = double(p->Ky) / (2.0 * M_PI);
  p->has_theta = D.theta != nullptr;
  p->block_off.assign(D.block_off, D.block_off + D.d + 1);
  p->ws = static_cast<char*>(workspace);
  p->ws_bytes = ws_bytes;
  p->ws_measure = measure != nullptr;

  // ---- binning: counting sort by tile inside every block -------------------
  const int64_t M = D.M;
  const int ntiles = p->tiles_x * p->tiles_y;
  std::vector<int32_t> key(M), cell(M);
  for (int64_t i = 0; i < M; ++i) {
    const double tu = double(D.omega_u[i]) * p->su_scale;
    const double tv = double(D.omega_v[i]) * p->sv_scale;
    const int cu0 = (int(std::floor(tu)) - 3) & (p->Kx - 1);
    const int cv0 = (int(std::floor(tv)) - 3) & (p->Ky - 1);
    key[i] = (cv0 / p->T) * p->tiles_x + (cu0 / p->T);
    cell[i] = cv0 * p->Kx + cu0;
  }
  p->perm_host.resize(M);
  std::vector<int64_t> cnt(ntiles + 1);
  // bins (block j, tile t) -> plan range, collected per tile in block order
  struct Bin { int64_t start, count; int32_t block; };
  std::vector<std::vector<Bin>> tile_bins(ntiles);
  for (int j = 0; j < p->d; ++j) {
    const int64_t b0 = p->block_off[j], b1 = p->block_off[j + 1];
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t i = b0; i < b1; ++i) cnt[key[i] + 1]++;
    for (int t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t i = b0; i < b1; ++i) p->perm_host[b0 + pos[key[i]]++] = int32_t(i);
    // inside each bin, order by first-tap cell (row-major within the tile):
    // neighbouring lanes then touch neighbouring cells
    for (int t = 0; t < ntiles; ++t) {
      int32_t* a = p->perm_host.data() + b0 + cnt[t];
      std::stable_sort(a, a + (cnt[t + 1] - cnt[t]),
                       [&](int32_t x, int32_t y) { return cell[x] < cell[y]; });
    }
    for (int t = 0; t < ntiles; ++t)
      if (cnt[t + 1] > cnt[t]) tile_bins[t].push_back({b0 + cnt[t], cnt[t + 1] - cnt[t], j});
  }
  // work items: each tile's visibilities (all blocks) cut into <= chunk_max
  // pieces, a piece being a list of per-block segments.  8 x 8 tiles (one
  // wave per item, work in batches of 64) take full chunk_max pieces and a
  // remainder, which needs the fewest batches; larger tiles (several waves
  // per item) take pieces of near-equal size, which balances the waves.
  std::vector<Item> items;
  std::vector<Seg> segs;
  std::vector<int32_t> tile_item_off(ntiles + 1, 0);
  for (int t = 0; t < ntiles; ++t) {
    int64_t total = 0;
    for (const Bin& b : tile_bins[t]) total += b.count;
    tile_item_off[t] = int32_t(items.size());
    if (total == 0) continue;
    size_t bi = 0;
    int64_t used = 0;   // visibilities of tile_bins[t][bi] already assigned
    int64_t left = total;
    while (left > 0) {
      const int64_t nit = (left + chunk_max - 1) / chunk_max;
      int64_t want = p->T == 8 ? std::min<int64_t>(left, chunk_max) : (left + nit - 1) / nit;
      Item it{};
      it.tx = t % p->tiles_x;
      it.ty = t / p->tiles_x;
      it.seg0 = int32_t(segs.size());
      while (want > 0 && int(segs.size()) - it.seg0 < MAX_ITEM_SEGS) {
        const Bin& b = tile_bins[t][bi];
        const int64_t take = std::min(want, b.count - used);
        segs.push_back({int32_t(b.start + used), int32_t(take), b.block, int32_t(items.size())});
        used += take;
        want -= take;
        left -= take;
        if (used == b.count) {
          ++bi;
          used = 0;
        }
      }
      it.seg1 = int32_t(segs.size());
      items.push_back(it);
    }
  }
  tile_item_off[ntiles] = int32_t(items.size());
  // fold order: the tiles of tile row ty go to XCD ty mod 8 (horizontal
  // neighbours, which share cache lines of the item regions, meet in one L2;
  // the dense rows are spread over all XCDs), and each XCD takes its tiles
  // by decreasing number of item regions to sum (own and left / upper /
  // upper-left halos), so the long sums start first.  The per-XCD lists of
  // fold workgroups (4 tile slots each) are padded to a common length with
  // -1 (no tile).
  std::vector<int32_t> fold_wg;
  std::vector<std::vector<int32_t>> fold_wg_lists;
  {
    std::vector<int32_t> work(ntiles);
    for (int t = 0; t < ntiles; ++t) {
      const int tx = t % p->tiles_x, ty = t / p->tiles_x;
      const int lx = (tx + p->tiles_x - 1) % p->tiles_x, uy = (ty + p->tiles_y - 1) % p->tiles_y;
      auto n = [&](int u) { return tile_item_off[u + 1] - tile_item_off[u]; };
      work[t] = n(t) + n(ty * p->tiles_x + lx) + n(uy * p->tiles_x + tx) + n(uy * p->tiles_x + lx);
    }
    std::vector<std::vector<int32_t>> lists(MAX_XCD);
    for (int t = 0; t < ntiles; ++t) lists[(t / p->tiles_x) % MAX_XCD].push_back(t);
    for (auto& l : lists)
      std::stable_sort(l.begin(), l.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
    for (auto& l : lists) {
      // workgroups of the 4-wave fold: a tile with more than FOLD_HEAVY item
      // regions to sum gets all four waves, the others go four to a
      // workgroup, in the same per-XCD order
      std::vector<int32_t> wg;
      for (size_t i = 0; i < l.size();) {
        if (work[l[i]] > FOLD_HEAVY) {
          wg.insert(wg.end(), {l[i], -2, -2, -2});
          ++i;
          continue;
        }
        int32_t e[4] = {-1, -1, -1, -1};
        for (int k = 0; k < 4 && i < l.size() && work[l[i]] <= FOLD_HEAVY; ++k) e[k] = l[i++];
        wg.insert(wg.end(), e, e + 4);
      }
      fold_wg_lists.push_back(wg);
    }
    size_t per_wg = 0;
    for (auto& w : fold_wg_lists) per_wg = std::max(per_wg, w.size());
    for (auto& w : fold_wg_lists) {
      w.resize(per_wg, -1);
      fold_wg.insert(fold_wg.end(), w.begin(), w.end());
    }
  }
  p->n_items = int(items.size());
  p->n_segs = int(segs.size());
  p->n_tiles = ntiles;
  // work-balanced XCD bands of the item launches: the cost of an item is
  // its 64-point batches plus one for staging and storing its region
  {
    std::vector<double> cost(p->n_items);
    for (int i = 0; i < p->n_items; ++i) {
      int64_t c = 0;
      for (int g = items[i].seg0; g < items[i].seg1; ++g) c += segs[g].count;
      cost[i] = double((c + 63) / 64) + 1.0;
    }
    auto split = [&](int unit) {
      XcdSplit sp{};
      sp.unit = unit;
      const int nu = (p->n_items + unit - 1) / unit;
      std::vector<double> pre(nu + 1, 0.0);
      for (int u = 0; u < nu; ++u) {
        double c = 0.0;
        for (int i = u * unit; i < std::min(p->n_items, (u + 1) * unit); ++i) c += cost[i];
        pre[u + 1] = pre[u] + c;
      }
      sp.off[0] = 0;
      sp.off[MAX_XCD] = nu;
      int u = 0;
      for (int k = 1; k < MAX_XCD; ++k) {
        const double target = pre[nu] * k / MAX_XCD;
        while (u < nu && pre[u] < target) ++u;
        sp.off[k] = u;
      }
      int longest = 0;
      for (int k = 0; k < MAX_XCD; ++k) longest = std::max(longest, sp.off[k + 1] - sp.off[k]);
      sp.launch = std::max(1, longest) * MAX_XCD;
      return sp;
    };
    p->split1 = split(1);
    p->split_degrid = split(PPD_DEGRID_RUN > 0 ? PPD_DEGRID_RUN : 1);
    p->split_grid = split(PPD_GRIDM_RUN * PPD_GRIDM_WPG);
  }
  p->n_tile_launch = ((ntiles + MAX_XCD - 1) / MAX_XCD) * MAX_XCD;
  p->items_host = items;
  p->segs_host = segs;
  p->bseg_off.assign(p->d + 1, 0);
  for (const Seg& sg : segs) p->bseg_off[sg.block + 1]++;
  for (int j = 0; j < p->d; ++j) p->bseg_off[j + 1] += p->bseg_off[j];
  std::vector<int32_t> bids(p->n_segs);
  {
    std::vector<int32_t> fill(p->bseg_off.begin(), p->bseg_off.end() - 1);
    for (int c = 0; c < p->n_segs; ++c) bids[fill[segs[c].block]++] = c;
  }

  // ---- host tables -----------------------------------------------------------
  std::vector<float> wu(M), wv(M), th;
  for (int64_t i = 0; i < M; ++i) {
    wu[i] = D.omega_u[p->perm_host[i]];
    wv[i] = D.omega_v[p->perm_host[i]];
  }
  if (D.theta) {
    th.resize(M);
    for (int64_t i = 0; i < M; ++i) th[i] = D.theta[p->perm_host[i]];
  }
  std::vector<int32_t> vblk(M);
  for (int j = 0; j < p->d; ++j)
    for (int64_t i = p->block_off[j]; i < p->block_off[j + 1]; ++i) vblk[i] = j;
  float kbc[KB_TAPS * KB_NC];
  kb_tap_polynomials(p->beta, kbc);
  std::vector<float> dpx(p->nx), dpy(p->ny);
  for (int c = 0; c < p->nx; ++c) dpx[c] = float(1.0 / kb_ft(double(c - p->nx / 2) / p->Kx, p->beta));
  for (int r = 0; r < p->ny; ++r) dpy[r] = float(1.0 / kb_ft(double(r - p->ny / 2) / p->Ky, p->beta));
  auto twiddles = [](int K) {
    std::vector<float2> t(K / 2);
    for (int k = 0; k < K / 2; ++k) {
      const double a = -2.0 * M_PI * double(k) / double(K);
      t[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
    return t;
  };
  std::vector<float2> twx = twiddles(p->Kx), twy = twiddles(p->Ky);
  std::vector<float> filt(8 * 2 * FILT_STRIDE, 0.0f);
  for (int q = 1; q <= 8; ++q) {
    double h[FILT_STRIDE];
    daubechies(q, h);
    const int L = 2 * q;
    for (int n = 0; n < L; ++n) {
      filt[(q - 1) * 2 * FILT_STRIDE + n] = float(h[n]);
      filt[(q - 1) * 2 * FILT_STRIDE + FILT_STRIDE + n] = float(((n & 1) ? -1.0 : 1.0) * h[L - 1 - n]);
    }
  }

  // chunks of the exact prox's Newton passes (SEC_CHUNK points, one block each)
  std::vector<int32_t> cstart, cblock, coff(p->d + 1, 0);
  for (int j = 0; j < p->d; ++j) {
    coff[j] = int32_t(cblock.size());
    for (int64_t s0 = p->block_off[j]; s0 < p->block_off[j + 1]; s0 += SEC_CHUNK) {
      cstart.push_back(int32_t(s0));
      cblock.push_back(j);
    }
  }
  coff[p->d] = int32_t(cblock.size());
  cstart.push_back(int32_t(M));
  p->n_sec_chunks = int(cblock.size());

  // persistent Algorithm 2: workgroup g owns plan-order points
  // [g PA_CHUNK, (g+1) PA_CHUNK); its first block, and each block's range of
  // workgroups (blocks are contiguous in plan order)
  p->pa_groups = int((M + PA_CHUNK - 1) / PA_CHUNK);
  std::vector<int32_t> wgb0(p->pa_groups), gfirst(p->d), glast(p->d), voff(p->d + 1);
  bool pa_fits = true;
  {
    int j = 0;
    for (int g = 0; g < p->pa_groups; ++g) {
      const int64_t a0 = int64_t(g) * PA_CHUNK, a1 = std::min<int64_t>(a0 + PA_CHUNK, M);
      while (p->block_off[j + 1] <= a0) ++j;
      wgb0[g] = j;
      int nb = 1;
      while (j + nb < p->d && p->block_off[j + nb] < a1) ++nb;
      if (nb > PA_MAXB) pa_fits = false;
    }
    for (int jj = 0; jj < p->d; ++jj) {
      gfirst[jj] = int32_t(p->block_off[jj] / PA_CHUNK);
      glast[jj] = int32_t((p->block_off[jj + 1] - 1) / PA_CHUNK);
    }
    for (int jj = 0; jj <= p->d; ++jj) voff[jj] = int32_t(p->block_off[jj]);
  }

  // ---- device memory -----------------------------------------------------------
  const size_t K2 = size_t(p->Kx) * p->Ky;
  const size_t N = size_t(p->nx) * p->ny;
  int st = PPD_OK;
  auto A = [&](int s) { if (st == PPD_OK) st = s; };
  A(dalloc(p, &p->wu, M));
  A(dalloc(p, &p->wv, M));
  if (D.theta) A(dalloc(p, &p->theta, M));
  A(dalloc(p, &p->perm, M));
  A(dalloc(p, &p->items, p->n_items));
  A(dalloc(p, &p->segs, p->n_segs));
  A(dalloc(p, &p->tile_item_off, ntiles + 1));
  A(dalloc(p, &p->fold_wg, fold_wg.size()));
  p->n_fold_wg = int(fold_wg.size() / 4);
  A(dalloc(p, &p->bseg_ids, p->n_segs));
  A(dalloc(p, &p->bseg_off_d, p->d + 1));
  A(dalloc(p, &p->bfac, p->d));
  A(dalloc(p, &p->gscratch, size_t(p->n_items) * (p->T + 7) * (p->T + 7)));
  A(dalloc(p, &p->vis_block, M));
  A(dalloc(p, &p->kbc, KB_TAPS * KB_NC));
  A(dalloc(p, &p->dpx, p->nx));
  A(dalloc(p, &p->dpy, p->ny));
  A(dalloc(p, &p->twx, p->Kx / 2));
  A(dalloc(p, &p->twy, p->Ky / 2));
  A(dalloc(p, &p->filt, filt.size()));
  A(dalloc(p, &p->grid_f, K2));
  A(dalloc(p, &p->grid_a, K2));
  A(dalloc(p, &p->half, size_t(p->ny) * p->Kx));
  A(dalloc(p, &p->half_f, size_t(p->ny) * p->Kx));
  A(dalloc(p, &p->ybuf, M));
  A(dalloc(p, &p->wbuf, M));
  A(dalloc(p, &p->gabuf, M));
  A(dalloc(p, &p->qbuf, M));
  A(dalloc(p, &p->sec_cstart, cstart.size()));
  A(dalloc(p, &p->sec_cblock, cblock.size()));
  A(dalloc(p, &p->sec_coff, coff.size()));
  A(dalloc(p, &p->sec_part, 4 * cblock.size()));
  A(dalloc(p, &p->sec_nu, 2 * size_t(p->d)));
  A(dalloc(p, &p->du_blk, p->d));
  A(dalloc(p, &p->voff_d, p->d + 1));
  A(dalloc(p, &p->pa_wgb0, p->pa_groups));
  A(dalloc(p, &p->pa_gfirst, p->d));
  A(dalloc(p, &p->pa_glast, p->d));
  A(dalloc(p, &p->pa_part, 2 * size_t(p->pa_groups) * PA_MAXB));
  A(dalloc(p, &p->pa_sync, PA_SYNC_WORDS));
  A(dalloc(p, &p->part, 2 * size_t(p->n_segs)));
  A(dalloc(p, &p->rpart, p->n_segs));
  A(dalloc(p, &p->eps_d, p->d));
  A(dalloc(p, &p->ppart, size_t(p->ny) * 4));
  A(dalloc(p, &p->stats_d, 8 + p->d));
  A(dalloc(p, &p->hist_cursor, 1));
  A(dalloc(p, &p->rj_d, p->d));
  // SARA temporaries: low-pass bands of levels 1..L-1 for 8 wavelet bases
  size_t ll = 0;
  for (int l = 1; l < levels; ++l) ll += N >> (2 * l);
  p->sara_ll_floats = ll;
  A(dalloc(p, &p->sara_ll, 8 * ll));
  A(dalloc(p, &p->sara_rec, 8 * ll));
  A(dalloc(p, &p->ut, N));
  A(dalloc(p, &p->img_tmp, N));
  A(dalloc(p, &p->vec_tmp, N));
  A(dalloc(p, &p->pl_part, 1024));
  A(dalloc(p, &p->res_sq, p->d));
  A(dalloc(p, &p->pl_scalar, 4));
  A(dalloc(p, &p->icount, N));
  A(dalloc(p, &p->imin, 1));
  if (measure) {
    *measure = (p->ws_used + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN;
    destroy_plan(p);
    return st;
  }
  p->stream = static_cast<hipStream_t>(stream);
  (void)hipGetDevice(&p->device);
  if (st != PPD_OK) {
    destroy_plan(p);
    return st;
  }
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (st == PPD_OK && hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
      st = fail(PPD_EDEVICE, "hipMemcpy upload failed");
  };
  up(p->wu, wu.data(), 4 * M);
  up(p->wv, wv.data(), 4 * M);
  if (D.theta) up(p->theta, th.data(), 4 * M);
  up(p->perm, p->perm_host.data(), 4 * M);
  up(p->items, items.data(), sizeof(Item) * p->n_items);
  up(p->segs, segs.data(), sizeof(Seg) * p->n_segs);
  up(p->tile_item_off, tile_item_off.data(), 4 * (ntiles + 1));
  up(p->fold_wg, fold_wg.data(), 4 * fold_wg.size());
  up(p->sec_cstart, cstart.data(), 4 * cstart.size());
  up(p->sec_cblock, cblock.data(), 4 * cblock.size());
  up(p->sec_coff, coff.data(), 4 * coff.size());
  up(p->bseg_ids, bids.data(), 4 * p->n_segs);
  up(p->bseg_off_d, p->bseg_off.data(), 4 * (p->d + 1));
  up(p->vis_block, vblk.data(), 4 * M);
  up(p->kbc, kbc, sizeof(kbc));
  up(p->dpx, dpx.data(), 4 * p->nx);
  up(p->dpy, dpy.data(), 4 * p->ny);
  up(p->twx, twx.data(), sizeof(float2) * twx.size());
  up(p->twy, twy.data(), sizeof(float2) * twy.size());
  up(p->filt, filt.data(), 4 * filt.size());
  up(p->voff_d, voff.data(), 4 * voff.size());
  up(p->pa_wgb0, wgb0.data(), 4 * wgb0.size());
  up(p->pa_gfirst, gfirst.data(), 4 * gfirst.size());
  up(p->pa_glast, glast.data(), 4 * glast.size());
  {
    const std::vector<uint32_t> zeros(PA_SYNC_WORDS, 0u);
    up(p->pa_sync, zeros.data(), sizeof(uint32_t) * zeros.size());
    const std::vector<uint64_t> empty(2 * size_t(p->pa_groups) * PA_MAXB, PA_EMPTY);
    up(p->pa_part, empty.data(), sizeof(uint64_t) * empty.size());
  }
  // the persistent launch needs all its workgroups on the device at once
  if (st == PPD_OK) {
    p->pa_ok = pa_fits && p->pa_groups <= alg2_persistent_capacity();
  }
  // mapped pinned host memory the final statistics reduction writes into
  if (st == PPD_OK && (hipHostMalloc(reinterpret_cast<void**>(&p->host_stats), sizeof(double) * (9 + p->d),
                                     hipHostMallocMapped) != hipSuccess ||
                       hipHostGetDevicePointer(reinterpret_cast<void**>(&p->host_stats_dev), p->host_stats, 0) !=
                           hipSuccess))
    st = fail(PPD_ENOMEM, "mapped pinned memory for the statistics read-back failed");
  // default priority on purpose: both streams of an iteration are equal
  if (st == PPD_OK && (hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess ||
                       hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
                       hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess))
    st = fail(PPD_EDEVICE, "creating the second stream failed");
  if (st == PPD_OK && hipDeviceSynchronize() != hipSuccess) st = fail(PPD_EDEVICE, "sync failed");
  if (st != PPD_OK) {
    destroy_plan(p);
    return st;
  }
  *out = p;
  return PPD_OK;
}

extern "C" {

int ppd_plan_create(ppd_plan** out, const ppd_plan_desc* desc, void* stream) {
  return create_plan(out, desc, stream, nullptr, 0, nullptr);
}

int ppd_plan_workspace_size(const ppd_plan_desc* desc, size_t* bytes) {
  if (!bytes) return fail(PPD_EINVAL, "ppd_plan_workspace_size: NULL bytes");
  *bytes = 0;
  ppd_plan* unused = nullptr;
  return create_plan(&unused, desc, nullptr, nullptr, 0, bytes);
}

int ppd_plan_create_ws(ppd_plan** out, const ppd_plan_desc* desc, void* workspace, size_t bytes, void* stream) {
  if (!out) return fail(PPD_EINVAL, "ppd_plan_create_ws: NULL plan");
  *out = nullptr;
  if (!workspace) return fail(PPD_EINVAL, "ppd_plan_create_ws: NULL workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN)
    return fail(PPD_EINVAL, "ppd_plan_create_ws: workspace must be 256-byte aligned");
  return create_plan(out, desc, stream, workspace, bytes, nullptr);
}

int ppd_plan_destroy(ppd_plan* plan) {
  destroy_plan(plan);
  return PPD_OK;
}

int ppd_plan_set_stream(ppd_plan* plan, void* stream) {
  if (!plan) return fail(PPD_EINVAL, "NULL plan");
  for (int k = 0; k < ppd::GRAPH_SLOTS; ++k) {
    if (plan->graph_exec[k]) (void)hipGraphExecDestroy(plan->graph_exec[k]);
    if (plan->graph[k]) (void)hipGraphDestroy(plan->graph[k]);
    plan->graph_exec[k] = nullptr;
    plan->graph[k] = nullptr;
    plan->graph_key[k].clear();
  }
  plan->stream = static_cast<hipStream_t>(stream);
  return PPD_OK;
}

int ppd_plan_get_info(const ppd_plan* p, ppd_plan_info* info) {
  if (!p || !info) return fail(PPD_EINVAL, "NULL argument");
  info->nx = p->nx;
  info->ny = p->ny;
  info->Kx = p->Kx;
  info->Ky = p->Ky;
  info->M = p->M;
  info->d = p->d;
  info->levels = p->levels;
  info->tile = p->T;
  info->chunk = p->chunk_max;
  info->n_chunks = p->n_items;
  info->kb_beta = p->beta;
  info->device_bytes = p->device_bytes;
  info->persistent = p->pa_ok ? 1 : 0;
  info->pad_ = 0;
  return PPD_OK;
}

int ppd_plan_permutation(const ppd_plan* p, int64_t* perm) {
  if (!p || !perm) return fail(PPD_EINVAL, "NULL argument");
  for (int64_t i = 0; i < p->M; ++i) perm[i] = p->perm_host[i];
  return PPD_OK;
}

int ppd_plan_permute(ppd_plan* p, int direction, const void* in, void* out, int elem_bytes) {
  if (!p || !in || !out) return fail(PPD_EINVAL, "NULL argument");
  if (direction != PPD_USER_TO_PLAN && direction != PPD_PLAN_TO_USER)
    return fail(PPD_EINVAL, "bad direction");
  if (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16)
    return fail(PPD_EINVAL, "elem_bytes must be 4, 8 or 16");
  if (in == out) return fail(PPD_EINVAL, "permute cannot run in place");
  return permute(p, direction, in, out, elem_bytes);
}

int ppd_timing_enable(ppd_plan* p, int on) {
  if (!p) return fail(PPD_EINVAL, "NULL plan");
  p->timing = on != 0;
  return PPD_OK;
}

int ppd_timing_reset(ppd_plan* p) {
  if (!p) return fail(PPD_EINVAL, "NULL plan");
  PPD_HIP(hipStreamSynchronize(p->stream));
  p->ev_pending.clear();
  for (int k = 0; k < KK_COUNT; ++k) {
    p->t_counts[k] = 0;
    p->t_ms[k] = 0.0;
  }
  return PPD_OK;
}

int ppd_timing_read(ppd_plan* p, int cap, const char** names, int64_t* counts, double* total_ms,
                    int* n_kinds) {
  if (!p || !n_kinds) return fail(PPD_EINVAL, "NULL argument");
  PPD_HIP(hipStreamSynchronize(p->stream));
  for (auto& pr : p->ev_pending) {
    float ms = 0.0f;
    PPD_HIP(hipEventElapsedTime(&ms, p->ev_pool[2 * pr.second], p->ev_pool[2 * pr.second + 1]));
    p->t_counts[pr.first]++;
    p->t_ms[pr.first] += ms;
  }
  p->ev_pending.clear();
  int n = 0;
  for (int k = 0; k < KK_COUNT; ++k) {
    if (p->t_counts[k] == 0) continue;
    if (n < cap) {
      if (names) names[n] = kernel_kind_name(k);
      if (counts) counts[n] = p->t_counts[k];
      if (total_ms) total_ms[n] = p->t_ms[k];
    }
    ++n;
  }
  *n_kinds = n;
  return PPD_OK;
}

}  // extern "C"

namespace ppd {

int timer_begin(ppd_plan* p, int kind, int* slot) {
  *slot = -1;
  if (!p->timing) return PPD_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  PPD_HIP(hipStreamIsCapturing(p->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return PPD_OK;
  const int idx = int(p->ev_pending.size());
  while (p->ev_pool.size() < size_t(2 * (idx + 1))) {
    hipEvent_t e;
    PPD_HIP(hipEventCreate(&e));
    p->ev_pool.push_back(e);
  }
  PPD_HIP(hipEventRecord(p->ev_pool[2 * idx], p->stream));
  p->ev_pending.push_back({kind, idx});
  *slot = idx;
  return PPD_OK;
}

int timer_end(ppd_plan* p, int slot) {
  if (slot < 0) return PPD_OK;
  PPD_HIP(hipEventRecord(p->ev_pool[2 * slot + 1], p->stream));
  return PPD_OK;
}

}  // namespace ppd
