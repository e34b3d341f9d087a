// Algorithm 2 (Sec. 4.1) without any device allocation: the same
// forward-backward iterations as ppd_ellipsoid_proj, for callers that
// cannot allocate (graph capture, serving loops), with every intermediate
// in one file-scope device array instead of a plan's buffers.
//
// The visibilities of block j are the contiguous range
// [block_off[j], block_off[j+1]); each block is cut into chunks of NA_CHUNK
// consecutive points, one workgroup each.  A step forms, per chunk, the
// partial sum of ||q - y_j||^2 with q = z - mu U (z - w); a second launch
// sums each block's chunk partials in a fixed order and stores the block's
// P_B factor; the next step first applies z <- P_B(q) with it.  All partial
// and factor slots are written before they are read in every call, so
// nothing has to start at zero.
#include <mutex>

#include "ppd_internal.h"

namespace ppd {
namespace {

constexpr int NA_CHUNK = 8192;        // points per workgroup
constexpr int NA_THREADS = 256;
constexpr int NA_MAX_BLOCKS = 4096;
constexpr int NA_MAX_CHUNKS = 65536;

// Layout of the array (byte offsets): eps [d] f64, block offsets [d+1] i64,
// chunk offsets [d+1] i32 (chunks of block j: [coff[j], coff[j+1])), block
// factors [d] (factor, inside) f64 pairs, chunk partials [n_chunks] f64.
constexpr size_t NA_OFF_EPS = 0;
constexpr size_t NA_OFF_BOFF = NA_OFF_EPS + 8 * NA_MAX_BLOCKS;
constexpr size_t NA_OFF_COFF = NA_OFF_BOFF + 8 * (NA_MAX_BLOCKS + 1);
constexpr size_t NA_OFF_FAC = (NA_OFF_COFF + 4 * (NA_MAX_BLOCKS + 1) + 255) / 256 * 256;
constexpr size_t NA_OFF_PART = NA_OFF_FAC + 16 * NA_MAX_BLOCKS;
constexpr size_t NA_BYTES = NA_OFF_PART + 8 * NA_MAX_CHUNKS;

// One copy per GPU, held until the process ends (about 0.7 MiB).  Host code
// never uses this name as an address: it takes the device address from
// hipGetSymbolAddress once per device (see scratch_for_device).
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

struct NaView {
  const double* eps;
  const int64_t* boff;
  const int32_t* coff;
  double2* fac;
  double* part;
};

__device__ __forceinline__ NaView na_view(unsigned char* base) {
  return {reinterpret_cast<const double*>(base + NA_OFF_EPS), reinterpret_cast<const int64_t*>(base + NA_OFF_BOFF),
          reinterpret_cast<const int32_t*>(base + NA_OFF_COFF), reinterpret_cast<double2*>(base + NA_OFF_FAC),
          reinterpret_cast<double*>(base + NA_OFF_PART)};
}

__device__ __forceinline__ double na_block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NA_THREADS / 64; ++k) s += red[k];
  return s;
}

// mode 0: partials of ||q - y||^2 from z; mode 1: z <- P_B(q) with the block
// factors, then partials of the next q; mode 2: z <- P_B(q) only.
__global__ __launch_bounds__(NA_THREADS) void k_na_step(int mode, int d, const double2* __restrict__ w,
                                                        const float2* __restrict__ y, const double* __restrict__ U,
                                                        double2* __restrict__ z, double mu,
                                                        unsigned char* __restrict__ base) {
  __shared__ double red[NA_THREADS / 64];
  const NaView s = na_view(base);
  const int c = blockIdx.x;
  int lo = 0, hi = d;   // the block of chunk c: the last j with coff[j] <= c
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s.coff[mid] <= c) lo = mid;
    else hi = mid;
  }
  const int j = lo;
  const int64_t i0 = s.boff[j] + int64_t(c - s.coff[j]) * NA_CHUNK;
  const int64_t i1 = min(i0 + NA_CHUNK, s.boff[j + 1]);
  const double2 bf = mode != 0 ? s.fac[j] : make_double2(1.0, 1.0);
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += NA_THREADS) {
    const double Ue = U[i], mU = mu * Ue;
    const double2 we = w[i];
    const float2 ye = y[i];
    double2 ze = z[i];
    if (mode != 0) {
      const double qx = ze.x - mU * (ze.x - we.x), qy = ze.y - mU * (ze.y - we.y);
      ze.x = bf.y != 0.0 ? qx : double(ye.x) + (qx - double(ye.x)) * bf.x;
      ze.y = bf.y != 0.0 ? qy : double(ye.y) + (qy - double(ye.y)) * bf.x;
      z[i] = ze;
    }
    if (mode != 2) {
      const double dx = (ze.x - mU * (ze.x - we.x)) - double(ye.x);
      const double dy = (ze.y - mU * (ze.y - we.y)) - double(ye.y);
      acc += dx * dx + dy * dy;
    }
  }
  if (mode != 2) {
    acc = na_block_sum(acc, red);
    if (threadIdx.x == 0) s.part[c] = acc;
  }
}

// Block j: r = sqrt(sum of its chunk partials in chunk order); the P_B
// factor (eps_j / r, 0) if r > eps_j, else (1, 1) (Sec. 3.3, eq. proj-L2).
__global__ __launch_bounds__(NA_THREADS) void k_na_factors(unsigned char* __restrict__ base) {
  __shared__ double red[NA_THREADS / 64];
  const NaView s = na_view(base);
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int c = s.coff[j] + int(threadIdx.x); c < s.coff[j + 1]; c += NA_THREADS) acc += s.part[c];
  acc = na_block_sum(acc, red);
  if (threadIdx.x == 0) {
    const double r = sqrt(acc), e = s.eps[j];
    s.fac[j] = r > e ? make_double2(e / r, 0.0) : make_double2(1.0, 1.0);
  }
}

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_na_mutex;
unsigned char* g_na_ptr[NA_MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_for_device(unsigned char** out) {
  int dev = 0;
  PPD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NA_MAX_DEVICES) return fail(PPD_EUNSUPPORTED, "device index beyond the supported count");
  std::lock_guard<std::mutex> lock(g_na_mutex);
  if (!g_na_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PPD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_na_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_na_ptr[dev];
  return PPD_OK;
}

}  // namespace
}  // namespace ppd

using namespace ppd;

extern "C" int ppd_ellipsoid_proj_noalloc(const double* w, const float* y, const double* U, int32_t d,
                                          const int64_t* block_off, const double* eps, int n_itr, double mu,
                                          double* zbar, void* stream) {
  if (!w || !y || !U || !block_off || !eps || !zbar)
    return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: NULL argument");
  if (d < 1 || d > NA_MAX_BLOCKS)
    return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: d must be in [1, " + std::to_string(NA_MAX_BLOCKS) + "]");
  if (n_itr < 1) return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: n_itr must be >= 1");
  if (!(mu > 0.0) || !std::isfinite(mu)) return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: mu must be > 0");
  if (block_off[0] != 0) return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: block_off[0] must be 0");
  int32_t coff[NA_MAX_BLOCKS + 1];
  coff[0] = 0;
  for (int j = 0; j < d; ++j) {
    const int64_t mj = block_off[j + 1] - block_off[j];
    if (mj < 1) return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: block_off must be strictly increasing");
    if (block_off[j + 1] >= (int64_t(1) << 40))
      return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: too many visibilities");
    if (!(eps[j] > 0.0) || !std::isfinite(eps[j]))
      return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: eps must be finite and > 0");
    const int64_t nc = coff[j] + (mj + NA_CHUNK - 1) / NA_CHUNK;
    if (nc > NA_MAX_CHUNKS)
      return fail(PPD_EINVAL, "ppd_ellipsoid_proj_noalloc: more than " + std::to_string(NA_MAX_CHUNKS) +
                                  " chunks of " + std::to_string(NA_CHUNK) + " points (about " +
                                  std::to_string(int64_t(NA_MAX_CHUNKS) * NA_CHUNK) + " visibilities)");
    coff[j + 1] = int32_t(nc);
  }
  const int nchunks = coff[d];
  unsigned char* base = nullptr;
  PPD_TRY(scratch_for_device(&base));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the block tables into the array (pageable host sources are staged by the
  // runtime before these calls return)
  PPD_HIP(hipMemcpyAsync(base + NA_OFF_EPS, eps, sizeof(double) * d, hipMemcpyHostToDevice, s));
  PPD_HIP(hipMemcpyAsync(base + NA_OFF_BOFF, block_off, sizeof(int64_t) * (d + 1), hipMemcpyHostToDevice, s));
  PPD_HIP(hipMemcpyAsync(base + NA_OFF_COFF, coff, sizeof(int32_t) * (d + 1), hipMemcpyHostToDevice, s));
  const double2* w2 = reinterpret_cast<const double2*>(w);
  const float2* y2 = reinterpret_cast<const float2*>(y);
  double2* z2 = reinterpret_cast<double2*>(zbar);
  hipLaunchKernelGGL(k_na_step, dim3(nchunks), dim3(NA_THREADS), 0, s, 0, d, w2, y2, U, z2, mu, base);
  hipLaunchKernelGGL(k_na_factors, dim3(d), dim3(NA_THREADS), 0, s, base);
  for (int k = 1; k < n_itr; ++k) {
    hipLaunchKernelGGL(k_na_step, dim3(nchunks), dim3(NA_THREADS), 0, s, 1, d, w2, y2, U, z2, mu, base);
    hipLaunchKernelGGL(k_na_factors, dim3(d), dim3(NA_THREADS), 0, s, base);
  }
  hipLaunchKernelGGL(k_na_step, dim3(nchunks), dim3(NA_THREADS), 0, s, 2, d, w2, y2, U, z2, mu, base);
  PPD_HIP(hipGetLastError());
  return PPD_OK;
}
