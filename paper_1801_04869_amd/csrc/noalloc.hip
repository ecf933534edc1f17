// Entry point that allocates nothing: the film magnetic moment of
// mag_observe for callers that cannot call hipMalloc (code under HIP graph
// capture, tight serving loops).  Its per-block partial sums live in a
// file-scope device array instead of context workspace; the host reaches
// that array only through the address hipGetSymbolAddress returns for the
// current device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/magfft.h"
#include "kern_common.h"

namespace mag {
namespace {

constexpr int kMomThreads = 256;
constexpr int kMomNpt = 8;                       // nodes per thread
constexpr int kMomBlockNodes = kMomThreads * kMomNpt;

// One slot per block of the partial-sum kernel.  Shared by every call on a
// device: calls that overlap on one device race on it.
__device__ __align__(256) double scratch[MAG_NOALLOC_MAX_PARTS];

constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (set up once per device).
double *scratch_ptr(int *err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = MAG_E_HIP;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      *err = MAG_E_HIP;
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *err = MAG_OK;
  return g_scratch_ptr[dev];
}

// part[b] = sum of g over nodes [b * kMomBlockNodes, (b + 1) * kMomBlockNodes),
// a fixed summation order (per thread in index order, then the block total).
__global__ void __launch_bounds__(kMomThreads) moment_parts(const double *__restrict__ g, long long n,
                                                            double *__restrict__ part) {
  __shared__ double red[kMomThreads / 64];
  const long long i0 = (long long)blockIdx.x * kMomBlockNodes + threadIdx.x;
  double v[kMomNpt];
#pragma unroll
  for (int k = 0; k < kMomNpt; ++k) {
    const long long i = i0 + (long long)k * kMomThreads;
    v[k] = i < n ? g[i] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kMomNpt; ++k) acc += v[k];
  const double s = block_total<kMomThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// m = (0, 0, dxdy * sum of part[0..nb)); one block, fixed order.
__global__ void __launch_bounds__(kMomThreads) moment_final(const double *__restrict__ part, int nb, double dxdy,
                                                            double *__restrict__ m) {
  __shared__ double sh[kMomThreads];
  const double s = fixed_sum256<kMomThreads>(part, nb, sh);
  if (threadIdx.x == 0) {
    m[0] = 0.0;
    m[1] = 0.0;
    m[2] = s * dxdy;
  }
}

}  // namespace

// Called by mag_create: the current device's scratch address is looked up at
// set-up time, before any capture the caller may start.
int noalloc_setup() {
  int err = MAG_OK;
  (void)scratch_ptr(&err);
  return err;
}

}  // namespace mag

extern "C" int mag_film_moment_noalloc(const double *g, int nx, int ny, double Lx, double Ly, double *m,
                                       void *hip_stream) {
  if (!g || !m) return MAG_E_ARG;
  if (nx < 1 || ny < 1 || !(Lx > 0) || !(Ly > 0) || !std::isfinite(Lx) || !std::isfinite(Ly)) return MAG_E_ARG;
  const long long n = (long long)nx * ny;
  const long long nb = (n + mag::kMomBlockNodes - 1) / mag::kMomBlockNodes;
  if (nb > MAG_NOALLOC_MAX_PARTS) return MAG_E_ARG;   // more than MAG_NOALLOC_MAX_PARTS * 2048 nodes
  int err = MAG_OK;
  double *part = mag::scratch_ptr(&err);
  if (!part) return err;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const double dxdy = (2.0 * Lx / nx) * (2.0 * Ly / ny);
  hipLaunchKernelGGL(mag::moment_parts, dim3((unsigned)nb), dim3(mag::kMomThreads), 0, s, g, n, part);
  hipLaunchKernelGGL(mag::moment_final, dim3(1), dim3(mag::kMomThreads), 0, s, part, (int)nb, dxdy, m);
  return hipGetLastError() == hipSuccess ? MAG_OK : MAG_E_HIP;
}
