// CPU emulation of the small part of the HIP runtime and device language the
// library uses.  TEST INFRASTRUCTURE ONLY: it lets the unmodified library
// sources run on the host under AddressSanitizer, one work-group at a time
// with one std::thread per work-item, so that every global, LDS and
// dynamic-LDS access is bounds-checked.  Nothing in the product links it.
#pragma once
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint3v { unsigned x, y, z; };
struct double2 { double x, y; };

namespace emu {
inline thread_local dim3 tIdx, bIdx;
inline dim3 bDim, gDim;
inline std::barrier<> *bar = nullptr;
inline unsigned char *dyn = nullptr;
}  // namespace emu

#define threadIdx (emu::tIdx)
#define blockIdx (emu::bIdx)
#define blockDim (emu::bDim)
#define gridDim (emu::gDim)
#define HIP_DYNAMIC_SHARED(type, var) type *var = reinterpret_cast<type *>(emu::dyn);

inline void __syncthreads() { emu::bar->arrive_and_wait(); }

// Cross-lane exchange within a 64-wide wavefront, emulated through a per-block
// buffer between two block barriers (all work-items of the block must call it
// together, which the library's uniform reductions do).
namespace emu {
inline std::vector<double> *xbuf = nullptr;
}
inline double __shfl_xor(double v, int mask, int width = 64) {
  const unsigned t = threadIdx.x + emu::bDim.x * (threadIdx.y + emu::bDim.y * threadIdx.z);
  (*emu::xbuf)[t] = v;
  __syncthreads();
  const unsigned base = t & ~63u;
  const double r = (*emu::xbuf)[base + ((t - base) ^ (unsigned)mask)];
  __syncthreads();
  (void)width;
  return r;
}

using std::exp;
using std::fabs;
using std::fmax;
using std::isfinite;
using std::isnan;
using std::log;
using std::sqrt;

typedef int hipError_t;
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };

// Fresh device allocations are filled with 0xff bytes (NaN for float and
// double) so that reads of never-written device memory show up in results.
inline hipError_t hipMalloc(void *p, size_t n) {
  void *q = std::malloc(n ? n : 1);
  std::memset(q, 0xff, n ? n : 1);
  *reinterpret_cast<void **>(p) = q;
  return hipSuccess;
}
template <typename T>
inline hipError_t hipMallocAsync(T **p, size_t n, hipStream_t) { return hipMalloc(p, n); }
inline float rsqrtf(float x) { return 1.0f / std::sqrt(x); }
#define __align__(n) alignas(n)
#define MAG_OPAQUE(x) asm volatile("" : "+m"(x))
#define MAG_WAVES_PER_EU(...)
#define hipHostMallocCoherent 0x40000000u
inline hipError_t hipHostMalloc(void *p, size_t n, unsigned = 0) { return hipMalloc(p, n); }
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipFreeAsync(void *p, hipStream_t) { std::free(p); return hipSuccess; }
inline hipError_t hipHostFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "emu"; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = nullptr; return 1; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0; return hipSuccess; }

template <typename... KA, typename... A>
void emu_launch(void (*k)(KA...), dim3 g, dim3 b, size_t shm, A... args) {
  const unsigned nt = b.x * b.y * b.z;
  emu::bDim = b;
  emu::gDim = g;
  std::vector<unsigned char> dynbuf;
  for (unsigned bz = 0; bz < g.z; ++bz)
    for (unsigned by = 0; by < g.y; ++by)
      for (unsigned bx = 0; bx < g.x; ++bx) {
        unsigned char *d = shm ? static_cast<unsigned char *>(std::malloc(shm)) : nullptr;
        if (d) std::memset(d, 0xff, shm);
        emu::dyn = d;
        std::barrier<> br((std::ptrdiff_t)nt);
        emu::bar = &br;
        std::vector<double> xb(((nt + 63) / 64) * 64, 0.0);
        emu::xbuf = &xb;
        std::vector<std::thread> th;
        th.reserve(nt);
        for (unsigned t = 0; t < nt; ++t)
          th.emplace_back([&, t]() {
            emu::tIdx = dim3(t % b.x, (t / b.x) % b.y, t / (b.x * b.y));
            emu::bIdx = dim3(bx, by, bz);
            k(args...);
            br.arrive_and_drop();
          });
        for (auto &x : th) x.join();
        std::free(d);
      }
}
#define hipLaunchKernelGGL(K, G, B, S, STREAM, ...) emu_launch(K, dim3(G), dim3(B), (size_t)(S), __VA_ARGS__)
