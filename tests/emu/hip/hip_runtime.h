// CPU emulation of the small part of the HIP runtime and device language the
// library uses.  TEST INFRASTRUCTURE ONLY: it lets the unmodified library
// sources run on the host under AddressSanitizer, one work-group at a time
// with one std::thread per work-item, so that every global, LDS and
// dynamic-LDS access is bounds-checked.  Nothing in the product links it.
//
// Device memory is modelled as a separate address space:
//  * hipMalloc / hipMallocAsync allocations are registered as DEVICE memory
//    and ASan-poisoned whenever host code runs, so a host read or write of
//    device memory stops the run with a use-after-poison report;
//  * hipHostMalloc allocations are registered as PINNED host memory
//    (readable by both sides);
//  * every pointer argument of a launch, and every pointer member of a
//    by-value struct argument, must be null or lie inside a live DEVICE or
//    PINNED allocation (a plain host pointer reaching a kernel is a GPU page
//    fault);
//  * every hipMemcpy* kind is checked against the registry;
//  * launch shapes are checked against the hardware limits (block <= 1024
//    work-items, grid.x * block.x < 2^32) and logged, so that the test can
//    compare them with the gfx950 code-object metadata of the same kernels
//    (max flat work-group size, static LDS).
#pragma once
#include <sanitizer/asan_interface.h>

#include <barrier>
#include <condition_variable>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <dlfcn.h>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <type_traits>
#include <utility>
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
struct float2 { float x, y; };

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
// the barrier and fence builtins (the emulated work-items are threads whose
// block barrier already orders every memory access)
#define __builtin_amdgcn_s_barrier() __syncthreads()
#define __builtin_amdgcn_fence(...) ((void)0)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)

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
// Stream capture: launches made while capturing are recorded and run when
// the graph is launched; synchronisation and copies during a capture are
// errors (they are not capturable on the device either).
namespace emu {
struct Graph {
  std::vector<std::function<void()>> ops;
};
inline bool capturing = false;
inline Graph *cap_graph = nullptr;
}  // namespace emu
typedef emu::Graph *hipGraph_t;
typedef emu::Graph *hipGraphExec_t;
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipStreamCaptureModeThreadLocal = 1 };
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };

// ------------------------------------------------------------ allocation registry
namespace emu {
enum Kind { HOST = 0, DEVICE = 1, PINNED = 2 };
struct Alloc {
  size_t n;
  int kind;
};
inline std::map<uintptr_t, Alloc> &reg() {
  static std::map<uintptr_t, Alloc> m;
  return m;
}
inline std::mutex &reg_mu() {
  static std::mutex m;
  return m;
}
inline int violations = 0;

[[noreturn]] inline void fail(const char *fmt, const void *p, const char *what) {
  fprintf(stderr, "EMU-VIOLATION: ");
  fprintf(stderr, fmt, p, what);
  fprintf(stderr, "\n");
  fflush(stderr);
  std::abort();
}

// Kind of the allocation holding p (HOST when none does); *base/*len when found.
inline int kind_of(const void *p, uintptr_t *base = nullptr, size_t *len = nullptr) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto &m = reg();
  auto it = m.upper_bound(a);
  if (it == m.begin()) return HOST;
  --it;
  if (a >= it->first && a < it->first + (it->second.n ? it->second.n : 1)) {
    if (base) *base = it->first;
    if (len) *len = it->second.n;
    return it->second.kind;
  }
  return HOST;
}

inline void poison_device(bool on) {
  for (auto &kv : reg())
    if (kv.second.kind == DEVICE && kv.second.n) {
      if (on) ASAN_POISON_MEMORY_REGION(reinterpret_cast<void *>(kv.first), kv.second.n);
      else ASAN_UNPOISON_MEMORY_REGION(reinterpret_cast<void *>(kv.first), kv.second.n);
    }
}

inline void *reg_alloc(size_t n, int kind) {
  void *q = std::malloc(n ? n : 1);
  std::memset(q, 0xff, n ? n : 1);   // NaN bytes: reads of never-written memory show up
  reg()[reinterpret_cast<uintptr_t>(q)] = Alloc{n, kind};
  if (kind == DEVICE && n) ASAN_POISON_MEMORY_REGION(q, n);
  return q;
}

inline hipError_t reg_free(void *p, int want) {
  if (!p) return hipSuccess;
  auto &m = reg();
  auto it = m.find(reinterpret_cast<uintptr_t>(p));
  if (it == m.end()) fail("free of %p, which is not the start of a live allocation (%s)", p, want == DEVICE ? "hipFree" : "hipHostFree");
  if (it->second.kind != want)
    fail("%p freed with the wrong call (%s)", p, want == DEVICE ? "hipFree on pinned memory" : "hipHostFree on device memory");
  if (it->second.n) ASAN_UNPOISON_MEMORY_REGION(p, it->second.n);
  m.erase(it);
  std::free(p);
  return hipSuccess;
}

// A pointer argument of a kernel: null, or inside a live device / pinned allocation.
inline void check_ptr(const void *p, const char *kname, int argi) {
  if (!p) return;
  const int k = kind_of(p);
  if (k == DEVICE || k == PINNED) return;
  char what[256];
  snprintf(what, sizeof what, "%s, argument %d", kname, argi);
  fail("host pointer %p passed to a kernel (%s)", p, what);
}

// Members of a by-value struct argument, found by aggregate decomposition
// (the kernel-argument structs are aggregates of scalars and pointers), so
// that padding bytes are never taken for addresses.
struct any_t {
  template <class U>
  constexpr operator U() const noexcept;
};
template <class T, class Seq, class = void>
struct ctor_n : std::false_type {};
template <class T, size_t... I>
struct ctor_n<T, std::index_sequence<I...>, std::void_t<decltype(T{((void)I, any_t{})...})>> : std::true_type {};
template <class T, size_t N = 0>
constexpr size_t field_count() {
  if constexpr (N < 24 && ctor_n<T, std::make_index_sequence<N + 1>>::value) return field_count<T, N + 1>();
  else return N;
}
#define EMU_FIELDS(N, ...)                     \
  if constexpr (n == N) {                      \
    const auto &[__VA_ARGS__] = t;             \
    emu_visit(f, __VA_ARGS__);                 \
  }
template <class F, class... X>
inline void emu_visit(F &&f, const X &...x) {
  (f(x), ...);
}
template <class T, class F>
inline void for_each_field(const T &t, F &&f) {
  constexpr size_t n = field_count<T>();
  static_assert(n >= 1 && n <= 16, "kernel-argument struct not decomposable");
  EMU_FIELDS(1, a0)
  EMU_FIELDS(2, a0, a1)
  EMU_FIELDS(3, a0, a1, a2)
  EMU_FIELDS(4, a0, a1, a2, a3)
  EMU_FIELDS(5, a0, a1, a2, a3, a4)
  EMU_FIELDS(6, a0, a1, a2, a3, a4, a5)
  EMU_FIELDS(7, a0, a1, a2, a3, a4, a5, a6)
  EMU_FIELDS(8, a0, a1, a2, a3, a4, a5, a6, a7)
  EMU_FIELDS(9, a0, a1, a2, a3, a4, a5, a6, a7, a8)
  EMU_FIELDS(10, a0, a1, a2, a3, a4, a5, a6, a7, a8, a9)
  EMU_FIELDS(11, a0, a1, a2, a3, a4, a5, a6, a7, a8, a9, a10)
  EMU_FIELDS(12, a0, a1, a2, a3, a4, a5, a6, a7, a8, a9, a10, a11)
  EMU_FIELDS(13, a0, a1, a2, a3, a4, a5, a6, a7, a8, a9, a10, a11, a12)
  EMU_FIELDS(14, a0, a1, a2, a3, a4, a5, a6, a7, a8, a9, a10, a11, a12, a13)
  EMU_FIELDS(15, a0, a1, a2, a3, a4, a5, a6, a7, a8, a9, a10, a11, a12, a13, a14)
  EMU_FIELDS(16, a0, a1, a2, a3, a4, a5, a6, a7, a8, a9, a10, a11, a12, a13, a14, a15)
}
#undef EMU_FIELDS

template <typename A>
inline void check_arg(const A &a, const char *kname, int argi) {
  if constexpr (std::is_pointer_v<A>) {
    check_ptr(reinterpret_cast<const void *>(a), kname, argi);
  } else if constexpr (std::is_class_v<A>) {
    for_each_field(a, [&](const auto &m) { check_arg(m, kname, argi); });
  }
}

// Launch log: one line per launch (kernel address relative to its object,
// grid, block, dynamic LDS), written when EMU_LAUNCH_LOG names a file.
inline FILE *launch_log() {
  static FILE *f = nullptr;
  static bool init = false;
  if (!init) {
    init = true;
    const char *p = getenv("EMU_LAUNCH_LOG");
    if (p && *p) f = fopen(p, "a");
  }
  return f;
}
}  // namespace emu

inline hipError_t hipMalloc(void *p, size_t n) {
  *reinterpret_cast<void **>(p) = emu::reg_alloc(n, emu::DEVICE);
  return hipSuccess;
}
template <typename T>
inline hipError_t hipMallocAsync(T **p, size_t n, hipStream_t) { return hipMalloc(p, n); }
inline float rsqrtf(float x) { return 1.0f / std::sqrt(x); }
// the bare gfx950 square-root instructions (1 ulp there; correctly rounded here)
#define __builtin_amdgcn_rsqf(x) (1.0f / std::sqrt((float)(x)))
#define __builtin_amdgcn_sqrtf(x) std::sqrt((float)(x))
#define __align__(n) alignas(n)
#define MAG_OPAQUE(x) asm volatile("" : "+m"(x))
#define MAG_WAVES_PER_EU(...)
#define hipHostMallocCoherent 0x40000000u
inline hipError_t hipHostMalloc(void *p, size_t n, unsigned = 0) {
  *reinterpret_cast<void **>(p) = emu::reg_alloc(n, emu::PINNED);
  return hipSuccess;
}
inline hipError_t hipFree(void *p) { return emu::reg_free(p, emu::DEVICE); }
inline hipError_t hipFreeAsync(void *p, hipStream_t) { return emu::reg_free(p, emu::DEVICE); }
inline hipError_t hipHostFree(void *p) { return emu::reg_free(p, emu::PINNED); }

namespace emu {
// Copy with the kind checked against the registry: a device side must be a
// device (or pinned) allocation holding all n bytes, a host side must not be
// device memory.
inline hipError_t checked_copy(void *d, const void *s, size_t n, hipMemcpyKind kind, const char *call) {
  if (capturing) fail("copy during stream capture (%p, %s)", d, call);
  if (n == 0) return hipSuccess;
  uintptr_t db = 0, sb = 0;
  size_t dl = 0, sl = 0;
  const int dk = kind_of(d, &db, &dl), sk = kind_of(s, &sb, &sl);
  auto need_dev = [&](int k, uintptr_t base, size_t len, const void *p, const char *side) {
    if (k != DEVICE && k != PINNED) fail("%p is not device memory (%s)", p, side);
    if (reinterpret_cast<uintptr_t>(p) + n > base + len) fail("copy runs past the end of the allocation at %p (%s)", p, side);
  };
  auto need_host = [&](int k, const void *p, const char *side) {
    if (k == DEVICE) fail("%p is device memory, the copy kind says host (%s)", p, side);
  };
  char w[128];
  switch (kind) {
    case hipMemcpyHostToDevice:
      snprintf(w, sizeof w, "%s H2D destination", call);
      need_dev(dk, db, dl, d, w);
      snprintf(w, sizeof w, "%s H2D source", call);
      need_host(sk, s, w);
      break;
    case hipMemcpyDeviceToHost:
      snprintf(w, sizeof w, "%s D2H source", call);
      need_dev(sk, sb, sl, s, w);
      snprintf(w, sizeof w, "%s D2H destination", call);
      need_host(dk, d, w);
      break;
    case hipMemcpyDeviceToDevice:
      snprintf(w, sizeof w, "%s D2D destination", call);
      need_dev(dk, db, dl, d, w);
      snprintf(w, sizeof w, "%s D2D source", call);
      need_dev(sk, sb, sl, s, w);
      break;
    case hipMemcpyHostToHost:
      snprintf(w, sizeof w, "%s H2H", call);
      need_host(dk, d, w);
      need_host(sk, s, w);
      break;
    default:
      if (dk == DEVICE) need_dev(dk, db, dl, d, call);
      if (sk == DEVICE) need_dev(sk, sb, sl, s, call);
      break;
  }
  if (dk == DEVICE) ASAN_UNPOISON_MEMORY_REGION(d, n);
  if (sk == DEVICE) ASAN_UNPOISON_MEMORY_REGION(const_cast<void *>(s), n);
  std::memmove(d, s, n);
  if (dk == DEVICE) poison_device(true);
  if (sk == DEVICE) poison_device(true);
  return hipSuccess;
}
}  // namespace emu

inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k) {
  return emu::checked_copy(d, s, n, k, "hipMemcpy");
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
  return emu::checked_copy(d, s, n, k, "hipMemcpyAsync");
}
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
  if (n == 0) return hipSuccess;
  uintptr_t b = 0;
  size_t l = 0;
  const int k = emu::kind_of(d, &b, &l);
  if (k != emu::DEVICE && k != emu::PINNED) emu::fail("hipMemsetAsync on %p, which is %s", d, "not device memory");
  if (reinterpret_cast<uintptr_t>(d) + n > b + l) emu::fail("hipMemsetAsync at %p runs past %s", d, "the end of its allocation");
  if (k == emu::DEVICE) ASAN_UNPOISON_MEMORY_REGION(d, n);
  std::memset(d, v, n);
  if (k == emu::DEVICE) emu::poison_device(true);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) {
  if (emu::capturing) emu::fail("hipStreamSynchronize during stream capture (%p, %s)", nullptr, "not capturable");
  return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  static int dummy[64];
  static int k = 0;
  *s = &dummy[(k++) & 63];
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
  *e = nullptr;
  return hipSuccess;
}
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, int) {
  if (emu::capturing) emu::fail("nested stream capture (%p, %s)", nullptr, "hipStreamBeginCapture");
  emu::capturing = true;
  emu::cap_graph = new emu::Graph();
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
  emu::capturing = false;
  *g = emu::cap_graph;
  emu::cap_graph = nullptr;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, void *, size_t) {
  *x = new emu::Graph(*g);
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
  for (auto &op : x->ops) op();
  return hipSuccess;
}
inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
// A `__device__` array is a host static here: its address is registered as
// device memory (poisoned for host code) the first time it is looked up.
#define HIP_SYMBOL(x) (x)
template <typename T>
inline hipError_t hipGetSymbolAddress(void **p, T &sym) {
  uintptr_t b = 0;
  size_t l = 0;
  if (emu::kind_of(&sym, &b, &l) != emu::DEVICE) {
    emu::reg()[reinterpret_cast<uintptr_t>(&sym)] = emu::Alloc{sizeof(T), emu::DEVICE};
    ASAN_POISON_MEMORY_REGION(&sym, sizeof(T));
  }
  *p = &sym;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "emu"; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = nullptr; return 1; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0; return hipSuccess; }

namespace emu {
// Persistent work-item threads, reused by every launch (a fresh thread per
// work-item would exhaust the sanitizer's thread registry on long runs).
// run(n, f) executes f(0..n-1) on the first n workers and waits for them.
struct Pool {
  std::vector<std::thread> th;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::function<void(unsigned)> job;
  unsigned njob = 0, remaining = 0;
  unsigned long long gen = 0;
  bool stop = false;
  void worker(unsigned i) {
    unsigned long long seen = 0;
    for (;;) {
      std::function<void(unsigned)> f;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || gen != seen; });
        if (stop) return;
        seen = gen;
        if (i >= njob) continue;
        f = job;
      }
      f(i);
      std::lock_guard<std::mutex> lk(mu);
      if (--remaining == 0) done_cv.notify_all();
    }
  }
  void run(unsigned n, std::function<void(unsigned)> f) {
    while (th.size() < n) {
      const unsigned i = (unsigned)th.size();
      th.emplace_back([this, i] { worker(i); });
    }
    std::unique_lock<std::mutex> lk(mu);
    job = std::move(f);
    njob = n;
    remaining = n;
    ++gen;
    cv.notify_all();
    done_cv.wait(lk, [&] { return remaining == 0; });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto &t : th) t.join();
  }
};
inline Pool &pool() {
  static Pool p;
  return p;
}
}  // namespace emu

template <typename... KA, typename... A>
void emu_launch(void (*k)(KA...), dim3 g, dim3 b, size_t shm, A... args) {
  const unsigned nt = b.x * b.y * b.z;
  Dl_info di{};
  dladdr(reinterpret_cast<void *>(k), &di);
  const uintptr_t off = reinterpret_cast<uintptr_t>(k) - reinterpret_cast<uintptr_t>(di.dli_fbase);
  char kname[64];
  snprintf(kname, sizeof kname, "kernel at +0x%lx", (unsigned long)off);
  if (nt == 0 || nt > 1024 || g.x == 0 || g.y == 0 || g.z == 0 || g.y > 65535 || g.z > 65535 ||
      (unsigned long long)g.x * b.x >= (1ull << 32))
    emu::fail("launch shape out of the hardware limits (%p, %s)", reinterpret_cast<void *>(k), kname);
  if (FILE *f = emu::launch_log()) {
    fprintf(f, "%lx %u %u %u %u %u %u %zu\n", (unsigned long)off, g.x, g.y, g.z, b.x, b.y, b.z, shm);
    fflush(f);
  }
  // kernel arguments converted to the kernel's parameter types, then checked
  std::tuple<std::decay_t<KA>...> conv(args...);
  {
    int i = 0;
    std::apply([&](const auto &...x) { (emu::check_arg(x, kname, i++), ...); }, conv);
  }
  auto run = [=]() mutable {
  emu::poison_device(false);
  emu::bDim = b;
  emu::gDim = g;
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
        emu::pool().run(nt, [&](unsigned t) {
          emu::tIdx = dim3(t % b.x, (t / b.x) % b.y, t / (b.x * b.y));
          emu::bIdx = dim3(bx, by, bz);
          std::apply(k, conv);
          br.arrive_and_drop();
        });
        std::free(d);
      }
  emu::poison_device(true);
  };
  if (emu::capturing) emu::cap_graph->ops.push_back(run);
  else run();
}
#define hipLaunchKernelGGL(K, G, B, S, STREAM, ...) emu_launch(K, dim3(G), dim3(B), (size_t)(S), __VA_ARGS__)

// Entry points for the test driver: device buffers and copies in the
// emulated device address space.
extern "C" {
inline __attribute__((visibility("default"), used)) void *emu_dev_alloc(size_t n) {
  void *p = nullptr;
  hipMalloc(&p, n);
  return p;
}
inline __attribute__((visibility("default"), used)) void emu_dev_free(void *p) { hipFree(p); }
inline __attribute__((visibility("default"), used)) void emu_h2d(void *d, const void *s, size_t n) {
  hipMemcpy(d, s, n, hipMemcpyHostToDevice);
}
inline __attribute__((visibility("default"), used)) void emu_d2h(void *d, const void *s, size_t n) {
  hipMemcpy(d, s, n, hipMemcpyDeviceToHost);
}
}
