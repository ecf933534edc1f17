// Device building blocks of the pencil FFTs (gfx950, wave64).
//
// A pencil of length N (a power of two, 8..4096, or three times a power of
// two, 12..768, whose first stage is a radix-12 DFT) is spread over TT = N / RMAX
// threads; thread j holds the RMAX values x[j + rho * TT] in registers.  The
// transform is a mixed-radix Stockham decimation-in-time: stage s combines
// sub-transforms of length Ns (product of the earlier radices) with radix R_s.
// Between stages the data goes through LDS; the first stage reads the
// register pattern above straight from global memory and the last stage
// leaves X[j + rho * TT] in registers, so a two-stage pencil costs one LDS
// exchange.  In-register DFTs of size 2..16 are unrolled radix-2 butterflies
// with compile-time twiddles, size 12 a prime-factor (3 x 4) composition
// without internal twiddles; inter-stage twiddles come from a table of
// exp(-2 pi i m / N) built on the host in double precision.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace mag {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------- compile-time loops
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int i, int n) {
  int r = 0;
  for (int b = 1; b < n; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// cos and sin of 2 pi m / 16
constexpr double kC1 = 0.92387953251128674;   // cos(pi/8)
constexpr double kC2 = 0.70710678118654752;   // cos(pi/4)
constexpr double kC3 = 0.38268343236508978;   // cos(3pi/8)
constexpr double kCos16[16] = {1, kC1, kC2, kC3, 0, -kC3, -kC2, -kC1, -1, -kC1, -kC2, -kC3, 0, kC3, kC2, kC1};
constexpr double kSin16[16] = {0, kC3, kC2, kC1, 1, kC1, kC2, kC3, 0, -kC3, -kC2, -kC1, -1, -kC1, -kC2, -kC3};

// a * exp(DIR * 2 pi i M / R), M a compile-time integer; DIR = -1 forward, +1 inverse.
template <int R, int DIR, int M, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (2 * m == R) {
    return {-a.x, -a.y};
  } else if constexpr (4 * m == R) {
    if constexpr (DIR < 0) return {a.y, -a.x};   // * (-i)
    else return {-a.y, a.x};                     // * (+i)
  } else if constexpr (4 * m == 3 * R) {
    if constexpr (DIR < 0) return {-a.y, a.x};
    else return {a.y, -a.x};
  } else {
    constexpr double c = kCos16[m * (16 / R)];
    constexpr double s = DIR * kSin16[m * (16 / R)];
    const T wr = (T)c, wi = (T)s;
    return {a.x * wr - a.y * wi, a.x * wi + a.y * wr};
  }
}

// In-register DFT of size 3, natural order: A_k = sum_n a_n w^(nk) with
// w = exp(DIR 2 pi i / 3) = -1/2 + DIR i sin(2 pi / 3).
template <int DIR, typename T>
__device__ __forceinline__ void dft3(cx<T>& a0, cx<T>& a1, cx<T>& a2) {
  const T h = (T)(DIR * 0.86602540378443865);   // DIR sin(2 pi / 3)
  const cx<T> t = a1 + a2, d = a1 - a2;
  const cx<T> m = {a0.x - (T)0.5 * t.x, a0.y - (T)0.5 * t.y};
  const cx<T> id = {-h * d.y, h * d.x};          // DIR i sin(2 pi / 3) (a1 - a2)
  a0 = a0 + t;
  a1 = m + id;
  a2 = m - id;
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v);

// In-register DFT of size 12 by the prime-factor (Good-Thomas) map 12 = 3 x 4:
// input index n = (4 n1 + 3 n2) mod 12, output index k = (4 k1 + 9 k2) mod 12,
// so that nk = 4 n1 k1 + 3 n2 k2 (mod 12): three-point DFTs over n1 for each
// n2, then four-point DFTs over n2 for each k1, with no twiddles between.
template <int DIR, typename T>
__device__ __forceinline__ void dft12(cx<T>* v) {
  cx<T> y[3][4];
  static_for<0, 4>([&](auto n2I) {
    constexpr int n2 = decltype(n2I)::value;
    cx<T> a0 = v[(3 * n2) % 12], a1 = v[(4 + 3 * n2) % 12], a2 = v[(8 + 3 * n2) % 12];
    dft3<DIR, T>(a0, a1, a2);
    y[0][n2] = a0;
    y[1][n2] = a1;
    y[2][n2] = a2;
  });
  static_for<0, 3>([&](auto k1I) {
    constexpr int k1 = decltype(k1I)::value;
    dft<4, DIR, T>(y[k1]);
    static_for<0, 4>([&](auto k2I) {
      constexpr int k2 = decltype(k2I)::value;
      v[(4 * k1 + 9 * k2) % 12] = y[k1][k2];
    });
  });
}

// In-register DFT of size R (2, 4, 8, 16 or 12), natural order in and out.
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 12) {
    dft12<DIR, T>(v);
  } else {
    static_for<0, ilog2(R)>([&](auto st) {
      constexpr int span = R >> (decltype(st)::value + 1);
      static_for<0, R / (2 * span)>([&](auto bi) {
        constexpr int base = decltype(bi)::value * 2 * span;
        static_for<0, span>([&](auto kk) {
          constexpr int k = decltype(kk)::value;
          const cx<T> a = v[base + k], b = v[base + k + span];
          v[base + k] = a + b;
          v[base + k + span] = rot<R, DIR, k*(R / (2 * span))>(a - b);
        });
      });
    });
    static_for<0, R>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      constexpr int j = bitrev(i, R);
      if constexpr (j > i) {
        const cx<T> t = v[i];
        v[i] = v[j];
        v[j] = t;
      }
    });
  }
}

// ---------------------------------------------------------------- plans
// A plan lists the radices of the stages (at most 4); RMAX is the largest and
// sets how many values each thread holds.  Plan<N> favours radix 16 (fewest
// LDS exchanges); Plan8<N> caps the radix at 8 (fewer registers per thread,
// more threads per pencil).
template <int N>
struct Plan;
template <int N>
struct Plan8;
#define MAG_PLAN(NAME, N_, S_, RMAX_, R0, R1, R2, R3)         \
  template <>                                                \
  struct NAME<N_> {                                          \
    static constexpr int S = S_, RMAX = RMAX_;               \
    static constexpr int R[4] = {R0, R1, R2, R3};            \
    static constexpr int TT = N_ / RMAX_;                    \
  };
MAG_PLAN(Plan, 8, 1, 8, 8, 1, 1, 1)
MAG_PLAN(Plan, 16, 1, 16, 16, 1, 1, 1)
MAG_PLAN(Plan, 32, 2, 8, 8, 4, 1, 1)
MAG_PLAN(Plan, 64, 2, 8, 8, 8, 1, 1)
MAG_PLAN(Plan, 128, 2, 16, 16, 8, 1, 1)
MAG_PLAN(Plan, 256, 2, 16, 16, 16, 1, 1)
MAG_PLAN(Plan, 512, 3, 8, 8, 8, 8, 1)
MAG_PLAN(Plan, 1024, 3, 16, 16, 16, 4, 1)
MAG_PLAN(Plan, 2048, 3, 16, 16, 16, 8, 1)
MAG_PLAN(Plan, 4096, 3, 16, 16, 16, 16, 1)
MAG_PLAN(Plan8, 8, 1, 8, 8, 1, 1, 1)
MAG_PLAN(Plan8, 16, 2, 8, 8, 2, 1, 1)
MAG_PLAN(Plan8, 32, 2, 8, 8, 4, 1, 1)
MAG_PLAN(Plan8, 64, 2, 8, 8, 8, 1, 1)
MAG_PLAN(Plan8, 128, 3, 8, 8, 8, 2, 1)
MAG_PLAN(Plan8, 256, 3, 8, 8, 8, 4, 1)
MAG_PLAN(Plan8, 512, 3, 8, 8, 8, 8, 1)
MAG_PLAN(Plan8, 1024, 4, 8, 8, 8, 8, 2)
MAG_PLAN(Plan8, 2048, 4, 8, 8, 8, 8, 4)
MAG_PLAN(Plan8, 4096, 4, 8, 8, 8, 8, 8)
// three times a power of two: a radix-12 first stage, twelve values per thread
MAG_PLAN(Plan8, 12, 1, 12, 12, 1, 1, 1)
MAG_PLAN(Plan8, 24, 2, 12, 12, 2, 1, 1)
MAG_PLAN(Plan8, 48, 2, 12, 12, 4, 1, 1)
MAG_PLAN(Plan8, 96, 3, 12, 12, 4, 2, 1)
MAG_PLAN(Plan8, 192, 3, 12, 12, 4, 4, 1)
MAG_PLAN(Plan8, 384, 4, 12, 12, 4, 4, 2)
MAG_PLAN(Plan8, 768, 4, 12, 12, 4, 4, 4)
#undef MAG_PLAN

// b mod n for b >= 0 (a mask when n is a power of two)
template <int n>
__device__ __forceinline__ int mod_len(int b) {
  if constexpr ((n & (n - 1)) == 0) return b & (n - 1);
  else return (int)((unsigned)b % (unsigned)n);
}

template <typename PL, int s>
constexpr int plan_ns() {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= PL::R[i];
  return ns;
}

// Work-group barrier for the LDS exchanges of the transforms: its fences are
// limited to the local address space, so the wave's outstanding global loads
// and stores need not complete first (a plain __syncthreads waits for every
// outstanding vector-memory operation, which would serialise a transform
// with the loads issued for the next one).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One pencil transform.  v[RMAX] holds x[j + rho*TT] on entry and X[j + rho*TT]
// on exit.  lre/lim: this pencil's LDS scratch (real and imaginary planes),
// element i at offset lidx(i).  tw: exp(-2 pi i m / N), m = 0..N-1.
// Every thread of the block must call this (it contains barriers).
template <int N, int DIR, typename P = Plan<N>, typename T, typename LIdx>
__device__ __forceinline__ void pencil_fft(cx<T>* v, int j, T* lre, T* lim, LIdx lidx,
                                           const cx<T>* __restrict__ tw) {
  constexpr int RMAX = P::RMAX, TT = P::TT, S = P::S;
  if constexpr (S > 1) lds_barrier();   // LDS may still be read by a previous use
  static_for<0, S>([&](auto sI) {
    constexpr int s = decltype(sI)::value;
    constexpr int R = P::R[s];
    constexpr int U = RMAX / R;
    constexpr int Ns = plan_ns<P, s>();
    if constexpr (s > 0) {
      lds_barrier();
#pragma unroll
      for (int rho = 0; rho < RMAX; ++rho) {
        const int o = lidx(j + rho * TT);
        v[rho] = {lre[o], lim[o]};
      }
      if constexpr (s < S - 1) lds_barrier();
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = j + u * TT;
      const int k = mod_len<Ns>(b);
      cx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[u + r * U];
      if constexpr (s > 0) {
        constexpr int tstep = N / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w = tw[r * k * tstep];
          a[r] = (DIR < 0) ? cmul(a[r], w) : cmulc(a[r], w);
        }
      }
      dft<R, DIR, T>(a);
      if constexpr (s < S - 1) {
        const int base = (b / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int o = lidx(base + r * Ns);
          lre[o] = a[r].x;
          lim[o] = a[r].y;
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u + r * U] = a[r];
      }
    }
  });
}

// Powers w^r, r = 1..R-1, of one twiddle w by products of lower powers
// (w^r = w^h w^(r-h), h the largest power of two below r): at most
// log2(R) multiplications deep, so the rounding error stays a few ulp.
template <int R, typename T>
__device__ __forceinline__ void twiddle_powers(cx<T> w, cx<T>* wp) {
  wp[1] = w;
  static_for<2, R>([&](auto rI) {
    constexpr int r = decltype(rI)::value;
    constexpr int h = 1 << (ilog2(r) - ((r & (r - 1)) == 0 ? 1 : 0));
    wp[r] = cmul(wp[h], wp[r - h]);
  });
}

// Offset of stage s's twiddles in a thread's preloaded set (stages 1..S-1,
// RMAX / R[s] entries each).
template <typename PL>
constexpr int plan_twoff(int s) {
  int o = 0;
  for (int i = 1; i < s; ++i) o += PL::RMAX / PL::R[i];
  return o;
}

// The inter-stage twiddle entries one thread of a pencil transform reads,
// loaded once into registers (they depend only on the thread's index j, and
// the inverse transform uses the same entries conjugated).  Issuing these
// loads with the data loads takes the table reads off the critical path
// between LDS exchanges.  LOCAL = true makes each entry opaque where a stage
// uses it, so that its powers are formed inside that stage (fewer live
// registers) instead of once for every stage and transform of the kernel.
template <typename PL, typename T, bool LOCAL = false>
struct TwPre {
  static constexpr int NW = plan_twoff<PL>(PL::S) > 0 ? plan_twoff<PL>(PL::S) : 1;
  cx<T> w[NW];
};

template <int N, typename PL, typename T, bool LOCAL>
__device__ __forceinline__ void tw_preload(TwPre<PL, T, LOCAL>& t, int j, const cx<T>* __restrict__ tw) {
  constexpr int RMAX = PL::RMAX, TT = PL::TT, S = PL::S;
  static_for<1, S>([&](auto sI) {
    constexpr int s = decltype(sI)::value;
    constexpr int R = PL::R[s];
    constexpr int U = RMAX / R;
    constexpr int Ns = plan_ns<PL, s>();
    constexpr int tstep = N / (Ns * R);
#pragma unroll
    for (int u = 0; u < U; ++u) t.w[plan_twoff<PL>(s) + u] = tw[mod_len<Ns>(j + u * TT) * tstep];
  });
}

template <typename PL, int s, typename T>
__device__ __forceinline__ cx<T> tw_get(const cx<T>* __restrict__ tw, int u, int idx) {
  (void)u;
  return tw[idx];
}
// Value barrier: the compiler must assume x changed here (no code is emitted).
#ifndef MAG_OPAQUE
#define MAG_OPAQUE(x) asm volatile("" : "+v"(x))
#endif

template <typename PL, int s, typename T, bool LOCAL>
__device__ __forceinline__ cx<T> tw_get(const TwPre<PL, T, LOCAL>& t, int u, int idx) {
  (void)idx;
  cx<T> w = t.w[plan_twoff<PL>(s) + u];
  if constexpr (LOCAL) {
    MAG_OPAQUE(w.x);
    MAG_OPAQUE(w.y);
  }
  return w;
}

// Same transform as pencil_fft, with the LDS exchange holding interleaved
// complex values (one access per element) and the inter-stage twiddles of a
// thread formed from a single table entry per stage (twiddle_powers).
// tw: the table itself or a TwPre set loaded by tw_preload for this j.
template <int N, int DIR, typename P = Plan<N>, typename T, typename LIdx, typename TW>
__device__ __forceinline__ void pencil_fft_cx(cx<T>* v, int j, cx<T>* lds, LIdx lidx, const TW& tw) {
  constexpr int RMAX = P::RMAX, TT = P::TT, S = P::S;
  if constexpr (S > 1) lds_barrier();   // LDS may still be read by a previous use
  static_for<0, S>([&](auto sI) {
    constexpr int s = decltype(sI)::value;
    constexpr int R = P::R[s];
    constexpr int U = RMAX / R;
    constexpr int Ns = plan_ns<P, s>();
    if constexpr (s > 0) {
      lds_barrier();
#pragma unroll
      for (int rho = 0; rho < RMAX; ++rho) v[rho] = lds[lidx(j + rho * TT)];
      if constexpr (s < S - 1) lds_barrier();
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = j + u * TT;
      const int k = mod_len<Ns>(b);
      cx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[u + r * U];
      if constexpr (s > 0) {
        constexpr int tstep = N / (Ns * R);
        cx<T> wp[R];
        twiddle_powers<R, T>(tw_get<P, s, T>(tw, u, k * tstep), wp);
#pragma unroll
        for (int r = 1; r < R; ++r) a[r] = (DIR < 0) ? cmul(a[r], wp[r]) : cmulc(a[r], wp[r]);
      }
      dft<R, DIR, T>(a);
      if constexpr (s < S - 1) {
        const int base = (b / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lidx(base + r * Ns)] = a[r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u + r * U] = a[r];
      }
    }
  });
}

}  // namespace mag
