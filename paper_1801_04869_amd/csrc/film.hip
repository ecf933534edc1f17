// Thin-film (2D) right-hand side: eq. (9) in the film on a staggered
// node/edge grid and the free-space iteration (10)-(12) of Prigozhin &
// Sokolovsky, Sec. 2.
//
// Layouts (x fastest): g, dh/dt, G on nodes [ny][nx]; half spectrum stored
// transposed, [kx][ny] with kx = nx/2 + 1, so that every pass reads and
// writes contiguous runs.  A right-hand side is
//   stencil       e = rho(|j|) j on the edges, dh/dt = -curl e on inside
//                 nodes (eq. (9)), and the shift A^0 of the first iterate
//   rows_fwd(H)   R2C of H - dh_e, sums of w1 (H - dh_e)
// then per inner iteration four passes (film_iteration below): the column
// pass with 2/|k|, a fused row pass (C2R G, gdot = G - C with C from the w1
// sums, R2C of gdot on free space), the column pass with |k|/2 (after the
// stop decision on the |gdot| sums), and a fused row pass (update (12) of H on
// free space, R2C of H - dh_e for the next iteration).  w1 = K1 1_out and
// w2 = K2 1_out turn the free-space means of (10) and (11) into dot products
// accumulated inside the row passes.  On exit gdot = G - C is written to the
// output in double precision.
#include <cmath>

#include "ctx.h"
#include "kern_common.h"

namespace mag {

namespace {

// Periodic index for -n <= i < 2n (grid lengths are powers of two or three
// times a power of two); P2: n is a power of two (a mask).
template <bool P2 = false>
__device__ __forceinline__ int wrap(int i, int n) {
  if constexpr (P2) return i & (n - 1);
  i = i < 0 ? i + n : i;
  return i >= n ? i - n : i;
}

// LDS exchange slot of complex element i of a pencil: one padding element
// after every 128 bytes (16 FP32 or 8 FP64 complex values); the pencil's
// pitch in elements.
template <typename T>
__device__ __forceinline__ int lds_pad(int i) {
  return sizeof(T) == 4 ? i + (i >> 4) : i + (i >> 3);
}
template <typename T>
constexpr int lds_pitch(int n) {
  return sizeof(T) == 4 ? n + n / 16 : n + n / 8;
}
// Square roots of the Fourier multipliers: in float the bare hardware
// instructions (within 1 ulp for the normal, positive |k|^2 they take),
// in double the correctly rounded library functions.
__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float mult_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double mult_sqrt(double x) { return sqrt(x); }

struct FilmGeom {
  int nx, ny, kx;
  double idx, idy;
};

template <typename T>
__device__ __forceinline__ T film_rho(T s, T jc, T e0, T nm1, T lmax) {
  if (!(s > (T)0)) return (T)0;
  T lg = log(s / jc);
  if constexpr (sizeof(T) == 4) lg = fminf(lg, lmax);
  return (e0 / jc) * exp(nm1 * lg);
}

struct FilmLaw {
  double e0, nm1, rho_out, lmax, jc0;
  int has_jc;
};

// e on the x-edge (p, q+1/2) or the y-edge (p+1/2, q) (orient 0 / 1);
// P2: nx and ny are powers of two.
template <typename T, bool P2>
__device__ __forceinline__ T film_edge_e(const double *__restrict__ g, const uint8_t *__restrict__ mat,
                                         const T *__restrict__ jc, const FilmGeom &G, const FilmLaw &law,
                                         int p, int q, int orient) {
  const int nx = G.nx, ny = G.ny;
  auto gv = [&](int pp, int qq) { return g[(long long)wrap<P2>(qq, ny) * nx + wrap<P2>(pp, nx)]; };
  auto jxv = [&](int pp, int qq) { return (gv(pp, qq + 1) - gv(pp, qq)) * G.idy; };
  auto jyv = [&](int pp, int qq) { return -(gv(pp + 1, qq) - gv(pp, qq)) * G.idx; };
  double jo, oth;
  long long c0 = (long long)wrap<P2>(q, ny) * nx + wrap<P2>(p, nx), c1;
  if (orient == 0) {
    jo = jxv(p, q);
    oth = 0.25 * (jyv(p - 1, q) + jyv(p, q) + jyv(p - 1, q + 1) + jyv(p, q + 1));
    c1 = (long long)wrap<P2>(q, ny) * nx + wrap<P2>(p - 1, nx);
  } else {
    jo = jyv(p, q);
    oth = 0.25 * (jxv(p, q - 1) + jxv(p, q) + jxv(p + 1, q - 1) + jxv(p + 1, q));
    c1 = (long long)wrap<P2>(q - 1, ny) * nx + wrap<P2>(p, nx);
  }
  const uint8_t m0 = mat[c0], m1 = mat[c1];
  if (m0 == 1 && m1 == 1) {
    const T jt = (T)jo, ot = (T)oth;
    const T s = sqrt(jt * jt + ot * ot);
    const T jce = law.has_jc ? (T)0.5 * (jc[c0] + jc[c1]) : (T)law.jc0;
    return film_rho(s, jce, (T)law.e0, (T)law.nm1, (T)law.lmax) * jt;
  }
  return (T)law.rho_out * (T)jo;
}

// dh_z/dt = -(d_x e_y - d_y e_x) at inside nodes (eq. (9)); free-space nodes
// keep the warm start (or take dh_e/dt).  Each thread handles kStencilNpt
// nodes kStencilThreads apart; one partial sum of H - dh_e over D per block
// (few enough blocks that every block of the next pass can add the partials
// itself: 1024 at 2048^2).  Four nodes per thread rather than eight put twice
// as many waves on the film's rows, whose nodes each gather their
// neighbourhood in a chain of dependent loads (21.8 -> 20.3 us at 2048^2).
constexpr int kStencilNpt = 4;
constexpr int kStencilThreads = 1024;

// FP32: two blocks of 16 waves per CU need at most 64 registers per lane
// (the general periodic wrap of grids of 3 * 2^k nodes needs more: one block).
// SPECTRAL: the film values of H have been written by the spectral passes
// and are only read here; the free space and the partial sums are the same.
template <typename T, bool SPECTRAL, bool P2>
__global__ void __launch_bounds__(kStencilThreads) MAG_WAVES_PER_EU(sizeof(T) == 4 && (P2 || SPECTRAL) ? 8 : 4) film_stencil(const double *__restrict__ g, const uint8_t *__restrict__ mat,
                                                    const uint8_t *__restrict__ flags, const T *__restrict__ jc,
                                                    T *__restrict__ H, FilmGeom G, FilmLaw law,
                                                    const IterState *__restrict__ it, int warm,
                                                    double *__restrict__ part) {
  __shared__ double red[kStencilThreads / 64];
  // a step that has already reached its end time launches nothing useful
  if (it->done) return;
  const double hde = it->hde;
  // after a failed attempt the free space restarts from dh_e/dt
  warm = warm && !it->cold;
  const long long n = (long long)G.nx * G.ny;
  const long long i0 = (long long)blockIdx.x * (kStencilThreads * kStencilNpt) + threadIdx.x;
  double acc = 0.0;
  // the flags (and warm starts) of all of this thread's nodes first, in one
  // batch: free-space nodes then need no further load
  uint8_t fl[kStencilNpt];
  T hw[kStencilNpt];
#pragma unroll
  for (int k = 0; k < kStencilNpt; ++k) {
    const long long i = i0 + (long long)k * kStencilThreads;
    const long long ic = i < n ? i : 0;
    fl[k] = flags[ic];
    hw[k] = (warm || SPECTRAL) ? H[ic] : (T)0;
  }
#pragma unroll 1
  for (int k = 0; k < kStencilNpt; ++k) {
    const long long i = i0 + (long long)k * kStencilThreads;
    if (i >= n) break;
    const int p = (int)(i % G.nx), q = (int)(i / G.nx);
    T h;
    if (SPECTRAL && (fl[k] & 1)) {
      h = hw[k];
    } else if (fl[k] & 1) {
      const T exq = film_edge_e<T, P2>(g, mat, jc, G, law, p, q, 0);
      const T exm = film_edge_e<T, P2>(g, mat, jc, G, law, p, q - 1, 0);
      const T eyp = film_edge_e<T, P2>(g, mat, jc, G, law, p, q, 1);
      const T eym = film_edge_e<T, P2>(g, mat, jc, G, law, p - 1, q, 1);
      const double curl = ((double)eyp - (double)eym) * G.idx - ((double)exq - (double)exm) * G.idy;
      h = (T)(-curl);
      H[i] = h;
    } else if (warm) {
      h = hw[k];
    } else {
      h = (T)hde;
      H[i] = h;
    }
    acc += (double)h - hde;
  }
  const double s = block_total<kStencilThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Launch shape of the row transforms.  The half spectrum is stored
// transposed, [kx][ny] (y fastest), so that the column pass reads contiguous
// columns; a row block of P rows therefore writes (reads) P consecutive
// complex values per wavenumber k, P chosen so that this run is at least 32
// bytes.  Consecutive row blocks are placed on the same XCD (see
// xcd_block) so that the runs of neighbouring blocks meet in one L2.  The block's LDS holds either the FFT exchange of its P rows (pitch
// lds_pitch<T>(M)) or the transposed [M+1][P+1] tile of its output, one after the
// other.
template <int M, typename T>
struct FilmRowShape {
  using PL = Plan8<M>;
  static constexpr int TT = PL::TT;
  static constexpr int PITCH = lds_pitch<T>(M);
  static constexpr int PMIN = 32 / (2 * (int)sizeof(T));
  static constexpr int PT = 256 / TT > 0 ? 256 / TT : 1;
  static constexpr int P = PT > PMIN ? PT : PMIN;
  static constexpr int SP = P + 1;                    // tile pitch (complex entries per k)
  static constexpr int XCH = 2 * P * PITCH;           // T entries of the FFT exchange
  static constexpr int STG = 2 * (M + 1) * SP;        // T entries of the tile
  static constexpr int LDS_T = XCH > STG ? XCH : STG;
  static constexpr int THREADS = P * TT;
  // Waves per SIMD that a square grid (ny = 2M rows) needs resident for its
  // row blocks to run in the fewest rounds on 256 CUs that LDS (160 KB per
  // CU) allows, spread evenly over those rounds: the register budget handed
  // to the compiler.
  static constexpr int TW_BYTES = sizeof(T) == 4 ? 2 * M * 2 * (int)sizeof(T) : 0;   // see row_twiddles
  static constexpr int BLOCKS_LDS_RAW = (160 * 1024) / (LDS_T * (int)sizeof(T) + TW_BYTES + 1024);
  static constexpr int BLOCKS_LDS = BLOCKS_LDS_RAW < 1 ? 1 : BLOCKS_LDS_RAW;
  static constexpr int BLOCKS_SQ = ((2 * M + P - 1) / P + 255) / 256;
  static constexpr int ROUNDS = (BLOCKS_SQ + BLOCKS_LDS - 1) / BLOCKS_LDS;
  static constexpr int BLOCKS_CU = (BLOCKS_SQ + ROUNDS - 1) / ROUNDS;
  static constexpr int WAVES_EU_RAW = BLOCKS_CU * ((THREADS + 63) / 64) / 4;
  static constexpr int WAVES_EU = WAVES_EU_RAW < 1 ? 1 : (WAVES_EU_RAW > 8 ? 8 : WAVES_EU_RAW);
  static_assert(THREADS <= 1024, "row block too large");
  static_assert(LDS_T * sizeof(T) <= 150 * 1024, "row block LDS too large");
};

// Partial sums passed between the passes of one iteration: `in` (nin values)
// are summed by every block that needs the total (fixed order, so all agree),
// `out` / `out2` receive one value per logical row block.  `iter` is the index
// of the current evaluation of (11) for the stop decision in the column pass.
struct Parts {
  const double *in;
  int nin;
  double *out;
  double *out2;
  int iter;
};

// Work-groups are dealt to the 8 XCDs round-robin (hardware block i runs on
// XCD i % 8).  Map them so that XCD x processes the contiguous logical range
// [x nblk/8, (x+1) nblk/8) when nblk is a multiple of 8.
__device__ __forceinline__ int xcd_block(int i, int nblk) {
  if (nblk & 7) return i;
  return (i & 7) * (nblk >> 3) + (i >> 3);
}

// Launch shape of the column pass: P contiguous columns of length NY per block,
// radix at most 8 (8 values per thread keeps the register count low enough
// for several blocks per compute unit).
template <int NY, typename T>
struct FilmColShape {
  using PL = Plan8<NY>;
  static constexpr int TT = PL::TT;
  static constexpr int P = 256 / TT > 0 ? 256 / TT : 1;
  static constexpr int PITCH = lds_pitch<T>(NY);
  static constexpr int LDS_T = 2 * P * PITCH;
  static constexpr int THREADS = P * TT;
  static_assert(LDS_T * sizeof(T) <= 150 * 1024, "column block LDS too large");
};

// Tile traffic of a row pass: entries (k, r), k = 0..M, r = 0..P-1, of the
// transposed spectrum S[k][q0 + r].  tile_fetch issues all of a work-item's
// loads into registers at once (one round trip to memory, not one per loop
// trip); tile_put stores them to the LDS tile [M+1][SP]; tile_store writes
// the tile back.  Rows past ny read entry 0 and are dropped.
template <typename T, int M, int P, int THREADS>
struct TileRegs {
  static constexpr int NE = (M + 1) * P, NU = (NE + THREADS - 1) / THREADS;
  cx<T> t[NU];
};

template <typename T, int M, int P, int THREADS>
__device__ __forceinline__ void tile_fetch(TileRegs<T, M, P, THREADS> &tr, const cx<T> *__restrict__ S, int ny,
                                           int q0) {
  using TR = TileRegs<T, M, P, THREADS>;
#pragma unroll
  for (int u = 0; u < TR::NU; ++u) {
    const int idx = threadIdx.x + u * THREADS;
    const int k = idx / P, r = idx % P;
    const bool ok = idx < TR::NE && q0 + r < ny;
    const cx<T> v = S[ok ? (long long)k * ny + q0 + r : 0];
    tr.t[u] = ok ? v : cx<T>{(T)0, (T)0};
  }
}

template <typename T, int M, int P, int SP, int THREADS>
__device__ __forceinline__ void tile_put(cx<T> *tile, const TileRegs<T, M, P, THREADS> &tr) {
  using TR = TileRegs<T, M, P, THREADS>;
#pragma unroll
  for (int u = 0; u < TR::NU; ++u) {
    const int idx = threadIdx.x + u * THREADS;
    if (idx < TR::NE) tile[(idx / P) * SP + idx % P] = tr.t[u];
  }
}

template <typename T, int M, int P, int SP, int THREADS>
__device__ __forceinline__ void tile_store(const cx<T> *tile, cx<T> *__restrict__ S, int ny, int q0) {
  constexpr int NE = (M + 1) * P, NU = (NE + THREADS - 1) / THREADS;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int idx = threadIdx.x + u * THREADS;
    const int k = idx / P, r = idx % P;
    if (idx < NE && q0 + r < ny) S[(long long)k * ny + q0 + r] = tile[k * SP + r];
  }
}

// FP32 row passes read the twiddle tables of the row transform (length M
// and the real-to-complex step) from LDS: the block fetches them with its
// other loads (row_tw_fetch), stores them (row_tw_put, which points twM and
// twN at the copies) and every first use follows a barrier.  FP64 reads them
// from memory (their LDS would cost a resident block per CU).
template <typename T, int M, int THREADS>
struct RowTw {
  static constexpr bool ON = sizeof(T) == 4;
  static constexpr int NU = (M + THREADS - 1) / THREADS;
  cx<T> m[ON ? NU : 1], n[ON ? NU : 1];
};

template <typename T, int M, int THREADS>
__device__ __forceinline__ void row_tw_fetch(RowTw<T, M, THREADS> &rt, const cx<T> *__restrict__ twM,
                                             const cx<T> *__restrict__ twN) {
  using RT = RowTw<T, M, THREADS>;
  if constexpr (RT::ON) {
#pragma unroll
    for (int u = 0; u < RT::NU; ++u) {
      const int i = threadIdx.x + u * THREADS;
      if (i < M) {
        rt.m[u] = twM[i];
        rt.n[u] = twN[i];
      }
    }
  }
}

template <typename T, int M, int THREADS>
__device__ __forceinline__ void row_tw_put(const RowTw<T, M, THREADS> &rt, const cx<T> *__restrict__ &twM,
                                           const cx<T> *__restrict__ &twN) {
  using RT = RowTw<T, M, THREADS>;
  if constexpr (RT::ON) {
    __shared__ __align__(16) cx<T> lm[M], ln[M];
#pragma unroll
    for (int u = 0; u < RT::NU; ++u) {
      const int i = threadIdx.x + u * THREADS;
      if (i < M) {
        lm[i] = rt.m[u];
        ln[i] = rt.n[u];
      }
    }
    twM = lm;
    twN = ln;
  }
}

// Row transforms (real-to-complex along x, output transposed).
// MODE 0: H rows (apply shift A on free space, write back, transform H - dh_e).
// MODE 1: G rows (gdot = G - C, per-block sums of |gdot| on free space,
//         transform gdot on free space).
// MODE 2: rows of a double array.
// MODE 5: rows of a double array minus A on free space (A summed from the
//         per-block sums pp.in when given, else it->A).
// MODE 3: rows of the float iterate xf minus dh_e (it->hde), per-block sums
//         of w1 (xf - dh_e) over all nodes (the final double evaluation).
// MODE 6: rows of X - it->C on film nodes (flag bit 0), 0 elsewhere (the film
//         cotangent of the transposed iteration, spectral form).
template <typename T, int M, int MODE>
__global__ void __launch_bounds__((FilmRowShape<M, T>::THREADS))
    film_rows_fwd(T *__restrict__ X, const double *__restrict__ xd, const uint8_t *__restrict__ flags,
                  cx<T> *__restrict__ S, const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN,
                  FilmGeom G, double hde, Parts pp, IterState *__restrict__ it, const T *__restrict__ w1,
                  const float *__restrict__ xf) {
  using RS = FilmRowShape<M, T>;
  using PL = typename RS::PL;
  constexpr int TT = RS::TT, P = RS::P, RMAX = PL::RMAX, PITCH = RS::PITCH, SP = RS::SP;
  __shared__ __align__(16) T lds[RS::LDS_T];
  __shared__ double red[2 * (RS::THREADS / 64)];
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  RowTw<T, M, RS::THREADS> rtw;
  row_tw_fetch(rtw, twM, twN);
  const int blk = xcd_block(blockIdx.x, (G.ny + P - 1) / P);
  const int q0 = blk * P;
  const int q = q0 + pr;
  const bool active = q < G.ny;
  const long long ro = (long long)(active ? q : 0) * G.nx;
  // MODE 0: this thread's nodes 2m, 2m+1 (m = j + rho TT) of H, their flags
  // and w1, all loaded before any is used (a row past ny reads row 0 and is
  // not used).  MODE 3: the same nodes of xf and w1.
  T h0[RMAX][2], w0[RMAX][2];
  uint16_t f0[RMAX];
  if constexpr (MODE == 3) {
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const long long o = ro + 2 * (j + rho * TT);
      const float2 hv = *reinterpret_cast<const float2 *>(xf + o);
      h0[rho][0] = (T)hv.x;
      h0[rho][1] = (T)hv.y;
      w0[rho][0] = w1[o];
      w0[rho][1] = w1[o + 1];
    }
  }
  if constexpr (MODE == 0) {
    const T *wsrc = w1 ? w1 : X;   // without w1 the values read are not used
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const long long o = ro + 2 * (j + rho * TT);
      h0[rho][0] = X[o];
      h0[rho][1] = X[o + 1];
      f0[rho] = *reinterpret_cast<const uint16_t *>(flags + o);
      w0[rho][0] = wsrc[o];
      w0[rho][1] = wsrc[o + 1];
    }
  }
  // the stop flag is tested once the loads above are issued (nothing is
  // written before the test)
  if (it->done) return;
  // MODE 0: the shift A of (10) from the previous update's sums (or the
  // stencil's, already reduced into it->A); MODE 1: C = free-space mean of G.
  double shift = 0.0;
  if constexpr (MODE == 0) {
    // the shift A^0 from the stencil's per-block sums (or the value in it->A)
    shift = pp.in ? parts_sum(pp.in, pp.nin) * it->inv_nout : it->A;
    if (pp.in && blockIdx.x == 0 && threadIdx.x == 0) it->A = shift;
  }
  if constexpr (MODE == 1) {
    shift = parts_sum(pp.in, pp.nin) * it->inv_nout;
    if (blockIdx.x == 0 && threadIdx.x == 0) it->C = shift;
  }
  if constexpr (MODE == 5) {
    // A from per-block sums of the input over D (or the value in it->A)
    shift = pp.in ? parts_sum(pp.in, pp.nin) * it->inv_nout : it->A;
    if (pp.in && blockIdx.x == 0 && threadIdx.x == 0) it->A = shift;
  }
  // MODE 0 and 3 subtract dh_e/dt of the iteration state
  if constexpr (MODE == 0 || MODE == 3) hde = it->hde;
  double acc = 0.0, acc_film = 0.0;
  cx<T> v[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    T val[2] = {(T)0, (T)0};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = 2 * (j + rho * TT) + e;
      if (!active) continue;
      if constexpr (MODE == 0) {
        T h = h0[rho][e];
        const bool film = (f0[rho] >> (8 * e)) & 1;
        if (!film) {
          h = (T)((double)h - shift);
          X[ro + p] = h;
        }
        val[e] = (T)((double)h - hde);
        if (w1) {
          const double t = (double)w0[rho][e] * ((double)h - hde);
          acc += t;
          if (film) acc_film += t;
        }
      } else if constexpr (MODE == 3) {
        const double x = (double)h0[rho][e] - hde;
        val[e] = (T)x;
        acc += (double)w0[rho][e] * x;
      } else if constexpr (MODE == 1) {
        const double gd = (double)X[ro + p] - shift;
        if (!(flags[ro + p] & 1)) {
          acc += fabs(gd);
          val[e] = (T)gd;
        }
      } else if constexpr (MODE == 6) {
        if (flags[ro + p] & 1) val[e] = (T)((double)X[ro + p] - it->C);
      } else if constexpr (MODE == 5) {
        const double y = xd[ro + p] - ((flags[ro + p] & 1) ? 0.0 : shift);
        val[e] = (T)y;
        if (w1) acc += (double)w1[ro + p] * y;
      } else {
        val[e] = (T)xd[ro + p];
      }
    }
    v[rho] = {val[0], val[1]};
  }
  row_tw_put(rtw, twM, twN);   // first read after the transform's entry barrier
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pr * PITCH;
  pencil_fft_cx<M, -1, PL>(v, j, xch, [](int i) { return lds_pad<T>(i); }, twM);
  // Half spectrum of the real row from the packed transform Z:
  // X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) W^k (Z[k] - conj Z[M-k]), W = exp(-2 pi i / 2M).
  __syncthreads();
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) xch[j + rho * TT] = v[rho];
  __syncthreads();
  cx<T> xk[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const int km = k == 0 ? 0 : M - k;
    const cx<T> zk = v[rho];
    const cx<T> zm = conj(xch[km]);
    const cx<T> sum = zk + zm, dif = zk - zm;
    const cx<T> wd = cmul(twN[k], dif);
    xk[rho] = {(T)0.5 * (sum.x + wd.y), (T)0.5 * (sum.y - wd.x)};
  }
  const cx<T> xm = {v[0].x - v[0].y, (T)0};   // X[M], meaningful in thread j = 0
  __syncthreads();
  cx<T> *tile = reinterpret_cast<cx<T> *>(lds);   // [M+1][SP]
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) tile[(j + rho * TT) * SP + pr] = xk[rho];
  if (j == 0) tile[M * SP + pr] = xm;
  __syncthreads();
  tile_store<T, M, P, SP, RS::THREADS>(tile, S, G.ny, q0);
  if constexpr (MODE == 1) {
    const double sblk = block_total<RS::THREADS>(acc, red);
    if (threadIdx.x == 0) pp.out[blk] = sblk;
  }
  if constexpr (MODE == 0) {
    // the film part of the sums stays fixed while the iteration only
    // changes H on free space: per-block values for the update passes
    if (pp.out2) {
      const double sf = block_total<RS::THREADS>(acc_film, red + RS::THREADS / 64);
      if (threadIdx.x == 0) pp.out2[blk] = sf;
    }
  }
  if constexpr (MODE == 0 || MODE == 3 || MODE == 5) {
    if (pp.out) {
      const double sblk = block_total<RS::THREADS>(acc, red);
      if (threadIdx.x == 0) pp.out[blk] = sblk;
    }
  }
}

// Partial sums of the fused transposed iteration: the free-space mean of the
// new iterate is c_new * (sum of in_new); that of the previous one c_old *
// (sum of in_old) (in_old == NULL: the first pass, which has no previous one).
struct AdjParts {
  const double *in_new, *in_old, *in_a;
  int nin;
  double c_new, c_old;
  double *out, *out2, *out3;
};

// Fused row passes of the transposed iteration (the adjoint of (10)-(12)):
// MODE 8: mu_new = C2R (first pass) or mu - C_old - lambda C2R; write mu_new;
//         nu = mu_new - C_new; sums over free space of |nu| (out) and of
//         w2 nu (out2), and on the first pass sums of |mu_new| over D (out3);
//         R2C of nu on free space.
// MODE 9: z = C2R on free space (0 on the film), zz = z - A_z on free space
//         with A_z = (sum of w2 nu) / #out (in_a); sums of w1 zz over D (out,
//         the next mean); R2C of zz.
template <typename T, int M, int MODE>
__global__ void __launch_bounds__((FilmRowShape<M, T>::THREADS))
    film_rows_adj(T *__restrict__ X, const uint8_t *__restrict__ flags, cx<T> *__restrict__ S,
                  const T *__restrict__ w, const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN,
                  FilmGeom G, double lam, AdjParts pp, IterState *__restrict__ it) {
  using RS = FilmRowShape<M, T>;
  using PL = typename RS::PL;
  constexpr int TT = RS::TT, P = RS::P, RMAX = PL::RMAX, PITCH = RS::PITCH, SP = RS::SP;
  __shared__ __align__(16) T lds[RS::LDS_T];
  __shared__ double red[3 * (RS::THREADS / 64)];
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  const int blk = xcd_block(blockIdx.x, (G.ny + P - 1) / P);
  const int q0 = blk * P;
  const int q = q0 + pr;
  const bool active = q < G.ny;
  const long long ro = (long long)(active ? q : 0) * G.nx;
  // tile, twiddles and partial sums fetched together, then stored
  cx<T> *tile = reinterpret_cast<cx<T> *>(lds);   // [M+1][SP]
  TileRegs<T, M, P, RS::THREADS> tr;
  tile_fetch(tr, S, G.ny, q0);
  RowTw<T, M, RS::THREADS> rtw;
  row_tw_fetch(rtw, twM, twN);
  if (it->done) return;   // after the loads are issued; nothing written before
  double c_new = 0.0, c_old = 0.0, a_z = 0.0;
  if constexpr (MODE == 8) {
    c_new = pp.c_new * parts_sum(pp.in_new, pp.nin);
    if (pp.in_old) c_old = pp.c_old * parts_sum(pp.in_old, pp.nin);
    if (blockIdx.x == 0 && threadIdx.x == 0) it->C = c_new;
  } else {
    a_z = parts_sum(pp.in_a, pp.nin) * it->inv_nout;
  }
  tile_put<T, M, P, SP, RS::THREADS>(tile, tr);
  row_tw_put(rtw, twM, twN);
  __syncthreads();
  cx<T> v[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const cx<T> a = tile[k * SP + pr];
    const cx<T> b = tile[(M - k) * SP + pr];
    const cx<T> sum = {a.x + b.x, a.y - b.y};
    const cx<T> dif = {a.x - b.x, a.y + b.y};
    const cx<T> wd = cmulc(dif, twN[k]);
    v[rho] = {sum.x - wd.y, sum.y + wd.x};
  }
  if constexpr (PL::S == 1) __syncthreads();
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pr * PITCH;
  pencil_fft_cx<M, +1, PL>(v, j, xch, [](int i) { return lds_pad<T>(i); }, twM);
  double acc = 0.0, acc2 = 0.0, acc3 = 0.0;
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    T u[2] = {(T)0, (T)0};
    const T val[2] = {v[rho].x, v[rho].y};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = 2 * (j + rho * TT) + e;
      if (!active) continue;
      const bool out = !(flags[ro + p] & 1);
      if constexpr (MODE == 8) {
        const double mu = pp.in_old ? (double)X[ro + p] - c_old - lam * (double)val[e] : (double)val[e];
        const T mut = (T)mu;
        X[ro + p] = mut;
        acc3 += fabs((double)mut);
        const double wv = (double)w[ro + p];   // loaded with the flag, not after it
        if (out) {
          const double nu = (double)mut - c_new;
          acc += fabs(nu);
          acc2 += wv * nu;
          u[e] = (T)nu;
        }
      } else {
        const double zz = out ? (double)val[e] - a_z : 0.0;
        acc += (double)w[ro + p] * zz;
        u[e] = (T)zz;
      }
    }
    v[rho] = {u[0], u[1]};
  }
  pencil_fft_cx<M, -1, PL>(v, j, xch, [](int i) { return lds_pad<T>(i); }, twM);
  __syncthreads();
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) xch[j + rho * TT] = v[rho];
  __syncthreads();
  cx<T> xk[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const int km = k == 0 ? 0 : M - k;
    const cx<T> zk = v[rho];
    const cx<T> zm = conj(xch[km]);
    const cx<T> sum = zk + zm, dif = zk - zm;
    const cx<T> wd = cmul(twN[k], dif);
    xk[rho] = {(T)0.5 * (sum.x + wd.y), (T)0.5 * (sum.y - wd.x)};
  }
  const cx<T> xm = {v[0].x - v[0].y, (T)0};
  __syncthreads();
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) tile[(j + rho * TT) * SP + pr] = xk[rho];
  if (j == 0) tile[M * SP + pr] = xm;
  __syncthreads();
  tile_store<T, M, P, SP, RS::THREADS>(tile, S, G.ny, q0);
  constexpr int NW = RS::THREADS / 64;
  const double s1 = block_total<RS::THREADS>(acc, red);
  if (threadIdx.x == 0) pp.out[blk] = s1;
  if constexpr (MODE == 8) {
    const double s2 = block_total<RS::THREADS>(acc2, red + NW);
    if (threadIdx.x == 0) pp.out2[blk] = s2;
    if (pp.out3) {
      const double s3 = block_total<RS::THREADS>(acc3, red + 2 * NW);
      if (threadIdx.x == 0) pp.out3[blk] = s3;
    }
  }
}

// Fused row pass of the forward iteration: complex-to-real of the transposed
// spectrum, a pointwise step, real-to-complex of the result (transposed out).
// The free-space means C and A are not summed over the field itself: since
// K1 and K2 are symmetric, sum_out K x = sum_D (K 1_out) x, so with
// w = K 1_out precomputed they come from dot products taken one pass earlier.
// MODE 6 (after the 2/|k| pass; w = w2, NaN on film nodes, so the flags are
//        not read): G = C2R; write G (if keep) or, at the last
//        evaluation of a fixed count, the result gdot = G - C to `res`
//        (double); C = (sum of w1 (H - dh_e))
//        / #out; gdot = G - C; sums over free space of |gdot| (out) and of
//        w2 gdot (out2); R2C of gdot on free space.
// MODE 7 (after the |k|/2 pass; w = w1, NaN on film nodes): V = C2R; on
//        free space H <- H - lambda V - A with A = -lambda (sum of w2 gdot) /
//        #out, the shift that restores (10) (sum_D (H - dh_e) was 0 before
//        the update); sums of w1 (H - dh_e) over D (out, the next C: the free
//        space part here plus the fixed film part per block, read from
//        out2); R2C of H - dh_e.
template <typename T, int M, int MODE>
__global__ void __launch_bounds__((FilmRowShape<M, T>::THREADS))
    MAG_WAVES_PER_EU(FilmRowShape<M, T>::WAVES_EU)
    film_rows_fused(T *__restrict__ X, const uint8_t *__restrict__ flags, cx<T> *__restrict__ S,
                    const T *__restrict__ w, const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN,
                    FilmGeom G, double lam, Parts pp, IterState *__restrict__ it, int keep,
                    double *__restrict__ res) {
  using RS = FilmRowShape<M, T>;
  using PL = typename RS::PL;
  constexpr int TT = RS::TT, P = RS::P, RMAX = PL::RMAX, PITCH = RS::PITCH, SP = RS::SP;
  __shared__ __align__(16) T lds[RS::LDS_T];
  __shared__ double red[2 * (RS::THREADS / 64)];
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  const int blk = xcd_block(blockIdx.x, (G.ny + P - 1) / P);
  const int q0 = blk * P;
  const int q = q0 + pr;
  const bool active = q < G.ny;
  const long long ro = (long long)(active ? q : 0) * G.nx;
  // Loads in the order they are needed (memory returns them in order): the
  // tile, the twiddles, the partial sums, then the weights of this thread's
  // nodes 2m, 2m+1 (m = j + rho TT; NaN on film nodes, so they carry the
  // free-space flag too; a row past ny reads row 0 and is not used), which
  // stay in flight while the tile is stored to LDS and transformed.
  cx<T> *tile = reinterpret_cast<cx<T> *>(lds);   // [M+1][SP]
  TileRegs<T, M, P, RS::THREADS> tr;
  tile_fetch(tr, S, G.ny, q0);
  RowTw<T, M, RS::THREADS> rtw;
  row_tw_fetch(rtw, twM, twN);
  // the stop flag is tested after the tile and twiddle loads are issued (they
  // do not depend on it and nothing is written before the test), so its load
  // does not delay theirs: -0.2 / -0.4 us on passes 2 / 4 at 2048^2
  if (it->done) return;
  const double hde = it->hde;
  double cst;
  if constexpr (MODE == 6) {
    cst = parts_sum(pp.in, pp.nin) * it->inv_nout;   // C
    if (blockIdx.x == 0 && threadIdx.x == 0) it->C = cst;
  } else {
    cst = -lam * parts_sum(pp.in, pp.nin) * it->inv_nout;   // A
  }
  T wpre[RMAX][2];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const long long o = ro + 2 * (j + rho * TT);
    wpre[rho][0] = w[o];
    wpre[rho][1] = w[o + 1];
  }
  tile_put<T, M, P, SP, RS::THREADS>(tile, tr);
  row_tw_put(rtw, twM, twN);
  __syncthreads();
  cx<T> v[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const cx<T> a = tile[k * SP + pr];
    const cx<T> b = tile[(M - k) * SP + pr];
    const cx<T> sum = {a.x + b.x, a.y - b.y};
    const cx<T> dif = {a.x - b.x, a.y + b.y};
    const cx<T> wd = cmulc(dif, twN[k]);
    v[rho] = {sum.x - wd.y, sum.y + wd.x};
  }
  if constexpr (PL::S == 1) __syncthreads();
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pr * PITCH;
  pencil_fft_cx<M, +1, PL>(v, j, xch, [](int i) { return lds_pad<T>(i); }, twM);
  double acc = 0.0, acc2 = 0.0;
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    T u[2] = {(T)0, (T)0};
    const T val[2] = {v[rho].x, v[rho].y};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = 2 * (j + rho * TT) + e;
      if (!active) continue;
      if constexpr (MODE == 6) {
        const double wv = (double)wpre[rho][e];
        const bool out = !isnan(wv);
        if (keep) X[ro + p] = val[e];
        if (res) res[ro + p] = (double)val[e] - cst;
        if (out) {
          const double gd = (double)val[e] - cst;
          acc += fabs(gd);
          acc2 += wv * gd;
          u[e] = (T)gd;
        }
      } else {
        // free space: update (12) and the free-space part of the w1 sums
        // (the film part, fixed, is added per block below)
        const double wv = (double)wpre[rho][e];
        T h = X[ro + p];
        if (!isnan(wv)) {
          h = (T)((double)h - lam * (double)val[e] - cst);
          X[ro + p] = h;
          acc += wv * ((double)h - hde);
        }
        u[e] = (T)((double)h - hde);
      }
    }
    v[rho] = {u[0], u[1]};
  }
  pencil_fft_cx<M, -1, PL>(v, j, xch, [](int i) { return lds_pad<T>(i); }, twM);
  __syncthreads();
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) xch[j + rho * TT] = v[rho];
  __syncthreads();
  cx<T> xk[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const int km = k == 0 ? 0 : M - k;
    const cx<T> zk = v[rho];
    const cx<T> zm = conj(xch[km]);
    const cx<T> sum = zk + zm, dif = zk - zm;
    const cx<T> wd = cmul(twN[k], dif);
    xk[rho] = {(T)0.5 * (sum.x + wd.y), (T)0.5 * (sum.y - wd.x)};
  }
  const cx<T> xm = {v[0].x - v[0].y, (T)0};
  __syncthreads();
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) tile[(j + rho * TT) * SP + pr] = xk[rho];
  if (j == 0) tile[M * SP + pr] = xm;
  __syncthreads();
  tile_store<T, M, P, SP, RS::THREADS>(tile, S, G.ny, q0);
  const double s1 = block_total<RS::THREADS>(acc, red);
  if constexpr (MODE == 6) {
    if (threadIdx.x == 0) pp.out[blk] = s1;
  } else {
    if (threadIdx.x == 0) pp.out[blk] = s1 + pp.out2[blk];
  }
  if constexpr (MODE == 6) {
    const double s2 = block_total<RS::THREADS>(acc2, red + RS::THREADS / 64);
    if (threadIdx.x == 0) pp.out2[blk] = s2;
  }
}

// Row transforms (complex-to-real along x, input transposed).
// MODE 0: write G, per-block sums of G over free space.
// MODE 1: V -> H -= lambda V on free space, per-block sums of H - dh_e over D.
// MODE 2: write hz = h_e + value (double).
// Transposed iteration (the adjoint of (10)-(12)):
// MODE 3: write the value on free space, 0 on the film; sums over free space.
// MODE 4: X <- X - C - lambda value; sums of the new X over free space.
// MODE 5: write the value; sums over free space, and sums of |value| over D
//         (second half of part).
// Final double evaluation:
// MODE 6: write gdot = value - C (double), C = (sum of pp.in) / #out; with
//         pp.out, sums of |gdot| over free space.
// Spectral form:
// MODE 7: write the value into X at film nodes (flag bit 0), nothing else.
// MODE 8: write -value (double).
template <typename T, int M, int MODE>
__global__ void __launch_bounds__((FilmRowShape<M, T>::THREADS))
    film_rows_inv(T *__restrict__ X, double *__restrict__ xd, const uint8_t *__restrict__ flags,
                  const cx<T> *__restrict__ S, const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN,
                  FilmGeom G, double hde, double lam, Parts pp, const IterState *__restrict__ it) {
  if (it->done) return;
  using RS = FilmRowShape<M, T>;
  using PL = typename RS::PL;
  constexpr int TT = RS::TT, P = RS::P, RMAX = PL::RMAX, PITCH = RS::PITCH, SP = RS::SP;
  __shared__ __align__(16) T lds[RS::LDS_T];
  __shared__ double red[2 * (RS::THREADS / 64)];
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  const int blk = xcd_block(blockIdx.x, (G.ny + P - 1) / P);
  const int q0 = blk * P;
  const int q = q0 + pr;
  const bool active = q < G.ny;
  const long long ro = (long long)(active ? q : 0) * G.nx;
  // MODE 4: the free-space mean of the iteration state; MODE 6: from the
  // per-block sums pp.in of the forward pass (MODE 3)
  double cmean = 0.0;
  if constexpr (MODE == 4) cmean = it->C;
  if constexpr (MODE == 6) cmean = parts_sum(pp.in, pp.nin) * it->inv_nout;
  double acc2 = 0.0;
  cx<T> *tile = reinterpret_cast<cx<T> *>(lds);   // [M+1][SP]
  {
    TileRegs<T, M, P, RS::THREADS> tr;
    tile_fetch(tr, S, G.ny, q0);
    RowTw<T, M, RS::THREADS> rtw;
    row_tw_fetch(rtw, twM, twN);
    tile_put<T, M, P, SP, RS::THREADS>(tile, tr);
    row_tw_put(rtw, twM, twN);
  }
  __syncthreads();
  // Z[k] = (X[k] + conj X[M-k]) + i W^{-k} (X[k] - conj X[M-k]); the inverse
  // transform of Z is x[2m] + i x[2m+1] times 2M.
  cx<T> v[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const cx<T> a = tile[k * SP + pr];
    const cx<T> b = tile[(M - k) * SP + pr];
    const cx<T> sum = {a.x + b.x, a.y - b.y};
    const cx<T> dif = {a.x - b.x, a.y + b.y};
    const cx<T> wd = cmulc(dif, twN[k]);
    v[rho] = {sum.x - wd.y, sum.y + wd.x};
  }
  if constexpr (PL::S == 1) __syncthreads();   // single-stage FFTs do not fence the tile
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pr * PITCH;
  pencil_fft_cx<M, +1, PL>(v, j, xch, [](int i) { return lds_pad<T>(i); }, twM);
  double acc = 0.0;
  if (active) {
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int m = j + rho * TT;
      const T val[2] = {v[rho].x, v[rho].y};
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int p = 2 * m + e;
        const bool out = !(flags[ro + p] & 1);
        if constexpr (MODE == 0) {
          X[ro + p] = val[e];
          if (out) acc += (double)val[e];
        } else if constexpr (MODE == 1) {
          T h = X[ro + p];
          if (out) {
            h = (T)((double)h - lam * (double)val[e]);
            X[ro + p] = h;
          }
          acc += (double)h - hde;
        } else if constexpr (MODE == 3) {
          X[ro + p] = out ? val[e] : (T)0;
          if (out) acc += (double)val[e];
        } else if constexpr (MODE == 4) {
          const T h = (T)((double)X[ro + p] - cmean - lam * (double)val[e]);
          X[ro + p] = h;
          if (out) acc += (double)h;
        } else if constexpr (MODE == 5) {
          X[ro + p] = val[e];
          if (out) acc += (double)val[e];
          acc2 += fabs((double)val[e]);
        } else if constexpr (MODE == 7) {
          if (!out) X[ro + p] = val[e];
        } else if constexpr (MODE == 8) {
          xd[ro + p] = -(double)val[e];
        } else if constexpr (MODE == 6) {
          const double gd = (double)val[e] - cmean;
          xd[ro + p] = gd;
          if (out) acc += fabs(gd);
        } else {
          xd[ro + p] = hde + (double)val[e];
        }
      }
    }
  }
  if constexpr (MODE != 2 && MODE != 7 && MODE != 8) {
    if (MODE != 6 || pp.out) {   // uniform over the block
      const double sblk = block_total<RS::THREADS>(acc, red);
      if (threadIdx.x == 0) pp.out[blk] = sblk;
    }
  }
  if constexpr (MODE == 5) {
    const double sblk2 = block_total<RS::THREADS>(acc2, red + RS::THREADS / 64);
    if (threadIdx.x == 0) pp.out2[blk] = sblk2;
  }
}

// Column pass on the transposed spectrum: forward y transform of contiguous
// columns, multiplier K(|k|) / N, inverse y transform.
// which = 0: 2/|k| (eq. (7) solved for g, 0 at k = 0); which = 1: |k|/2 (eq. (12)).
// The kx = 0 and kx = M (= nx/2) columns of the half spectrum of real rows are
// real; they travel as the real and imaginary parts of one complex column,
// processed by pencil 0 of block 0, so the pass covers kx - 1 = M pencils
// (M divides evenly over the compute units at the usual sizes).  With
// Z = a + i b (a, b real) and Zh its transform, the two spectra are
// (Zh[k] + conj Zh[-k]) / 2 and (Zh[k] - conj Zh[-k]) / (2i), so the product
// with the multipliers m0 (kx = 0) and mM (kx = M) is
//   W[k] = (m0 + mM)/2 Zh[k] + (m0 - mM)/2 conj Zh[-k],
// whose inverse transform is out0 + i outM.
template <typename T, int NY>
__global__ void __launch_bounds__((FilmColShape<NY, T>::THREADS))
    film_cols(cx<T> *__restrict__ S, int kx, const double *__restrict__ k2x, const double *__restrict__ k2y,
              double inv_n, int which, const cx<T> *__restrict__ tw, Parts pp, IterState *__restrict__ it,
              IterState *mirror) {
  using CS = FilmColShape<NY, T>;
  using PL = typename CS::PL;
  constexpr int TT = CS::TT, P = CS::P, RMAX = PL::RMAX, PITCH = CS::PITCH;
  __shared__ __align__(16) T lds[CS::LDS_T];
  if (pp.in) {
    // Stop test of Sec. 2.3 on the residual sums of the previous pass: every
    // block takes the same decision; block 0 records it.  The flag of an
    // earlier stop is tested once the sums are loaded.
    const double r = parts_sum(pp.in, pp.nin) * it->inv_nout;
    if (it->done) return;
    const int iters = pp.iter + 1;
    const int fixed = it->fixed;
    const int done = !isfinite(r) ? 2 : (fixed > 0 ? (iters >= fixed ? 1 : 0) : (r < it->thr ? 1 : 0));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      it->r = r;
      it->iters = iters;
      it->done = done;
      if (done == 2) it->fail = 1;
      *mirror = *it;
    }
    if (done) return;
  }
  const int pcol = threadIdx.x / TT, j = threadIdx.x % TT;
  // FP64 forms the twiddle powers inside each stage (register budget of 4
  // blocks per CU); FP32 leaves the compiler free to keep them for the
  // inverse transform.
  TwPre<PL, T, (sizeof(T) > 4)> twp;
  tw_preload<NY, PL>(twp, j, tw);
  const int col = blockIdx.x * P + pcol;
  const bool active = col < kx - 1;
  const bool pair_block = blockIdx.x == 0;          // uniform over the block
  const bool packed = pair_block && pcol == 0;
  cx<T> *base = S + (long long)(active ? col : 0) * NY;
  cx<T> *base_m = S + (long long)(kx - 1) * NY;
  cx<T> v[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int y = j + rho * TT;
    if (packed) v[rho] = {base[y].x, base_m[y].x};
    else v[rho] = active ? base[y] : cx<T>{(T)0, (T)0};
  }
  // |k|^2 terms of the multiplier, loaded with the column
  T ky2[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) ky2[rho] = (T)k2y[j + rho * TT];
  const T kxx = (T)k2x[active ? col : 0], kxm = (T)k2x[kx - 1];
  // without a decision in this pass the stop flag is tested once the
  // column's loads are issued (nothing is written before the test)
  if (!pp.in && it->done) return;
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pcol * PITCH;
  auto lidx = [](int i) { return lds_pad<T>(i); };
  pencil_fft_cx<NY, -1, PL>(v, j, xch, lidx, twp);
  // multiplier in the compute precision: |k|^2 = kx^2 + ky^2
  const T c1 = (T)(2.0 * inv_n), c2 = (T)(0.5 * inv_n);
  auto mult = [&](T kk2) -> T {
    if (which == 0) return kk2 > (T)0 ? c1 * inv_sqrt(kk2) : (T)0;
    return c2 * mult_sqrt(kk2);
  };
  if (pair_block) {
    __syncthreads();   // the transform's last LDS reads are done
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) xch[lidx(j + rho * TT)] = v[rho];
    __syncthreads();
  }
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    const T m0 = mult(kxx + ky2[rho]);
    if (packed) {
      const cx<T> zm = conj(xch[lidx(k == 0 ? 0 : NY - k)]);
      const T mm = mult(kxm + ky2[rho]);
      const T hp = (T)0.5 * (m0 + mm), hm = (T)0.5 * (m0 - mm);
      v[rho] = {hp * v[rho].x + hm * zm.x, hp * v[rho].y + hm * zm.y};
    } else {
      v[rho] = scale(v[rho], m0);
    }
  }
  pencil_fft_cx<NY, +1, PL>(v, j, xch, lidx, twp);
  if (packed) {
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      base[j + rho * TT] = {v[rho].x, (T)0};
      base_m[j + rho * TT] = {v[rho].y, (T)0};
    }
  } else if (active) {
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) base[j + rho * TT] = v[rho];
  }
}

// Column passes of the spectral form (Sec. 2.2).  A derivative d/dx_a is
// the symbol i s_a, s_a = k_a exp(-|k|^2 sigma^2 / 2) / N (N = nx ny, the
// normalisation of the two transforms), with k_a the signed wavenumber of
// axis a and its Nyquist value set to 0 (an odd symbol has no real value
// there): kxs, kys.  The Gaussian factor is separable: fx[kx] fy[ky] with
// fx = exp(-kx^2 sigma^2 / 2), fy = exp(-ky^2 sigma^2 / 2) from tables.  The symbols are Hermitian, so the packed kx = 0 / kx = M
// pencil is split by the identity of film_cols with complex multipliers,
//   W[k] = (m0 + mM)/2 Zh[k] + (m0 - mM)/2 conj Zh[-k].
// OP 0 (gradient): from the spectrum of g in S, the spectra of j_x = d_y g
//      (to S) and j_y = -d_x g (to S2), eq. (2) at the nodes.
// OP 1 (curl): from the spectra of e_x (S) and e_y (S2), the spectrum of
//      dh_z/dt = d_y e_x - d_x e_y (to S), eq. (9).
template <typename T, int NY, int OP>
__global__ void __launch_bounds__((FilmColShape<NY, T>::THREADS))
    film_cols_spec(cx<T> *__restrict__ S, cx<T> *__restrict__ S2, int kx, const double *__restrict__ fx,
                   const double *__restrict__ fy, const double *__restrict__ kxs, const double *__restrict__ kys,
                   double inv_n, const cx<T> *__restrict__ tw, const IterState *__restrict__ it) {
  using CS = FilmColShape<NY, T>;
  using PL = typename CS::PL;
  constexpr int TT = CS::TT, P = CS::P, RMAX = PL::RMAX, PITCH = CS::PITCH;
  __shared__ __align__(16) T lds[CS::LDS_T];
  const int pcol = threadIdx.x / TT, j = threadIdx.x % TT;
  // two columns held at once (OP 0: the two results, OP 1: the two inputs):
  // twiddle powers formed per stage, which keeps 4 waves per SIMD in FP32
  TwPre<PL, T, true> twp;
  tw_preload<NY, PL>(twp, j, tw);
  const int col = blockIdx.x * P + pcol;
  const bool active = col < kx - 1;
  const bool pair_block = blockIdx.x == 0;   // uniform over the block
  const bool packed = pair_block && pcol == 0;
  const long long co = (long long)(active ? col : 0) * NY, cm = (long long)(kx - 1) * NY;
  // OP 0: v = the spectrum of g; OP 1: v = e_x, u = e_y
  cx<T> v[RMAX], u[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int y = j + rho * TT;
    if (packed) v[rho] = {S[co + y].x, S[cm + y].x};
    else v[rho] = active ? S[co + y] : cx<T>{(T)0, (T)0};
    if constexpr (OP == 1) {
      if (packed) u[rho] = {S2[co + y].x, S2[cm + y].x};
      else u[rho] = active ? S2[co + y] : cx<T>{(T)0, (T)0};
    }
  }
  T fyv[RMAX], kya[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    fyv[rho] = (T)fy[j + rho * TT];
    kya[rho] = (T)kys[j + rho * TT];
  }
  const T fxc = (T)(fx[active ? col : 0] * inv_n), fxm = (T)(fx[kx - 1] * inv_n);
  const T kxa = (T)kxs[active ? col : 0], kxam = (T)kxs[kx - 1];
  if (it->done) return;
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pcol * PITCH;
  auto lidx = [](int i) { return lds_pad<T>(i); };
  pencil_fft_cx<NY, -1, PL>(v, j, xch, lidx, twp);
  // (each transform starts with a barrier: a column has at least two stages)
  if constexpr (OP == 1) pencil_fft_cx<NY, -1, PL>(u, j, xch, lidx, twp);
  // the packed pencil reads the mirrored entries conj Zh[-k] of a transform
  // from the LDS (block 0 only; the next transform starts with a barrier)
  auto mirror_to_lds = [&](const cx<T> *w) {
    if (pair_block) {
      lds_barrier();
#pragma unroll
      for (int rho = 0; rho < RMAX; ++rho) xch[lidx(j + rho * TT)] = w[rho];
      lds_barrier();
    }
  };
  // i (hp Z + hm conj Z[-k]) with hp = (s0 + sM) / 2, hm = (s0 - sM) / 2; i s0 Z off the packed pencil
  auto apply = [&](const cx<T> &z, int k, T s0, T sm) -> cx<T> {
    if (packed) {
      const cx<T> zm = conj(xch[lidx(k == 0 ? 0 : NY - k)]);
      const T hp = (T)0.5 * (s0 + sm), hm = (T)0.5 * (s0 - sm);
      return {-(hp * z.y + hm * zm.y), hp * z.x + hm * zm.x};
    }
    return {-s0 * z.y, s0 * z.x};
  };
  // the filter (times 1/N) at (kx, ky) and, on the packed pencil, at (M, ky)
  auto filt = [&](int rho, T &f0, T &fm) {
    f0 = fxc * fyv[rho];
    fm = fxm * fyv[rho];
  };
  mirror_to_lds(v);
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int k = j + rho * TT;
    T f0, fm;
    filt(rho, f0, fm);
    if constexpr (OP == 0) {
      u[rho] = apply(v[rho], k, -kxa * f0, -kxam * fm);       // j_y = -d_x g
    }
    v[rho] = apply(v[rho], k, kya[rho] * f0, kya[rho] * fm);  // j_x = d_y g, or d_y e_x
  }
  if constexpr (OP == 1) {
    mirror_to_lds(u);
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      T f0, fm;
      filt(rho, f0, fm);
      const cx<T> b = apply(u[rho], j + rho * TT, kxa * f0, kxam * fm);   // d_x e_y
      v[rho] = {v[rho].x - b.x, v[rho].y - b.y};
    }
  }
  pencil_fft_cx<NY, +1, PL>(v, j, xch, lidx, twp);
  auto store = [&](cx<T> *__restrict__ D, const cx<T> *w) {
    if (packed) {
#pragma unroll
      for (int rho = 0; rho < RMAX; ++rho) {
        D[co + j + rho * TT] = {w[rho].x, (T)0};
        D[cm + j + rho * TT] = {w[rho].y, (T)0};
      }
    } else if (active) {
#pragma unroll
      for (int rho = 0; rho < RMAX; ++rho) D[co + j + rho * TT] = w[rho];
    }
  };
  store(S, v);
  if constexpr (OP == 0) {
    pencil_fft_cx<NY, +1, PL>(u, j, xch, lidx, twp);
    store(S2, u);
  }
}

// Per-node critical current of the spectral form: the mean of the four cells
// around node (p, q) (summed in the order (p,q), (p-1,q), (p,q-1),
// (p-1,q-1)) where all four are superconducting, NaN at every other node
// (rho_out applies there).
template <typename T>
__global__ void __launch_bounds__(256) film_node_jc(const uint8_t *__restrict__ mat, const T *__restrict__ jc,
                                                    T *__restrict__ jcn, FilmGeom G, FilmLaw law) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long n = (long long)G.nx * G.ny;
  if (i >= n) return;
  const int p = (int)(i % G.nx), q = (int)(i / G.nx);
  const long long r0 = (long long)q * G.nx, rm = (long long)wrap(q - 1, G.ny) * G.nx;
  const int pm = wrap(p - 1, G.nx);
  const long long c[4] = {r0 + p, r0 + pm, rm + p, rm + pm};
  bool sc = true;
#pragma unroll
  for (int a = 0; a < 4; ++a) sc = sc && mat[c[a]] == 1;
  const T v = law.has_jc ? (T)0.25 * (jc[c[0]] + jc[c[1]] + jc[c[2]] + jc[c[3]]) : (T)law.jc0;
  jcn[i] = sc ? v : (T)NAN;
}

// Row pass of the spectral form between its two column passes: C2R of the
// spectra of j_x (S) and j_y (S2) along x, e = rho(|j|) j at each node (the
// power law (3) where jcn is a number, rho_out where it is NaN), R2C of e_x
// (to S) and e_y (to S2).  Same tiles, twiddles and packing as
// film_rows_fused; the two components pass through the LDS one after the
// other.
template <typename T, int M>
__global__ void __launch_bounds__((FilmRowShape<M, T>::THREADS))
    MAG_WAVES_PER_EU(FilmRowShape<M, T>::WAVES_EU)
    film_rows_node_e(cx<T> *__restrict__ S, cx<T> *__restrict__ S2, const T *__restrict__ jcn,
                     const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN, FilmGeom G, FilmLaw law,
                     const IterState *__restrict__ it) {
  using RS = FilmRowShape<M, T>;
  using PL = typename RS::PL;
  constexpr int TT = RS::TT, P = RS::P, RMAX = PL::RMAX, PITCH = RS::PITCH, SP = RS::SP;
  __shared__ __align__(16) T lds[RS::LDS_T];
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  const int blk = xcd_block(blockIdx.x, (G.ny + P - 1) / P);
  const int q0 = blk * P;
  const int q = q0 + pr;
  const long long ro = (long long)(q < G.ny ? q : 0) * G.nx;
  cx<T> *tile = reinterpret_cast<cx<T> *>(lds);   // [M+1][SP]
  TileRegs<T, M, P, RS::THREADS> t1, t2;
  tile_fetch(t1, S, G.ny, q0);
  tile_fetch(t2, S2, G.ny, q0);
  RowTw<T, M, RS::THREADS> rtw;
  row_tw_fetch(rtw, twM, twN);
  if (it->done) return;
  T jn[RMAX][2];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const long long o = ro + 2 * (j + rho * TT);
    jn[rho][0] = jcn[o];
    jn[rho][1] = jcn[o + 1];
  }
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pr * PITCH;
  auto lidx = [](int i) { return lds_pad<T>(i); };
  // C2R of the tile: Z[k] = (X[k] + conj X[M-k]) + i W^{-k} (X[k] - conj X[M-k]);
  // its inverse transform holds the values of nodes 2m, 2m+1
  auto c2r = [&](cx<T> *vv) {
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int k = j + rho * TT;
      const cx<T> a = tile[k * SP + pr];
      const cx<T> b = tile[(M - k) * SP + pr];
      const cx<T> sum = {a.x + b.x, a.y - b.y};
      const cx<T> dif = {a.x - b.x, a.y + b.y};
      const cx<T> wd = cmulc(dif, twN[k]);
      vv[rho] = {sum.x - wd.y, sum.y + wd.x};
    }
    if constexpr (PL::S == 1) __syncthreads();   // single-stage FFTs do not fence the tile
    pencil_fft_cx<M, +1, PL>(vv, j, xch, lidx, twM);
  };
  // R2C of the node values in vv into the tile, then to D
  auto r2c_store = [&](cx<T> *vv, cx<T> *__restrict__ D) {
    pencil_fft_cx<M, -1, PL>(vv, j, xch, lidx, twM);
    __syncthreads();
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) xch[j + rho * TT] = vv[rho];
    __syncthreads();
    cx<T> xk[RMAX];
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int k = j + rho * TT;
      const int km = k == 0 ? 0 : M - k;
      const cx<T> zk = vv[rho];
      const cx<T> zm = conj(xch[km]);
      const cx<T> sum = zk + zm, dif = zk - zm;
      const cx<T> wd = cmul(twN[k], dif);
      xk[rho] = {(T)0.5 * (sum.x + wd.y), (T)0.5 * (sum.y - wd.x)};
    }
    const cx<T> xm = {vv[0].x - vv[0].y, (T)0};
    __syncthreads();
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) tile[(j + rho * TT) * SP + pr] = xk[rho];
    if (j == 0) tile[M * SP + pr] = xm;
    __syncthreads();
    tile_store<T, M, P, SP, RS::THREADS>(tile, D, G.ny, q0);
  };
  tile_put<T, M, P, SP, RS::THREADS>(tile, t1);
  row_tw_put(rtw, twM, twN);
  __syncthreads();
  cx<T> jx[RMAX], jy[RMAX];
  c2r(jx);
  __syncthreads();   // the transform's last LDS reads are done
  tile_put<T, M, P, SP, RS::THREADS>(tile, t2);
  __syncthreads();
  c2r(jy);
  const T e0 = (T)law.e0, nm1 = (T)law.nm1, lmax = (T)law.lmax, rout = (T)law.rho_out;
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const T ax[2] = {jx[rho].x, jx[rho].y}, ay[2] = {jy[rho].x, jy[rho].y};
    T ex[2], ey[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const T jcv = jn[rho][e];
      const T r = isnan(jcv) ? rout : film_rho(sqrt(ax[e] * ax[e] + ay[e] * ay[e]), jcv, e0, nm1, lmax);
      ex[e] = r * ax[e];
      ey[e] = r * ay[e];
    }
    jx[rho] = {ex[0], ex[1]};
    jy[rho] = {ey[0], ey[1]};
  }
  __syncthreads();   // the second C2R's last LDS reads are done
  r2c_store(jx, S);
  __syncthreads();   // the tile has been read out
  r2c_store(jy, S2);
}

// Row pass of the transposed spectral form: C2R of the spectra of j_x (Sj),
// j_y (Sj2), a = d_y hbar (S) and b = -d_x hbar (S2), so that e_bar =
// (-a, -b); then at each node j_bar = rho e_bar + rho (n-1) (j.e_bar) j / |j|^2
// and the cotangent of the node jc, -n rho (j.e_bar) / jc, at power-law nodes
// (jcn a number), j_bar = rho_out e_bar elsewhere; R2C of j_bar_x (to S) and
// j_bar_y (to S2); the node jc cotangent to cn (if not null).  The four tiles
// pass through the LDS one after the other.
// (Four transformed rows are held at once: a register budget of 2 waves per
// SIMD in FP32 with eight values per work-item, 1 otherwise, so that nothing
// spills.)
template <typename T, int M>
__global__ void __launch_bounds__((FilmRowShape<M, T>::THREADS))
    MAG_WAVES_PER_EU(sizeof(T) == 4 && FilmRowShape<M, T>::PL::RMAX <= 8 ? 2 : 1)
    film_rows_node_ebar(cx<T> *__restrict__ S, cx<T> *__restrict__ S2, const cx<T> *__restrict__ Sj,
                        const cx<T> *__restrict__ Sj2, const T *__restrict__ jcn, double *__restrict__ cn,
                        const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN, FilmGeom G, FilmLaw law,
                        const IterState *__restrict__ it) {
  using RS = FilmRowShape<M, T>;
  using PL = typename RS::PL;
  constexpr int TT = RS::TT, P = RS::P, RMAX = PL::RMAX, PITCH = RS::PITCH, SP = RS::SP;
  __shared__ __align__(16) T lds[RS::LDS_T];
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  const int blk = xcd_block(blockIdx.x, (G.ny + P - 1) / P);
  const int q0 = blk * P;
  const int q = q0 + pr;
  const bool active = q < G.ny;
  const long long ro = (long long)(active ? q : 0) * G.nx;
  cx<T> *tile = reinterpret_cast<cx<T> *>(lds);   // [M+1][SP]
  RowTw<T, M, RS::THREADS> rtw;
  row_tw_fetch(rtw, twM, twN);
  if (it->done) return;
  T jn[RMAX][2];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const long long o = ro + 2 * (j + rho * TT);
    jn[rho][0] = jcn[o];
    jn[rho][1] = jcn[o + 1];
  }
  cx<T> *xch = reinterpret_cast<cx<T> *>(lds) + pr * PITCH;
  auto lidx = [](int i) { return lds_pad<T>(i); };
  bool tw_ready = false;
  // C2R of the spectrum Src along the block's rows into vv (nodes 2m, 2m+1)
  auto c2r = [&](const cx<T> *__restrict__ Src, cx<T> *vv) {
    TileRegs<T, M, P, RS::THREADS> tr;
    tile_fetch(tr, Src, G.ny, q0);
    __syncthreads();   // the previous use of the LDS is done
    tile_put<T, M, P, SP, RS::THREADS>(tile, tr);
    if (!tw_ready) row_tw_put(rtw, twM, twN);
    tw_ready = true;
    __syncthreads();
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int k = j + rho * TT;
      const cx<T> a = tile[k * SP + pr];
      const cx<T> b = tile[(M - k) * SP + pr];
      const cx<T> sum = {a.x + b.x, a.y - b.y};
      const cx<T> dif = {a.x - b.x, a.y + b.y};
      const cx<T> wd = cmulc(dif, twN[k]);
      vv[rho] = {sum.x - wd.y, sum.y + wd.x};
    }
    if constexpr (PL::S == 1) __syncthreads();
    pencil_fft_cx<M, +1, PL>(vv, j, xch, lidx, twM);
  };
  auto r2c_store = [&](cx<T> *vv, cx<T> *__restrict__ D) {
    pencil_fft_cx<M, -1, PL>(vv, j, xch, lidx, twM);
    __syncthreads();
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) xch[j + rho * TT] = vv[rho];
    __syncthreads();
    cx<T> xk[RMAX];
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int k = j + rho * TT;
      const int km = k == 0 ? 0 : M - k;
      const cx<T> zk = vv[rho];
      const cx<T> zm = conj(xch[km]);
      const cx<T> sum = zk + zm, dif = zk - zm;
      const cx<T> wd = cmul(twN[k], dif);
      xk[rho] = {(T)0.5 * (sum.x + wd.y), (T)0.5 * (sum.y - wd.x)};
    }
    const cx<T> xm = {vv[0].x - vv[0].y, (T)0};
    __syncthreads();
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) tile[(j + rho * TT) * SP + pr] = xk[rho];
    if (j == 0) tile[M * SP + pr] = xm;
    __syncthreads();
    tile_store<T, M, P, SP, RS::THREADS>(tile, D, G.ny, q0);
  };
  cx<T> jx[RMAX], jy[RMAX], ax[RMAX], ay[RMAX];
  c2r(Sj, jx);
  c2r(Sj2, jy);
  c2r(S, ax);
  c2r(S2, ay);
  const T e0 = (T)law.e0, nm1 = (T)law.nm1, lmax = (T)law.lmax, rout = (T)law.rho_out, nex = (T)(law.nm1 + 1.0);
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const T jxv[2] = {jx[rho].x, jx[rho].y}, jyv[2] = {jy[rho].x, jy[rho].y};
    const T ex[2] = {-ax[rho].x, -ax[rho].y}, ey[2] = {-ay[rho].x, -ay[rho].y};
    T bx[2], by[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const T jcv = jn[rho][e];
      T c_node = (T)0;
      if (isnan(jcv)) {
        bx[e] = rout * ex[e];
        by[e] = rout * ey[e];
      } else {
        const T s2 = jxv[e] * jxv[e] + jyv[e] * jyv[e];
        const T r = film_rho(sqrt(s2), jcv, e0, nm1, lmax);
        const T jd = jxv[e] * ex[e] + jyv[e] * ey[e];
        const T fac = s2 > (T)0 ? r * nm1 * jd / s2 : (T)0;
        bx[e] = r * ex[e] + fac * jxv[e];
        by[e] = r * ey[e] + fac * jyv[e];
        c_node = -nex * r * jd / jcv;
      }
      if (cn && active) cn[ro + 2 * (j + rho * TT) + e] = (double)c_node;
    }
    jx[rho] = {bx[0], bx[1]};
    jy[rho] = {by[0], by[1]};
  }
  __syncthreads();   // the last C2R's LDS reads are done
  r2c_store(jx, S);
  __syncthreads();
  r2c_store(jy, S2);
}

// Cotangent of the cell jc map from that of the node jc (node (p, q) takes
// the mean of cells (p,q), (p-1,q), (p,q-1), (p-1,q-1)): cell (p, q)
// collects a quarter of nodes (p,q), (p+1,q), (p,q+1), (p+1,q+1), times jc0.
__global__ void __launch_bounds__(256) film_cell_jcbar(const double *__restrict__ cn, double *__restrict__ jcbar,
                                                       FilmGeom G, double scale) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long n = (long long)G.nx * G.ny;
  if (i >= n) return;
  const int p = (int)(i % G.nx), q = (int)(i / G.nx);
  const long long r0 = (long long)q * G.nx, r1 = (long long)wrap(q + 1, G.ny) * G.nx;
  const int p1 = wrap(p + 1, G.nx);
  jcbar[i] = 0.25 * scale * (cn[r0 + p] + cn[r0 + p1] + cn[r1 + p] + cn[r1 + p1]);
}

__global__ void __launch_bounds__(64) vjp_gate_k(const IterState *__restrict__ it, IterState *__restrict__ gate) {
  if (threadIdx.x == 0) {
    *gate = IterState{};
    gate->C = it->C;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) film_out(const T *__restrict__ Gm, double *__restrict__ out, long long n,
                                                const IterState *__restrict__ it) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = (double)Gm[i] - it->C;
}

// Final evaluation of a MAG_MIXED_FINAL64 right-hand side.  gate->done is
// the skip flag of its kernels; dh_e/dt and 1/#out are copied from the
// iteration state.
// decide = 0 (stop test, or a fixed count of one): it runs once the float
//   iteration has stopped after at least one evaluation (a stop, the count
//   reached, or a non-finite residual); the launches of an unfinished block
//   of iterations return at once.
// decide = 1 (fixed count of two or more): the float iteration has skipped
//   its last evaluation, and this one takes the decision in its place; it
//   runs unless the iteration has already stopped (a non-finite residual).
// Either way nothing runs in a step that has reached its end time.
__global__ void __launch_bounds__(64) final64_gate_k(const IterState *__restrict__ it, IterState *__restrict__ gate,
                                                     int decide) {
  if (threadIdx.x == 0) {
    gate->done = decide ? (it->done ? 1 : 0) : ((it->done && it->iters > 0) ? 0 : 1);
    gate->hde = it->hde;
    gate->inv_nout = it->inv_nout;
  }
}

// The decision after the final evaluation at a fixed count: residual mean of
// |gdot| over free space from the per-block sums, the count, done (2 for a
// non-finite residual, which also sets the sticky failure flag).
__global__ void __launch_bounds__(64) final64_decide_k(const double *__restrict__ part, int np,
                                                       IterState *__restrict__ it, IterState *mirror,
                                                       const IterState *__restrict__ gate, int iters) {
  if (gate->done) return;
  const double r = parts_sum(part, np) * gate->inv_nout;
  if (threadIdx.x == 0) {
    const int done = isfinite(r) ? 1 : 2;
    it->r = r;
    it->iters = iters;
    it->done = done;
    if (done == 2) it->fail = 1;
    *mirror = *it;
  }
}

__global__ void __launch_bounds__(256) film_current(const double *__restrict__ g, double *__restrict__ j, int nx,
                                                    int ny, double idx, double idy) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long n = (long long)nx * ny;
  if (i >= n) return;
  const int p = (int)(i % nx), q = (int)(i / nx);
  const double g0 = g[i];
  j[i] = (g[(long long)wrap(q + 1, ny) * nx + p] - g0) * idy;
  j[i + n] = -(g[(long long)q * nx + wrap(p + 1, nx)] - g0) * idx;
}

__global__ void __launch_bounds__(256) sum_blocks(const double *__restrict__ x, long long n,
                                                  double *__restrict__ part) {
  __shared__ double red[4];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const double s = block_total<256>(i < n ? x[i] : 0.0, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Per-block sums of x over kSumWideThreads * kSumWideNpt consecutive entries
// (512 blocks at 2048^2, few enough for a consuming pass to add them itself);
// a thread's loads are issued together, its values added in index order.
constexpr int kSumWideThreads = 1024;
constexpr int kSumWideNpt = 8;
__global__ void __launch_bounds__(kSumWideThreads) sum_wide(const double *__restrict__ x, long long n,
                                                           double *__restrict__ part) {
  __shared__ double red[kSumWideThreads / 64];
  const long long i0 = (long long)blockIdx.x * (kSumWideThreads * kSumWideNpt) + threadIdx.x;
  double v[kSumWideNpt];
#pragma unroll
  for (int k = 0; k < kSumWideNpt; ++k) {
    const long long i = i0 + (long long)k * kSumWideThreads;
    v[k] = i < n ? x[i] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kSumWideNpt; ++k) acc += v[k];
  const double s = block_total<kSumWideThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ------------------------------------------------------------ adjoint stencil
// Transpose of g -> dh_in (eqs. (2), (3), (9)).  For the x-edge (p, q+1/2)
// and the y-edge (p+1/2, q) of node (p, q): the cotangent of e from the
// film-node cotangent hbar = (mu - C) on inside nodes, then the partials of
// e = rho(|j|) j: with s = |j| = sqrt(j_own^2 + oth^2),
//   de/dj_own = rho (1 + (n-1) j_own^2 / s^2),   de/doth = rho (n-1) j_own oth / s^2,
//   de/djc_edge = -n e / jc_edge   (superconducting edges; rho_out elsewhere).
// Stored per edge (double): ebar de/dj_own, ebar de/doth, ebar de/djc.
// gv(pp, qq), mv(pp, qq), jv(pp, qq): g at node (pp, qq), material and jc of
// cell (pp, qq); coordinates not wrapped.
template <typename T, typename GV, typename MV, typename JV>
__device__ __forceinline__ void film_edge_vjp(GV gv, MV mv, JV jv, const FilmGeom &G, const FilmLaw &law, int p,
                                              int q, int orient, double ebar, double *own, double *oth_bar,
                                              double *jc_bar) {
  auto jxv = [&](int pp, int qq) { return (gv(pp, qq + 1) - gv(pp, qq)) * G.idy; };
  auto jyv = [&](int pp, int qq) { return -(gv(pp + 1, qq) - gv(pp, qq)) * G.idx; };
  double jo, oth;
  int p1, q1;   // the other cell of the edge
  if (orient == 0) {
    jo = jxv(p, q);
    oth = 0.25 * (jyv(p - 1, q) + jyv(p, q) + jyv(p - 1, q + 1) + jyv(p, q + 1));
    p1 = p - 1;
    q1 = q;
  } else {
    jo = jyv(p, q);
    oth = 0.25 * (jxv(p, q - 1) + jxv(p, q) + jxv(p + 1, q - 1) + jxv(p + 1, q));
    p1 = p;
    q1 = q - 1;
  }
  if (mv(p, q) == 1 && mv(p1, q1) == 1) {
    const T jt = (T)jo, ot = (T)oth;
    const T s = sqrt(jt * jt + ot * ot);
    const T jce = law.has_jc ? (T)0.5 * (jv(p, q) + jv(p1, q1)) : (T)law.jc0;
    const T nm1 = (T)law.nm1;
    T a, b;
    if (s > (T)0) {
      const T rho = film_rho(s, jce, (T)law.e0, nm1, (T)law.lmax);
      const T is2 = (T)1 / (s * s);
      a = rho * ((T)1 + nm1 * jt * jt * is2);
      b = rho * nm1 * jt * ot * is2;
      *jc_bar = ebar * (double)(-(nm1 + (T)1) * rho * jt / jce);
    } else {
      a = nm1 == (T)0 ? (T)law.e0 / jce : (T)0;
      b = (T)0;
      *jc_bar = 0.0;
    }
    *own = ebar * (double)a;
    *oth_bar = ebar * (double)b;
  } else {
    *own = ebar * law.rho_out;
    *oth_bar = 0.0;
    *jc_bar = 0.0;
  }
}

// Fused stencil transpose on a kVjpTile^2 tile of nodes: g (two-node halo)
// and the film-node cotangent hbar = mu - C (one node beyond the far sides)
// are staged in LDS; the edge terms of the x- and y-edge of every node of the
// tile and a one-node halo are computed into LDS (edges whose cotangent is 0,
// all of them away from the film, are skipped); then, per node, the
// edge-current cotangents (own part plus a quarter of the neighbour-mean parts
// of the four other-orientation edges that average this edge into their |j|),
// g_bar by the transpose of eq. (2), and the cell jc_bar from its four edges
// (edge jc = mean of two cells).
constexpr int kVjpTile = 16;

template <typename T>
__global__ void __launch_bounds__(kVjpTile * kVjpTile)
    film_vjp_stencil(const double *__restrict__ g, const uint8_t *__restrict__ mat,
                     const uint8_t *__restrict__ flags, const T *__restrict__ jc, const T *__restrict__ mu,
                     FilmGeom G, FilmLaw law, double *__restrict__ gbar, double *__restrict__ jcbar, double jc0,
                     const IterState *__restrict__ it) {
  constexpr int B = kVjpTile, NT = B * B;
  constexpr int GW = B + 4;   // g on [p0-2, p0+B+2)
  constexpr int HW = B + 3;   // hbar on [p0-1, p0+B+2)
  constexpr int EW = B + 2;   // edge terms on [p0-1, p0+B+1)
  __shared__ double gs[GW * GW];
  __shared__ double hs[HW * HW];
  __shared__ T es[6][EW * EW];   // own_x, oth_x, own_y, oth_y, jc_x, jc_y
  const int p0 = blockIdx.x * B, q0 = blockIdx.y * B;
  const double C = it->C;
  // staging loads issued together (one round trip), then stored
  constexpr int NG = (GW * GW + NT - 1) / NT, NH = (HW * HW + NT - 1) / NT;
  double gl[NG];
  uint8_t fh[NH];
  T muh[NH];
#pragma unroll
  for (int u = 0; u < NG; ++u) {
    const int k = threadIdx.x + u * NT, kc = k < GW * GW ? k : 0;
    gl[u] = g[(long long)wrap(q0 - 2 + kc / GW, G.ny) * G.nx + wrap(p0 - 2 + kc % GW, G.nx)];
  }
#pragma unroll
  for (int u = 0; u < NH; ++u) {
    const int k = threadIdx.x + u * NT, kc = k < HW * HW ? k : 0;
    const long long idx = (long long)wrap(q0 - 1 + kc / HW, G.ny) * G.nx + wrap(p0 - 1 + kc % HW, G.nx);
    fh[u] = flags[idx];
    muh[u] = mu[idx];
  }
#pragma unroll
  for (int u = 0; u < NG; ++u)
    if (threadIdx.x + u * NT < GW * GW) gs[threadIdx.x + u * NT] = gl[u];
#pragma unroll
  for (int u = 0; u < NH; ++u)
    if (threadIdx.x + u * NT < HW * HW) hs[threadIdx.x + u * NT] = (fh[u] & 1) ? (double)muh[u] - C : 0.0;
  __syncthreads();
  // material and jc are read from memory only for edges next to the film
  auto gv = [&](int pp, int qq) { return gs[(qq - q0 + 2) * GW + (pp - p0 + 2)]; };
  auto cell = [&](int pp, int qq) { return (long long)wrap(qq, G.ny) * G.nx + wrap(pp, G.nx); };
  auto mv = [&](int pp, int qq) { return mat[cell(pp, qq)]; };
  auto jv = [&](int pp, int qq) { return jc[cell(pp, qq)]; };
  auto hb = [&](int pp, int qq) { return hs[(qq - q0 + 1) * HW + (pp - p0 + 1)]; };
  for (int k = threadIdx.x; k < EW * EW; k += NT) {
    const int p = p0 - 1 + k % EW, q = q0 - 1 + k / EW;
    // dh(p,q) = -[(e_y(p,q) - e_y(p-1,q))/dx - (e_x(p,q) - e_x(p,q-1))/dy]
    const double h0 = hb(p, q);
    const double ebx = (h0 - hb(p, q + 1)) * G.idy;
    const double eby = (hb(p + 1, q) - h0) * G.idx;
    double o = 0.0, b = 0.0, cj = 0.0;
    if (ebx != 0.0) film_edge_vjp<T>(gv, mv, jv, G, law, p, q, 0, ebx, &o, &b, &cj);
    es[0][k] = (T)o;
    es[1][k] = (T)b;
    es[4][k] = (T)cj;
    o = b = cj = 0.0;
    if (eby != 0.0) film_edge_vjp<T>(gv, mv, jv, G, law, p, q, 1, eby, &o, &b, &cj);
    es[2][k] = (T)o;
    es[3][k] = (T)b;
    es[5][k] = (T)cj;
  }
  __syncthreads();
  const int p = p0 + threadIdx.x % B, q = q0 + threadIdx.x / B;
  auto E = [&](int pl, int pp, int qq) { return (double)es[pl][(qq - q0 + 1) * EW + (pp - p0 + 1)]; };
  // x-edge (pp, qq) is averaged into the y-edges (pp, qq), (pp, qq+1), (pp-1, qq), (pp-1, qq+1)
  auto jbx = [&](int pp, int qq) {
    return E(0, pp, qq) + 0.25 * (E(3, pp, qq) + E(3, pp, qq + 1) + E(3, pp - 1, qq) + E(3, pp - 1, qq + 1));
  };
  // y-edge (pp, qq) is averaged into the x-edges (pp, qq), (pp+1, qq), (pp, qq-1), (pp+1, qq-1)
  auto jby = [&](int pp, int qq) {
    return E(2, pp, qq) + 0.25 * (E(1, pp, qq) + E(1, pp + 1, qq) + E(1, pp, qq - 1) + E(1, pp + 1, qq - 1));
  };
  const long long i = (long long)q * G.nx + p;
  // j_x(p,q) = (g(p,q+1) - g(p,q))/dy,  j_y(p,q) = -(g(p+1,q) - g(p,q))/dx
  gbar[i] = (jbx(p, q - 1) - jbx(p, q)) * G.idy + (jby(p, q) - jby(p - 1, q)) * G.idx;
  if (jcbar) jcbar[i] = jc0 * 0.5 * (E(4, p, q) + E(4, p + 1, q) + E(5, p, q) + E(5, p, q + 1));
}

}  // namespace

// ================================================================= host side
static FilmGeom fgeom(mag_ctx *c) {
  FilmGeom G;
  G.nx = c->n[0];
  G.ny = c->n[1];
  G.kx = c->kx;
  G.idx = 1.0 / c->d[0];
  G.idy = 1.0 / c->d[1];
  return G;
}

#define FILM_SWITCH_M(M_, ...)                            \
  switch (M_) {                                            \
    case 8: { constexpr int MM = 8; __VA_ARGS__; } break;         \
    case 24: { constexpr int MM = 24; __VA_ARGS__; } break;       \
    case 48: { constexpr int MM = 48; __VA_ARGS__; } break;       \
    case 96: { constexpr int MM = 96; __VA_ARGS__; } break;       \
    case 192: { constexpr int MM = 192; __VA_ARGS__; } break;     \
    case 384: { constexpr int MM = 384; __VA_ARGS__; } break;     \
    case 16: { constexpr int MM = 16; __VA_ARGS__; } break;       \
    case 32: { constexpr int MM = 32; __VA_ARGS__; } break;       \
    case 64: { constexpr int MM = 64; __VA_ARGS__; } break;       \
    case 128: { constexpr int MM = 128; __VA_ARGS__; } break;     \
    case 256: { constexpr int MM = 256; __VA_ARGS__; } break;     \
    case 512: { constexpr int MM = 512; __VA_ARGS__; } break;     \
    case 1024: { constexpr int MM = 1024; __VA_ARGS__; } break;   \
    default: return set_error(c, MAG_E_ARG, "unsupported length %d", M_); \
  }

#define FILM_SWITCH_N(N_, ...)                            \
  switch (N_) {                                            \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;       \
    case 48: { constexpr int NN = 48; __VA_ARGS__; } break;       \
    case 96: { constexpr int NN = 96; __VA_ARGS__; } break;       \
    case 192: { constexpr int NN = 192; __VA_ARGS__; } break;     \
    case 384: { constexpr int NN = 384; __VA_ARGS__; } break;     \
    case 768: { constexpr int NN = 768; __VA_ARGS__; } break;     \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;       \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;       \
    case 128: { constexpr int NN = 128; __VA_ARGS__; } break;     \
    case 256: { constexpr int NN = 256; __VA_ARGS__; } break;     \
    case 512: { constexpr int NN = 512; __VA_ARGS__; } break;     \
    case 1024: { constexpr int NN = 1024; __VA_ARGS__; } break;   \
    case 2048: { constexpr int NN = 2048; __VA_ARGS__; } break;   \
    default: return set_error(c, MAG_E_ARG, "unsupported length %d", N_); \
  }

template <typename T>
struct FilmPtrs {
  T *H, *G;
  cx<T> *S;
  const cx<T> *twM, *twY, *twN;
  const double *k2x, *k2y;
  const double *kxs, *kys;   // signed wavenumbers, Nyquist set to 0 (spectral derivatives)
  T *w1, *w2;   // K1 1_out and K2 1_out (w2: NaN on film nodes)
  T *w1f;       // K1 1_out with NaN on film nodes
};

// The double pointers of a MAG_MIXED_FINAL64 context are those of its final
// evaluation: the spectrum buffer (allocated for double), the double
// twiddles and w1 in double; it has no double iterate, G, w2 or w1f.
template <typename T>
static FilmPtrs<T> fptrs(mag_ctx *c) {
  FilmPtrs<T> f;
  const bool final64 = sizeof(T) == 8 && c->prec != MAG_FP64;
  f.H = final64 ? nullptr : reinterpret_cast<T *>(c->d_H);
  f.G = final64 ? nullptr : reinterpret_cast<T *>(c->d_G);
  f.S = reinterpret_cast<cx<T> *>(c->d_S);
  const cx<T> *tw = reinterpret_cast<const cx<T> *>(final64 ? c->d_tw64 : c->d_tw);
  f.twM = tw + c->tw_off[0];
  f.twY = tw + c->tw_off[1];
  f.twN = tw + c->tw_off[3];
  f.k2x = c->d_sym + c->sym_off[0];
  f.k2y = c->d_sym + c->sym_off[1];
  f.kxs = c->d_sym + c->sym_off[2];
  f.kys = c->d_sym + c->sym_off[3];
  f.w1 = reinterpret_cast<T *>(final64 ? c->d_w64 : c->d_w);
  f.w2 = (f.w1 && !final64) ? f.w1 + c->nnode : nullptr;
  f.w1f = (f.w1 && !final64) ? f.w1 + 2 * c->nnode : nullptr;
  return f;
}

// Number of row blocks (partial sums per row pass) of the current grid.
template <typename T>
static int film_row_blocks(mag_ctx *c) {
  const FilmGeom G = fgeom(c);
  int nb = 0;
  FILM_SWITCH_M(G.nx / 2, { nb = (G.ny + FilmRowShape<MM, T>::P - 1) / FilmRowShape<MM, T>::P; });
  return nb;
}

// Regions of d_part used by the passes of one iteration (nb row blocks each).
struct PartRegions {
  double *C, *R, *A, *X, *F;
  int nb;
};

static int film_stencil_blocks(mag_ctx *c) {
  return (int)((c->nnode + kStencilThreads * kStencilNpt - 1) / (kStencilThreads * kStencilNpt));
}

template <typename T>
static PartRegions film_regions(mag_ctx *c) {
  PartRegions r;
  r.nb = film_row_blocks<T>(c);
  r.C = c->d_part;
  r.R = c->d_part + r.nb;
  r.A = c->d_part + 2 * r.nb;
  r.X = c->d_part + 3 * r.nb;   // stencil partials (film_stencil_blocks of them)
  r.F = r.X + film_stencil_blocks(c);
  return r;
}

static Parts parts(const double *in, int nin, double *out, double *out2 = nullptr, int iter = 0) {
  Parts p;
  p.in = in;
  p.nin = nin;
  p.out = out;
  p.out2 = out2;
  p.iter = iter;
  return p;
}

template <typename T, int MODE>
static int film_fwd(mag_ctx *c, T *X, const double *xd, double hde, Parts pp, int kid, IterState *its = nullptr,
                    const float *xf = nullptr, cx<T> *dst = nullptr) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  ProfLaunch ps(c, kid);
  FILM_SWITCH_M(G.nx / 2, {
    using RS = FilmRowShape<MM, T>;
    const int nblk = (G.ny + RS::P - 1) / RS::P;
    MAG_TIMED_LAUNCH(ps, (film_rows_fwd<T, MM, MODE>), dim3(nblk), dim3(RS::THREADS), 0, c->stream, X, xd,
                       c->d_flags, dst ? dst : f.S, f.twM, f.twN, G, hde, pp, its ? its : c->d_it,
                       ((MODE == 0 || MODE == 3 || MODE == 5) && pp.out) ? (const T *)f.w1 : (const T *)nullptr, xf);
  });
  return MAG_OK;
}

template <typename T, int MODE>
static int film_inv(mag_ctx *c, T *X, double *xd, double hde, Parts pp, int kid, IterState *its = nullptr,
                    const cx<T> *src = nullptr) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  ProfLaunch ps(c, kid);
  FILM_SWITCH_M(G.nx / 2, {
    using RS = FilmRowShape<MM, T>;
    const int nblk = (G.ny + RS::P - 1) / RS::P;
    MAG_TIMED_LAUNCH(ps, (film_rows_inv<T, MM, MODE>), dim3(nblk), dim3(RS::THREADS), 0, c->stream, X, xd,
                       c->d_flags, src ? src : f.S, f.twM, f.twN, G, hde, c->lambda, pp, its ? its : c->d_it);
  });
  return MAG_OK;
}

template <typename T, int MODE>
static int film_fused(mag_ctx *c, T *X, const T *w, Parts pp, int kid, int keep = 1, double *out = nullptr) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  ProfLaunch ps(c, kid);
  FILM_SWITCH_M(G.nx / 2, {
    using RS = FilmRowShape<MM, T>;
    const int nblk = (G.ny + RS::P - 1) / RS::P;
    MAG_TIMED_LAUNCH(ps, (film_rows_fused<T, MM, MODE>), dim3(nblk), dim3(RS::THREADS), 0, c->stream, X, c->d_flags,
                       f.S, w, f.twM, f.twN, G, c->lambda, pp, c->d_it, keep, out);
  });
  return MAG_OK;
}

template <typename T, int MODE>
static int film_adj(mag_ctx *c, T *X, const T *w, AdjParts pp) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  ProfLaunch ps(c, K_VJP);
  FILM_SWITCH_M(G.nx / 2, {
    using RS = FilmRowShape<MM, T>;
    const int nblk = (G.ny + RS::P - 1) / RS::P;
    MAG_TIMED_LAUNCH(ps, (film_rows_adj<T, MM, MODE>), dim3(nblk), dim3(RS::THREADS), 0, c->stream, X, c->d_flags,
                       f.S, w, f.twM, f.twN, G, c->lambda, pp, c->d_it);
  });
  return MAG_OK;
}

// which = 0: 2/|k|; which = 1: |k|/2.  pp.in != NULL: take the stop decision
// of evaluation pp.iter from the residual sums pp.in first.
template <typename T>
static int film_col(mag_ctx *c, int which, Parts pp = parts(nullptr, 0, nullptr), IterState *its = nullptr,
                    int kid = K_FILM_COLS) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  ProfLaunch ps(c, kid);
  FILM_SWITCH_N(G.ny, {
    using CS = FilmColShape<NN, T>;
    const int nblk = (G.kx - 1 + CS::P - 1) / CS::P;   // the kx = 0 and kx = M columns share a pencil
    MAG_TIMED_LAUNCH(ps, (film_cols<T, NN>), dim3(nblk), dim3(CS::THREADS), 0, c->stream, f.S, G.kx, f.k2x, f.k2y,
                       1.0 / (double)c->nnode, which, f.twY, pp, its ? its : c->d_it, c->h_it);
  });
  return MAG_OK;
}

// Column pass of the spectral form (OP 0: gradient of g, OP 1: curl of e).
template <typename T, int OP>
static int film_col_spec(mag_ctx *c, int kid, cx<T> *Sa = nullptr, cx<T> *Sb = nullptr,
                         const IterState *its = nullptr) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  if (!c->d_filt) return set_error(c, MAG_E_STATE, "spectral form without its filter tables");
  ProfLaunch ps(c, kid);
  FILM_SWITCH_N(G.ny, {
    using CS = FilmColShape<NN, T>;
    const int nblk = (G.kx - 1 + CS::P - 1) / CS::P;
    MAG_TIMED_LAUNCH(ps, (film_cols_spec<T, NN, OP>), dim3(nblk), dim3(CS::THREADS), 0, c->stream, Sa ? Sa : f.S,
                     Sb ? Sb : reinterpret_cast<cx<T> *>(c->d_S2), G.kx, (const double *)c->d_filt,
                     (const double *)c->d_filt + G.kx, f.kxs, f.kys, 1.0 / (double)c->nnode, f.twY,
                     its ? its : (const IterState *)c->d_it);
  });
  return MAG_OK;
}

// The spectrum of g in S becomes the spectra of j_x (S) and j_y (S2).
template <typename T>
static int film_spectral_current(mag_ctx *c, const double *state, int kid) {
  int rc;
  if ((rc = film_fwd<T, 2>(c, nullptr, state, 0.0, parts(nullptr, 0, nullptr), kid))) return rc;
  return film_col_spec<T, 0>(c, kid);
}

static FilmLaw film_law(const mag_ctx *c);

// The film values of dh_z/dt in the spectral form, written into H at the
// film nodes: j from g, e = rho(|j|) j at the nodes, d_y e_x - d_x e_y.
template <typename T>
static int film_spectral_film_values(mag_ctx *c, const double *state) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  const FilmLaw law = film_law(c);
  if (!c->d_S2 || !c->d_jcn) return set_error(c, MAG_E_STATE, "spectral form without its buffers");
  if (c->jcn_gen != c->gen) {
    // the per-node jc follows the material and the jc map
    ProfScope ps(c, K_FILM_SPECTRAL);
    hipLaunchKernelGGL((film_node_jc<T>), dim3((unsigned)((c->nnode + 255) / 256)), dim3(256), 0, c->stream,
                       c->d_mat, reinterpret_cast<const T *>(c->d_jc), reinterpret_cast<T *>(c->d_jcn), G, law);
    MAG_HIP(c, hipGetLastError());
    c->jcn_gen = c->gen;
  }
  int rc;
  if ((rc = film_spectral_current<T>(c, state, K_FILM_SPECTRAL))) return rc;
  {
    ProfLaunch ps(c, K_FILM_SPECTRAL);
    FILM_SWITCH_M(G.nx / 2, {
      using RS = FilmRowShape<MM, T>;
      const int nblk = (G.ny + RS::P - 1) / RS::P;
      MAG_TIMED_LAUNCH(ps, (film_rows_node_e<T, MM>), dim3(nblk), dim3(RS::THREADS), 0, c->stream, f.S,
                       reinterpret_cast<cx<T> *>(c->d_S2), reinterpret_cast<const T *>(c->d_jcn), f.twM, f.twN, G,
                       law, (const IterState *)c->d_it);
    });
  }
  if ((rc = film_col_spec<T, 1>(c, K_FILM_SPECTRAL))) return rc;
  return film_inv<T, 7>(c, f.H, nullptr, 0.0, parts(nullptr, 0, nullptr), K_FILM_SPECTRAL);
}

// One inner iteration i (evaluation i of (11), then the update (12)), four
// passes over the spectrum:
//   (i = 0: rows_fwd  H: shift A^0 from the stencil sums, R2C of H - dh_e,
//                     sums of w1 (H - dh_e))
//   cols       2/|k|
//   fused 6    G, C from the w1 sums, gdot = G - C, sums of |gdot| and of
//              w2 gdot over free space, R2C of gdot on free space
//   cols       stop decision on the |gdot| sums, then |k|/2
//   fused 7    H <- H - lambda V - A on free space (A from the w2 sums),
//              sums of w1 (H - dh_e), R2C of H - dh_e (next iteration)
// At a fixed count the last evaluation writes gdot to `out` itself and the
// update that no evaluation would use is not launched (the column pass still
// records the residual and the count); otherwise G is kept for film_out.
// MAG_MIXED_FINAL64 at a fixed count of two or more: the last evaluation of
// (11) is the double one of film_final64, which also takes the decision.
static bool final64_decides(const mag_ctx *c) { return c->prec == MAG_MIXED_FINAL64 && c->fixed_iters >= 2; }

template <typename T>
static int film_iteration(mag_ctx *c, double hde, int i, int nbs, double *out) {
  if (final64_decides(c) && i == c->fixed_iters - 1) return MAG_OK;
  const FilmPtrs<T> f = fptrs<T>(c);
  const PartRegions pr = film_regions<T>(c);
  int rc;
  if (i == 0 && (rc = film_fwd<T, 0>(c, f.H, nullptr, hde, parts(pr.X, nbs, pr.C, pr.F), K_FILM_ROWS_FWD_H)))
    return rc;
  if ((rc = film_col<T>(c, 0))) return rc;
  const bool last_fixed = c->fixed_iters > 0 && i == c->fixed_iters - 1;
  if ((rc = film_fused<T, 6>(c, f.G, f.w2, parts(pr.C, pr.nb, pr.R, pr.A), K_FILM_ROWS_INV_G,
                             c->fixed_iters <= 0 ? 1 : 0, last_fixed ? out : nullptr)))
    return rc;
  if ((rc = film_col<T>(c, 1, parts(pr.R, pr.nb, nullptr, nullptr, i)))) return rc;
  if (last_fixed) return MAG_OK;
  return film_fused<T, 7>(c, f.H, f.w1f, parts(pr.A, pr.nb, pr.C, pr.F), K_FILM_ROWS_INV_UPD);
}

// The returned dg/dt of a MAG_MIXED_FINAL64 right-hand side: (11) once more
// in double from the float iterate H the iteration stopped at,
// gdot = K1 (H - dh_e) - C, with C the free-space mean of K1 (H - dh_e)
// (Sec. 2.2) taken as <w1, H - dh_e> / #out.  Three passes: R2C rows of
// H - dh_e with the w1 sums, the 2/|k| column pass, C2R rows writing
// gdot to out.  At a fixed count of two or more it stands in for the float
// iteration's last evaluation and takes the decision (final64_decide_k).
// The double spectrum reuses the spectrum buffer, which the float iteration
// no longer needs.  Enqueued only.
static int film_final64(mag_ctx *c, double *out) {
  const PartRegions pr = film_regions<float>(c);
  const int nb64 = film_row_blocks<double>(c);
  double *part = pr.F + pr.nb;   // after the regions of the float iteration: w1 sums
  double *rpart = part + nb64;   // |gdot| sums
  if (rpart + nb64 > c->d_part + c->npart) return set_error(c, MAG_E_STATE, "partial-sum buffer too small");
  const int decide = final64_decides(c) ? 1 : 0;
  {
    ProfScope ps(c, K_FILM_FINAL64);
    hipLaunchKernelGGL(final64_gate_k, dim3(1), dim3(64), 0, c->stream, c->d_it, c->d_it64, decide);
  }
  int rc;
  if ((rc = film_fwd<double, 3>(c, nullptr, nullptr, 0.0, parts(nullptr, 0, part), K_FILM_FINAL64, c->d_it64,
                                reinterpret_cast<const float *>(c->d_H))))
    return rc;
  if ((rc = film_col<double>(c, 0, parts(nullptr, 0, nullptr), c->d_it64, K_FILM_FINAL64))) return rc;
  if ((rc = film_inv<double, 6>(c, nullptr, out, 0.0, parts(part, nb64, decide ? rpart : nullptr), K_FILM_FINAL64,
                                c->d_it64)))
    return rc;
  if (decide) {
    ProfScope ps(c, K_FILM_FINAL64);
    hipLaunchKernelGGL(final64_decide_k, dim3(1), dim3(64), 0, c->stream, (const double *)rpart, nb64, c->d_it,
                       c->h_it, (const IterState *)c->d_it64, c->fixed_iters);
  }
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

static FilmLaw film_law(const mag_ctx *c) {
  FilmLaw law;
  law.e0 = c->e0;
  law.nm1 = c->nexp - 1.0;
  law.rho_out = c->rho_out;
  law.lmax = std::log(1e30) / (c->nexp - 1.0 > 1e-12 ? c->nexp - 1.0 : 1e-12);
  law.jc0 = c->jc0;
  law.has_jc = c->has_jc_map ? 1 : 0;
  return law;
}

// The film values of dh_z/dt (eq. (9)), the free-space start and the partial
// sums of H - dh_e: the staggered stencil, or in the spectral form (Sec.
// 2.2) the film values from the spectral passes, then the same stencil
// kernel for the free space and the sums.
template <typename T>
static int film_stencil_pass(mag_ctx *c, const double *state, int warm) {
  FilmPtrs<T> f = fptrs<T>(c);
  const FilmGeom G = fgeom(c);
  const FilmLaw law = film_law(c);
  const int nbs = film_stencil_blocks(c);
  if (c->deriv == 0) {
    ProfLaunch ps(c, K_FILM_STENCIL);
    const bool p2 = !(G.nx & (G.nx - 1)) && !(G.ny & (G.ny - 1));
    if (p2)
      MAG_TIMED_LAUNCH(ps, (film_stencil<T, false, true>), dim3(nbs), dim3(kStencilThreads), 0, c->stream, state,
                       c->d_mat, c->d_flags, reinterpret_cast<const T *>(c->d_jc), f.H, G, law, c->d_it, warm,
                       film_regions<T>(c).X);
    else
      MAG_TIMED_LAUNCH(ps, (film_stencil<T, false, false>), dim3(nbs), dim3(kStencilThreads), 0, c->stream, state,
                       c->d_mat, c->d_flags, reinterpret_cast<const T *>(c->d_jc), f.H, G, law, c->d_it, warm,
                       film_regions<T>(c).X);
    return MAG_OK;
  }
  if (int rc = film_spectral_film_values<T>(c, state)) return rc;
  ProfLaunch ps(c, K_FILM_STENCIL);
  MAG_TIMED_LAUNCH(ps, (film_stencil<T, true, false>), dim3(nbs), dim3(kStencilThreads), 0, c->stream, state, c->d_mat,
                   c->d_flags, reinterpret_cast<const T *>(c->d_jc), f.H, G, law, c->d_it, warm, film_regions<T>(c).X);
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

// The right-hand side with a fixed inner count, enqueued only: the iteration
// state (dh_e/dt included) has been set on the device by the caller, the
// free-space iterate holds the warm start, and the last evaluation writes
// `out`.  No host synchronisation and no host-side decision, so the launches
// can be captured in a graph.
template <typename T>
static int film_rhs_enqueue_t(mag_ctx *c, const double *state, double *out) {
  const int nbs = film_stencil_blocks(c);
  if (int rc = film_stencil_pass<T>(c, state, 1)) return rc;
  for (int i = 0; i < c->fixed_iters; ++i) {
    c->cur_iter = i;
    if (int rc = film_iteration<T>(c, 0.0, i, nbs, out)) return rc;
  }
  c->cur_iter = -1;
  if (c->prec == MAG_MIXED_FINAL64)
    if (int rc = film_final64(c, out)) return rc;
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int film_rhs_enqueue(mag_ctx *c, const double *state, double *out) {
  if (c->fixed_iters <= 0) return set_error(c, MAG_E_STATE, "an enqueued right-hand side needs a fixed count");
  return c->prec == MAG_FP64 ? film_rhs_enqueue_t<double>(c, state, out) : film_rhs_enqueue_t<float>(c, state, out);
}

template <typename T>
static int film_rhs_t(mag_ctx *c, const double *state, double t, double *out, int *n_inner) {
  double hd[3];
  field_hdot(c, t, hd);
  const double hde = hd[2];
  const FilmGeom G = fgeom(c);
  FilmPtrs<T> f = fptrs<T>(c);
  IterState is{};
  is.fixed = c->fixed_iters;
  is.thr = c->tol * (std::fabs(hde) > 1.0 ? std::fabs(hde) : 1.0);
  is.inv_nout = c->nout > 0 ? 1.0 / (double)c->nout : 0.0;
  is.hde = hde;
  if (int rc0 = run_iter_init(c, is)) return rc0;
  const FilmLaw law = film_law(c);
  const long long n = c->nnode;
  const int nbs = film_stencil_blocks(c);
  int rc = film_stencil_pass<T>(c, state, c->warm_valid ? 1 : 0);
  if (rc) return rc;
  MAG_HIP(c, hipGetLastError());
  const int kmax = c->fixed_iters > 0 ? c->fixed_iters : c->max_inner;
  int issued = 0;
  int block = c->fixed_iters > 0 ? c->fixed_iters : (c->last_iters > 0 ? c->last_iters : 1);
  bool done = false;
  while (issued < kmax) {
    const int k = block < kmax - issued ? block : kmax - issued;
    for (int i = 0; i < k; ++i) {
      c->cur_iter = issued + i;
      if ((rc = film_iteration<T>(c, hde, issued + i, nbs, out))) return rc;
    }
    c->cur_iter = -1;
    issued += k;
    // out = G - C, enqueued before the poll: right whenever this block ends
    // the iteration (it is enqueued again after a further block otherwise);
    // at a fixed count the last evaluation has written it already.  The
    // final double evaluation runs only if the block ends the iteration.
    if (c->prec == MAG_MIXED_FINAL64) {
      if ((rc = film_final64(c, out))) return rc;
    } else if (c->fixed_iters <= 0) {
      ProfScope ps(c, K_MISC);
      hipLaunchKernelGGL((film_out<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, f.G, out, n,
                         c->d_it);
    }
    MAG_HIP(c, hipGetLastError());
    if (c->rhs_async && issued >= kmax) {
      // fixed count, no host scalar wanted: return without waiting; the
      // status is checked by mag_rhs_status
      c->async_pending = true;
      c->last_iters = kmax;
      c->warm_valid = true;
      if (n_inner) *n_inner = kmax;
      return MAG_OK;
    }
    MAG_HIP(c, hipStreamSynchronize(c->stream));
    if (c->h_it->done) {
      done = true;
      break;
    }
    block = 1;
  }
  const int used = c->h_it->iters;
  prof_drop_after(c, used);
  if (n_inner) *n_inner = used;
  if (!done) {
    c->warm_valid = false;
    return set_error(c, MAG_NOT_CONVERGED, "inner iteration not converged after %d iterations (r = %g)", used,
                     c->h_it->r);
  }
  if (!std::isfinite(c->h_it->r) || !std::isfinite(c->h_it->C)) {
    c->warm_valid = false;
    return set_error(c, MAG_E_NUMERIC, "non-finite residual");
  }
  c->last_iters = used;
  c->warm_valid = true;
  return MAG_OK;
}

int film_rhs(mag_ctx *c, const double *state, double t, double *out, int *n_inner) {
  return c->prec == MAG_FP64 ? film_rhs_t<double>(c, state, t, out, n_inner)
                             : film_rhs_t<float>(c, state, t, out, n_inner);
}

template <typename T>
static int film_observe_t(mag_ctx *c, const double *state, double t, double *hz, double *j, double *m) {
  const FilmGeom G = fgeom(c);
  const long long n = c->nnode;
  const int nb = (int)((n + 255) / 256);
  double he[3];
  field_h(c, t, he);
  IterState is{};
  if (int rc0 = run_iter_init(c, is)) return rc0;
  int rc, nblk = 0;
  if (hz) {
    if ((rc = film_fwd<T, 2>(c, nullptr, state, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
    if ((rc = film_col<T>(c, 1))) return rc;
    if ((rc = film_inv<T, 2>(c, nullptr, hz, he[2], parts(nullptr, 0, nullptr), K_MISC))) return rc;
  }
  if (j && c->deriv == 1) {
    // j_x = d_y g and j_y = -d_x g at the nodes (spectral form)
    if ((rc = film_spectral_current<T>(c, state, K_MISC))) return rc;
    if ((rc = film_inv<T, 2>(c, nullptr, j, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
    if ((rc = film_inv<T, 2>(c, nullptr, j + n, 0.0, parts(nullptr, 0, nullptr), K_MISC, nullptr,
                             reinterpret_cast<const cx<T> *>(c->d_S2))))
      return rc;
  }
  ProfScope ps(c, K_MISC);
  if (j && c->deriv == 0)
    hipLaunchKernelGGL(film_current, dim3(nb), dim3(256), 0, c->stream, state, j, G.nx, G.ny, G.idx, G.idy);
  // m_z = sum g dx dy: fixed-order two-level sum
  hipLaunchKernelGGL(sum_blocks, dim3(nb), dim3(256), 0, c->stream, state, n, c->d_part);
  std::vector<double> parts(nb);
  MAG_HIP(c, hipGetLastError());
  MAG_HIP(c, hipMemcpyAsync(parts.data(), c->d_part, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += parts[i];
  m[0] = 0.0;
  m[1] = 0.0;
  m[2] = s * c->d[0] * c->d[1];
  return MAG_OK;
}

int film_observe(mag_ctx *c, const double *state, double t, double *hz, double *j, double *m) {
  return c->prec == MAG_FP64 ? film_observe_t<double>(c, state, t, hz, j, m)
                             : film_observe_t<float>(c, state, t, hz, j, m);
}

// Transpose of g -> h_z (post-processing of Sec. 2.1): the multiplier |k|/2 is
// real and even, so the transpose is the same map without h_e.
template <typename T>
static int film_hz_transpose_t(mag_ctx *c, const double *hz_bar, double *state_bar) {
  IterState is{};
  if (int rc0 = run_iter_init(c, is)) return rc0;
  int rc, nblk = 0;
  if ((rc = film_fwd<T, 2>(c, nullptr, hz_bar, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
  if ((rc = film_col<T>(c, 1))) return rc;
  if ((rc = film_inv<T, 2>(c, nullptr, state_bar, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int film_hz_transpose(mag_ctx *c, const double *hz_bar, double *state_bar) {
  return c->prec == MAG_FP64 ? film_hz_transpose_t<double>(c, hz_bar, state_bar)
                             : film_hz_transpose_t<float>(c, hz_bar, state_bar);
}

// ------------------------------------------------------------------ adjoint
// Vector-Jacobian product of film_rhs: the transposed iteration
//   mu = Q^T ybar;  repeat  nu = S^T mu,  mu = nu - lambda Q^T P_out K2 P_out nu
// (Q^T z = K1 (z - m_out sum_D z), S^T z = z - mean_out z), stopped after the
// forward's fixed count or when mean_out |nu| < tol mean_D |Q^T ybar|, then
// the stencil transpose on the film part of S^T mu.
// Transpose of the spectral form's film values (the film cotangent Mu - C
// from the transposed iteration) to the state and the jc map.  The passes
// run under their own iteration state (the transposed iteration's is done).
template <typename T>
static int film_spectral_vjp(mag_ctx *c, const double *state, const T *Mu, double *gbar, double *jcbar) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  const FilmLaw law = film_law(c);
  if (!c->d_S2 || !c->d_jcn || !c->d_S34 || !c->d_cn || !c->d_itv)
    return set_error(c, MAG_E_STATE, "spectral form without its buffers");
  cx<T> *S = f.S, *S2 = reinterpret_cast<cx<T> *>(c->d_S2);
  cx<T> *S3 = reinterpret_cast<cx<T> *>(c->d_S34), *S4 = S3 + c->nspec;
  IterState *gate = c->d_itv;
  {
    ProfScope ps(c, K_VJP);
    hipLaunchKernelGGL(vjp_gate_k, dim3(1), dim3(64), 0, c->stream, (const IterState *)c->d_it, gate);
    if (c->jcn_gen != c->gen) {
      hipLaunchKernelGGL((film_node_jc<T>), dim3((unsigned)((c->nnode + 255) / 256)), dim3(256), 0, c->stream,
                         c->d_mat, reinterpret_cast<const T *>(c->d_jc), reinterpret_cast<T *>(c->d_jcn), G, law);
      c->jcn_gen = c->gen;
    }
  }
  int rc;
  // the spectra of j_x, j_y (from g) to S3, S4
  if ((rc = film_fwd<T, 2>(c, nullptr, state, 0.0, parts(nullptr, 0, nullptr), K_VJP, gate, nullptr, S3))) return rc;
  if ((rc = film_col_spec<T, 0>(c, K_VJP, S3, S4, gate))) return rc;
  // the spectra of d_y hbar, -d_x hbar (hbar = Mu - C on the film) to S, S2
  if ((rc = film_fwd<T, 6>(c, const_cast<T *>(Mu), nullptr, 0.0, parts(nullptr, 0, nullptr), K_VJP, gate))) return rc;
  if ((rc = film_col_spec<T, 0>(c, K_VJP, S, S2, gate))) return rc;
  {
    ProfLaunch ps(c, K_VJP);
    FILM_SWITCH_M(G.nx / 2, {
      using RS = FilmRowShape<MM, T>;
      const int nblk = (G.ny + RS::P - 1) / RS::P;
      MAG_TIMED_LAUNCH(ps, (film_rows_node_ebar<T, MM>), dim3(nblk), dim3(RS::THREADS), 0, c->stream, S, S2,
                       (const cx<T> *)S3, (const cx<T> *)S4, reinterpret_cast<const T *>(c->d_jcn),
                       jcbar ? c->d_cn : nullptr, f.twM, f.twN, G, law, (const IterState *)gate);
    });
  }
  // g_bar = -(d_y jbar_x - d_x jbar_y)
  if ((rc = film_col_spec<T, 1>(c, K_VJP, S, S2, gate))) return rc;
  if ((rc = film_inv<T, 8>(c, nullptr, gbar, 0.0, parts(nullptr, 0, nullptr), K_VJP, gate))) return rc;
  if (jcbar) {
    ProfScope ps(c, K_VJP);
    hipLaunchKernelGGL(film_cell_jcbar, dim3((unsigned)((c->nnode + 255) / 256)), dim3(256), 0, c->stream,
                       (const double *)c->d_cn, jcbar, G, c->jc0);
  }
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

template <typename T>
static int film_rhs_vjp_t(mag_ctx *c, const double *state, const double *ybar, double *gbar, double *jcbar) {
  const FilmGeom G = fgeom(c);
  const FilmPtrs<T> f = fptrs<T>(c);
  const long long n = c->nnode;
  T *Mu = f.G;   // the forward's G is scratch between calls
  IterState is{};
  is.fixed = c->fixed_iters;
  is.inv_nout = c->nout > 0 ? 1.0 / (double)c->nout : 0.0;
  is.sum0 = c->tol / (double)n;
  int rc;
  if ((rc = run_iter_init(c, is))) return rc;
  // regions of d_part: residual, w2 sums, w1 sums (two, alternating), scale,
  // sums of ybar
  const int pnb = film_row_blocks<T>(c);
  double *Rr = c->d_part, *Rw2 = c->d_part + pnb, *Rw1[2] = {c->d_part + 2 * pnb, c->d_part + 3 * pnb},
         *Rsc = c->d_part + 4 * pnb, *Ry = c->d_part + 5 * pnb;
  const int nyb = (int)((n + kSumWideThreads * kSumWideNpt - 1) / (kSumWideThreads * kSumWideNpt));
  {
    ProfScope ps(c, K_VJP);
    hipLaunchKernelGGL(sum_wide, dim3(nyb), dim3(kSumWideThreads), 0, c->stream, ybar, n, Ry);
  }
  const double inv_nout = is.inv_nout, lam = c->lambda;
  // mu0 = K1 (ybar - A on free space), A = sum_D ybar / #out from the sums
  // above; C0 = <w1, ybar - A 1_out> / #out
  if ((rc = film_fwd<T, 5>(c, nullptr, ybar, 0.0, parts(Ry, nyb, Rw1[0]), K_VJP))) return rc;
  if ((rc = film_col<T>(c, 0))) return rc;
  {
    AdjParts ap{Rw1[0], nullptr, nullptr, pnb, inv_nout, 0.0, Rr, Rw2, Rsc};
    if ((rc = film_adj<T, 8>(c, Mu, f.w2, ap))) return rc;
  }
  // thr = tol mean_D |mu0| (the stop test of a fixed count does not use it)
  if (c->fixed_iters <= 0 && (rc = run_finalize_mean(c, pnb, 2, (int)(Rsc - c->d_part)))) return rc;
  MAG_HIP(c, hipGetLastError());
  const int kmax = c->fixed_iters > 0 ? c->fixed_iters : c->max_inner;
  int issued = 0;
  int block = c->fixed_iters > 0 ? c->fixed_iters : (c->last_iters > 0 ? c->last_iters : 1);
  bool done = false;
  while (issued < kmax) {
    const int k = block < kmax - issued ? block : kmax - issued;
    for (int i = 0; i < k; ++i) {
      const int ii = issued + i;
      c->cur_iter = ii;
      // stop test on |nu|, then |k|/2 of P_out nu
      if ((rc = film_col<T>(c, 1, parts(Rr, pnb, nullptr, nullptr, ii)))) return rc;
      {
        AdjParts ap{nullptr, nullptr, Rw2, pnb, 0.0, 0.0, Rw1[(ii + 1) & 1], nullptr, nullptr};
        if ((rc = film_adj<T, 9>(c, nullptr, f.w1, ap))) return rc;   // z, z - A_z, R2C
      }
      if ((rc = film_col<T>(c, 0))) return rc;                            // 2/|k|
      {
        AdjParts ap{Rw1[(ii + 1) & 1], Rw1[ii & 1], nullptr, pnb, -lam * inv_nout,
                    ii == 0 ? inv_nout : -lam * inv_nout, Rr, Rw2, nullptr};
        if ((rc = film_adj<T, 8>(c, Mu, f.w2, ap))) return rc;
      }
    }
    c->cur_iter = -1;
    issued += k;
    MAG_HIP(c, hipGetLastError());
    MAG_HIP(c, hipStreamSynchronize(c->stream));
    if (c->h_it->done) {
      done = true;
      break;
    }
    block = 1;
  }
  const int used = c->h_it->iters;
  prof_drop_after(c, used);
  if (!done)
    return set_error(c, MAG_NOT_CONVERGED, "transposed iteration not converged after %d iterations (r = %g)", used,
                     c->h_it->r);
  if (!std::isfinite(c->h_it->r) || !std::isfinite(c->h_it->C))
    return set_error(c, MAG_E_NUMERIC, "non-finite value in the transposed iteration");
  FilmLaw law;
  law.e0 = c->e0;
  law.nm1 = c->nexp - 1.0;
  law.rho_out = c->rho_out;
  law.lmax = std::log(1e30) / (c->nexp - 1.0 > 1e-12 ? c->nexp - 1.0 : 1e-12);
  law.jc0 = c->jc0;
  law.has_jc = c->has_jc_map ? 1 : 0;
  if (c->deriv == 1) return film_spectral_vjp<T>(c, state, Mu, gbar, jcbar);
  {
    ProfLaunch ps(c, K_VJP);
    MAG_TIMED_LAUNCH(ps, (film_vjp_stencil<T>), dim3(G.nx / kVjpTile, G.ny / kVjpTile), dim3(kVjpTile * kVjpTile),
                     0, c->stream, state, c->d_mat, c->d_flags, reinterpret_cast<const T *>(c->d_jc), Mu, G, law,
                     gbar, jcbar, c->jc0, c->d_it);
  }
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int film_rhs_vjp(mag_ctx *c, const double *state, double, const double *out_bar, double *state_bar,
                 double *jc_bar) {
  return c->prec == MAG_FP64 ? film_rhs_vjp_t<double>(c, state, out_bar, state_bar, jc_bar)
                             : film_rhs_vjp_t<float>(c, state, out_bar, state_bar, jc_bar);
}

// ------------------------------------------------------------------ setup
// The spectral form's buffers: a second half spectrum and the per-node jc
// (forward); two more half spectra, the node jc cotangent and an iteration
// state (VJP).  Allocated with the grid or when the form is chosen, never
// inside a right-hand side or a VJP.
int film_spectral_alloc(mag_ctx *c) {
  const size_t ts = c->prec == MAG_FP64 ? 8 : 4;
  const long long n = c->nnode;
  if (!c->d_S2) MAG_HIP(c, hipMalloc(&c->d_S2, c->nspec * 2 * ts));
  if (!c->d_jcn) MAG_HIP(c, hipMalloc(&c->d_jcn, n * ts));
  if (!c->d_S34) MAG_HIP(c, hipMalloc(&c->d_S34, 2 * c->nspec * 2 * ts));
  if (!c->d_cn) MAG_HIP(c, hipMalloc(&c->d_cn, n * sizeof(double)));
  if (!c->d_itv) MAG_HIP(c, hipMalloc(&c->d_itv, sizeof(IterState)));
  // the Gaussian factors per axis, exp(-k^2 sigma^2 / 2) over the half
  // spectrum in x and the full spectrum in y, sigma by default sqrt(dx^2 + dy^2)
  // (Sec. 2.2); refilled whenever the grid or sigma changes
  const double sig = c->dsigma < 0 ? std::hypot(c->d[0], c->d[1]) : c->dsigma;
  const int nx = c->n[0], ny = c->n[1];
  std::vector<double> tab;
  for (int m = 0; m < c->kx; ++m) {
    const double k = 2.0 * M_PI * (double)m / (nx * c->d[0]);
    tab.push_back(std::exp(-0.5 * sig * sig * k * k));
  }
  for (int m = 0; m < ny; ++m) {
    const double k = 2.0 * M_PI * (double)(m < (ny + 1) / 2 ? m : m - ny) / (ny * c->d[1]);
    tab.push_back(std::exp(-0.5 * sig * sig * k * k));
  }
  if (!c->d_filt) MAG_HIP(c, hipMalloc(&c->d_filt, tab.size() * sizeof(double)));
  MAG_HIP(c, hipMemcpy(c->d_filt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  return MAG_OK;
}

int film_alloc(mag_ctx *c) {
  const size_t ts = c->prec == MAG_FP64 ? 8 : 4;
  const long long n = c->nnode;
  MAG_HIP(c, hipMalloc(&c->d_H, n * ts));
  MAG_HIP(c, hipMalloc(&c->d_G, n * ts));
  // a MAG_MIXED_FINAL64 context runs its final evaluation in this buffer
  MAG_HIP(c, hipMalloc(&c->d_S, c->nspec * 2 * (c->prec == MAG_MIXED_FINAL64 ? sizeof(double) : ts)));
  MAG_HIP(c, hipMalloc(&c->d_flags, n));
  MAG_HIP(c, hipMalloc(&c->d_mat, n));
  // 256-node blocks, or the regions of row blocks and stencil blocks of an
  // iteration and the final double evaluation's row blocks
  c->npart = (int)((n + 255) / 256 + 3 * c->n[1] + 16);
  MAG_HIP(c, hipMalloc(&c->d_part, (size_t)c->npart * sizeof(double)));
  MAG_HIP(c, hipMalloc(&c->d_w, 3 * n * ts));
  MAG_HIP(c, hipMemsetAsync(c->d_H, 0, n * ts, c->stream));
  MAG_HIP(c, hipMemsetAsync(c->d_G, 0, n * ts, c->stream));
  if (c->deriv == 1)
    if (int rc = film_spectral_alloc(c)) return rc;
  if (c->prec == MAG_MIXED_FINAL64) {
    MAG_HIP(c, hipMalloc(&c->d_it64, sizeof(IterState)));
    MAG_HIP(c, hipMemsetAsync(c->d_it64, 0, sizeof(IterState), c->stream));
    MAG_HIP(c, hipMalloc(&c->d_w64, n * sizeof(double)));
  }
  // |k|^2 per axis: k = 2 pi fftfreq(n, d)
  const int nx = c->n[0], ny = c->n[1];
  std::vector<double> sym;
  c->sym_off[0] = 0;
  for (int m = 0; m < c->kx; ++m) {
    const double k = 2.0 * M_PI * (double)(m <= nx / 2 ? m : m - nx) / (nx * c->d[0]);
    sym.push_back(k * k);
  }
  c->sym_off[1] = (long long)sym.size();
  for (int m = 0; m < ny; ++m) {
    const double k = 2.0 * M_PI * (double)(m < (ny + 1) / 2 ? m : m - ny) / (ny * c->d[1]);
    sym.push_back(k * k);
  }
  // signed wavenumbers of the spectral derivatives, the Nyquist value of
  // each axis set to 0: x over the half spectrum, then y
  c->sym_off[2] = (long long)sym.size();
  for (int m = 0; m < c->kx; ++m)
    sym.push_back(m == nx / 2 ? 0.0 : 2.0 * M_PI * (double)m / (nx * c->d[0]));
  c->sym_off[3] = (long long)sym.size();
  for (int m = 0; m < ny; ++m)
    sym.push_back(m == ny / 2 ? 0.0 : 2.0 * M_PI * (double)(m < (ny + 1) / 2 ? m : m - ny) / (ny * c->d[1]));
  MAG_HIP(c, hipMalloc(&c->d_sym, sym.size() * sizeof(double)));
  MAG_HIP(c, hipMemcpy(c->d_sym, sym.data(), sym.size() * sizeof(double), hipMemcpyHostToDevice));
  return MAG_OK;
}

namespace {
template <typename T>
__global__ void __launch_bounds__(256) from_double_k(const double *__restrict__ src, T *__restrict__ dst,
                                                     long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}
}  // namespace

// tmp: device double[2n], the indicator in the first half.
// w = K 1_out in the compute precision; with mark_film, film nodes hold a
// NaN instead, so that a pass that needs w only on free space reads its
// free-space flag from w itself.
template <typename T>
__global__ void __launch_bounds__(256) weights_k(const double *__restrict__ src, T *__restrict__ dst,
                                                 const uint8_t *__restrict__ flags, int mark_film, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  dst[i] = (mark_film && (flags[i] & 1)) ? (T)NAN : (T)src[i];
}

template <typename T>
static int film_weights_t(mag_ctx *c, double *tmp) {
  const long long n = c->nnode;
  T *w = reinterpret_cast<T *>(c->d_w);
  IterState is{};
  int rc;
  if ((rc = run_iter_init(c, is))) return rc;
  for (int which = 0; which < 2; ++which) {
    if ((rc = film_fwd<T, 2>(c, nullptr, tmp, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
    if ((rc = film_col<T>(c, which))) return rc;
    if ((rc = film_inv<T, 2>(c, nullptr, tmp + n, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
    ProfScope ps(c, K_MISC);
    hipLaunchKernelGGL((weights_k<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, tmp + n,
                       w + which * n, c->d_flags, which, n);
    if (which == 0)
      hipLaunchKernelGGL((weights_k<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, tmp + n,
                         w + 2 * n, c->d_flags, 1, n);
  }
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

// w1 = K1 1_out in double for the final evaluation of a MAG_MIXED_FINAL64
// context (tmp as for film_weights_t).
static int film_weights64(mag_ctx *c, double *tmp) {
  const long long n = c->nnode;
  IterState is{};
  int rc;
  if ((rc = run_iter_init(c, is))) return rc;
  if ((rc = film_fwd<double, 2>(c, nullptr, tmp, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
  if ((rc = film_col<double>(c, 0))) return rc;
  if ((rc = film_inv<double, 2>(c, nullptr, tmp + n, 0.0, parts(nullptr, 0, nullptr), K_MISC))) return rc;
  ProfScope ps(c, K_MISC);
  hipLaunchKernelGGL((weights_k<double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, tmp + n,
                     c->d_w64, c->d_flags, 0, n);
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int film_domain(mag_ctx *c) {
  const int nx = c->n[0], ny = c->n[1];
  const long long n = c->nnode;
  const std::vector<uint8_t> &m = c->h_mat;
  std::vector<uint8_t> fl(n, 0);
  auto F = [&](int p, int q) { return m[(long long)((q % ny + ny) % ny) * nx + (p % nx + nx) % nx] != 0; };
  long long nin = 0;
  for (int q = 0; q < ny; ++q)
    for (int p = 0; p < nx; ++p) {
      const bool in = F(p, q) && F(p - 1, q) && F(p, q - 1) && F(p - 1, q - 1);
      fl[(long long)q * nx + p] = in ? 1 : 0;
      nin += in;
    }
  if (nin == 0) return set_error(c, MAG_E_ARG, "material has no inside node: empty film");
  if (nin == n) return set_error(c, MAG_E_ARG, "material leaves no free-space node");
  c->nout = n - nin;
  for (int a = 0; a < 2; ++a) {
    c->box0[a] = 0;
    c->box1[a] = c->n[a] - 1;
  }
  MAG_HIP(c, hipMemcpy(c->d_flags, fl.data(), n, hipMemcpyHostToDevice));
  MAG_HIP(c, hipMemcpy(c->d_mat, m.data(), n, hipMemcpyHostToDevice));
  c->warm_valid = false;
  // w1 = K1 1_out and w2 = K2 1_out (free-space indicator through the two
  // Fourier multipliers), used to take the free-space means of the iteration
  // as dot products.
  std::vector<double> ind(n);
  for (long long i = 0; i < n; ++i) ind[i] = fl[i] ? 0.0 : 1.0;
  double *tmp = nullptr;
  MAG_HIP(c, hipMalloc(&tmp, 2 * n * sizeof(double)));
  MAG_HIP(c, hipMemcpy(tmp, ind.data(), n * sizeof(double), hipMemcpyHostToDevice));
  int rc = c->prec == MAG_FP64 ? film_weights_t<double>(c, tmp) : film_weights_t<float>(c, tmp);
  if (!rc && c->prec == MAG_MIXED_FINAL64) rc = film_weights64(c, tmp);
  if (rc) {
    (void)hipFree(tmp);
    return rc;
  }
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  MAG_HIP(c, hipFree(tmp));
  return MAG_OK;
}

}  // namespace mag
