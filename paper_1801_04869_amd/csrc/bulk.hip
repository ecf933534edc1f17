// Bulk (3D) right-hand side on a Yee lattice: Faraday's law with the power law
// in the sample and iteration (18) with the Biot-Savart operator Phi of
// eq. (17) in free space (Sec. 3.1 of Prigozhin & Sokolovsky).
//
// Layouts (x fastest): state/iterate [3][nz][ny][nx] on edges, current/e on
// faces, half spectrum [3][nz][ny][kx] with kx = nx/2 + 1.
//
// One inner iteration = five passes over the half spectrum:
//   x_fwd   curl of the iterate, masked to inside faces, real-to-complex rows
//           (only rows of the pruning box; values outside it are zero)
//   y_fwd   complex transforms along y (only z-planes of the box)
//   z_phi   forward z transform, lattice Phi symbol (3x3, with 1/N), inverse z
//   y_inv   inverse transforms along y (all planes)
//   x_inv   complex-to-real rows, free-space update dh = dh_e + Phi[jdot],
//           per-block sums of |dh_new - dh_old| over free-space edges
// followed by a one-block finalize that applies the stop test of Sec. 3.1.
#include <cmath>
#include <cstring>

#include "ctx.h"
#include "kern_common.h"

namespace mag {

namespace {

__device__ __forceinline__ int wrap(int i, int n) { return i & (n - 1); }

struct BulkGeom {
  int nx, ny, nz, kx;
  int b0x, b0y, b0z, b1x, b1y, b1z;   // pruning box (node indices, inclusive)
  double idx, idy, idz;               // 1/d
};

// Box-local index of a stencil neighbour.  When the box spans a whole
// periodic axis (b0 = 0, b1 = n - 1) its two halo layers are copies of the
// last and first interior layers; fold them onto the interior.
__device__ __forceinline__ int fold(int l, int b0, int b1, int n) {
  if (b0 == 0 && b1 == n - 1) return ((l - 1 + n) % n) + 1;
  return l;
}

// ------------------------------------------------------------ stencil pass
// All grids are one-dimensional with 256 threads per block; box indices use
// 32-bit arithmetic (the host checks that the box holds fewer than 2^31 points).
constexpr int kBlk = 256;

struct BoxIdx {
  int lx, ly, lz;
};
__device__ __forceinline__ BoxIdx box_index(int tid, int bx, int by) {
  BoxIdx b;
  b.lx = tid % bx;
  const int t = tid / bx;
  b.ly = t % by;
  b.lz = t / by;
  return b;
}

// j = curl h on the faces of the extended box [b0-1, b1+1] (double arithmetic
// from the double state, stored in T).
template <typename T>
__global__ void __launch_bounds__(kBlk) bulk_curl_box(const double *__restrict__ h, T *__restrict__ jb,
                                                      BulkGeom g, int bx, int by, int bz) {
  const int nbox = bx * by * bz;
  const int tid = blockIdx.x * kBlk + threadIdx.x;
  if (tid >= nbox) return;
  const BoxIdx b = box_index(tid, bx, by);
  const int p = wrap(g.b0x - 1 + b.lx, g.nx), q = wrap(g.b0y - 1 + b.ly, g.ny), r = wrap(g.b0z - 1 + b.lz, g.nz);
  const long long N = (long long)g.nx * g.ny * g.nz;
  const double *hx = h, *hy = h + N, *hz = h + 2 * N;
  auto at = [&](int pp, int qq, int rr) {
    return ((long long)wrap(rr, g.nz) * g.ny + wrap(qq, g.ny)) * g.nx + wrap(pp, g.nx);
  };
  const long long o = at(p, q, r);
  const double jx = (hz[at(p, q + 1, r)] - hz[o]) * g.idy - (hy[at(p, q, r + 1)] - hy[o]) * g.idz;
  const double jy = (hx[at(p, q, r + 1)] - hx[o]) * g.idz - (hz[at(p + 1, q, r)] - hz[o]) * g.idx;
  const double jz = (hy[at(p + 1, q, r)] - hy[o]) * g.idx - (hx[at(p, q + 1, r)] - hx[o]) * g.idy;
  jb[tid] = (T)jx;
  jb[tid + nbox] = (T)jy;
  jb[tid + 2 * nbox] = (T)jz;
}

// Power law on inside faces.  rho = (e0/jc)(s/jc)^(n-1) evaluated as
// (e0/jc) exp((n-1) log(s/jc)); in float the exponent is clamped so that the
// factor stays below 1e30.  Non-inside faces get e = 0 (never used).
template <typename T>
__device__ __forceinline__ T power_rho(T s, T jc, T e0, T nm1, T lmax) {
  if (!(s > (T)0)) return (T)0;
  T lg = log(s / jc);
  if constexpr (sizeof(T) == 4) lg = fminf(lg, lmax);
  return (e0 / jc) * exp(nm1 * lg);
}

template <typename T>
__global__ void __launch_bounds__(kBlk) bulk_efield_box(const T *__restrict__ jb, T *__restrict__ eb,
                                                        const uint8_t *__restrict__ mat,
                                                        const T *__restrict__ jc, BulkGeom g, int bx,
                                                        int by, int bz, T e0, T nm1, T rho_out, T lmax,
                                                        int has_jc, T jc0) {
  const int nbox = bx * by * bz;
  const int tid = blockIdx.x * kBlk + threadIdx.x;
  if (tid >= nbox) return;
  const BoxIdx b = box_index(tid, bx, by);
  const int lx = b.lx, ly = b.ly, lz = b.lz;
  const T *jx = jb, *jy = jb + nbox, *jz = jb + 2 * nbox;
  const bool interior = lx > 0 && ly > 0 && lz > 0 && lx < bx - 1 && ly < by - 1 && lz < bz - 1;
  if (!interior) {
    eb[tid] = eb[tid + nbox] = eb[tid + 2 * nbox] = (T)0;
    return;
  }
  const int p = wrap(g.b0x - 1 + lx, g.nx), q = wrap(g.b0y - 1 + ly, g.ny), r = wrap(g.b0z - 1 + lz, g.nz);
  auto L = [&](int a, int bb, int cc) { return (cc * by + bb) * bx + a; };
  auto cell = [&](int pp, int qq, int rr) {
    return ((long long)wrap(rr, g.nz) * g.ny + wrap(qq, g.ny)) * g.nx + wrap(pp, g.nx);
  };
  const int o = tid;
  // neighbours of an a-face among b-faces: offsets {-1,0} along a, {0,+1} along b
  const T jxo = jx[o], jyo = jy[o], jzo = jz[o];
  const T jy_at_x = (T)0.25 * (jy[L(lx - 1, ly, lz)] + jyo + jy[L(lx - 1, ly + 1, lz)] + jy[L(lx, ly + 1, lz)]);
  const T jz_at_x = (T)0.25 * (jz[L(lx - 1, ly, lz)] + jzo + jz[L(lx - 1, ly, lz + 1)] + jz[L(lx, ly, lz + 1)]);
  const T jx_at_y = (T)0.25 * (jx[L(lx, ly - 1, lz)] + jxo + jx[L(lx + 1, ly - 1, lz)] + jx[L(lx + 1, ly, lz)]);
  const T jz_at_y = (T)0.25 * (jz[L(lx, ly - 1, lz)] + jzo + jz[L(lx, ly - 1, lz + 1)] + jz[L(lx, ly, lz + 1)]);
  const T jx_at_z = (T)0.25 * (jx[L(lx, ly, lz - 1)] + jxo + jx[L(lx + 1, ly, lz - 1)] + jx[L(lx + 1, ly, lz)]);
  const T jy_at_z = (T)0.25 * (jy[L(lx, ly, lz - 1)] + jyo + jy[L(lx, ly + 1, lz - 1)] + jy[L(lx, ly + 1, lz)]);
  const T s0 = sqrt(jxo * jxo + jy_at_x * jy_at_x + jz_at_x * jz_at_x);
  const T s1 = sqrt(jyo * jyo + jx_at_y * jx_at_y + jz_at_y * jz_at_y);
  const T s2 = sqrt(jzo * jzo + jx_at_z * jx_at_z + jy_at_z * jy_at_z);
  const long long c0 = cell(p, q, r);
  const uint8_t m0 = mat[c0];
  auto face_e = [&](long long cn, T s, T jv) -> T {
    const uint8_t m1 = mat[cn];
    if (m0 == 1 && m1 == 1) {
      const T jcf = has_jc ? (T)0.5 * (jc[c0] + jc[cn]) : jc0;
      return power_rho(s, jcf, e0, nm1, lmax) * jv;
    }
    if (m0 != 0 && m1 != 0) return rho_out * jv;
    return (T)0;
  };
  eb[o] = face_e(cell(p - 1, q, r), s0, jxo);
  eb[o + nbox] = face_e(cell(p, q - 1, r), s1, jyo);
  eb[o + 2 * nbox] = face_e(cell(p, q, r - 1), s2, jzo);
}

// dh/dt = -curl^T e on inside edges (backward differences inside the box).
template <typename T>
__global__ void __launch_bounds__(kBlk) bulk_hdot_in(const T *__restrict__ eb, T *__restrict__ H,
                                                     const uint8_t *__restrict__ flags, BulkGeom g, int bx,
                                                     int by, int bz) {
  const int nbox = bx * by * bz;
  const int tid = blockIdx.x * kBlk + threadIdx.x;
  if (tid >= nbox) return;
  const BoxIdx b = box_index(tid, bx, by);
  const int lx = b.lx, ly = b.ly, lz = b.lz;
  if (lx == 0 || ly == 0 || lz == 0 || lx == bx - 1 || ly == by - 1 || lz == bz - 1) return;
  const int p = wrap(g.b0x - 1 + lx, g.nx), q = wrap(g.b0y - 1 + ly, g.ny), r = wrap(g.b0z - 1 + lz, g.nz);
  const long long N = (long long)g.nx * g.ny * g.nz;
  const long long gi = ((long long)r * g.ny + q) * g.nx + p;
  const uint8_t f = flags[gi];
  if (!(f & 0x38)) return;
  auto L = [&](int a, int bb, int cc) {
    return (fold(cc, g.b0z, g.b1z, g.nz) * by + fold(bb, g.b0y, g.b1y, g.ny)) * bx + fold(a, g.b0x, g.b1x, g.nx);
  };
  const T *ex = eb, *ey = eb + nbox, *ez = eb + 2 * nbox;
  const int o = tid;
  if (f & 0x08) {
    const double v = (double(ez[o]) - double(ez[L(lx, ly - 1, lz)])) * g.idy -
                     (double(ey[o]) - double(ey[L(lx, ly, lz - 1)])) * g.idz;
    H[gi] = (T)(-v);
  }
  if (f & 0x10) {
    const double v = (double(ex[o]) - double(ex[L(lx, ly, lz - 1)])) * g.idz -
                     (double(ez[o]) - double(ez[L(lx - 1, ly, lz)])) * g.idx;
    H[gi + N] = (T)(-v);
  }
  if (f & 0x20) {
    const double v = (double(ey[o]) - double(ey[L(lx - 1, ly, lz)])) * g.idx -
                     (double(ex[o]) - double(ex[L(lx, ly - 1, lz)])) * g.idy;
    H[gi + 2 * N] = (T)(-v);
  }
}

// Free-space edges take dh_e/dt (first call or after a failed iteration).
template <typename T>
__global__ void __launch_bounds__(kBlk) bulk_init_out(T *__restrict__ H, const uint8_t *__restrict__ flags,
                                                      long long N, double h0, double h1, double h2) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  if (i >= N) return;
  const uint8_t f = flags[i];
  if (!(f & 0x08)) H[i] = (T)h0;
  if (!(f & 0x10)) H[i + N] = (T)h1;
  if (!(f & 0x20)) H[i + 2 * N] = (T)h2;
}

// ------------------------------------------------------------ x_fwd
// Rows (q, r) of the box for the three components: block b handles rows
// (b % nblk) * P .. of component b / nblk.  jdot = curl H on inside faces.
template <typename T, int M>
__global__ void __launch_bounds__((RowShape<M, T>::THREADS))
    bulk_x_fwd(const T *__restrict__ H, const uint8_t *__restrict__ flags, cx<T> *__restrict__ S,
               const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN, BulkGeom g, int nblk,
               const IterState *__restrict__ it) {
  if (it->done) return;
  using RS = RowShape<M, T>;
  constexpr int TT = RS::TT, P = RS::P, RMAX = Plan<M>::RMAX;
  constexpr int PITCH = RS::PITCH;
  __shared__ T lre[P * PITCH], lim[P * PITCH];
  const int c = blockIdx.x / nblk;
  const int rb = blockIdx.x - c * nblk;
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  const int nrow_y = g.b1y - g.b0y + 1, nrow_z = g.b1z - g.b0z + 1;
  const int row = rb * P + pr;
  const bool active = row < nrow_y * nrow_z;
  const int q = g.b0y + (active ? row % nrow_y : 0), r = g.b0z + (active ? row / nrow_y : 0);
  const long long N = (long long)g.nx * g.ny * g.nz;
  const T *Hx = H, *Hy = H + N, *Hz = H + 2 * N;
  const long long rowo = ((long long)r * g.ny + q) * g.nx;
  const long long rowq1 = ((long long)r * g.ny + wrap(q + 1, g.ny)) * g.nx;
  const long long rowr1 = ((long long)wrap(r + 1, g.nz) * g.ny + q) * g.nx;
  const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
  const uint8_t bit = (uint8_t)(1u << c);
  cx<T> v[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    T val[2] = {(T)0, (T)0};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = 2 * (j + rho * TT) + e;
      if (active && p >= g.b0x && p <= g.b1x && (flags[rowo + p] & bit)) {
        const int p1 = wrap(p + 1, g.nx);
        T jv;
        if (c == 0) jv = (Hz[rowq1 + p] - Hz[rowo + p]) * idy - (Hy[rowr1 + p] - Hy[rowo + p]) * idz;
        else if (c == 1) jv = (Hx[rowr1 + p] - Hx[rowo + p]) * idz - (Hz[rowo + p1] - Hz[rowo + p]) * idx;
        else jv = (Hy[rowo + p1] - Hy[rowo + p]) * idx - (Hx[rowq1 + p] - Hx[rowo + p]) * idy;
        val[e] = jv;
      }
    }
    v[rho] = {val[0], val[1]};
  }
  T *mre = lre + pr * PITCH, *mim = lim + pr * PITCH;
  pencil_fft<M, -1>(v, j, mre, mim, [](int i) { return i + (i >> 4); }, twM);
  cx<T> *dst = S + (long long)c * g.kx * g.ny * g.nz + ((long long)r * g.ny + q) * g.kx;
  r2c_finish<M>(v, j, mre, mim, twN, dst, active);
}

// ------------------------------------------------------------ column transforms
// In-place complex transforms of length NN along a strided axis.  Pencil
// (col, plane) of component cc: element i at S + cc*comp_stride +
// plane*plane_stride + i*estride + col, for col < ncols and planes
// [plane0, plane0 + nplanes); block b covers component b / (ngrp*nplanes).
// Inputs outside [lo, hi] are taken as zero (zero padding).
template <typename T, int NN, int DIR>
__global__ void __launch_bounds__((ColShape<NN, T>::THREADS))
    col_fft(cx<T> *__restrict__ S, long long comp_stride, long long plane_stride, long long estride,
            int ncols, int plane0, int nplanes, int lo, int hi, const cx<T> *__restrict__ tw,
            const IterState *__restrict__ it) {
  if (it->done) return;
  using CS = ColShape<NN, T>;
  constexpr int TT = CS::TT, P = CS::P, RMAX = Plan<NN>::RMAX;
  HIP_DYNAMIC_SHARED(unsigned char, smem_raw)
  T *lre = reinterpret_cast<T *>(smem_raw), *lim = lre + NN * P;
  const int pcol = threadIdx.x % P, j = threadIdx.x / P;
  const int ngrp = (ncols + P - 1) / P;
  const int per_comp = ngrp * nplanes;
  const int cc = blockIdx.x / per_comp;
  const int bi = blockIdx.x - cc * per_comp;
  const int grp = bi % ngrp, plane = plane0 + bi / ngrp;
  const int col = grp * P + pcol;
  const bool active = col < ncols;
  cx<T> *base = S + (long long)cc * comp_stride + (long long)plane * plane_stride + (active ? col : 0);
  cx<T> v[RMAX];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int i = j + rho * TT;
    v[rho] = (active && i >= lo && i <= hi) ? base[(long long)i * estride] : cx<T>{(T)0, (T)0};
  }
  pencil_fft<NN, DIR>(v, j, lre, lim, [pcol](int i) { return i * P + pcol; }, tw);
  if (!active) return;
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) base[(long long)(j + rho * TT) * estride] = v[rho];
}

// ------------------------------------------------------------ z pass with Phi
// Symbol tables (double): dm[a] complex backward-difference symbol per axis
// index, k2[a] = 4 sin^2(theta/2)/d^2 per axis index.
struct PhiTables {
  const double2 *dmx, *dmy, *dmz;
  const double *k2x, *k2y, *k2z;
  double inv_n;   // 1 / (nx ny nz)
};

// z pencils of P consecutive kx at one ky.  LDS holds the three transformed
// components of the block's pencils (each thread keeps only one component in
// registers at a time) plus one exchange area for the transforms.
template <int NZ, typename T>
struct ZShape {
  static constexpr int TT = Plan<NZ>::TT;
  static constexpr int PW = sizeof(T) == 8 ? 8 : 16;
  static constexpr int PL = pow2floor(kLdsBudget / (4 * NZ * 2 * (int)sizeof(T)));
  static constexpr int PT = 1024 / TT;
  static constexpr int P0 = PW < PL ? PW : PL;
  static constexpr int P = P0 < PT ? P0 : PT;
  static constexpr int THREADS = P * TT;
  static constexpr int LDS_BYTES = 4 * NZ * P * 2 * (int)sizeof(T);
};

template <typename T, int NZ>
__global__ void __launch_bounds__((ZShape<NZ, T>::THREADS))
    bulk_z_phi(cx<T> *__restrict__ S, long long comp_stride, int kx, int ny, int lo, int hi,
               const cx<T> *__restrict__ tw, PhiTables tb, const IterState *__restrict__ it) {
  if (it->done) return;
  using ZS = ZShape<NZ, T>;
  constexpr int TT = ZS::TT, P = ZS::P, RMAX = Plan<NZ>::RMAX;
  constexpr int SL = 2 * NZ * P;   // one slice (real then imaginary plane)
  HIP_DYNAMIC_SHARED(unsigned char, smem_raw)
  T *lds = reinterpret_cast<T *>(smem_raw);
  T *xre = lds + 3 * SL, *xim = xre + NZ * P;   // exchange area
  const int pcol = threadIdx.x % P, j = threadIdx.x / P;
  const int ngrp = (kx + P - 1) / P;
  const int grp = blockIdx.x % ngrp, ky = blockIdx.x / ngrp;
  const int col = grp * P + pcol;
  const bool active = col < kx;
  const long long estride = (long long)ny * kx;
  cx<T> *base = S + (long long)ky * kx + (active ? col : 0);
  auto lidx = [pcol](int i) { return i * P + pcol; };
  cx<T> v[RMAX];
  // forward transforms; each thread stores its own outputs (kz = j + rho TT)
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int i = j + rho * TT;
      v[rho] = (active && i >= lo && i <= hi) ? base[c * comp_stride + (long long)i * estride]
                                              : cx<T>{(T)0, (T)0};
    }
    pencil_fft<NZ, -1>(v, j, xre, xim, lidx, tw);
    T *fre = lds + c * SL, *fim = fre + NZ * P;
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int o = (j + rho * TT) * P + pcol;
      fre[o] = v[rho].x;
      fim[o] = v[rho].y;
    }
  }
  // Phi_x = (dy Fz - dz Fy) / |kappa|^2, cyclic; 1/N folded in.  Only the
  // thread's own entries are touched, so no barrier is needed.
  const double2 dxv = tb.dmx[active ? col : 0], dyv = tb.dmy[ky];
  const double k2xy = tb.k2x[active ? col : 0] + tb.k2y[ky];
#pragma unroll
  for (int rho = 0; rho < RMAX; ++rho) {
    const int kz = j + rho * TT;
    const int o = kz * P + pcol;
    const double2 dzv = tb.dmz[kz];
    const double kk = k2xy + tb.k2z[kz];
    const double inv = kk > 0.0 ? tb.inv_n / kk : 0.0;
    const cx<T> dx = {(T)(dxv.x * inv), (T)(dxv.y * inv)};
    const cx<T> dy = {(T)(dyv.x * inv), (T)(dyv.y * inv)};
    const cx<T> dz = {(T)(dzv.x * inv), (T)(dzv.y * inv)};
    const cx<T> Fx = {lds[o], lds[o + NZ * P]};
    const cx<T> Fy = {lds[SL + o], lds[SL + o + NZ * P]};
    const cx<T> Fz = {lds[2 * SL + o], lds[2 * SL + o + NZ * P]};
    const cx<T> Px = cmul(dy, Fz) - cmul(dz, Fy);
    const cx<T> Py = cmul(dz, Fx) - cmul(dx, Fz);
    const cx<T> Pz = cmul(dx, Fy) - cmul(dy, Fx);
    lds[o] = Px.x;
    lds[o + NZ * P] = Px.y;
    lds[SL + o] = Py.x;
    lds[SL + o + NZ * P] = Py.y;
    lds[2 * SL + o] = Pz.x;
    lds[2 * SL + o + NZ * P] = Pz.y;
  }
  for (int c = 0; c < 3; ++c) {
    const T *fre = lds + c * SL, *fim = fre + NZ * P;
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int o = (j + rho * TT) * P + pcol;
      v[rho] = {fre[o], fim[o]};
    }
    pencil_fft<NZ, +1>(v, j, xre, xim, lidx, tw);
    if (active) {
#pragma unroll
      for (int rho = 0; rho < RMAX; ++rho) base[c * comp_stride + (long long)(j + rho * TT) * estride] = v[rho];
    }
  }
}

// ------------------------------------------------------------ x_inv + update
// All rows of the three components: block b handles rows (b % nblk) * P .. of
// component b / nblk and writes its partial sum to part[b].
template <typename T, int M>
__global__ void __launch_bounds__((RowShape<M, T>::THREADS))
    bulk_x_inv(T *__restrict__ H, const uint8_t *__restrict__ flags, const cx<T> *__restrict__ S,
               const cx<T> *__restrict__ twM, const cx<T> *__restrict__ twN, BulkGeom g, int nblk, double hd0,
               double hd1, double hd2, double *__restrict__ part, const IterState *__restrict__ it) {
  if (it->done) return;
  using RS = RowShape<M, T>;
  constexpr int TT = RS::TT, P = RS::P, RMAX = Plan<M>::RMAX;
  constexpr int PITCH = RS::PITCH;
  __shared__ T lre[P * PITCH], lim[P * PITCH];
  __shared__ double red[RS::THREADS];
  const int c = blockIdx.x / nblk;
  const int rb = blockIdx.x - c * nblk;
  const int pr = threadIdx.x / TT, j = threadIdx.x % TT;
  const int nrows = g.ny * g.nz;
  const int row = rb * P + pr;
  const bool active = row < nrows;
  const int q = active ? row % g.ny : 0, r = active ? row / g.ny : 0;
  const long long N = (long long)g.nx * g.ny * g.nz;
  const cx<T> *src = S + (long long)c * g.kx * g.ny * g.nz + ((long long)r * g.ny + q) * g.kx;
  cx<T> v[RMAX];
  c2r_start<M>(v, j, src, twN, active);
  T *mre = lre + pr * PITCH, *mim = lim + pr * PITCH;
  pencil_fft<M, +1>(v, j, mre, mim, [](int i) { return i + (i >> 4); }, twM);
  const double hde = c == 0 ? hd0 : (c == 1 ? hd1 : hd2);
  const uint8_t bit = (uint8_t)(8u << c);
  double acc = 0.0;
  if (active) {
    T *Hc = H + (long long)c * N + ((long long)r * g.ny + q) * g.nx;
    const uint8_t *fr = flags + ((long long)r * g.ny + q) * g.nx;
#pragma unroll
    for (int rho = 0; rho < RMAX; ++rho) {
      const int m = j + rho * TT;
      const T ph[2] = {v[rho].x, v[rho].y};
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int p = 2 * m + e;
        if (!(fr[p] & bit)) {
          const T hn = (T)(hde + (double)ph[e]);
          const T ho = Hc[p];
          acc += fabs((double)hn - (double)ho);
          Hc[p] = hn;
        }
      }
    }
  }
  const double s = block_sum<RS::THREADS>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(kBlk) to_double_k(const T *__restrict__ src, double *__restrict__ dst, long long n) {
  const long long i = (long long)blockIdx.x * kBlk + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

}  // namespace

// ================================================================= host side
template <typename T>
static BulkGeom geom(mag_ctx *c) {
  BulkGeom g;
  g.nx = c->n[0];
  g.ny = c->n[1];
  g.nz = c->n[2];
  g.kx = c->kx;
  g.b0x = c->box0[0];
  g.b0y = c->box0[1];
  g.b0z = c->box0[2];
  g.b1x = c->box1[0];
  g.b1y = c->box1[1];
  g.b1z = c->box1[2];
  g.idx = 1.0 / c->d[0];
  g.idy = 1.0 / c->d[1];
  g.idz = 1.0 / c->d[2];
  return g;
}

#define MAG_SWITCH_M(M_, ...)                  \
  switch (M_) {                                 \
    case 8: { constexpr int MM = 8; __VA_ARGS__; } break;       \
    case 16: { constexpr int MM = 16; __VA_ARGS__; } break;     \
    case 32: { constexpr int MM = 32; __VA_ARGS__; } break;     \
    case 64: { constexpr int MM = 64; __VA_ARGS__; } break;     \
    case 128: { constexpr int MM = 128; __VA_ARGS__; } break;   \
    case 256: { constexpr int MM = 256; __VA_ARGS__; } break;   \
    case 512: { constexpr int MM = 512; __VA_ARGS__; } break;   \
    case 1024: { constexpr int MM = 1024; __VA_ARGS__; } break; \
    default: return set_error(c, MAG_E_ARG, "unsupported length %d", M_); \
  }

#define MAG_SWITCH_N(N_, ...)                  \
  switch (N_) {                                 \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;     \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;     \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;     \
    case 128: { constexpr int NN = 128; __VA_ARGS__; } break;   \
    case 256: { constexpr int NN = 256; __VA_ARGS__; } break;   \
    case 512: { constexpr int NN = 512; __VA_ARGS__; } break;   \
    case 1024: { constexpr int NN = 1024; __VA_ARGS__; } break; \
    case 2048: { constexpr int NN = 2048; __VA_ARGS__; } break; \
    default: return set_error(c, MAG_E_ARG, "unsupported length %d", N_); \
  }

template <typename T>
static int bulk_launch_col(mag_ctx *c, int dir, int n_axis, long long plane_stride, long long estride,
                           int plane0, int nplanes, int lo, int hi, const cx<T> *tw, int kid) {
  cx<T> *S = reinterpret_cast<cx<T> *>(c->d_S);
  ProfScope ps(c, kid);
  MAG_SWITCH_N(n_axis, {
    using CS = ColShape<NN, T>;
    const int ngrp = (c->kx + CS::P - 1) / CS::P;
    dim3 grid(3 * ngrp * nplanes);
    const size_t lds = (size_t)2 * NN * CS::P * sizeof(T);
    if (dir < 0)
      hipLaunchKernelGGL((col_fft<T, NN, -1>), grid, dim3(CS::THREADS), lds, c->stream, S, c->nspec,
                         plane_stride, estride, c->kx, plane0, nplanes, lo, hi, tw, c->d_it);
    else
      hipLaunchKernelGGL((col_fft<T, NN, +1>), grid, dim3(CS::THREADS), lds, c->stream, S, c->nspec,
                         plane_stride, estride, c->kx, plane0, nplanes, lo, hi, tw, c->d_it);
  });
  return MAG_OK;
}

template <typename T>
static int bulk_iteration(mag_ctx *c, const double hd[3]) {
  const BulkGeom g = geom<T>(c);
  const T *Hc = reinterpret_cast<const T *>(c->d_H);
  T *H = reinterpret_cast<T *>(c->d_H);
  cx<T> *S = reinterpret_cast<cx<T> *>(c->d_S);
  const cx<T> *tw = reinterpret_cast<const cx<T> *>(c->d_tw);
  const cx<T> *twM = tw + c->tw_off[0], *twY = tw + c->tw_off[1], *twZ = tw + c->tw_off[2],
              *twN = tw + c->tw_off[3];
  const int M = c->n[0] / 2;
  // x_fwd on box rows
  {
    ProfScope ps(c, K_BULK_X_FWD);
    const int nrows = (g.b1y - g.b0y + 1) * (g.b1z - g.b0z + 1);
    MAG_SWITCH_M(M, {
      using RS = RowShape<MM, T>;
      const int nb_rows = (nrows + RS::P - 1) / RS::P;
      hipLaunchKernelGGL((bulk_x_fwd<T, MM>), dim3(3 * nb_rows), dim3(RS::THREADS), 0, c->stream, Hc, c->d_flags,
                         S, twM, twN, g, nb_rows, c->d_it);
    });
  }
  // y forward on box z-planes, inputs y in the box
  int rc = bulk_launch_col<T>(c, -1, g.ny, (long long)g.ny * g.kx, g.kx, g.b0z, g.b1z - g.b0z + 1, g.b0y,
                              g.b1y, twY, K_BULK_Y_FWD);
  if (rc) return rc;
  // z pass with Phi
  {
    ProfScope ps(c, K_BULK_Z_PHI);
    PhiTables tb;
    const double *sym = c->d_sym;
    tb.dmx = reinterpret_cast<const double2 *>(sym + c->sym_off[0]);
    tb.dmy = reinterpret_cast<const double2 *>(sym + c->sym_off[1]);
    tb.dmz = reinterpret_cast<const double2 *>(sym + c->sym_off[2]);
    tb.k2x = sym + c->sym_off[3];
    tb.k2y = sym + c->sym_off[4];
    tb.k2z = sym + c->sym_off[5];
    tb.inv_n = 1.0 / (double)c->nnode;
    MAG_SWITCH_N(g.nz, {
      using ZS = ZShape<NN, T>;
      const int ngrp = (g.kx + ZS::P - 1) / ZS::P;
      hipLaunchKernelGGL((bulk_z_phi<T, NN>), dim3(ngrp * g.ny), dim3(ZS::THREADS), (size_t)ZS::LDS_BYTES,
                         c->stream, S, c->nspec, g.kx, g.ny, g.b0z, g.b1z, twZ, tb, c->d_it);
    });
  }
  // y inverse on all planes
  rc = bulk_launch_col<T>(c, +1, g.ny, (long long)g.ny * g.kx, g.kx, 0, g.nz, 0, g.ny - 1, twY, K_BULK_Y_INV);
  if (rc) return rc;
  // x_inv + update + partial residuals
  int nblk = 0;
  {
    ProfScope ps(c, K_BULK_X_INV_UPD);
    const int nrows = g.ny * g.nz;
    MAG_SWITCH_M(M, {
      using RS = RowShape<MM, T>;
      nblk = (nrows + RS::P - 1) / RS::P;
      hipLaunchKernelGGL((bulk_x_inv<T, MM>), dim3(3 * nblk), dim3(RS::THREADS), 0, c->stream, H, c->d_flags, S,
                         twM, twN, g, nblk, hd[0], hd[1], hd[2], c->d_part, c->d_it);
    });
  }
  return run_finalize_stop(c, nblk * 3);
}

template <typename T>
static int bulk_rhs_t(mag_ctx *c, const double *state, double t, double *out, int *n_inner) {
  double hd[3];
  field_hdot(c, t, hd);
  const double hmag = std::sqrt(hd[0] * hd[0] + hd[1] * hd[1] + hd[2] * hd[2]);
  const BulkGeom g = geom<T>(c);
  T *H = reinterpret_cast<T *>(c->d_H);
  // reset the iteration state
  IterState is{};
  is.done = 0;
  is.iters = 0;
  is.fixed = c->fixed_iters;
  is.thr = c->tol * (hmag > 1.0 ? hmag : 1.0);
  is.inv_nout = c->nout > 0 ? 1.0 / (double)c->nout : 0.0;
  if (int rc0 = run_iter_init(c, is)) return rc0;
  if (!c->warm_valid) {
    ProfScope ps(c, K_MISC);
    const long long N = c->nnode;
    hipLaunchKernelGGL((bulk_init_out<T>), dim3((unsigned)((N + kBlk - 1) / kBlk)), dim3(kBlk), 0, c->stream, H,
                       c->d_flags, N, hd[0], hd[1], hd[2]);
  }
  // stencil: j, e, dh_in on the box
  const int bx = c->boxn[0], by = c->boxn[1], bz = c->boxn[2];
  const long long nbox = c->boxvol;
  T *jb = reinterpret_cast<T *>(c->d_box), *eb = jb + 3 * nbox;
  const unsigned nb = (unsigned)((nbox + kBlk - 1) / kBlk);
  {
    ProfScope ps(c, K_BULK_CURL);
    hipLaunchKernelGGL((bulk_curl_box<T>), dim3(nb), dim3(kBlk), 0, c->stream, state, jb, g, bx, by, bz);
  }
  {
    ProfScope ps(c, K_BULK_EFIELD);
    const double lmax = std::log(1e30) / (c->nexp - 1.0 > 1e-12 ? c->nexp - 1.0 : 1e-12);
    hipLaunchKernelGGL((bulk_efield_box<T>), dim3(nb), dim3(kBlk), 0, c->stream, jb, eb, c->d_mat,
                       reinterpret_cast<const T *>(c->d_jc), g, bx, by, bz, (T)c->e0, (T)(c->nexp - 1.0),
                       (T)c->rho_out, (T)lmax, c->has_jc_map ? 1 : 0, (T)c->jc0);
  }
  {
    ProfScope ps(c, K_BULK_HDOT_IN);
    hipLaunchKernelGGL((bulk_hdot_in<T>), dim3(nb), dim3(kBlk), 0, c->stream, eb, H, c->d_flags, g, bx, by, bz);
  }
  MAG_HIP(c, hipGetLastError());
  // inner iterations in blocks, one host poll per block
  const int kmax = c->fixed_iters > 0 ? c->fixed_iters : c->max_inner;
  int issued = 0;
  int block = c->fixed_iters > 0 ? c->fixed_iters : (c->last_iters > 0 ? c->last_iters : 1);
  bool done = false;
  while (issued < kmax) {
    const int nb_it = block < kmax - issued ? block : kmax - issued;
    for (int k = 0; k < nb_it; ++k) {
      c->cur_iter = issued + k;
      int rc = bulk_iteration<T>(c, hd);
      if (rc) return rc;
    }
    c->cur_iter = -1;
    issued += nb_it;
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
  if (n_inner) *n_inner = used;
  if (!done) {
    c->warm_valid = false;
    return set_error(c, MAG_NOT_CONVERGED, "inner iteration not converged after %d iterations (r = %g)",
                     used, c->h_it->r);
  }
  c->last_iters = used;
  c->warm_valid = true;
  if (!std::isfinite(c->h_it->r)) {
    c->warm_valid = false;
    return set_error(c, MAG_E_NUMERIC, "non-finite residual");
  }
  return run_to_double(c, c->d_H, out, 3 * c->nnode);
}

int bulk_rhs(mag_ctx *c, const double *state, double t, double *out, int *n_inner) {
  return c->prec == MAG_FP64 ? bulk_rhs_t<double>(c, state, t, out, n_inner)
                             : bulk_rhs_t<float>(c, state, t, out, n_inner);
}

template <typename T>
int run_to_double_t(mag_ctx *c, const void *src, double *dst, long long n) {
  ProfScope ps(c, K_MISC);
  hipLaunchKernelGGL((to_double_k<T>), dim3((unsigned)((n + kBlk - 1) / kBlk)), dim3(kBlk), 0, c->stream,
                     reinterpret_cast<const T *>(src), dst, n);
  MAG_HIP(c, hipGetLastError());
  return MAG_OK;
}

int run_to_double(mag_ctx *c, const void *src, double *dst, long long n) {
  return c->prec == MAG_FP64 ? run_to_double_t<double>(c, src, dst, n) : run_to_double_t<float>(c, src, dst, n);
}

// ------------------------------------------------------------------ setup
int bulk_alloc(mag_ctx *c) {
  const size_t ts = c->prec == MAG_FP64 ? 8 : 4;
  const long long N = c->nnode;
  MAG_HIP(c, hipMalloc(&c->d_H, 3 * N * ts));
  MAG_HIP(c, hipMalloc(&c->d_S, 3 * c->nspec * 2 * ts));
  MAG_HIP(c, hipMalloc(&c->d_flags, N));
  MAG_HIP(c, hipMalloc(&c->d_mat, N));
  // per-block partials: at most one x_inv block per row, times 3 components
  c->npart = (int)(3LL * c->n[1] * c->n[2] + 16);
  MAG_HIP(c, hipMalloc(&c->d_part, (size_t)c->npart * sizeof(double)));
  MAG_HIP(c, hipMemsetAsync(c->d_H, 0, 3 * N * ts, c->stream));
  // symbol tables: dm (complex) for x (kx entries), y, z; k2 for x, y, z
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  std::vector<double> sym;
  auto theta = [](int m, int n) { return 2.0 * M_PI * (double)(m <= n / 2 ? m : m - n) / (double)n; };
  auto add_dm = [&](int cnt, int n, double d, int slot) {
    c->sym_off[slot] = (long long)sym.size();
    for (int m = 0; m < cnt; ++m) {
      const double th = theta(m, n);
      sym.push_back((1.0 - std::cos(th)) / d);   // (1 - exp(-i th)) / d = (1 - cos th + i sin th) / d
      sym.push_back(std::sin(th) / d);
    }
  };
  auto add_k2 = [&](int cnt, int n, double d, int slot) {
    c->sym_off[slot] = (long long)sym.size();
    for (int m = 0; m < cnt; ++m) {
      const double s = std::sin(0.5 * theta(m, n));
      sym.push_back(4.0 * s * s / (d * d));
    }
  };
  add_dm(c->kx, nx, c->d[0], 0);
  add_dm(ny, ny, c->d[1], 1);
  add_dm(nz, nz, c->d[2], 2);
  add_k2(c->kx, nx, c->d[0], 3);
  add_k2(ny, ny, c->d[1], 4);
  add_k2(nz, nz, c->d[2], 5);
  MAG_HIP(c, hipMalloc(&c->d_sym, sym.size() * sizeof(double)));
  MAG_HIP(c, hipMemcpy(c->d_sym, sym.data(), sym.size() * sizeof(double), hipMemcpyHostToDevice));
  return MAG_OK;
}

// Classify faces/edges from the host copy of the material and size the box.
int bulk_domain(mag_ctx *c) {
  const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
  const long long N = c->nnode;
  const std::vector<uint8_t> &m = c->h_mat;
  std::vector<uint8_t> fl(N, 0);
  auto F = [&](int p, int q, int r) -> bool {
    return m[((long long)(r & (nz - 1)) * ny + (q & (ny - 1))) * nx + (p & (nx - 1))] != 0;
  };
  long long nin = 0;
  int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
  for (int r = 0; r < nz; ++r)
    for (int q = 0; q < ny; ++q)
      for (int p = 0; p < nx; ++p) {
        uint8_t f = 0;
        const bool c0 = F(p, q, r);
        if (c0 && F(p - 1, q, r)) f |= 1;
        if (c0 && F(p, q - 1, r)) f |= 2;
        if (c0 && F(p, q, r - 1)) f |= 4;
        // x-edge: cells (p,q-1,r-1),(p,q,r-1),(p,q-1,r),(p,q,r)
        if (c0 && F(p, q - 1, r) && F(p, q, r - 1) && F(p, q - 1, r - 1)) f |= 8;
        if (c0 && F(p - 1, q, r) && F(p, q, r - 1) && F(p - 1, q, r - 1)) f |= 16;
        if (c0 && F(p - 1, q, r) && F(p, q - 1, r) && F(p - 1, q - 1, r)) f |= 32;
        fl[((long long)r * ny + q) * nx + p] = f;
        nin += ((f >> 3) & 1) + ((f >> 4) & 1) + ((f >> 5) & 1);
        if (f) {
          const int idx[3] = {p, q, r};
          for (int a = 0; a < 3; ++a) {
            if (idx[a] < lo[a]) lo[a] = idx[a];
            if (idx[a] > hi[a]) hi[a] = idx[a];
          }
        }
      }
  if (hi[0] < 0) return set_error(c, MAG_E_ARG, "material has no inside face: empty sample");
  for (int a = 0; a < 3; ++a) {
    // the box must leave room for the one-cell halo of the stencil; otherwise use the whole axis
    if (lo[a] < 2 || hi[a] > c->n[a] - 3) {
      lo[a] = 0;
      hi[a] = c->n[a] - 1;
    }
    c->box0[a] = lo[a];
    c->box1[a] = hi[a];
    c->boxn[a] = hi[a] - lo[a] + 3;
  }
  c->nout = 3 * N - nin;
  MAG_HIP(c, hipMemcpy(c->d_flags, fl.data(), N, hipMemcpyHostToDevice));
  MAG_HIP(c, hipMemcpy(c->d_mat, m.data(), N, hipMemcpyHostToDevice));
  const size_t ts = c->prec == MAG_FP64 ? 8 : 4;
  c->boxvol = (long long)c->boxn[0] * c->boxn[1] * c->boxn[2];
  if (3 * c->boxvol >= (1LL << 31)) return set_error(c, MAG_E_ARG, "sample box too large (%lld points)", c->boxvol);
  if (c->d_box) (void)hipFree(c->d_box);
  c->d_box = nullptr;
  MAG_HIP(c, hipMalloc(&c->d_box, 6 * c->boxvol * ts));
  c->warm_valid = false;
  return MAG_OK;
}

}  // namespace mag

// ================================================================= observables
namespace mag {
namespace {

// j = curl h on all faces (double) and per-block sums of the moment terms
// (1/2) r x j dV, each component of r x j summed over the faces carrying the
// current component involved; positions relative to the box centre.
__global__ void __launch_bounds__(256) bulk_obs_k(const double *__restrict__ h, double *__restrict__ j, int nx,
                                                  int ny, int nz, double dx, double dy, double dz, double Lx,
                                                  double Ly, double Lz, double *__restrict__ part) {
  __shared__ double red[256];
  const long long N = (long long)nx * ny * nz;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double mx = 0, my = 0, mz = 0;
  if (i < N) {
    const int p = (int)(i % nx), q = (int)((i / nx) % ny), r = (int)(i / ((long long)nx * ny));
    auto at = [&](int pp, int qq, int rr) {
      return ((long long)(rr & (nz - 1)) * ny + (qq & (ny - 1))) * nx + (pp & (nx - 1));
    };
    const double *hx = h, *hy = h + N, *hz = h + 2 * N;
    const double jx = (hz[at(p, q + 1, r)] - hz[i]) / dy - (hy[at(p, q, r + 1)] - hy[i]) / dz;
    const double jy = (hx[at(p, q, r + 1)] - hx[i]) / dz - (hz[at(p + 1, q, r)] - hz[i]) / dx;
    const double jz = (hy[at(p + 1, q, r)] - hy[i]) / dx - (hx[at(p, q + 1, r)] - hx[i]) / dy;
    if (j) {
      j[i] = jx;
      j[i + N] = jy;
      j[i + 2 * N] = jz;
    }
    const double x = -Lx + p * dx, y = -Ly + q * dy, z = -Lz + r * dz;
    const double xh = x + 0.5 * dx, yh = y + 0.5 * dy, zh = z + 0.5 * dz;
    // x-face (x, yh, zh), y-face (xh, y, zh), z-face (xh, yh, z)
    mx = yh * jz - zh * jy;
    my = zh * jx - xh * jz;
    mz = xh * jy - yh * jx;
  }
  const double sx = block_sum<256>(mx, red);
  if (threadIdx.x == 0) part[3 * blockIdx.x] = sx;
  __syncthreads();
  const double sy = block_sum<256>(my, red);
  if (threadIdx.x == 0) part[3 * blockIdx.x + 1] = sy;
  __syncthreads();
  const double sz = block_sum<256>(mz, red);
  if (threadIdx.x == 0) part[3 * blockIdx.x + 2] = sz;
}

}  // namespace

int bulk_observe(mag_ctx *c, const double *state, double t, double *hz, double *j, double *m) {
  (void)t;
  const long long N = c->nnode;
  const int nb = (int)((N + 255) / 256);
  double *part = nullptr;
  MAG_HIP(c, hipMallocAsync((void **)&part, (size_t)nb * 3 * sizeof(double), c->stream));
  if (hz) MAG_HIP(c, hipMemcpyAsync(hz, state + 2 * N, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  ProfScope ps(c, K_MISC);
  hipLaunchKernelGGL(bulk_obs_k, dim3(nb), dim3(256), 0, c->stream, state, j, c->n[0], c->n[1], c->n[2], c->d[0],
                     c->d[1], c->d[2], c->L[0], c->L[1], c->L[2], part);
  MAG_HIP(c, hipGetLastError());
  std::vector<double> hp((size_t)nb * 3);
  MAG_HIP(c, hipMemcpyAsync(hp.data(), part, (size_t)nb * 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MAG_HIP(c, hipFreeAsync(part, c->stream));
  MAG_HIP(c, hipStreamSynchronize(c->stream));
  double s[3] = {0, 0, 0};
  for (int b = 0; b < nb; ++b)
    for (int a = 0; a < 3; ++a) s[a] += hp[3 * b + a];
  const double dV = c->d[0] * c->d[1] * c->d[2];
  for (int a = 0; a < 3; ++a) m[a] = 0.5 * dV * s[a];
  return MAG_OK;
}

int bulk_rhs_vjp(mag_ctx *c, const double *, double, const double *, double *, double *) {
  return set_error(c, MAG_E_STATE, "bulk VJP not available yet");
}


}  // namespace mag
