// Union of orthonormal wavelet bases as the spatial prior: W_s x = (Psi_1 x, ..., Psi_8 x) / sqrt(8),
// Psi_n the J-level periodic 2-D discrete wavelet transform with Daubechies' filter of n vanishing
// moments (the prior MUFFIN's IUWT replaces and is compared with, Sec. 3 and Sec. 4, Fig. 3).
//
// Coefficients of basis n sit in the pyramid layout of an N x N plane: after level l the
// approximation LL_l is the top-left (N / 2^l)^2 block, and the level's HL, LH and HH blocks sit to
// its right, below it and diagonally.  A level filters along the columns index first (lo/hi),
// then along the rows index (LL, LH from lo; HL, HH from hi):
//   lo[r][c] = sum_k h_k x[r][(2c + k) mod n],   hi with g_k = (-1)^k h_{F-1-k}
//   LL[r][c] = sum_k h_k lo[(2r + k) mod n][c], LH with g, HL and HH likewise from hi.
// The adjoint (= inverse, each basis being orthonormal) runs the transposes coarse to fine:
//   x[p] = sum over k with p - k even of h_k a[(p - k) / 2 mod m] + g_k d[(p - k) / 2 mod m].
//
// One launch per level.  The analysis launch of level 1 loads a tile of d once and runs all eight
// bases on it; later levels read each basis's approximation, which the previous level wrote to a
// work buffer.  The dual step of eq. (anaylsespat) is fused into the analysis epilogue:
// u <- rho sat(u + coef w) + (1 - rho) u with coef = sigma mu_s / sqrt(8).  The adjoint's finest
// level sums the eight bases in registers and writes W_s^dagger u once.
//
// Filters are built on the host from Daubechies' construction: the roots y_k of
// P_n(y) = sum_{k<n} C(n-1+k, k) y^k (Durand-Kerner iteration in long double), each mapped to the
// root z inside the unit circle of z^2 - (2 - 4y) z + 1 = 0, and h proportional to
// (1 + z)^n prod_k (z - z_k), scaled to sum sqrt(2) and ordered largest taps first.
#include "common.h"

#include <cmath>
#include <complex>
#include <type_traits>
#include <vector>

namespace mf {

namespace {

constexpr int TO = 32;                      // output coefficients per analysis tile side
constexpr int FMAX = 2 * kUobBases;         // longest filter (8 vanishing moments: 16 taps)
constexpr int SA = 2 * TO + FMAX - 2;       // input rows / columns of an analysis tile
constexpr int TA = 64;                      // output pixels per adjoint tile side
constexpr int CWA = TA / 2 + FMAX / 2 + 1;  // coefficient rows / columns of an adjoint tile
constexpr int NOUT = (TO * TO + 255) / 256; // analysis outputs per thread
constexpr int NLD = (SA * SA + 255) / 256;  // analysis tile entries per thread
constexpr int NPPH = (TA / 2 * TA / 2 + 255) / 256;  // adjoint output pixel pairs per thread and half tile
constexpr int NPP = 2 * NPPH;                          // ... and per tile
constexpr int kUobAllBasesBlocks = 2048;  // blocks a level needs before one block runs all bases

__device__ __forceinline__ float satf_u(float u) { return fminf(1.f, fmaxf(-1.f, u)); }
// v mod n in [0, n) for any v
__device__ __forceinline__ int wrap_any(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}
// v mod n for v in [-n, 2n): two selects, no branch
__device__ __forceinline__ int wrap_once(int v, int n) {
  v += v < 0 ? n : 0;
  return v >= n ? v - n : v;
}
// i / d for 0 <= i < 2^20 and 1 <= d <= 2^10 through the float reciprocal of d: the quotient's
// error stays below 0.5 / d, so rounding i + 1/2 down gives the exact floor
__device__ __forceinline__ int div_small(int i, float inv_d) { return (int)(((float)i + 0.5f) * inv_d); }

// Calls fn with the filter length F (2, 4, ..., 16) as a compile-time constant, so that the tap
// loops unroll and the taps of the block's basis sit in scalar registers.
template <class Fn>
__device__ __forceinline__ void with_len(int F, Fn&& fn) {
  switch (F) {
    case 2: fn(std::integral_constant<int, 2>{}); break;
    case 4: fn(std::integral_constant<int, 4>{}); break;
    case 6: fn(std::integral_constant<int, 6>{}); break;
    case 8: fn(std::integral_constant<int, 8>{}); break;
    case 10: fn(std::integral_constant<int, 10>{}); break;
    case 12: fn(std::integral_constant<int, 12>{}); break;
    case 14: fn(std::integral_constant<int, 14>{}); break;
    default: fn(std::integral_constant<int, 16>{}); break;
  }
}

// ------------------------------------------------------------------ analysis (one level)
// Grid: x = tiles of the level's m x m output, y = channel, z = basis, or z = 1 for a block that
// runs all bases on its tile (the level's input then either is shared by all bases, level 1, or
// is each basis's own approximation, whose next tile is loaded while the current basis is
// filtered).  MODE: UOB_DUAL (dual step into U), UOB_STORE (coefficients times scale into out),
// UOB_ABS (FP64 sum of |coefficient| times scale into partial).
template <int MODE>
__global__ void __launch_bounds__(256) k_uob_an(UobLevelArgs a) {
  __shared__ float tin[SA][SA + 1];
  __shared__ float lo[SA][TO + 1], hi[SA][TO + 1];
  const int n = a.n, m = n >> 1;
  const int to = m < TO ? m : TO;
  const float inv_to = 1.f / (float)to;
  const int tiles_x = (m + to - 1) / to;
  const int R0 = (blockIdx.x / tiles_x) * to, C0 = (blockIdx.x % tiles_x) * to;
  const int l = blockIdx.y;
  const bool shared = a.shared_input != 0;
  const bool all_bases = gridDim.z == 1;
  const int b_first = all_bases ? 0 : blockIdx.z, b_last = all_bases ? kUobBases : blockIdx.z + 1;
  // input tile: rows 2R0 .. 2R0 + S - 1 (mod n), same for columns, S set by the longest filter;
  // 2R0 + S - 1 < 2n once n >= SA.  Entry i = tid + 256 q of the tile (row i / S, column i mod S)
  // is the same plane offset for every basis: computed once.
  const int S = 2 * to + FMAX - 2;
  const float inv_S = 1.f / (float)S;
  const bool one_wrap = n >= SA;
  int toff[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    int i = threadIdx.x + 256 * q;
    i = i < S * S ? i : S * S - 1;
    const int r = div_small(i, inv_S), c = i - r * S;
    const int gy = one_wrap ? wrap_once(2 * R0 + r, n) : wrap_any(2 * R0 + r, n);
    const int gx = one_wrap ? wrap_once(2 * C0 + c, n) : wrap_any(2 * C0 + c, n);
    toff[q] = MF_CHK(gy, n) * a.in_ld + MF_CHK(gx, n);
  }
  float treg[NLD];  // a tile in registers, on its way to LDS
  auto fetch_tile = [&](int b) __attribute__((always_inline)) {
    const float* base = a.in + (long long)l * a.in_cs + (long long)b * a.in_bs;
#pragma unroll
    for (int q = 0; q < NLD; ++q) treg[q] = base[toff[q]];
  };
  auto put_tile = [&](int tid) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int i = tid + 256 * q;
      if (i < S * S) {
        const int r = div_small(i, inv_S);
        tin[MF_CHK(r, S)][MF_CHK(i - r * S, S)] = treg[q];
      }
    }
  };
  double acc = 0.0;
  // the dual-plane entries a thread updates (HL, LH, HH, and LL at the coarsest level), one basis
  // ahead of the filtering
  float unext[NOUT][4];
  auto fetch_u = [&](int b, int tid) __attribute__((always_inline)) {
    const float* U = a.U + (long long)l * a.u_cs + (long long)b * a.u_bs;
#pragma unroll
    for (int q = 0; q < NOUT; ++q) {
      const int i = tid + 256 * q;
      const int r = div_small(i, inv_to), c = i - r * to;
      const bool ok = i < to * to && R0 + r < m && C0 + c < m;
      const int gr = MF_CHK(ok ? R0 + r : 0, m), gc = MF_CHK(ok ? C0 + c : 0, m);
      unext[q][0] = U[(long long)gr * a.N + m + gc];
      unext[q][1] = U[(long long)(m + gr) * a.N + gc];
      unext[q][2] = U[(long long)(m + gr) * a.N + m + gc];
      unext[q][3] = a.last ? U[(long long)gr * a.N + gc] : 0.f;
    }
  };
  if constexpr (MODE == UOB_DUAL) fetch_u(b_first, threadIdx.x);
  fetch_tile(b_first);
#pragma unroll 1
  for (int b = b_first; b < b_last; ++b) {
    // the thread index, opaque to the compiler inside the basis loop: the addresses are
    // recomputed per basis instead of being hoisted out of the loop into registers
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    // tin is read by the row pass only, which every wave has left (barrier before the column pass)
    if (b == b_first || !shared) put_tile(tid);
    if (!shared && b + 1 < b_last) fetch_tile(b + 1);
    const long long pb = (long long)l * a.u_cs + (long long)b * a.u_bs;
    float uold[NOUT][4];  // this basis's dual entries; the next basis's are fetched into unext
    if constexpr (MODE == UOB_DUAL) {
#pragma unroll
      for (int q = 0; q < NOUT; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) uold[q][t] = unext[q][t];
      if (b + 1 < b_last) fetch_u(b + 1, tid);
    }
    lds_barrier();
    with_len(a.f.len[b], [&](auto Fc) {
      constexpr int F = decltype(Fc)::value;
      float hk[F], gk[F];
#pragma unroll
      for (int k = 0; k < F; ++k) hk[k] = a.f.h[b][k], gk[k] = a.f.g[b][k];
      const int Sr = 2 * to + F - 2;
      // along the columns index: lo / hi for every loaded row
      for (int i = tid; i < Sr * to; i += 256) {
        const int r = div_small(i, inv_to), c = i - r * to;
        float sl = 0.f, sh = 0.f;
#pragma unroll
        for (int k = 0; k < F; ++k) {
          const float v = tin[MF_CHK(r, S)][MF_CHK(2 * c + k, S)];
          sl = fmaf(hk[k], v, sl);
          sh = fmaf(gk[k], v, sh);
        }
        lo[MF_CHK(r, SA)][MF_CHK(c, to)] = sl;
        hi[r][c] = sh;
      }
      lds_barrier();
      // along the rows index: the four subbands of each output coefficient of the tile
#pragma unroll
      for (int q = 0; q < NOUT; ++q) {
        const int i = tid + 256 * q;
        const int r = div_small(i, inv_to), c = i - r * to;
        const int gr = R0 + r, gc = C0 + c;
        if (i >= to * to || gr >= m || gc >= m) continue;
        float ll = 0.f, lh = 0.f, hl = 0.f, hh = 0.f;
#pragma unroll
        for (int k = 0; k < F; ++k) {
          const float vl = lo[MF_CHK(2 * r + k, Sr)][MF_CHK(c, to)], vh = hi[2 * r + k][c];
          ll = fmaf(hk[k], vl, ll);
          lh = fmaf(gk[k], vl, lh);
          hl = fmaf(hk[k], vh, hl);
          hh = fmaf(gk[k], vh, hh);
        }
        // pyramid positions in the N x N plane of basis b: HL (gr, m + gc), LH (m + gr, gc), HH (m + gr, m + gc)
        const long long pos[3] = {(long long)gr * a.N + m + gc, (long long)(m + gr) * a.N + gc,
                                  (long long)(m + gr) * a.N + m + gc};
        const float w[3] = {hl, lh, hh};
        const long long lpos = (long long)gr * a.N + gc;
#ifdef MF_CHECKED
        for (int t = 0; t < 3; ++t) (void)MF_CHK(pos[t], (long long)a.N * a.N);
#endif
        if constexpr (MODE == UOB_DUAL) {
#pragma unroll
          for (int t = 0; t < 3; ++t) {
            const float u = uold[q][t];
            a.U[pb + pos[t]] = a.rho * satf_u(u + a.coef * w[t]) + (1.f - a.rho) * u;
          }
          if (a.last) {
            const float u = uold[q][3];
            a.U[pb + lpos] = a.rho * satf_u(u + a.coef * ll) + (1.f - a.rho) * u;
          }
        } else if constexpr (MODE == UOB_STORE) {
          float* op = a.out + (long long)l * a.out_cs + (long long)b * a.out_bs;
#pragma unroll
          for (int t = 0; t < 3; ++t) op[pos[t]] = a.scale * w[t];
          if (a.last) op[lpos] = a.scale * ll;
        } else {
#pragma unroll
          for (int t = 0; t < 3; ++t) acc += fabs((double)(a.scale * w[t]));
          if (a.last) acc += fabs((double)(a.scale * ll));
        }
        if (!a.last)
          a.llout[(long long)l * a.ll_cs + (long long)b * a.ll_bs + MF_CHK((long long)gr * m + gc, (long long)m * m)] = ll;
      }
    });
    // lo / hi (and an unshared tin) are next written after this wave has passed the barrier
    // between the row and column passes, and read after the next barrier
  }
  if constexpr (MODE == UOB_ABS) {
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0)
      a.partial[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
  }
}

// ------------------------------------------------------------------ adjoint (one level)
// Level with coefficient side m and output side n = 2m, tiles of TA x TA output pixels.  The
// approximation comes from in (row stride in_ld; at the coarsest level, the LL block of the dual
// planes), the details from the dual planes' level blocks.  ACCUM: the output level is the image;
// the eight bases are summed in registers and written once, times scale.  Otherwise the output is
// the next finer approximation of each basis, for one basis (grid z = basis) or all of them.
//
// Output pixel p takes the taps k of its own parity: coefficient (p - k) / 2 = (p - par) / 2 - kk
// for k = 2 kk + par, par = p mod 2.  The two pixels 2j and 2j + 1 read the same coefficients, so
// a thread computes them together: every LDS read feeds two FMAs, taps stay in scalar registers.
template <bool ACCUM>
__global__ void __launch_bounds__(256) k_uob_adj(UobLevelArgs a) {
  __shared__ float cf[4][CWA][CWA + 1];  // LL, LH, HL, HH coefficient tiles
  __shared__ float lo[TA / 2][CWA + 1], hi[TA / 2][CWA + 1];  // one half of the tile's rows
  const int m = a.n >> 1, n = a.n;
  const int to = n < TA ? n : TA;
  const int HR = ((to >> 1) + 1) & ~1;  // output rows per half (even; TA / 2 for full tiles)
  const float inv_hto = 1.f / (float)(to >> 1);
  const int tiles_x = (n + to - 1) / to;
  const int R0 = (blockIdx.x / tiles_x) * to, C0 = (blockIdx.x % tiles_x) * to;
  const int l = blockIdx.y;
  // coefficient index range of the tile along each axis: i0 .. i0 + CWA - 1 (mod m), with
  // i0 >= -FMAX / 2 and i0 + CWA - 1 <= m once m >= CWA
  const int i0t = (R0 - FMAX) / 2, j0t = (C0 - FMAX) / 2;
  const bool one_wrap = m >= CWA;
  const bool all_bases = gridDim.z == 1;  // always with ACCUM
  const int b_first = all_bases ? 0 : blockIdx.z, b_last = all_bases ? kUobBases : blockIdx.z + 1;
  float accv[NPP][2];
#pragma unroll
  for (int q = 0; q < NPP; ++q) accv[q][0] = accv[q][1] = 0.f;
  // Staging of the four coefficient tiles of a basis: wave w loads subband w (LL, LH, HL, HH), one
  // tile row per load, one column per lane (lanes past CWA load column CWA - 1 and discard it).
  // A row's source address is wave-uniform; a lane's column is fixed.
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cl = lane < CWA ? lane : CWA - 1;
  const int gc = MF_CHK(one_wrap ? wrap_once(j0t + cl, m) : wrap_any(j0t + cl, m), m);
  // the subband's rows within its plane: the LL block of in (row stride in_ld), or the level's
  // LH (rows m.., columns 0..), HL (rows 0.., columns m..) or HH block of the dual planes
  const long long sub_off = wave == 1 ? (long long)m * a.N : wave == 2 ? (long long)m : (long long)m * a.N + m;
  const long long sub_ld = wave == 0 ? (long long)a.in_ld : (long long)a.N;
  // one basis's tile rows of this lane, in registers: the next basis's are loaded while the
  // current one is filtered (the barriers below wait for LDS traffic only)
  float creg[CWA];
  auto fetch = [&](int b, int i0) __attribute__((always_inline)) {
    const float* base = wave == 0 ? a.in + (long long)l * a.in_cs + (long long)b * a.in_bs
                                  : a.U + (long long)l * a.u_cs + (long long)b * a.u_bs + sub_off;
    int gr = wrap_any(i0, m);  // coefficient row of tile row 0, then advanced one row per load
#pragma unroll
    for (int t = 0; t < CWA; ++t) {
      creg[t] = base[(long long)MF_CHK(gr, m) * sub_ld + gc];
      gr = gr + 1 == m ? 0 : gr + 1;
    }
  };
  fetch(b_first, i0t);
#pragma unroll 1
  for (int b = b_first; b < b_last; ++b) {
    // the tile origin and the thread index, opaque to the compiler inside the basis loop: the
    // addresses are recomputed per basis instead of being hoisted out of the loop into registers
    int i0 = i0t, tid = threadIdx.x;
    asm volatile("" : "+s"(i0), "+v"(tid));
    // cf is read by the row pass only, which every wave has left (barrier before the column pass)
    if (lane < CWA) {
#pragma unroll
      for (int t = 0; t < CWA; ++t) cf[wave][t][lane] = creg[t];
    }
    lds_barrier();
    if (b + 1 < b_last) fetch(b + 1, i0);
    with_len(a.f.len[b], [&](auto Fc) {
      constexpr int H = decltype(Fc)::value / 2;
      float he[H], ho[H], ge[H], go[H];  // taps of even and odd index
#pragma unroll
      for (int kk = 0; kk < H; ++kk) {
        he[kk] = a.f.h[b][2 * kk], ho[kk] = a.f.h[b][2 * kk + 1];
        ge[kk] = a.f.g[b][2 * kk], go[kk] = a.f.g[b][2 * kk + 1];
      }
      // two halves of HR output rows each, so that lo and hi hold HR rows (a quarter of the LDS)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // along the rows index, output rows R0 + 2 rp and R0 + 2 rp + 1 together (same coefficient
        // rows ib - kk, ib = rp + FMAX / 2): lo from (LL, LH), hi from (HL, HH)
        for (int i = tid; i < (HR >> 1) * CWA; i += 256) {
          const int rl = i / CWA, c = i - rl * CWA;  // row pair within the half
          const int rp = h * (HR >> 1) + rl;
          if (2 * rp >= to) break;
          const int ib = rp + FMAX / 2;
          float le = 0.f, lodd = 0.f, hev = 0.f, hodd = 0.f;
#pragma unroll
          for (int kk = 0; kk < H; ++kk) {
            const float vll = cf[0][MF_CHK(ib - kk, CWA)][MF_CHK(c, CWA)], vlh = cf[1][ib - kk][c];
            const float vhl = cf[2][ib - kk][c], vhh = cf[3][ib - kk][c];
            le = fmaf(he[kk], vll, fmaf(ge[kk], vlh, le));
            lodd = fmaf(ho[kk], vll, fmaf(go[kk], vlh, lodd));
            hev = fmaf(he[kk], vhl, fmaf(ge[kk], vhh, hev));
            hodd = fmaf(ho[kk], vhl, fmaf(go[kk], vhh, hodd));
          }
          lo[2 * rl][c] = le;
          lo[MF_CHK(2 * rl + 1, HR)][c] = lodd;
          hi[2 * rl][c] = hev;
          hi[2 * rl + 1][c] = hodd;
        }
        lds_barrier();
        // along the columns index, output pixels C0 + 2 cp and C0 + 2 cp + 1 of row r together
        // (same columns jb - kk of lo and hi, jb = cp + FMAX / 2)
#pragma unroll
        for (int q = 0; q < NPPH; ++q) {
          const int i = tid + 256 * q;
          const int rl = div_small(i, inv_hto), cp = i - rl * (to >> 1);
          const int r = h * HR + rl;
          if (rl >= HR || r >= to) continue;
          const int jb = cp + FMAX / 2;
          float xe = 0.f, xo = 0.f;
#pragma unroll
          for (int kk = 0; kk < H; ++kk) {
            const float vl = lo[MF_CHK(rl, HR)][MF_CHK(jb - kk, CWA)], vh = hi[rl][jb - kk];
            xe = fmaf(he[kk], vl, fmaf(ge[kk], vh, xe));
            xo = fmaf(ho[kk], vl, fmaf(go[kk], vh, xo));
          }
          if (ACCUM) {
            accv[h * NPPH + q][0] += xe;
            accv[h * NPPH + q][1] += xo;
          } else if (R0 + r < n && C0 + 2 * cp < n) {
            float* o = a.llout + (long long)l * a.ll_cs + (long long)b * a.ll_bs +
                       MF_CHK((long long)(R0 + r) * n + C0 + 2 * cp, (long long)n * n - 1);
            o[0] = xe;
            o[1] = xo;
          }
        }
        if (h == 0) lds_barrier();  // the second half rewrites lo and hi
      }
    });
    // lo and hi are next written after the barrier that follows the next basis's tile store
  }
  if (ACCUM) {
#pragma unroll
    for (int q = 0; q < NPP; ++q) {
      const int i = threadIdx.x + 256 * (q % NPPH);
      const int rl = div_small(i, inv_hto), cp = i - rl * (to >> 1);
      const int r = (q / NPPH) * HR + rl;
      if (rl >= HR || r >= to) continue;
      if (R0 + r < n && C0 + 2 * cp < n) {
        float* o = a.out + (long long)l * a.out_cs + MF_CHK((long long)(R0 + r) * a.N + C0 + 2 * cp, (long long)a.N * a.N - 1);
        o[0] = a.scale * accv[q][0];
        o[1] = a.scale * accv[q][1];
      }
    }
  }
}

// ------------------------------------------------------------------ filters (host)
// Roots of sum_k c_k y^k (c_{deg} != 0) by Durand-Kerner iteration.
std::vector<std::complex<long double>> poly_roots(const std::vector<long double>& c) {
  using cd = std::complex<long double>;
  const int deg = (int)c.size() - 1;
  std::vector<cd> r(deg);
  if (deg <= 0) return r;
  for (int i = 0; i < deg; ++i) r[i] = std::pow(cd(0.4L, 0.9L), i);
  auto eval = [&](cd y) {
    cd s = 0;
    for (int k = deg; k >= 0; --k) s = s * y + c[k];
    return s / c[deg];
  };
  for (int it = 0; it < 2000; ++it) {
    long double delta = 0;
    for (int i = 0; i < deg; ++i) {
      cd den = 1;
      for (int j = 0; j < deg; ++j)
        if (j != i) den *= (r[i] - r[j]);
      const cd step = eval(r[i]) / den;
      r[i] -= step;
      delta = std::max(delta, std::abs(step));
    }
    if (delta < 1e-18L) break;
  }
  return r;
}

std::vector<double> daubechies_lowpass(int n) {
  using cd = std::complex<long double>;
  std::vector<long double> coef(n);
  for (int k = 0; k < n; ++k) {
    long double bin = 1;  // C(n - 1 + k, k)
    for (int i = 1; i <= k; ++i) bin = bin * (n - 1 + i) / i;
    coef[k] = bin;
  }
  std::vector<cd> poly{cd(1)};
  auto mul = [&](cd c0, cd c1) {  // poly *= (c0 + c1 z)
    std::vector<cd> out(poly.size() + 1, cd(0));
    for (size_t i = 0; i < poly.size(); ++i) {
      out[i] += poly[i] * c0;
      out[i + 1] += poly[i] * c1;
    }
    poly.swap(out);
  };
  for (int i = 0; i < n; ++i) mul(cd(1), cd(1));
  for (const cd& y : poly_roots(coef)) {
    // z^2 - (2 - 4y) z + 1 = 0: the two roots are reciprocal; keep the one inside the unit circle
    const cd bq = -(cd(2) - cd(4) * y);
    const cd disc = std::sqrt(bq * bq - cd(4));
    cd z1 = (-bq + disc) / cd(2), z2 = (-bq - disc) / cd(2);
    const cd z = std::abs(z1) < std::abs(z2) ? z1 : z2;
    mul(-z, cd(1));
  }
  std::vector<long double> h(poly.size());
  long double sum = 0;
  for (size_t i = 0; i < poly.size(); ++i) {
    h[i] = poly[i].real();
    sum += h[i];
  }
  std::vector<double> out(h.size());
  for (size_t i = 0; i < h.size(); ++i) out[i] = (double)(h[i] * std::sqrt(2.0L) / sum);
  if (std::fabs(out.front()) < std::fabs(out.back())) std::reverse(out.begin(), out.end());
  return out;
}

}  // namespace

UobFilters uob_filters() {
  UobFilters f{};
  for (int b = 0; b < kUobBases; ++b) {
    const std::vector<double> h = daubechies_lowpass(b + 1);
    const int F = (int)h.size();
    f.len[b] = F;
    for (int k = 0; k < F; ++k) {
      f.h[b][k] = (float)h[k];
      f.g[b][k] = (float)((k & 1) ? -h[F - 1 - k] : h[F - 1 - k]);
    }
  }
  return f;
}

int uob_lowpass(int n, double* h, int len) {
  if (n < 1 || n > kUobBases || !h || len < 2 * n) return set_error("uob_lowpass: bad arguments"), MUFFIN_EINVAL;
  const std::vector<double> v = daubechies_lowpass(n);
  for (int k = 0; k < 2 * n; ++k) h[k] = v[k];
  return MUFFIN_OK;
}

int launch_uob_an(int mode, const UobLevelArgs& a, int nch, double* partial, int* nblocks_out, hipStream_t st) {
  const int m = a.n >> 1;
  const int to = m < TO ? m : TO;
  const int tiles = ((m + to - 1) / to) * ((m + to - 1) / to);
  // one block per (tile, channel) runs all bases when that still gives the chip several blocks per
  // slot; otherwise one block per basis
  const bool all_bases = a.shared_input || (a.all_bases < 0 ? (long long)tiles * nch >= kUobAllBasesBlocks : a.all_bases != 0);
  const dim3 grid((unsigned)tiles, (unsigned)nch, all_bases ? 1u : (unsigned)kUobBases);
  if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y * grid.z);
  if (mode == UOB_ABS && (long long)grid.x * grid.y * grid.z > kMaxPartials)
    return set_error("uob: too many blocks for the partial sums"), MUFFIN_EINVAL;
  UobLevelArgs b = a;
  b.partial = partial;
  switch (mode) {
    case UOB_DUAL: hipLaunchKernelGGL(k_uob_an<UOB_DUAL>, grid, dim3(256), 0, st, b); break;
    case UOB_STORE: hipLaunchKernelGGL(k_uob_an<UOB_STORE>, grid, dim3(256), 0, st, b); break;
    case UOB_ABS: hipLaunchKernelGGL(k_uob_an<UOB_ABS>, grid, dim3(256), 0, st, b); break;
    default: return set_error("uob: bad mode"), MUFFIN_EINVAL;
  }
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int launch_uob_adj(bool accum, const UobLevelArgs& a, int nch, hipStream_t st) {
  const int n = a.n;
  const int to = n < TA ? n : TA;
  const int tiles = ((n + to - 1) / to) * ((n + to - 1) / to);
  const bool all_bases = accum || (a.all_bases < 0 ? (long long)tiles * nch >= kUobAllBasesBlocks : a.all_bases != 0);
  const dim3 grid((unsigned)tiles, (unsigned)nch, all_bases ? 1u : (unsigned)kUobBases);
  if (accum) hipLaunchKernelGGL(k_uob_adj<true>, grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_uob_adj<false>, grid, dim3(256), 0, st, a);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

#ifdef MF_CHECKED
int oob_take_uob(unsigned long long* n) { return oob_take_here(n); }
#endif

}  // namespace mf
