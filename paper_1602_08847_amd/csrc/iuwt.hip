// Isotropic undecimated wavelet transform (B3-spline a trous, periodic boundary) building blocks.
//
// H_j is the separable smoothing by [1, 4, 6, 4, 1] / 16 with taps s = 2^j apart along each axis.
// Every kernel is the band kernel below with a fused epilogue:
//   SM_SMOOTH      out = H_j A                           (c_{j+1} = H_j c_j)
//   SM_SUBADD      out = E + H_j (A - B)                 (adjoint Horner step)
//   SM_DETAIL      w = E - H_j A, u <- rho sat(u + coef w) + (1 - rho) u     (second generation)
//   SM_DETAIL_ABS  partial = sum |E - H_j A|             (objective, FP64)
//   SM_DETAIL1     out2 = H_j A and u update with w = A - H_j A              (first generation)
//   DB_ANALYSIS    c' = H_j c (written to out2), w = c - H_j c', u update     (second generation)
//   DB_ADJOINT     out = u + H_j (a - H_j u)  (A = u, B = a)                  (second generation)
//   DB_ANALYSIS_C  DB_ANALYSIS whose c' feeds the coarse plane's dual update (out2 = that plane)
//                  instead of being stored: the last scale of the analysis
// Workgroups are ordered so that each XCD (blocks b, b + 8, ...) walks a contiguous range of
// bands, keeping neighbouring bands' edge rows in its own L2.
#include "common.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

namespace mf {

__device__ __forceinline__ float satf(float u) { return fminf(1.f, fmaxf(-1.f, u)); }

__device__ __forceinline__ double block_sum_atrous(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;
}

struct AtrousArgs {
  PlaneRef A, B, E, F;
  PlaneOut out, out2, out3, out4;
  int N, j, TX, TY;
  int tiles_x, tiles_per_ch, nblocks;
  float coef, rho, coef2;
  double* partial;
  // the residue classes mod 2^j of a band are split over ncg workgroups (0 or 1: one workgroup
  // per band); tiles_per_ch counts (band, class group) tiles
  int ncg;
};

// The rounding of the filter and of the dual update is written out (the power-of-two weights scale
// exactly, the 3/8 tap and the step are fused): every kernel, whichever way the compiler lays out its
// inlined copies, then rounds them alike, which keeps the one-scale and fused launches bit-identical.
__device__ __forceinline__ float b3(float c0, float c1, float c2, float c3, float c4) {
  return __builtin_fmaf(0.375f, c2, 0.0625f * (c0 + c4) + 0.25f * (c1 + c3));
}

// relaxed dual update rho * sat(u + coef w) + (1 - rho) u
__device__ __forceinline__ float dual_upd(float u, float w, float coef, float rho) {
  return __builtin_fmaf(rho, satf(__builtin_fmaf(coef, w, u)), (1.f - rho) * u);
}

// Band kernel: one workgroup of N threads owns rows [y0, y0 + TY) of one channel, thread x owns
// column x.  Rows are visited residue class by residue class modulo s, so the vertical 5-tap
// filter is a sliding window of five registers fed by one coalesced row load per step (the first
// four steps of a class only fill the window).  Steps are grouped in rounds of KR; the KR vertical
// results of a round go through LDS for the horizontal taps (x +- s, x +- 2s, periodic).  Double-
// smoothing modes chain a second window over the first stage's output in the same class, two
// steps behind, which extends the first stage by 2s rows on each side of the band.
//
// The schedule is kept cheap for the scalar unit, which issues the uniform bookkeeping of all the
// waves of a SIMD: each class is padded to whole rounds, so every step loads, filters and shifts
// its windows the same way and only the stores test whether the step is a real output; the rows
// of the load streams are byte offsets advanced by s rows per step with one conditional wrap (a
// full modulo is taken once per class).  The next round's loads are all issued before the current
// round is computed, so their latency overlaps the LDS passes and barriers.
template <int KR>
struct BandPre {
  float a[KR], b[KR], e[KR], u[KR], u2[KR];
};

template <int MODE, int KR>
__device__ __forceinline__ void band_body(const AtrousArgs& a) {
  constexpr bool ANA = (MODE == DB_ANALYSIS || MODE == DB_ANALYSIS_C);
  constexpr bool DBL = (ANA || MODE == DB_ADJOINT);
  // which load streams a mode has: a at step row (t - 2)s, e at (t - 4)s, u at (t - 4)s or, for the
  // analysis, (t - 6)s (the stage-2 row)
  constexpr bool LB = (MODE == SM_SUBADD);
  constexpr bool LE = (MODE == SM_SUBADD || MODE == SM_DETAIL || MODE == SM_DETAIL_ABS || MODE == DB_ADJOINT);
  constexpr bool LU = (MODE == SM_DETAIL || MODE == SM_DETAIL1);
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  float* buf1 = sm;                            // [2][KR][N] single stage, [KR][N] double
  float* buf2 = sm + (DBL ? KR : 2 * KR) * N;  // [KR][N]
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, tile = b - ch * a.tiles_per_ch;
  // tile = (band, class group): the workgroup runs classes [r_lo, r_hi) of its band's rows
  const int ncg = a.ncg > 1 ? a.ncg : 1;
  const int band = tile / ncg, r_lo = (tile - band * ncg) * (s / ncg), r_hi = r_lo + s / ncg;
  const int y0 = band * TY, y1 = y0 + TY;
  const int E1 = DBL ? 2 * s : 0;
  const char* __restrict__ A = reinterpret_cast<const char*>(a.A.p + ch * a.A.cs);
  const char* __restrict__ B =
      (MODE == SM_SUBADD || MODE == DB_ADJOINT) ? reinterpret_cast<const char*>(a.B.p + ch * a.B.cs) : nullptr;
  const char* __restrict__ E = (MODE == SM_SUBADD || MODE == SM_DETAIL || MODE == SM_DETAIL_ABS)
                                   ? reinterpret_cast<const char*>(a.E.p + ch * a.E.cs)
                                   : nullptr;
  float* __restrict__ O = a.out.p ? a.out.p + ch * a.out.cs : nullptr;
  float* __restrict__ O2 = a.out2.p ? a.out2.p + ch * a.out2.cs : nullptr;
  const int xm2 = ((x - 2 * s) % N + N) % N, xm1 = ((x - s) % N + N) % N;
  const int xp1 = (x + s) % N, xp2 = (x + 2 * s) % N;
  // bytes; a step of s rows is a step of s mod N rows on the periodic plane
  const int rowb = N * 4, planeb = N * N * 4, stepb = (s % N) * rowb;
  const unsigned xb = (unsigned)x * 4u;
  auto at = [&](const char* base, int off) -> float {
    return *reinterpret_cast<const float*>(base + MF_CHK(off, planeb) + xb);
  };
  auto put = [&](float* base, int y, float v) {  // row y of the band
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + MF_CHK(y, N) * rowb + xb) = v;
  };
  // class r: stage-1 outputs at rows first(r) + m s, m < M1(r); steps t = m + 4, padded to rounds
  auto nsteps = [&](int r) -> int {
    const int v = TY + 2 * E1 - r;
    return v > 0 ? ((v + s - 1) >> jj) + 4 : 0;
  };
  auto padded = [&](int ns) -> int { return (ns + KR - 1) / KR * KR; };
  auto rowoff = [&](int y) -> int {  // byte offset of row y mod N
    y %= N;
    return (y < 0 ? y + N : y) * rowb;
  };
  auto adv = [&](int& o) {
    o += stepb;
    if (o >= planeb) o -= planeb;
  };
  // load stream: the next round to load is steps [lt, lt + KR) of class lr
  int lr = 0, lt = 0, oa = 0, oe = 0, ou = 0;
  auto start_class = [&](int r) {
    const int f = y0 + r - E1;
    oa = rowoff(f - 2 * s);
    if constexpr (LE || LU || MODE == DB_ANALYSIS_C) oe = rowoff(f - 4 * s);
    if constexpr (ANA) ou = rowoff(f - 6 * s);
  };
  auto load_round = [&](BandPre<KR>& P) {
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      P.a[kk] = at(A, oa);
      if constexpr (LB) P.b[kk] = at(B, oa);
      if constexpr (LE) P.e[kk] = at(MODE == DB_ADJOINT ? B : E, oe);
      if constexpr (LU) P.u[kk] = at(reinterpret_cast<const char*>(O), oe);
      if constexpr (ANA) P.u[kk] = at(reinterpret_cast<const char*>(O), ou);
      if constexpr (MODE == DB_ANALYSIS_C) P.u2[kk] = at(reinterpret_cast<const char*>(O2), oe);
      adv(oa);
      if constexpr (LE || LU || MODE == DB_ANALYSIS_C) adv(oe);
      if constexpr (ANA) adv(ou);
    }
  };
  auto advance_load = [&]() {
    lt += KR;
    if (lt >= padded(nsteps(lr))) {
      lt = 0;
      do {
        ++lr;
      } while (lr < r_hi && nsteps(lr) == 0);
      if (lr < r_hi) start_class(lr);
    }
  };
  double acc = 0.0;
  int round = 0;
  float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f;
  float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
  // round of steps [t0, t0 + KR) of a class with ns real steps whose first stage-1 row is first
  auto process = [&](const BandPre<KR>& cur, int t0, int ns, int first) {
    float pv[KR], cen1[KR], cen2[KR];
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      float w4 = cur.a[kk];
      if constexpr (MODE == SM_SUBADD) w4 -= cur.b[kk];
      pv[kk] = b3(w0, w1, w2, w3, w4);
      cen1[kk] = w2;
      cen2[kk] = w0;
      w0 = w1;
      w1 = w2;
      w2 = w3;
      w3 = w4;
    }
    float* L1 = buf1 + (DBL ? 0 : (round & 1) * KR * N);
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) L1[kk * N + x] = pv[kk];
    lds_barrier();
    float P[KR];
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      const float* row = L1 + kk * N;
      P[kk] = b3(row[xm2], row[xm1], row[x], row[xp1], row[xp2]);
    }
    if constexpr (!DBL) {
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int m = t0 + kk - 4;
        if (m < 0 || t0 + kk >= ns) continue;
        const int y = first + m * s;  // inside the band
        const float v = P[kk];
        if constexpr (MODE == SM_SMOOTH) {
          put(O, y, v);
        } else if constexpr (MODE == SM_SUBADD) {
          put(O, y, cur.e[kk] + v);
        } else if constexpr (MODE == SM_DETAIL || MODE == SM_DETAIL1) {
          const float e = (MODE == SM_DETAIL) ? cur.e[kk] : cen1[kk];
          const float w = e - v;
          const float u = cur.u[kk];
          put(O, y, dual_upd(u, w, a.coef, a.rho));
          if (MODE == SM_DETAIL1) put(O2, y, v);
        } else {
          acc += fabs((double)cur.e[kk] - (double)v);
        }
      }
    } else {
      float rv[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int m = t0 + kk - 4;
        float qin = P[kk];
        if constexpr (MODE == DB_ADJOINT) qin = cur.e[kk] - qin;
        if constexpr (ANA) {
          const int y = first + m * s;
          if (m >= 0 && t0 + kk < ns && y >= y0 && y < y1) {
            if constexpr (MODE == DB_ANALYSIS_C) {
              const float u2 = cur.u2[kk];
              put(O2, y, dual_upd(u2, qin, a.coef2, a.rho));
            } else {
              put(O2, y, qin);
            }
          }
        }
        rv[kk] = b3(q0, q1, q2, q3, qin);
        q0 = q1;
        q1 = q2;
        q2 = q3;
        q3 = qin;
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) buf2[kk * N + x] = rv[kk];
      lds_barrier();
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int m = t0 + kk - 4;
        if (m < 4 || t0 + kk >= ns) continue;
        const float* row = buf2 + kk * N;
        const float R = b3(row[xm2], row[xm1], row[x], row[xp1], row[xp2]);
        const int y = first + (m - 2) * s;  // stage-2 row, inside the band
        if constexpr (MODE == DB_ADJOINT) {
          put(O, y, cen2[kk] + R);
        } else {
          const float w = cen2[kk] - R;
          const float u = cur.u[kk];
          put(O, y, dual_upd(u, w, a.coef, a.rho));
        }
      }
    }
    ++round;
  };
  int r = r_lo;
  while (r < r_hi && nsteps(r) == 0) ++r;
  if (r < r_hi) {
    lr = r;
    start_class(lr);
    int pt = 0, pns = nsteps(r), pfirst = y0 + r - E1;
    BandPre<KR> cur, nxt;
    load_round(cur);
    advance_load();
    while (true) {
      // past the last class the load stream reads further rows of the plane, unused
      load_round(nxt);
      advance_load();
      process(cur, pt, pns, pfirst);
      pt += KR;
      if (pt >= padded(pns)) {
        do {
          ++r;
        } while (r < r_hi && nsteps(r) == 0);
        if (r >= r_hi) break;
        pt = 0;
        pns = nsteps(r);
        pfirst = y0 + r - E1;
      }
      cur = nxt;
    }
  }
  if constexpr (MODE == SM_DETAIL_ABS) {
    const double tot = block_sum_atrous(acc);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = tot;
  }
}

template <int MODE, int KR>
__global__ void __launch_bounds__(1024) k_band(AtrousArgs a) {
  band_body<MODE, KR>(a);
}

// The autotuner's timing launches run the same code under a symbol of their own, so that a
// profile of a run keeps the trials of other band heights apart from the iteration's launches.
template <int MODE, int KR>
__global__ void __launch_bounds__(1024) k_band_trial(AtrousArgs a) {
  band_body<MODE, KR>(a);
}

// ------------------------------------------------------------------ pairs of scales
// Two consecutive scales j, j + 1 in one pass, so the plane between them (c_{j+1} of the analysis,
// the running sum of the adjoint) never leaves the chip.  With s = 2^j the rows are visited
// residue class by residue class modulo s, where H_j has its taps 1 and 2 class steps apart and
// H_{j+1} 2 and 4: each vertical filter is a register window (5 entries for H_j, 9 for H_{j+1})
// and each horizontal filter a pass through LDS.  Load index i of class r is row
// y0 + r + (i - HALO) s; the chained stages of the second generation need HALO = 10 class steps
// of halo on either side.
//   PR_ANALYSIS:  c1 = H_j c (index t - 2 after loading c(t)), w_j = c - H_j c1 (t - 4),
//                 c2 = H_{j+1} c1 (t - 6), w_{j+1} = c1 - H_{j+1} c2 (t - 10)
//   PR_ADJOINT:   h = H_{j+1} u_{j+1} (t - 4), a' = u_{j+1} + H_{j+1}(a - h) (t - 8),
//                 a'' = u_j + H_j(a' - H_j u_j) (t - 10)
// The first generation smooths once per scale, so its pairs need 6 class steps of halo:
//   P1_ANALYSIS:  c1 = H_j c (t - 2), w_j = c - c1 (t - 2), c2 = H_{j+1} c1 (t - 6),
//                 w_{j+1} = c1 - c2 (t - 6)
//   P1_ADJOINT:   a' = u_{j+1} + H_{j+1}(a - u_{j+1}) (t - 4), a'' = u_j + H_j(a' - u_j) (t - 6)
// Every stage performs the same operations in the same order as the one-scale kernels, so the
// results are identical to running them one after the other.
template <int KR>
struct PairPre {
  float p0[KR], p1[KR], p2[KR], p3[KR];
};

template <int MODE, int KR>
__device__ __forceinline__ void pair_body(const AtrousArgs& a) {
  constexpr bool G1 = (MODE == P1_ANALYSIS || MODE == P1_ANALYSIS_C || MODE == P1_ADJOINT);
  constexpr bool ADJ = (MODE == PR_ADJOINT || MODE == P1_ADJOINT);
  constexpr bool CO = (MODE == PR_ANALYSIS_C || MODE == P1_ANALYSIS_C);
  constexpr int HALO = G1 ? 6 : 10;
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  float* bA = sm;
  float* bB = sm + KR * N;
  float* bC = sm + 2 * KR * N;
  float* bD = sm + 3 * KR * N;
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, tile = b - ch * a.tiles_per_ch;
  // tile = (band, class group): the workgroup runs classes [r_lo, r_hi) of rows [y0, y0 + TY)
  const int ncg = a.ncg > 1 ? a.ncg : 1;
  const int band = tile / ncg, cgi = tile - band * ncg;
  const int y0 = band * TY;
  const int r_lo = cgi * (s / ncg), r_hi = r_lo + s / ncg;
  const char* __restrict__ A = reinterpret_cast<const char*>(a.A.p + ch * a.A.cs);
  const char* __restrict__ Bp = ADJ ? reinterpret_cast<const char*>(a.B.p + ch * a.B.cs) : nullptr;
  const char* __restrict__ Ep = ADJ ? reinterpret_cast<const char*>(a.E.p + ch * a.E.cs) : nullptr;
  float* __restrict__ O = a.out.p + ch * a.out.cs;
  float* __restrict__ O2 = ADJ ? nullptr : a.out2.p + ch * a.out2.cs;
  float* __restrict__ O3 = ADJ ? nullptr : a.out3.p + ch * a.out3.cs;
  auto modx = [&](int v) { return (v % N + N) % N; };
  const int xm1 = modx(x - s), xm2 = modx(x - 2 * s), xm4 = modx(x - 4 * s);
  const int xp1 = modx(x + s), xp2 = modx(x + 2 * s), xp4 = modx(x + 4 * s);
  auto hj = [&](const float* row) { return b3(row[xm2], row[xm1], row[x], row[xp1], row[xp2]); };
  auto hj1 = [&](const float* row) { return b3(row[xm4], row[xm2], row[x], row[xp2], row[xp4]); };
  const int rowb = N * 4, planeb = N * N * 4, stepb = (s % N) * rowb;
  const unsigned xb = (unsigned)x * 4u;
  auto at = [&](const char* base, int off) -> float {
    return *reinterpret_cast<const float*>(base + MF_CHK(off, planeb) + xb);
  };
  auto put = [&](float* base, int y, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + MF_CHK(y, N) * rowb + xb) = v;
  };
  auto upd = [&](float u, float w, float coef) { return dual_upd(u, w, coef, a.rho); };
  auto nsteps = [&](int r) -> int {
    const int v = TY - r;
    return v > 0 ? ((v + s - 1) >> jj) + 2 * HALO : 0;
  };
  auto padded = [&](int ns) -> int { return (ns + KR - 1) / KR * KR; };
  auto rowoff = [&](int y) -> int {
    y %= N;
    return (y < 0 ? y + N : y) * rowb;
  };
  auto adv = [&](int& o) {
    o += stepb;
    if (o >= planeb) o -= planeb;
  };
  // load streams: p0 at index t, p1 at t - D1, p2 at t - D2, p3 at t - 6 (coarse plane).  Second
  // generation: p1 at t - 4, p2 at t - 6 (adjoint: u_j) or t - 10 (analysis: u_{j+1}); first
  // generation: analysis u_j at t - 2 and u_{j+1} at t - 6, adjoint a at t and u_j at t - 4
  constexpr int D1 = G1 ? (ADJ ? 0 : 2) : 4;
  constexpr int D2 = G1 ? (ADJ ? 4 : 6) : (ADJ ? 6 : 10);
  int lr = 0, lt = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0;
  auto start_class = [&](int r) {
    const int f = y0 + r - HALO * s;
    o0 = rowoff(f);
    o1 = rowoff(f - D1 * s);
    o2 = rowoff(f - D2 * s);
    if constexpr (CO) o3 = rowoff(f - 6 * s);
  };
  auto load_round = [&](PairPre<KR>& P) {
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      P.p0[kk] = at(A, o0);
      if constexpr (ADJ) {
        P.p1[kk] = at(Ep, o1);
        P.p2[kk] = at(Bp, o2);
      } else {
        P.p1[kk] = at(reinterpret_cast<const char*>(O), o1);
        P.p2[kk] = at(reinterpret_cast<const char*>(O2), o2);
        if constexpr (CO) P.p3[kk] = at(reinterpret_cast<const char*>(O3), o3);
      }
      adv(o0);
      adv(o1);
      adv(o2);
      if constexpr (CO) adv(o3);
    }
  };
  auto advance_load = [&]() {
    lt += KR;
    if (lt >= padded(nsteps(lr))) {
      lt = 0;
      do {
        ++lr;
      } while (lr < r_hi && nsteps(lr) == 0);
      if (lr < r_hi) start_class(lr);
    }
  };
  // windows, oldest first
  float wa[9], wb[9], wc[5], wd[5], we[5];
#pragma unroll
  for (int i = 0; i < 9; ++i) wa[i] = wb[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) wc[i] = wd[i] = we[i] = 0.f;
  auto push9 = [](float (&w)[9], float v) {
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = w[i + 1];
    w[8] = v;
  };
  auto push5 = [](float (&w)[5], float v) {
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = w[i + 1];
    w[4] = v;
  };
  auto v9 = [](const float (&w)[9]) { return b3(w[0], w[2], w[4], w[6], w[8]); };
  auto v5 = [](const float (&w)[5]) { return b3(w[0], w[1], w[2], w[3], w[4]); };
  // round of steps [t0, t0 + KR) of a class with ns steps whose load index 0 is row first
  auto process = [&](const PairPre<KR>& cur, int t0, int ns, int first) {
    if constexpr (G1 && ADJ) {
      // wa: a - u_{j+1} (t-8..t), wd: u_{j+1} (t-4..t), wc: a' - u_j (t-8..t-4), we: u_j (t-8..t-4)
      float pv1[KR], cuh[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        push9(wa, cur.p1[kk] - cur.p0[kk]);
        pv1[kk] = v9(wa);
        push5(wd, cur.p0[kk]);
        cuh[kk] = wd[0];
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bA[kk * N + x] = pv1[kk];
      lds_barrier();
      float pv2[KR], cul[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const float a1 = cuh[kk] + hj1(bA + kk * N);  // a' at t - 4
        push5(wc, a1 - cur.p2[kk]);
        pv2[kk] = v5(wc);
        push5(we, cur.p2[kk]);
        cul[kk] = we[2];  // u_j at t - 6
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bB[kk * N + x] = pv2[kk];
      lds_barrier();
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int t = t0 + kk;
        if (t >= 2 * HALO && t < ns) put(O, first + (t - HALO) * s, cul[kk] + hj(bB + kk * N));
      }
    } else if constexpr (G1) {
      // wc: c (t-4..t), wa: c1 (t-10..t-2)
      float pv1[KR], cc2[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        push5(wc, cur.p0[kk]);
        pv1[kk] = v5(wc);
        cc2[kk] = wc[2];
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bA[kk * N + x] = pv1[kk];
      lds_barrier();
      float pv2[KR], cc6[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int t = t0 + kk;
        const float c1 = hj(bA + kk * N);  // c1 at t - 2
        if (t >= HALO + 2 && t < ns - HALO + 2) put(O, first + (t - 2) * s, upd(cur.p1[kk], cc2[kk] - c1, a.coef));
        push9(wa, c1);
        pv2[kk] = v9(wa);
        cc6[kk] = wa[4];
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bB[kk * N + x] = pv2[kk];
      lds_barrier();
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int t = t0 + kk;
        const float c2 = hj1(bB + kk * N);  // c2 at t - 6
        if (t >= 2 * HALO && t < ns) {
          put(O2, first + (t - HALO) * s, upd(cur.p2[kk], cc6[kk] - c2, a.coef));
          if constexpr (CO) {
            put(O3, first + (t - HALO) * s, upd(cur.p3[kk], c2, a.coef2));
          } else {
            put(O3, first + (t - HALO) * s, c2);
          }
        }
      }
    } else if constexpr (ADJ) {
      // wa: u_{j+1} (t-8..t), wc: u_j (t-10..t-6), wb: a - H_{j+1} u_{j+1} (t-12..t-4),
      // wd: a' - H_j u_j (t-12..t-8)
      float pv1[KR], pv3[KR], cuh[KR], cul[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        push9(wa, cur.p0[kk]);
        pv1[kk] = v9(wa);
        cuh[kk] = wa[0];
        push5(wc, cur.p2[kk]);
        pv3[kk] = v5(wc);
        cul[kk] = wc[0];
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        bA[kk * N + x] = pv1[kk];
        bB[kk * N + x] = pv3[kk];
      }
      lds_barrier();
      float pv2[KR], h0[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const float h1 = hj1(bA + kk * N);
        h0[kk] = hj(bB + kk * N);
        push9(wb, cur.p1[kk] - h1);
        pv2[kk] = v9(wb);
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bC[kk * N + x] = pv2[kk];
      lds_barrier();
      float pv4[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const float a1 = cuh[kk] + hj1(bC + kk * N);
        push5(wd, a1 - h0[kk]);
        pv4[kk] = v5(wd);
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bD[kk * N + x] = pv4[kk];
      lds_barrier();
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int t = t0 + kk;
        if (t >= 2 * HALO && t < ns) put(O, first + (t - HALO) * s, cul[kk] + hj(bD + kk * N));
      }
    } else {
      // wc: c (t-4..t), wa: c1 (t-10..t-2), wb: c2 (t-14..t-6)
      float pv1[KR], cc4[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        push5(wc, cur.p0[kk]);
        pv1[kk] = v5(wc);
        cc4[kk] = wc[0];
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bA[kk * N + x] = pv1[kk];
      lds_barrier();
      float pv2[KR], pv3[KR], cc10[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        push9(wa, hj(bA + kk * N));
        pv2[kk] = b3(wa[4], wa[5], wa[6], wa[7], wa[8]);
        pv3[kk] = v9(wa);
        cc10[kk] = wa[0];
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        bB[kk * N + x] = pv2[kk];
        bC[kk * N + x] = pv3[kk];
      }
      lds_barrier();
      float pv4[KR];
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int t = t0 + kk;
        const float w = cc4[kk] - hj(bB + kk * N);
        if (t >= HALO + 4 && t < ns - 6) put(O, first + (t - 4) * s, upd(cur.p1[kk], w, a.coef));
        const float c2 = hj1(bC + kk * N);
        if (t >= HALO + 6 && t < ns - 4) {
          if constexpr (CO) {
            put(O3, first + (t - 6) * s, upd(cur.p3[kk], c2, a.coef2));
          } else {
            put(O3, first + (t - 6) * s, c2);
          }
        }
        push9(wb, c2);
        pv4[kk] = v9(wb);
      }
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) bD[kk * N + x] = pv4[kk];
      lds_barrier();
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) {
        const int t = t0 + kk;
        if (t >= 2 * HALO && t < ns)
          put(O2, first + (t - HALO) * s, upd(cur.p2[kk], cc10[kk] - hj1(bD + kk * N), a.coef));
      }
    }
  };
  int r = r_lo;
  while (r < r_hi && nsteps(r) == 0) ++r;
  if (r < r_hi) {
    lr = r;
    start_class(lr);
    int pt = 0, pns = nsteps(r), pfirst = y0 + r - HALO * s;
    PairPre<KR> cur, nxt;
    load_round(cur);
    advance_load();
    while (true) {
      load_round(nxt);  // past the last class: further rows of the planes, unused
      advance_load();
      process(cur, pt, pns, pfirst);
      pt += KR;
      if (pt >= padded(pns)) {
        do {
          ++r;
        } while (r < r_hi && nsteps(r) == 0);
        if (r >= r_hi) break;
        pt = 0;
        pns = nsteps(r);
        pfirst = y0 + r - HALO * s;
      }
      cur = nxt;
    }
  }
}

template <int MODE, int KR>
__global__ void __launch_bounds__(1024) k_pair(AtrousArgs a) {
  pair_body<MODE, KR>(a);
}

template <int MODE, int KR>
__global__ void __launch_bounds__(1024) k_pair_trial(AtrousArgs a) {
  pair_body<MODE, KR>(a);
}

// ------------------------------------------------------------------ triples of scales
// Three consecutive scales j, j + 1, j + 2 in one pass, in the pairs' visiting order: with s = 2^j,
// H_j, H_{j+1} and H_{j+2} have their vertical taps 1 and 2, 2 and 4, 4 and 8 class steps apart
// (windows of 5, 9 and 17 entries), one row per step.  Load index i of class r is row
// y0 + r + (i - 22) s; with c loaded at index t the one-stage-per-step schedule is
//   TR_ANALYSIS:  c1 = H_j c (index t - 2), w_j = c - H_j c1 (t - 4),
//                 c2 = H_{j+1} c1 (t - 6), w_{j+1} = c1 - H_{j+1} c2 (t - 10),
//                 c3 = H_{j+2} c2 (t - 14), w_{j+2} = c2 - H_{j+2} c3 (t - 22)
//   TR_ADJOINT:   a1 = u_{j+2} + H_{j+2}(a - H_{j+2} u_{j+2}) (t - 16),
//                 a2 = u_{j+1} + H_{j+1}(a1 - H_{j+1} u_{j+1}) (t - 20),
//                 a3 = u_j + H_j(a2 - H_j u_j) (t - 22)
// and both kernels run these stages skewed over consecutive steps (below).  As with the pairs,
// every stage repeats the one-scale kernels' operations in their order.
struct TriPre {
  float p0, p1, p2, p3, p4;
};

// compile-time step residue of an unrolled step loop
template <int P>
using Phase = std::integral_constant<int, P>;

// Analysis triple, skewed: at step T it runs stage 1 of step T, stage 2 of T - 1, ..., stage 5 of
// T - 4, each stage reading the LDS rows the stage before it wrote in the previous step (two sets
// of rows, by step parity), so one barrier per step serves all five.  With t the step a stage
// works for and c loaded at index t:
//   S1: c into the window of H_j (vertical part of c1 = H_j c at t - 2)
//   S2: c1 (t - 2); vertical parts of H_j c1 (t - 4) and of c2 = H_{j+1} c1 (t - 6)
//   S3: w_j = c - H_j c1 (t - 4) and the dual step of u_j; c2 (t - 6); vertical parts of
//       H_{j+1} c2 (t - 10) and of c3 = H_{j+2} c2 (t - 14)
//   S4: w_{j+1} = c1 - H_{j+1} c2 (t - 10) and the dual step of u_{j+1}; c3 (t - 14), stored (or
//       the coarse plane's dual step); vertical part of H_{j+2} c3 (t - 22)
//   S5: w_{j+2} = c2 - H_{j+2} c3 (t - 22) and the dual step of u_{j+2}
// c, c1 and c2 wait two steps between the stage that has them and the one that uses them (two-slot
// rings), and the u streams are loaded at the indices where their stage reaches them.  The windows
// are phase windows as in the adjoint triple (the loop is unrolled four times), and the operations
// are those of the one-scale kernels in their order.
template <int RS, bool CO>
__device__ __forceinline__ void triple_an_body(const AtrousArgs& a) {
  constexpr int HALO = 22, SKEW = 4;
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, tile = b - ch * a.tiles_per_ch;
  // tile = (band, class group): the workgroup runs classes [r_lo, r_hi) of its band's rows
  const int ncg = a.ncg > 1 ? a.ncg : 1;
  const int band = tile / ncg, r_lo = (tile - band * ncg) * (s / ncg), r_hi = r_lo + s / ncg;
  const int y0 = band * TY;
  const char* __restrict__ A = reinterpret_cast<const char*>(a.A.p + ch * a.A.cs);
  float* __restrict__ O = a.out.p + ch * a.out.cs;
  float* __restrict__ O2 = a.out2.p + ch * a.out2.cs;
  float* __restrict__ O3 = a.out3.p + ch * a.out3.cs;
  float* __restrict__ O4 = a.out4.p + ch * a.out4.cs;
  auto modx = [&](int v) { return (v % N + N) % N; };
  const int xm1 = modx(x - s), xm2 = modx(x - 2 * s), xm4 = modx(x - 4 * s), xm8 = modx(x - 8 * s);
  const int xp1 = modx(x + s), xp2 = modx(x + 2 * s), xp4 = modx(x + 4 * s), xp8 = modx(x + 8 * s);
  auto h0 = [&](const float* row) { return b3(row[xm2], row[xm1], row[x], row[xp1], row[xp2]); };
  auto h1 = [&](const float* row) { return b3(row[xm4], row[xm2], row[x], row[xp2], row[xp4]); };
  auto h2 = [&](const float* row) { return b3(row[xm8], row[xm4], row[x], row[xp4], row[xp8]); };
  const int rowb = N * 4, planeb = N * N * 4, stepb = (s % N) * rowb;
  const unsigned xb = (unsigned)x * 4u;
  auto at = [&](const char* base, int off) -> float {
    // streaming loads (the stores stay cached: the next launch reads c_{j+3})
    return ld_stream(reinterpret_cast<const float*>(base + MF_CHK(off, planeb) + xb));
  };
  auto put = [&](float* base, int y, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + MF_CHK(y, N) * rowb + xb) = v;
  };
  auto upd = [&](float u, float w, float coef) { return dual_upd(u, w, coef, a.rho); };
  auto nsteps = [&](int r) -> int {
    const int v = TY - r;
    return v > 0 ? ((v + s - 1) >> jj) + 2 * HALO + SKEW : 0;
  };
  auto rowoff = [&](int y) -> int {
    y %= N;
    return (y < 0 ? y + N : y) * rowb;
  };
  auto adv = [&](int& o) {
    o += stepb;
    if (o >= planeb) o -= planeb;
  };
  // load streams (load index of step T): p0 c (T), p1 u_j (T - 6), p2 u_{j+1} (T - 13),
  // p3 u_{j+2} (T - 26), p4 coarse plane (T - 17)
  constexpr int D1 = 6, D2 = 13, D3 = 26, D4 = 17;
  int lr = 0, lt = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0, o4 = 0;
  auto start_class = [&](int r) {
    const int f = y0 + r - HALO * s;
    o0 = rowoff(f);
    o1 = rowoff(f - D1 * s);
    o2 = rowoff(f - D2 * s);
    o3 = rowoff(f - D3 * s);
    if constexpr (CO) o4 = rowoff(f - D4 * s);
  };
  auto load_step = [&](TriPre& P) {
    P.p0 = at(A, o0);
    P.p1 = at(reinterpret_cast<const char*>(O), o1);
    P.p2 = at(reinterpret_cast<const char*>(O2), o2);
    P.p3 = at(reinterpret_cast<const char*>(O3), o3);
    if constexpr (CO) P.p4 = at(reinterpret_cast<const char*>(O4), o4);
    adv(o0);
    adv(o1);
    adv(o2);
    adv(o3);
    if constexpr (CO) adv(o4);
  };
  auto advance_load = [&]() {
    ++lt;
    if (lt >= nsteps(lr)) {
      lt = 0;
      do {
        ++lr;
      } while (lr < r_hi && nsteps(lr) == 0);
      if (lr < r_hi) start_class(lr);
    }
  };
  // windows, oldest first: c (S1), c1 by residue mod 2 (S2), c2 and c3 by residue mod 4 (S3, S4)
  float wc[5], v1[2][5], v2[4][5], v3[4][5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    wc[i] = 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) v1[q][i] = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) v2[q][i] = v3[q][i] = 0.f;
  }
  // two-step rings (slot = residue mod 2): c (S1 -> S3), c1 (S2 -> S4), c2 (S3 -> S5)
  float r0[2] = {0.f, 0.f}, r1[2] = {0.f, 0.f}, r2[2] = {0.f, 0.f};
  auto push = [](float (&w)[5], float v) {
    w[0] = w[1];
    w[1] = w[2];
    w[2] = w[3];
    w[3] = w[4];
    w[4] = v;
  };
  auto v5 = [](const float (&w)[5]) { return b3(w[0], w[1], w[2], w[3], w[4]); };
  // step T (residue P mod 4); stage k works for step T - k + 1, whose load index 0 is row first
  // of a class with ns steps (T counts within the class, which the skew does not cross: SKEW
  // extra steps at the end of every class drain it)
  auto process = [&](auto ph, const TriPre& cur, int T, int ns, int first) {
    constexpr int P = decltype(ph)::value, P2 = P & 1;
    float* wr = sm + P2 * 6 * RS;        // rows written this step
    float* rd = sm + (P2 ^ 1) * 6 * RS;  // rows written last step
    const int lo = HALO, hi = ns - HALO - SKEW;  // load indices of the band's own rows
    const float cc0 = r0[P2], cc1 = r1[P2], cc2 = r2[P2];  // written two steps ago
    // S5, step T - 4: u_{j+2} at T - 26
    {
      const float w2 = cc2 - h2(rd + 5 * RS);
      if (T - 26 >= lo && T - 26 < hi) put(O3, first + (T - 26) * s, upd(cur.p3, w2, a.coef));
    }
    __builtin_amdgcn_sched_barrier(0);
    // S4, step T - 3: u_{j+1} at T - 13, c3 at T - 17
    {
      const float w1 = cc1 - h1(rd + 3 * RS);
      if (T - 13 >= lo && T - 13 < hi) put(O2, first + (T - 13) * s, upd(cur.p2, w1, a.coef));
      const float c3 = h2(rd + 4 * RS);
      if (T - 17 >= lo && T - 17 < hi) {
        if constexpr (CO) {
          put(O4, first + (T - 17) * s, upd(cur.p4, c3, a.coef2));
        } else {
          put(O4, first + (T - 17) * s, c3);
        }
      }
      push(v3[P], c3);
      wr[5 * RS + x] = v5(v3[P]);
    }
    __builtin_amdgcn_sched_barrier(0);
    // S3, step T - 2: u_j at T - 6, c2
    {
      const float w0 = cc0 - h0(rd + RS);
      if (T - 6 >= lo && T - 6 < hi) put(O, first + (T - 6) * s, upd(cur.p1, w0, a.coef));
      const float c2 = h1(rd + 2 * RS);
      push(v2[P], c2);
      r2[P2] = v2[P][0];
      wr[3 * RS + x] = b3(v2[P][2], v2[(P + 2) & 3][3], v2[P][3], v2[(P + 2) & 3][4], v2[P][4]);
      wr[4 * RS + x] = v5(v2[P]);
    }
    __builtin_amdgcn_sched_barrier(0);
    // S2, step T - 1: c1
    {
      const float c1 = h0(rd);
      push(v1[P2], c1);
      r1[P2] = v1[P2][0];
      wr[RS + x] = b3(v1[P2][2], v1[P2 ^ 1][3], v1[P2][3], v1[P2 ^ 1][4], v1[P2][4]);
      wr[2 * RS + x] = v5(v1[P2]);
    }
    // S1, step T: c
    push(wc, cur.p0);
    r0[P2] = wc[0];
    wr[x] = v5(wc);
    lds_barrier();
  };
  int r = r_lo;
  while (r < r_hi && nsteps(r) == 0) ++r;
  if (r < r_hi) {
    lr = r;
    start_class(lr);
    int pt = 0, pns = nsteps(r), pfirst = y0 + r - HALO * s;
    auto next_step = [&]() -> bool {  // false when the band is done
      if (++pt >= pns) {
        do {
          ++r;
        } while (r < r_hi && nsteps(r) == 0);
        if (r >= r_hi) return false;
        pt = 0;
        pns = nsteps(r);
        pfirst = y0 + r - HALO * s;
      }
      return true;
    };
    // Loads three steps ahead, four buffers taking turns, so that no copy waits for a load in
    // flight.  The scheduling barriers keep each step's loads from moving up into earlier steps.
    TriPre q0, q1, q2, q3;
    load_step(q0);
    advance_load();
    load_step(q1);
    advance_load();
    load_step(q2);
    advance_load();
    while (true) {
      load_step(q3);  // past the last class: further rows of the planes, unused
      advance_load();
      process(Phase<0>{}, q0, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q0);
      advance_load();
      process(Phase<1>{}, q1, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q1);
      advance_load();
      process(Phase<2>{}, q2, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q2);
      advance_load();
      process(Phase<3>{}, q3, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// Adjoint triple with phase windows.  A window whose filter taps lie d steps apart (d = 4 for
// H_{j+2}, 2 for H_{j+1}) is kept as d windows of five entries, one per step residue mod d, and a
// step shifts only the one of its own residue: 4 register moves instead of 16 or 8.  The main loop
// is unrolled four times so that every residue, the LDS parity and the slots of the 1-, 2- and
// 4-step delay lines are compile-time constants (the 3-step line still shifts).  The values and
// the operations on them are those of the shifting form, in the same order.
// LDS rows are RS floats apart (RS >= N, a compile-time constant), so every row and slot offset is
// an instruction immediate: with the residues fixed, nothing per row has to be held in a register.
template <int RS>
__device__ __forceinline__ void triple_adj_body(const AtrousArgs& a) {
  constexpr int HALO = 22, SKEW = 4;
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, tile = b - ch * a.tiles_per_ch;
  // tile = (band, class group): the workgroup runs classes [r_lo, r_hi) of its band's rows
  const int ncg = a.ncg > 1 ? a.ncg : 1;
  const int band = tile / ncg, r_lo = (tile - band * ncg) * (s / ncg), r_hi = r_lo + s / ncg;
  const int y0 = band * TY;
  const char* __restrict__ A = reinterpret_cast<const char*>(a.A.p + ch * a.A.cs);
  const char* __restrict__ Bp = reinterpret_cast<const char*>(a.B.p + ch * a.B.cs);
  const char* __restrict__ Ep = reinterpret_cast<const char*>(a.E.p + ch * a.E.cs);
  const char* __restrict__ Fp = reinterpret_cast<const char*>(a.F.p + ch * a.F.cs);
  float* __restrict__ O = a.out.p + ch * a.out.cs;
  auto modx = [&](int v) { return (v % N + N) % N; };
  const int xm1 = modx(x - s), xm2 = modx(x - 2 * s), xm4 = modx(x - 4 * s), xm8 = modx(x - 8 * s);
  const int xp1 = modx(x + s), xp2 = modx(x + 2 * s), xp4 = modx(x + 4 * s), xp8 = modx(x + 8 * s);
  auto h0 = [&](const float* row) { return b3(row[xm2], row[xm1], row[x], row[xp1], row[xp2]); };
  auto h1 = [&](const float* row) { return b3(row[xm4], row[xm2], row[x], row[xp2], row[xp4]); };
  auto h2 = [&](const float* row) { return b3(row[xm8], row[xm4], row[x], row[xp4], row[xp8]); };
  const int rowb = N * 4, planeb = N * N * 4, stepb = (s % N) * rowb;
  const unsigned xb = (unsigned)x * 4u;
  auto at = [&](const char* base, int off) -> float {
    // streaming: every row is read once, and the new sum is next read two launches later
    return ld_stream(reinterpret_cast<const float*>(base + MF_CHK(off, planeb) + xb));
  };
  auto put = [&](float* base, int y, float v) {
    st_stream(reinterpret_cast<float*>(reinterpret_cast<char*>(base) + MF_CHK(y, N) * rowb + xb), v);
  };
  auto nsteps = [&](int r) -> int {
    const int v = TY - r;
    return v > 0 ? ((v + s - 1) >> jj) + 2 * HALO + SKEW : 0;
  };
  auto rowoff = [&](int y) -> int {
    y %= N;
    return (y < 0 ? y + N : y) * rowb;
  };
  auto adv = [&](int& o) {
    o += stepb;
    if (o >= planeb) o -= planeb;
  };
  // load streams (load index of step t): p0 u_{j+2} (t), p1 a (t - 8), p2 u_{j+1} (t - 12),
  // p3 u_j (t - 18)
  int lr = 0, lt = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0;
  auto start_class = [&](int r) {
    const int f = y0 + r - HALO * s;
    o0 = rowoff(f);
    o1 = rowoff(f - 8 * s);
    o2 = rowoff(f - 12 * s);
    o3 = rowoff(f - 18 * s);
  };
  auto load_step = [&](TriPre& P) {
    P.p0 = at(A, o0);
    P.p1 = at(Fp, o1);
    P.p2 = at(Bp, o2);
    P.p3 = at(Ep, o3);
    adv(o0);
    adv(o1);
    adv(o2);
    adv(o3);
  };
  auto advance_load = [&]() {
    ++lt;
    if (lt >= nsteps(lr)) {
      lt = 0;
      do {
        ++lr;
      } while (lr < r_hi && nsteps(lr) == 0);
      if (lr < r_hi) start_class(lr);
    }
  };
  // windows, oldest first: u_{j+2} and a - H_{j+2} u_{j+2} by residue mod 4, u_{j+1} and
  // a1 - H_{j+1} u_{j+1} by residue mod 2, u_j and a2 - H_j u_j
  float ua[4][5], ub[4][5], va[2][5], vb[2][5], wa[5], wb[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int q = 0; q < 4; ++q) ua[q][i] = ub[q][i] = 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) va[q][i] = vb[q][i] = 0.f;
    wa[i] = wb[i] = 0.f;
  }
  // delay lines: dA, dC one step, in registers; in LDS, four slots per line indexed by the residue
  // (a line of d steps reads slot P - d before step P writes slot P; each thread reads only its
  // own column): dE two steps, dU1 three, dU0 four.  u_{j+2} two steps before the oldest entry of
  // ua[P] is the oldest entry of ua[P + 2], which was last pushed two steps ago.
  float dA = 0.f, dC = 0.f;
  float* dE = sm + 12 * RS;
  float* dU1 = sm + 16 * RS;
  float* dU0 = sm + 20 * RS;
#pragma unroll
  for (int q = 0; q < 4; ++q) dE[q * RS + x] = dU1[q * RS + x] = dU0[q * RS + x] = 0.f;
  auto push = [](float (&w)[5], float v) {
    w[0] = w[1];
    w[1] = w[2];
    w[2] = w[3];
    w[3] = w[4];
    w[4] = v;
  };
  auto v5 = [](const float (&w)[5]) { return b3(w[0], w[1], w[2], w[3], w[4]); };
  // step t (residue P mod 4) of a class with ns steps whose load index 0 is row first.  At step
  // T: stage 1 of step T, stage 2 of T - 1, stage 3 of T - 2, stage 4 of T - 3 and the output of
  // T - 4, where step t is the one-step-per-stage schedule's step t.
  auto process = [&](auto ph, const TriPre& cur, int t, int ns, int first) {
    constexpr int P = decltype(ph)::value, P2 = P & 1;
    float* wr = sm + P2 * 6 * RS;        // written this step
    float* rd = sm + (P2 ^ 1) * 6 * RS;  // written last step
    // Each stage reads its horizontal filters of last step's rows just before it needs them (the
    // scheduling barriers keep the compiler from issuing all thirty LDS reads at once, which would
    // hold thirty more registers).  Stage 1 of T - 1 wrote rows 0, 2, 4; stage 2 of T - 2 row 1,
    // stage 3 of T - 3 row 3, stage 4 of T - 4 row 5.
    // stage 1, step T
    push(ua[P], cur.p0);
    push(va[P2], cur.p2);
    push(wa, cur.p3);
    wr[x] = v5(ua[P]);
    wr[2 * RS + x] = v5(va[P2]);
    wr[4 * RS + x] = v5(wa);
    __builtin_amdgcn_sched_barrier(0);
    // stage 2, step T - 1: a - H_{j+2} u_{j+2}
    const float hA = h2(rd);
    const float a_old = dA;
    dA = cur.p1;
    push(ub[P], a_old - hA);
    wr[RS + x] = v5(ub[P]);
    __builtin_amdgcn_sched_barrier(0);
    // stage 3, step T - 2: a1 = u_{j+2} + H_{j+2}(...), then a1 - H_{j+1} u_{j+1}
    const float gB = h2(rd + RS), hC = h1(rd + 2 * RS);
    const float a1 = ua[(P + 2) & 3][0] + gB;
    const float c_old = dC;
    dC = hC;
    push(vb[P2], a1 - c_old);
    wr[3 * RS + x] = v5(vb[P2]);
    __builtin_amdgcn_sched_barrier(0);
    // stage 4, step T - 3: a2 = u_{j+1} + H_{j+1}(...), then a2 - H_j u_j
    const float gD = h1(rd + 3 * RS), hE = h0(rd + 4 * RS);
    const float u1 = dU1[((P + 1) & 3) * RS + x];
    dU1[P * RS + x] = va[P2][0];
    const float a2 = u1 + gD;
    const float e_old = dE[((P + 2) & 3) * RS + x];
    dE[P * RS + x] = hE;
    push(wb, a2 - e_old);
    wr[5 * RS + x] = v5(wb);
    __builtin_amdgcn_sched_barrier(0);
    // output, step T - 4: u_j + H_j(...)
    const float gF = h0(rd + 5 * RS);
    const float u0 = dU0[P * RS + x];
    dU0[P * RS + x] = wa[0];
    const float out = u0 + gF;
    const int to = t - SKEW;
    if (to >= 2 * HALO && to < ns - SKEW) put(O, first + (to - HALO) * s, out);
    lds_barrier();
  };
  int r = r_lo;
  while (r < r_hi && nsteps(r) == 0) ++r;
  if (r < r_hi) {
    lr = r;
    start_class(lr);
    int pt = 0, pns = nsteps(r), pfirst = y0 + r - HALO * s;
    auto next_step = [&]() -> bool {  // false when the band is done
      if (++pt >= pns) {
        do {
          ++r;
        } while (r < r_hi && nsteps(r) == 0);
        if (r >= r_hi) return false;
        pt = 0;
        pns = nsteps(r);
        pfirst = y0 + r - HALO * s;
      }
      return true;
    };
    // Loads three steps ahead, four buffers taking turns, so that no copy waits for a load in
    // flight.  The scheduling barriers keep each step's loads from moving up into earlier steps.
    TriPre q0, q1, q2, q3;
    load_step(q0);
    advance_load();
    load_step(q1);
    advance_load();
    load_step(q2);
    advance_load();
    while (true) {
      load_step(q3);  // past the last class: further rows of the planes, unused
      advance_load();
      process(Phase<0>{}, q0, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q0);
      advance_load();
      process(Phase<1>{}, q1, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q1);
      advance_load();
      process(Phase<2>{}, q2, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q2);
      advance_load();
      process(Phase<3>{}, q3, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int RS, bool CO>
__global__ void __launch_bounds__(1024) k_triple_an(AtrousArgs a) {
  triple_an_body<RS, CO>(a);
}

template <int RS, bool CO>
__global__ void __launch_bounds__(1024) k_triple_an_trial(AtrousArgs a) {
  triple_an_body<RS, CO>(a);
}

template <int RS>
__global__ void __launch_bounds__(1024) k_triple_adj(AtrousArgs a) {
  triple_adj_body<RS>(a);
}

template <int RS>
__global__ void __launch_bounds__(1024) k_triple_adj_trial(AtrousArgs a) {
  triple_adj_body<RS>(a);
}

constexpr int kAdjRows = 24;  // LDS rows of the adjoint triple: 2 x 6 stage rows, 3 x 4 delay slots
constexpr int kAnRows = 12;   // LDS rows of the analysis triple: 2 x 6 stage rows
// row stride of the triples' LDS rows: the smallest of 64, 256, 1024 floats that holds a row
static int tri_row_stride(int N) { return N <= 64 ? 64 : (N <= 256 ? 256 : 1024); }

// ------------------------------------------------------------------ fused pair
// The last analysis pair of an iteration (scales j, j + 1 and the coarse plane's dual step) and
// the first adjoint pair of the next iteration, which works on exactly the planes the analysis
// has just updated, in one pass.  Stages, for analysis step t (c_j loaded at index t):
//   A1  c into the window of H_j (vertical part of c1 = H_j c at t - 2)
//   A2  c1 (t - 2); vertical parts of H_j c1 (t - 4) and of c2 = H_{j+1} c1 (t - 6)
//   A3  w_j (t - 4): new u_j; c2 (t - 6): new coarse plane u_c; vertical part of H_{j+1} c2
//   A4  w_{j+1} (t - 10): new u_{j+1}
//   B1  (adjoint index tau = t - 10) vertical parts of H_{j+1} u_{j+1} (tau - 4) and of
//       H_j u_j (tau - 8)
//   B2  h = H_{j+1} u_{j+1}; vertical part of H_{j+1}(u_c - h) (tau - 8)
//   B3  a' = u_{j+1} + H_{j+1}(u_c - h) (tau - 8); vertical part of H_j(a' - H_j u_j)
//   B4  a'' = u_j + H_j(a' - H_j u_j) (tau - 10 = t - 20)
// They are skewed like the triples: wall step T runs A1 for t = T, A2 for T - 1, A3 for T - 2, A4
// and B1 for T - 3, B2 for T - 4, B3 for T - 5 and B4 for T - 6, each stage reading the LDS rows
// its predecessor wrote in the previous step (two sets of rows, by step parity), so one barrier
// per step serves all of them.  The new u_j and u_c wait 13 and 10 steps for B1 and B2 in LDS
// rings (each thread reads back only what it wrote); the other carried values wait in registers.
// The old dual planes are read from B, E, F and the new ones written to out, out2, out3 (two
// buffers, so that a band's halo always reads old values); a'' goes to out4.  Windows are phase
// windows, the loop is unrolled four times and the LDS rows are RS floats apart (see the
// triples).  Every stage repeats the operations of the analysis pair and the adjoint pair in
// their order: planes and a'' are bit-identical to the two separate launches.
struct FusedPre {
  float p0, p1, p2, p3;
};
constexpr int kFusedDJ = 13, kFusedDC = 10;          // delays of the new u_j and u_c
constexpr int kFusedRows = 16 + kFusedDJ + kFusedDC;  // LDS rows: 2 x 8 stage rows, the two rings

template <int RS>
__device__ __forceinline__ void fused_body(const AtrousArgs& a) {
  constexpr int HALO = 20;  // 10 class steps for the analysis, 10 for the adjoint
  constexpr int SKEW = 6;   // the last stage works for the step six steps back
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  float* ringJ = sm + 16 * RS;
  float* ringC = sm + (16 + kFusedDJ) * RS;
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, tile = b - ch * a.tiles_per_ch;
  // tile = (band, class group): the workgroup runs classes [r_lo, r_hi) of its band's rows
  const int ncg = a.ncg > 1 ? a.ncg : 1;
  const int band = tile / ncg, r_lo = (tile - band * ncg) * (s / ncg), r_hi = r_lo + s / ncg;
  const int y0 = band * TY;
  const char* __restrict__ A = reinterpret_cast<const char*>(a.A.p + ch * a.A.cs);
  const char* __restrict__ Bp = reinterpret_cast<const char*>(a.B.p + ch * a.B.cs);
  const char* __restrict__ Ep = reinterpret_cast<const char*>(a.E.p + ch * a.E.cs);
  const char* __restrict__ Fp = reinterpret_cast<const char*>(a.F.p + ch * a.F.cs);
  float* __restrict__ O = a.out.p + ch * a.out.cs;
  float* __restrict__ O2 = a.out2.p + ch * a.out2.cs;
  float* __restrict__ O3 = a.out3.p + ch * a.out3.cs;
  float* __restrict__ O4 = a.out4.p + ch * a.out4.cs;
  auto modx = [&](int v) { return (v % N + N) % N; };
  const int xm1 = modx(x - s), xm2 = modx(x - 2 * s), xm4 = modx(x - 4 * s);
  const int xp1 = modx(x + s), xp2 = modx(x + 2 * s), xp4 = modx(x + 4 * s);
  auto hj = [&](const float* row) { return b3(row[xm2], row[xm1], row[x], row[xp1], row[xp2]); };
  auto hj1 = [&](const float* row) { return b3(row[xm4], row[xm2], row[x], row[xp2], row[xp4]); };
  const int rowb = N * 4, planeb = N * N * 4, stepb = (s % N) * rowb;
  const unsigned xb = (unsigned)x * 4u;
  auto at = [&](const char* base, int off) -> float {
    return *reinterpret_cast<const float*>(base + MF_CHK(off, planeb) + xb);
  };
  auto put = [&](float* base, int y, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + MF_CHK(y, N) * rowb + xb) = v;
  };
  auto upd = [&](float u, float w, float coef) { return dual_upd(u, w, coef, a.rho); };
  auto nsteps = [&](int r) -> int {
    const int v = TY - r;
    return v > 0 ? ((v + s - 1) >> jj) + 2 * HALO + SKEW : 0;
  };
  auto rowoff = [&](int y) -> int {
    y %= N;
    return (y < 0 ? y + N : y) * rowb;
  };
  auto adv = [&](int& o) {
    o += stepb;
    if (o >= planeb) o -= planeb;
  };
  // load streams (load index of wall step T): p0 c (T), p1 old u_j (T - 6), p2 old u_{j+1}
  // (T - 13), p3 old coarse plane (T - 8)
  constexpr int D1 = 6, D2 = 13, D3 = 8;
  int lr = 0, lt = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0;
  auto start_class = [&](int r) {
    const int f = y0 + r - HALO * s;
    o0 = rowoff(f);
    o1 = rowoff(f - D1 * s);
    o2 = rowoff(f - D2 * s);
    o3 = rowoff(f - D3 * s);
  };
  auto load_step = [&](FusedPre& P) {
    P.p0 = at(A, o0);
    P.p1 = at(Bp, o1);
    P.p2 = at(Ep, o2);
    P.p3 = at(Fp, o3);
    adv(o0);
    adv(o1);
    adv(o2);
    adv(o3);
  };
  auto advance_load = [&]() {
    ++lt;
    if (lt >= nsteps(lr)) {
      lt = 0;
      do {
        ++lr;
      } while (lr < r_hi && nsteps(lr) == 0);
      if (lr < r_hi) start_class(lr);
    }
  };
  // windows, oldest first (9-entry windows with taps two steps apart as two phase windows):
  // wc c (A1), wa c1 (A2), wb c2 (A3), ya new u_{j+1} (B1), yc new u_j (B1), yb u_c - h (B2),
  // yd a' - H_j u_j (B3)
  float wc[5], wa[2][5], wb[2][5], ya[2][5], yb[2][5], yc[5], yd[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    wc[i] = yc[i] = yd[i] = 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) wa[q][i] = wb[q][i] = ya[q][i] = yb[q][i] = 0.f;
  }
  // register rings: c (A1 -> A3) and c1 (A2 -> A4) two steps, u_{j+1} (B1 -> B3) two steps, u_j
  // (B1 -> B4) three steps in four slots, H_j u_j (B2 -> B3) one step in two slots
  float r4[2] = {0.f, 0.f}, r10[2] = {0.f, 0.f}, rh[2] = {0.f, 0.f}, rl[4] = {0.f, 0.f, 0.f, 0.f};
  float rh0[2] = {0.f, 0.f};
#pragma unroll
  for (int i = 0; i < kFusedDJ; ++i) ringJ[i * RS + x] = 0.f;
#pragma unroll
  for (int i = 0; i < kFusedDC; ++i) ringC[i * RS + x] = 0.f;
  int rj = 0, rc = 0;  // ring slots of the current step
  auto push = [](float (&w)[5], float v) {
    w[0] = w[1];
    w[1] = w[2];
    w[2] = w[3];
    w[3] = w[4];
    w[4] = v;
  };
  auto v5 = [](const float (&w)[5]) { return b3(w[0], w[1], w[2], w[3], w[4]); };
  // wall step T (residue P mod 4) of a class with ns steps whose load index 0 is row first
  auto process = [&](auto ph, const FusedPre& cur, int T, int ns, int first) {
    constexpr int P = decltype(ph)::value, P2 = P & 1, Q2 = P2 ^ 1;
    float* wr = sm + P2 * 8 * RS;  // rows written this step: 0..3 analysis, 4..7 adjoint
    float* rd = sm + Q2 * 8 * RS;  // rows written last step
    const int lo = HALO, hi = ns - HALO - SKEW;  // load indices of the band's own rows
    // carried values, all written before this step
    const float cc4 = r4[P2], cc10 = r10[P2], cuh = rh[P2], cul = rl[(P + 1) & 3], h0 = rh0[Q2];
    const float uj_b1 = ringJ[rj * RS + x];  // new u_j of 13 steps ago
    const float uc_b2 = ringC[rc * RS + x];  // new u_c of 10 steps ago
    // B4, t = T - 6: a'' at T - 26
    {
      const float out = cul + hj(rd + 7 * RS);
      if (T - 26 >= lo && T - 26 < hi) put(O4, first + (T - 26) * s, out);
    }
    __builtin_amdgcn_sched_barrier(0);
    // B3, t = T - 5: a' and a' - H_j u_j
    {
      const float a1 = cuh + hj1(rd + 6 * RS);
      push(yd, a1 - h0);
      wr[7 * RS + x] = v5(yd);
    }
    __builtin_amdgcn_sched_barrier(0);
    // B2, t = T - 4: u_c - H_{j+1} u_{j+1}, and H_j u_j for B3
    {
      const float h1 = hj1(rd + 4 * RS);
      rh0[P2] = hj(rd + 5 * RS);
      push(yb[P2], uc_b2 - h1);
      wr[6 * RS + x] = v5(yb[P2]);
    }
    __builtin_amdgcn_sched_barrier(0);
    // A4 and B1, t = T - 3: new u_{j+1} at T - 13, then the adjoint's vertical parts
    {
      const float nu1 = upd(cur.p2, cc10 - hj1(rd + 3 * RS), a.coef);
      if (T - 13 >= lo && T - 13 < hi) put(O2, first + (T - 13) * s, nu1);
      push(ya[P2], nu1);
      rh[P2] = ya[P2][0];
      wr[4 * RS + x] = v5(ya[P2]);
      push(yc, uj_b1);
      rl[P] = yc[0];
      wr[5 * RS + x] = v5(yc);
    }
    __builtin_amdgcn_sched_barrier(0);
    // A3, t = T - 2: new u_j at T - 6 and coarse plane at T - 8; c2
    {
      const float nuj = upd(cur.p1, cc4 - hj(rd + RS), a.coef);
      if (T - 6 >= lo && T - 6 < hi) put(O, first + (T - 6) * s, nuj);
      const float c2 = hj1(rd + 2 * RS);
      const float nuc = upd(cur.p3, c2, a.coef2);
      if (T - 8 >= lo && T - 8 < hi) put(O3, first + (T - 8) * s, nuc);
      push(wb[P2], c2);
      wr[3 * RS + x] = v5(wb[P2]);
      ringJ[rj * RS + x] = nuj;
      ringC[rc * RS + x] = nuc;
    }
    __builtin_amdgcn_sched_barrier(0);
    // A2, t = T - 1: c1
    {
      push(wa[P2], hj(rd));
      r10[P2] = wa[P2][0];
      wr[RS + x] = b3(wa[P2][2], wa[Q2][3], wa[P2][3], wa[Q2][4], wa[P2][4]);
      wr[2 * RS + x] = v5(wa[P2]);
    }
    // A1, t = T: c
    push(wc, cur.p0);
    r4[P2] = wc[0];
    wr[x] = v5(wc);
    rj = rj + 1 == kFusedDJ ? 0 : rj + 1;
    rc = rc + 1 == kFusedDC ? 0 : rc + 1;
    lds_barrier();
  };
  int r = r_lo;
  while (r < r_hi && nsteps(r) == 0) ++r;
  if (r < r_hi) {
    lr = r;
    start_class(lr);
    int pt = 0, pns = nsteps(r), pfirst = y0 + r - HALO * s;
    auto next_step = [&]() -> bool {  // false when the band is done
      if (++pt >= pns) {
        do {
          ++r;
        } while (r < r_hi && nsteps(r) == 0);
        if (r >= r_hi) return false;
        pt = 0;
        pns = nsteps(r);
        pfirst = y0 + r - HALO * s;
      }
      return true;
    };
    // loads three steps ahead, four buffers taking turns (see the triples)
    FusedPre q0, q1, q2, q3;
    load_step(q0);
    advance_load();
    load_step(q1);
    advance_load();
    load_step(q2);
    advance_load();
    while (true) {
      load_step(q3);  // past the last class: further rows of the planes, unused
      advance_load();
      process(Phase<0>{}, q0, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q0);
      advance_load();
      process(Phase<1>{}, q1, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q1);
      advance_load();
      process(Phase<2>{}, q2, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
      load_step(q2);
      advance_load();
      process(Phase<3>{}, q3, pt, pns, pfirst);
      if (!next_step()) break;
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int RS>
__global__ void __launch_bounds__(1024) k_fused(AtrousArgs a) {
  fused_body<RS>(a);
}

template <int RS>
__global__ void __launch_bounds__(1024) k_fused_trial(AtrousArgs a) {
  fused_body<RS>(a);
}

constexpr int kKR = 8;   // rows per round, single-smoothing modes
constexpr int kKR2 = 4;  // rows per round, double-smoothing modes (keeps them within 128 VGPRs)
constexpr int kKRP = 2;  // rows per round, pair kernels (keeps them within 128 VGPRs)

static int band_rows_default(int N, int j) {
  // about 32 s rows per band (band edges cost 4s or 8s extra row loads per class), at least 64
  int target = 32 << j;
  if (target < 64) target = 64;
  int TY = 1;
  while (TY * 2 <= target && TY * 2 <= N) TY *= 2;
  while (N % TY) TY >>= 1;
  return TY;
}

static bool is_pair(int mode) {
  return mode == PR_ANALYSIS || mode == PR_ANALYSIS_C || mode == PR_ADJOINT || mode == P1_ANALYSIS ||
         mode == P1_ANALYSIS_C || mode == P1_ADJOINT;
}
static bool is_triple(int mode) { return mode == TR_ANALYSIS || mode == TR_ANALYSIS_C || mode == TR_ADJOINT; }

static int triple_rows_default(int N, int j) {
  // the triples' halo is 22 s rows on either side: about 128 s rows per band, at least 256
  int target = 128 << j;
  if (target < 256) target = 256;
  int TY = 1;
  while (TY * 2 <= target && TY * 2 <= N) TY *= 2;
  while (N % TY) TY >>= 1;
  return TY;
}

static int pair_rows_default(int N, int j) {
  // the pairs' halo is 10 s rows on either side: about 64 s rows per band, at least 128
  int target = 64 << j;
  if (target < 128) target = 128;
  int TY = 1;
  while (TY * 2 <= target && TY * 2 <= N) TY *= 2;
  while (N % TY) TY >>= 1;
  return TY;
}

// Band heights chosen by the autotuner, per (N, scale, kernel class); process-wide.
static std::mutex g_tune_mu;
static std::map<long long, int> g_tune;
static long long tune_key(int N, int j, int cls) { return ((long long)N << 16) | (j << 8) | cls; }

int atrous_class(int mode) {
  switch (mode) {
    case DB_ANALYSIS:
    case DB_ANALYSIS_C: return 0;
    case DB_ADJOINT: return 1;
    case SM_DETAIL1: return 2;
    case SM_SUBADD: return 3;
    case PR_ANALYSIS:
    case PR_ANALYSIS_C: return 5;
    case PR_ADJOINT: return 6;
    case TR_ANALYSIS:
    case TR_ANALYSIS_C: return 7;
    case TR_ADJOINT: return 8;
    case PR_FUSED: return 9;
    case P1_ANALYSIS:
    case P1_ANALYSIS_C: return 10;
    case P1_ADJOINT: return 11;
    default: return 4;
  }
}

int atrous_band_rows(int N, int j, int mode) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(N, j, atrous_class(mode)));
  if (it != g_tune.end()) return it->second;
  if (is_triple(mode) || mode == PR_FUSED) return triple_rows_default(N, j);  // halos of 21 and 22 steps
  return is_pair(mode) ? pair_rows_default(N, j) : band_rows_default(N, j);
}

// For a launch over nch channels: without a tuned value, the default band height is halved (down
// to 16 rows, as long as it divides N) while the launch would have fewer than kMinBandWaves waves
// (N / 64 waves per band), so that few channels of a small image still fill the GPU; the
// autotuner's measurements on such sizes pick heights of that order.
// A launch first splits each band's residue classes mod 2^j over more workgroups (class groups, up
// to 8): that adds no halo rows, where a lower band adds a halo per class.  The objective's
// reduction (one partial sum per workgroup) keeps one workgroup per band.
constexpr long long kMinBandWaves = 2048;
constexpr int kMaxClassGroups = 8;
static void default_tiles(int N, int j, int mode, int nch, int& TY, int& ncg) {
  TY = atrous_band_rows(N, j, mode);
  ncg = 1;
  const int maxg = mode != SM_DETAIL_ABS ? std::min(1 << j, kMaxClassGroups) : 1;
  const long long wpb = (N + 63) / 64;
  while ((long long)nch * (N / TY) * ncg * wpb < kMinBandWaves) {
    if (ncg < maxg) ncg *= 2;
    else if (TY > 16 && N % (TY / 2) == 0) TY /= 2;
    else break;
  }
}

int atrous_band_rows(int N, int j, int mode, int nch) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(N, j, atrous_class(mode)));
    if (it != g_tune.end()) return it->second;
  }
  int TY, ncg;
  default_tiles(N, j, mode, nch, TY, ncg);
  return TY;
}

int atrous_set_band_rows(int N, int j, int mode, int TY) {
  if (TY != 0 && (TY < 1 || TY > N || N % TY)) return set_error("band rows must divide N"), MUFFIN_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (TY == 0) g_tune.erase(tune_key(N, j, atrous_class(mode)));
  else g_tune[tune_key(N, j, atrous_class(mode))] = TY;
  return MUFFIN_OK;
}

// Class groups (the residue classes mod 2^j of a band split over that many workgroups): with tuned
// band rows, the tuned groups (1 if none were recorded); else the default.
static std::map<long long, int> g_tune_cg;

// Both choices for one kernel class (the codes of atrous_class) at once, as a caller restores them.
int atrous_set_tiles(int N, int j, int cls, int TY, int ncg) {
  if (cls < 0 || cls > 11 || cls == 4) return set_error("band tiles: unknown kernel family"), MUFFIN_EINVAL;
  if (TY != 0 && (TY < 1 || TY > N || N % TY)) return set_error("band rows must divide N"), MUFFIN_EINVAL;
  if (ncg != 0 && (ncg < 1 || ncg > std::min(1 << j, kMaxClassGroups) || (ncg & (ncg - 1))))
    return set_error("class groups must be a power of two up to min(2^j, 8)"), MUFFIN_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const long long k = tune_key(N, j, cls);
  if (TY == 0) g_tune.erase(k);
  else g_tune[k] = TY;
  if (ncg <= 1) g_tune_cg.erase(k);
  else g_tune_cg[k] = ncg;
  return MUFFIN_OK;
}

int atrous_class_groups(int N, int j, int mode, int nch) {
  if (mode == SM_DETAIL_ABS) return 1;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const long long k = tune_key(N, j, atrous_class(mode));
    if (g_tune.count(k)) {
      auto it = g_tune_cg.find(k);
      return it != g_tune_cg.end() ? it->second : 1;
    }
  }
  int TY, ncg;
  default_tiles(N, j, mode, nch, TY, ncg);
  return ncg;
}

int atrous_set_class_groups(int N, int j, int mode, int ncg) {
  if (mode == SM_DETAIL_ABS && ncg > 1) return set_error("class groups: not for the reduction"), MUFFIN_EINVAL;
  if (ncg != 0 && (ncg < 1 || ncg > std::min(1 << j, kMaxClassGroups) || (ncg & (ncg - 1))))
    return set_error("class groups must be a power of two up to min(2^j, 8)"), MUFFIN_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (ncg <= 1) g_tune_cg.erase(tune_key(N, j, atrous_class(mode)));
  else g_tune_cg[tune_key(N, j, atrous_class(mode))] = ncg;
  return MUFFIN_OK;
}

bool atrous_double_fits(int N, int j, int* TXo, int* TYo) {
  if (TXo) *TXo = N;
  if (TYo) *TYo = atrous_band_rows(N, j, DB_ANALYSIS);
  return true;
}

int launch_atrous(int mode, int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneOut out, PlaneOut out2,
                  float coef, float rho, double* partial, int* nblocks_out, hipStream_t st, int trial,
                  float coef2) {
  AtrousArgs a;
  a.A = A;
  a.B = B;
  a.E = E;
  a.out = out;
  a.out2 = out2;
  a.N = N;
  a.j = j;
  a.coef = coef;
  a.rho = rho;
  a.coef2 = coef2;
  a.partial = partial;
  const bool dbl = (mode == DB_ANALYSIS || mode == DB_ADJOINT || mode == DB_ANALYSIS_C);
  if (N > 1024) return set_error("atrous: N > 1024"), MUFFIN_EINVAL;
  a.TX = N;
  a.TY = atrous_band_rows(N, j, mode, nch);
  a.ncg = atrous_class_groups(N, j, mode, nch);
  if (a.ncg < 1 || a.ncg > (1 << j)) return set_error("atrous: bad class groups"), MUFFIN_EINVAL;
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY * a.ncg;
  const long long nb = (long long)a.tiles_per_ch * nch;
  if (nb > 0x7fffffffLL) return set_error("atrous: grid too large"), MUFFIN_EINVAL;
  if (nblocks_out) *nblocks_out = (int)nb;
  if (mode == SM_DETAIL_ABS && nb > kMaxPartials) {
    set_error("atrous: too many blocks for the partial-sum buffer");
    return MUFFIN_EINVAL;
  }
  a.nblocks = (int)nb;
  const int s = 1 << j;
  const size_t shm = sizeof(float) * (size_t)2 * (dbl ? kKR2 : kKR) * N;
  const dim3 grid((unsigned)nb), block((unsigned)N);
  if (trial) {
    switch (mode) {
      case SM_SUBADD: hipLaunchKernelGGL((k_band_trial<SM_SUBADD, kKR>), grid, block, shm, st, a); break;
      case SM_DETAIL1: hipLaunchKernelGGL((k_band_trial<SM_DETAIL1, kKR>), grid, block, shm, st, a); break;
      case DB_ANALYSIS: hipLaunchKernelGGL((k_band_trial<DB_ANALYSIS, kKR2>), grid, block, shm, st, a); break;
      case DB_ADJOINT: hipLaunchKernelGGL((k_band_trial<DB_ADJOINT, kKR2>), grid, block, shm, st, a); break;
      case DB_ANALYSIS_C:
        hipLaunchKernelGGL((k_band_trial<DB_ANALYSIS_C, kKR2>), grid, block, shm, st, a);
        break;
      default: set_error("atrous: no trial variant for this mode"); return MUFFIN_EINVAL;
    }
    MF_HIP(hipGetLastError());
    return MUFFIN_OK;
  }
  switch (mode) {
    case SM_SMOOTH: hipLaunchKernelGGL((k_band<SM_SMOOTH, kKR>), grid, block, shm, st, a); break;
    case SM_SUBADD: hipLaunchKernelGGL((k_band<SM_SUBADD, kKR>), grid, block, shm, st, a); break;
    case SM_DETAIL: hipLaunchKernelGGL((k_band<SM_DETAIL, kKR>), grid, block, shm, st, a); break;
    case SM_DETAIL_ABS: hipLaunchKernelGGL((k_band<SM_DETAIL_ABS, kKR>), grid, block, shm, st, a); break;
    case SM_DETAIL1: hipLaunchKernelGGL((k_band<SM_DETAIL1, kKR>), grid, block, shm, st, a); break;
    case DB_ANALYSIS: hipLaunchKernelGGL((k_band<DB_ANALYSIS, kKR2>), grid, block, shm, st, a); break;
    case DB_ADJOINT: hipLaunchKernelGGL((k_band<DB_ADJOINT, kKR2>), grid, block, shm, st, a); break;
    case DB_ANALYSIS_C: hipLaunchKernelGGL((k_band<DB_ANALYSIS_C, kKR2>), grid, block, shm, st, a); break;
    default: set_error("atrous: bad mode"); return MUFFIN_EINVAL;
  }
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int launch_pair(int mode, int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneOut out, PlaneOut out2,
                PlaneOut out3, float coef, float rho, float coef2, hipStream_t st, int trial) {
  if (!is_pair(mode)) return set_error("pair: bad mode"), MUFFIN_EINVAL;
  if (N > 1024) return set_error("pair: N > 1024"), MUFFIN_EINVAL;
  AtrousArgs a{};
  a.A = A;
  a.B = B;
  a.E = E;
  a.out = out;
  a.out2 = out2;
  a.out3 = out3;
  a.N = N;
  a.j = j;
  a.coef = coef;
  a.rho = rho;
  a.coef2 = coef2;
  a.TX = N;
  a.TY = atrous_band_rows(N, j, mode, nch);
  a.ncg = atrous_class_groups(N, j, mode, nch);
  if (a.ncg < 1 || a.ncg > (1 << j)) return set_error("pair: bad class groups"), MUFFIN_EINVAL;
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY * a.ncg;
  const long long nb = (long long)a.tiles_per_ch * nch;
  if (nb > 0x7fffffffLL) return set_error("pair: grid too large"), MUFFIN_EINVAL;
  a.nblocks = (int)nb;
  const size_t shm = sizeof(float) * (size_t)4 * kKRP * N;
  const dim3 grid((unsigned)nb), block((unsigned)N);
  switch (mode) {
    case PR_ANALYSIS:
      if (trial) hipLaunchKernelGGL((k_pair_trial<PR_ANALYSIS, kKRP>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_pair<PR_ANALYSIS, kKRP>), grid, block, shm, st, a);
      break;
    case PR_ANALYSIS_C:
      if (trial) hipLaunchKernelGGL((k_pair_trial<PR_ANALYSIS_C, kKRP>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_pair<PR_ANALYSIS_C, kKRP>), grid, block, shm, st, a);
      break;
    case P1_ANALYSIS:
      if (trial) hipLaunchKernelGGL((k_pair_trial<P1_ANALYSIS, kKRP>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_pair<P1_ANALYSIS, kKRP>), grid, block, shm, st, a);
      break;
    case P1_ANALYSIS_C:
      if (trial) hipLaunchKernelGGL((k_pair_trial<P1_ANALYSIS_C, kKRP>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_pair<P1_ANALYSIS_C, kKRP>), grid, block, shm, st, a);
      break;
    case P1_ADJOINT:
      if (trial) hipLaunchKernelGGL((k_pair_trial<P1_ADJOINT, kKRP>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_pair<P1_ADJOINT, kKRP>), grid, block, shm, st, a);
      break;
    default:
      if (trial) hipLaunchKernelGGL((k_pair_trial<PR_ADJOINT, kKRP>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_pair<PR_ADJOINT, kKRP>), grid, block, shm, st, a);
      break;
  }
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int launch_triple(int mode, int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneRef F, PlaneOut out,
                  PlaneOut out2, PlaneOut out3, PlaneOut out4, float coef, float rho, float coef2, hipStream_t st,
                  int trial) {
  if (!is_triple(mode)) return set_error("triple: bad mode"), MUFFIN_EINVAL;
  if (N > 1024) return set_error("triple: N > 1024"), MUFFIN_EINVAL;
  AtrousArgs a{};
  a.A = A;
  a.B = B;
  a.E = E;
  a.F = F;
  a.out = out;
  a.out2 = out2;
  a.out3 = out3;
  a.out4 = out4;
  a.N = N;
  a.j = j;
  a.coef = coef;
  a.rho = rho;
  a.coef2 = coef2;
  a.TX = N;
  a.TY = atrous_band_rows(N, j, mode, nch);
  a.ncg = atrous_class_groups(N, j, mode, nch);
  if (a.ncg < 1 || a.ncg > (1 << j)) return set_error("triple: bad class groups"), MUFFIN_EINVAL;
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY * a.ncg;
  const long long nb = (long long)a.tiles_per_ch * nch;
  if (nb > 0x7fffffffLL) return set_error("triple: grid too large"), MUFFIN_EINVAL;
  a.nblocks = (int)nb;
  const dim3 grid((unsigned)nb), block((unsigned)N);
  if (mode == TR_ADJOINT) {
    const int RS = tri_row_stride(N);
    const size_t shma = sizeof(float) * kAdjRows * (size_t)RS;
    switch (RS) {
      case 64:
        if (trial) hipLaunchKernelGGL(k_triple_adj_trial<64>, grid, block, shma, st, a);
        else hipLaunchKernelGGL(k_triple_adj<64>, grid, block, shma, st, a);
        break;
      case 256:
        if (trial) hipLaunchKernelGGL(k_triple_adj_trial<256>, grid, block, shma, st, a);
        else hipLaunchKernelGGL(k_triple_adj<256>, grid, block, shma, st, a);
        break;
      default:
        if (trial) hipLaunchKernelGGL(k_triple_adj_trial<1024>, grid, block, shma, st, a);
        else hipLaunchKernelGGL(k_triple_adj<1024>, grid, block, shma, st, a);
    }
    MF_HIP(hipGetLastError());
    return MUFFIN_OK;
  }
  const int RS = tri_row_stride(N);
  const size_t shm = sizeof(float) * kAnRows * (size_t)RS;
  const bool co = mode == TR_ANALYSIS_C;
#define MF_TRI_AN(rs)                                                                              \
  if (co) {                                                                                        \
    if (trial) hipLaunchKernelGGL((k_triple_an_trial<rs, true>), grid, block, shm, st, a);         \
    else hipLaunchKernelGGL((k_triple_an<rs, true>), grid, block, shm, st, a);                     \
  } else {                                                                                         \
    if (trial) hipLaunchKernelGGL((k_triple_an_trial<rs, false>), grid, block, shm, st, a);        \
    else hipLaunchKernelGGL((k_triple_an<rs, false>), grid, block, shm, st, a);                    \
  }
  switch (RS) {
    case 64: MF_TRI_AN(64) break;
    case 256: MF_TRI_AN(256) break;
    default: MF_TRI_AN(1024)
  }
#undef MF_TRI_AN
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int launch_fused_pair(int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneRef F, PlaneOut out,
                      PlaneOut out2, PlaneOut out3, PlaneOut out4, float coef, float rho, float coef2,
                      hipStream_t st, int trial) {
  if (N > 1024) return set_error("fused pair: N > 1024"), MUFFIN_EINVAL;
  AtrousArgs a{};
  a.A = A;
  a.B = B;
  a.E = E;
  a.F = F;
  a.out = out;
  a.out2 = out2;
  a.out3 = out3;
  a.out4 = out4;
  a.N = N;
  a.j = j;
  a.coef = coef;
  a.rho = rho;
  a.coef2 = coef2;
  a.TX = N;
  a.TY = atrous_band_rows(N, j, PR_FUSED, nch);
  a.ncg = atrous_class_groups(N, j, PR_FUSED, nch);
  if (a.ncg < 1 || a.ncg > (1 << j)) return set_error("fused pair: bad class groups"), MUFFIN_EINVAL;
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY * a.ncg;
  const long long nb = (long long)a.tiles_per_ch * nch;
  if (nb > 0x7fffffffLL) return set_error("fused pair: grid too large"), MUFFIN_EINVAL;
  a.nblocks = (int)nb;
  const int RS = tri_row_stride(N);
  const size_t shm = sizeof(float) * kFusedRows * (size_t)RS;
  const dim3 grid((unsigned)nb), block((unsigned)N);
  switch (RS) {
    case 64:
      if (trial) hipLaunchKernelGGL(k_fused_trial<64>, grid, block, shm, st, a);
      else hipLaunchKernelGGL(k_fused<64>, grid, block, shm, st, a);
      break;
    case 256:
      if (trial) hipLaunchKernelGGL(k_fused_trial<256>, grid, block, shm, st, a);
      else hipLaunchKernelGGL(k_fused<256>, grid, block, shm, st, a);
      break;
    default:
      if (trial) hipLaunchKernelGGL(k_fused_trial<1024>, grid, block, shm, st, a);
      else hipLaunchKernelGGL(k_fused<1024>, grid, block, shm, st, a);
  }
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int atrous_init_attrs() {
  const int shm = (int)(sizeof(float) * 2 * kKR * 1024);
  MF_HIP(hipFuncSetAttribute((const void*)k_band<SM_SMOOTH, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band<SM_SUBADD, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band<SM_DETAIL, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band<SM_DETAIL_ABS, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band<SM_DETAIL1, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band<DB_ANALYSIS, kKR2>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band<DB_ADJOINT, kKR2>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band<DB_ANALYSIS_C, kKR2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band_trial<DB_ANALYSIS_C, kKR2>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  const int shmp = (int)(sizeof(float) * 4 * kKRP * 1024);
  MF_HIP(hipFuncSetAttribute((const void*)k_pair<PR_ANALYSIS, kKRP>, hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair<PR_ANALYSIS_C, kKRP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair<PR_ADJOINT, kKRP>, hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair_trial<PR_ANALYSIS, kKRP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair_trial<PR_ANALYSIS_C, kKRP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair_trial<PR_ADJOINT, kKRP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair<P1_ANALYSIS, kKRP>, hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair<P1_ANALYSIS_C, kKRP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair<P1_ADJOINT, kKRP>, hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair_trial<P1_ANALYSIS, kKRP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair_trial<P1_ANALYSIS_C, kKRP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_pair_trial<P1_ADJOINT, kKRP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shmp));
  MF_HIP(hipFuncSetAttribute((const void*)k_band_trial<SM_SUBADD, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shm));
  const int shma = (int)(sizeof(float) * kAdjRows * 1024);
  MF_HIP(hipFuncSetAttribute((const void*)k_triple_adj<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, shma));
  MF_HIP(hipFuncSetAttribute((const void*)k_triple_adj_trial<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shma));
  const int shmf = (int)(sizeof(float) * kFusedRows * 1024);
  MF_HIP(hipFuncSetAttribute((const void*)k_fused<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, shmf));
  MF_HIP(hipFuncSetAttribute((const void*)k_fused_trial<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, shmf));
  MF_HIP(hipFuncSetAttribute((const void*)k_band_trial<SM_DETAIL1, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band_trial<DB_ANALYSIS, kKR2>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_band_trial<DB_ADJOINT, kKR2>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  return MUFFIN_OK;
}

// ------------------------------------------------------------------ pointwise plane kernels
struct PointArgs {
  PlaneRef A, E;
  PlaneOut out;
  long long npix;
  float coef, rho;
  double* partial;
};

template <int MODE>
__global__ void __launch_bounds__(256) k_point(PointArgs a) {
  const int ch = blockIdx.y;
  const float* A = a.A.p + ch * a.A.cs;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.npix; i += (long long)gridDim.x * blockDim.x) {
    if constexpr (MODE == PT_DETAIL1 || MODE == PT_COARSE) {
      const float w = (MODE == PT_DETAIL1) ? a.E.p[ch * a.E.cs + i] - A[i] : A[i];
      float* up = a.out.p + ch * a.out.cs + i;
      const float u = *up;
      *up = dual_upd(u, w, a.coef, a.rho);
    } else if constexpr (MODE == PT_ABS_DIFF) {
      acc += fabs((double)a.E.p[ch * a.E.cs + i] - (double)A[i]);
    } else if constexpr (MODE == PT_ABS) {
      acc += fabs((double)A[i]);
    } else if constexpr (MODE == PT_COPY) {
      a.out.p[ch * a.out.cs + i] = a.coef * A[i];
    } else {
      a.out.p[ch * a.out.cs + i] = a.E.p[ch * a.E.cs + i] - A[i];
    }
  }
  if constexpr (MODE == PT_ABS_DIFF || MODE == PT_ABS) {
    const double tot = block_sum_atrous(acc);
    if (threadIdx.x == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = tot;
  }
}

int launch_pointwise(int mode, int N, int nch, PlaneRef A, PlaneRef E, PlaneOut out, float coef, float rho,
                     double* partial, int* nblocks_out, hipStream_t st) {
  PointArgs a;
  a.A = A;
  a.E = E;
  a.out = out;
  a.npix = (long long)N * N;
  a.coef = coef;
  a.rho = rho;
  a.partial = partial;
  long long bx = (a.npix + 255) / 256;
  if (bx > 1024) bx = 1024;
  const dim3 grid((unsigned)bx, (unsigned)nch);
  if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y);
  if ((mode == PT_ABS_DIFF || mode == PT_ABS) && (long long)grid.x * grid.y > kMaxPartials) {
    set_error("pointwise: too many blocks for the partial-sum buffer");
    return MUFFIN_EINVAL;
  }
  switch (mode) {
    case PT_DETAIL1: hipLaunchKernelGGL(k_point<PT_DETAIL1>, grid, dim3(256), 0, st, a); break;
    case PT_COARSE: hipLaunchKernelGGL(k_point<PT_COARSE>, grid, dim3(256), 0, st, a); break;
    case PT_ABS_DIFF: hipLaunchKernelGGL(k_point<PT_ABS_DIFF>, grid, dim3(256), 0, st, a); break;
    case PT_ABS: hipLaunchKernelGGL(k_point<PT_ABS>, grid, dim3(256), 0, st, a); break;
    case PT_COPY: hipLaunchKernelGGL(k_point<PT_COPY>, grid, dim3(256), 0, st, a); break;
    case PT_SUB: hipLaunchKernelGGL(k_point<PT_SUB>, grid, dim3(256), 0, st, a); break;
    default: set_error("pointwise: bad mode"); return MUFFIN_EINVAL;
  }
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

__global__ void __launch_bounds__(256) k_clamp_pos(float* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    x[i] = fmaxf(x[i], 0.f);
}

int launch_clamp_pos(float* x, long long n, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_clamp_pos, dim3((unsigned)nb), dim3(256), 0, st, x, n);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

__global__ void __launch_bounds__(256) k_scale_channels(float* __restrict__ x, const float* __restrict__ w,
                                                        long long npix, long long cs) {
  const float s = w[blockIdx.y];
  float* xc = x + (long long)blockIdx.y * cs;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < npix; i += (long long)gridDim.x * 256)
    xc[i] *= s;
}

int launch_scale_channels(float* x, const float* chan_w, long long npix, long long cs, int nch, hipStream_t st) {
  long long nb = (npix + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_scale_channels, dim3((unsigned)nb, (unsigned)nch), dim3(256), 0, st, x, chan_w, npix, cs);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

#ifdef MF_CHECKED
int oob_take_iuwt(unsigned long long* n) { return oob_take_here(n); }
#endif

}  // namespace mf
