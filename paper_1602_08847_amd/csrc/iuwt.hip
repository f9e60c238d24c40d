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

#include <map>
#include <mutex>

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
  const int ch = b / a.tiles_per_ch, band = b - ch * a.tiles_per_ch;
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
    return *reinterpret_cast<const float*>(base + off + xb);
  };
  auto put = [&](float* base, int y, float v) {  // row y of the band
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + y * rowb + xb) = v;
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
      } while (lr < s && nsteps(lr) == 0);
      if (lr < s) start_class(lr);
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
  int r = 0;
  while (r < s && nsteps(r) == 0) ++r;
  if (r < s) {
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
        } while (r < s && nsteps(r) == 0);
        if (r >= s) break;
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
// y0 + r + (i - 10) s; the chained stages need 10 class steps of halo on either side.
//   PR_ANALYSIS:  c1 = H_j c (index t - 2 after loading c(t)), w_j = c - H_j c1 (t - 4),
//                 c2 = H_{j+1} c1 (t - 6), w_{j+1} = c1 - H_{j+1} c2 (t - 10)
//   PR_ADJOINT:   h = H_{j+1} u_{j+1} (t - 4), a' = u_{j+1} + H_{j+1}(a - h) (t - 8),
//                 a'' = u_j + H_j(a' - H_j u_j) (t - 10)
// Every stage performs the same operations in the same order as the one-scale kernels, so the
// results are identical to running them one after the other.
template <int KR>
struct PairPre {
  float p0[KR], p1[KR], p2[KR], p3[KR];
};

template <int MODE, int KR>
__device__ __forceinline__ void pair_body(const AtrousArgs& a) {
  constexpr bool ADJ = (MODE == PR_ADJOINT);
  constexpr bool CO = (MODE == PR_ANALYSIS_C);
  constexpr int HALO = 10;
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  float* bA = sm;
  float* bB = sm + KR * N;
  float* bC = sm + 2 * KR * N;
  float* bD = sm + 3 * KR * N;
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, band = b - ch * a.tiles_per_ch;
  const int y0 = band * TY;
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
    return *reinterpret_cast<const float*>(base + off + xb);
  };
  auto put = [&](float* base, int y, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + y * rowb + xb) = v;
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
  // load streams: p0 at index t, p1 at t - 4, p2 at t - 6 (adjoint: u_j) or t - 10 (analysis:
  // u_{j+1}), p3 at t - 6 (coarse plane)
  int lr = 0, lt = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0;
  auto start_class = [&](int r) {
    const int f = y0 + r - HALO * s;
    o0 = rowoff(f);
    o1 = rowoff(f - 4 * s);
    o2 = rowoff(f - (ADJ ? 6 : 10) * s);
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
      } while (lr < s && nsteps(lr) == 0);
      if (lr < s) start_class(lr);
    }
  };
  // windows, oldest first
  float wa[9], wb[9], wc[5], wd[5];
#pragma unroll
  for (int i = 0; i < 9; ++i) wa[i] = wb[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) wc[i] = wd[i] = 0.f;
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
    if constexpr (ADJ) {
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
  int r = 0;
  while (r < s && nsteps(r) == 0) ++r;
  if (r < s) {
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
        } while (r < s && nsteps(r) == 0);
        if (r >= s) break;
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
// Three consecutive scales j, j + 1, j + 2 in one pass, the same way as the pairs: with s = 2^j,
// H_j, H_{j+1} and H_{j+2} have their vertical taps 1 and 2, 2 and 4, 4 and 8 class steps apart
// (windows of 5, 9 and 17 entries), one row per round, four LDS barriers per row.  Load index i of
// class r is row y0 + r + (i - 22) s.
//   TR_ANALYSIS:  c1 = H_j c (index t - 2 after loading c(t)), w_j = c - H_j c1 (t - 4),
//                 c2 = H_{j+1} c1 (t - 6), w_{j+1} = c1 - H_{j+1} c2 (t - 10),
//                 c3 = H_{j+2} c2 (t - 14), w_{j+2} = c2 - H_{j+2} c3 (t - 22)
//   TR_ADJOINT:   a1 = u_{j+2} + H_{j+2}(a - H_{j+2} u_{j+2}) (t - 16),
//                 a2 = u_{j+1} + H_{j+1}(a1 - H_{j+1} u_{j+1}) (t - 20),
//                 a3 = u_j + H_j(a2 - H_j u_j) (t - 22)
// As with the pairs, every stage repeats the one-scale kernels' operations in their order.
struct TriPre {
  float p0, p1, p2, p3, p4;
};

template <int MODE>
__device__ __forceinline__ void triple_body(const AtrousArgs& a) {
  constexpr bool ADJ = (MODE == TR_ADJOINT);
  constexpr bool CO = (MODE == TR_ANALYSIS_C);
  constexpr int HALO = 22;
  // the adjoint runs its four stages skewed over four consecutive steps (one barrier per step,
  // double-buffered LDS); the analysis runs them one after the other within a step
  constexpr int SKEW = ADJ ? 4 : 0;
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  float* bA = sm;
  float* bB = sm + N;
  float* bC = sm + 2 * N;
  float* bD = sm + 3 * N;
  float* bE = sm + 4 * N;
  float* bF = sm + 5 * N;
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, band = b - ch * a.tiles_per_ch;
  const int y0 = band * TY;
  const char* __restrict__ A = reinterpret_cast<const char*>(a.A.p + ch * a.A.cs);
  const char* __restrict__ Bp = ADJ ? reinterpret_cast<const char*>(a.B.p + ch * a.B.cs) : nullptr;
  const char* __restrict__ Ep = ADJ ? reinterpret_cast<const char*>(a.E.p + ch * a.E.cs) : nullptr;
  const char* __restrict__ Fp = ADJ ? reinterpret_cast<const char*>(a.F.p + ch * a.F.cs) : nullptr;
  float* __restrict__ O = a.out.p + ch * a.out.cs;
  float* __restrict__ O2 = ADJ ? nullptr : a.out2.p + ch * a.out2.cs;
  float* __restrict__ O3 = ADJ ? nullptr : a.out3.p + ch * a.out3.cs;
  float* __restrict__ O4 = ADJ ? nullptr : a.out4.p + ch * a.out4.cs;
  auto modx = [&](int v) { return (v % N + N) % N; };
  const int xm1 = modx(x - s), xm2 = modx(x - 2 * s), xm4 = modx(x - 4 * s), xm8 = modx(x - 8 * s);
  const int xp1 = modx(x + s), xp2 = modx(x + 2 * s), xp4 = modx(x + 4 * s), xp8 = modx(x + 8 * s);
  auto h0 = [&](const float* row) { return b3(row[xm2], row[xm1], row[x], row[xp1], row[xp2]); };
  auto h1 = [&](const float* row) { return b3(row[xm4], row[xm2], row[x], row[xp2], row[xp4]); };
  auto h2 = [&](const float* row) { return b3(row[xm8], row[xm4], row[x], row[xp4], row[xp8]); };
  const int rowb = N * 4, planeb = N * N * 4, stepb = (s % N) * rowb;
  const unsigned xb = (unsigned)x * 4u;
  auto at = [&](const char* base, int off) -> float {
    return *reinterpret_cast<const float*>(base + off + xb);
  };
  auto put = [&](float* base, int y, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + y * rowb + xb) = v;
  };
  auto upd = [&](float u, float w, float coef) { return dual_upd(u, w, coef, a.rho); };
  // steps of class r: its M rows plus the halo on both sides, plus SKEW steps that drain the
  // skewed stages
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
  // load streams (load index of step t):
  //   analysis  p0 c (t), p1 u_j (t - 4), p2 u_{j+1} (t - 10), p3 u_{j+2} (t - 22), p4 coarse (t - 14)
  //   adjoint   p0 u_{j+2} (t), p1 a (t - 8), p2 u_{j+1} (t - 12), p3 u_j (t - 18)
  constexpr int D1 = ADJ ? 8 : 4, D2 = ADJ ? 12 : 10, D3 = ADJ ? 18 : 22, D4 = 14;
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
    if constexpr (ADJ) {
      P.p1 = at(Fp, o1);
      P.p2 = at(Bp, o2);
      P.p3 = at(Ep, o3);
    } else {
      P.p1 = at(reinterpret_cast<const char*>(O), o1);
      P.p2 = at(reinterpret_cast<const char*>(O2), o2);
      P.p3 = at(reinterpret_cast<const char*>(O3), o3);
      if constexpr (CO) P.p4 = at(reinterpret_cast<const char*>(O4), o4);
    }
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
      } while (lr < s && nsteps(lr) == 0);
      if (lr < s) start_class(lr);
    }
  };
  // windows, oldest first
  float w17a[17], w17b[17], w9a[9], w9b[9], w5a[5], w5b[5];
#pragma unroll
  for (int i = 0; i < 17; ++i) w17a[i] = w17b[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 9; ++i) w9a[i] = w9b[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) w5a[i] = w5b[i] = 0.f;
  auto push = [](auto& w, float v) {
    constexpr int n = sizeof(w) / sizeof(w[0]);
#pragma unroll
    for (int i = 0; i < n - 1; ++i) w[i] = w[i + 1];
    w[n - 1] = v;
  };
  auto v17 = [](const float (&w)[17]) { return b3(w[0], w[4], w[8], w[12], w[16]); };
  auto v9 = [](const float (&w)[9]) { return b3(w[0], w[2], w[4], w[6], w[8]); };
  auto v5 = [](const float (&w)[5]) { return b3(w[0], w[1], w[2], w[3], w[4]); };
  // delay lines of the skewed adjoint: value of step T - 1 first
  float dA[1] = {0.f}, dC[1] = {0.f}, dE[2] = {0.f, 0.f};
  float dU2[2] = {0.f, 0.f}, dU1[3] = {0.f, 0.f, 0.f}, dU0[4] = {0.f, 0.f, 0.f, 0.f};
  auto delay = [](auto& d, float v) -> float {  // returns the value of D steps ago, stores v
    constexpr int n = sizeof(d) / sizeof(d[0]);
    const float out = d[n - 1];
#pragma unroll
    for (int i = n - 1; i > 0; --i) d[i] = d[i - 1];
    d[0] = v;
    return out;
  };
  int par = 0;  // LDS parity of the skewed adjoint
  // step t of a class with ns steps whose load index 0 is row first
  auto process = [&](const TriPre& cur, int t, int ns, int first) {
    if constexpr (ADJ) {
      // At step T: stage 1 of step T, stage 2 of T - 1, stage 3 of T - 2, stage 4 of T - 3 and the
      // output of T - 4, where step t is the one-step-per-stage schedule's step t:
      //   w17a: u_{j+2} (t-16..t), w9a: u_{j+1} (t-20..t-12), w5a: u_j (t-22..t-18),
      //   w17b: a - H_{j+2} u_{j+2} (t-24..t-8), w9b: a1 - H_{j+1} u_{j+1} (t-24..t-16),
      //   w5b: a2 - H_j u_j (t-24..t-20)
      float* wr = sm + par * 6 * N;        // written this step
      float* rd = sm + (par ^ 1) * 6 * N;  // written last step
      const float hA = h2(rd), hC = h1(rd + 2 * N), hE = h0(rd + 4 * N);  // stage 1 of T - 1
      const float gB = h2(rd + N);      // stage 2 of T - 2
      const float gD = h1(rd + 3 * N);  // stage 3 of T - 3
      const float gF = h0(rd + 5 * N);  // stage 4 of T - 4
      // stage 1, step T
      push(w17a, cur.p0);
      push(w9a, cur.p2);
      push(w5a, cur.p3);
      wr[x] = v17(w17a);
      wr[2 * N + x] = v9(w9a);
      wr[4 * N + x] = v5(w5a);
      // stage 2, step T - 1: a - H_{j+2} u_{j+2}
      push(w17b, delay(dA, cur.p1) - hA);
      wr[N + x] = v17(w17b);
      // stage 3, step T - 2: a1 = u_{j+2} + H_{j+2}(...), then a1 - H_{j+1} u_{j+1}
      const float a1 = delay(dU2, w17a[0]) + gB;
      push(w9b, a1 - delay(dC, hC));
      wr[3 * N + x] = v9(w9b);
      // stage 4, step T - 3: a2 = u_{j+1} + H_{j+1}(...), then a2 - H_j u_j
      const float a2 = delay(dU1, w9a[0]) + gD;
      push(w5b, a2 - delay(dE, hE));
      wr[5 * N + x] = v5(w5b);
      // output, step T - 4: u_j + H_j(...)
      const float out = delay(dU0, w5a[0]) + gF;
      const int to = t - SKEW;
      if (to >= 2 * HALO && to < ns - SKEW) put(O, first + (to - HALO) * s, out);
      lds_barrier();
      par ^= 1;
    } else {
      // w5a: c (t-4..t), w9a: c1 (t-10..t-2), w17a: c2 (t-22..t-6), w17b: c3 (t-30..t-14)
      push(w5a, cur.p0);
      const float cc0 = w5a[0];
      bA[x] = v5(w5a);
      lds_barrier();
      push(w9a, h0(bA));
      const float cc1 = w9a[0];
      bB[x] = b3(w9a[4], w9a[5], w9a[6], w9a[7], w9a[8]);
      bC[x] = v9(w9a);
      lds_barrier();
      const float wj = cc0 - h0(bB);
      if (t >= HALO + 4 && t < ns - 18) put(O, first + (t - 4) * s, upd(cur.p1, wj, a.coef));
      push(w17a, h1(bC));
      const float cc2 = w17a[0];
      bD[x] = b3(w17a[8], w17a[10], w17a[12], w17a[14], w17a[16]);
      bE[x] = v17(w17a);
      lds_barrier();
      const float wj1 = cc1 - h1(bD);
      if (t >= HALO + 10 && t < ns - 12) put(O2, first + (t - 10) * s, upd(cur.p2, wj1, a.coef));
      const float c3 = h2(bE);
      if (t >= HALO + 14 && t < ns - 8) {
        if constexpr (CO) {
          put(O4, first + (t - 14) * s, upd(cur.p4, c3, a.coef2));
        } else {
          put(O4, first + (t - 14) * s, c3);
        }
      }
      push(w17b, c3);
      bF[x] = v17(w17b);
      lds_barrier();
      if (t >= 2 * HALO && t < ns) put(O3, first + (t - HALO) * s, upd(cur.p3, cc2 - h2(bF), a.coef));
    }
  };
  int r = 0;
  while (r < s && nsteps(r) == 0) ++r;
  if (r < s) {
    lr = r;
    start_class(lr);
    int pt = 0, pns = nsteps(r), pfirst = y0 + r - HALO * s;
    auto next_step = [&]() -> bool {  // false when the band is done
      if (++pt >= pns) {
        do {
          ++r;
        } while (r < s && nsteps(r) == 0);
        if (r >= s) return false;
        pt = 0;
        pns = nsteps(r);
        pfirst = y0 + r - HALO * s;
      }
      return true;
    };
    if constexpr (ADJ) {
      // loads one step ahead (two would not fit the adjoint's registers)
      TriPre cur, nxt;
      load_step(cur);
      advance_load();
      while (true) {
        load_step(nxt);  // past the last class: further rows of the planes, unused
        advance_load();
        process(cur, pt, pns, pfirst);
        if (!next_step()) break;
        cur = nxt;
      }
      return;
    }
    // loads run two steps ahead of the computation; the loop is unrolled three times so the three
    // buffers keep fixed roles and no register copy waits for a load in flight
    TriPre q0, q1, q2;
    load_step(q0);
    advance_load();
    load_step(q1);
    advance_load();
    while (true) {
      load_step(q2);  // past the last class: further rows of the planes, unused
      advance_load();
      process(q0, pt, pns, pfirst);
      if (!next_step()) break;
      load_step(q0);
      advance_load();
      process(q1, pt, pns, pfirst);
      if (!next_step()) break;
      load_step(q1);
      advance_load();
      process(q2, pt, pns, pfirst);
      if (!next_step()) break;
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(1024) k_triple(AtrousArgs a) {
  triple_body<MODE>(a);
}

template <int MODE>
__global__ void __launch_bounds__(1024) k_triple_trial(AtrousArgs a) {
  triple_body<MODE>(a);
}

// ------------------------------------------------------------------ fused pair
// The last analysis pair of an iteration (scales j, j + 1 and the coarse plane's dual step) and
// the first adjoint pair of the next iteration, which works on exactly the planes the analysis
// has just updated, in one pass.  With t the load index of c_j:
//   analysis:  c1 = H_j c (t - 2), w_j (t - 4), c2 = H_{j+1} c1 (t - 6), w_{j+1} (t - 10), giving
//              the new u_j (t - 4), coarse plane u_c (t - 6) and u_{j+1} (t - 10)
//   adjoint, one step behind, on those values (index T = t - 11 of u_{j+1}):
//              h = H_{j+1} u_{j+1} (T - 4), a' = u_{j+1} + H_{j+1}(u_c - h) (T - 8),
//              a'' = u_j + H_j(a' - H_j u_j) (T - 10 = t - 21)
// The new u_j and u_c wait 13 and 9 steps until the adjoint reaches them, in LDS rings of one
// slot per step (each thread reads back only what it wrote, so the rings need no barrier).  The four stages of a step share three LDS barriers: the analysis and adjoint stages of
// one phase read rows written in the phase before.  The old planes are read from B, E, F and the
// new ones written to out, out2, out3, so a band's halo always reads the values its neighbours
// are replacing; a'' goes to out4.  Every stage repeats the operations of the analysis pair and
// the adjoint pair in their order: planes and a'' are bit-identical to the two launches.
struct FusedPre {
  float p0, p1, p2, p3;
};

__device__ __forceinline__ void fused_body(const AtrousArgs& a) {
  constexpr int HALO = 20;  // 10 class steps for the analysis, 10 for the adjoint
  constexpr int SKEW = 1;   // the adjoint stages run one step behind
  extern __shared__ float sm[];
  const int N = a.N, jj = a.j, s = 1 << jj, x = threadIdx.x, TY = a.TY;
  float* bA = sm;  // analysis rows
  float* bB = sm + N;
  float* bC = sm + 2 * N;
  float* bD = sm + 3 * N;
  float* qA = sm + 4 * N;  // adjoint rows
  float* qB = sm + 5 * N;
  float* qC = sm + 6 * N;
  float* qD = sm + 7 * N;
  constexpr int DJ = 13, DC = 9;  // delays of the new u_j and u_c
  float* ringJ = sm + 8 * N;      // [DJ][N]
  float* ringC = sm + (8 + DJ) * N;  // [DC][N]
  const int b = xcd_remap(blockIdx.x, a.nblocks);
  const int ch = b / a.tiles_per_ch, band = b - ch * a.tiles_per_ch;
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
    return *reinterpret_cast<const float*>(base + off + xb);
  };
  auto put = [&](float* base, int y, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + y * rowb + xb) = v;
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
  // load streams: p0 c (t), p1 old u_j (t - 4), p2 old u_{j+1} (t - 10), p3 old coarse (t - 6)
  int lr = 0, lt = 0, o0 = 0, o1 = 0, o2 = 0, o3 = 0;
  auto start_class = [&](int r) {
    const int f = y0 + r - HALO * s;
    o0 = rowoff(f);
    o1 = rowoff(f - 4 * s);
    o2 = rowoff(f - 10 * s);
    o3 = rowoff(f - 6 * s);
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
      } while (lr < s && nsteps(lr) == 0);
      if (lr < s) start_class(lr);
    }
  };
  // windows, oldest first.  Analysis: wc c (t-4..t), wa c1 (t-10..t-2), wb c2 (t-14..t-6).
  // Adjoint: ya u_{j+1} (T-8..T), yc u_j (T-10..T-6), yb u_c - h (T-12..T-4), yd a' - H_j u_j
  // (T-12..T-8).
  float wc[5], wa[9], wb[9], ya[9], yb[9], yc[5], yd[5];
#pragma unroll
  for (int i = 0; i < 9; ++i) wa[i] = wb[i] = ya[i] = yb[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) wc[i] = yc[i] = yd[i] = 0.f;
  // ring slots of the current step; the new u_{j+1} of the last step
#pragma unroll
  for (int i = 0; i < DJ; ++i) ringJ[i * N + x] = 0.f;
#pragma unroll
  for (int i = 0; i < DC; ++i) ringC[i * N + x] = 0.f;
  int rj = 0, rc = 0;
  float pend1 = 0.f;
  auto push = [](auto& w, float v) {
    constexpr int n = sizeof(w) / sizeof(w[0]);
#pragma unroll
    for (int i = 0; i < n - 1; ++i) w[i] = w[i + 1];
    w[n - 1] = v;
  };
  auto v9 = [](const float (&w)[9]) { return b3(w[0], w[2], w[4], w[6], w[8]); };
  auto v5 = [](const float (&w)[5]) { return b3(w[0], w[1], w[2], w[3], w[4]); };
  // step t of a class with ns steps whose load index 0 is row first; index i is a row of the band
  // when HALO <= i < ns - HALO - SKEW
  auto process = [&](const FusedPre& cur, int t, int ns, int first) {
    const int lo = HALO, hi = ns - HALO - SKEW;
    // phase 1: analysis H_j of c (vertical); adjoint H_{j+1} of u_{j+1} and H_j of u_j (vertical)
    push(wc, cur.p0);
    const float cc4 = wc[0];
    bA[x] = v5(wc);
    push(ya, pend1);
    const float cuh = ya[0];
    qA[x] = v9(ya);
    push(yc, ringJ[rj * N + x]);  // u_j of 13 steps ago
    const float cul = yc[0];
    qB[x] = v5(yc);
    lds_barrier();
    // phase 2: c1, the vertical parts of H_j c1 and H_{j+1} c1; u_c - H_{j+1} u_{j+1}
    push(wa, hj(bA));
    const float cc10 = wa[0];
    bB[x] = b3(wa[4], wa[5], wa[6], wa[7], wa[8]);
    bC[x] = v9(wa);
    const float h1 = hj1(qA);
    const float h0 = hj(qB);
    push(yb, ringC[rc * N + x] - h1);  // u_c of 9 steps ago
    qC[x] = v9(yb);
    lds_barrier();
    // phase 3: new u_j and coarse plane, vertical H_{j+1} of c2; a' and a' - H_j u_j
    const float nuj = upd(cur.p1, cc4 - hj(bB), a.coef);
    if (t - 4 >= lo && t - 4 < hi) put(O, first + (t - 4) * s, nuj);
    const float c2 = hj1(bC);
    const float nuc = upd(cur.p3, c2, a.coef2);
    if (t - 6 >= lo && t - 6 < hi) put(O3, first + (t - 6) * s, nuc);
    push(wb, c2);
    bD[x] = v9(wb);
    const float a1 = cuh + hj1(qC);
    push(yd, a1 - h0);
    qD[x] = v5(yd);
    ringJ[rj * N + x] = nuj;
    ringC[rc * N + x] = nuc;
    rj = rj + 1 == DJ ? 0 : rj + 1;
    rc = rc + 1 == DC ? 0 : rc + 1;
    lds_barrier();
    // phase 4: new u_{j+1}; a''
    const float nu1 = upd(cur.p2, cc10 - hj1(bD), a.coef);
    if (t - 10 >= lo && t - 10 < hi) put(O2, first + (t - 10) * s, nu1);
    pend1 = nu1;
    if (t - 21 >= lo && t - 21 < hi) put(O4, first + (t - 21) * s, cul + hj(qD));
  };
  int r = 0;
  while (r < s && nsteps(r) == 0) ++r;
  if (r < s) {
    lr = r;
    start_class(lr);
    int pt = 0, pns = nsteps(r), pfirst = y0 + r - HALO * s;
    FusedPre cur, nxt;
    load_step(cur);
    advance_load();
    while (true) {
      load_step(nxt);  // past the last class: further rows of the planes, unused
      advance_load();
      process(cur, pt, pns, pfirst);
      if (++pt >= pns) {
        do {
          ++r;
        } while (r < s && nsteps(r) == 0);
        if (r >= s) break;
        pt = 0;
        pns = nsteps(r);
        pfirst = y0 + r - HALO * s;
      }
      cur = nxt;
    }
  }
}

__global__ void __launch_bounds__(1024) k_fused(AtrousArgs a) { fused_body(a); }
constexpr int kFusedRows = 8 + 13 + 9;  // LDS rows of N floats: eight stage rows, the two rings

__global__ void __launch_bounds__(1024) k_fused_trial(AtrousArgs a) { fused_body(a); }

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

static bool is_pair(int mode) { return mode == PR_ANALYSIS || mode == PR_ANALYSIS_C || mode == PR_ADJOINT; }
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

int atrous_set_band_rows(int N, int j, int mode, int TY) {
  if (TY != 0 && (TY < 1 || TY > N || N % TY)) return set_error("band rows must divide N"), MUFFIN_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (TY == 0) g_tune.erase(tune_key(N, j, atrous_class(mode)));
  else g_tune[tune_key(N, j, atrous_class(mode))] = TY;
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
  a.TY = atrous_band_rows(N, j, mode);
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY;
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
  a.TY = atrous_band_rows(N, j, mode);
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY;
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
  a.TY = atrous_band_rows(N, j, mode);
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY;
  const long long nb = (long long)a.tiles_per_ch * nch;
  if (nb > 0x7fffffffLL) return set_error("triple: grid too large"), MUFFIN_EINVAL;
  a.nblocks = (int)nb;
  const size_t shm = sizeof(float) * (size_t)(mode == TR_ADJOINT ? 12 : 6) * N;
  const dim3 grid((unsigned)nb), block((unsigned)N);
  switch (mode) {
    case TR_ANALYSIS:
      if (trial) hipLaunchKernelGGL((k_triple_trial<TR_ANALYSIS>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_triple<TR_ANALYSIS>), grid, block, shm, st, a);
      break;
    case TR_ANALYSIS_C:
      if (trial) hipLaunchKernelGGL((k_triple_trial<TR_ANALYSIS_C>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_triple<TR_ANALYSIS_C>), grid, block, shm, st, a);
      break;
    default:
      if (trial) hipLaunchKernelGGL((k_triple_trial<TR_ADJOINT>), grid, block, shm, st, a);
      else hipLaunchKernelGGL((k_triple<TR_ADJOINT>), grid, block, shm, st, a);
      break;
  }
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
  a.TY = atrous_band_rows(N, j, PR_FUSED);
  a.tiles_x = 1;
  a.tiles_per_ch = N / a.TY;
  const long long nb = (long long)a.tiles_per_ch * nch;
  if (nb > 0x7fffffffLL) return set_error("fused pair: grid too large"), MUFFIN_EINVAL;
  a.nblocks = (int)nb;
  const size_t shm = sizeof(float) * kFusedRows * (size_t)N;
  const dim3 grid((unsigned)nb), block((unsigned)N);
  if (trial) hipLaunchKernelGGL(k_fused_trial, grid, block, shm, st, a);
  else hipLaunchKernelGGL(k_fused, grid, block, shm, st, a);
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
  MF_HIP(hipFuncSetAttribute((const void*)k_band_trial<SM_SUBADD, kKR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             shm));
  const int shmf = (int)(sizeof(float) * kFusedRows * 1024);
  MF_HIP(hipFuncSetAttribute((const void*)k_fused, hipFuncAttributeMaxDynamicSharedMemorySize, shmf));
  MF_HIP(hipFuncSetAttribute((const void*)k_fused_trial, hipFuncAttributeMaxDynamicSharedMemorySize, shmf));
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

}  // namespace mf
