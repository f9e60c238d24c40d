// Stockham FFT core shared by the FFT-convolution passes and the spectral (cosine) kernel.
//
// Every 1-D transform is a self-sorting (Stockham) decimation-in-time FFT held in LDS: at each
// stage of radix R over a span Ns (product of the earlier radices), butterfly b reads the R
// inputs b + r N/R, multiplies input r by w^(r k), k = b mod Ns, w = exp(-2 pi i / (Ns R)),
// takes an R-point DFT in registers and writes output r to (b / Ns) Ns R + k + r Ns.
#pragma once
#include "common.h"

namespace mf {

// ------------------------------------------------------------------ radix plans
template <int N>
struct Plan;
#define MF_PLAN(n, nst_, r0, r1, r2, rmax)                             \
  template <>                                                          \
  struct Plan<n> {                                                     \
    static constexpr int nst = nst_;                                   \
    static constexpr int rad[3] = {r0, r1, r2};                        \
    static constexpr int T = n / rmax; /* threads per transform */     \
  };
MF_PLAN(8, 1, 8, 1, 1, 8)
MF_PLAN(16, 1, 16, 1, 1, 16)
MF_PLAN(32, 2, 8, 4, 1, 8)
MF_PLAN(64, 2, 8, 8, 1, 8)
MF_PLAN(128, 2, 16, 8, 1, 16)
MF_PLAN(256, 2, 16, 16, 1, 16)
MF_PLAN(512, 3, 8, 8, 8, 8)
MF_PLAN(1024, 3, 16, 16, 4, 16)
MF_PLAN(12, 2, 4, 3, 1, 4)
MF_PLAN(24, 2, 8, 3, 1, 8)
MF_PLAN(48, 3, 4, 4, 3, 4)  // not (16, 3): an even thread count per transform (12, not 3)
MF_PLAN(96, 3, 8, 4, 3, 8)
MF_PLAN(192, 3, 8, 8, 3, 8)
MF_PLAN(384, 3, 16, 8, 3, 16)
MF_PLAN(768, 3, 16, 16, 3, 16)
#undef MF_PLAN

template <int N>
constexpr int span_before(int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= Plan<N>::rad[i];
  return p;
}

// LDS addressing: one padding slot every 32 complex entries breaks power-of-two strides;
// the per-transform stride is odd so that transforms side by side fall in different banks.
__host__ __device__ constexpr int lpad(int i) { return i + (i >> 5); }
template <int N>
constexpr int lstride() {
  int s = lpad(N - 1) + 1;
  return (s & 1) ? s : s + 1;
}

// ------------------------------------------------------------------ butterflies
// Multiply by -i (forward) or +i (inverse).
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
  const float c = -0.5f;
  const float s = 0.86602540378443864676f;  // sqrt(3)/2
  float2 t = cadd(v[1], v[2]);
  float2 d = csub(v[1], v[2]);
  float2 m = make_float2(v[0].x + c * t.x, v[0].y + c * t.y);
  // (-/+ i) s d
  float2 r = rot90<INV>(d);
  v[0] = cadd(v[0], t);
  v[1] = make_float2(m.x + s * r.x, m.y + s * r.y);
  v[2] = make_float2(m.x - s * r.x, m.y - s * r.y);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = rot90<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  // even/odd split: E = DFT4(v0,v2,v4,v6), O = DFT4(v1,v3,v5,v7); y_k = E_k + w8^k O_k
  dft4<INV>(v[0], v[2], v[4], v[6]);
  dft4<INV>(v[1], v[3], v[5], v[7]);
  const float h = 0.70710678118654752440f;
  float2 o1 = v[3], o2 = v[5], o3 = v[7];
  // w8 = (h, -h) forward, (h, h) inverse
  o1 = INV ? make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y)) : make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
  o2 = rot90<INV>(o2);
  o3 = INV ? make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y)) : make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <bool INV>
__device__ __forceinline__ void dft16(float2* v) {
  // n = 4 n1 + n2, k = k1 + 4 k2: inner 4-point DFTs over n1, twiddle w16^(n2 k1), outer over n2.
  float2 b[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
    dft4<INV>(a0, a1, a2, a3);
    b[n2][0] = a0;
    b[n2][1] = a1;
    b[n2][2] = a2;
    b[n2][3] = a3;
  }
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f, h = 0.70710678118654752440f;
  const float sg = INV ? 1.f : -1.f;
  // w16^m for m = n2 * k1, m in {1,2,3,4,6,9}
  const float2 w1 = make_float2(c1, sg * s1), w2 = make_float2(h, sg * h), w3 = make_float2(s1, sg * c1);
  const float2 w6 = make_float2(-h, sg * h), w9 = make_float2(-c1, -sg * s1);
  b[1][1] = cmul(b[1][1], w1);
  b[1][2] = cmul(b[1][2], w2);
  b[1][3] = cmul(b[1][3], w3);
  b[2][1] = cmul(b[2][1], w2);
  b[2][2] = rot90<INV>(b[2][2]);
  b[2][3] = cmul(b[2][3], w6);
  b[3][1] = cmul(b[3][1], w3);
  b[3][2] = cmul(b[3][2], w6);
  b[3][3] = cmul(b[3][3], w9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = b[0][k1], a1 = b[1][k1], a2 = b[2][k1], a3 = b[3][k1];
    dft4<INV>(a0, a1, a2, a3);
    v[k1] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
  if constexpr (R == 2) dft2<INV>(v[0], v[1]);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 16) dft16<INV>(v);
}

// ------------------------------------------------------------------ LDS Stockham transform
// One N-point transform of buf (LDS, lpad addressing) by T cooperating threads, t in [0, T).
// All threads of the workgroup must call it (it synchronises the workgroup).
template <int N, bool INV, int S = 0>
__device__ __forceinline__ void fft_lds(float2* buf, int t, bool active, const float2* __restrict__ tw) {
  if constexpr (S == 0) {
    // a kernel with two transforms would otherwise have the second one's twiddle loads merged
    // into the first and kept live in registers in between: offset the table by an opaque zero
    int zero = 0;
    asm volatile("" : "+s"(zero));
    tw += zero;
  }
  if constexpr (S < Plan<N>::nst) {
    constexpr int T = Plan<N>::T;
    constexpr int R = Plan<N>::rad[S];
    constexpr int Ns = span_before<N>(S);
    constexpr int NB = N / R;
    constexpr int PER = (NB + T - 1) / T;
    constexpr int TWS = N / (Ns * R);  // twiddle table stride
    float2 v[PER][R];
    // the stage's twiddles (a table in global memory, cache-resident) are requested first, so they
    // arrive while the LDS reads and the barrier complete
    float2 w[PER][R];
    if constexpr (Ns > 1) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int k = (t + i * T) % Ns;
        if constexpr (R >= 8) {
          // w^r from the table's w, w^2, w^4 (and w^8): at most three products per twiddle
#pragma unroll
          for (int r = 1; r < R; r *= 2) w[i][r] = tw[MF_CHK(r * k * TWS, N)];
#pragma unroll
          for (int r = 3; r < R; ++r) {
            if ((r & (r - 1)) == 0) continue;
            const int hi = 1 << (31 - __builtin_clz(r));
            w[i][r] = cmul(w[i][hi], w[i][r - hi]);
          }
        } else {
#pragma unroll
          for (int r = 1; r < R; ++r) w[i][r] = tw[MF_CHK(r * k * TWS, N)];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = t + i * T;
      if (active && (PER * T == NB || b < NB)) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = buf[lpad(MF_CHK(b + r * NB, N))];
      }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = t + i * T;
      if (active && (PER * T == NB || b < NB)) {
        const int k = b % Ns;
        if constexpr (Ns > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 wr = w[i][r];
            if (INV) wr.y = -wr.y;
            v[i][r] = cmul(v[i][r], wr);
          }
        }
        dftR<R, INV>(v[i]);
        const int base = (b / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lpad(MF_CHK(base + r * Ns, N))] = v[i][r];
      }
    }
    lds_barrier();
    fft_lds<N, INV, S + 1>(buf, t, active, tw);
  }
}

}  // namespace mf
