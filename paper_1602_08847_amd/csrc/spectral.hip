// Per-pixel spectral work: the fused step that takes the paper's master-node role (Sec. 3),
//   t   = mu_l V W^T                   (spectral adjoint of the dual, orthonormal DCT-III)
//   x~  = (x - tau (q + t))_+          (primal proximal step; q = gradient + mu_s W_s^dagger u)
//   d   = 2 x~ - x
//   V   <- rho sat(V + sigma mu_l d W) + (1 - rho) V      (spectral dual step, DCT-II)
//   x   <- rho x~ + (1 - rho) x
// A workgroup owns a run of pixels across all L channels; it reads x, q and V once and writes x, d
// and V once.  When L has an FFT plan the two cosine transforms go through an L-point complex
// FFT in LDS (reordering of the spectrum into even samples followed by reversed odd samples,
// then a quarter-sample phase factor, Makhoul 1980), two pixels packed per transform as real and
// imaginary parts.  Other L use dense products with a cosine table, each thread accumulating
// four outputs so every LDS read feeds four FMAs.
#include "fft_core.h"

#include <cmath>
#include <complex>
#include <vector>

namespace mf {

constexpr int PX = 32;  // pixels per workgroup

__device__ __forceinline__ float satf_s(float u) { return fminf(1.f, fmaxf(-1.f, u)); }

__global__ void __launch_bounds__(256) k_spectral_step(SpectralArgs a) {
  extern __shared__ float sm[];
  const int L = a.L;
  float* Vs = sm;           // [L][PX]
  float* Ds = sm + L * PX;  // [L][PX]
  const int p = threadIdx.x & (PX - 1);
  const int g = threadIdx.x >> 5;  // 0..7
  const long long pix0 = (long long)blockIdx.x * PX;
  const long long pix = pix0 + p;
  const bool pv = pix < a.npix;
  for (int idx = threadIdx.x; idx < L * PX; idx += 256) {
    const int l = idx / PX, pp = idx % PX;
    const long long q = pix0 + pp;
    Vs[idx] = (q < a.npix) ? a.V[(long long)l * a.cs + q] : 0.f;
  }
  lds_barrier();
  // primal step, channel rows l = g + 8 i (four per pass)
  for (int lb = g; lb < L; lb += 32) {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    int ls[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ls[i] = lb + 8 * i;
    for (int k = 0; k < L; ++k) {
      const float v = Vs[k * PX + p];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (ls[i] < L) acc[i] = fmaf(a.W[ls[i] * L + k], v, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int l = ls[i];
      if (l < L) {
        float d = 0.f;
        if (pv) {
          const long long o = (long long)l * a.cs + pix;
          const float x = a.X[o];
          const float t = a.mu_l * acc[i];
          const float xt = fmaxf(x - a.tau * (a.Q[o] + t), 0.f);
          d = 2.f * xt - x;
          a.D[o] = d;
          a.X[o] = a.rho * xt + (1.f - a.rho) * x;
        }
        Ds[l * PX + p] = d;
      }
    }
  }
  lds_barrier();
  // spectral dual step, coefficient rows k = g + 8 i
  for (int kb = g; kb < L; kb += 32) {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    int ks[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ks[i] = kb + 8 * i;
    for (int l = 0; l < L; ++l) {
      const float dv = Ds[l * PX + p];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (ks[i] < L) acc[i] = fmaf(a.WT[ks[i] * L + l], dv, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = ks[i];
      if (k < L && pv) {
        const float v = Vs[k * PX + p];
        a.V[(long long)k * a.cs + pix] = a.rho * satf_s(v + a.smu_l * acc[i]) + (1.f - a.rho) * v;
      }
    }
  }
}


// Channel counts without an FFT plan, L <= 256: the same step with the two cosine transforms as
// dense products.  A workgroup owns 64 pixels, one per lane, and stages their dual spectra across
// all L channels in LDS.  A wave computes CW channels at a time, so the cosine-table entries it
// needs are the same in every lane (scalar loads) and each LDS read feeds CW FMAs; the sums run
// over k in order, as in k_spectral_step.  The k loops are unrolled sixteen times, so that each
// table row is read sixteen entries per scalar load.
//
// One LDS array serves both products: the primal step reads V from it and keeps the d of its own
// channels in registers (at most MAXM chunks of CW per wave); once every wave is done with V, d
// replaces it, and the dual step reads each thread's few V entries back from global memory.  With
// half the LDS per workgroup, twice as many workgroups fit on a CU to hide the LDS and
// scalar-load latency.
constexpr int PXM = 64;
constexpr int kMatMaxL = 256;
// the cosine tables are read-only for the whole launch: read them through the constant address
// space, so that the wave-uniform reads become scalar loads
typedef const float __attribute__((address_space(4)))* const_fp;

template <int CW, int MAXM>
__global__ void __launch_bounds__(256) k_spectral_mat(SpectralArgs a) {
  extern __shared__ float sm[];  // [L][PXM]: V during the primal step, then d
  const int L = a.L;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long npix = a.npix, cs = a.cs;
  const long long pix = (long long)blockIdx.x * PXM + lane;
  const bool pok = pix < npix;
  for (int l = wv; l < L; l += 4) sm[l * PXM + lane] = pok ? a.V[(long long)l * cs + pix] : 0.f;
  lds_barrier();
  // primal step, channels l0 .. l0 + CW - 1 of this wave for l0 = wv CW + 4 CW m
  float dreg[MAXM][CW];
#pragma unroll
  for (int m = 0; m < MAXM; ++m) {
    const int l0 = wv * CW + 4 * CW * m;
#pragma unroll
    for (int c = 0; c < CW; ++c) dreg[m][c] = 0.f;
    if (l0 >= L) continue;
    float xr[CW], qr[CW], acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const long long o = (long long)min(l0 + c, L - 1) * cs + (pok ? pix : 0);
      xr[c] = a.X[o];  // fetched now, used after the sums
      qr[c] = a.Q[o];
      acc[c] = 0.f;
    }
    const_fp Wr[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) Wr[c] = (const_fp)(a.W + (long long)min(l0 + c, L - 1) * L);
#pragma unroll 16
    for (int k = 0; k < L; ++k) {
      const float v = sm[k * PXM + lane];
#pragma unroll
      for (int c = 0; c < CW; ++c) acc[c] = fmaf(Wr[c][k], v, acc[c]);
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int l = l0 + c;
      if (l >= L || !pok) continue;
      const long long o = (long long)l * cs + pix;
      const float x = xr[c];
      const float tv = a.mu_l * acc[c];
      const float xt = fmaxf(x - a.tau * (qr[c] + tv), 0.f);
      const float d = 2.f * xt - x;
      a.D[o] = d;
      a.X[o] = a.rho * xt + (1.f - a.rho) * x;
      dreg[m][c] = d;
    }
  }
  lds_barrier();  // every wave is done with V
#pragma unroll
  for (int m = 0; m < MAXM; ++m) {
    const int l0 = wv * CW + 4 * CW * m;
#pragma unroll
    for (int c = 0; c < CW; ++c)
      if (l0 + c < L) sm[(l0 + c) * PXM + lane] = dreg[m][c];
  }
  lds_barrier();
  // spectral dual step, coefficients k0 .. k0 + CW - 1 of this wave
  for (int k0 = wv * CW; k0 < L; k0 += 4 * CW) {
    float acc[CW];
    const_fp Wr[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      acc[c] = 0.f;
      Wr[c] = (const_fp)(a.WT + (long long)min(k0 + c, L - 1) * L);
    }
#pragma unroll 16
    for (int l = 0; l < L; ++l) {
      const float dv = sm[l * PXM + lane];
#pragma unroll
      for (int c = 0; c < CW; ++c) acc[c] = fmaf(Wr[c][l], dv, acc[c]);
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int k = k0 + c;
      if (k >= L) break;
      if (pok) {
        float* vp = a.V + (long long)k * cs + pix;
        const float v = *vp;
        *vp = a.rho * satf_s(v + a.smu_l * acc[c]) + (1.f - a.rho) * v;
      }
    }
  }
}

// ------------------------------------------------------------------ FFT-based fused step
// Orthonormal DCT-II of a length-L spectrum x: v = (x_0, x_2, ..., x_{L-2}, x_{L-1}, ..., x_3, x_1),
// X_k = s_k Re(exp(-i pi k / 2L) FFT(v)_k).  Its inverse: Y_k = s_k h_k X_k (h_0 = 1, h_k = 1/2),
// V_k = exp(i pi k / 2L) (Y_k - i Y_{L-k}) (Y_L = 0), v = unnormalised inverse FFT of V, and x is
// read back from v with the same reordering.
// the largest power of two <= v (v >= 1)
constexpr int pow2_floor(int v) { return v < 2 ? 1 : 2 * pow2_floor(v / 2); }

template <int L>
struct SpecGeom {
  static constexpr int T = Plan<L>::T;
  // transforms (pixel pairs) per block: a power of two, so that a block's pixels span whole
  // 128-byte lines of every channel plane (T = 12 or 24 with L = 3 * 2^a would otherwise give 42
  // or 20 pixels per block)
  static constexpr int NF = pow2_floor(256 / T);
  static constexpr int PXB = 2 * NF;                        // pixels per block
  // odd transform stride: the per-pixel steps read one entry of each of 16 transforms at once
  static constexpr int LS = lstride<L>();
  static constexpr int NT = NF * T;                       // threads per block
  static constexpr int PER = (L * PXB + NT - 1) / NT;     // (channel, pixel) elements per thread
  static constexpr size_t shm = sizeof(float2) * (NF * LS + L);  // transforms, then the twiddles
};

__device__ __forceinline__ int dct_slot(int l, int L) { return (l & 1) ? L - 1 - (l >> 1) : (l >> 1); }

template <int L>
__global__ void __launch_bounds__(256) k_spectral_fft(SpectralArgs a) {
  using G = SpecGeom<L>;
  constexpr int T = G::T, NF = G::NF, PXB = G::PXB, LS = G::LS;
  constexpr int NT = NF * T;
  constexpr int PER = G::PER;
  extern __shared__ float2 buf[];  // [NF][LS] transforms; pixel p is part p & 1 of transform p / 2
  float2* twl = buf + NF * LS;     // [L] twiddle table, copied once so the stages read it from LDS
  for (int i = threadIdx.x; i < L; i += NT) twl[i] = a.twL[i];
  const long long npix = a.npix, cs = a.cs;
  const long long pix0 = (long long)blockIdx.x * PXB;
  // Element i of a thread is (channel, pixel) = (idx / PXB, idx % PXB), idx = threadIdx.x + i NT.
  // When NT is a multiple of PXB the pixel is the same for all i and the channel steps by
  // NT / PXB, so every access is a uniform base for i plus one byte offset per thread.
  constexpr bool FIXP = (NT % PXB) == 0;
  constexpr int LSTEP = FIXP ? NT / PXB : 1;
  const int l0 = threadIdx.x / PXB, p0 = threadIdx.x - l0 * PXB;
  const bool q0ok = pix0 + p0 < npix;
  const unsigned voff = FIXP ? (unsigned)(((long long)l0 * cs + pix0 + p0) * 4) : 0u;
  const long long cstride = (long long)LSTEP * cs * 4;
  auto el_l = [&](int i) -> int { return FIXP ? l0 + i * LSTEP : (threadIdx.x + i * NT) / PXB; };
  auto el_p = [&](int i) -> int { return FIXP ? p0 : (threadIdx.x + i * NT) % PXB; };
  auto el_ok = [&](int i) -> bool {
    if constexpr (FIXP) return q0ok;
    const int idx = threadIdx.x + i * NT;
    return idx < L * PXB && pix0 + idx % PXB < npix;
  };
  auto el_ptr = [&](const float* base, int i) -> const float* {
    if constexpr (FIXP) return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + i * cstride + voff);
    return base + (long long)el_l(i) * cs + pix0 + el_p(i);
  };
  auto el_out = [&](float* base, int i) -> float* { return const_cast<float*>(el_ptr(base, i)); };
  // V of the thread's elements, kept in registers for the dual step.  X, q, V and d are each
  // touched once per iteration here, so the kernel's global accesses are streaming.
  float vreg[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) vreg[i] = el_ok(i) ? ld_stream(el_ptr(a.V, i)) : 0.f;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (FIXP || threadIdx.x + i * NT < L * PXB) {
      const int p = el_p(i);
      reinterpret_cast<float*>(buf + MF_CHK(p >> 1, NF) * LS + lpad(MF_CHK(el_l(i), L)))[p & 1] = vreg[i];
    }
  }
  lds_barrier();
  const int f = threadIdx.x / T, t = threadIdx.x - f * T;
  float2* fb = buf + f * LS;
  {
    // t = mu_l * DCT-III(V), pre-twiddle in place: slot k becomes exp(i pi k / 2L) (Y_k - i Y_{L-k})
    // with Y = s h mu_l V (Y_L = 0), for both packed pixels; one thread owns slots k and L - k
    const float c0 = a.mu_l * sqrtf(1.f / L), c1 = a.mu_l * rsqrtf(2.f * L);
    auto twiddled = [&](float2 yk, float2 ym, int k) -> float2 {  // yk = Y_k, ym = Y_{L-k} of (a, b)
      const float2 e = a.csL[k];
      const float2 Va = make_float2(yk.x * e.x + ym.x * e.y, yk.x * e.y - ym.x * e.x);
      const float2 Vb = make_float2(yk.y * e.x + ym.y * e.y, yk.y * e.y - ym.y * e.x);
      return make_float2(Va.x - Vb.y, Va.y + Vb.x);
    };
    for (int k = t; 2 * k <= L; k += T) {
      const float2 zk = fb[lpad(k)];
      if (k == 0) {
        fb[lpad(0)] = twiddled(make_float2(zk.x * c0, zk.y * c0), make_float2(0.f, 0.f), 0);
      } else {
        const float2 zm = fb[lpad(MF_CHK(L - k, L))];
        const float2 yk = make_float2(zk.x * c1, zk.y * c1), ym = make_float2(zm.x * c1, zm.y * c1);
        fb[lpad(k)] = twiddled(yk, ym, k);
        if (2 * k != L) fb[lpad(L - k)] = twiddled(ym, yk, L - k);
      }
    }
  }
  lds_barrier();
  fft_lds<L, true>(fb, t, true, twl);
  // primal step per (channel, pixel); x and q are fetched here, all at once, and d goes back into
  // the same slot for the forward transform
  float xreg[PER], qreg[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    xreg[i] = el_ok(i) ? ld_stream(el_ptr(a.X, i)) : 0.f;
    qreg[i] = el_ok(i) ? ld_stream(el_ptr(a.Q, i)) : 0.f;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (!FIXP && threadIdx.x + i * NT >= L * PXB) continue;
    const int l = el_l(i), p = el_p(i);
    float* slot = reinterpret_cast<float*>(buf + MF_CHK(p >> 1, NF) * LS + lpad(MF_CHK(dct_slot(l, L), L))) + (p & 1);
    const float tv = *slot;
    float d = 0.f;
    if (el_ok(i)) {
      const float x = xreg[i];
      const float xt = fmaxf(x - a.tau * (qreg[i] + tv), 0.f);
      d = 2.f * xt - x;
      st_stream(el_out(a.D, i), d);
      st_stream(el_out(a.X, i), a.rho * xt + (1.f - a.rho) * x);
    }
    *slot = d;
  }
  lds_barrier();
  fft_lds<L, false>(fb, t, true, twl);
  // spectral dual step per (coefficient, pixel): element i now stands for coefficient k = el_l(i)
  const float s0 = a.smu_l * sqrtf(1.f / L), s1 = a.smu_l * sqrtf(2.f / L);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (!FIXP && threadIdx.x + i * NT >= L * PXB) continue;
    const int k = el_l(i), p = el_p(i);
    const float2* fp = buf + (p >> 1) * LS;
    const float2 zk = fp[lpad(k)];
    const float2 zm = cconj(fp[lpad(MF_CHK(k ? L - k : 0, L))]);
    float2 v;
    if ((p & 1) == 0) {
      v = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    } else {
      v = make_float2(0.5f * (zk.y - zm.y), -0.5f * (zk.x - zm.x));
    }
    const float2 e = a.csL[k];
    const float c = (v.x * e.x + v.y * e.y) * (k ? s1 : s0);
    if (el_ok(i)) {
      const float vo = vreg[i];
      st_stream(el_out(a.V, i), a.rho * satf_s(vo + c) + (1.f - a.rho) * vo);
    }
  }
}

// ------------------------------------------------------------------ Bluestein form of the same step
// For L without an FFT plan the L-point DFTs of the step above run as circular convolutions of a
// length M >= 2L - 1 with an FFT plan (Bluestein's chirp-z identity nk = (n^2 + k^2 - (k - n)^2) / 2):
//   DFT_L(z)_k = c_k sum_{n<L} (z_n c_n) conj(c_{k-n}),   c_n = exp(-i pi n^2 / L),
// i.e. a = z c zero-padded to M, the chirp b_j = conj(c_j) (|j| < L, stored at j mod M), and
// DFT_L(z)_k = c_k IFFT_M(FFT_M(a) FFT_M(b))_k / M for k < L.  The unnormalised inverse DFT is
// conj(DFT_L(conj z)).  The table a.blu holds exp(-2 pi i m / M) (m < M), B = FFT_M(b) and c_n
// (n < L), all from FP64 on the host.
template <int M>
struct BluGeom {
  static constexpr int T = Plan<M>::T;
  static constexpr int NF = (256 / T) > 0 ? (256 / T) : 1;  // transforms (pixel pairs) per block
  static constexpr int PXB = 2 * NF;                        // pixels per block
  static constexpr int LS = lstride<M>();
  static constexpr int NT = NF * T;                          // threads per block (256)
  static constexpr int LMAX = M / 2;                         // largest L served: 2L - 1 <= M (M even)
  static constexpr int PER = (LMAX * PXB + NT - 1) / NT;     // (channel, pixel) elements per thread, at most
  static constexpr size_t shm = sizeof(float2) * (NF * LS + 2 * M + LMAX);
  static_assert(NT % PXB == 0, "a thread keeps one pixel");
};

// The Stockham transform of fft_core.h with the pointwise steps around it folded into its first
// loads and last stores: pre(n, v) is applied to input n as the first stage reads it, post(k, v)
// to output k as the last stage writes it.  Same stages, twiddles and barriers as fft_lds.
template <int N, bool INV, int S = 0, class Pre, class Post>
__device__ __forceinline__ void fft_io(float2* buf, int t, const float2* __restrict__ tw, const Pre& pre,
                                       const Post& post) {
  if constexpr (S == 0) {
    int zero = 0;  // keeps the two transforms' twiddle loads apart (as in fft_lds)
    asm volatile("" : "+s"(zero));
    tw += zero;
  }
  if constexpr (S < Plan<N>::nst) {
    constexpr int T = Plan<N>::T;
    constexpr int R = Plan<N>::rad[S];
    constexpr int Ns = span_before<N>(S);
    constexpr int NB = N / R;
    constexpr int PER = (NB + T - 1) / T;
    constexpr int TWS = N / (Ns * R);
    constexpr bool LAST = S + 1 == Plan<N>::nst;
    float2 v[PER][R];
    float2 w[PER][R];
    if constexpr (Ns > 1) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int k = (t + i * T) % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) w[i][r] = tw[MF_CHK(r * k * TWS, N)];
      }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = t + i * T;
      if (PER * T == NB || b < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          v[i][r] = buf[lpad(MF_CHK(b + r * NB, N))];
          if constexpr (S == 0) v[i][r] = pre(b + r * NB, v[i][r]);
        }
      }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = t + i * T;
      if (PER * T == NB || b < NB) {
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
        for (int r = 0; r < R; ++r) {
          const int pos = MF_CHK(base + r * Ns, N);
          buf[lpad(pos)] = LAST ? post(pos, v[i][r]) : v[i][r];
        }
      }
    }
    lds_barrier();
    fft_io<N, INV, S + 1>(buf, t, tw, pre, post);
  }
}

// One L-point DFT (INV: unnormalised inverse) of slots [0, L) of the transform at fb by its T
// threads, through the length-M convolution; slots [L, M) are ignored on entry and left
// unspecified.  The caller has synchronised the workgroup since fb was last written.
template <int M, bool INV>
__device__ __forceinline__ void blu_dft(float2* fb, int t, int L, const float2* twm, const float2* bh,
                                        const float2* ch) {
  const float inv_m = 1.f / (float)M;
  // FFT_M of a = z c (n < L; INV: conj z), zero beyond, times B
  fft_io<M, false>(
      fb, t, twm,
      [&](int n, float2 z) {
        const float2 c = ch[n < L ? n : 0];
        return n < L ? cmul(INV ? cconj(z) : z, c) : make_float2(0.f, 0.f);
      },
      [&](int k, float2 z) { return cmul(z, bh[k]); });
  // inverse FFT_M, then c_k / M on k < L (INV: conjugated)
  fft_io<M, true>(
      fb, t, twm, [](int, float2 z) { return z; },
      [&](int k, float2 z) {
        const float2 c = ch[k < L ? k : 0];
        const float2 y = cmul(z, c);
        return k < L ? make_float2(y.x * inv_m, (INV ? -y.y : y.y) * inv_m) : z;
      });
}

template <int M>
__global__ void __launch_bounds__(256) k_spectral_blu(SpectralArgs a) {
  using G = BluGeom<M>;
  constexpr int T = G::T, NF = G::NF, PXB = G::PXB, LS = G::LS, NT = G::NT, PER = G::PER;
  const int L = a.L;
  extern __shared__ float2 buf[];  // [NF][LS] transforms, then twiddles [M], B [M], chirp [L]
  float2* twm = buf + NF * LS;
  float2* bh = twm + M;
  float2* ch = bh + M;
  for (int i = threadIdx.x; i < 2 * M + L; i += NT) twm[MF_CHK(i, 2 * M + G::LMAX)] = a.blu[i];
  const long long npix = a.npix, cs = a.cs;
  const long long pix0 = (long long)blockIdx.x * PXB;
  // element i of a thread: channel l0 + i LSTEP of pixel p0 (valid while the channel is < L)
  constexpr int LSTEP = NT / PXB;
  const int l0 = threadIdx.x / PXB, p0 = threadIdx.x - l0 * PXB;
  const bool pok = pix0 + p0 < npix;
  const long long pbase = l0 * cs + pix0 + p0;
  const long long cstep = (long long)LSTEP * cs;
  const int f = threadIdx.x / T, t = threadIdx.x - f * T;
  float2* fb = buf + f * LS;
  float* my = reinterpret_cast<float*>(buf + (p0 >> 1) * LS) + (p0 & 1);  // part p0 & 1 of its transform
  float vreg[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int l = l0 + i * LSTEP;
    vreg[i] = (l < L && pok) ? ld_stream(a.V + pbase + i * cstep) : 0.f;
    if (l < L) my[2 * lpad(MF_CHK(l, L))] = vreg[i];
  }
  lds_barrier();
  {
    // t = mu_l * DCT-III(V): slot k becomes exp(i pi k / 2L) (Y_k - i Y_{L-k}), Y = s h mu_l V
    // (Y_L = 0), for both packed pixels; one thread owns slots k and L - k
    const float c0 = a.mu_l * sqrtf(1.f / L), c1 = a.mu_l * rsqrtf(2.f * L);
    auto twiddled = [&](float2 yk, float2 ym, int k) -> float2 {
      const float2 e = a.csL[k];
      const float2 Va = make_float2(yk.x * e.x + ym.x * e.y, yk.x * e.y - ym.x * e.x);
      const float2 Vb = make_float2(yk.y * e.x + ym.y * e.y, yk.y * e.y - ym.y * e.x);
      return make_float2(Va.x - Vb.y, Va.y + Vb.x);
    };
    for (int k = t; 2 * k <= L; k += T) {
      const float2 zk = fb[lpad(k)];
      if (k == 0) {
        fb[lpad(0)] = twiddled(make_float2(zk.x * c0, zk.y * c0), make_float2(0.f, 0.f), 0);
      } else {
        const float2 zm = fb[lpad(MF_CHK(L - k, L))];
        const float2 yk = make_float2(zk.x * c1, zk.y * c1), ym = make_float2(zm.x * c1, zm.y * c1);
        fb[lpad(k)] = twiddled(yk, ym, k);
        if (2 * k != L) fb[lpad(L - k)] = twiddled(ym, yk, L - k);
      }
    }
  }
  lds_barrier();
  blu_dft<M, true>(fb, t, L, twm, bh, ch);
  // primal step per (channel, pixel); d goes back into the same slot for the forward transform
  float xreg[PER], qreg[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const bool ok = l0 + i * LSTEP < L && pok;
    xreg[i] = ok ? ld_stream(a.X + pbase + i * cstep) : 0.f;
    qreg[i] = ok ? ld_stream(a.Q + pbase + i * cstep) : 0.f;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int l = l0 + i * LSTEP;
    if (l >= L) continue;
    float* slot = my + 2 * lpad(MF_CHK(dct_slot(l, L), L));
    const float tv = *slot;
    float d = 0.f;
    if (pok) {
      const float x = xreg[i];
      const float xt = fmaxf(x - a.tau * (qreg[i] + tv), 0.f);
      d = 2.f * xt - x;
      st_stream(a.D + pbase + i * cstep, d);
      st_stream(a.X + pbase + i * cstep, a.rho * xt + (1.f - a.rho) * x);
    }
    *slot = d;
  }
  lds_barrier();
  blu_dft<M, false>(fb, t, L, twm, bh, ch);
  // spectral dual step per (coefficient, pixel): element i now stands for coefficient k
  const float s0 = a.smu_l * sqrtf(1.f / L), s1 = a.smu_l * sqrtf(2.f / L);
  const float2* fp = buf + (p0 >> 1) * LS;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int k = l0 + i * LSTEP;
    if (k >= L) continue;
    const float2 zk = fp[lpad(k)];
    const float2 zm = cconj(fp[lpad(MF_CHK(k ? L - k : 0, L))]);
    float2 v;
    if ((p0 & 1) == 0) {
      v = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    } else {
      v = make_float2(0.5f * (zk.y - zm.y), -0.5f * (zk.x - zm.x));
    }
    const float2 e = a.csL[k];
    const float c = (v.x * e.x + v.y * e.y) * (k ? s1 : s0);
    if (pok) {
      const float vo = vreg[i];
      st_stream(a.V + pbase + i * cstep, a.rho * satf_s(vo + c) + (1.f - a.rho) * vo);
    }
  }
}

template <int M>
static int spectral_blu_n(const SpectralArgs& a, hipStream_t st) {
  using G = BluGeom<M>;
  const long long nblk = (a.npix + G::PXB - 1) / G::PXB;
  hipLaunchKernelGGL(k_spectral_blu<M>, dim3((unsigned)nblk), dim3(G::NT), G::shm, st, a);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

template <int M>
static int spectral_blu_attr() {
  MF_HIP(hipFuncSetAttribute((const void*)k_spectral_blu<M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)BluGeom<M>::shm));
  return MUFFIN_OK;
}

// Default choice between the Bluestein step and the cosine-table products, from their measured
// times on a 512 x 512 image (the products cost L^2 per pixel and transform, the Bluestein step
// grows with M): the products are faster below 110 channels and from 129 to 215 channels (M = 384
// and 512); beyond 256 channels only the direct kernel is left, which the Bluestein step beats.
bool spectral_blu_default(int L) {
  if (!spectral_blu_m(L)) return false;
  return (L >= 110 && L <= 128) || L >= 216;
}

int spectral_blu_m(int L) {
  if (L < kBluMinL || L > 512 || spectral_has_fft(L)) return 0;
  for (int M : {64, 96, 128, 192, 256, 384, 512, 768, 1024})  // the FFT plans of even thread count
    if (M >= 2 * L - 1) return M;
  return 0;
}

std::vector<float2> spectral_blu_table(int L) {
  const int M = spectral_blu_m(L);
  std::vector<float2> out;
  if (!M) return out;
  out.resize((size_t)2 * M + L);
  std::vector<std::complex<double>> b(M, 0.0), chirp(L);
  for (int n = 0; n < L; ++n) {
    const long long r = ((long long)n * n) % (2LL * L);  // exp(-i pi n^2 / L) has period 2L in n^2
    chirp[n] = std::polar(1.0, -M_PI * (double)r / L);
  }
  for (int j = 0; j < L; ++j) {
    b[j] = std::conj(chirp[j]);
    if (j) b[M - j] = std::conj(chirp[j]);
  }
  for (int m = 0; m < M; ++m) {
    const double th = -2.0 * M_PI * m / M;
    out[m] = make_float2((float)std::cos(th), (float)std::sin(th));
  }
  for (int k = 0; k < M; ++k) {  // B = FFT_M(b), directly in FP64 (M <= 1024, once per context)
    std::complex<double> acc = 0.0;
    for (int j = 0; j < M; ++j) {
      if (b[j] == 0.0) continue;
      acc += b[j] * std::polar(1.0, -2.0 * M_PI * (double)(((long long)j * k) % M) / M);
    }
    out[M + k] = make_float2((float)acc.real(), (float)acc.imag());
  }
  for (int n = 0; n < L; ++n) out[2 * M + n] = make_float2((float)chirp[n].real(), (float)chirp[n].imag());
  return out;
}

template <int L>
static int spectral_fft_n(const SpectralArgs& a, hipStream_t st) {
  using G = SpecGeom<L>;
  const long long nblk = (a.npix + G::PXB - 1) / G::PXB;
  hipLaunchKernelGGL(k_spectral_fft<L>, dim3((unsigned)nblk), dim3(G::NF * G::T), G::shm, st, a);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

template <int L>
static int spectral_fft_attr() {
  MF_HIP(hipFuncSetAttribute((const void*)k_spectral_fft<L>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)SpecGeom<L>::shm));
  return MUFFIN_OK;
}

bool spectral_has_fft(int L) {
  switch (L) {
    case 8: case 16: case 32: case 64: case 128: case 256: case 512:
    case 12: case 24: case 48: case 96: case 192: case 384:
      return true;
    default:
      return false;
  }
}

#define MF_SPEC_DISPATCH(L, fn, ...)        \
  switch (L) {                              \
    case 8: return fn<8>(__VA_ARGS__);      \
    case 16: return fn<16>(__VA_ARGS__);    \
    case 32: return fn<32>(__VA_ARGS__);    \
    case 64: return fn<64>(__VA_ARGS__);    \
    case 128: return fn<128>(__VA_ARGS__);  \
    case 256: return fn<256>(__VA_ARGS__);  \
    case 512: return fn<512>(__VA_ARGS__);  \
    case 12: return fn<12>(__VA_ARGS__);    \
    case 24: return fn<24>(__VA_ARGS__);    \
    case 48: return fn<48>(__VA_ARGS__);    \
    case 96: return fn<96>(__VA_ARGS__);    \
    case 192: return fn<192>(__VA_ARGS__);  \
    case 384: return fn<384>(__VA_ARGS__);  \
    default: break;                         \
  }

int launch_spectral_step(const SpectralArgs& a, hipStream_t st) {
  if (a.use_fft) {
    MF_SPEC_DISPATCH(a.L, spectral_fft_n, a, st)
  }
  if (a.blu) {
    switch (spectral_blu_m(a.L)) {
      case 64: return spectral_blu_n<64>(a, st);
      case 96: return spectral_blu_n<96>(a, st);
      case 128: return spectral_blu_n<128>(a, st);
      case 192: return spectral_blu_n<192>(a, st);
      case 256: return spectral_blu_n<256>(a, st);
      case 384: return spectral_blu_n<384>(a, st);
      case 512: return spectral_blu_n<512>(a, st);
      case 768: return spectral_blu_n<768>(a, st);
      case 1024: return spectral_blu_n<1024>(a, st);
      default: return set_error("spectral: no Bluestein length for L"), MUFFIN_EINVAL;
    }
  }
  if (a.L <= kMatMaxL) {
    // one LDS array of L x PXM; each wave keeps the d of up to MAXM chunks of 8 channels
    const size_t shm = sizeof(float) * (size_t)a.L * PXM;
    const long long nblk = (a.npix + PXM - 1) / PXM;
    if (a.L <= 64) hipLaunchKernelGGL((k_spectral_mat<8, 2>), dim3((unsigned)nblk), dim3(256), shm, st, a);
    else if (a.L <= 128) hipLaunchKernelGGL((k_spectral_mat<8, 4>), dim3((unsigned)nblk), dim3(256), shm, st, a);
    else hipLaunchKernelGGL((k_spectral_mat<8, 8>), dim3((unsigned)nblk), dim3(256), shm, st, a);
    MF_HIP(hipGetLastError());
    return MUFFIN_OK;
  }
  const size_t shm = sizeof(float) * 2 * (size_t)a.L * PX;
  const long long nblk = (a.npix + PX - 1) / PX;
  hipLaunchKernelGGL(k_spectral_step, dim3((unsigned)nblk), dim3(256), shm, st, a);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// out[i] = sum_j M[i][j] in[j] per pixel (M = W^T: forward DCT-II; M = W: inverse), or the FP64
// sum of |out| per workgroup.
template <bool ABS>
__global__ void __launch_bounds__(256) k_pix_matvec(const float* __restrict__ in, float* __restrict__ out,
                                                    const float* __restrict__ M, long long npix, long long cs, int L,
                                                    double* __restrict__ partial) {
  // 64 pixels per workgroup, one per lane; a wave computes 8 output rows at a time from
  // wave-uniform matrix rows (scalar loads), each LDS read feeding 8 FMAs; sums run over j in order
  constexpr int CW = 8;
  extern __shared__ float sm[];
  float* Is = sm;  // [L][PXM]
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long pix = (long long)blockIdx.x * PXM + lane;
  const bool pok = pix < npix;
  for (int l = wv; l < L; l += 4) Is[l * PXM + lane] = pok ? in[(long long)l * cs + pix] : 0.f;
  lds_barrier();
  double acc_abs = 0.0;
  for (int i0 = wv * CW; i0 < L; i0 += 4 * CW) {
    float acc[CW];
    const_fp Mr[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      acc[c] = 0.f;
      Mr[c] = (const_fp)(M + (long long)min(i0 + c, L - 1) * L);
    }
#pragma unroll 4
    for (int j = 0; j < L; ++j) {
      const float v = Is[j * PXM + lane];
#pragma unroll
      for (int c = 0; c < CW; ++c) acc[c] = fmaf(Mr[c][j], v, acc[c]);
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      const int r = i0 + c;
      if (r < L && pok) {
        if (ABS) acc_abs += fabs((double)acc[c]);
        else out[(long long)r * cs + pix] = acc[c];
      }
    }
  }
  if constexpr (ABS) {
    for (int off = 32; off > 0; off >>= 1) acc_abs += __shfl_down(acc_abs, off, 64);
    __shared__ double red[4];
    if (lane == 0) red[wv] = acc_abs;
    lds_barrier();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

int launch_dct(const float* in, float* out, const float* Wmat, long long npix, long long cs, int L, hipStream_t st) {
  const size_t shm = sizeof(float) * (size_t)L * PXM;
  const long long nblk = (npix + PXM - 1) / PXM;
  hipLaunchKernelGGL(k_pix_matvec<false>, dim3((unsigned)nblk), dim3(256), shm, st, in, out, Wmat, npix, cs, L,
                     (double*)nullptr);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int launch_dct_abs(const float* in, const float* WT, long long npix, long long cs, int L, double* partial,
                   int* nblocks_out,
                   hipStream_t st) {
  const size_t shm = sizeof(float) * (size_t)L * PXM;
  const long long nblk = (npix + PXM - 1) / PXM;
  if (nblk > kMaxPartials) {
    set_error("dct_abs: too many blocks for the partial-sum buffer");
    return MUFFIN_EINVAL;
  }
  if (nblocks_out) *nblocks_out = (int)nblk;
  hipLaunchKernelGGL(k_pix_matvec<true>, dim3((unsigned)nblk), dim3(256), shm, st, in, (float*)nullptr, WT, npix,
                     cs, L, partial);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int spectral_direct_attrs(int L) {
  const int shm = (int)(sizeof(float) * 2 * (size_t)L * PX);
  MF_HIP(hipFuncSetAttribute((const void*)k_spectral_step, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_spectral_mat<8, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(float) * kMatMaxL * PXM)));
  MF_HIP(hipFuncSetAttribute((const void*)k_pix_matvec<false>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_pix_matvec<true>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  return MUFFIN_OK;
}

int spectral_init_attrs(int L) {
  MF_TRY(spectral_direct_attrs(L));
  if (spectral_has_fft(L)) {
    MF_SPEC_DISPATCH(L, spectral_fft_attr)
  }
  switch (spectral_blu_m(L)) {
    case 64: MF_TRY(spectral_blu_attr<64>()); break;
    case 96: MF_TRY(spectral_blu_attr<96>()); break;
    case 128: MF_TRY(spectral_blu_attr<128>()); break;
    case 192: MF_TRY(spectral_blu_attr<192>()); break;
    case 256: MF_TRY(spectral_blu_attr<256>()); break;
    case 384: MF_TRY(spectral_blu_attr<384>()); break;
    case 512: MF_TRY(spectral_blu_attr<512>()); break;
    case 768: MF_TRY(spectral_blu_attr<768>()); break;
    case 1024: MF_TRY(spectral_blu_attr<1024>()); break;
    default: break;
  }
  return MUFFIN_OK;
}

#ifdef MF_CHECKED
int oob_take_spectral(unsigned long long* n) { return oob_take_here(n); }
#endif

}  // namespace mf
