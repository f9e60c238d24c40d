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
template <int L>
struct SpecGeom {
  static constexpr int T = Plan<L>::T;
  static constexpr int NF = (256 / T) > 0 ? (256 / T) : 1;  // transforms (pixel pairs) per block
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
      reinterpret_cast<float*>(buf + (p >> 1) * LS + lpad(el_l(i)))[p & 1] = vreg[i];
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
        const float2 zm = fb[lpad(L - k)];
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
    float* slot = reinterpret_cast<float*>(buf + (p >> 1) * LS + lpad(dct_slot(l, L))) + (p & 1);
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
    const float2 zm = cconj(fp[lpad(k ? L - k : 0)]);
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
  return MUFFIN_OK;
}

}  // namespace mf
