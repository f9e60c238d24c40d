// Per-pixel spectral work: the fused step that takes the paper's master-node role (Sec. 3),
//   t   = mu_l V W^T                   (spectral adjoint of the dual, orthonormal DCT-III)
//   x~  = (x - tau (q + t))_+          (primal proximal step; q = gradient + mu_s W_s^dagger u)
//   d   = 2 x~ - x
//   V   <- rho sat(V + sigma mu_l d W) + (1 - rho) V      (spectral dual step, DCT-II)
//   x   <- rho x~ + (1 - rho) x
// A workgroup owns 32 pixels across all L channels: it stages their V spectra and their d spectra
// in LDS ([L][32] each), reads x and q once, and writes x, d and V once.  The length-L cosine
// transforms are dense products with a cosine table, each thread accumulating four outputs so
// every LDS read feeds four FMAs.
#include "common.h"

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
    Vs[idx] = (q < a.npix) ? a.V[(long long)l * a.npix + q] : 0.f;
  }
  __syncthreads();
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
          const long long o = (long long)l * a.npix + pix;
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
  __syncthreads();
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
        a.V[(long long)k * a.npix + pix] = a.rho * satf_s(v + a.smu_l * acc[i]) + (1.f - a.rho) * v;
      }
    }
  }
}

int launch_spectral_step(const SpectralArgs& a, hipStream_t st) {
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
                                                    const float* __restrict__ M, long long npix, int L,
                                                    double* __restrict__ partial) {
  extern __shared__ float sm[];
  float* Is = sm;  // [L][PX]
  const int p = threadIdx.x & (PX - 1);
  const int g = threadIdx.x >> 5;
  const long long pix0 = (long long)blockIdx.x * PX;
  const long long pix = pix0 + p;
  for (int idx = threadIdx.x; idx < L * PX; idx += 256) {
    const int l = idx / PX, pp = idx % PX;
    const long long q = pix0 + pp;
    Is[idx] = (q < npix) ? in[(long long)l * npix + q] : 0.f;
  }
  __syncthreads();
  double acc_abs = 0.0;
  for (int ib = g; ib < L; ib += 32) {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < L; ++j) {
      const float v = Is[j * PX + p];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (ib + 8 * i < L) acc[i] = fmaf(M[(ib + 8 * i) * L + j], v, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ib + 8 * i;
      if (r < L && pix < npix) {
        if (ABS) acc_abs += fabs((double)acc[i]);
        else out[(long long)r * npix + pix] = acc[i];
      }
    }
  }
  if constexpr (ABS) {
    for (int off = 32; off > 0; off >>= 1) acc_abs += __shfl_down(acc_abs, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc_abs;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

int launch_dct(const float* in, float* out, const float* Wmat, long long npix, int L, hipStream_t st) {
  const size_t shm = sizeof(float) * (size_t)L * PX;
  const long long nblk = (npix + PX - 1) / PX;
  hipLaunchKernelGGL(k_pix_matvec<false>, dim3((unsigned)nblk), dim3(256), shm, st, in, out, Wmat, npix, L,
                     (double*)nullptr);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int launch_dct_abs(const float* in, const float* WT, long long npix, int L, double* partial, int* nblocks_out,
                   hipStream_t st) {
  const size_t shm = sizeof(float) * (size_t)L * PX;
  const long long nblk = (npix + PX - 1) / PX;
  if (nblk > kMaxPartials) {
    set_error("dct_abs: too many blocks for the partial-sum buffer");
    return MUFFIN_EINVAL;
  }
  if (nblocks_out) *nblocks_out = (int)nblk;
  hipLaunchKernelGGL(k_pix_matvec<true>, dim3((unsigned)nblk), dim3(256), shm, st, in, (float*)nullptr, WT, npix,
                     L, partial);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int spectral_init_attrs(int L) {
  const int shm = (int)(sizeof(float) * 2 * (size_t)L * PX);
  MF_HIP(hipFuncSetAttribute((const void*)k_spectral_step, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_pix_matvec<false>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_pix_matvec<true>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  return MUFFIN_OK;
}

}  // namespace mf
