// Isotropic undecimated wavelet transform (B3-spline a trous, periodic boundary) building blocks.
//
// H_j is the separable smoothing by [1, 4, 6, 4, 1] / 16 with taps 2^j apart along each axis.
// A workgroup owns a TX x TY output tile of one channel; it loads the tile plus a halo of 2^(j+1)
// pixels on every side (wrapped periodically) into LDS, filters the columns into a second LDS
// buffer, filters the rows, and applies one of the fused epilogues:
//   AT_SMOOTH      out = H_j A                           (analysis: c_{j+1} = H_j c_j)
//   AT_SUBADD      out = E + H_j (A - B)                 (adjoint Horner step, both generations)
//   AT_DETAIL      w = E - H_j A, u <- rho sat(u + coef w) + (1 - rho) u   (gen-2 detail + dual step)
//   AT_DETAIL_ABS  partial = sum |E - H_j A|             (objective, FP64)
#include "common.h"

namespace mf {

__device__ __forceinline__ int wrapi(int v, int N) {
  v %= N;
  return v < 0 ? v + N : v;
}

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
  PlaneRef A, B, E;
  PlaneOut out;
  int N, j, TX, TY;
  int tiles_x, tiles_y;
  float coef, rho;
  double* partial;
};

template <int MODE>
__global__ void __launch_bounds__(256) k_atrous(AtrousArgs a) {
  extern __shared__ float sm[];
  const int N = a.N;
  const int s = 1 << a.j;      // tap spacing
  const int h = 2 * s;         // halo
  const int TX = a.TX, TY = a.TY;
  const int W = TX + 2 * h, Hh = TY + 2 * h;
  float* in = sm;              // [Hh][W]
  float* mid = sm + Hh * W;    // [TY][W]
  const int tile = blockIdx.x;
  const int ch = blockIdx.y;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int x0 = tx * TX, y0 = ty * TY;
  const float* A = a.A.p + ch * a.A.cs;
  const float* B = (MODE == AT_SUBADD) ? a.B.p + ch * a.B.cs : nullptr;
  for (int idx = threadIdx.x; idx < Hh * W; idx += blockDim.x) {
    const int yy = idx / W, xx = idx - yy * W;
    const long long g = (long long)wrapi(y0 - h + yy, N) * N + wrapi(x0 - h + xx, N);
    float v = A[g];
    if (MODE == AT_SUBADD) v -= B[g];
    in[idx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TY * W; idx += blockDim.x) {
    const int yy = idx / W, xx = idx - yy * W;
    const float* c = in + yy * W + xx;  // taps at rows yy + {0, s, 2s, 3s, 4s}
    mid[idx] = 0.0625f * (c[0] + c[4 * s * W]) + 0.25f * (c[s * W] + c[3 * s * W]) + 0.375f * c[2 * s * W];
  }
  __syncthreads();
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < TY * TX; idx += blockDim.x) {
    const int yy = idx / TX, xx = idx - yy * TX;
    const float* c = mid + yy * W + xx;
    const float v = 0.0625f * (c[0] + c[4 * s]) + 0.25f * (c[s] + c[3 * s]) + 0.375f * c[2 * s];
    const long long g = (long long)(y0 + yy) * N + (x0 + xx);
    if constexpr (MODE == AT_SMOOTH) {
      a.out.p[ch * a.out.cs + g] = v;
    } else if constexpr (MODE == AT_SUBADD) {
      a.out.p[ch * a.out.cs + g] = a.E.p[ch * a.E.cs + g] + v;
    } else if constexpr (MODE == AT_DETAIL) {
      const float w = a.E.p[ch * a.E.cs + g] - v;
      float* up = a.out.p + ch * a.out.cs + g;
      const float u = *up;
      *up = a.rho * satf(u + a.coef * w) + (1.f - a.rho) * u;
    } else {
      acc += fabs((double)a.E.p[ch * a.E.cs + g] - (double)v);
    }
  }
  if constexpr (MODE == AT_DETAIL_ABS) {
    const double tot = block_sum_atrous(acc);
    if (threadIdx.x == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = tot;
  }
}

static void tile_shape(int N, int j, int& TX, int& TY) {
  // widest row tile that divides N (coalesced rows), height chosen to bound LDS
  TX = 64;
  while (N % TX) TX >>= 1;
  const int h = 2 << j;
  TY = 32;
  while (TY > 4 && (size_t)((TY + 2 * h) * (TX + 2 * h) + TY * (TX + 2 * h)) * 4 > 96 * 1024) TY >>= 1;
  while (N % TY) TY >>= 1;
}

int launch_atrous(int mode, int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneOut out, float coef,
                  float rho, double* partial, int* nblocks_out, hipStream_t st) {
  AtrousArgs a;
  a.A = A;
  a.B = B;
  a.E = E;
  a.out = out;
  a.N = N;
  a.j = j;
  tile_shape(N, j, a.TX, a.TY);
  a.tiles_x = N / a.TX;
  a.tiles_y = N / a.TY;
  a.coef = coef;
  a.rho = rho;
  a.partial = partial;
  const int h = 2 << j;
  const size_t shm = sizeof(float) * ((size_t)(a.TY + 2 * h) * (a.TX + 2 * h) + (size_t)a.TY * (a.TX + 2 * h));
  if (shm > 144 * 1024) {
    set_error("atrous: scale too coarse for the LDS tile");
    return MUFFIN_EINVAL;
  }
  const dim3 grid((unsigned)(a.tiles_x * a.tiles_y), (unsigned)nch);
  if (nblocks_out) *nblocks_out = (int)(grid.x * grid.y);
  if (mode == AT_DETAIL_ABS && (long long)grid.x * grid.y > kMaxPartials) {
    set_error("atrous: too many blocks for the partial-sum buffer");
    return MUFFIN_EINVAL;
  }
  switch (mode) {
    case AT_SMOOTH: hipLaunchKernelGGL(k_atrous<AT_SMOOTH>, grid, dim3(256), shm, st, a); break;
    case AT_SUBADD: hipLaunchKernelGGL(k_atrous<AT_SUBADD>, grid, dim3(256), shm, st, a); break;
    case AT_DETAIL: hipLaunchKernelGGL(k_atrous<AT_DETAIL>, grid, dim3(256), shm, st, a); break;
    case AT_DETAIL_ABS: hipLaunchKernelGGL(k_atrous<AT_DETAIL_ABS>, grid, dim3(256), shm, st, a); break;
    default: set_error("atrous: bad mode"); return MUFFIN_EINVAL;
  }
  MF_HIP(hipGetLastError());
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
      *up = a.rho * satf(u + a.coef * w) + (1.f - a.rho) * u;
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

int atrous_init_attrs() {
  const int shm = 144 * 1024;  // leaves room for the static LDS of the reduction variants
  MF_HIP(hipFuncSetAttribute((const void*)k_atrous<AT_SMOOTH>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_atrous<AT_SUBADD>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_atrous<AT_DETAIL>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_atrous<AT_DETAIL_ABS>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
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
                                                        long long npix) {
  const float s = w[blockIdx.y];
  float* xc = x + (long long)blockIdx.y * npix;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < npix; i += (long long)gridDim.x * 256)
    xc[i] *= s;
}

int launch_scale_channels(float* x, const float* chan_w, long long npix, int nch, hipStream_t st) {
  long long nb = (npix + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_scale_channels, dim3((unsigned)nb, (unsigned)nch), dim3(256), 0, st, x, chan_w, npix);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

}  // namespace mf
