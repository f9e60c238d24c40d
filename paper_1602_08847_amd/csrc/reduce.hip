// FP64 reductions on the device: block partials are written by the producing kernels and
// finished here in a fixed order, so every result is deterministic.
#include "common.h"

#include <cmath>

namespace mf {

__global__ void __launch_bounds__(1024) k_reduce_sum(const double* __restrict__ partial, int n,
                                                     double* __restrict__ dst, int accumulate) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *dst = accumulate ? *dst + red[0] : red[0];
}

int launch_reduce_sum(const double* partial, int n, double* dst, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(1024), 0, st, partial, n, dst, accumulate);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

__global__ void __launch_bounds__(256) k_max_partial(const float* __restrict__ x, long long n, double scale,
                                                     double* __restrict__ partial) {
  __shared__ double red[256];
  double m = -INFINITY;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    m = fmax(m, (double)x[i] * scale);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_max_final(const double* __restrict__ partial, int n, double* __restrict__ dst) {
  __shared__ double red[1024];
  double m = -INFINITY;
  for (int i = threadIdx.x; i < n; i += 1024) m = fmax(m, partial[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dst = red[0];
}

int launch_reduce_max(const float* x, long long n, double scale, double* partial, double* dst, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_max_partial, dim3((unsigned)nb), dim3(256), 0, st, x, n, scale, partial);
  MF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(1024), 0, st, partial, (int)nb, dst);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// Symbol of W_s^dagger diag(omega) W_s at DFT frequency (k1, k2): plane j+1 has symbol
// prod_{i<j} h_i (1 - h_j^g) (g = 1 or 2 by generation), the coarse plane prod_{i<J} h_i, where
// h_i = b(2^i w1) b(2^i w2) and b(w) = 3/8 + cos(w)/2 + cos(2w)/8 is the B3 filter response.
__device__ double b3_resp(double w) { return 0.375 + 0.5 * cos(w) + 0.125 * cos(2.0 * w); }

__global__ void __launch_bounds__(256) k_frame_symbol(int N, int J, int gen, double omega_coarse,
                                                      double* __restrict__ partial) {
  __shared__ double red[256];
  const long long n = (long long)N * N;
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double w1 = 2.0 * M_PI * (double)(i / N) / N, w2 = 2.0 * M_PI * (double)(i % N) / N;
    double prod = 1.0, tot = 0.0;
    for (int j = 0; j < J; ++j) {
      const double sc = (double)(1 << j);
      const double h = b3_resp(sc * w1) * b3_resp(sc * w2);
      const double g = prod * (gen == 1 ? 1.0 - h : 1.0 - h * h);
      tot += g * g;
      prod *= h;
    }
    tot += omega_coarse * prod * prod;
    m = fmax(m, tot);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

int launch_frame_bound(int N, int J, int gen, double omega_coarse, double* partial, double* dst, hipStream_t st) {
  long long nb = ((long long)N * N + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_frame_symbol, dim3((unsigned)nb), dim3(256), 0, st, N, J, gen, omega_coarse, partial);
  MF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(1024), 0, st, partial, (int)nb, dst);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

__global__ void __launch_bounds__(256) k_nonfinite(const float* __restrict__ x, long long n, double* __restrict__ partial) {
  __shared__ double red[256];
  double c = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    c += isfinite(x[i]) ? 0.0 : 1.0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

int launch_count_nonfinite(const float* x, long long n, double* partial, double* dst, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)nb), dim3(256), 0, st, x, n, partial);
  MF_HIP(hipGetLastError());
  return launch_reduce_sum(partial, (int)nb, dst, 1, st);
}

}  // namespace mf
