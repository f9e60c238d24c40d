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

// Squared distances for the convergence norms and the SNR: over nplanes planes of npix floats
// (plane k of a at a + k acs, of b at b + k bcs), partial[blk] = sum (a - b)^2 and
// partial[nblk + blk] = sum a^2, in FP64 (b == NULL reads as 0).
__global__ void __launch_bounds__(256) k_diff_norms(const float* __restrict__ a, long long acs,
                                                    const float* __restrict__ b, long long bcs, long long npix,
                                                    double* __restrict__ partial) {
  __shared__ double r0[256], r1[256];
  const long long k = blockIdx.y;
  const float* ap = a + k * acs;
  const float* bp = b ? b + k * bcs : nullptr;
  double sd = 0.0, sa = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < npix; i += (long long)gridDim.x * 256) {
    const double av = (double)ap[i];
    const double d = bp ? av - (double)bp[i] : av;
    sd += d * d;
    sa += av * av;
  }
  r0[threadIdx.x] = sd;
  r1[threadIdx.x] = sa;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long long nblk = (long long)gridDim.x * gridDim.y;
    const long long blk = k * gridDim.x + blockIdx.x;
    partial[blk] = r0[0];
    partial[nblk + blk] = r1[0];
  }
}

int launch_diff_norms(const float* a, long long acs, const float* b, long long bcs, long long npix, int nplanes,
                      double* partial, double* dst_diff, double* dst_a, int accumulate, hipStream_t st) {
  if (nplanes < 1 || npix < 1) return set_error("diff_norms: empty operand"), MUFFIN_EINVAL;
  if (nplanes > 65535) return set_error("diff_norms: too many planes"), MUFFIN_EINVAL;
  long long per = (npix + 4 * 256 - 1) / (4 * 256);
  if (per > 64) per = 64;
  while (per > 1 && per * nplanes * 2 > kMaxPartials) per >>= 1;
  const long long nblk = per * nplanes;
  if (2 * nblk > kMaxPartials) return set_error("diff_norms: too many blocks for the partial sums"), MUFFIN_EINVAL;
  hipLaunchKernelGGL(k_diff_norms, dim3((unsigned)per, (unsigned)nplanes), dim3(256), 0, st, a, acs, b, bcs, npix,
                     partial);
  MF_HIP(hipGetLastError());
  MF_TRY(launch_reduce_sum(partial, (int)nblk, dst_diff, accumulate, st));
  return launch_reduce_sum(partial + nblk, (int)nblk, dst_a, accumulate, st);
}

}  // namespace mf
