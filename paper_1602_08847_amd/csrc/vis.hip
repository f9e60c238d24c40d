// Visibility-domain data term (Sec. 2, eq. (viseq)): Phi maps a channel image to its K complex
// visibilities, v_k = sum_p x_p / n_p exp(-2 pi i (u_k l_p + v_k m_p + w_k n_p)), with (u, v, w) the
// baseline in wavelengths of the channel and (l, m, n) the direction cosines of pixel p
// (n = sqrt(1 - l^2 - m^2)); the w n term is the direction-dependent effect that keeps Phi from
// being a Fourier transform.  The data term 1/2 ||v - Phi x||^2 has the gradient
// Re Phi^H (Phi x - v).
//
// Both directions are direct sums over all (visibility, pixel) pairs, evaluated exactly rather
// than through a gridded approximation.  Each pair costs one phase and one complex exponential,
// so the kernels are bound by VALU issue, not by memory:
//  * the phase is formed in FP64 (two FMAs with the per-row or per-visibility part hoisted), its
//    integer number of turns dropped exactly (v_fract_f64), and the fraction converted to FP32;
//  * the hardware sine and cosine take the angle in turns, so no range reduction is left;
//  * products and sums are FP32.
// Forward (k_vis_fwd): a lane holds one visibility and a wave walks a band of image rows, so the
// pixel data (l_j, n_ij, x_ij / n_ij) are uniform across the wave and come in through scalar loads.
// The bands' partial sums are added in a fixed order by k_vis_resid, which subtracts the data and
// stores the residual next to the baseline.  Adjoint (k_vis_adj): a lane holds four neighbouring
// pixels of one row and walks all visibilities, whose baseline and residual are again wave-uniform
// scalar loads; the epilogue applies 1/n and adds the spatial adjoint term of the primal step.
#include "common.h"

namespace mf {

typedef const double __attribute__((address_space(4)))* cdp;
typedef const float __attribute__((address_space(4)))* cfp;
typedef const VisPt __attribute__((address_space(4)))* cvp;

// cos and sin of 2 pi ph for a phase ph in turns
__device__ __forceinline__ void cis_turns(double ph, float& c, float& s) {
  const float f = (float)__builtin_amdgcn_fract(ph);
  c = __builtin_amdgcn_cosf(f);
  s = __builtin_amdgcn_sinf(f);
}

// XN[l][p] = X[l][p] / n_p over the dense N x N planes (X in slots of cs floats).
__global__ void __launch_bounds__(256) k_vis_xn(const float* __restrict__ X, long long cs,
                                                const float* __restrict__ invn, float* __restrict__ XN,
                                                long long np) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long l = blockIdx.y;
  if (p < np) XN[l * np + MF_CHK(p, np)] = X[l * cs + p] * invn[p];
}

int launch_vis_xn(const float* X, long long cs, const float* invn, float* XN, int N, int L, hipStream_t st) {
  const long long np = (long long)N * N;
  hipLaunchKernelGGL(k_vis_xn, dim3((unsigned)((np + 255) / 256), (unsigned)L), dim3(256), 0, st, X, cs, invn, XN,
                     np);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// Rows per band of the forward pass: enough bands that L x ceil(K / 64) x bands waves fill the
// GPU several times over (eight waves per SIMD of 256 compute units).
int vis_chunks(int N, int K, int L) {
  const long long waves = (long long)L * ((K + 63) / 64);
  long long C = (8192 + waves - 1) / waves;
  if (C < 1) C = 1;
  if (C > N) C = N;
  const long long R = (N + C - 1) / C;
  return (int)((N + R - 1) / R);
}

// part[c][l][k] = sum over the rows of band c of x_ij / n_ij exp(-2 pi i phase), one wave per
// (64 visibilities, band, channel); waves with the same channel and band are adjacent.
__global__ void __launch_bounds__(256) k_vis_fwd(const VisPt* __restrict__ vp, const float* __restrict__ XN,
                                                 const double* __restrict__ lt, const double* __restrict__ nt,
                                                 float2* __restrict__ part, int N, int K, int L, int G, int C,
                                                 int R) {
  const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  const int lane = threadIdx.x & 63;
  if (wave >= L * G * C) return;
  const int g = wave % G;
  const int c = (wave / G) % C;
  const int l = wave / (G * C);
  const int k = g * 64 + lane;
  const bool ok = k < K;
  const VisPt p = vp[(long long)l * K + MF_CHK(ok ? k : K - 1, K)];
  const double u = p.u, v = p.v, w = p.w;
  float are = 0.f, aim = 0.f;
  const int i0 = c * R, i1 = min(N, i0 + R);
  const long long np = (long long)N * N;
  const cdp lrow = (cdp)lt;
  for (int i = i0; i < i1; ++i) {
    const double vm = v * lrow[MF_CHK(i, N)];
    const cdp nrow = (cdp)(nt + (long long)i * N);
    const cfp xrow = (cfp)(XN + (long long)l * np + (long long)i * N);
    for (int j = 0; j < N; j += 8) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const double ph = fma(u, lrow[MF_CHK(j + t, N)], fma(w, nrow[MF_CHK(j + t, N)], vm));
        float cc, ss;
        cis_turns(ph, cc, ss);
        const float x = xrow[j + t];
        are = fmaf(x, cc, are);
        aim = fmaf(-x, ss, aim);
      }
    }
  }
  if (ok) part[((long long)c * L + l) * K + k] = make_float2(are, aim);
}

int launch_vis_fwd(const VisPt* vp, const float* XN, const double* lt, const double* nt, float2* part, int N, int K,
                   int L, int C, hipStream_t st) {
  if (N % 8) return set_error("visibility kernels need N to be a multiple of 8"), MUFFIN_EINVAL;
  const int G = (K + 63) / 64;
  const int R = (N + C - 1) / C;
  if ((long long)(C - 1) * R >= N) return set_error("visibility forward: empty row band"), MUFFIN_EINVAL;
  const long long waves = (long long)L * G * C;
  hipLaunchKernelGGL(k_vis_fwd, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, vp, XN, lt, nt, part, N, K, L,
                     G, C, R);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// r = sum_c part[c] + vsign vis (vis may be NULL), stored in vp (and in rout when it is not NULL);
// partial[block] = 1/2 sum |r|^2 in FP64 when partial is not NULL.
__global__ void __launch_bounds__(256) k_vis_resid(const float2* __restrict__ part, int C, long long LK,
                                                   const float2* __restrict__ vis, float vsign,
                                                   VisPt* __restrict__ vp, double* __restrict__ partial,
                                                   float2* __restrict__ rout) {
  __shared__ double red[256];
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (t < LK) {
    float re = 0.f, im = 0.f;
    for (int c = 0; c < C; ++c) {
      const float2 q = part[(long long)c * LK + t];
      re += q.x;
      im += q.y;
    }
    if (vis) {
      re = fmaf(vsign, vis[t].x, re);
      im = fmaf(vsign, vis[t].y, im);
    }
    vp[MF_CHK(t, LK)].rre = re;
    vp[t].rim = im;
    if (rout) rout[t] = make_float2(re, im);
    e = (double)re * re + (double)im * im;
  }
  if (!partial) return;
  red[threadIdx.x] = e;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = 0.5 * red[0];
}

int launch_vis_resid(const float2* part, int C, int L, int K, const float2* vis, float vsign, VisPt* vp,
                     double* partial, int* nblocks, float2* rout, hipStream_t st) {
  const long long LK = (long long)L * K;
  const long long nb = (LK + 255) / 256;
  if (partial && nb > kMaxPartials) return set_error("visibility residual: too many blocks"), MUFFIN_EINVAL;
  hipLaunchKernelGGL(k_vis_resid, dim3((unsigned)nb), dim3(256), 0, st, part, C, LK, vis, vsign, vp, partial, rout);
  MF_HIP(hipGetLastError());
  if (nblocks) *nblocks = (int)nb;
  return MUFFIN_OK;
}

// out[l][p] = (1/n_p) Re sum_k r_k exp(+2 pi i phase_kp) (+ s_scale sadd[l][p]); four pixels of one
// row per lane.
__global__ void __launch_bounds__(256) k_vis_adj(const VisPt* __restrict__ vp, int K, const double* __restrict__ lt,
                                                 const double* __restrict__ nt, const float* __restrict__ invn,
                                                 int N, float* __restrict__ out, long long out_cs,
                                                 const float* __restrict__ sadd, long long s_cs, float s_scale) {
  const long long np = (long long)N * N;
  const long long l = blockIdx.y;
  const long long p0 = 4 * ((long long)blockIdx.x * 256 + threadIdx.x);
  if (p0 >= np) return;
  const int i = (int)(p0 / N), j0 = (int)(p0 - (long long)i * N);
  const double m = lt[MF_CHK(i, N)];
  double lj[4], nj[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    lj[t] = lt[MF_CHK(j0 + t, N)];
    nj[t] = nt[MF_CHK(p0 + t, np)];
  }
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const cvp vq = (cvp)(vp + l * K);
#pragma unroll 2
  for (int k = 0; k < K; ++k) {
    const double u = vq[k].u, v = vq[k].v, w = vq[k].w;  // wave-uniform: scalar loads
    const float a = vq[k].rre, b = vq[k].rim;
    const double vm = v * m;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double ph = fma(u, lj[t], fma(w, nj[t], vm));
      float cc, ss;
      cis_turns(ph, cc, ss);
      acc[t] = fmaf(a, cc, acc[t]);
      acc[t] = fmaf(-b, ss, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float q = acc[t] * invn[p0 + t];
    if (sadd) q = fmaf(s_scale, sadd[l * s_cs + p0 + t], q);
    out[l * out_cs + p0 + t] = q;
  }
}

int launch_vis_adj(const VisPt* vp, int K, int L, const double* lt, const double* nt, const float* invn, int N,
                   float* out, long long out_cs, const float* sadd, long long s_cs, float s_scale, hipStream_t st) {
  if (N % 8) return set_error("visibility kernels need N to be a multiple of 8"), MUFFIN_EINVAL;
  const long long np = (long long)N * N;
  const long long nb = (np / 4 + 255) / 256;
  hipLaunchKernelGGL(k_vis_adj, dim3((unsigned)nb, (unsigned)L), dim3(256), 0, st, vp, K, lt, nt, invn, N, out,
                     out_cs, sadd, s_cs, s_scale);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// x[l][p] *= f over the dense planes of a cube in slots of cs floats.
__global__ void __launch_bounds__(256) k_vis_scale(float* __restrict__ x, long long cs, long long np, float f) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p < np) x[(long long)blockIdx.y * cs + p] *= f;
}

int launch_vis_scale(float* x, long long cs, int N, int L, float f, hipStream_t st) {
  const long long np = (long long)N * N;
  hipLaunchKernelGGL(k_vis_scale, dim3((unsigned)((np + 255) / 256), (unsigned)L), dim3(256), 0, st, x, cs, np, f);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

#ifdef MF_CHECKED
int oob_take_vis(unsigned long long* n) { return oob_take_here(n); }
#endif

}  // namespace mf
