// Visibility-domain data term (Sec. 2, eq. (viseq)): Phi maps a channel image to its K complex
// visibilities, v_k = sum_p x_p / n_p exp(-2 pi i (u_k l_p + v_k m_p + w_k n_p)), with (u, v, w) the
// baseline in wavelengths of the channel and (l, m, n) the direction cosines of pixel p
// (n = sqrt(1 - l^2 - m^2)); the w n term is the direction-dependent effect that keeps Phi from
// being a Fourier transform.  The data term w_l/2 ||v - Phi x||^2 (w_l the channel's weight) has
// the gradient w_l Re Phi^H (Phi x - v).
//
// Both directions are direct sums over all (visibility, pixel) pairs, evaluated exactly rather
// than through a gridded approximation.  Each pair costs one phase and one complex exponential,
// so the kernels are bound by VALU issue, not by memory:
//  * the phase is formed in FP64 (two FMAs with the per-row or per-visibility part hoisted), its
//    integer number of turns dropped exactly (v_fract_f64), and the fraction converted to FP32;
//  * the hardware sine and cosine take the angle in turns, so no range reduction is left;
//  * products and sums are FP32.
// Forward (k_vis_fwd): a lane holds one visibility and a wave walks a band of image rows, so the
// pixel data (l_j, n_ij, x_ij / n_ij) are the same for every lane: they are staged in LDS and read
// as broadcasts.  The bands' partial sums are added in a fixed order by k_vis_resid, which
// subtracts the data and stores the residual next to the baseline.  Adjoint (k_vis_adj): a lane
// holds four neighbouring pixels of one row and walks all visibilities, whose baseline and residual
// are again staged in LDS; the epilogue applies 1/n and adds the spatial adjoint term of the primal
// step.
#include "common.h"

namespace mf {

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

// Row bands of the forward pass: enough that L x ceil(K / 256) x 4 x bands waves fill the GPU four
// times over at eight waves per SIMD (256 compute units), so that the last round's tail is short.
int vis_chunks(int N, int K, int L) {
  const long long waves = (long long)L * ((K + 255) / 256) * 4;
  long long C = (32768 + waves - 1) / waves;
  if (C < 1) C = 1;
  if (C > N) C = N;
  const long long R = (N + C - 1) / C;
  return (int)((N + R - 1) / R);
}

// Four pixels of one staged image row as the forward pass reads them: l_j, n_ij, x_ij / n_ij.
struct PixQuad {
  double lj[4], nj[4];
  float xj[4];
  __device__ __forceinline__ void load(const double* sl, const double* nrow, const float* xrow, int j, int N) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      lj[t] = sl[MF_CHK(j + t, N)];
      nj[t] = nrow[MF_CHK(j + t, N)];
      xj[t] = xrow[MF_CHK(j + t, N)];
    }
  }
  // sum += x exp(-2 pi i phase), phase = u l + w n + vm; even pixels into slot 0, odd into slot 1
  __device__ __forceinline__ void accumulate(double u, double w, double vm, float* are, float* aim) const {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double ph = fma(u, lj[t], fma(w, nj[t], vm));
      float cc, ss;
      cis_turns(ph, cc, ss);
      are[t & 1] = fmaf(xj[t], cc, are[t & 1]);
      aim[t & 1] = fmaf(-xj[t], ss, aim[t & 1]);
    }
  }
};

// part[c][l][k] = sum over the rows of band c of x_ij / n_ij exp(-2 pi i phase).  A workgroup is
// four waves on the same channel and band, each with 64 visibilities: the band's rows are staged
// once per workgroup in LDS (l_j for the whole image, then n_ij and x_ij / n_ij row by row, two
// row buffers), and every wave reads them as broadcasts.  The next row is fetched into registers
// while the current one is summed.
__global__ void __launch_bounds__(256) k_vis_fwd(const VisPt* __restrict__ vp, const float* __restrict__ XN,
                                                 const double* __restrict__ lt, const double* __restrict__ nt,
                                                 float2* __restrict__ part, int N, int K, int L, int G4, int C,
                                                 int R) {
  extern __shared__ double vsm[];  // [N] l, [2][N] n, then [2][N] floats x / n
  double* sl = vsm;
  double* sn = vsm + N;
  float* sx = (float*)(vsm + 3 * N);
  const int b = blockIdx.x;
  const int gq = b % G4, c = (b / G4) % C, l = b / (G4 * C);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = (gq * 4 + wv) * 64 + lane;
  const bool ok = k < K;
  const VisPt p = vp[(long long)l * K + MF_CHK(ok ? k : K - 1, K)];
  const double u = p.u, v = p.v, w = p.w;
  const int i0 = c * R, i1 = min(N, i0 + R);
  const long long np = (long long)N * N;
  const float* xplane = XN + (long long)l * np;
  constexpr int kPer = 4;  // pixels of a row per thread (N <= 1024)
  double nreg[kPer];
  float xreg[kPer];
  for (int j = threadIdx.x; j < N; j += 256) sl[MF_CHK(j, N)] = lt[j];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int j = threadIdx.x + 256 * q;
    if (j < N) {
      nreg[q] = nt[(long long)i0 * N + j];
      xreg[q] = xplane[(long long)i0 * N + j];
    }
  }
  float are[2] = {0.f, 0.f}, aim[2] = {0.f, 0.f};
  for (int i = i0; i < i1; ++i) {
    const int buf = (i - i0) & 1;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int j = threadIdx.x + 256 * q;
      if (j < N) {
        sn[buf * N + MF_CHK(j, N)] = nreg[q];
        sx[buf * N + MF_CHK(j, N)] = xreg[q];
      }
    }
    lds_barrier();  // row i staged (and, for the other buffer, row i - 1 no longer read)
    if (i + 1 < i1) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int j = threadIdx.x + 256 * q;
        if (j < N) {
          nreg[q] = nt[(long long)(i + 1) * N + j];
          xreg[q] = xplane[(long long)(i + 1) * N + j];
        }
      }
    }
    const double vm = v * lt[MF_CHK(i, N)];
    const double* nrow = sn + buf * N;
    const float* xrow = sx + buf * N;
    // two register sets of four pixels: one set is read from LDS while the other is summed
    // (N is a multiple of 8)
    PixQuad A, B;
    A.load(sl, nrow, xrow, 0, N);
    for (int j = 0; j < N; j += 8) {
      B.load(sl, nrow, xrow, j + 4, N);
      A.accumulate(u, w, vm, are, aim);
      A.load(sl, nrow, xrow, j + 8 < N ? j + 8 : j, N);
      B.accumulate(u, w, vm, are, aim);
    }
  }
  if (ok) part[((long long)c * L + l) * K + k] = make_float2(are[0] + are[1], aim[0] + aim[1]);
}

int launch_vis_fwd(const VisPt* vp, const float* XN, const double* lt, const double* nt, float2* part, int N, int K,
                   int L, int C, hipStream_t st) {
  if (N % 8 || N > 1024) return set_error("visibility kernels need N a multiple of 8, at most 1024"), MUFFIN_EINVAL;
  const int G4 = (K + 255) / 256;
  const int R = (N + C - 1) / C;
  if ((long long)(C - 1) * R >= N) return set_error("visibility forward: empty row band"), MUFFIN_EINVAL;
  const long long blocks = (long long)L * G4 * C;
  const size_t shm = sizeof(double) * 3 * N + sizeof(float) * 2 * N;
  hipLaunchKernelGGL(k_vis_fwd, dim3((unsigned)blocks), dim3(256), shm, st, vp, XN, lt, nt, part, N, K, L, G4, C, R);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// r = sum_c part[c] + vsign vis (vis may be NULL); vp receives w_l r (w_l = cw[l], or 1 when cw is
// NULL) and rout, when it is not NULL, r itself; partial[block] = 1/2 sum w_l |r|^2 in FP64 when
// partial is not NULL.  Grid-stride over the L K visibilities, so that the number of partial sums
// stays bounded.
__global__ void __launch_bounds__(256) k_vis_resid(const float2* __restrict__ part, int C, long long LK, int K,
                                                   const float2* __restrict__ vis, float vsign,
                                                   const float* __restrict__ cw, VisPt* __restrict__ vp,
                                                   double* __restrict__ partial, float2* __restrict__ rout) {
  __shared__ double red[256];
  double e = 0.0;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < LK; t += (long long)gridDim.x * 256) {
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
    const float wl = cw ? cw[t / K] : 1.f;
    vp[MF_CHK(t, LK)].rre = wl * re;
    vp[t].rim = wl * im;
    if (rout) rout[t] = make_float2(re, im);
    e += (double)wl * ((double)re * re + (double)im * im);
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

int launch_vis_resid(const float2* part, int C, int L, int K, const float2* vis, float vsign, const float* cw,
                     VisPt* vp, double* partial, int* nblocks, float2* rout, hipStream_t st) {
  const long long LK = (long long)L * K;
  long long nb = (LK + 255) / 256;
  if (nb > 16384) nb = 16384;
  hipLaunchKernelGGL(k_vis_resid, dim3((unsigned)nb), dim3(256), 0, st, part, C, LK, K, vis, vsign, cw, vp, partial,
                     rout);
  MF_HIP(hipGetLastError());
  if (nblocks) *nblocks = (int)nb;
  return MUFFIN_OK;
}

// out[l][p] = (1/n_p) Re sum_k r_k exp(+2 pi i phase_kp) (+ s_scale sadd[l][p]); four pixels of one
// row per lane.  The channel's visibilities pass through LDS in chunks of 256 (one 32-byte record
// per thread, two buffers, the next chunk fetched into registers while the current one is summed);
// every wave reads them as broadcasts.
constexpr int kVisChunk = 256;

__global__ void __launch_bounds__(256) k_vis_adj(const VisPt* __restrict__ vp, int K, const double* __restrict__ lt,
                                                 const double* __restrict__ nt, const float* __restrict__ invn,
                                                 int N, float* __restrict__ out, long long out_cs,
                                                 const float* __restrict__ sadd, long long s_cs, float s_scale) {
  // a record is moved as two float4 (the records are 32-byte aligned): a VisPt held in a variable
  // across the loop would be kept in scratch memory
  __shared__ float4 sv4[2][kVisChunk][2];
  const long long np = (long long)N * N;
  const long long l = blockIdx.y;
  const long long p0 = 4 * ((long long)blockIdx.x * 256 + threadIdx.x);
  const bool active = p0 < np;  // every thread takes part in the staging and the barriers
  const long long pc = active ? p0 : 0;
  const int i = (int)(pc / N), j0 = (int)(pc - (long long)i * N);
  const double m = lt[MF_CHK(i, N)];
  double lj[4], nj[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    lj[t] = lt[MF_CHK(j0 + t, N)];
    nj[t] = nt[MF_CHK(pc + t, np)];
  }
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const float4* vl = (const float4*)(vp + l * K);
  const int nchunks = (K + kVisChunk - 1) / kVisChunk;
  const int k1 = MF_CHK(min((int)threadIdx.x, K - 1), K);
  float4 pre0 = vl[2 * k1], pre1 = vl[2 * k1 + 1];
  sv4[0][threadIdx.x][0] = pre0;
  sv4[0][threadIdx.x][1] = pre1;
  // the pixel geometry is consumed here, so that its loads have landed before the chunk loop:
  // otherwise the loop's first use waits on every load in flight, the next chunk's included
#pragma unroll
  for (int t = 0; t < 4; ++t) asm volatile("" ::"v"(lj[t]), "v"(nj[t]));
  asm volatile("" ::"v"(m));
  lds_barrier();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int k0 = ch * kVisChunk, n = min(kVisChunk, K - k0);
    const bool more = ch + 1 < nchunks;
    if (more) {
      const int kn = MF_CHK(min(k0 + kVisChunk + (int)threadIdx.x, K - 1), K);
      pre0 = vl[2 * kn];
      pre1 = vl[2 * kn + 1];
    }
    const VisPt* cur = (const VisPt*)&sv4[ch & 1][0][0];
#pragma unroll 2
    for (int kk = 0; kk < n; ++kk) {
      const double vm = cur[kk].v * m;
      const double u = cur[kk].u, w = cur[kk].w;
      const float a = cur[kk].rre, b = cur[kk].rim;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double ph = fma(u, lj[t], fma(w, nj[t], vm));
        float cc, ss;
        cis_turns(ph, cc, ss);
        acc[t] = fmaf(a, cc, acc[t]);
        acc[t] = fmaf(-b, ss, acc[t]);
      }
    }
    if (more) {  // that buffer was last read before the previous barrier
      sv4[(ch + 1) & 1][threadIdx.x][0] = pre0;
      sv4[(ch + 1) & 1][threadIdx.x][1] = pre1;
    }
    lds_barrier();
  }
  if (!active) return;
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
