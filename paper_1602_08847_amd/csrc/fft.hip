// Real 2-D FFT convolution passes for the data term (Algorithm 1, eq. (grad)).
//
// A channel's gradient H^dagger H x is C2R(P . R2C(x)) with P = w |H(k)|^2 / N^2, computed in
// three passes over a column-blocked half spectrum ([ncb][N][CB] per channel, pitch = ncb CB):
//   1. rows:    two real rows packed as one complex row, one N-point complex FFT, then split;
//   2. columns: CB columns per workgroup, N-point forward FFT, pointwise multiply, inverse FFT;
//   3. rows:    Hermitian completion of two rows, inverse FFT, real/imaginary parts are the rows,
//               fused epilogue (gradient, plain store, or FP64 residual energy).
// The 1-D transforms are the LDS Stockham FFTs of fft_core.h.
#include "fft_core.h"

#include <cmath>

namespace mf {

// columns per block of the half spectrum (and per workgroup of the column pass)
template <int N>
constexpr int col_block() {
  constexpr int T = Plan<N>::T;
  constexpr int cb = 512 / T;
  return cb < 8 ? 8 : (cb > 32 ? 32 : cb);
}

// ------------------------------------------------------------------ pass 1: rows, real -> half spectrum
template <int N>
__global__ void __launch_bounds__(256) k_rows_r2c(const float* __restrict__ x, long long cs, float2* __restrict__ S,
                                                  int pitch, long long npairs, const float2* __restrict__ tw,
                                                  int shift) {
  constexpr int T = Plan<N>::T;
  constexpr int NI = N / T;  // entries of one transform per thread
  constexpr int FPB = (256 / T) > 0 ? (256 / T) : 1;
  constexpr int LS = lstride<N>();
  __shared__ float2 lds[FPB * LS];
  const int f = threadIdx.x / T, t = threadIdx.x % T;
  const long long pair = (long long)blockIdx.x * FPB + f;
  const bool active = (f < FPB) && (pair < npairs);
  float2* buf = lds + (f < FPB ? f : 0) * LS;
  long long ch = 0;
  int r0 = 0;
  if (active) {
    ch = pair / (N / 2);
    r0 = 2 * (int)(pair % (N / 2));
    const float* xc = x + ch * cs;
    int ra = r0, rb = r0 + 1;
    if (shift) {
      ra = (ra + N / 2) % N;
      rb = (rb + N / 2) % N;
    }
    const float* pa = xc + (long long)ra * N;
    const float* pb = xc + (long long)rb * N;
    // all N/T loads of the thread in flight at once, then into LDS; x is read once per pass
    // (streaming), while the half spectrum this pass writes stays cached for the next pass
    float va[NI], vb[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int c = shift ? (t + i * T + N / 2) % N : t + i * T;
      va[i] = ld_stream(pa + c);
      vb[i] = ld_stream(pb + c);
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) buf[lpad(t + i * T)] = make_float2(va[i], vb[i]);
  }
  lds_barrier();
  fft_lds<N, false>(buf, t, active, tw);
  if (active) {
    // blocked half spectrum: entry (row, col) at ((ch ncb + col / CB) N + row) CB + col % CB, so
    // the transform pair's rows r0, r0 + 1 are neighbours within every column block
    constexpr int CB = col_block<N>();
    float2* sblk = S + (ch * N) * (long long)pitch + (long long)r0 * CB;
    for (int k = t; k <= N / 2; k += T) {
      const float2 zk = buf[lpad(k)];
      const float2 zm = cconj(buf[lpad((N - k) % N)]);
      // A = (Z_k + conj Z_{N-k}) / 2,  B = (Z_k - conj Z_{N-k}) / (2i)
      const float2 a = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
      const float2 d = csub(zk, zm);
      const float2 bb = make_float2(0.5f * d.y, -0.5f * d.x);
      float2* e = sblk + (long long)(k / CB) * N * CB + k % CB;
      e[0] = a;
      e[CB] = bb;
    }
  }
}

// ------------------------------------------------------------------ pass 2: columns

template <int N, int MODE>
// two workgroups per CU: the register budget is capped at 128 for power-of-two sizes (their
// radix-16/8 plans fit without spills; the radix-3 plans would spill, so they keep the default)
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu((N & (N - 1)) == 0 ? 4 : 1))) k_cols(float2* __restrict__ S, int pitch, int ncb,
                                              const float2* __restrict__ tw, const float* __restrict__ Mr,
                                              const float2* __restrict__ Mc, float scale,
                                              float2* __restrict__ outT) {
  constexpr int T = Plan<N>::T;
  constexpr int CB = col_block<N>();
  constexpr int LS = lstride<N>();
  extern __shared__ float2 lds[];
  float2* twl = lds + CB * LS;  // [N] twiddle table, copied once so the stages read it from LDS
  for (int i = threadIdx.x; i < N; i += CB * T) twl[i] = tw[i];
  // consecutive column blocks of a channel run on one XCD
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int ch = blk / ncb;
  const int c0 = (blk % ncb) * CB;
  const int nthr = CB * T;
  constexpr int NI = N / T;  // entries per thread: N * CB / nthr
  // the block's CB columns are one contiguous [N][CB] run of the blocked half spectrum; entry i of
  // the thread is element threadIdx.x + i * nthr of it: row r0 + i * (nthr / CB), column cc
  constexpr int RSTEP = nthr / CB;
  const int r0 = threadIdx.x / CB, cc = threadIdx.x % CB;
  float2* Sb = S + (long long)ch * N * pitch + (long long)c0 * N;
  auto sent = [&](int i) -> float2* { return Sb + threadIdx.x + i * nthr; };
  {
    // all loads of the thread in flight at once, then into LDS
    float2 v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) v[i] = *sent(i);
#pragma unroll
    for (int i = 0; i < NI; ++i) lds[cc * LS + lpad(r0 + i * RSTEP)] = v[i];
  }
  const int f = threadIdx.x / T, t = threadIdx.x % T;
  const long long mrow = ((long long)ch * pitch + c0 + f) * N;  // transposed multiplier row
  // the multiplier: fetched after the forward transform, all of the thread's entries at once (held
  // across the transform it would cost an occupancy step)
  float mr[MODE == COL_REAL ? NI : 1];
  float2 mc[(MODE == COL_CPLX || MODE == COL_CPLX_CONJ) ? NI : 1];
  lds_barrier();
  float2* buf = lds + f * LS;
  fft_lds<N, false>(buf, t, true, twl);
  __builtin_amdgcn_sched_barrier(0);  // the multiplier loads stay after the transform
  if constexpr (MODE == COL_REAL) {
    const float* __restrict__ mp = Mr + mrow + t;
#pragma unroll
    for (int i = 0; i < NI; ++i) mr[i] = ld_stream(mp + i * T);  // constant, read once per pass
  }
  if constexpr (MODE == COL_CPLX || MODE == COL_CPLX_CONJ) {
    const float2* __restrict__ mp = Mc + mrow + t;
#pragma unroll
    for (int i = 0; i < NI; ++i) mc[i] = mp[i * T];
  }
  if constexpr (MODE == COL_FWD) {
#pragma unroll
    for (int i = 0; i < NI; ++i) outT[mrow + t + i * T] = buf[lpad(t + i * T)];
    return;
  } else {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int r = t + i * T;
      float2 v = buf[lpad(r)];
      if constexpr (MODE == COL_REAL) {
        v = cscale(v, mr[i] * scale);
      } else {
        float2 m = mc[i];
        if (MODE == COL_CPLX_CONJ) m.y = -m.y;
        v = cscale(cmul(v, m), scale);
      }
      buf[lpad(r)] = v;
    }
    // fft_lds begins with reads of this thread group's own entries only after a barrier
    lds_barrier();
    fft_lds<N, true>(buf, t, true, twl);
#pragma unroll
    for (int i = 0; i < NI; ++i) *sent(i) = lds[cc * LS + lpad(r0 + i * RSTEP)];
  }
}

// ------------------------------------------------------------------ pass 3: rows, half spectrum -> real
__device__ __forceinline__ double block_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  lds_barrier();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
  }
  return s;
}

template <int N, int EPI>
__global__ void __launch_bounds__(256) k_rows_c2r(const float2* __restrict__ S, int pitch, long long npairs,
                                                  const float2* __restrict__ tw, float* __restrict__ out,
                                                  long long cs, const float* __restrict__ b, const float* __restrict__ s,
                                                  float s_scale, const float* __restrict__ y,
                                                  const float* __restrict__ chan_w, double* __restrict__ partial,
                                                  PrimalEpi pe) {
  constexpr int T = Plan<N>::T;
  constexpr int NI = N / T;  // entries of one transform per thread
  constexpr int FPB = (256 / T) > 0 ? (256 / T) : 1;
  constexpr int LS = lstride<N>();
  __shared__ float2 lds[FPB * LS];
  const int f = threadIdx.x / T, t = threadIdx.x % T;
  const long long pair = (long long)blockIdx.x * FPB + f;
  const bool active = (f < FPB) && (pair < npairs);
  float2* buf = lds + (f < FPB ? f : 0) * LS;
  long long ch = 0;
  int r0 = 0;
  long long o0 = 0, o1 = 0;
  // epilogue operands of the thread's outputs, fetched after the transform, all at once
  constexpr int NE = (EPI == EPI_STORE) ? 1 : NI;
  constexpr int NX = (EPI == EPI_PRIMAL) ? NI : 1;
  float e0[NE], e1[NE], s0[NE], s1[NE], x0[NX], x1[NX];
  if (active) {
    ch = pair / (N / 2);
    r0 = 2 * (int)(pair % (N / 2));
    o0 = ch * cs + (long long)r0 * N;
    o1 = o0 + N;
    constexpr int CB = col_block<N>();
    const float2* sblk = S + (ch * N) * (long long)pitch + (long long)r0 * CB;  // blocked layout
    // entries above N/2 are the conjugates of stored ones (Hermitian symmetry of real rows)
    float2 va[NI], vb[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int k = t + i * T;
      const int ks = k <= N / 2 ? k : N - k;
      const float2* e = sblk + (long long)(ks / CB) * N * CB + ks % CB;
      va[i] = e[0];
      vb[i] = e[CB];
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int k = t + i * T;
      float2 a = va[i], bb = vb[i];
      if (k == 0 || k == N / 2) {
        a.y = 0.f;
        bb.y = 0.f;
      } else if (k > N / 2) {
        a = cconj(a);
        bb = cconj(bb);
      }
      // Z = A + i B
      buf[lpad(k)] = make_float2(a.x - bb.y, a.y + bb.x);
    }
  }
  lds_barrier();
  fft_lds<N, true>(buf, t, active, tw);
  __builtin_amdgcn_sched_barrier(0);  // the epilogue loads stay after the transform
  double acc = 0.0;
  if (active) {
    if constexpr (EPI != EPI_STORE) {
      const float* __restrict__ ep = ((EPI == EPI_GRAD || EPI == EPI_PRIMAL) ? b : y) + o0 + t;
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        e0[i] = ld_stream(ep + i * T);  // b or y, and below the adjoint term: read once (streaming)
        e1[i] = ld_stream(ep + N + i * T);
      }
      if ((EPI == EPI_GRAD || EPI == EPI_PRIMAL) && s) {
        const float* __restrict__ sp = s + o0 + t;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          s0[i] = ld_stream(sp + i * T);
          s1[i] = ld_stream(sp + N + i * T);
        }
      }
      if constexpr (EPI == EPI_PRIMAL) {
        const float* __restrict__ xp = out + o0 + t;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          x0[i] = ld_stream(xp + i * T);
          x1[i] = ld_stream(xp + N + i * T);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int n = t + i * T;
      const float2 z = buf[lpad(n)];
      if constexpr (EPI == EPI_STORE) {
        out[o0 + n] = z.x;
        out[o1 + n] = z.y;
      } else if constexpr (EPI == EPI_GRAD) {
        float g0 = z.x - e0[i], g1 = z.y - e1[i];
        if (s) {
          g0 += s_scale * s0[i];
          g1 += s_scale * s1[i];
        }
        out[o0 + n] = g0;
        out[o1 + n] = g1;
      } else if constexpr (EPI == EPI_PRIMAL) {
        // q as in EPI_GRAD, then the primal step of the spectral kernel with its term t = 0
        float q0 = z.x - e0[i], q1 = z.y - e1[i];
        if (s) {
          q0 += s_scale * s0[i];
          q1 += s_scale * s1[i];
        }
        const float tau = pe.tau_ch[ch];
        const float xa = x0[i], xb = x1[i];
        const float ta = fmaxf(xa - tau * q0, 0.f), tb = fmaxf(xb - tau * q1, 0.f);
        st_stream(pe.D + o0 + n, 2.f * ta - xa);
        st_stream(pe.D + o1 + n, 2.f * tb - xb);
        st_stream(out + o0 + n, pe.rho * ta + (1.f - pe.rho) * xa);
        st_stream(out + o1 + n, pe.rho * tb + (1.f - pe.rho) * xb);
      } else {
        const double r0d = (double)z.x - (double)e0[i];
        const double r1d = (double)z.y - (double)e1[i];
        acc += r0d * r0d + r1d * r1d;
      }
    }
    if constexpr (EPI == EPI_RESID) acc *= 0.5 * (chan_w ? (double)chan_w[ch] : 1.0);
  }
  if constexpr (EPI == EPI_RESID) {
    const double tot = block_sum_d(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
  }
}

// ------------------------------------------------------------------ host side
bool fft_supported(int N) {
  switch (N) {
    case 8: case 16: case 32: case 64: case 128: case 256: case 512: case 1024:
    case 12: case 24: case 48: case 96: case 192: case 384: case 768:
      return true;
    default:
      return false;
  }
}

template <int N>
static FftGeom geom_of() {
  FftGeom g;
  g.N = N;
  g.CB = col_block<N>();
  g.ncb = (N / 2 + 1 + g.CB - 1) / g.CB;
  g.pitch = g.ncb * g.CB;
  return g;
}

FftGeom fft_geom(int N) {
  switch (N) {
#define MF_G(n) case n: return geom_of<n>();
    MF_G(8) MF_G(16) MF_G(32) MF_G(64) MF_G(128) MF_G(256) MF_G(512) MF_G(1024)
    MF_G(12) MF_G(24) MF_G(48) MF_G(96) MF_G(192) MF_G(384) MF_G(768)
#undef MF_G
    default: return FftGeom{};
  }
}

std::vector<float2> fft_twiddles(int N) {
  std::vector<float2> tw(N);
  for (int m = 0; m < N; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)N;
    tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return tw;
}

template <int N>
static int rows_r2c_n(const float* x, long long cs, float2* S, int nch, const FftGeom& g, const float2* tw, bool shift,
                      hipStream_t st) {
  constexpr int T = Plan<N>::T;
  constexpr int FPB = (256 / T) > 0 ? (256 / T) : 1;
  const long long npairs = (long long)nch * (N / 2);
  const long long nblk = (npairs + FPB - 1) / FPB;
  hipLaunchKernelGGL(k_rows_r2c<N>, dim3((unsigned)nblk), dim3(FPB * T), 0, st, x, cs, S, g.pitch, npairs, tw,
                     shift ? 1 : 0);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

template <int N>
static int cols_n(float2* S, int nch, const FftGeom& g, const float2* tw, int mode, const float* Mr,
                  const float2* Mc, float scale, float2* outT, hipStream_t st) {
  constexpr int T = Plan<N>::T;
  constexpr int CB = col_block<N>();
  constexpr int LS = lstride<N>();
  const size_t shm = sizeof(float2) * (CB * LS + N);  // columns, then the twiddle table
  const dim3 grid((unsigned)(nch * g.ncb)), block(CB * T);
  switch (mode) {
    case COL_FWD:
      hipLaunchKernelGGL((k_cols<N, COL_FWD>), grid, block, shm, st, S, g.pitch, g.ncb, tw, Mr, Mc, scale, outT);
      break;
    case COL_REAL:
      hipLaunchKernelGGL((k_cols<N, COL_REAL>), grid, block, shm, st, S, g.pitch, g.ncb, tw, Mr, Mc, scale, outT);
      break;
    case COL_CPLX:
      hipLaunchKernelGGL((k_cols<N, COL_CPLX>), grid, block, shm, st, S, g.pitch, g.ncb, tw, Mr, Mc, scale, outT);
      break;
    case COL_CPLX_CONJ:
      hipLaunchKernelGGL((k_cols<N, COL_CPLX_CONJ>), grid, block, shm, st, S, g.pitch, g.ncb, tw, Mr, Mc, scale,
                         outT);
      break;
    default:
      set_error("launch_cols: bad mode");
      return MUFFIN_EINVAL;
  }
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

template <int N>
static int rows_c2r_n(const float2* S, int nch, const FftGeom& g, const float2* tw, int epi, float* out,
                      long long cs, const float* b, const float* s, float s_scale, const float* y, const float* chan_w,
                      double* partial, int* nblocks_out, hipStream_t st, const PrimalEpi& pe) {
  constexpr int T = Plan<N>::T;
  constexpr int FPB = (256 / T) > 0 ? (256 / T) : 1;
  const long long npairs = (long long)nch * (N / 2);
  const long long nblk = (npairs + FPB - 1) / FPB;
  if (nblocks_out) *nblocks_out = (int)nblk;
  if (epi == EPI_RESID && nblk > kMaxPartials) {
    set_error("rows_c2r: too many blocks for the partial-sum buffer");
    return MUFFIN_EINVAL;
  }
  const dim3 grid((unsigned)nblk), block(FPB * T);
  switch (epi) {
    case EPI_STORE:
      hipLaunchKernelGGL((k_rows_c2r<N, EPI_STORE>), grid, block, 0, st, S, g.pitch, npairs, tw, out, cs, b, s, s_scale,
                         y, chan_w, partial, pe);
      break;
    case EPI_GRAD:
      hipLaunchKernelGGL((k_rows_c2r<N, EPI_GRAD>), grid, block, 0, st, S, g.pitch, npairs, tw, out, cs, b, s, s_scale,
                         y, chan_w, partial, pe);
      break;
    case EPI_RESID:
      hipLaunchKernelGGL((k_rows_c2r<N, EPI_RESID>), grid, block, 0, st, S, g.pitch, npairs, tw, out, cs, b, s, s_scale,
                         y, chan_w, partial, pe);
      break;
    case EPI_PRIMAL:
      if (!pe.D || !pe.tau_ch) return set_error("rows_c2r: primal epilogue needs D and tau"), MUFFIN_EINVAL;
      hipLaunchKernelGGL((k_rows_c2r<N, EPI_PRIMAL>), grid, block, 0, st, S, g.pitch, npairs, tw, out, cs, b, s,
                         s_scale, y, chan_w, partial, pe);
      break;
    default:
      set_error("rows_c2r: bad epilogue");
      return MUFFIN_EINVAL;
  }
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

#define MF_DISPATCH(N, call) \
  switch (N) {               \
    case 8: return call<8>;  \
    case 16: return call<16>; \
    case 32: return call<32>; \
    case 64: return call<64>; \
    case 128: return call<128>; \
    case 256: return call<256>; \
    case 512: return call<512>; \
    case 1024: return call<1024>; \
    case 12: return call<12>; \
    case 24: return call<24>; \
    case 48: return call<48>; \
    case 96: return call<96>; \
    case 192: return call<192>; \
    case 384: return call<384>; \
    case 768: return call<768>; \
    default: set_error("unsupported FFT size"); return MUFFIN_EINVAL; \
  }

int launch_rows_r2c(const float* x, long long cs, float2* S, int nch, const FftGeom& g, const float2* tw,
                    bool shift, hipStream_t st) {
  if (cs < (long long)g.N * g.N) return set_error("rows_r2c: channel stride below N*N"), MUFFIN_EINVAL;
#define CALL(n) rows_r2c_n<n>(x, cs, S, nch, g, tw, shift, st)
  switch (g.N) {
    case 8: return CALL(8);
    case 16: return CALL(16);
    case 32: return CALL(32);
    case 64: return CALL(64);
    case 128: return CALL(128);
    case 256: return CALL(256);
    case 512: return CALL(512);
    case 1024: return CALL(1024);
    case 12: return CALL(12);
    case 24: return CALL(24);
    case 48: return CALL(48);
    case 96: return CALL(96);
    case 192: return CALL(192);
    case 384: return CALL(384);
    case 768: return CALL(768);
    default: set_error("unsupported FFT size"); return MUFFIN_EINVAL;
  }
#undef CALL
}

int launch_cols(float2* S, int nch, const FftGeom& g, const float2* tw, int mode, const float* Mr,
                const float2* Mc, float scale, float2* outT, hipStream_t st) {
#define CALL(n) cols_n<n>(S, nch, g, tw, mode, Mr, Mc, scale, outT, st)
  switch (g.N) {
    case 8: return CALL(8);
    case 16: return CALL(16);
    case 32: return CALL(32);
    case 64: return CALL(64);
    case 128: return CALL(128);
    case 256: return CALL(256);
    case 512: return CALL(512);
    case 1024: return CALL(1024);
    case 12: return CALL(12);
    case 24: return CALL(24);
    case 48: return CALL(48);
    case 96: return CALL(96);
    case 192: return CALL(192);
    case 384: return CALL(384);
    case 768: return CALL(768);
    default: set_error("unsupported FFT size"); return MUFFIN_EINVAL;
  }
#undef CALL
}

int launch_rows_c2r(const float2* S, int nch, const FftGeom& g, const float2* tw, int epi, float* out,
                    long long cs, const float* b, const float* s, float s_scale, const float* y,
                    const float* chan_w, double* partial, int* nblocks_out, hipStream_t st, const PrimalEpi& pe) {
  if (cs < (long long)g.N * g.N) return set_error("rows_c2r: channel stride below N*N"), MUFFIN_EINVAL;
#define CALL(n) rows_c2r_n<n>(S, nch, g, tw, epi, out, cs, b, s, s_scale, y, chan_w, partial, nblocks_out, st, pe)
  switch (g.N) {
    case 8: return CALL(8);
    case 16: return CALL(16);
    case 32: return CALL(32);
    case 64: return CALL(64);
    case 128: return CALL(128);
    case 256: return CALL(256);
    case 512: return CALL(512);
    case 1024: return CALL(1024);
    case 12: return CALL(12);
    case 24: return CALL(24);
    case 48: return CALL(48);
    case 96: return CALL(96);
    case 192: return CALL(192);
    case 384: return CALL(384);
    case 768: return CALL(768);
    default: set_error("unsupported FFT size"); return MUFFIN_EINVAL;
  }
#undef CALL
}
#undef MF_DISPATCH

template <int N>
static int attrs_n() {
  constexpr int shm = (int)(sizeof(float2) * (col_block<N>() * lstride<N>() + N));
  MF_HIP(hipFuncSetAttribute((const void*)k_cols<N, COL_FWD>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_cols<N, COL_REAL>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_cols<N, COL_CPLX>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  MF_HIP(hipFuncSetAttribute((const void*)k_cols<N, COL_CPLX_CONJ>, hipFuncAttributeMaxDynamicSharedMemorySize, shm));
  return MUFFIN_OK;
}

int fft_init_attrs(int N) {
  switch (N) {
    case 8: return attrs_n<8>();
    case 16: return attrs_n<16>();
    case 32: return attrs_n<32>();
    case 64: return attrs_n<64>();
    case 128: return attrs_n<128>();
    case 256: return attrs_n<256>();
    case 512: return attrs_n<512>();
    case 1024: return attrs_n<1024>();
    case 12: return attrs_n<12>();
    case 24: return attrs_n<24>();
    case 48: return attrs_n<48>();
    case 96: return attrs_n<96>();
    case 192: return attrs_n<192>();
    case 384: return attrs_n<384>();
    case 768: return attrs_n<768>();
    default: set_error("unsupported FFT size"); return MUFFIN_EINVAL;
  }
}

// P = w_l |H|^2 * scale on the transposed half spectrum.
__global__ void __launch_bounds__(256) k_power_spectrum(const float2* __restrict__ H, float* __restrict__ P,
                                                        const float* __restrict__ w, long long per_ch, float scale) {
  const int ch = blockIdx.y;
  const float s = scale * (w ? w[ch] : 1.f);
  const long long o = (long long)ch * per_ch;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < per_ch; i += (long long)gridDim.x * 256) {
    const float2 h = H[o + i];
    P[o + i] = s * (h.x * h.x + h.y * h.y);
  }
}

int launch_power_spectrum(const float2* Hhat_T, float* P_T, const float* chan_w, long long per_ch, int nch,
                          float scale, hipStream_t st) {
  long long nb = (per_ch + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_power_spectrum, dim3((unsigned)nb, (unsigned)nch), dim3(256), 0, st, Hhat_T, P_T, chan_w,
                     per_ch, scale);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

#ifdef MF_CHECKED
int oob_take_fft(unsigned long long* n) { return oob_take_here(n); }
#endif

}  // namespace mf
