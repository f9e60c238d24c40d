// Internal declarations shared by the HIP translation units of libmuffin.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "muffin.h"

namespace mf {

void set_error(const std::string& msg);

#define MF_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::mf::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return MUFFIN_EHIP;                                                         \
    }                                                                             \
  } while (0)

#define MF_TRY(expr)             \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != MUFFIN_OK) return rc_; \
  } while (0)

// Workgroup barrier ordering LDS only: unlike __syncthreads() it does not wait for this wave's
// outstanding global loads and stores, so prefetched rows stay in flight across it.  Use it only
// where the data exchanged through the barrier lives in LDS.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------------ checked build
// Built with -DMF_CHECKED (build.build_checked), MF_CHK(i, n) counts an index i outside [0, n) in
// this translation unit's device counter and yields 0 in its place, so the access stays in bounds
// and the kernel runs on; in the normal build it is i itself.  muffin_debug_oob sums and clears the
// counters of every translation unit.
#ifdef MF_CHECKED
static __device__ unsigned long long mf_oob_count;  // one per translation unit
__device__ __forceinline__ long long mf_chk(long long i, long long n) {
  if (i < 0 || i >= n) {
    atomicAdd(&mf_oob_count, 1ull);
    return 0;
  }
  return i;
}
#define MF_CHK(i, n) (static_cast<decltype(i)>(::mf::mf_chk((long long)(i), (long long)(n))))
// This translation unit's count since the last call, then zero.
static inline int oob_take_here(unsigned long long* n) {
  MF_HIP(hipMemcpyFromSymbol(n, HIP_SYMBOL(mf_oob_count), sizeof(*n)));
  const unsigned long long zero = 0;
  MF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(mf_oob_count), &zero, sizeof(zero)));
  return MUFFIN_OK;
}
#else
#define MF_CHK(i, n) (i)
#endif
// Per translation unit (checked build): its count since the last call, then zero.
int oob_take_fft(unsigned long long* n);
int oob_take_iuwt(unsigned long long* n);
int oob_take_spectral(unsigned long long* n);
int oob_take_uob(unsigned long long* n);
int oob_take_vis(unsigned long long* n);

// XCD-aware block order.  Consecutive workgroup ids are dealt round-robin to the 8 XCDs, each
// with its own L2; this maps id b to logical block xcd_remap(b) so that XCD x (ids b = x, x + 8,
// ...) walks one contiguous range of logical blocks, and neighbouring blocks that share cache
// lines or halo rows meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int x = b & 7, i = b >> 3;
  return x * per + (x < rem ? x : rem) + i;
}

// Streaming (nontemporal) global accesses: the line is marked for early eviction instead of being
// kept in L2 and the Infinity Cache.  They pay where the data is not read again soon (a plane the
// next launch does not touch) and cost where it is: a kernel that re-reads its own halo rows, or a
// launch whose output the very next launch reads, loses the cache hits.  Which kernels use them is
// decided by measurement, kernel by kernel.
__device__ __forceinline__ float ld_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }

// ------------------------------------------------------------------ complex helpers
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// ------------------------------------------------------------------ FFT geometry
// Column blocking of the half spectrum: the N/2+1 columns in ncb blocks of CB, pitch = ncb * CB.
struct FftGeom {
  int N = 0;
  int CB = 8;       // columns per block in the column pass
  int ncb = 0;      // column blocks
  int pitch = 0;    // columns over all blocks (>= N/2 + 1); a channel holds N * pitch entries
};
bool fft_supported(int N);
FftGeom fft_geom(int N);
// Twiddle table exp(-2 pi i m / N), m = 0..N-1, built in FP64 on the host.
std::vector<float2> fft_twiddles(int N);

// Row pass, real -> half spectrum.  x: nch planes of N x N, channel stride cs floats (>= N*N);
// S: column-blocked [nch][ncb][N][CB] (entry (row, col) of a channel at
// ((col / CB) N + row) CB + col % CB).  With shift, the input is read with an (N/2, N/2) circular
// shift (ifftshift of a centred PSF).
int launch_rows_r2c(const float* x, long long cs, float2* S, int nch, const FftGeom& g, const float2* tw,
                    bool shift, hipStream_t st);

enum ColMode { COL_FWD = 0, COL_REAL = 1, COL_CPLX = 2, COL_CPLX_CONJ = 3 };
// Column pass over the half spectrum: forward FFT along rows, then (mode != COL_FWD) multiply by
// M (real [nch][pitch][N] or complex [nch][pitch][N], transposed) times scale, then inverse FFT.
// For COL_FWD the forward result is written transposed to outT ([nch][pitch][N]) instead of S.
int launch_cols(float2* S, int nch, const FftGeom& g, const float2* tw, int mode, const float* Mr,
                const float2* Mc, float scale, float2* outT, hipStream_t st);

enum RowEpi { EPI_STORE = 0, EPI_GRAD = 1, EPI_RESID = 2, EPI_PRIMAL = 3 };
// Operands of the primal epilogue: the relaxed primal step of one channel when the spectral weight
// is zero (the spectral term t vanishes, so the step needs no other channel).
struct PrimalEpi {
  float* D = nullptr;             // d = 2 x~ - x, channel stride cs
  const float* tau_ch = nullptr;  // [nch] primal step of each channel's cube
  float rho = 1.f;
};
// Row pass, half spectrum -> real, with an epilogue per pixel (g = inverse transform); out, b, s
// and y are nch planes of N x N with channel stride cs floats:
//   EPI_STORE : out = g
//   EPI_GRAD  : out = g - b + s_scale * s      (s may be NULL)
//   EPI_RESID : partial[block] = sum over the block of 0.5 * w_l * (g - y)^2   (FP64)
//   EPI_PRIMAL: q = g - b + s_scale * s, x~ = (x - tau q)_+ with x = out; D = 2 x~ - x and
//               out = rho x~ + (1 - rho) x (the primal step and relaxation at mu_lambda = 0)
int launch_rows_c2r(const float2* S, int nch, const FftGeom& g, const float2* tw, int epi,
                    float* out, long long cs, const float* b, const float* s, float s_scale, const float* y,
                    const float* chan_w, double* partial, int* nblocks_out, hipStream_t st,
                    const PrimalEpi& pe = PrimalEpi{});

// ------------------------------------------------------------------ IUWT (a trous)
// Pointer + channel stride (in floats) of one plane per channel.
struct PlaneRef {
  const float* p = nullptr;
  long long cs = 0;
};
struct PlaneOut {
  float* p = nullptr;
  long long cs = 0;
};
enum AtrousMode {
  SM_SMOOTH = 0,      // out = H_j(A)
  SM_SUBADD = 1,      // out = E + H_j(A - B)
  SM_DETAIL = 2,      // w = E - H_j(A);  u(out) <- rho*sat(u + coef*w) + (1-rho)*u
  SM_DETAIL_ABS = 3,  // partial[block] = sum |E - H_j(A)|
  SM_DETAIL1 = 4,     // out2 = H_j(A); w = A - H_j(A); u(out) update  (first generation)
  DB_ANALYSIS = 5,    // out2 = c' = H_j(A); w = A - H_j(c'); u(out) update  (second generation)
  DB_ADJOINT = 6,     // out = A + H_j(B - H_j(A))  (A = u_j, B = a; second generation Horner step)
  DB_ANALYSIS_C = 7,  // DB_ANALYSIS at the last scale with the coarse plane's dual update fused:
                      // u2(out2) <- rho*sat(u2 + coef2*c') + (1-rho)*u2 instead of storing c'
  // two consecutive scales j, j+1 in one pass (second generation):
  PR_ANALYSIS = 8,    // A = c_j; out = u_j, out2 = u_{j+1} (dual updates); out3 = c_{j+2} = H_{j+1} H_j c_j
  PR_ANALYSIS_C = 9,  // PR_ANALYSIS with c_{j+2} feeding the coarse plane's dual update (out3, coef2)
  PR_ADJOINT = 10,    // A = u_{j+1}, B = u_j, E = a: out = two Horner steps, scale j+1 then j
  // three consecutive scales j, j+1, j+2 in one pass (second generation):
  TR_ANALYSIS = 11,   // A = c_j; out, out2, out3 = u_j, u_{j+1}, u_{j+2} (dual updates); out4 = c_{j+3}
  TR_ANALYSIS_C = 12, // TR_ANALYSIS with c_{j+3} feeding the coarse plane's dual update (out4, coef2)
  TR_ADJOINT = 13,    // A = u_{j+2}, B = u_{j+1}, E = u_j, F = a: out = Horner steps j+2, j+1, j
  // the last analysis pair (scales j, j+1, coarse plane) fused with the next iteration's first
  // adjoint pair over the planes it has just updated:
  PR_FUSED = 14,      // A = c_j; B, E, F = old u_j, u_{j+1}, coarse; out, out2, out3 = new ones;
                      // out4 = two Horner steps (scale j+1 then j) starting from the new coarse plane
  // two consecutive scales j, j+1 in one pass (first generation):
  P1_ANALYSIS = 15,   // A = c_j; out = u_j, out2 = u_{j+1} (dual updates, w = c - H c); out3 = c_{j+2}
  P1_ANALYSIS_C = 16, // P1_ANALYSIS with c_{j+2} feeding the coarse plane's dual update (out3, coef2)
  P1_ADJOINT = 17     // A = u_{j+1}, B = u_j, E = a: out = u_j + H_j(a' - u_j), a' = u_{j+1} + H_{j+1}(a - u_{j+1})
};
// launch of a pair kernel: j is the finer scale of the pair
int launch_pair(int mode, int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneOut out, PlaneOut out2,
                PlaneOut out3, float coef, float rho, float coef2, hipStream_t st, int trial = 0);
// launch of the fused pair (PR_FUSED): j is the finer scale of the pair
int launch_fused_pair(int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneRef F, PlaneOut out,
                      PlaneOut out2, PlaneOut out3, PlaneOut out4, float coef, float rho, float coef2,
                      hipStream_t st, int trial = 0);
// launch of a triple kernel: j is the finest of its three scales
int launch_triple(int mode, int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneRef F, PlaneOut out,
                  PlaneOut out2, PlaneOut out3, PlaneOut out4, float coef, float rho, float coef2, hipStream_t st,
                  int trial = 0);
// band height (rows per workgroup) of the band kernels, default or autotuned; set_band_rows records
// an autotuned choice for (N, j, kernel class of mode)
int atrous_band_rows(int N, int j, int mode);
// The band height a launch over nch channels uses: the tuned one, else the default made small
// enough for the launch to fill the GPU.
int atrous_band_rows(int N, int j, int mode, int nch);
int atrous_set_band_rows(int N, int j, int mode, int TY);
// residue-class groups per band of the pair kernels (each group its own workgroup) for a launch
// over nch channels: the tuned value with the tuned band rows, else the default with the default rows
int atrous_class_groups(int N, int j, int mode, int nch);
int atrous_set_class_groups(int N, int j, int mode, int ncg);
// band rows (0: default) and class groups (0 or 1: none) of one kernel class at once
int atrous_set_tiles(int N, int j, int cls, int TY, int ncg);
int atrous_class(int mode);
// true if the double-smoothing kernels fit in LDS at scale j for image side N
bool atrous_double_fits(int N, int j, int* TX, int* TY);
int launch_atrous(int mode, int N, int nch, int j, PlaneRef A, PlaneRef B, PlaneRef E, PlaneOut out,
                  PlaneOut out2, float coef, float rho, double* partial, int* nblocks_out, hipStream_t st,
                  int trial = 0,  // trial: the autotuner's timing launch (same code, own symbol)
                  float coef2 = 0.f);  // DB_ANALYSIS_C: the coarse plane's dual step sigma*mu_s*omega
enum PointMode {
  PT_DETAIL1 = 0,  // w = E - A; u update (first-generation detail, no smoothing)
  PT_COARSE = 1,   // w = A; u update
  PT_ABS_DIFF = 2, // partial = sum |E - A|
  PT_ABS = 3,      // partial = sum |A|
  PT_COPY = 4,     // out = coef * A
  PT_SUB = 5       // out = E - A
};
int launch_pointwise(int mode, int N, int nch, PlaneRef A, PlaneRef E, PlaneOut out, float coef,
                     float rho, double* partial, int* nblocks_out, hipStream_t st);

// ------------------------------------------------------------------ spectral (per pixel)
struct SpectralArgs {
  float* X;
  const float* Q;
  float* V;
  float* D;
  const float* W;   // [L][L] W[l][k] = s_k cos(pi (2l+1) k / 2L)
  const float* WT;  // [L][L] transpose
  const float2* twL;  // FFT twiddles exp(-2 pi i m / L)
  const float2* csL;  // exp(i pi k / 2L)
  long long npix;     // N*N
  long long cs;       // floats between the channel planes of X, Q, V and D (>= npix)
  int L;
  int use_fft;        // 1: FFT-based cosine transforms (L has an FFT plan), 0: cosine table
  float tau, mu_l, smu_l, rho;
  const float2* blu = nullptr;  // Bluestein table of L (spectral_blu_table), or null: cosine table
};
bool spectral_has_fft(int L);
// Bluestein length M (the shortest FFT plan of even thread count with M >= 2L - 1) for L without
// an FFT plan, kBluMinL <= L <= 512; else 0.
constexpr int kBluMinL = 16;
int spectral_blu_m(int L);
// Whether the spectral step of L channels takes the Bluestein form by default (else cosine tables).
bool spectral_blu_default(int L);
// exp(-2 pi i m / M) (m < M), FFT_M of the chirp conj(c_j), and c_n = exp(-i pi n^2 / L) (n < L).
std::vector<float2> spectral_blu_table(int L);
int launch_spectral_step(const SpectralArgs& a, hipStream_t st);
// out = X W_lambda (inverse = false) or X W_lambda^dagger (inverse = true), per pixel; in and out
// hold L planes of npix pixels with channel stride cs floats.
int launch_dct(const float* in, float* out, const float* Wmat, long long npix, long long cs, int L,
               hipStream_t st);
// partial[block] = sum |X W_lambda| over the block's pixels.
int launch_dct_abs(const float* in, const float* WT, long long npix, long long cs, int L, double* partial,
                   int* nblocks_out, hipStream_t st);

// ------------------------------------------------------------------ union of wavelet bases
// The spatial prior as a union of the first kUobBases orthonormal Daubechies bases (scaled by
// 1/sqrt(kUobBases)), each a J-level periodic 2-D DWT in pyramid layout; see uob.hip.
constexpr int kUobBases = 8;
struct UobFilters {
  float h[kUobBases][2 * kUobBases];  // scaling filters (basis b has 2 (b + 1) taps)
  float g[kUobBases][2 * kUobBases];  // wavelet filters g_k = (-1)^k h_{F-1-k}
  int len[kUobBases];
};
UobFilters uob_filters();
// Daubechies scaling filter with n vanishing moments (2n taps) in FP64, from the library's own
// construction (for host-side checks)
int uob_lowpass(int n, double* h, int len);
enum UobMode { UOB_DUAL = 0, UOB_STORE = 1, UOB_ABS = 2 };
// One level of the analysis (input side n -> four m x m subbands, m = n / 2) or of the adjoint
// (coefficient side m -> output side n), over nch channels.
struct UobLevelArgs {
  UobFilters f;
  const float* in = nullptr;  // analysis: level input (d, or the previous approximation); adjoint: approximation
  long long in_cs = 0, in_bs = 0;  // channel and basis strides of in (in_bs = 0: one input for all bases)
  int in_ld = 0;                   // row stride of in
  int n = 0;                       // analysis: input side; adjoint: output side
  int N = 0;                       // side (and row stride) of the dual planes and of out
  int shared_input = 0;            // analysis: one input tile for all bases (level 1)
  int last = 0;                    // analysis: the coarsest level (its approximation is a coefficient too)
  int all_bases = -1;              // after level 1: one block runs every basis (1), one per basis (0), by size (-1)
  float* U = nullptr;              // dual planes [channel][basis][N][N]
  long long u_cs = 0, u_bs = 0;
  float* llout = nullptr;          // next approximation of each (channel, basis), dense rows
  long long ll_cs = 0, ll_bs = 0;
  float* out = nullptr;            // UOB_STORE: coefficients (strides out_cs, out_bs); adjoint: the image
  long long out_cs = 0, out_bs = 0;
  float coef = 0.f, rho = 1.f, scale = 1.f;
  double* partial = nullptr;
};
int launch_uob_an(int mode, const UobLevelArgs& a, int nch, double* partial, int* nblocks_out, hipStream_t st);
int launch_uob_adj(bool accum, const UobLevelArgs& a, int nch, hipStream_t st);

// ------------------------------------------------------------------ reductions (FP64)
// dst[slot] (+)= sum(partial[0..n)) in a fixed order.
int launch_reduce_sum(const double* partial, int n, double* dst, int accumulate, hipStream_t st);
// dst = max over a float array (times scale) in FP64.
int launch_reduce_max(const float* x, long long n, double scale, double* partial, double* dst,
                      hipStream_t st);
// dst = max over the N x N frequency grid of sum_k omega_k |g_k|^2 (IUWT frame symbol).
int launch_frame_bound(int N, int J, int gen, double omega_coarse, double* partial, double* dst,
                       hipStream_t st);
// Scan for non-finite values; dst[0] += count (as double).
int launch_count_nonfinite(const float* x, long long n, double* partial, double* dst,
                           hipStream_t st);
// Over nplanes planes of npix floats (plane k of a at a + k acs, of b at b + k bcs; b may be NULL
// for zeros): dst_diff (+)= sum (a - b)^2 and dst_a (+)= sum a^2, in FP64 in a fixed order.
int launch_diff_norms(const float* a, long long acs, const float* b, long long bcs, long long npix, int nplanes,
                      double* partial, double* dst_diff, double* dst_a, int accumulate, hipStream_t st);
constexpr int kMaxPartials = 1 << 20;

// ------------------------------------------------------------------ visibility-domain data term
// One visibility of one channel (Sec. 2, eq. (viseq)): the baseline in wavelengths of the channel,
// and the residual (Phi x - v) that the forward pass leaves for the adjoint.  32 bytes, so that a
// wave-uniform visibility is one scalar load.
struct VisPt {
  double u, v, w;
  float rre, rim;
};
static_assert(sizeof(VisPt) == 32, "VisPt must stay 32 bytes");
// Row bands of the forward pass for N x N images, K visibilities and L channels.
int vis_chunks(int N, int K, int L);
// XN = X / n per pixel (X in slots of cs floats, XN dense planes).
int launch_vis_xn(const float* X, long long cs, const float* invn, float* XN, int N, int L, hipStream_t st);
// part[c][l][k]: band c's share of Phi_l (XN n)_k, C = vis_chunks(N, K, L) bands.
int launch_vis_fwd(const VisPt* vp, const float* XN, const double* lt, const double* nt, float2* part, int N, int K,
                   int L, int C, hipStream_t st);
// r = sum of the C bands + vsign vis (vis NULL: 0); vp receives w_l r (channel weights cw, NULL for 1)
// and rout (unless NULL) r; with partial, 1/2 w_l |r|^2 block sums (*nblocks of them).
int launch_vis_resid(const float2* part, int C, int L, int K, const float2* vis, float vsign, const float* cw,
                     VisPt* vp, double* partial, int* nblocks, float2* rout, hipStream_t st);
// out = Re Phi^H r (+ s_scale sadd), planes out_cs (sadd: s_cs) floats apart.
int launch_vis_adj(const VisPt* vp, int K, int L, const double* lt, const double* nt, const float* invn, int N,
                   float* out, long long out_cs, const float* sadd, long long s_cs, float s_scale, hipStream_t st);
// x *= f over the N x N planes of L channels in slots of cs floats.
int launch_vis_scale(float* x, long long cs, int N, int L, float f, hipStream_t st);

}  // namespace mf
