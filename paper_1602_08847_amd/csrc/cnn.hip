// Warm-start CNN: four 3x3 convolutions 1 -> 32 -> 32 -> 32 -> 1, circular padding, bias, ReLU
// after the first three layers; BF16 weights and activations, FP32 accumulation, activations
// rounded to BF16 (nearest, ties to even) when stored.  Training uses MSE and Adam on FP32
// master weights.
//
// The two 32 -> 32 layers are implicit GEMMs on v_mfma_f32_32x32x16_bf16 (gfx950):
//   forward  z[p][o]  = b[o] + sum_{tap, c} W[o][c][tap] a[p + tap][c]   M = 32 pixels, N = 32 o, K = 9 x 32
//   data     dx[p][c] = sum_{tap, o} W[o][c][tap] dz[p - tap][o]         the forward kernel with taps
//                                                                          mirrored and W transposed
//   weight   dW[tap][o][c] = sum_p dz[p][o] a[p + tap][c]                M = 32 o, N = 32 c, K = pixels
// The forward edge layers use the same product: layer 1 with its nine taps as K (padded to 16),
// layer 4 with its nine taps as the output columns (padded to 32) followed by a nine-point sum.
// Operand lane layout of the 32x32x16 BF16 MFMA (checked on the device): A[i][k] sits in lane
// i + 32 (k / 8), element k % 8; B[k][j] in lane j + 32 (k / 8), element k % 8; D[i][j] in lane
// j + 32 ((i / 4) % 2), register (i % 4) + 4 (i / 8).
// Activations are NHWC BF16 ([pixel][32]); network inputs and outputs are FP32 planes [B][N][N].
#include "common.h"

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

namespace mf {

constexpr int FC = 32;  // feature channels
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }
__device__ __forceinline__ bool bf_pos(uint16_t h) { return h != 0 && (h & 0x8000u) == 0; }
__device__ __forceinline__ int wrapn(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

// ------------------------------------------------------------------ 32 -> 32 layers, MFMA
enum MmaMode { MM_ACT = 0, MM_Z = 1, MM_DMASK = 2, MM_DRAW = 3 };
constexpr int TPX = 32, TROWS = 8;      // output tile: 32 pixels x 8 rows per workgroup
constexpr int PSTR = 40;                // LDS pixel stride in bf16 (80 bytes: conflict-free 16-byte reads)

// in: NHWC BF16 activations (or gradients); wg: [9][32 j][32 k] BF16 with B[k][j] = wg[tap][j][k];
// the tap offset applied to the input is +(dy, dx) for tap = (dy + 1) * 3 + (dx + 1).
constexpr int kTileChunks = (TROWS + 2) * (TPX + 2) * 4;  // 16-byte chunks of a haloed input tile
constexpr int kTileLoads = (kTileChunks + 255) / 256;     // of them per thread

// 16-byte chunk k of the haloed input tile t (one-pixel periodic halo)
__device__ __forceinline__ const u16x8* tile_chunk(const uint16_t* in, long long t, int k, int N) {
  const int tiles_x = N / TPX, tiles_y = N / TROWS;
  const int tx = (int)(t % tiles_x);
  const long long rest = t / tiles_x;
  const int ty = (int)(rest % tiles_y);
  const long long b = rest / tiles_y;
  const int q = k & 3, pix = k >> 2;
  const int r = pix / (TPX + 2), c = pix - r * (TPX + 2);
  const int gy = wrapn(ty * TROWS + r - 1, N), gx = wrapn(tx * TPX + c - 1, N);
  return reinterpret_cast<const u16x8*>(in + b * (long long)N * N * FC + ((long long)gy * N + gx) * FC + q * 8);
}

__device__ __forceinline__ void stage_weights(uint16_t* tw, const uint16_t* wg) {
  for (int i = threadIdx.x; i < 9 * FC * 4; i += 256) {  // 9 x 32 rows of 64 bytes
    const int row = i >> 2, q = i & 3;
    *reinterpret_cast<u16x8*>(tw + row * PSTR + q * 8) = *reinterpret_cast<const u16x8*>(wg + row * FC + q * 8);
  }
}

// The MFMA sums of output row r of a tile (32 pixels x 32 outputs) from its haloed input tile tc
// and the weights tw, both in LDS.
__device__ __forceinline__ f32x16 conv_row(const uint16_t* tc, const uint16_t* tw, int r) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 31, kh8 = (lane >> 5) * 8;
  f32x16 acc = {};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3, dx = tap % 3;  // input offset +1 (halo)
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      const u16x8 av = *reinterpret_cast<const u16x8*>(tc + ((r + dy) * (TPX + 2) + li + dx) * PSTR + kh * 16 + kh8);
      const u16x8 bv = *reinterpret_cast<const u16x8*>(tw + (tap * FC + li) * PSTR + kh * 16 + kh8);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                    acc, 0, 0, 0);
    }
  }
  return acc;
}

// The same for the two output rows r0 and r0 + 1 together: each weight operand read feeds both rows.
__device__ __forceinline__ void conv_rows2(const uint16_t* tc, const uint16_t* tw, int r0, f32x16 (&acc)[2]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 31, kh8 = (lane >> 5) * 8;
  acc[0] = f32x16{};
  acc[1] = f32x16{};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3, dx = tap % 3;  // input offset +1 (halo)
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
      const u16x8 bv = *reinterpret_cast<const u16x8*>(tw + (tap * FC + li) * PSTR + kh * 16 + kh8);
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        const u16x8 av =
            *reinterpret_cast<const u16x8*>(tc + ((r0 + tt + dy) * (TPX + 2) + li + dx) * PSTR + kh * 16 + kh8);
        acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                          __builtin_bit_cast(bf16x8, bv), acc[tt], 0, 0, 0);
      }
    }
  }
}

// The MFMA sums of tile t (8 rows of 32 pixels x 32 outputs: wave w owns rows 2w, 2w + 1) and the
// epilogue of MODE.
template <int MODE>
__device__ __forceinline__ void conv_tile(const uint16_t* tc, const uint16_t* tw, long long t,
                                          const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                                          uint16_t* __restrict__ out16, float* __restrict__ out32, int N) {
  const int tiles_x = N / TPX, tiles_y = N / TROWS;
  const int tx = (int)(t % tiles_x);
  const long long rest = t / tiles_x;
  const int ty = (int)(rest % tiles_y);
  const long long b = rest / tiles_y;
  const int x0 = tx * TPX, y0 = ty * TROWS;
  const long long n2 = (long long)N * N;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31;
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int r = 2 * w + tt;  // output row within the tile
    const f32x16 acc = conv_row(tc, tw, r);
    const int y = y0 + r;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);  // pixel within the 32-pixel row segment
      const int j = li;                                        // output channel
      const long long pix = b * n2 + (long long)y * N + x0 + i;
      float v = acc[e];
      if constexpr (MODE == MM_ACT) {
        out16[pix * FC + j] = f2bf(fmaxf(v + bias[j], 0.f));
      } else if constexpr (MODE == MM_Z) {
        out32[((b * FC + j) * N + y) * (long long)N + x0 + i] = v + bias[j];
      } else if constexpr (MODE == MM_DMASK) {
        out16[pix * FC + j] = bf_pos(mask[pix * FC + j]) ? f2bf(v) : (uint16_t)0;
      } else {
        out32[((b * FC + j) * N + y) * (long long)N + x0 + i] = v;
      }
    }
  }
}

// Tile t of the image batch: 8 rows x 32 pixels at (x0, y0) of image b.
struct TileAt {
  long long b;
  int x0, y0;
};
__device__ __forceinline__ TileAt tile_at(long long t, int N) {
  const int tiles_x = N / TPX, tiles_y = N / TROWS;
  const long long rest = t / tiles_x;
  return TileAt{rest / tiles_y, (int)(t % tiles_x) * TPX, (int)(rest % tiles_y) * TROWS};
}

// One tile per workgroup (the backward and single-layer modes).
template <int MODE>
__global__ void __launch_bounds__(256) k_conv_mma(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wg,
                                                  const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                                                  uint16_t* __restrict__ out16, float* __restrict__ out32, int N,
                                                  int nimg) {
  __shared__ __attribute__((aligned(16))) uint16_t tin[(TROWS + 2) * (TPX + 2) * PSTR];
  __shared__ __attribute__((aligned(16))) uint16_t tw[9 * FC * PSTR];
  (void)nimg;
  stage_weights(tw, wg);
  for (int k = threadIdx.x; k < kTileChunks; k += 256)
    *reinterpret_cast<u16x8*>(tin + (k >> 2) * PSTR + (k & 3) * 8) = *tile_chunk(in, blockIdx.x, k, N);
  __syncthreads();
  conv_tile<MODE>(tin, tw, blockIdx.x, bias, mask, out16, out32, N);
}

// Forward activations, persistent: each workgroup stages the weights once and walks the tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...; the next tile's input loads are in flight while the
// MFMAs of the current one run, in registers.  Its barriers (and those of the persistent edge-layer
// kernels) order LDS only: a tile's output stores and the next tile's loads stay in flight across
// them.  (The other modes keep one tile per workgroup.)
constexpr int kConvBlocks = 768;  // three resident workgroups per CU
unsigned conv_grid(long long tiles, int blocks = kConvBlocks) { return (unsigned)(tiles < blocks ? tiles : blocks); }
// the edge layers' persistent grids: as many workgroups as fit on a CU (LDS 21 KB and 39 KB)
constexpr int kConv1Blocks = 256 * 6, kConv4Blocks = 256 * 4;

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_conv_act(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wg,
                                                  const float* __restrict__ bias, uint16_t* __restrict__ out16, int N,
                                                  int nimg) {
  // one tile buffer (50 KB of LDS with the weights: three workgroups per CU); the next tile waits
  // in registers until every wave is done with the current one
  __shared__ __attribute__((aligned(16))) uint16_t tin[(TROWS + 2) * (TPX + 2) * PSTR];
  __shared__ __attribute__((aligned(16))) uint16_t tw[9 * FC * PSTR];
  const long long ntiles = (long long)nimg * (N / TPX) * (N / TROWS);
  stage_weights(tw, wg);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 31;
  const float bj = bias[li];
  u16x8 pre[kTileLoads];
  auto fetch = [&](long long tt) {
#pragma unroll
    for (int m = 0; m < kTileLoads; ++m) {
      const int k = threadIdx.x + 256 * m;
      pre[m] = *tile_chunk(in, tt, k < kTileChunks ? k : kTileChunks - 1, N);
    }
  };
  long long t = blockIdx.x;
  if (t < ntiles) fetch(t);
  for (; t < ntiles; t += gridDim.x) {
#pragma unroll
    for (int m = 0; m < kTileLoads; ++m) {
      const int k = threadIdx.x + 256 * m;
      if (k < kTileChunks) *reinterpret_cast<u16x8*>(tin + (k >> 2) * PSTR + (k & 3) * 8) = pre[m];
    }
    lds_barrier();  // the tile is in place
    if (t + gridDim.x < ntiles) fetch(t + gridDim.x);  // in flight during the products
    f32x16 acc[2];
    conv_rows2(tin, tw, 2 * w, acc);
    lds_barrier();  // every wave is done reading the tile: it now stages the outputs
    // this wave's two rows, 64 pixels x 32 channels (BF16, pixel stride PSTR), then 16-byte stores
    // of one pixel's 8 channels
    uint16_t* os = tin + w * 2 * TPX * PSTR;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);  // pixel within the segment; channel li
        os[(tt * TPX + i) * PSTR + li] = f2bf(fmaxf(acc[tt][e] + bj, 0.f));
      }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    const TileAt ta = tile_at(t, N);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = lane + 64 * q;  // pixel ch / 4 of the two rows, channels 8 (ch % 4) ..
      const int px = ch >> 2, part = ch & 3;
      const int y = ta.y0 + 2 * w + px / TPX;
      *reinterpret_cast<u16x8*>(out16 + (ta.b * (long long)N * N + (long long)y * N + ta.x0 + px % TPX) * FC +
                                part * 8) = *reinterpret_cast<const u16x8*>(os + px * PSTR + part * 8);
    }
    lds_barrier();  // every wave is done with its staged outputs before the next tile overwrites them
  }
}

// Inference, layers 1 and 2 in one pass: layer 1 is computed on the haloed 10 x 34 tile of a1 from a
// 12 x 36 tile of x (MFMA as in k_conv1_mma, two overlapping 32-pixel segments per row) straight
// into LDS, and layer 2 reads it there as k_conv_act reads its input tile; a1 never reaches
// memory.  Every product and rounding is the one of the separate kernels, so a2 is the same bit for
// bit.  Persistent, with the next tile's x in registers.
constexpr int kX12 = (TROWS + 4) * (TPX + 4);  // haloed x tile of the fused pass
constexpr int kX12Loads = (kX12 + 255) / 256;
__global__ void __launch_bounds__(256) k_conv12_act(const float* __restrict__ x, const float* __restrict__ w1b,
                                                    const float* __restrict__ b1, const uint16_t* __restrict__ wg,
                                                    const float* __restrict__ b2, uint16_t* __restrict__ out16, int N,
                                                    int nimg) {
  constexpr int XW = TPX + 4, TW = TPX + 2;
  __shared__ uint16_t xs[kX12];
  __shared__ __attribute__((aligned(16))) uint16_t tin[(TROWS + 2) * TW * PSTR];
  __shared__ __attribute__((aligned(16))) uint16_t tw[9 * FC * PSTR];
  const long long ntiles = (long long)nimg * (N / TPX) * (N / TROWS);
  const long long n2 = (long long)N * N;
  stage_weights(tw, wg);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 31, kb = (lane >> 5) * 8;
  u16x8 bv1;  // layer 1: B[k][j] = W1[j][tap k]
#pragma unroll
  for (int e = 0; e < 8; ++e) bv1[e] = kb + e < 9 ? f2bf(w1b[(kb + e) * FC + li]) : (uint16_t)0;
  const float bias1 = b1[li], bias2 = b2[li];
  float pre[kX12Loads];
  auto fetch = [&](long long tt) {
    const TileAt ta = tile_at(tt, N);
    const float* xb = x + ta.b * n2;
#pragma unroll
    for (int m = 0; m < kX12Loads; ++m) {
      int i = threadIdx.x + 256 * m;
      i = i < kX12 ? i : kX12 - 1;
      const int r = i / XW, c = i - r * XW;
      pre[m] = xb[(long long)wrapn(ta.y0 + r - 2, N) * N + wrapn(ta.x0 + c - 2, N)];
    }
  };
  long long t = blockIdx.x;
  if (t < ntiles) fetch(t);
  for (; t < ntiles; t += gridDim.x) {
#pragma unroll
    for (int m = 0; m < kX12Loads; ++m) {
      const int i = threadIdx.x + 256 * m;
      if (i < kX12) xs[i] = f2bf(pre[m]);
    }
    lds_barrier();  // x is in place, and every wave is done with the previous tile's outputs
    if (t + gridDim.x < ntiles) fetch(t + gridDim.x);
    // layer 1 on a1 rows 0..9 (image rows y0 - 1 ..), columns 0..33, items (row, segment)
    for (int it = w; it < 2 * (TROWS + 2); it += 4) {
      const int r = it >> 1, c0 = (it & 1) ? 2 : 0;
      u16x8 av;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kb + e;  // a1 (r, c0 + li) reads x tile row r + k / 3, column c0 + li + k % 3
        av[e] = k < 9 ? xs[(r + k / 3) * XW + c0 + li + k % 3] : (uint16_t)0;
      }
      f32x16 a = {};
      a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv1), a,
                                                  0, 0, 0);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);  // pixel c0 + i of the row; channel li
        if (c0 == 0 || c0 + i >= TPX) tin[(r * TW + c0 + i) * PSTR + li] = f2bf(fmaxf(a[e] + bias1, 0.f));
      }
    }
    lds_barrier();  // a1 is in place
    f32x16 acc[2];
    conv_rows2(tin, tw, 2 * w, acc);
    lds_barrier();  // every wave is done reading a1: the tile now stages the outputs
    uint16_t* os = tin + w * 2 * TPX * PSTR;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);
        os[(tt * TPX + i) * PSTR + li] = f2bf(fmaxf(acc[tt][e] + bias2, 0.f));
      }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    const TileAt ta = tile_at(t, N);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = lane + 64 * q;
      const int px = ch >> 2, part = ch & 3;
      const int y = ta.y0 + 2 * w + px / TPX;
      *reinterpret_cast<u16x8*>(out16 + (ta.b * n2 + (long long)y * N + ta.x0 + px % TPX) * FC + part * 8) =
          *reinterpret_cast<const u16x8*>(os + px * PSTR + part * 8);
    }
  }
}

// ------------------------------------------------------------------ edge layers on the MFMA
// Layer 1 (1 -> 32): z[p][o] = b[o] + sum_tap W1[o][tap] bf16(x[p + tap]) as one 32x32x16 product
// per 32-pixel row segment, A[i][k] = bf16(x[pixel i + offset of tap k]) (k < 9; zero for k >= 9),
// B[k][j] = W1[j][tap k].  Persistent workgroups walk the 8-row x 32-pixel tiles (wave w: rows 2w,
// 2w + 1); the next tile's haloed x is loaded while the current one is multiplied.
// mode 0: a1 = bf16(relu(z)) NHWC, staged per wave in LDS so that every store is 16 bytes of one
// pixel; mode 1: z FP32 [B][32][N][N].
constexpr int kX1 = (TROWS + 2) * (TPX + 2);     // haloed x tile
constexpr int kX1Loads = (kX1 + 255) / 256;
__global__ void __launch_bounds__(256) k_conv1_mma(const float* __restrict__ x, const float* __restrict__ w1b,
                                                   const float* __restrict__ b1, uint16_t* __restrict__ a1,
                                                   float* __restrict__ zout, int N, int nimg, int mode) {
  constexpr int TW = TPX + 2;
  __shared__ uint16_t xs[kX1];
  __shared__ __attribute__((aligned(16))) uint16_t os[4][2 * TPX * PSTR];  // per wave: 2 rows x 32 pixels
  const long long ntiles = (long long)nimg * (N / TPX) * (N / TROWS);
  const long long n2 = (long long)N * N;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, kb = (lane >> 5) * 8;  // this lane's k = kb .. kb + 7
  u16x8 bv;
#pragma unroll
  for (int e = 0; e < 8; ++e) bv[e] = kb + e < 9 ? f2bf(w1b[(kb + e) * FC + li]) : (uint16_t)0;
  const float bias = b1[li];
  float pre[kX1Loads];
  auto fetch = [&](long long t) {
    const TileAt ta = tile_at(t, N);
    const float* xb = x + ta.b * n2;
#pragma unroll
    for (int m = 0; m < kX1Loads; ++m) {
      int i = threadIdx.x + 256 * m;
      i = i < kX1 ? i : kX1 - 1;
      const int r = i / TW, c = i - r * TW;
      pre[m] = xb[(long long)wrapn(ta.y0 + r - 1, N) * N + wrapn(ta.x0 + c - 1, N)];
    }
  };
  long long t = blockIdx.x;
  if (t < ntiles) fetch(t);
  for (; t < ntiles; t += gridDim.x) {
#pragma unroll
    for (int m = 0; m < kX1Loads; ++m) {
      const int i = threadIdx.x + 256 * m;
      if (i < kX1) xs[i] = f2bf(pre[m]);
    }
    lds_barrier();
    if (t + gridDim.x < ntiles) fetch(t + gridDim.x);  // in flight during the products
    const TileAt ta = tile_at(t, N);
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int r = 2 * w + tt;  // output row within the tile
      u16x8 av;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kb + e;  // tap k reads tile row r + k / 3, column li + k % 3 (halo offset +1)
        av[e] = k < 9 ? xs[(r + k / 3) * TW + li + k % 3] : (uint16_t)0;
      }
      f32x16 acc = {};
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                    acc, 0, 0, 0);
      const int y = ta.y0 + r;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);  // pixel within the segment; channel li
        const float v = acc[e] + bias;
        if (mode == 0) os[w][(tt * TPX + i) * PSTR + li] = f2bf(fmaxf(v, 0.f));
        else zout[((ta.b * FC + li) * N + y) * (long long)N + ta.x0 + i] = v;
      }
    }
    if (mode == 0) {
      // this wave's two rows: 64 pixels x four 16-byte chunks, read back across lanes
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ch = lane + 64 * q;  // chunk: pixel ch / 4 of the two rows, channels 8 (ch % 4) ..
        const int px = ch >> 2, part = ch & 3;
        const int y = ta.y0 + 2 * w + px / TPX;
        const u16x8 v = *reinterpret_cast<const u16x8*>(&os[w][px * PSTR + part * 8]);
        *reinterpret_cast<u16x8*>(a1 + (ta.b * n2 + (long long)y * N + ta.x0 + px % TPX) * FC + part * 8) = v;
      }
    }
    lds_barrier();  // xs and os are rewritten for the next tile
  }
}

// Layer 4 (32 -> 1): z[p] = b4 + sum_tap Y[p + offset(tap)][tap] with Y[q][tap] = sum_c W4[tap][c] a3[q][c].
// Y of the tile's haloed 10 x 34 pixels comes from 32x32x16 products (A[i][k] = a3[pixel i][k] over
// two halves of the 32 channels, B[k][j] = W4[tap j][k] for j < 9, zero beyond) into LDS; each
// row of 34 takes two overlapping segments (columns 0..31 and 2..33, the second keeping 32 and 33).
// Then one thread per output pixel adds the bias and its nine Y terms in tap order.  Persistent
// workgroups; the next tile's activations are loaded while the current one is multiplied.
__global__ void __launch_bounds__(256) k_conv4_mma(const uint16_t* __restrict__ a3, const float* __restrict__ w4b,
                                                   const float* __restrict__ b4, float* __restrict__ z, int N,
                                                   int nimg) {
  constexpr int TW = TPX + 2, YS = 9;
  __shared__ __attribute__((aligned(16))) uint16_t tin[(TROWS + 2) * TW * PSTR];
  __shared__ float ys[(TROWS + 2) * TW * YS];
  const long long ntiles = (long long)nimg * (N / TPX) * (N / TROWS);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, kh8 = (lane >> 5) * 8;
  u16x8 bv[2];
#pragma unroll
  for (int kh = 0; kh < 2; ++kh)
#pragma unroll
    for (int e = 0; e < 8; ++e) bv[kh][e] = li < 9 ? f2bf(w4b[li * FC + kh * 16 + kh8 + e]) : (uint16_t)0;
  const float bias = b4[0];
  u16x8 pre[kTileLoads];
  auto fetch = [&](long long t) {
#pragma unroll
    for (int m = 0; m < kTileLoads; ++m) {
      const int k = threadIdx.x + 256 * m;
      pre[m] = *tile_chunk(a3, t, k < kTileChunks ? k : kTileChunks - 1, N);
    }
  };
  long long t = blockIdx.x;
  if (t < ntiles) fetch(t);
  for (; t < ntiles; t += gridDim.x) {
#pragma unroll
    for (int m = 0; m < kTileLoads; ++m) {
      const int k = threadIdx.x + 256 * m;
      if (k < kTileChunks) *reinterpret_cast<u16x8*>(tin + (k >> 2) * PSTR + (k & 3) * 8) = pre[m];
    }
    lds_barrier();
    if (t + gridDim.x < ntiles) fetch(t + gridDim.x);  // in flight during the products
    // (row, segment) items 0 .. 19, wave w takes w, w + 4, ...
    for (int it = w; it < 2 * (TROWS + 2); it += 4) {
      const int r = it >> 1, c0 = (it & 1) ? 2 : 0;
      f32x16 acc = {};
#pragma unroll
      for (int kh = 0; kh < 2; ++kh) {
        const u16x8 av = *reinterpret_cast<const u16x8*>(tin + (r * TW + c0 + li) * PSTR + kh * 16 + kh8);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                      __builtin_bit_cast(bf16x8, bv[kh]), acc, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int i = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);  // pixel within the segment; tap li
        if (li < 9 && (c0 == 0 || c0 + i >= TPX)) ys[(r * TW + c0 + i) * YS + li] = acc[e];
      }
    }
    lds_barrier();
    const TileAt ta = tile_at(t, N);
    const int r = threadIdx.x / TPX, c = threadIdx.x % TPX;
    float acc = bias;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc += ys[((r + tap / 3) * TW + c + tap % 3) * YS + tap];
    z[ta.b * (long long)N * N + (long long)(ta.y0 + r) * N + ta.x0 + c] = acc;
    // tin is rewritten next only after every wave has passed the barrier above (its products are
    // done), ys only after the barrier that follows the next tile's store
  }
}

// ------------------------------------------------------------------ weight gradient, MFMA
// dW[tap][o][c] = sum_p dz[p][o] a[p + tap][c], db[o] = sum_p dz[p][o].  A workgroup of three
// waves walks 32-pixel row segments; wave w owns the taps of row offset dy = w - 1.  Each
// segment stages dz transposed ([o][32 px]) and a transposed for the three rows and three
// column shifts ([row][dx][c][32 px]), so every operand is one aligned 16-byte LDS read.
// Partial sums per workgroup: partial[blk][tap * 1024 + o * 32 + c] and [9216 + o].
constexpr int WPART = 9 * FC * FC + FC;
__global__ void __launch_bounds__(192) k_wgrad_mma(const uint16_t* __restrict__ dz, const uint16_t* __restrict__ a,
                                                   float* __restrict__ partial, int N, long long nseg) {
  __shared__ __attribute__((aligned(16))) uint16_t dzT[FC * PSTR];
  __shared__ __attribute__((aligned(16))) uint16_t aT[3 * 3 * FC * PSTR];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, kh8 = (lane >> 5) * 8;
  const long long n2 = (long long)N * N;
  const int segs_x = N / TPX;
  f32x16 acc[3] = {{}, {}, {}};
  float dbacc = 0.f;
  for (long long sgi = blockIdx.x; sgi < nseg; sgi += gridDim.x) {
    const int sx = (int)(sgi % segs_x);
    const long long rowid = sgi / segs_x;  // b * N + y
    const long long b = rowid / N;
    const int y = (int)(rowid - b * N), x0 = sx * TPX;
    const uint16_t* dzb = dz + b * n2 * FC;
    const uint16_t* ab = a + b * n2 * FC;
    // dz segment, transposed: 32 px x 4 chunks of 8 channels
    for (int i = threadIdx.x; i < TPX * 4; i += 192) {
      const int px = i >> 2, q = i & 3;
      const u16x8 v = *reinterpret_cast<const u16x8*>(dzb + ((long long)y * N + x0 + px) * FC + q * 8);
#pragma unroll
      for (int e = 0; e < 8; ++e) dzT[(q * 8 + e) * PSTR + px] = v[e];
    }
    // a rows y-1, y, y+1 and columns x0-1 .. x0+32, scattered to the three column shifts
    for (int i = threadIdx.x; i < 3 * (TPX + 2) * 4; i += 192) {
      const int q = i & 3, rest = i >> 2;
      const int r = rest / (TPX + 2), c = rest - r * (TPX + 2);
      const int gy = wrapn(y + r - 1, N), gx = wrapn(x0 + c - 1, N);
      const u16x8 v = *reinterpret_cast<const u16x8*>(ab + ((long long)gy * N + gx) * FC + q * 8);
#pragma unroll
      for (int dxi = 0; dxi < 3; ++dxi) {
        const int px = c - dxi;  // a[x + dx] with dx = dxi - 1 sits at column c = x - x0 + dxi
        if (px >= 0 && px < TPX) {
#pragma unroll
          for (int e = 0; e < 8; ++e) aT[((r * 3 + dxi) * FC + q * 8 + e) * PSTR + px] = v[e];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int dxi = 0; dxi < 3; ++dxi) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const u16x8 av = *reinterpret_cast<const u16x8*>(dzT + li * PSTR + ks * 16 + kh8);
        const u16x8 bv = *reinterpret_cast<const u16x8*>(aT + ((w * 3 + dxi) * FC + li) * PSTR + ks * 16 + kh8);
        acc[dxi] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                           __builtin_bit_cast(bf16x8, bv), acc[dxi], 0, 0, 0);
      }
    }
    if (w == 1 && lane < 32) {
      float s = 0.f;
      for (int px = 0; px < TPX; ++px) s += bf2f(dzT[lane * PSTR + px]);
      dbacc += s;
    }
    __syncthreads();
  }
  float* pb = partial + (long long)blockIdx.x * WPART;
#pragma unroll
  for (int dxi = 0; dxi < 3; ++dxi) {
    const int tap = w * 3 + dxi;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int o = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);
      pb[tap * FC * FC + o * FC + li] = acc[dxi][e];
    }
  }
  if (w == 1 && lane < 32) pb[9 * FC * FC + lane] = dbacc;
}

// dz4 = bf16(2 (z - t) / M); partial[block] = sum (z - t)^2 (FP64)
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ z, const float* __restrict__ tgt,
                                             float* __restrict__ dz, double* __restrict__ partial, long long P,
                                             float scale) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < P; p += (long long)gridDim.x * 256) {
    const float r = z[p] - tgt[p];
    s += (double)r * r;
    dz[p] = bfround(scale * r);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Layer 4 data gradient: da3[p][c] = sum_tap W4[tap][c] dz4[p - tap]; mode 0: masked by a3 > 0 and
// rounded to BF16 (NHWC); mode 1: FP32 [B][32][N][N] without mask.
__global__ void __launch_bounds__(256) k_conv4_bwd_data(const float* __restrict__ dz4, const float* __restrict__ w4b,
                                                        const uint16_t* __restrict__ a3, uint16_t* __restrict__ dz3,
                                                        float* __restrict__ dx32, int N, long long P, int mode) {
  __shared__ float sw[9 * FC];
  for (int i = threadIdx.x; i < 9 * FC; i += 256) sw[i] = w4b[i];
  __syncthreads();
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const long long n2 = (long long)N * N;
  const long long b = p / n2;
  const int yx = (int)(p - b * n2), y = yx / N, xx = yx - y * N;
  float d[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = wrapn(y - (t / 3 - 1), N), xq = wrapn(xx - (t % 3 - 1), N);
    d[t] = dz4[b * n2 + (long long)yy * N + xq];
  }
  u16x8 out[4];
  u16x8 m[4];
  if (mode == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) m[q] = reinterpret_cast<const u16x8*>(a3 + p * FC)[q];
  }
#pragma unroll
  for (int c = 0; c < FC; ++c) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) s = fmaf(sw[t * FC + c], d[t], s);
    if (mode == 0) out[c / 8][c % 8] = bf_pos(m[c / 8][c % 8]) ? f2bf(s) : (uint16_t)0;
    else dx32[((b * FC + c) * N + y) * (long long)N + xx] = s;
  }
  if (mode == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) reinterpret_cast<u16x8*>(dz3 + p * FC)[q] = out[q];
  }
}

// Weight gradients of the single-channel layers, VALU.  Thread (g, c): c = lane % 32 is the
// feature channel, g = tid / 32 one of 8 pixel groups.
//   layer 4: dW4[tap][c] = sum_p dz4[p] a3[p + tap][c], db4 = sum_p dz4[p]
//   layer 1: dW1[tap][o] = sum_p dz1[p][o] x[p + tap],   db1[o] = sum_p dz1[p][o]
// partial[blk][tap * 32 + c] (9 x 32) and [288 + c] (bias; layer 4 uses entry 288 only).
constexpr int SPART = 9 * FC + FC;
template <int LAYER>
__global__ void __launch_bounds__(256) k_wgrad_single(const float* __restrict__ dzs, const uint16_t* __restrict__ act,
                                                      const uint16_t* __restrict__ dzm, const float* __restrict__ xin,
                                                      float* __restrict__ partial, int N, long long P) {
  __shared__ float red[8][SPART];
  const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long long n2 = (long long)N * N;
  float acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (long long p = (long long)blockIdx.x * 8 + g; p < P; p += (long long)gridDim.x * 8) {
    const long long b = p / n2;
    const int yx = (int)(p - b * n2), y = yx / N, xx = yx - y * N;
    const float d = (LAYER == 4) ? dzs[p] : bf2f(dzm[p * FC + c]);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const long long q = b * n2 + (long long)wrapn(y + t / 3 - 1, N) * N + wrapn(xx + t % 3 - 1, N);
      const float v = (LAYER == 4) ? bf2f(act[q * FC + c]) : bfround(xin[q]);
      acc[t] = fmaf(d, v, acc[t]);
    }
    acc[9] += d;
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) red[g][t * FC + c] = acc[t];
  red[g][9 * FC + c] = acc[9];
  __syncthreads();
  for (int i = threadIdx.x; i < SPART; i += 256) {
    float s = 0.f;
    for (int k = 0; k < 8; ++k) s += red[k][i];
    partial[(long long)blockIdx.x * SPART + i] = s;
  }
}

// out[map(i)] = sum_blk partial[blk][i] for i < n, in FP64.  A workgroup reduces 32 consecutive
// entries; its 8 thread groups take every 8th block (group g: blocks g, g + 8, ... in order), and
// the 8 group sums are added in group order, so the result does not depend on timing.
// map: 0 identity; 1: [tap][o][c] -> [o][c][tap] (32 x 32 layers, bias after 9216);
// 2: [tap][c] -> [c][tap] (single-channel layers, bias at 288 (layer 4: only entry 288 used)).
constexpr int kRedEntries = 32, kRedGroups = 8;  // entries per workgroup, block groups per entry
__global__ void __launch_bounds__(256) k_reduce_partials(const float* __restrict__ partial, int stride, int n,
                                                         int nblk, float* __restrict__ out, int map) {
  __shared__ double red[kRedGroups][kRedEntries];
  const int e = threadIdx.x % kRedEntries, g = threadIdx.x / kRedEntries;
  const int i = blockIdx.x * kRedEntries + e;
  double s = 0.0;
  if (i < n)
    for (int k = g; k < nblk; k += kRedGroups) s += partial[(long long)k * stride + i];
  red[g][e] = s;
  __syncthreads();
  if (g != 0 || i >= n) return;
  s = red[0][e];
  for (int q = 1; q < kRedGroups; ++q) s += red[q][e];
  int dst = i;
  if (map == 1 && i < 9 * FC * FC) {
    const int tap = i / (FC * FC), o = (i / FC) % FC, c = i % FC;
    dst = (o * FC + c) * 9 + tap;
  } else if (map == 2 && i < 9 * FC) {
    const int tap = i / FC, c = i % FC;
    dst = c * 9 + tap;
  }
  out[dst] = (float)s;
}

// Adam on FP32 master weights.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Derived BF16 weights from the FP32 master parameters (layout of the parameter vector:
// w1[32][1][3][3] b1[32] w2[32][32][3][3] b2[32] w3[32][32][3][3] b3[32] w4[1][32][3][3] b4[1]).
struct CnnOffsets {
  static constexpr int w1 = 0, b1 = 288, w2 = 320, b2 = 9536, w3 = 9568, b3 = 18784, w4 = 18816, b4 = 19104,
                       total = 19105;
};
__global__ void __launch_bounds__(256) k_prep_weights(const float* __restrict__ prm, float* __restrict__ w1b,
                                                      uint16_t* __restrict__ w2f, uint16_t* __restrict__ w2d,
                                                      uint16_t* __restrict__ w3f, uint16_t* __restrict__ w3d,
                                                      float* __restrict__ w4b) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < 9 * FC * FC) {
    const int tap = i / (FC * FC), j = (i / FC) % FC, k = i % FC;
    // forward: B[k = c][j = o] = W[o][c][tap]
    w2f[i] = f2bf(prm[CnnOffsets::w2 + (j * FC + k) * 9 + tap]);
    w3f[i] = f2bf(prm[CnnOffsets::w3 + (j * FC + k) * 9 + tap]);
    // data gradient: B[k = o][j = c] = W[o][c][8 - tap]
    w2d[i] = f2bf(prm[CnnOffsets::w2 + (k * FC + j) * 9 + (8 - tap)]);
    w3d[i] = f2bf(prm[CnnOffsets::w3 + (k * FC + j) * 9 + (8 - tap)]);
  }
  if (i < 9 * FC) {
    const int tap = i / FC, c = i % FC;
    w1b[i] = bfround(prm[CnnOffsets::w1 + c * 9 + tap]);
    w4b[i] = bfround(prm[CnnOffsets::w4 + c * 9 + tap]);
  }
}

// x / s_l per plane (input normalisation of the warm start)
// out[b][p] = x[b xcs + p] / s[b sstride] over nimg planes of n2 pixels (x has channel stride xcs)
__global__ void __launch_bounds__(256) k_scale_planes(const float* __restrict__ x, long long xcs,
                                                      const float* __restrict__ s, int sstride,
                                                      float* __restrict__ out, long long n2, int nimg) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n2 * nimg) return;
  const long long b = i / n2;
  out[i] = x[b * xcs + (i - b * n2)] / s[b * sstride];
}

}  // namespace mf

// ================================================================== C ABI
using namespace mf;

struct muffin_cnn {
  int device = 0;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  float *prm = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  float *w1b = nullptr, *w4b = nullptr;
  uint16_t *w2f = nullptr, *w2d = nullptr, *w3f = nullptr, *w3d = nullptr;
  long long cap = 0;  // pixel capacity of the workspaces
  float* xin = nullptr;
  uint16_t *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *g3 = nullptr, *g2 = nullptr, *g1 = nullptr;
  float *z4 = nullptr, *dz4 = nullptr;
  float* partial = nullptr;
  double* dpart = nullptr;
  double* dres = nullptr;
  long long t = 0;
};

namespace {
constexpr int kWgradBlocks = 1024;
constexpr int kSingleBlocks = 1024;
constexpr long long kChunkPixels = 16ll << 20;  // pixels per inference chunk

struct CnnScope {
  muffin_cnn* c;
  bool ok;
  explicit CnnScope(muffin_cnn* c_) : c(c_) {
    ok = hipEventRecord(c->ev_in, c->user) == hipSuccess && hipStreamWaitEvent(c->st, c->ev_in, 0) == hipSuccess;
  }
  ~CnnScope() {
    if (hipEventRecord(c->ev_out, c->st) == hipSuccess) (void)hipStreamWaitEvent(c->user, c->ev_out, 0);
  }
};

template <typename T>
int dal(T** p, size_t n) {
  if (hipMalloc((void**)p, sizeof(T) * (n ? n : 1)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation failed");
    return MUFFIN_ENOMEM;
  }
  return MUFFIN_OK;
}

void free_ws(muffin_cnn* c) {
  void* ps[] = {c->xin, c->a1, c->a2, c->a3, c->g3, c->g2, c->g1, c->z4, c->dz4};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  c->xin = nullptr;
  c->a1 = c->a2 = c->a3 = c->g3 = c->g2 = c->g1 = nullptr;
  c->z4 = c->dz4 = nullptr;
  c->cap = 0;
}

int ensure_ws(muffin_cnn* c, long long P) {
  if (P <= c->cap) return MUFFIN_OK;
  MF_HIP(hipStreamSynchronize(c->st));
  free_ws(c);
  MF_TRY(dal(&c->xin, P));
  MF_TRY(dal(&c->a1, P * FC));
  MF_TRY(dal(&c->a2, P * FC));
  MF_TRY(dal(&c->a3, P * FC));
  MF_TRY(dal(&c->g3, P * FC));
  MF_TRY(dal(&c->g2, P * FC));
  MF_TRY(dal(&c->g1, P * FC));
  MF_TRY(dal(&c->z4, P));
  MF_TRY(dal(&c->dz4, P));
  c->cap = P;
  return MUFFIN_OK;
}

int check_shape(int B, int N) {
  if (B < 1 || N < 32 || N > 4096 || N % TPX || N % TROWS)
    return set_error("CNN: need B >= 1 and N a multiple of 32 (32 <= N <= 4096)"), MUFFIN_EINVAL;
  return MUFFIN_OK;
}

int prep_weights(muffin_cnn* c) {
  hipLaunchKernelGGL(k_prep_weights, dim3((9 * FC * FC + 255) / 256), dim3(256), 0, c->st, c->prm, c->w1b, c->w2f,
                     c->w2d, c->w3f, c->w3d, c->w4b);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

// forward of P pixels (B images) from FP32 input planes into the activation planes a1, a2, a3
// (BF16, 32 features per pixel; a3 may be a1, which layer 3 no longer reads) and the output z
int forward_into(muffin_cnn* c, const float* x, int B, int N, uint16_t* a1, uint16_t* a2, uint16_t* a3, float* z) {
  const unsigned tiles = (unsigned)((long long)B * (N / TPX) * (N / TROWS));
  hipLaunchKernelGGL(k_conv1_mma, dim3(conv_grid(tiles, kConv1Blocks)), dim3(256), 0, c->st, x, c->w1b, c->prm + CnnOffsets::b1,
                     a1, (float*)nullptr, N, B, 0);
  hipLaunchKernelGGL(k_conv_act, dim3(conv_grid(tiles)), dim3(256), 0, c->st, a1, c->w2f, c->prm + CnnOffsets::b2, a2,
                     N, B);
  hipLaunchKernelGGL(k_conv_act, dim3(conv_grid(tiles)), dim3(256), 0, c->st, a2, c->w3f, c->prm + CnnOffsets::b3, a3,
                     N, B);
  hipLaunchKernelGGL(k_conv4_mma, dim3(conv_grid(tiles, kConv4Blocks)), dim3(256), 0, c->st, a3, c->w4b, c->prm + CnnOffsets::b4,
                     z, N, B);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// inference of B images: layers 1 and 2 in one pass into a2, layer 3 into a3 (may alias nothing
// else the pass reads), layer 4 into z; a1 is never formed
int forward_infer(muffin_cnn* c, const float* x, int B, int N, uint16_t* a2, uint16_t* a3, float* z) {
  const unsigned tiles = (unsigned)((long long)B * (N / TPX) * (N / TROWS));
  hipLaunchKernelGGL(k_conv12_act, dim3(conv_grid(tiles)), dim3(256), 0, c->st, x, c->w1b, c->prm + CnnOffsets::b1,
                     c->w2f, c->prm + CnnOffsets::b2, a2, N, B);
  hipLaunchKernelGGL(k_conv_act, dim3(conv_grid(tiles)), dim3(256), 0, c->st, a2, c->w3f, c->prm + CnnOffsets::b3, a3,
                     N, B);
  hipLaunchKernelGGL(k_conv4_mma, dim3(conv_grid(tiles, kConv4Blocks)), dim3(256), 0, c->st, a3, c->w4b,
                     c->prm + CnnOffsets::b4, z, N, B);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// forward with the network's own workspaces; activations kept for training
int forward(muffin_cnn* c, const float* x, int B, int N) { return forward_into(c, x, B, N, c->a1, c->a2, c->a3, c->z4); }

// ------------------------------------------------------------------ allocation-free inference
// Workspace of muffin_cnn_predict_noalloc: two BF16 activation planes of kNoAllocPixels pixels
// with 32 features each (128 MiB), one copy per GPU, held until the process ends.  Host code
// never uses the array's name as an address: the device address of each GPU's copy is looked up
// once per device (scratch_setup) and kept in scratch_dev.
constexpr long long kNoAllocPixels = 1ll << 20;
__device__ __align__(256) uint16_t scratch[2 * kNoAllocPixels * FC];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
uint16_t* scratch_dev[kMaxDevices] = {};

// with device dev current: record the address of its copy of scratch (once per device)
int scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return set_error("CNN: device index out of range"), MUFFIN_EINVAL;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_dev[dev]) return MUFFIN_OK;
  void* p = nullptr;
  MF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return set_error("CNN: no device address for the inference workspace"), MUFFIN_EHIP;
  scratch_dev[dev] = static_cast<uint16_t*>(p);
  return MUFFIN_OK;
}

uint16_t* scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? scratch_dev[dev] : nullptr;
}

int reduce_into(muffin_cnn* c, int stride, int n, int nblk, float* out, int map) {
  hipLaunchKernelGGL(k_reduce_partials, dim3((n + kRedEntries - 1) / kRedEntries), dim3(256), 0, c->st, c->partial,
                     stride, n, nblk, out, map);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

// loss and gradient (into c->grad) for targets tgt; x is the FP32 input
int loss_grad(muffin_cnn* c, const float* x, const float* tgt, int B, int N, double* loss) {
  const long long P = (long long)B * N * N;
  MF_TRY(forward(c, x, B, N));
  hipLaunchKernelGGL(k_mse, dim3(1024), dim3(256), 0, c->st, c->z4, tgt, c->dz4, c->dpart, P, (float)(2.0 / (double)P));
  MF_TRY(launch_reduce_sum(c->dpart, 1024, c->dres, 0, c->st));
  // layer 4
  hipLaunchKernelGGL(k_wgrad_single<4>, dim3(kSingleBlocks), dim3(256), 0, c->st, c->dz4, c->a3,
                     (const uint16_t*)nullptr, (const float*)nullptr, c->partial, N, P);
  MF_TRY(reduce_into(c, SPART, 9 * FC, kSingleBlocks, c->grad + CnnOffsets::w4, 2));
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, c->st, c->partial + 9 * FC, SPART, 1, kSingleBlocks,
                     c->grad + CnnOffsets::b4, 0);
  hipLaunchKernelGGL(k_conv4_bwd_data, dim3(nb256(P)), dim3(256), 0, c->st, c->dz4, c->w4b, c->a3, c->g3,
                     (float*)nullptr, N, P, 0);
  const unsigned tiles = (unsigned)((long long)B * (N / TPX) * (N / TROWS));
  const long long nseg = (long long)B * N * (N / TPX);
  const unsigned wb = (unsigned)(nseg < kWgradBlocks ? nseg : kWgradBlocks);
  // layer 3
  hipLaunchKernelGGL(k_wgrad_mma, dim3(wb), dim3(192), 0, c->st, c->g3, c->a2, c->partial, N, nseg);
  MF_TRY(reduce_into(c, WPART, WPART, (int)wb, c->grad + CnnOffsets::w3, 1));
  hipLaunchKernelGGL((k_conv_mma<MM_DMASK>), dim3(tiles), dim3(256), 0, c->st, c->g3, c->w3d, (const float*)nullptr,
                     c->a2, c->g2, (float*)nullptr, N, B);
  // layer 2
  hipLaunchKernelGGL(k_wgrad_mma, dim3(wb), dim3(192), 0, c->st, c->g2, c->a1, c->partial, N, nseg);
  MF_TRY(reduce_into(c, WPART, WPART, (int)wb, c->grad + CnnOffsets::w2, 1));
  hipLaunchKernelGGL((k_conv_mma<MM_DMASK>), dim3(tiles), dim3(256), 0, c->st, c->g2, c->w2d, (const float*)nullptr,
                     c->a1, c->g1, (float*)nullptr, N, B);
  // layer 1
  hipLaunchKernelGGL(k_wgrad_single<1>, dim3(kSingleBlocks), dim3(256), 0, c->st, (const float*)nullptr,
                     (const uint16_t*)nullptr, c->g1, x, c->partial, N, P);
  MF_TRY(reduce_into(c, SPART, SPART, kSingleBlocks, c->grad + CnnOffsets::w1, 2));
  MF_HIP(hipGetLastError());
  if (loss) {
    double h = 0;
    MF_HIP(hipMemcpyAsync(&h, c->dres, sizeof(double), hipMemcpyDeviceToHost, c->st));
    MF_HIP(hipStreamSynchronize(c->st));
    *loss = h / (double)P;
  }
  return MUFFIN_OK;
}

// host-side counter-based normal generator (splitmix64 + Box-Muller) for the initial weights
double normal_draw(uint64_t seed, uint64_t i) {
  auto mix = [](uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  };
  const double u1 = ((mix(seed * 0x100000001b3ull + 2 * i) >> 11) + 1.0) / 9007199254740993.0;
  const double u2 = (mix(seed * 0x100000001b3ull + 2 * i + 1) >> 11) / 9007199254740992.0;
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
}

}  // namespace

extern "C" {

int muffin_cnn_create(muffin_cnn** out, int32_t features, uint64_t seed, void* hip_stream) {
  if (!out) return set_error("out is NULL"), MUFFIN_EINVAL;
  *out = nullptr;
  if (features != FC) return set_error("CNN: only 32 feature channels are built"), MUFFIN_EINVAL;
  muffin_cnn* c = new (std::nothrow) muffin_cnn();
  if (!c) return set_error("host allocation failed"), MUFFIN_ENOMEM;
  c->user = (hipStream_t)hip_stream;
  auto fail = [&](int rc) {
    muffin_cnn_free(c);
    return rc;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return fail((set_error("CNN: no current device"), MUFFIN_EHIP));
  if (const int rc0 = scratch_setup(c->device)) return fail(rc0);
  if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
    return fail((set_error("CNN: stream or event creation failed"), MUFFIN_EHIP));
  const int n = CnnOffsets::total;
  int rc = MUFFIN_OK;
  if ((rc = dal(&c->prm, n)) || (rc = dal(&c->grad, n)) || (rc = dal(&c->m, n)) || (rc = dal(&c->v, n)) ||
      (rc = dal(&c->w1b, 9 * FC)) || (rc = dal(&c->w4b, 9 * FC)) || (rc = dal(&c->w2f, 9 * FC * FC)) ||
      (rc = dal(&c->w2d, 9 * FC * FC)) || (rc = dal(&c->w3f, 9 * FC * FC)) || (rc = dal(&c->w3d, 9 * FC * FC)) ||
      (rc = dal(&c->partial, (size_t)kWgradBlocks * WPART)) || (rc = dal(&c->dpart, 1024)) || (rc = dal(&c->dres, 4)))
    return fail(rc);
  // He-normal weights (std sqrt(2 / fan_in)), zero biases
  std::vector<float> h(n, 0.f);
  uint64_t k = 0;
  auto fill = [&](int off, int cnt, int fan_in) {
    const double sd = std::sqrt(2.0 / fan_in);
    for (int i = 0; i < cnt; ++i) h[off + i] = (float)(sd * normal_draw(seed, k++));
  };
  fill(CnnOffsets::w1, 288, 9);
  fill(CnnOffsets::w2, 9216, 288);
  fill(CnnOffsets::w3, 9216, 288);
  fill(CnnOffsets::w4, 288, 288);
  if (hipMemcpy(c->prm, h.data(), sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->m, 0, sizeof(float) * n) != hipSuccess || hipMemset(c->v, 0, sizeof(float) * n) != hipSuccess)
    return fail((set_error("CNN: upload failed"), MUFFIN_EHIP));
  if ((rc = prep_weights(c)) || hipStreamSynchronize(c->st) != hipSuccess) return fail(rc ? rc : MUFFIN_EHIP);
  *out = c;
  return MUFFIN_OK;
}

void muffin_cnn_free(muffin_cnn* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  free_ws(c);
  void* ps[] = {c->prm, c->grad, c->m, c->v, c->w1b, c->w4b, c->w2f, c->w2d, c->w3f, c->w3d, c->partial, c->dpart,
                c->dres};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->st) (void)hipStreamDestroy(c->st);
  delete c;
}

int muffin_cnn_param_count(muffin_cnn* c, int32_t* n) {
  if (!c || !n) return set_error("bad arguments"), MUFFIN_EINVAL;
  *n = CnnOffsets::total;
  return MUFFIN_OK;
}

int muffin_cnn_get_params(muffin_cnn* c, float* params, int32_t n) {
  if (!c || !params || n != CnnOffsets::total) return set_error("bad arguments"), MUFFIN_EINVAL;
  CnnScope s(c);
  MF_HIP(hipMemcpyAsync(params, c->prm, sizeof(float) * n, hipMemcpyDeviceToHost, c->st));
  MF_HIP(hipStreamSynchronize(c->st));
  return MUFFIN_OK;
}

int muffin_cnn_set_params(muffin_cnn* c, const float* params, int32_t n) {
  if (!c || !params || n != CnnOffsets::total) return set_error("bad arguments"), MUFFIN_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return set_error("CNN: non-finite parameter"), MUFFIN_ENONFINITE;
  CnnScope s(c);
  MF_HIP(hipMemcpyAsync(c->prm, params, sizeof(float) * n, hipMemcpyHostToDevice, c->st));
  MF_HIP(hipMemsetAsync(c->m, 0, sizeof(float) * n, c->st));
  MF_HIP(hipMemsetAsync(c->v, 0, sizeof(float) * n, c->st));
  c->t = 0;
  MF_TRY(prep_weights(c));
  MF_HIP(hipStreamSynchronize(c->st));
  return MUFFIN_OK;
}

int muffin_cnn_predict(muffin_cnn* c, const float* in, float* out, int32_t B, int32_t N) {
  if (!c || !in || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  MF_TRY(check_shape(B, N));
  CnnScope s(c);
  const long long n2 = (long long)N * N;
  long long chunk = kChunkPixels / n2;
  if (chunk < 1) chunk = 1;
  if (chunk > B) chunk = B;
  MF_TRY(ensure_ws(c, chunk * n2));
  for (long long b0 = 0; b0 < B; b0 += chunk) {
    const int nb = (int)((B - b0) < chunk ? (B - b0) : chunk);
    MF_TRY(forward_infer(c, in + b0 * n2, nb, N, c->a2, c->a1, out + b0 * n2));
  }
  return MUFFIN_OK;
}

int muffin_cnn_predict_noalloc(muffin_cnn* c, const float* in, float* out, int32_t B, int32_t N) {
  if (!c || !in || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  MF_TRY(check_shape(B, N));
  const long long n2 = (long long)N * N;
  if (n2 > kNoAllocPixels)
    return set_error("CNN: the allocation-free inference takes planes of at most 2^20 pixels (N <= 1024)"),
           MUFFIN_EINVAL;
  uint16_t* ws = scratch_of(c->device);
  if (!ws) return set_error("CNN: inference workspace not set up on this device"), MUFFIN_EHIP;
  uint16_t* a1 = ws;
  uint16_t* a2 = ws + kNoAllocPixels * FC;
  CnnScope s(c);
  const long long chunk = (kNoAllocPixels / n2) < B ? (kNoAllocPixels / n2) : B;
  for (long long b0 = 0; b0 < B; b0 += chunk) {
    const int nb = (int)((B - b0) < chunk ? (B - b0) : chunk);
    MF_TRY(forward_infer(c, in + b0 * n2, nb, N, a2, a1, out + b0 * n2));
  }
  return MUFFIN_OK;
}

int muffin_cnn_loss_grad(muffin_cnn* c, const float* in, const float* target, int32_t B, int32_t N, double* loss,
                         float* grad) {
  if (!c || !in || !target) return set_error("bad arguments"), MUFFIN_EINVAL;
  MF_TRY(check_shape(B, N));
  CnnScope s(c);
  MF_TRY(ensure_ws(c, (long long)B * N * N));
  MF_TRY(loss_grad(c, in, target, B, N, loss));
  if (grad) {
    MF_HIP(hipMemcpyAsync(grad, c->grad, sizeof(float) * CnnOffsets::total, hipMemcpyDeviceToHost, c->st));
    MF_HIP(hipStreamSynchronize(c->st));
  }
  return MUFFIN_OK;
}

int muffin_cnn_train_step(muffin_cnn* c, const float* in, const float* target, int32_t B, int32_t N, float lr,
                          double* loss) {
  if (!c || !in || !target || !(lr > 0)) return set_error("bad arguments"), MUFFIN_EINVAL;
  MF_TRY(check_shape(B, N));
  CnnScope s(c);
  MF_TRY(ensure_ws(c, (long long)B * N * N));
  MF_TRY(loss_grad(c, in, target, B, N, loss));
  c->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)c->t)), c2 = (float)(1.0 - std::pow(0.999, (double)c->t));
  hipLaunchKernelGGL(k_adam, dim3((CnnOffsets::total + 255) / 256), dim3(256), 0, c->st, c->prm, c->grad, c->m, c->v,
                     CnnOffsets::total, lr, b1, b2, 1e-8f, c1, c2);
  MF_HIP(hipGetLastError());
  MF_TRY(prep_weights(c));
  return MUFFIN_OK;
}

int muffin_cnn_layer(muffin_cnn* c, int32_t layer, int32_t op, const float* x, const float* dz, float* out,
                     float* dparams, int32_t B, int32_t N) {
  if (!c || layer < 1 || layer > 4 || (op != 0 && op != 1) || !x || !out) return set_error("bad arguments"), MUFFIN_EINVAL;
  if (op == 1 && (!dz || !dparams)) return set_error("bad arguments"), MUFFIN_EINVAL;
  MF_TRY(check_shape(B, N));
  CnnScope s(c);
  const long long P = (long long)B * N * N, n2 = (long long)N * N;
  MF_TRY(ensure_ws(c, P));
  const int cin = (layer == 1) ? 1 : FC, cout = (layer == 4) ? 1 : FC;
  // stage x: FP32 [B][cin][N][N] -> BF16 NHWC (layers 2-4) or FP32 plane (layer 1)
  std::vector<float> hx((size_t)P * cin);
  MF_HIP(hipMemcpyAsync(hx.data(), x, sizeof(float) * hx.size(), hipMemcpyDeviceToHost, c->st));
  std::vector<float> hdz;
  if (op == 1) {
    hdz.resize((size_t)P * cout);
    MF_HIP(hipMemcpyAsync(hdz.data(), dz, sizeof(float) * hdz.size(), hipMemcpyDeviceToHost, c->st));
  }
  MF_HIP(hipStreamSynchronize(c->st));
  auto to_bf = [](float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  };
  auto nhwc = [&](const std::vector<float>& src) {
    std::vector<uint16_t> d((size_t)P * FC);
    for (long long b = 0; b < B; ++b)
      for (int ch = 0; ch < FC; ++ch)
        for (long long q = 0; q < n2; ++q) d[(size_t)((b * n2 + q) * FC + ch)] = to_bf(src[(size_t)((b * FC + ch) * n2 + q)]);
    return d;
  };
  const unsigned tiles = (unsigned)((long long)B * (N / TPX) * (N / TROWS));
  if (cin == FC) {
    auto v = nhwc(hx);
    MF_HIP(hipMemcpyAsync(c->a2, v.data(), sizeof(uint16_t) * v.size(), hipMemcpyHostToDevice, c->st));
  } else {
    MF_HIP(hipMemcpyAsync(c->xin, hx.data(), sizeof(float) * P, hipMemcpyHostToDevice, c->st));
  }
  if (op == 0) {
    if (layer == 1)
      hipLaunchKernelGGL(k_conv1_mma, dim3(conv_grid(tiles, kConv1Blocks)), dim3(256), 0, c->st, c->xin, c->w1b,
                         c->prm + CnnOffsets::b1, (uint16_t*)nullptr, out, N, B, 1);
    else if (layer == 4)
      hipLaunchKernelGGL(k_conv4_mma, dim3(conv_grid(tiles, kConv4Blocks)), dim3(256), 0, c->st, c->a2, c->w4b,
                         c->prm + CnnOffsets::b4, out, N, B);
    else
      hipLaunchKernelGGL((k_conv_mma<MM_Z>), dim3(tiles), dim3(256), 0, c->st, c->a2, layer == 2 ? c->w2f : c->w3f,
                         c->prm + (layer == 2 ? CnnOffsets::b2 : CnnOffsets::b3), (const uint16_t*)nullptr,
                         (uint16_t*)nullptr, out, N, B);
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(c->st));
    return MUFFIN_OK;
  }
  // backward: dz rounded to BF16; dx without activation mask; parameter gradients to dparams
  const int nw = cout * cin * 9 + cout;
  float* gtmp = c->grad;  // reuse the gradient buffer as scratch
  if (cout == FC) {
    auto v = nhwc(hdz);
    MF_HIP(hipMemcpyAsync(c->g3, v.data(), sizeof(uint16_t) * v.size(), hipMemcpyHostToDevice, c->st));
  } else {
    std::vector<float> r(hdz.size());
    for (size_t i = 0; i < r.size(); ++i) {
      uint32_t u = (uint32_t)to_bf(hdz[i]) << 16;
      std::memcpy(&r[i], &u, 4);
    }
    MF_HIP(hipMemcpyAsync(c->dz4, r.data(), sizeof(float) * P, hipMemcpyHostToDevice, c->st));
  }
  const long long nseg = (long long)B * N * (N / TPX);
  const unsigned wb = (unsigned)(nseg < kWgradBlocks ? nseg : kWgradBlocks);
  if (layer == 4) {
    hipLaunchKernelGGL(k_wgrad_single<4>, dim3(kSingleBlocks), dim3(256), 0, c->st, c->dz4, c->a2,
                       (const uint16_t*)nullptr, (const float*)nullptr, c->partial, N, P);
    MF_TRY(reduce_into(c, SPART, 9 * FC, kSingleBlocks, gtmp, 2));
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, c->st, c->partial + 9 * FC, SPART, 1, kSingleBlocks,
                       gtmp + 9 * FC, 0);
    hipLaunchKernelGGL(k_conv4_bwd_data, dim3(nb256(P)), dim3(256), 0, c->st, c->dz4, c->w4b, (const uint16_t*)nullptr,
                       (uint16_t*)nullptr, out, N, P, 1);
  } else if (layer == 1) {
    hipLaunchKernelGGL(k_wgrad_single<1>, dim3(kSingleBlocks), dim3(256), 0, c->st, (const float*)nullptr,
                       (const uint16_t*)nullptr, c->g3, c->xin, c->partial, N, P);
    MF_TRY(reduce_into(c, SPART, SPART, kSingleBlocks, gtmp, 2));
    MF_HIP(hipMemsetAsync(out, 0, sizeof(float) * P, c->st));  // input gradient of layer 1 is not used
  } else {
    hipLaunchKernelGGL(k_wgrad_mma, dim3(wb), dim3(192), 0, c->st, c->g3, c->a2, c->partial, N, nseg);
    MF_TRY(reduce_into(c, WPART, WPART, (int)wb, gtmp, 1));
    hipLaunchKernelGGL((k_conv_mma<MM_DRAW>), dim3(tiles), dim3(256), 0, c->st, c->g3, layer == 2 ? c->w2d : c->w3d,
                       (const float*)nullptr, (const uint16_t*)nullptr, (uint16_t*)nullptr, out, N, B);
  }
  MF_HIP(hipGetLastError());
  MF_HIP(hipMemcpyAsync(dparams, gtmp, sizeof(float) * nw, hipMemcpyDeviceToHost, c->st));
  MF_HIP(hipStreamSynchronize(c->st));
  return MUFFIN_OK;
}

}  // extern "C"

// Warm start of a reconstruction context: each dirty channel is divided by the sum of its PSF over
// the 9 x 9 window at the PSF origin (the gain of the PSF main lobe over the network's receptive
// field), the network runs, and max(output, 0) becomes X.
namespace mf {
__global__ void __launch_bounds__(256) k_psf_lobe(const float* __restrict__ psf, long long cs,
                                                  float* __restrict__ out, int N, int radius) {
  __shared__ float red[256];
  const int l = blockIdx.x, w = 2 * radius + 1;
  const float* p = psf + (long long)l * cs;
  float s = 0.f;
  for (int i = threadIdx.x; i < w * w; i += 256) {
    const int dy = i / w - radius, dx = i % w - radius;
    s += p[(long long)wrapn(N / 2 + dy, N) * N + wrapn(N / 2 + dx, N)];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[l] = red[0];
}

// The network's inference ordered against another stream (a reconstruction context's): the
// network's stream waits for the work enqueued on ``after`` so far, and ``after`` waits for the
// inference, without synchronising the host.
int cnn_predict_after(muffin_cnn* net, const float* in, float* out, int B, int N, hipStream_t after) {
  hipStream_t saved = net->user;
  net->user = after;
  const int rc = muffin_cnn_predict(net, in, out, B, N);
  net->user = saved;
  return rc;
}

int launch_psf_lobe(const float* psf, long long cs, float* out, int N, int L, int radius, hipStream_t st) {
  hipLaunchKernelGGL(k_psf_lobe, dim3(L), dim3(256), 0, st, psf, cs, out, N, radius);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}

int cnn_warm_input(const float* Y, long long cs, const float* scale, float* out, int N, int L, hipStream_t st) {
  const long long n2 = (long long)N * N;
  hipLaunchKernelGGL(k_scale_planes, dim3(nb256(n2 * L)), dim3(256), 0, st, Y, cs, scale, 1, out, n2, L);
  MF_HIP(hipGetLastError());
  return MUFFIN_OK;
}
}  // namespace mf
