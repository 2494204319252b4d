// Kernels of the convolutional surrogate (C ABI in include/qla_nn.h): BF16
// implicit-GEMM 3x3 circular convolutions on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation), their weight gradients, and
// the elementwise pieces of a U-net step (pooling, upsampling, activation,
// input packing, relative-L2 loss, Adam).
//
// MFMA 32x32x16 operand layout (lane l of the wave): A supplies row l % 32
// and the eight K values 8*(l / 32) .. +7; B supplies column l % 32 and the
// same eight K values; the 16 FP32 results of lane l are column l % 32,
// rows 8*(r / 4) + 4*(l / 32) + r % 4 for r = 0..15.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "qla_nn.h"

extern "C" const char* qla_last_error(void);

namespace qnn {

// the library's per-thread error message (defined with the step ABI)
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr float kLeakySlope = 0.125f;

__host__ __device__ inline float bf2f(uint16_t v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }

// round to nearest even; NaN stays NaN
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<uint16_t>((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

__device__ inline int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Blocks are dealt round-robin to the 8 XCDs (block b to XCD b % 8). The
// pipelined and window convolutions take tiles l, l + n, l + 2n, ... with
// l this function of their block index: each XCD then holds a contiguous
// run of l, so the tiles in flight on one XCD are image neighbours whose
// halo rows its L2 shares. A permutation of 0 .. n-1.
__device__ inline int xcd_band(int b, int n) {
  const int per = n / 8, rem = n % 8, xcd = b % 8, k8 = b / 8;
  return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
}

// ---------------------------------------------------------------------------
// Forward 3x3 circular convolution as an implicit GEMM. A wave computes 32
// pixels x 32*NT output channels; a block is 4 waves along the pixels.
// ---------------------------------------------------------------------------
template <int NT, bool OUT_FP32>
__global__ void __launch_bounds__(256) conv_fwd_kernel(int P, int H, int W, const uint16_t* __restrict__ x,
                                                       int cin, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, int act,
                                                       void* __restrict__ y, int y_ld, int c_store) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m0 = (blockIdx.x * 4 + wave) * 32;
  if (m0 >= P) return;
  const int n0 = blockIdx.y * 32 * NT;
  const int HW = H * W;
  const int p = m0 + (lane & 31);
  const int pc = p < P ? p : P - 1;
  const int b = pc / HW;
  const int rem = pc - b * HW;
  const int yy = rem / W;
  const int xx = rem - yy * W;
  int nb[9];
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
      nb[(dy + 1) * 3 + (dx + 1)] = b * HW + wrapi(yy + dy, H) * W + wrapi(xx + dx, W);
  const int kg = (lane >> 5) * 8;
  const int K = 9 * cin;
  f32x16 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.0f;
  const uint16_t* wl[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) wl[j] = w + static_cast<int64_t>(n0 + j * 32 + (lane & 31)) * K + kg;
#pragma unroll 1
  for (int t = 0; t < 9; ++t) {
    const uint16_t* xr = x + static_cast<int64_t>(nb[t]) * cin + kg;
#pragma unroll 2
    for (int c0 = 0; c0 < cin; c0 += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(xr + c0);
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(wl[j] + t * cin + c0);
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int col = n0 + j * 32 + (lane & 31);
    if (col >= c_store) continue;
    const float bsum = bias ? bias[col] : 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
      if (row >= P) continue;
      float v = acc[j][r] + bsum;
      if (act == QNN_ACT_LEAKY) v = v > 0.0f ? v : kLeakySlope * v;
      if constexpr (OUT_FP32)
        static_cast<float*>(y)[static_cast<int64_t>(row) * y_ld + col] = v;
      else
        static_cast<uint16_t*>(y)[static_cast<int64_t>(row) * y_ld + col] = f2bf(v);
    }
  }
}

// ---------------------------------------------------------------------------
// Forward 3x3 circular convolution, persistent and software-pipelined. A
// block loops over tiles of 128*MT output pixels (TH rows x TW columns of
// one image, TW in {16, 32, 64}) for 32*NT output channels, taking the
// input channels 16 at a time. Each step (tile, chunk) stages in LDS the
// input tile with its one-pixel halo and the chunk's weights (9 taps x
// 32*NT channels x 16), from registers loaded during the previous step's
// MFMAs: apart from a block's first step no wave waits on memory, across
// chunks and across tiles alike. A wave computes 32*MT pixels x 32*NT
// channels; per tap it reads MT A and NT B operands from LDS (16 bytes a
// lane, rows 48 bytes apart, which spreads 16 lanes over all banks) for
// MT*NT MFMAs.
// ---------------------------------------------------------------------------
constexpr int kStageStride = 24;   // LDS elements per staged pixel or weight row (16 + 8 pad)

template <int MT, int NT>
struct PipeConv {
  static constexpr int kPix = 128 * MT;
  static constexpr int kBN = 32 * NT;
  // staged pixels (TH + 2) * (TW + 2), largest over TW in {16, 32, 64}
  static constexpr int kIn16 = (kPix / 16 + 2) * 18;
  static constexpr int kIn32 = (kPix / 32 + 2) * 34;
  static constexpr int kIn64 = (kPix / 64 + 2) * 66;
  static constexpr int kMaxIn = kIn16 > kIn32 ? (kIn16 > kIn64 ? kIn16 : kIn64) : (kIn32 > kIn64 ? kIn32 : kIn64);
  // 16-byte staging pieces per thread (pieces are dealt in groups of 16)
  static constexpr int kInItems = (2 * ((kMaxIn + 7) / 8 * 8) + 255) / 256;
  static constexpr int kWRows = 9 * kBN;
  static constexpr int kWItems = (2 * ((kWRows + 7) / 8 * 8) + 255) / 256;
  // output staging: per wave 32*MT pixels x (32*NT + 8) BF16 (16-byte rows)
  static constexpr int kERow = 32 * NT + 8;
  static constexpr int kStage = (kMaxIn + kWRows) * kStageStride;
  static constexpr int kOut = 4 * 32 * MT * kERow;
  static constexpr int kSmem = kStage > kOut ? kStage : kOut;
};

// The end of a tile in the persistent convolution kernels: bias, activation
// and the store of the block's 128*MT pixels x 32*NT channels from n0 (wave
// w holds tile pixels (w*MT + mt)*32 .. +31), leaving acc zeroed. BF16
// results (every channel stored, 16-byte aligned rows) pass through LDS as
// [pixel][channel] rows from E (which may alias the staged operands: every
// wave is waited for first) and leave as 16 bytes (8 channels of one pixel)
// per lane, plus the skip input when given (`add`, or with ADD_REGS the
// caller's registers add_regs[k] holding piece k of the lane's stores);
// FP32 results pass through E too, 32 pixels of a wave at a time, and only
// channels below c_store are stored.
template <int MT, int NT, bool OUT_FP32, bool ADD_REGS = false, bool POOL = false>
__device__ __forceinline__ void tile_epilogue(f32x16 (&acc)[MT][NT], uint16_t* E0, int tile, int tiles_x, int tiles_y,
                                              int tw_shift, int TH, int H, int W, int n0,
                                              const float* __restrict__ bias, int act, void* __restrict__ y, int y_ld,
                                              int c_store, const uint16_t* __restrict__ add,
                                              const u32x4* add_regs = nullptr, uint16_t* __restrict__ pool = nullptr) {
  constexpr int kERow = 32 * NT + 8;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int TW = 1 << tw_shift;
  const int tx0 = (tile % tiles_x) << tw_shift;
  const int t2 = tile / tiles_x;
  const int ty0 = (t2 % tiles_y) * TH;
  const int b = t2 / tiles_y;
  if constexpr (!OUT_FP32) {
    __syncthreads();    // every wave is done with the staged operands
    uint16_t* const E = E0 + wave * (32 * MT) * kERow;
    const bool leaky = act == QNN_ACT_LEAKY;
#pragma unroll
    for (int jn = 0; jn < NT; ++jn) {
      const int cl = jn * 32 + (lane & 31);
      const float bsum = bias ? bias[n0 + cl] : 0.0f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
          const int m = mt * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);   // rows m, m + 1
          f32x2 v = {acc[mt][jn][r] + bsum, acc[mt][jn][r + 1] + bsum};
          acc[mt][jn][r] = 0.0f;
          acc[mt][jn][r + 1] = 0.0f;
          if (leaky) {
            // the leaky ReLU as max(v, v / 8)
            v[0] = fmaxf(v[0], kLeakySlope * v[0]);
            v[1] = fmaxf(v[1], kLeakySlope * v[1]);
          }
          // round to nearest even (the hardware conversion); the pair is
          // taken apart as one 32-bit word (indexing the BF16 vector
          // itself miscompiles: the second element is lost)
          const uint32_t pk = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
          E[m * kERow + cl] = static_cast<uint16_t>(pk);
          E[(m + 1) * kERow + cl] = static_cast<uint16_t>(pk >> 16);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2 * MT * NT; ++k) {
      const int q = lane + 64 * k;
      const int pm = q / (4 * NT), g = q % (4 * NT);
      const int j = wave * 32 * MT + pm;
      const int oy = ty0 + (j >> tw_shift);
      if (oy < H) {
        const int o = ((b * H + oy) * W + tx0 + (j & (TW - 1))) * y_ld + n0 + g * 8;
        u32x4 v = *reinterpret_cast<const u32x4*>(E + pm * kERow + g * 8);
        if (ADD_REGS || add) {
          // the stored BF16 result plus the skip input, rounded once more
          const u32x4 e = ADD_REGS ? add_regs[k] : *reinterpret_cast<const u32x4*>(add + o);
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const float lo = bf2f(static_cast<uint16_t>(v[h])) + bf2f(static_cast<uint16_t>(e[h]));
            const float hi = bf2f(static_cast<uint16_t>(v[h] >> 16)) + bf2f(static_cast<uint16_t>(e[h] >> 16));
            v[h] = static_cast<uint32_t>(f2bf(lo)) | (static_cast<uint32_t>(f2bf(hi)) << 16);
          }
        }
        *reinterpret_cast<u32x4*>(static_cast<uint16_t*>(y) + o) = v;
      }
    }
    if constexpr (POOL) {
      // 2x2 means of the stored results (no skip input), from the wave's rows
      // of E: the wave's 64 pixels are 64 / TW whole tile rows starting at an
      // even image row, i.e. 16 pooled pixels x 32 NT channels; each lane
      // takes 8 channels of one pooled pixel, summed in the order of
      // qnn_avgpool2 and rounded the same way. Pool rows are y_ld long.
      static_assert(MT == 2, "whole tile rows per wave");
      const int hw = TW >> 1;
      const int r0 = ty0 + ((wave * 64) >> tw_shift);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        const int q = lane + 64 * k;
        const int pp = q / (4 * NT), g = q % (4 * NT);
        const int pr = pp / hw, pc = pp - pr * hw;
        if (r0 + 2 * pr < H) {
          const uint16_t* e = E + (2 * pr * TW + 2 * pc) * kERow + g * 8;
          const u32x4 v00 = *reinterpret_cast<const u32x4*>(e);
          const u32x4 v01 = *reinterpret_cast<const u32x4*>(e + kERow);
          const u32x4 v10 = *reinterpret_cast<const u32x4*>(e + TW * kERow);
          const u32x4 v11 = *reinterpret_cast<const u32x4*>(e + (TW + 1) * kERow);
          float f[8];
#pragma unroll
          for (int h = 0; h < 4; ++h) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              const int sh = 16 * s;
              f[2 * h + s] = 0.25f * (bf2f(static_cast<uint16_t>(v00[h] >> sh)) +
                                      bf2f(static_cast<uint16_t>(v01[h] >> sh)) +
                                      bf2f(static_cast<uint16_t>(v10[h] >> sh)) +
                                      bf2f(static_cast<uint16_t>(v11[h] >> sh)));
            }
          }
          u32x4 o;
#pragma unroll
          for (int h = 0; h < 4; ++h)
            o[h] = static_cast<uint32_t>(f2bf(f[2 * h])) | (static_cast<uint32_t>(f2bf(f[2 * h + 1])) << 16);
          const int64_t po = ((static_cast<int64_t>(b) * (H >> 1) + ((r0 >> 1) + pr)) * (W >> 1) +
                              (tx0 >> 1) + pc) * y_ld + n0 + g * 8;
          *reinterpret_cast<u32x4*>(pool + po) = o;
        }
      }
    }
  } else {
    // FP32 results, one 32-pixel half of the wave's pixels at a time: the
    // wave writes them to its rows of E as [pixel][channel] (rows of 32 NT +
    // 4 floats), then stores the channels n0 .. c_store - 1 of each pixel,
    // consecutive lanes on consecutive elements
    constexpr int kFRow = 32 * NT + 4;
    float* const E = reinterpret_cast<float*>(E0) + wave * 32 * kFRow;
    const int cnt = c_store - n0 < 32 * NT ? c_store - n0 : 32 * NT;   // channels stored (may be <= 0)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      __syncthreads();    // the staged operands, or the previous half's rows, are free
#pragma unroll
      for (int jn = 0; jn < NT; ++jn) {
        const int cl = jn * 32 + (lane & 31);
        const float bsum = (bias && cl < cnt) ? bias[n0 + cl] : 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float v = acc[mt][jn][r] + bsum;
          acc[mt][jn][r] = 0.0f;
          if (act == QNN_ACT_LEAKY) v = v > 0.0f ? v : kLeakySlope * v;
          E[((r >> 2) * 8 + (lane >> 5) * 4 + (r & 3)) * kFRow + cl] = v;
        }
      }
      __syncthreads();
      for (int i = lane; i < 32 * cnt; i += 64) {
        const int pm = i / cnt, c = i - pm * cnt;
        const int j = (wave * MT + mt) * 32 + pm;
        const int oy = ty0 + (j >> tw_shift);
        if (oy < H)
          static_cast<float*>(y)[((b * H + oy) * W + tx0 + (j & (TW - 1))) * y_ld + n0 + c] = E[pm * kFRow + c];
      }
    }
  }
}

// One 32-pixel half (mt) of a wave's results written as scaled FP32 planes
// (see tile_epilogue_planes), leaving a zeroed.
__device__ __forceinline__ void planes_half(f32x16& a, float* E, int mt, int MT, int tx0, int ty0, int b,
                                            int tw_shift, int H, int W, float bsum, int act, float* __restrict__ q,
                                            int nq, float sc) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cl = lane & 31;
  // the accumulators are read from a copy and cleared as one vector (element
  // stores under the branches below put them in scratch memory)
  const f32x16 av = a;
  a = f32x16{};
  __syncthreads();    // the staged operands, or the previous half's rows, are free
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float v = av[r] + bsum;
    if (act == QNN_ACT_LEAKY) v = v > 0.0f ? v : kLeakySlope * v;
    if (cl < nq) E[cl * 33 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3)] = v;
  }
  __syncthreads();
  const int j = (wave * MT + mt) * 32 + cl;
  const int oy = ty0 + (j >> tw_shift);
  if (oy < H) {
    const int64_t pix = static_cast<int64_t>(oy) * W + tx0 + (j & ((1 << tw_shift) - 1));
    for (int c = lane >> 5; c < nq; c += 2)
      q[(static_cast<int64_t>(b) * nq + c) * H * W + pix] = E[c * 33 + cl] * sc;
  }
}

// The end of a tile for results written as per-sample scaled FP32 planes
// (32 output channels, n0 = 0): q[(b * nq + c) * H * W + pixel] = scale[b] *
// act(bias + acc) for channels c < nq, leaving acc zeroed. Each half of a
// wave's pixels passes through LDS as [channel][pixel] (rows of 33 floats
// from E0), and each lane then stores one pixel of a plane: consecutive
// lanes on consecutive pixels of one image row (TW >= 32: a half is one
// row segment; TW = 16: two).
template <int MT>
__device__ __forceinline__ void tile_epilogue_planes(f32x16 (&acc)[MT][1], uint16_t* E0, int tile, int tiles_x,
                                                     int tiles_y, int tw_shift, int TH, int H, int W,
                                                     const float* __restrict__ bias, int act,
                                                     float* __restrict__ q, int nq,
                                                     const float* __restrict__ scale) {
  static_assert(MT == 1 || MT == 2, "one or two halves");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tx0 = (tile % tiles_x) << tw_shift;
  const int t2 = tile / tiles_x;
  const int ty0 = (t2 % tiles_y) * TH;
  const int b = t2 / tiles_y;
  const float sc = scale[b];
  float* const E = reinterpret_cast<float*>(E0) + wave * 32 * 33;
  const int cl = lane & 31;
  const float bsum = (bias && cl < nq) ? bias[cl] : 0.0f;
  planes_half(acc[0][0], E, 0, MT, tx0, ty0, b, tw_shift, H, W, bsum, act, q, nq, sc);
  if constexpr (MT == 2) planes_half(acc[1][0], E, 1, MT, tx0, ty0, b, tw_shift, H, W, bsum, act, q, nq, sc);
}

template <int MT, int NT, bool OUT_FP32>
__global__ void __launch_bounds__(256) conv_fwd_pipe_kernel(int H, int W, int tw_shift, int tiles,
                                                            const uint16_t* __restrict__ x, int cin,
                                                            const uint16_t* __restrict__ w,
                                                            const float* __restrict__ bias, int act,
                                                            void* __restrict__ y, int y_ld, int c_store, int up,
                                                            const uint16_t* __restrict__ add) {
  using PC = PipeConv<MT, NT>;
  // staged input tile and weights; at the end of a tile, the waves' outputs
  __shared__ __attribute__((aligned(16))) uint16_t smem[PC::kSmem];
  static_assert(PC::kSmem >= 4 * 32 * (32 * NT + 4) * 2, "FP32 epilogue rows exceed the staging area");
  uint16_t* const lin = smem;
  uint16_t* const lw = smem + PC::kMaxIn * kStageStride;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int TW = 1 << tw_shift;
  const int TH = PC::kPix >> tw_shift;
  const int TWp = TW + 2;
  const int nstaged = (TH + 2) * TWp;
  const int tiles_x = W >> tw_shift;
  const int tiles_y = (H + TH - 1) / TH;
  const int n0 = blockIdx.y * PC::kBN;
  const int K = 9 * cin;
  const int nchunks = cin >> 4;
  const int kh = (lane >> 5) * 8;
  const bool tall = TH > H;    // rows of a tile may wrap more than once

  // this thread's staging pieces, fixed for the whole kernel. Piece i is
  // half (i / 8) % 2 (8 channels) of staged row 8 (i / 16) + i % 8, so that
  // eight consecutive lanes write eight rows 48 bytes apart (all banks).
  // Input rows are the staged pixels, packed as tile row << 16 | column << 1
  // | half; weight rows are (output channel, tap) pairs, channel-major, the
  // order of the weights in memory. A negative LDS offset marks a piece past
  // the end.
  int in_p[PC::kInItems], in_d[PC::kInItems];
#pragma unroll
  for (int k = 0; k < PC::kInItems; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int pi = (i >> 4) * 8 + (i & 7), half = (i >> 3) & 1;
    const int r = pi / TWp;
    in_p[k] = (r << 16) | ((pi - r * TWp) << 1) | half;
    in_d[k] = pi < nstaged ? pi * kStageStride + half * 8 : -1;
  }
  int w_s[PC::kWItems], w_d[PC::kWItems];
#pragma unroll
  for (int k = 0; k < PC::kWItems; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int row = (i >> 4) * 8 + (i & 7), half = (i >> 3) & 1;
    const int co = row / 9, tap = row - co * 9;
    w_d[k] = row < PC::kWRows ? row * kStageStride + half * 8 : -1;
    w_s[k] = (n0 + co) * K + tap * cin + half * 8;
  }
  // this lane's A rows (tile pixels), as staged-tile offsets of tap (0, 0)
  int a_off[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int j = (wave * MT + mt) * 32 + (lane & 31);
    a_off[mt] = ((j >> tw_shift) * TWp + (j & (TW - 1))) * kStageStride + kh;
  }
  // this lane's B row: output channel lane % 32 of each 32-channel group
  const int b_off = (lane & 31) * 9 * kStageStride + kh;

  u32x4 sin[PC::kInItems], swt[PC::kWItems];
#define QNN_PIPE_FETCH(T, CH)                                                                       \
  {                                                                                                 \
    const int tx0_ = ((T) % tiles_x) << tw_shift;                                                   \
    const int t2_ = (T) / tiles_x;                                                                  \
    const int ty0_ = (t2_ % tiles_y) * TH;                                                          \
    const int img_ = (t2_ / tiles_y) * (H >> up);                                                  \
    _Pragma("unroll") for (int k = 0; k < PC::kInItems; ++k) {                                      \
      if (in_d[k] >= 0) {                                                                           \
        /* periodic; with tiles taller than the image, rows may lie several H past the end */    \
        int yy = ty0_ - 1 + (in_p[k] >> 16);                                                        \
        if (tall)                                                                                   \
          yy = (yy + H) % H;                                                                        \
        else                                                                                        \
          yy = yy < 0 ? yy + H : (yy >= H ? yy - H : yy);                                           \
        int xx = tx0_ - 1 + ((in_p[k] >> 1) & 0x7fff);                                              \
        xx = xx < 0 ? xx + W : (xx >= W ? xx - W : xx);                                             \
        /* an upsampled input is read at (yy / 2, xx / 2) of the half-size */                     \
        /* image; element offsets fit 31 bits (checked on the host) */                             \
        const int src = ((img_ + (yy >> up)) * (W >> up) + (xx >> up)) * cin + (CH) * 16 + (in_p[k] & 1) * 8; \
        sin[k] = *reinterpret_cast<const u32x4*>(x + src);                                          \
      }                                                                                             \
    }                                                                                               \
    _Pragma("unroll") for (int k = 0; k < PC::kWItems; ++k) {                                       \
      if (w_d[k] >= 0) swt[k] = *reinterpret_cast<const u32x4*>(w + w_s[k] + (CH) * 16);            \
    }                                                                                               \
  }

  f32x16 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int jn = 0; jn < NT; ++jn)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mt][jn][r] = 0.0f;

  const int first = xcd_band(blockIdx.x, gridDim.x);
  const int my_tiles = (tiles - 1 - first) / static_cast<int>(gridDim.x) + 1;
  const int steps = my_tiles * nchunks;
  int tile = first, chunk = 0;
  QNN_PIPE_FETCH(tile, chunk)
  for (int s = 0; s < steps; ++s) {
    __syncthreads();      // every wave is done with the previous step's LDS
#pragma unroll
    for (int k = 0; k < PC::kInItems; ++k)
      if (in_d[k] >= 0) *reinterpret_cast<u32x4*>(lin + in_d[k]) = sin[k];
#pragma unroll
    for (int k = 0; k < PC::kWItems; ++k)
      if (w_d[k] >= 0) *reinterpret_cast<u32x4*>(lw + w_d[k]) = swt[k];
    __syncthreads();
    int ntile = tile, nchunk = chunk + 1;
    if (nchunk == nchunks) {
      nchunk = 0;
      ntile += gridDim.x;
    }
    if (s + 1 < steps) QNN_PIPE_FETCH(ntile, nchunk)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;   // offsets +1 into the staged tile
      bf16x8 a[MT], bv[NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        a[mt] = *reinterpret_cast<const bf16x8*>(lin + a_off[mt] + (dy * TWp + dx) * kStageStride);
#pragma unroll
      for (int jn = 0; jn < NT; ++jn)
        bv[jn] = *reinterpret_cast<const bf16x8*>(lw + (jn * 32 * 9 + tap) * kStageStride + b_off);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int jn = 0; jn < NT; ++jn)
          acc[mt][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], bv[jn], acc[mt][jn], 0, 0, 0);
    }
    if (chunk == nchunks - 1)
      tile_epilogue<MT, NT, OUT_FP32>(acc, smem, tile, tiles_x, tiles_y, tw_shift, TH, H, W, n0, bias, act, y, y_ld,
                                      c_store, add);
    tile = ntile;
    chunk = nchunk;
  }
}
#undef QNN_PIPE_FETCH

// ---------------------------------------------------------------------------
// Forward 3x3 circular convolution with resident weights, for the layers
// whose weights fit in LDS beside one tile: 16*KC input channels (KC in
// {2, 3, 4}), 32*NT output channels a block (NT in {1, 2}), tiles of 256
// pixels (TH x TW, TW in {16, 32}). The block's weights are staged once and
// stay; each step stages a whole tile with all its input channels, loaded
// into registers during the previous tile's MFMAs. The only memory traffic
// of a step is then the tile itself, in one batch of loads two to four
// times as large as a step of the pipelined kernel has in flight, with a
// fraction of its barriers: these layers are bound by the bytes a CU keeps
// in flight, not by the matrix cores. The MFMAs run in the pipelined
// kernel's order (16-channel chunks outer, taps inner), so the results are
// bitwise the same.
// ---------------------------------------------------------------------------
template <int KC, int NT>
struct ResConv {
  static constexpr int kCin = 16 * KC;
  static constexpr int kParts = 2 * KC;              // 16-byte pieces per staged row
  static constexpr int kRow = 16 * KC + 8;           // LDS elements per row: an odd multiple of 16 bytes
  // pieces are dealt to lanes in groups of kGroup rows x 2 pieces (KC = 3) or
  // kGroup rows x 1 piece, which puts every eight consecutive lanes on eight
  // distinct 16-byte bank groups
  static constexpr int kGroup = KC == 3 ? 4 : 8;
  static constexpr int kMaxIn = 10 * 34;             // staged pixels for TW = 32 (TW = 16: 18 * 18)
  static constexpr int kInItems = ((kMaxIn + kGroup - 1) / kGroup * kGroup * kParts + 255) / 256;
  static constexpr int kWRows = 9 * 32 * NT;
  static constexpr int kIn = kMaxIn * kRow;
  static constexpr int kOut = 4 * 64 * (32 * NT + 8);   // the epilogue's [pixel][channel] rows
  static constexpr int kSmem = kWRows * kRow + (kIn > kOut ? kIn : kOut);
};

template <int KC, int NT, bool OUT_FP32, bool PLANES = false, bool POOL = false>
__global__ void __launch_bounds__(256) conv_fwd_res_kernel(int H, int W, int tw_shift, int tiles,
                                                           const uint16_t* __restrict__ x,
                                                           const uint16_t* __restrict__ w,
                                                           const float* __restrict__ bias, int act,
                                                           void* __restrict__ y, int y_ld, int c_store,
                                                           const uint16_t* __restrict__ add,
                                                           const float* __restrict__ scale,
                                                           uint16_t* __restrict__ pool) {
  static_assert(!PLANES || (NT == 1 && OUT_FP32), "planes: 32 output channels, FP32");
  static_assert(!POOL || !OUT_FP32, "pooling: BF16 results");
  using RC = ResConv<KC, NT>;
  constexpr int cin = RC::kCin;
  __shared__ __attribute__((aligned(16))) uint16_t smem[RC::kSmem];
  uint16_t* const lw = smem;                         // [co * 9 + tap][cin], resident
  uint16_t* const lin = smem + RC::kWRows * RC::kRow;   // staged tile; then the epilogue's rows
  static_assert(RC::kSmem - RC::kWRows * RC::kRow >= 4 * 32 * (32 * NT + 4) * 2,
                "FP32 epilogue rows exceed the staging area");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int TW = 1 << tw_shift;
  const int TH = 256 >> tw_shift;
  const int TWp = TW + 2;
  const int nstaged = (TH + 2) * TWp;
  const int tiles_x = W >> tw_shift;
  const int tiles_y = (H + TH - 1) / TH;
  const int n0 = blockIdx.y * 32 * NT;
  const int kh = (lane >> 5) * 8;
  const bool tall = TH > H;    // rows of a tile may wrap more than once

  // this thread's staging pieces, fixed for the whole kernel: piece i is
  // part (i / G) % parts of staged row G (i / (G parts)) + i % G (G rows per
  // group; with KC = 3 the parts pair up within eight lanes), packed as tile
  // row << 16 | column << 4 | part; a negative LDS offset marks a piece past
  // the end
  int in_p[RC::kInItems], in_d[RC::kInItems];
#pragma unroll
  for (int k = 0; k < RC::kInItems; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int pi = (i / (RC::kGroup * RC::kParts)) * RC::kGroup + i % RC::kGroup;
    const int part = (i / RC::kGroup) % RC::kParts;
    const int r = pi / TWp;
    in_p[k] = (r << 16) | ((pi - r * TWp) << 4) | part;
    in_d[k] = pi < nstaged ? pi * RC::kRow + part * 8 : -1;
  }
  // this lane's A rows (tile pixels 64 * wave + 32 * mt + lane % 32) and B
  // row (output channel lane % 32 of each 32-channel group)
  int a_off[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int j = (wave * 2 + mt) * 32 + (lane & 31);
    a_off[mt] = ((j >> tw_shift) * TWp + (j & (TW - 1))) * RC::kRow + kh;
  }
  const int b_off = (lane & 31) * 9 * RC::kRow + kh;

  u32x4 sin[RC::kInItems];
  auto fetch = [&](int t) {
    const int tx0 = (t % tiles_x) << tw_shift;
    const int t2 = t / tiles_x;
    const int ty0 = (t2 % tiles_y) * TH;
    const int img = (t2 / tiles_y) * H;
#pragma unroll
    for (int k = 0; k < RC::kInItems; ++k) {
      if (in_d[k] >= 0) {
        int yy = ty0 - 1 + (in_p[k] >> 16);
        if (tall)
          yy = (yy + H) % H;
        else
          yy = yy < 0 ? yy + H : (yy >= H ? yy - H : yy);
        int xx = tx0 - 1 + ((in_p[k] >> 4) & 0xfff);
        xx = xx < 0 ? xx + W : (xx >= W ? xx - W : xx);
        // element offsets fit 31 bits (checked on the host)
        sin[k] = *reinterpret_cast<const u32x4*>(x + ((img + yy) * W + xx) * cin + (in_p[k] & 15) * 8);
      }
    }
  };

  // (round-robin tiles: an XCD-banded order measured 1-4 % slower here)
  int tile = blockIdx.x;   // the grid never exceeds the tile count
  fetch(tile);
  // the block's weights, rows (co, tap) contiguous in memory
  for (int i = threadIdx.x; i < RC::kWRows * RC::kParts; i += 256) {
    const int row = i / RC::kParts, part = i - row * RC::kParts;
    *reinterpret_cast<u32x4*>(lw + row * RC::kRow + part * 8) =
        *reinterpret_cast<const u32x4*>(w + (n0 * 9 + row) * cin + part * 8);
  }
  f32x16 acc[2][NT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int jn = 0; jn < NT; ++jn)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mt][jn][r] = 0.0f;

  for (; tile < tiles; tile += gridDim.x) {
    __syncthreads();      // every wave is done with the previous tile's LDS
#pragma unroll
    for (int k = 0; k < RC::kInItems; ++k)
      if (in_d[k] >= 0) *reinterpret_cast<u32x4*>(lin + in_d[k]) = sin[k];
    __syncthreads();
    if (tile + static_cast<int>(gridDim.x) < tiles) fetch(tile + gridDim.x);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;   // offsets +1 into the staged tile
        bf16x8 a[2], bv[NT];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          a[mt] = *reinterpret_cast<const bf16x8*>(lin + a_off[mt] + (dy * TWp + dx) * RC::kRow + kc * 16);
#pragma unroll
        for (int jn = 0; jn < NT; ++jn)
          bv[jn] = *reinterpret_cast<const bf16x8*>(lw + b_off + (jn * 32 * 9 + tap) * RC::kRow + kc * 16);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int jn = 0; jn < NT; ++jn)
            acc[mt][jn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], bv[jn], acc[mt][jn], 0, 0, 0);
      }
    }
    if constexpr (PLANES)
      tile_epilogue_planes<2>(acc, lin, tile, tiles_x, tiles_y, tw_shift, TH, H, W, bias, act,
                              static_cast<float*>(y), c_store, scale);
    else
      tile_epilogue<2, NT, OUT_FP32, false, POOL>(acc, lin, tile, tiles_x, tiles_y, tw_shift, TH, H, W, n0, bias, act,
                                                  y, y_ld, c_store, add, nullptr, pool);
  }
}

// ---------------------------------------------------------------------------
// Forward 3x3 circular convolution of a nearest-neighbour upsampled input,
// plus an optional skip input: y = act(bias + conv3x3(up2(x), w)) + add, for
// 16*KC input channels (x at half resolution; KC in {4, 8}) and 32 output
// channels a block, tiles of 256 output pixels (TH x TW, TW in {16, 32}).
// Tile rows and columns start at even coordinates, so the tile reads the
// fixed half-resolution window (TH/2 + 2) x (TW/2 + 2), staged once per
// tile instead of once per output pixel it feeds (a quarter of the bytes);
// the tap offsets into that window depend on the lane only. The weights
// stay in LDS, and each step loads the next tile's window and skip input
// into registers during the current tile's MFMAs, the skip input in the
// pieces the epilogue stores. Bitwise the same as the pipelined kernel
// with the upsampling folded in (same MFMA operands, same order).
// ---------------------------------------------------------------------------
template <int KC>
struct UpConv {
  static constexpr int kCin = 16 * KC;
  static constexpr int kParts = 2 * KC;                // 16-byte pieces per staged row
  static constexpr int kRow = kCin + 8;                // an odd multiple of 16 bytes
  static constexpr int kMaxIn = 6 * 18;                // TW = 32: 6 x 18 (TW = 16: 10 x 10)
  static constexpr int kInItems = ((kMaxIn + 7) / 8 * 8 * kParts + 255) / 256;
  static constexpr int kWRows = 9 * 32;
  static constexpr int kIn = kMaxIn * kRow;
  static constexpr int kOut = 4 * 64 * 40;
  static constexpr int kSmem = kWRows * kRow + (kIn > kOut ? kIn : kOut);
};

template <int KC, bool ADD>
__global__ void __launch_bounds__(256) conv_fwd_up_kernel(int H, int W, int tw_shift, int tiles,
                                                          const uint16_t* __restrict__ x,
                                                          const uint16_t* __restrict__ w,
                                                          const float* __restrict__ bias, int act,
                                                          uint16_t* __restrict__ y, int y_ld,
                                                          const uint16_t* __restrict__ add) {
  using UC = UpConv<KC>;
  constexpr int cin = UC::kCin;
  __shared__ __attribute__((aligned(16))) uint16_t smem[UC::kSmem];
  uint16_t* const lw = smem;                           // [co * 9 + tap][cin], resident
  uint16_t* const lin = smem + UC::kWRows * UC::kRow;  // staged window; then the epilogue's rows
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int TW = 1 << tw_shift;
  const int TH = 256 >> tw_shift;
  const int Hh = H >> 1, Wh = W >> 1;                  // the input's size
  const int SW = TW / 2 + 2;                           // staged window: (TH/2 + 2) x SW
  const int nstaged = (TH / 2 + 2) * SW;
  const int tiles_x = W >> tw_shift;
  const int tiles_y = (H + TH - 1) / TH;
  const int n0 = blockIdx.y * 32;
  const int kh = (lane >> 5) * 8;
  const bool tall = TH / 2 + 2 > Hh;   // window rows may wrap more than once

  // staging pieces: piece i is part (i / 8) % parts of window row
  // 8 (i / (8 parts)) + i % 8 (eight consecutive lanes on eight rows an odd
  // number of 16-byte units apart: distinct bank groups), packed as row << 16
  // | column << 4 | part
  int in_p[UC::kInItems], in_d[UC::kInItems];
#pragma unroll
  for (int k = 0; k < UC::kInItems; ++k) {
    const int i = threadIdx.x + 256 * k;
    const int pi = (i / (8 * UC::kParts)) * 8 + (i & 7), part = (i >> 3) % UC::kParts;
    const int r = pi / SW;
    in_p[k] = (r << 16) | ((pi - r * SW) << 4) | part;
    in_d[k] = pi < nstaged ? pi * UC::kRow + part * 8 : -1;
  }
  // this lane's A rows: tile pixel (r, c) reads, for tap (dy, dx), the
  // window element (((r + dy) >> 1) + 1, ((c + dx) >> 1) + 1)
  int a_row[2][3], a_col[2][3];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int j = (wave * 2 + mt) * 32 + (lane & 31);
    const int r = j >> tw_shift, c = j & (TW - 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a_row[mt][d] = (((r + d - 1) >> 1) + 1) * SW * UC::kRow;
      a_col[mt][d] = (((c + d - 1) >> 1) + 1) * UC::kRow + kh;
    }
  }
  const int b_off = (lane & 31) * 9 * UC::kRow + kh;

  u32x4 sin[UC::kInItems];
  u32x4 sadd[ADD ? 4 : 1];
  auto fetch = [&](int t) {
    const int tx0 = (t % tiles_x) << tw_shift;
    const int t2 = t / tiles_x;
    const int ty0 = (t2 % tiles_y) * TH;
    const int b = t2 / tiles_y;
#pragma unroll
    for (int k = 0; k < UC::kInItems; ++k) {
      if (in_d[k] >= 0) {
        int hy = (ty0 >> 1) - 1 + (in_p[k] >> 16);
        if (tall)
          hy = (hy + Hh) % Hh;
        else
          hy = hy < 0 ? hy + Hh : (hy >= Hh ? hy - Hh : hy);
        int hx = (tx0 >> 1) - 1 + ((in_p[k] >> 4) & 0xfff);
        hx = hx < 0 ? hx + Wh : (hx >= Wh ? hx - Wh : hx);
        // element offsets fit 31 bits (checked on the host)
        sin[k] = *reinterpret_cast<const u32x4*>(x + ((b * Hh + hy) * Wh + hx) * cin + (in_p[k] & 15) * 8);
      }
    }
    if constexpr (ADD) {
      // the skip input in the epilogue's store pieces: piece k of a lane is
      // channels 8 (q % 4) .. +7 of tile pixel 64 wave + q / 4, q = lane + 64 k
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q = lane + 64 * k;
        const int j = wave * 64 + (q >> 2);
        const int oy = ty0 + (j >> tw_shift);
        if (oy < H)
          sadd[k] = *reinterpret_cast<const u32x4*>(
              add + ((b * H + oy) * W + tx0 + (j & (TW - 1))) * y_ld + n0 + (q & 3) * 8);
      }
    }
  };

  int tile = xcd_band(blockIdx.x, gridDim.x);   // the grid never exceeds the tile count
  fetch(tile);
  for (int i = threadIdx.x; i < UC::kWRows * UC::kParts; i += 256) {
    const int row = i / UC::kParts, part = i - row * UC::kParts;
    *reinterpret_cast<u32x4*>(lw + row * UC::kRow + part * 8) =
        *reinterpret_cast<const u32x4*>(w + (n0 * 9 + row) * cin + part * 8);
  }
  f32x16 acc[2][1];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[mt][0][r] = 0.0f;

  for (; tile < tiles; tile += gridDim.x) {
    __syncthreads();      // every wave is done with the previous tile's LDS
#pragma unroll
    for (int k = 0; k < UC::kInItems; ++k)
      if (in_d[k] >= 0) *reinterpret_cast<u32x4*>(lin + in_d[k]) = sin[k];
    u32x4 cadd[ADD ? 4 : 1];
    if constexpr (ADD) {
#pragma unroll
      for (int k = 0; k < 4; ++k) cadd[k] = sadd[k];
    }
    __syncthreads();
    if (tile + static_cast<int>(gridDim.x) < tiles) fetch(tile + gridDim.x);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
        bf16x8 a[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          a[mt] = *reinterpret_cast<const bf16x8*>(lin + a_row[mt][dy] + a_col[mt][dx] + kc * 16);
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(lw + b_off + tap * UC::kRow + kc * 16);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
          acc[mt][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mt], bv, acc[mt][0], 0, 0, 0);
      }
    }
    // (BF16 results store every channel: no c_store)
    tile_epilogue<2, 1, false, ADD>(acc, lin, tile, tiles_x, tiles_y, tw_shift, TH, H, W, n0, bias, act, y, y_ld, 0,
                                    nullptr, cadd);
  }
}

__global__ void flip_kernel(const uint16_t* __restrict__ w, int cout, int cin, uint16_t* __restrict__ wt) {
  const int64_t n = static_cast<int64_t>(cout) * 9 * cin;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int ci = static_cast<int>(i % cin);
    const int t = static_cast<int>((i / cin) % 9);
    const int co = static_cast<int>(i / (9 * static_cast<int64_t>(cin)));
    wt[(static_cast<int64_t>(ci) * 9 + (8 - t)) * cout + co] = w[i];
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[co][k] = sum_p dy[p][co] * x[nbr(p, t)][ci], k = t*cin+ci,
// an MFMA GEMM (M = c_out, N = 9*c_in, K = pixels). A block (4 waves) owns a
// 32x32 tile of dW and a range of pixels; waves take interleaved 16-pixel
// chunks (each within one image row, W % 16 == 0), then fold through LDS.
// ---------------------------------------------------------------------------
constexpr int kWgradPixelsPerBlock = 4096;

// ROWS: W % 16 == 0, so a 16-pixel chunk lies in one image row and its
// neighbours are found once per chunk; otherwise every pixel is decoded
// (and bounds-checked) on its own.
template <bool ROWS>
__global__ void __launch_bounds__(256) wgrad_kernel(int P, int H, int W, const uint16_t* __restrict__ x,
                                                    int cin, const uint16_t* __restrict__ dy,
                                                    int cout, float* __restrict__ part,
                                                    float* __restrict__ bpart) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int co0 = blockIdx.x * 32;
  const int k0 = blockIdx.y * 32;
  const int split = blockIdx.z;
  const int K = 9 * cin;
  const int HW = H * W;
  // columns past 9*c_in (when it is not a multiple of 32) compute zeros and
  // are not stored
  const bool kvalid = k0 + (lane & 31) < K;
  const int kk = kvalid ? k0 + (lane & 31) : K - 1;
  const int t = kk / cin;
  const int ci = kk - t * cin;
  const int tdy = t / 3 - 1, tdx = t % 3 - 1;
  const int co = co0 + (lane & 31);
  const int half = (lane >> 5) * 8;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  float bsum = 0.0f;
  const int pbeg = split * kWgradPixelsPerBlock;
  const int pend = min(P, pbeg + kWgradPixelsPerBlock);
  for (int p0 = pbeg + wave * 16; p0 < pend; p0 += 64) {
    bf16x8 a, bb;
    if constexpr (ROWS) {
      // the chunk's row: image b, row yy, columns xb .. xb+15
      const int b = p0 / HW;
      const int rem = p0 - b * HW;
      const int yy = rem / W;
      const int xb = rem - yy * W;
      const int ysrc = wrapi(yy + tdy, H);
      const int64_t rowbase = static_cast<int64_t>(b) * HW + static_cast<int64_t>(ysrc) * W;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint16_t dv = dy[static_cast<int64_t>(p0 + half + j) * cout + co];
        bsum += bf2f(dv);
        a[j] = __builtin_bit_cast(__bf16, dv);
        const int xs = wrapi(xb + half + j + tdx, W);
        const uint16_t xv = x[(rowbase + xs) * cin + ci];
        bb[j] = __builtin_bit_cast(__bf16, kvalid ? xv : static_cast<uint16_t>(0));
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int pp = p0 + half + j;
        uint16_t dv = 0, xv = 0;
        if (pp < pend) {
          dv = dy[static_cast<int64_t>(pp) * cout + co];
          const int b = pp / HW;
          const int rem = pp - b * HW;
          const int yy = rem / W;
          const int xx = rem - yy * W;
          const int64_t src = static_cast<int64_t>(b) * HW + static_cast<int64_t>(wrapi(yy + tdy, H)) * W +
                              wrapi(xx + tdx, W);
          if (kvalid) xv = x[src * cin + ci];
        }
        bsum += bf2f(dv);
        a[j] = __builtin_bit_cast(__bf16, dv);
        bb[j] = __builtin_bit_cast(__bf16, xv);
      }
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
  }
  // fold the four waves
  __shared__ float sh[4][16][64];
  __shared__ float shb[4][64];
#pragma unroll
  for (int r = 0; r < 16; ++r) sh[wave][r][lane] = acc[r];
  shb[wave][lane] = bsum;
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v = sh[0][r][lane] + sh[1][r][lane] + sh[2][r][lane] + sh[3][r][lane];
      const int row = (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);     // co within the tile
      if (kvalid) part[(static_cast<int64_t>(split) * cout + co0 + row) * K + k0 + (lane & 31)] = v;
    }
    if (bpart && blockIdx.y == 0 && lane < 32) {
      const float v = shb[0][lane] + shb[1][lane] + shb[2][lane] + shb[3][lane] +
                      shb[0][lane + 32] + shb[1][lane + 32] + shb[2][lane + 32] + shb[3][lane + 32];
      bpart[static_cast<int64_t>(split) * cout + co0 + lane] = v;
    }
  }
}

// Weight gradient, staged: a block owns 32*A output channels x 128 columns k
// of dW (per wave A 32 x 32 MFMA tiles sharing one B operand) and a range of
// pixels, taken 128 at a time. Each thread loads a group of 8 pixels x 8
// channels of dy or of the tap-shifted input (eight 16-byte loads), turns it
// into 8 channels x 8 pixels with byte permutes, and writes it to LDS as 16-
// byte rows, pixel index fastest, so that every MFMA operand (eight
// consecutive pixels of one channel or column) is one 16-byte LDS read. The
// next chunk's loads are in flight during the current chunk's MFMAs. Needs
// 16-byte aligned x and dy and W % 8 == 0 (a group then lies in one image
// row); the block's pixel range is a multiple of 128.
constexpr int kWtChunk = 128;                 // pixels per staged chunk
constexpr int kWtStride = kWtChunk + 8;       // LDS row stride (elements): rows 272 bytes apart

template <int A>
__global__ void __launch_bounds__(256) wgrad_lds_kernel(int P, int H, int W, const uint16_t* __restrict__ x,
                                                        int cin, const uint16_t* __restrict__ dy, int cout,
                                                        int pps, float* __restrict__ part,
                                                        float* __restrict__ bpart) {
  __shared__ __attribute__((aligned(16))) uint16_t dyT[32 * A * kWtStride];
  __shared__ __attribute__((aligned(16))) uint16_t xT[128 * kWtStride];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tid = threadIdx.x;
  // Blocks are dealt round-robin to the 8 XCDs. Regroup them so that each
  // XCD takes a contiguous run of (channel block, column block, pixel range)
  // triples, pixel range slowest: the blocks that read the same pixels for
  // other taps and channels then run on the same XCD and share its L2.
  const int ncx = gridDim.x, ncy = gridDim.y;
  const int nblk = ncx * ncy * static_cast<int>(gridDim.z);
  const int id = blockIdx.x + ncx * (blockIdx.y + ncy * blockIdx.z);
  const int per = nblk / 8, rem = nblk % 8, xcd = id % 8, k8 = id / 8;
  const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
  const int bx = logical % ncx, by = (logical / ncx) % ncy;
  const int co0 = bx * 32 * A;
  const int kb0 = by * 128;
  const int split = logical / (ncx * ncy);
  const int K = 9 * cin;
  const int pbeg = split * pps;
  const int pend = min(P, pbeg + pps);
  const int half = (lane >> 5) * 8;
  // this thread's groups: pixels 8 pg .. 8 pg + 7 of every chunk; input
  // columns kb0 + 8 kc .. + 7 (one tap, 8 channels); for the first 64 A
  // threads also dy channels co0 + 8 kc .. + 7
  const int pg = tid & 15, kc = tid >> 4;
  const int k = kb0 + 8 * kc;
  const bool kvalid = k < K;
  const int tap = kvalid ? k / cin : 0;
  const int ci = k - tap * cin;
  const int ty = tap / 3 - 1, tx = tap % 3 - 1;
  const bool dgrp = tid < 64 * A;
  // image, row and column of the group's first pixel in the next chunk
  int gb, gy, gx;
  {
    const int p = pbeg + 8 * pg;
    const int HW = H * W;
    gb = p / HW;
    gy = (p - gb * HW) / W;
    gx = p - gb * HW - gy * W;
  }
  u32x4 xr[8], dr[8];
  auto fetch = [&](int pc) {
    const int p = pc + 8 * pg;
    const bool live = p < pend;
#pragma unroll
    for (int i = 0; i < 8; ++i) xr[i] = u32x4{0, 0, 0, 0};
    if (live && kvalid) {
      int sy = gy + ty;
      sy = sy < 0 ? sy + H : (sy >= H ? sy - H : sy);
      const int rowbase = (gb * H + sy) * W;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        int sx = gx + i + tx;
        sx = sx < 0 ? sx + W : (sx >= W ? sx - W : sx);
        // element offsets fit 31 bits (checked on the host)
        xr[i] = *reinterpret_cast<const u32x4*>(x + (rowbase + sx) * cin + ci);
      }
    }
    if (dgrp) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        dr[i] = live ? *reinterpret_cast<const u32x4*>(dy + (p + i) * cout + co0 + 8 * kc) : u32x4{0, 0, 0, 0};
    }
    // advance the group by one chunk
    gx += kWtChunk;
    while (gx >= W) {
      gx -= W;
      if (++gy == H) {
        gy = 0;
        ++gb;
      }
    }
  };
  // 8 pixels x 8 channels (one 16-byte row per pixel) -> 8 channels x 8
  // pixels: word w of channel row j holds pixels 2w (low half) and 2w + 1
  auto put = [&](const u32x4 (&g)[8], uint16_t* dst) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
      u32x4 o;
#pragma unroll
      for (int w = 0; w < 4; ++w) o[w] = __builtin_amdgcn_perm(g[2 * w + 1][j >> 1], g[2 * w][j >> 1], sel);
      *reinterpret_cast<u32x4*>(dst + j * kWtStride) = o;
    }
  };

  f32x16 acc[A];
#pragma unroll
  for (int a = 0; a < A; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[a][r] = 0.0f;
  float bsum[A];
#pragma unroll
  for (int a = 0; a < A; ++a) bsum[a] = 0.0f;
  const bool want_bias = bpart && by == 0 && wave == 0;
  if (pbeg < pend) fetch(pbeg);
  for (int pc = pbeg; pc < pend; pc += kWtChunk) {
    __syncthreads();      // every wave is done with the previous chunk
    put(xr, xT + (8 * kc) * kWtStride + 8 * pg);
    if (dgrp) put(dr, dyT + (8 * kc) * kWtStride + 8 * pg);
    __syncthreads();
    if (pc + kWtChunk < pend) fetch(pc + kWtChunk);
#pragma unroll
    for (int s = 0; s < kWtChunk / 16; ++s) {
      const u32x4 braw = *reinterpret_cast<const u32x4*>(xT + (32 * wave + (lane & 31)) * kWtStride + 16 * s + half);
#pragma unroll
      for (int a = 0; a < A; ++a) {
        const u32x4 araw = *reinterpret_cast<const u32x4*>(dyT + (32 * a + (lane & 31)) * kWtStride + 16 * s + half);
        if (want_bias) {
#pragma unroll
          for (int w = 0; w < 4; ++w)
            bsum[a] += bf2f(static_cast<uint16_t>(araw[w])) + bf2f(static_cast<uint16_t>(araw[w] >> 16));
        }
        acc[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, araw),
                                                         __builtin_bit_cast(bf16x8, braw), acc[a], 0, 0, 0);
      }
    }
  }
  const int kcol = kb0 + 32 * wave + (lane & 31);
#pragma unroll
  for (int a = 0; a < A; ++a) {
    if (kcol < K) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);     // co within the tile
        part[(static_cast<int64_t>(split) * cout + co0 + 32 * a + row) * K + kcol] = acc[a][r];
      }
    }
    if (want_bias) {
      // lanes l and l + 32 hold the two pixel halves of channel l
      const float tot = bsum[a] + __shfl_xor(bsum[a], 32);
      if (lane < 32) bpart[static_cast<int64_t>(split) * cout + co0 + 32 * a + lane] = tot;
    }
  }
}

// The weight (and bias) gradient from the per-range partial sums, in one
// pass and a fixed order. part holds nsplit slices of n floats (bpart
// nsplit slices of nb); with G = min(nsplit, 16) groups, group g sums the
// slices g, g + G, g + 2G, ... in that order, and the result is 0 plus the
// groups in increasing g. A block owns 64 elements (weights first, then
// bias): its four waves take four groups each, reading 64 consecutive
// floats per load, and the first wave adds the groups up from LDS.
__global__ void __launch_bounds__(256) wgrad_sum_kernel(const float* __restrict__ part,
                                                        const float* __restrict__ bpart, int nsplit, int G,
                                                        int64_t n, int nb, float* __restrict__ dw,
                                                        float* __restrict__ dbias) {
  __shared__ float gs[16][64];
  const int e = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + e;
  const bool live = i < n + nb;
  const bool is_w = i < n;
  const float* src = is_w ? part + i : bpart + (i - n);
  const int64_t stride = is_w ? n : nb;
  for (int g = w; g < G; g += 4) {
    float s = 0.0f;
    if (live) {
      s = src[static_cast<int64_t>(g) * stride];
#pragma unroll 4
      for (int k = g + G; k < nsplit; k += G) s += src[static_cast<int64_t>(k) * stride];
    }
    gs[g][e] = s;
  }
  __syncthreads();
  if (w == 0 && live) {
    float s = 0.0f;
    for (int g = 0; g < G; ++g) s += gs[g][e];
    if (is_w)
      dw[i] = s;
    else
      dbias[i - n] = s;
  }
}

// ---------------------------------------------------------------------------
// Elementwise pieces.
// ---------------------------------------------------------------------------
#define QNN_GRID_STRIDE(i, n)                                                                  \
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < (n);       \
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)

__global__ void leaky_bwd_kernel(int64_t n, const uint16_t* __restrict__ y, const uint16_t* dy, uint16_t* dz) {
  QNN_GRID_STRIDE(i, n) {
    const float g = bf2f(dy[i]);
    dz[i] = f2bf(bf2f(y[i]) > 0.0f ? g : kLeakySlope * g);
  }
}

__global__ void add_kernel(int64_t n, const uint16_t* a, const uint16_t* b, uint16_t* y) {
  QNN_GRID_STRIDE(i, n) { y[i] = f2bf(bf2f(a[i]) + bf2f(b[i])); }
}

__global__ void avgpool2_kernel(int B, int H, int W, int C, const uint16_t* __restrict__ x, uint16_t* __restrict__ y) {
  const int h = H / 2, w = W / 2;
  const int64_t n = static_cast<int64_t>(B) * h * w * C;
  QNN_GRID_STRIDE(i, n) {
    const int c = static_cast<int>(i % C);
    int64_t q = i / C;
    const int xo = static_cast<int>(q % w);
    q /= w;
    const int yo = static_cast<int>(q % h);
    const int b = static_cast<int>(q / h);
    const int64_t base = ((static_cast<int64_t>(b) * H + 2 * yo) * W + 2 * xo) * C + c;
    const float s = bf2f(x[base]) + bf2f(x[base + C]) + bf2f(x[base + static_cast<int64_t>(W) * C]) +
                    bf2f(x[base + static_cast<int64_t>(W) * C + C]);
    y[i] = f2bf(0.25f * s);
  }
}

__global__ void avgpool2_bwd_kernel(int B, int H, int W, int C, const uint16_t* __restrict__ dy,
                                    uint16_t* __restrict__ dx, int accumulate) {
  const int h = H / 2, w = W / 2;
  const int64_t n = static_cast<int64_t>(B) * H * W * C;
  QNN_GRID_STRIDE(i, n) {
    const int c = static_cast<int>(i % C);
    int64_t q = i / C;
    const int xx = static_cast<int>(q % W);
    q /= W;
    const int yy = static_cast<int>(q % H);
    const int b = static_cast<int>(q / H);
    const float g = 0.25f * bf2f(dy[((static_cast<int64_t>(b) * h + yy / 2) * w + xx / 2) * C + c]);
    dx[i] = f2bf(accumulate ? bf2f(dx[i]) + g : g);
  }
}

__global__ void upsample2_kernel(int B, int h, int w, int C, const uint16_t* __restrict__ x, uint16_t* __restrict__ y) {
  const int H = 2 * h, W = 2 * w;
  const int64_t n = static_cast<int64_t>(B) * H * W * C;
  QNN_GRID_STRIDE(i, n) {
    const int c = static_cast<int>(i % C);
    int64_t q = i / C;
    const int xx = static_cast<int>(q % W);
    q /= W;
    const int yy = static_cast<int>(q % H);
    const int b = static_cast<int>(q / H);
    y[i] = x[((static_cast<int64_t>(b) * h + yy / 2) * w + xx / 2) * C + c];
  }
}

__global__ void upsample2_bwd_kernel(int B, int h, int w, int C, const uint16_t* __restrict__ dy, uint16_t* __restrict__ dx) {
  const int W = 2 * w;
  const int64_t n = static_cast<int64_t>(B) * h * w * C;
  QNN_GRID_STRIDE(i, n) {
    const int c = static_cast<int>(i % C);
    int64_t q = i / C;
    const int xo = static_cast<int>(q % w);
    q /= w;
    const int yo = static_cast<int>(q % h);
    const int b = static_cast<int>(q / h);
    const int64_t base = ((static_cast<int64_t>(b) * 2 * h + 2 * yo) * W + 2 * xo) * C + c;
    const float s = bf2f(dy[base]) + bf2f(dy[base + C]) + bf2f(dy[base + static_cast<int64_t>(W) * C]) +
                    bf2f(dy[base + static_cast<int64_t>(W) * C + C]);
    dx[i] = f2bf(s);
  }
}

// 8-channel vector forms of the elementwise kernels (C % 8 == 0, 16-byte
// aligned tensors): one thread moves 16 bytes per tensor, with the same
// per-element arithmetic as the scalar forms above.
__device__ inline void ld8(const uint16_t* p, float (&f)[8]) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[2 * k] = bf2f(static_cast<uint16_t>(w[k] & 0xffffu));
    f[2 * k + 1] = bf2f(static_cast<uint16_t>(w[k] >> 16));
  }
}

__device__ inline void st8(uint16_t* p, const float (&f)[8]) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = static_cast<uint32_t>(f2bf(f[2 * k])) | (static_cast<uint32_t>(f2bf(f[2 * k + 1])) << 16);
  *reinterpret_cast<uint4*>(p) = make_uint4(w[0], w[1], w[2], w[3]);
}

__global__ void leaky_bwd_v8_kernel(int64_t n8, const uint16_t* __restrict__ y, const uint16_t* dy, uint16_t* dz) {
  QNN_GRID_STRIDE(i, n8) {
    float a[8], g[8];
    ld8(y + 8 * i, a);
    ld8(dy + 8 * i, g);
#pragma unroll
    for (int k = 0; k < 8; ++k) g[k] = a[k] > 0.0f ? g[k] : kLeakySlope * g[k];
    st8(dz + 8 * i, g);
  }
}

__global__ void add_v8_kernel(int64_t n8, const uint16_t* a, const uint16_t* b, uint16_t* y) {
  QNN_GRID_STRIDE(i, n8) {
    float u[8], v[8];
    ld8(a + 8 * i, u);
    ld8(b + 8 * i, v);
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k] = u[k] + v[k];
    st8(y + 8 * i, u);
  }
}

// one thread per (coarse pixel, 8-channel group)
__global__ void avgpool2_v8_kernel(int B, int H, int W, int C, const uint16_t* __restrict__ x, uint16_t* __restrict__ y) {
  const int h = H / 2, w = W / 2, G = C / 8;
  const int64_t n = static_cast<int64_t>(B) * h * w * G;
  QNN_GRID_STRIDE(i, n) {
    const int g = static_cast<int>(i % G);
    const int64_t pix = i / G;
    const int xo = static_cast<int>(pix % w);
    const int64_t r = pix / w;
    const int yo = static_cast<int>(r % h);
    const int64_t b = r / h;
    const int64_t base = ((b * H + 2 * yo) * W + 2 * xo) * C + 8 * g;
    const int64_t row = static_cast<int64_t>(W) * C;
    float a[8], c1[8], c2[8], c3[8];
    ld8(x + base, a);
    ld8(x + base + C, c1);
    ld8(x + base + row, c2);
    ld8(x + base + row + C, c3);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0.25f * (a[k] + c1[k] + c2[k] + c3[k]);
    st8(y + pix * C + 8 * g, a);
  }
}

__global__ void avgpool2_bwd_v8_kernel(int B, int H, int W, int C, const uint16_t* __restrict__ dy,
                                       uint16_t* __restrict__ dx, int accumulate) {
  const int h = H / 2, w = W / 2, G = C / 8;
  const int64_t n = static_cast<int64_t>(B) * h * w * G;
  QNN_GRID_STRIDE(i, n) {
    const int g = static_cast<int>(i % G);
    const int64_t pix = i / G;
    const int xo = static_cast<int>(pix % w);
    const int64_t r = pix / w;
    const int yo = static_cast<int>(r % h);
    const int64_t b = r / h;
    float d[8];
    ld8(dy + pix * C + 8 * g, d);
#pragma unroll
    for (int k = 0; k < 8; ++k) d[k] = 0.25f * d[k];
    const int64_t base = ((b * H + 2 * yo) * W + 2 * xo) * C + 8 * g;
    const int64_t off[4] = {0, C, static_cast<int64_t>(W) * C, static_cast<int64_t>(W) * C + C};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float o[8];
      if (accumulate) {
        ld8(dx + base + off[j], o);
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = o[k] + d[k];
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = d[k];
      }
      st8(dx + base + off[j], o);
    }
  }
}

__global__ void upsample2_v8_kernel(int B, int h, int w, int C, const uint16_t* __restrict__ x, uint16_t* __restrict__ y) {
  const int W = 2 * w, G = C / 8;
  const int64_t n = static_cast<int64_t>(B) * h * w * G;
  QNN_GRID_STRIDE(i, n) {
    const int g = static_cast<int>(i % G);
    const int64_t pix = i / G;
    const int xo = static_cast<int>(pix % w);
    const int64_t r = pix / w;
    const int yo = static_cast<int>(r % h);
    const int64_t b = r / h;
    const uint4 v = *reinterpret_cast<const uint4*>(x + pix * C + 8 * g);
    const int64_t base = ((b * 2 * h + 2 * yo) * W + 2 * xo) * C + 8 * g;
    const int64_t row = static_cast<int64_t>(W) * C;
    *reinterpret_cast<uint4*>(y + base) = v;
    *reinterpret_cast<uint4*>(y + base + C) = v;
    *reinterpret_cast<uint4*>(y + base + row) = v;
    *reinterpret_cast<uint4*>(y + base + row + C) = v;
  }
}

__global__ void upsample2_bwd_v8_kernel(int B, int h, int w, int C, const uint16_t* __restrict__ dy,
                                        uint16_t* __restrict__ dx) {
  const int W = 2 * w, G = C / 8;
  const int64_t n = static_cast<int64_t>(B) * h * w * G;
  QNN_GRID_STRIDE(i, n) {
    const int g = static_cast<int>(i % G);
    const int64_t pix = i / G;
    const int xo = static_cast<int>(pix % w);
    const int64_t r = pix / w;
    const int yo = static_cast<int>(r % h);
    const int64_t b = r / h;
    const int64_t base = ((b * 2 * h + 2 * yo) * W + 2 * xo) * C + 8 * g;
    const int64_t row = static_cast<int64_t>(W) * C;
    float a[8], c1[8], c2[8], c3[8];
    ld8(dy + base, a);
    ld8(dy + base + C, c1);
    ld8(dy + base + row, c2);
    ld8(dy + base + row + C, c3);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = a[k] + c1[k] + c2[k] + c3[k];
    st8(dx + pix * C + 8 * g, a);
  }
}

// Per-sample max |q|: a 2D grid of blocks per sample, each folding its
// share with an unsigned atomic max on the float's bits (|q| >= 0, whose bit
// patterns order like the values); absmax_init clears, absmax_fix turns 0
// into 1.
__global__ void absmax_init_kernel(int B, float* __restrict__ scale) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) scale[b] = 0.0f;
}

template <bool VEC>
__global__ void __launch_bounds__(256) absmax_kernel(int H, int W, const float* __restrict__ q,
                                                     const int32_t* __restrict__ idx, float* __restrict__ scale) {
  const int b = blockIdx.y;
  const int64_t n = 6 * static_cast<int64_t>(H) * W;
  const float* qs = q + (idx ? idx[b] : b) * n;
  float m = 0.0f;
  const int64_t first = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  if constexpr (VEC) {
    // 16-byte loads, four in flight per thread (the maximum does not depend
    // on the order)
    const float4* q4 = reinterpret_cast<const float4*>(qs);
#pragma unroll 4
    for (int64_t i = first; i < n / 4; i += stride) {
      const float4 v = q4[i];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
  } else {
    for (int64_t i = first; i < n; i += stride) m = fmaxf(m, fabsf(qs[i]));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __shared__ float sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    atomicMax(reinterpret_cast<unsigned int*>(scale + b), __float_as_uint(m));
  }
}

__global__ void absmax_fix_kernel(int B, float* __restrict__ scale) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B && !(scale[b] > 0.0f)) scale[b] = 1.0f;
}

constexpr int kInCh = 48;

// One thread per pixel computes its 48 input channels (see qnn_pack_input).
// dx, dy: the displacement reduced to [0, W) and [0, H). Element offsets
// within a sample's planes fit 31 bits (checked on the host).
__global__ void __launch_bounds__(256) pack_input_kernel(int B, int H, int W, const float* __restrict__ q,
                                                         const int32_t* __restrict__ idx_q,
                                                         const float* __restrict__ n,
                                                         const int32_t* __restrict__ idx_n,
                                                         const float* __restrict__ scale, float n_shift,
                                                         float n_scale, int dx, int dy, uint16_t* __restrict__ x) {
  // a block packs 256 consecutive pixels at a time: each thread computes
  // its pixel's 48 channels into LDS, then the block stores the 24 KiB run
  // in 16-byte pieces, consecutive lanes on consecutive pieces
  __shared__ __attribute__((aligned(16))) uint16_t stage[256 * kInCh];
  const int HW = H * W;
  const int64_t total = static_cast<int64_t>(B) * HW;
  for (int64_t p0 = static_cast<int64_t>(blockIdx.x) * 256; p0 < total; p0 += static_cast<int64_t>(gridDim.x) * 256) {
    const int64_t p = p0 + threadIdx.x;
    __syncthreads();    // the previous run's stores have read the stage
    if (p < total) {
      const int b = static_cast<int>(p / HW);
      const int s = static_cast<int>(p - static_cast<int64_t>(b) * HW);
      const int yy = s / W, xx = s - (s / W) * W;
      const float* qb = q + static_cast<int64_t>(idx_q ? idx_q[b] : b) * 6 * HW;
      const float* nb = n + static_cast<int64_t>(idx_n ? idx_n[b] : b) * 3 * HW;
      const float sc = scale[b];
      // the four displaced source pixels, periodic
      const int xm = xx >= dx ? xx - dx : xx - dx + W;
      const int xp = xx + dx < W ? xx + dx : xx + dx - W;
      const int ym = yy >= dy ? yy - dy : yy - dy + H;
      const int yp = yy + dy < H ? yy + dy : yy + dy - H;
      const int src[4] = {yy * W + xm, yy * W + xp, ym * W + xx, yp * W + xx};
      float v[kInCh];
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = qb[c * HW + s] / sc;
#pragma unroll
      for (int c = 0; c < 3; ++c) v[6 + c] = (nb[c * HW + s] - n_shift) / n_scale;
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[9 + 6 * k + c] = qb[c * HW + src[k]] / sc;
#pragma unroll
      for (int c = 33; c < kInCh; ++c) v[c] = 0.0f;
#pragma unroll
      for (int g = 0; g < kInCh / 8; ++g) {
        float f[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) f[j] = v[8 * g + j];
        st8(stage + threadIdx.x * kInCh + 8 * g, f);
      }
    }
    __syncthreads();
    const int64_t pieces = (total - p0 < 256 ? total - p0 : 256) * (kInCh / 8);
#pragma unroll
    for (int k = 0; k < kInCh / 8; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < pieces)
        *reinterpret_cast<uint4*>(x + p0 * kInCh + 8 * i) = *reinterpret_cast<const uint4*>(stage + 8 * i);
    }
  }
}

// one thread per pixel: the pixel's 6 output channels are adjacent in y
__global__ void unpack_output_kernel(int B, int H, int W, const float* __restrict__ y, int y_ld,
                                     const float* __restrict__ scale, float* __restrict__ q) {
  const int64_t HW = static_cast<int64_t>(H) * W;
  const int64_t total = B * HW;
  QNN_GRID_STRIDE(p, total) {
    const int b = static_cast<int>(p / HW);
    const int64_t s = p - b * HW;
    const float* yp = y + p * y_ld;
    const float sc = scale[b];
#pragma unroll
    for (int c = 0; c < 6; ++c) q[(b * 6 + c) * HW + s] = yp[c] * sc;
  }
}

// relative L2: per-sample partial sums of (pred-target)^2 and target^2, the
// target being lattice sample idx_t[b] divided by scale[b]
__global__ void __launch_bounds__(256) rel_l2_partial_kernel(int H, int W, const float* __restrict__ pred, int pred_ld,
                                                             const float* __restrict__ target,
                                                             const int32_t* __restrict__ idx_t,
                                                             const float* __restrict__ scale,
                                                             double* __restrict__ work) {
  const int b = blockIdx.y;
  const int64_t HW = static_cast<int64_t>(H) * W;
  const float* tb = target + (idx_t ? idx_t[b] : b) * 6 * HW;
  const double inv = 1.0 / static_cast<double>(scale ? scale[b] : 1.0f);
  double num = 0.0, den = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < 6 * HW;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(i / HW);
    const int64_t s = i - c * HW;
    const double t = static_cast<double>(tb[i]) * inv;
    const double d = static_cast<double>(pred[(b * HW + s) * pred_ld + c]) - t;
    num += d * d;
    den += t * t;
  }
  for (int o = 32; o > 0; o >>= 1) {
    num += __shfl_xor(num, o);
    den += __shfl_xor(den, o);
  }
  __shared__ double sh[2][4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = num;
    sh[1][wv] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nb = gridDim.x;
    work[(static_cast<int64_t>(b) * nb + blockIdx.x) * 2 + 0] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    work[(static_cast<int64_t>(b) * nb + blockIdx.x) * 2 + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

// one thread per sample folds its partials; thread 0 then forms the loss
__global__ void rel_l2_final_kernel(int B, int nb, double* __restrict__ work, double* __restrict__ loss,
                                    double* __restrict__ per_sample) {
  __shared__ double rel2[1024];
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    double num = 0.0, den = 0.0;
    for (int k = 0; k < nb; ++k) {
      num += work[(static_cast<int64_t>(b) * nb + k) * 2 + 0];
      den += work[(static_cast<int64_t>(b) * nb + k) * 2 + 1];
    }
    // folded (num, den) of sample b go to the front of the workspace
    work[2 * static_cast<int64_t>(B) * nb + 2 * b + 0] = num;
    work[2 * static_cast<int64_t>(B) * nb + 2 * b + 1] = den;
    const double r = den > 0.0 ? num / den : 0.0;
    if (b < 1024) rel2[b] = r;
    if (per_sample) per_sample[b] = sqrt(r);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < B && b < 1024; ++b) s += rel2[b];
    *loss = s / B;
  }
}

// One thread per pixel: the gradient of its 6 channels, zeros in the rest of
// the d_ld-channel row (16-byte pieces when VEC: d_ld % 8 == 0, aligned).
template <bool VEC>
__global__ void rel_l2_grad_kernel(int B, int H, int W, int nb, const float* __restrict__ pred, int pred_ld,
                                   const float* __restrict__ target, const int32_t* __restrict__ idx_t,
                                   const float* __restrict__ scale, const double* __restrict__ work,
                                   uint16_t* __restrict__ dpred, int d_ld) {
  const int64_t HW = static_cast<int64_t>(H) * W;
  const int64_t total = B * HW;
  QNN_GRID_STRIDE(p, total) {
    const int b = static_cast<int>(p / HW);
    const int64_t s = p - b * HW;
    const double den = work[2 * static_cast<int64_t>(B) * nb + 2 * b + 1];
    const double inv = 1.0 / static_cast<double>(scale ? scale[b] : 1.0f);
    const float* tb = target + static_cast<int64_t>(idx_t ? idx_t[b] : b) * 6 * HW + s;
    uint16_t gv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double t = static_cast<double>(tb[c * HW]) * inv;
      const double d = static_cast<double>(pred[p * pred_ld + c]) - t;
      gv[c] = f2bf(den > 0.0 ? static_cast<float>(2.0 * d / (den * B)) : 0.0f);
    }
    uint16_t* row = dpred + p * d_ld;
    if constexpr (VEC) {
      const u32x4 first = {static_cast<uint32_t>(gv[0]) | (static_cast<uint32_t>(gv[1]) << 16),
                           static_cast<uint32_t>(gv[2]) | (static_cast<uint32_t>(gv[3]) << 16),
                           static_cast<uint32_t>(gv[4]) | (static_cast<uint32_t>(gv[5]) << 16), 0u};
      *reinterpret_cast<u32x4*>(row) = first;
      for (int c = 8; c < d_ld; c += 8) *reinterpret_cast<u32x4*>(row + c) = u32x4{0u, 0u, 0u, 0u};
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) row[c] = gv[c];
      for (int c = 6; c < d_ld; ++c) row[c] = 0;
    }
  }
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, uint16_t* __restrict__ pb, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  QNN_GRID_STRIDE(i, n) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f2bf(pi);
  }
}

// per-sample comparison: kCompareBlocks partial blocks per sample write
// (sum d^2, sum a^2, sum r^2) to work; compare_final folds them
constexpr int kCompareBlocks = 64;

__global__ void __launch_bounds__(256) compare_kernel(int64_t m, const float* __restrict__ a, const float* __restrict__ r,
                                                      double* __restrict__ work) {
  const int b = blockIdx.y;
  const float* ab = a + b * m;
  const float* rb = r + b * m;
  double dd = 0.0, aa = 0.0, rr = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < m;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double x = ab[i], y = rb[i];
    dd += (x - y) * (x - y);
    aa += x * x;
    rr += y * y;
  }
  for (int o = 32; o > 0; o >>= 1) {
    dd += __shfl_xor(dd, o);
    aa += __shfl_xor(aa, o);
    rr += __shfl_xor(rr, o);
  }
  __shared__ double sh[3][4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = dd;
    sh[1][wv] = aa;
    sh[2][wv] = rr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* w = work + (static_cast<int64_t>(b) * kCompareBlocks + blockIdx.x) * 3;
    w[0] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    w[1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    w[2] = sh[2][0] + sh[2][1] + sh[2][2] + sh[2][3];
  }
}

__global__ void compare_final_kernel(int B, const double* __restrict__ work, double* __restrict__ rel,
                                     double* __restrict__ en) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double dd = 0.0, aa = 0.0, rr = 0.0;
  for (int k = 0; k < kCompareBlocks; ++k) {
    const double* w = work + (static_cast<int64_t>(b) * kCompareBlocks + k) * 3;
    dd += w[0];
    aa += w[1];
    rr += w[2];
  }
  rel[b] = rr > 0.0 ? sqrt(dd / rr) : sqrt(dd);
  en[b] = rr > 0.0 ? fabs(aa - rr) / rr : aa;
}

// compute units of the device the library first launched on, queried once
// (thread-safe static initialisation)
int cu_count() {
  static const int cus = [] {
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    return n > 0 ? n : 1;
  }();
  return cus;
}

// Launch of the pipelined forward kernel: grid.y channel groups of 32*NT;
// grid.x persistent blocks, as many as stay resident at once (times
// `waves`, capped by the tile count).
template <int MT, int NT>
void conv_pipe_launch(int B, int H, int W, const uint16_t* x, int cin, int up, const uint16_t* w, const float* bias,
                      int act, const uint16_t* add, void* y, bool y_fp32, int y_ld, int c_store, int c_out,
                      float waves, hipStream_t st) {
  // resident blocks per CU of the two instances, queried once (thread-safe
  // static initialisation)
  const int cus = cu_count();
  static const int res_bf16 = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_pipe_kernel<MT, NT, false>, 256, 0);
    return n > 0 ? n : 1;
  }();
  static const int res_fp32 = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_pipe_kernel<MT, NT, true>, 256, 0);
    return n > 0 ? n : 1;
  }();
  const int res = y_fp32 ? res_fp32 : res_bf16;
  const int TW = W < 64 ? W : 64;
  const int tws = TW == 64 ? 6 : (TW == 32 ? 5 : 4);
  const int TH = PipeConv<MT, NT>::kPix / TW;
  const int64_t tiles = static_cast<int64_t>(B) * (W / TW) * ((H + TH - 1) / TH);
  const int gy = c_out / PipeConv<MT, NT>::kBN;
  int64_t gx = static_cast<int64_t>(waves * cus * res / gy);
  if (gx < 1) gx = 1;
  if (gx > tiles) gx = tiles;
  dim3 grid(static_cast<unsigned>(gx), gy);
  if (y_fp32)
    hipLaunchKernelGGL((conv_fwd_pipe_kernel<MT, NT, true>), grid, dim3(256), 0, st, H, W, tws, static_cast<int>(tiles),
                       x, cin, w, bias, act, y, y_ld, c_store, up, add);
  else
    hipLaunchKernelGGL((conv_fwd_pipe_kernel<MT, NT, false>), grid, dim3(256), 0, st, H, W, tws, static_cast<int>(tiles),
                       x, cin, w, bias, act, y, y_ld, c_store, up, add);
}

// the pipelined kernel's tiles: W a multiple of TW = min(W, 64) in {16, 32, 64}
inline bool pipe_fits(int W) { return W % 16 == 0 && (W >= 64 ? W % 64 == 0 : (W == 16 || W == 32)); }

bool conv_pipe(int mt, int nt, int B, int H, int W, const uint16_t* x, int cin, int up, const uint16_t* w,
               const float* bias, int act, const uint16_t* add, void* y, bool y_fp32, int y_ld, int c_store,
               int c_out, float waves, hipStream_t st) {
  if (!pipe_fits(W) || c_out % (32 * nt)) return false;
  // BF16 results leave in 16-byte pieces: every channel stored, whole
  // 8-channel groups per row, 16-byte aligned rows
  if (!y_fp32 && (c_store != c_out || y_ld % 8 || (reinterpret_cast<uintptr_t>(y) & 15))) return false;
#define QNN_PIPE(M, N)                                                                                   \
  if (mt == M && nt == N) {                                                                              \
    conv_pipe_launch<M, N>(B, H, W, x, cin, up, w, bias, act, add, y, y_fp32, y_ld, c_store, c_out, waves, st); \
    return true;                                                                                         \
  }
  QNN_PIPE(1, 1) QNN_PIPE(1, 2) QNN_PIPE(2, 1) QNN_PIPE(2, 2)
#undef QNN_PIPE
  return false;
}

// The resident-weight kernel (16*KC input channels, 32*NT output channels
// a block): tiles of TW = tw columns (32, or 16) x 256 / tw rows, grid.x
// persistent blocks as many as stay resident at once (times `waves`, capped
// by the tile count).
template <int KC, int NT>
void conv_res_launch(int B, int H, int W, const uint16_t* x, const uint16_t* w, const float* bias, int act,
                     const uint16_t* add, void* y, bool y_fp32, int y_ld, int c_store, int c_out, int tw,
                     float waves, hipStream_t st, uint16_t* pool = nullptr) {
  const int cus = cu_count();
  static const int res_bf16 = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_res_kernel<KC, NT, false>, 256, 0);
    return n > 0 ? n : 1;
  }();
  static const int res_fp32 = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_res_kernel<KC, NT, true>, 256, 0);
    return n > 0 ? n : 1;
  }();
  static const int res_pool = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_res_kernel<KC, NT, false, false, true>, 256, 0);
    return n > 0 ? n : 1;
  }();
  const int res = y_fp32 ? res_fp32 : (pool ? res_pool : res_bf16);
  const int tws = tw == 32 ? 5 : 4;
  const int TH = 256 / tw;
  const int64_t tiles = static_cast<int64_t>(B) * (W / tw) * ((H + TH - 1) / TH);
  const int gy = c_out / (32 * NT);
  int64_t gx = static_cast<int64_t>(waves * cus * res / gy);
  if (gx < 1) gx = 1;
  if (gx > tiles) gx = tiles;
  dim3 grid(static_cast<unsigned>(gx), gy);
  if (y_fp32)
    hipLaunchKernelGGL((conv_fwd_res_kernel<KC, NT, true>), grid, dim3(256), 0, st, H, W, tws,
                       static_cast<int>(tiles), x, w, bias, act, y, y_ld, c_store, add, nullptr, nullptr);
  else if (pool)
    hipLaunchKernelGGL((conv_fwd_res_kernel<KC, NT, false, false, true>), grid, dim3(256), 0, st, H, W, tws,
                       static_cast<int>(tiles), x, w, bias, act, y, y_ld, c_store, add, nullptr, pool);
  else
    hipLaunchKernelGGL((conv_fwd_res_kernel<KC, NT, false>), grid, dim3(256), 0, st, H, W, tws,
                       static_cast<int>(tiles), x, w, bias, act, y, y_ld, c_store, add, nullptr, nullptr);
}

// The resident-weight kernel writing nq scaled FP32 planes (32 output
// channels), grid as above.
template <int KC>
void conv_res_planes_launch(int B, int H, int W, const uint16_t* x, const uint16_t* w, const float* bias, int act,
                            const float* scale, int nq, float* q, int tw, hipStream_t st) {
  const int cus = cu_count();
  static const int res = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_res_kernel<KC, 1, true, true>, 256, 0);
    return n > 0 ? n : 1;
  }();
  const int tws = tw == 32 ? 5 : 4;
  const int TH = 256 / tw;
  const int64_t tiles = static_cast<int64_t>(B) * (W / tw) * ((H + TH - 1) / TH);
  int64_t gx = static_cast<int64_t>(cus) * res;
  if (gx > tiles) gx = tiles;
  hipLaunchKernelGGL((conv_fwd_res_kernel<KC, 1, true, true>), dim3(static_cast<unsigned>(gx), 1), dim3(256), 0, st,
                     H, W, tws, static_cast<int>(tiles), x, w, bias, act, q, 0, nq, nullptr, scale, nullptr);
}

// the resident-weight kernel where it applies: 32 or 48 input channels with
// 32-channel blocks (nt = 1), 32 or 64 with 64-channel blocks (nt = 2), W a
// multiple of the tile width tw (32 or 16), and BF16 results leaving in
// 16-byte pieces as in the pipelined kernel
bool conv_res(int B, int H, int W, const uint16_t* x, int cin, const uint16_t* w, const float* bias, int act,
              const uint16_t* add, void* y, bool y_fp32, int y_ld, int c_store, int c_out, int nt, int tw,
              float waves, hipStream_t st, uint16_t* pool = nullptr) {
  if ((tw != 16 && tw != 32) || W % tw || (nt != 1 && nt != 2) || c_out % (32 * nt)) return false;
  if (!y_fp32 && (c_store != c_out || y_ld % 8 || (reinterpret_cast<uintptr_t>(y) & 15))) return false;
  if (pool && (y_fp32 || add || (H & 1) || (W & 1) || (reinterpret_cast<uintptr_t>(pool) & 15))) return false;
#define QNN_RES(C, N)                                                                                             \
  if (cin == 16 * (C) && nt == (N)) {                                                                            \
    conv_res_launch<C, N>(B, H, W, x, w, bias, act, add, y, y_fp32, y_ld, c_store, c_out, tw, waves, st, pool);  \
    return true;                                                                                                  \
  }
  QNN_RES(2, 1) QNN_RES(3, 1) QNN_RES(2, 2) QNN_RES(4, 2)
#undef QNN_RES
  return false;
}

// The upsampling kernel (16*KC input channels at half resolution, BF16
// out): tiles of tw columns (32, or 16) x 256 / tw rows, grid.x persistent
// blocks as many as stay resident at once (capped by the tile count).
template <int KC>
void conv_up_launch(int B, int H, int W, const uint16_t* x, const uint16_t* w, const float* bias, int act,
                    const uint16_t* add, uint16_t* y, int y_ld, int c_out, int tw, float waves, hipStream_t st) {
  const int cus = cu_count();
  static const int res_add = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_up_kernel<KC, true>, 256, 0);
    return n > 0 ? n : 1;
  }();
  static const int res_plain = [] {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, conv_fwd_up_kernel<KC, false>, 256, 0);
    return n > 0 ? n : 1;
  }();
  const int tws = tw == 32 ? 5 : 4;
  const int TH = 256 / tw;
  const int64_t tiles = static_cast<int64_t>(B) * (W / tw) * ((H + TH - 1) / TH);
  const int gy = c_out / 32;
  int64_t gx = static_cast<int64_t>(waves * cus * (add ? res_add : res_plain) / gy);
  if (gx < 1) gx = 1;
  if (gx > tiles) gx = tiles;
  dim3 grid(static_cast<unsigned>(gx), gy);
  if (add)
    hipLaunchKernelGGL((conv_fwd_up_kernel<KC, true>), grid, dim3(256), 0, st, H, W, tws, static_cast<int>(tiles), x,
                       w, bias, act, y, y_ld, add);
  else
    hipLaunchKernelGGL((conv_fwd_up_kernel<KC, false>), grid, dim3(256), 0, st, H, W, tws, static_cast<int>(tiles), x,
                       w, bias, act, y, y_ld, add);
}

bool conv_up(int B, int H, int W, const uint16_t* x, int cin, const uint16_t* w, const float* bias, int act,
             const uint16_t* add, uint16_t* y, int y_ld, int c_out, int tw, float waves, hipStream_t st) {
  if ((tw != 16 && tw != 32) || W % tw || (H & 1) || c_out % 32 || y_ld % 8) return false;
  if (cin == 64)
    conv_up_launch<4>(B, H, W, x, w, bias, act, add, y, y_ld, c_out, tw, waves, st);
  else if (cin == 128)
    conv_up_launch<8>(B, H, W, x, w, bias, act, add, y, y_ld, c_out, tw, waves, st);
  else
    return false;
  return true;
}

// Tile shape of the pipelined kernel for a layer: 256-pixel tiles x 64
// channels when that gives two or more blocks per CU, else 128-pixel tiles;
// the layers with the fewest pixels split the channels finest.
// Weight-gradient geometry of the staged kernel: a = 32-channel output tiles
// per block (2 when c_out allows), and the pixel range of a block (pps, a
// multiple of the 128-pixel chunk) chosen so that the blocks fill the chip
// once: at most kWgradResident of them, the blocks both instances keep
// resident on the 256 CUs of an MI355X (three each, bound by LDS). Past that
// a second, partial round of blocks would take as long as the first. nsplit
// ranges (each leaves one partial dW in the workspace).
constexpr int64_t kWgradResident = 3 * 256;

void wgrad_split(int P, int c_in, int c_out, int& a, int& nsplit, int& pps) {
  a = (c_out % 64 == 0) ? 2 : 1;
  const int64_t blocks_xy = static_cast<int64_t>(c_out / (32 * a)) * ((9 * c_in + 127) / 128);
  int64_t want = kWgradResident / blocks_xy;
  const int64_t chunks = (P + kWtChunk - 1) / kWtChunk;
  if (want > chunks) want = chunks;
  if (want < 1) want = 1;
  const int64_t per = (P + want - 1) / want;
  pps = static_cast<int>((per + kWtChunk - 1) / kWtChunk * kWtChunk);
  nsplit = static_cast<int>((P + pps - 1) / pps);
}

void pipe_shape(int B, int H, int W, int c_out, int& m, int& n) {
  const int TW = W < 64 ? W : 64;
  auto blocks = [&](int mt, int nt) {
    const int TH = 128 * mt / TW;
    return static_cast<int64_t>(B) * (W / TW) * ((H + TH - 1) / TH) * (c_out / (32 * nt));
  };
  const int nt = (c_out % 64 == 0) ? 2 : 1;
  m = 1;
  n = 1;
  if (blocks(2, nt) >= 512) m = 2, n = nt;
  else if (blocks(1, nt) >= 256) n = nt;
}

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  QNN_GRID_STRIDE(i, n) { y[i] = f2bf(x[i]); }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  return static_cast<int>(g < 1 ? 1 : g);
}

int launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("qnn: %s: %s", what, hipGetErrorString(e));
    return QNN_EDEVICE;
  }
  return QNN_OK;
}

int bad(const char* what) {
  set_error("qnn: %s", what);
  return QNN_EINVAL;
}

}  // namespace qnn

using namespace qnn;

extern "C" {

// the vector (16-byte) kernels need 16-byte alignment of every tensor
static bool a16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int qnn_conv3x3_fwd(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t c_in, const uint16_t* w,
                    const float* bias, int32_t c_out, int32_t act, void* y, int32_t y_fp32, int32_t y_ld,
                    int32_t c_store, void* hip_stream) {
  if (B < 1 || H < 1 || W < 1 || !x || !w || !y) return bad("conv3x3_fwd: bad size or null pointer");
  if (c_in < 16 || c_in % 16 || c_out < 32 || c_out % 32) return bad("conv3x3_fwd: c_in % 16, c_out % 32");
  if (c_store < 1 || c_store > c_out || y_ld < c_store) return bad("conv3x3_fwd: bad c_store / y_ld");
  if (act != QNN_ACT_NONE && act != QNN_ACT_LEAKY) return bad("conv3x3_fwd: unknown activation");
  if (!a16(x) || !a16(w)) return bad("conv3x3_fwd: x and w must be 16-byte aligned");
  const int64_t P64 = static_cast<int64_t>(B) * H * W;
  if (P64 * (c_in > y_ld ? c_in : y_ld) >= (int64_t{1} << 31)) return bad("conv3x3_fwd: tensor too large");
  const int P = static_cast<int>(P64);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the resident-weight kernel for the layers whose weights fit in LDS
  // (with 64 output channels only for grids of a tile per CU or more: it
  // keeps fewer blocks resident), else the pipelined kernel where its tiles
  // fit, else the pixel-list kernel
  {
    const int tw = W % 32 == 0 ? 32 : 16;
    const int64_t tiles = static_cast<int64_t>(B) * (W / tw) * ((H + 256 / tw - 1) / (256 / tw));
    const bool narrow = c_out == 32;
    const bool wide = c_out == 64 && (c_in == 32 || c_in == 64) && tiles >= 256;
    if ((narrow || wide) && conv_res(B, H, W, x, c_in, w, bias, act, nullptr, y, y_fp32 != 0, y_ld, c_store, c_out,
                                     c_in == 64 ? 2 : 1, tw, 1.0f, st))
      return launched("conv3x3_fwd");
  }
  if (pipe_fits(W)) {
    int m, n;
    pipe_shape(B, H, W, c_out, m, n);
    if (conv_pipe(m, n, B, H, W, x, c_in, 0, w, bias, act, nullptr, y, y_fp32 != 0, y_ld, c_store, c_out, 1.0f, st))
      return launched("conv3x3_fwd");
  }
  const int nt = (c_out % 64 == 0) ? 2 : 1;
  dim3 grid((P + 127) / 128, c_out / (32 * nt));
  if (nt == 2) {
    if (y_fp32) hipLaunchKernelGGL((conv_fwd_kernel<2, true>), grid, dim3(256), 0, st, P, H, W, x, c_in, w, bias, act, y, y_ld, c_store);
    else hipLaunchKernelGGL((conv_fwd_kernel<2, false>), grid, dim3(256), 0, st, P, H, W, x, c_in, w, bias, act, y, y_ld, c_store);
  } else {
    if (y_fp32) hipLaunchKernelGGL((conv_fwd_kernel<1, true>), grid, dim3(256), 0, st, P, H, W, x, c_in, w, bias, act, y, y_ld, c_store);
    else hipLaunchKernelGGL((conv_fwd_kernel<1, false>), grid, dim3(256), 0, st, P, H, W, x, c_in, w, bias, act, y, y_ld, c_store);
  }
  return launched("conv3x3_fwd");
}

int qnn_conv3x3_fwd_fused(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t c_in, int32_t up,
                          const uint16_t* w, const float* bias, int32_t c_out, int32_t act, const uint16_t* add,
                          uint16_t* y, int32_t y_ld, void* hip_stream) {
  if (B < 1 || H < 1 || W < 1 || !x || !w || !y) return bad("conv3x3_fwd_fused: bad size or null pointer");
  if (c_in < 16 || c_in % 16 || c_out < 32 || c_out % 32) return bad("conv3x3_fwd_fused: c_in % 16, c_out % 32");
  if (act != QNN_ACT_NONE && act != QNN_ACT_LEAKY) return bad("conv3x3_fwd_fused: unknown activation");
  if (up != 0 && up != 1) return bad("conv3x3_fwd_fused: up must be 0 or 1");
  if (up && ((H | W) & 1)) return bad("conv3x3_fwd_fused: an upsampled input needs even H and W");
  if (!pipe_fits(W)) return bad("conv3x3_fwd_fused: W must be 16, 32 or a multiple of 64");
  if (y_ld < c_out || y_ld % 8) return bad("conv3x3_fwd_fused: y_ld must be >= c_out and a multiple of 8");
  if (!a16(x) || !a16(w) || !a16(y) || (add && !a16(add)))
    return bad("conv3x3_fwd_fused: tensors must be 16-byte aligned");
  const int64_t P64 = static_cast<int64_t>(B) * H * W;
  if (P64 * (c_in > y_ld ? c_in : y_ld) >= (int64_t{1} << 31)) return bad("conv3x3_fwd_fused: tensor too large");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the upsampling kernel for 64 -> 32 channels, and for 128 -> 64 on 2^20
  // pixels or more (below that its one block per CU falls behind), with
  // 16-wide tiles (the skip input's rows are read in shorter runs but the
  // window is smaller); else the pipelined kernel
  const bool up_narrow = c_in == 64 && c_out == 32;
  const bool up_wide = c_in == 128 && c_out == 64 && P64 >= (int64_t{1} << 20);
  if (up && (up_narrow || up_wide) && conv_up(B, H, W, x, c_in, w, bias, act, add, y, y_ld, c_out, 16, 1.0f, st))
    return launched("conv3x3_fwd_fused");
  int m, n;
  pipe_shape(B, H, W, c_out, m, n);
  if (!conv_pipe(m, n, B, H, W, x, c_in, up, w, bias, act, add, y, false, y_ld, c_out, c_out, 1.0f, st))
    return bad("conv3x3_fwd_fused: shape not supported");
  return launched("conv3x3_fwd_fused");
}

int qnn_conv3x3_fwd_planes(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t c_in, const uint16_t* w,
                           const float* bias, int32_t c_out, int32_t act, const float* scale, int32_t n_planes,
                           float* q, void* hip_stream) {
  if (B < 1 || H < 1 || W < 1 || !x || !w || !scale || !q) return bad("conv3x3_fwd_planes: bad size or null pointer");
  if ((c_in != 32 && c_in != 48) || c_out != 32) return bad("conv3x3_fwd_planes: c_in must be 32 or 48, c_out 32");
  if (W % 16) return bad("conv3x3_fwd_planes: W must be a multiple of 16");
  if (n_planes < 1 || n_planes > 32) return bad("conv3x3_fwd_planes: n_planes must be 1..32");
  if (act != QNN_ACT_NONE && act != QNN_ACT_LEAKY) return bad("conv3x3_fwd_planes: unknown activation");
  if (!a16(x) || !a16(w)) return bad("conv3x3_fwd_planes: x and w must be 16-byte aligned");
  const int64_t P64 = static_cast<int64_t>(B) * H * W;
  if (P64 * c_in >= (int64_t{1} << 31)) return bad("conv3x3_fwd_planes: tensor too large");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int tw = W % 32 == 0 ? 32 : 16;
  if (c_in == 32)
    conv_res_planes_launch<2>(B, H, W, x, w, bias, act, scale, n_planes, q, tw, st);
  else
    conv_res_planes_launch<3>(B, H, W, x, w, bias, act, scale, n_planes, q, tw, st);
  return launched("conv3x3_fwd_planes");
}

int qnn_conv3x3_fwd_pool(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t c_in, const uint16_t* w,
                         const float* bias, int32_t c_out, int32_t act, uint16_t* y, uint16_t* pool,
                         void* hip_stream) {
  if (B < 1 || H < 2 || W < 2 || !x || !w || !y || !pool) return bad("conv3x3_fwd_pool: bad size or null pointer");
  if ((H | W) & 1) return bad("conv3x3_fwd_pool: H and W must be even");
  if (c_in < 16 || c_in % 16 || c_out < 32 || c_out % 32) return bad("conv3x3_fwd_pool: c_in % 16, c_out % 32");
  if (act != QNN_ACT_NONE && act != QNN_ACT_LEAKY) return bad("conv3x3_fwd_pool: unknown activation");
  if (!a16(x) || !a16(w) || !a16(y) || !a16(pool)) return bad("conv3x3_fwd_pool: tensors must be 16-byte aligned");
  const int64_t P64 = static_cast<int64_t>(B) * H * W;
  if (P64 * (c_in > c_out ? c_in : c_out) >= (int64_t{1} << 31)) return bad("conv3x3_fwd_pool: tensor too large");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // pooled in the resident-weight kernel's epilogue where that kernel runs
  // (the same choice as qnn_conv3x3_fwd), else the two separate calls
  {
    const int tw = W % 32 == 0 ? 32 : 16;
    const int64_t tiles = static_cast<int64_t>(B) * (W / tw) * ((H + 256 / tw - 1) / (256 / tw));
    const bool narrow = c_out == 32;
    const bool wide = c_out == 64 && (c_in == 32 || c_in == 64) && tiles >= 256;
    if ((narrow || wide) && conv_res(B, H, W, x, c_in, w, bias, act, nullptr, y, false, c_out, c_out, c_out,
                                     c_in == 64 ? 2 : 1, tw, 1.0f, st, pool))
      return launched("conv3x3_fwd_pool");
  }
  const int rc = qnn_conv3x3_fwd(B, H, W, x, c_in, w, bias, c_out, act, y, 0, c_out, c_out, hip_stream);
  if (rc != QNN_OK) return rc;
  return qnn_avgpool2(B, H, W, c_out, y, pool, hip_stream);
}

int qnn_conv3x3_flip(const uint16_t* w, int32_t c_out, int32_t c_in, uint16_t* wt, void* hip_stream) {
  if (!w || !wt || c_out < 1 || c_in < 1) return bad("conv3x3_flip: bad size or null pointer");
  const int64_t n = static_cast<int64_t>(c_out) * 9 * c_in;
  hipLaunchKernelGGL(flip_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), w, c_out, c_in, wt);
  return launched("conv3x3_flip");
}

int64_t qnn_wgrad_work_floats(int32_t B, int32_t H, int32_t W, int32_t c_in, int32_t c_out) {
  const int64_t P = static_cast<int64_t>(B) * H * W;
  if (P < 1 || P >= (int64_t{1} << 31) || c_in < 1 || c_out < 32) return 0;
  const int64_t old_split = (P + kWgradPixelsPerBlock - 1) / kWgradPixelsPerBlock;
  int a, nsplit, pps;
  wgrad_split(static_cast<int>(P), c_in, c_out, a, nsplit, pps);
  const int64_t most = nsplit > old_split ? nsplit : old_split;
  return most * c_out * (9 * static_cast<int64_t>(c_in) + 1);
}

int qnn_conv3x3_wgrad(int32_t B, int32_t H, int32_t W, const uint16_t* x, int32_t c_in, const uint16_t* dy,
                      int32_t c_out, float* dw, float* dbias, float* work, void* hip_stream) {
  if (B < 1 || H < 1 || W < 1 || !x || !dy || !dw || !work) return bad("conv3x3_wgrad: bad size or null pointer");
  if (c_in < 16 || c_in % 16 || c_out < 32 || c_out % 32) return bad("conv3x3_wgrad: c_in % 16, c_out % 32");
  const int64_t P64 = static_cast<int64_t>(B) * H * W;
  if (P64 * (c_in > c_out ? c_in : c_out) >= (int64_t{1} << 31)) return bad("conv3x3_wgrad: tensor too large");
  const int P = static_cast<int>(P64);
  const int K = 9 * c_in;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int nsplit;
  float* part = work;
  float* bpart;
  if (a16(x) && a16(dy) && W % 8 == 0) {
    int a, pps;
    wgrad_split(P, c_in, c_out, a, nsplit, pps);
    bpart = work + static_cast<int64_t>(nsplit) * c_out * K;
    dim3 g(c_out / (32 * a), (K + 127) / 128, nsplit);
    if (a == 2)
      hipLaunchKernelGGL((wgrad_lds_kernel<2>), g, dim3(256), 0, st, P, H, W, x, c_in, dy, c_out, pps, part, dbias ? bpart : nullptr);
    else
      hipLaunchKernelGGL((wgrad_lds_kernel<1>), g, dim3(256), 0, st, P, H, W, x, c_in, dy, c_out, pps, part, dbias ? bpart : nullptr);
  } else {
    nsplit = (P + kWgradPixelsPerBlock - 1) / kWgradPixelsPerBlock;
    bpart = work + static_cast<int64_t>(nsplit) * c_out * K;
    if (W % 16 == 0)
      hipLaunchKernelGGL((wgrad_kernel<true>), dim3(c_out / 32, (K + 31) / 32, nsplit), dim3(256), 0, st, P, H, W, x, c_in, dy, c_out, part, dbias ? bpart : nullptr);
    else
      hipLaunchKernelGGL((wgrad_kernel<false>), dim3(c_out / 32, (K + 31) / 32, nsplit), dim3(256), 0, st, P, H, W, x, c_in, dy, c_out, part, dbias ? bpart : nullptr);
  }
  // the partial sums, weights and bias in one pass (a fixed order, so the
  // result is the same on every call)
  const int64_t n = static_cast<int64_t>(c_out) * K;
  const int nb = dbias ? c_out : 0;
  const int G = nsplit < 16 ? nsplit : 16;
  hipLaunchKernelGGL(wgrad_sum_kernel, dim3(static_cast<unsigned>((n + nb + 63) / 64)), dim3(256), 0, st, part, bpart,
                     nsplit, G, n, nb, dw, dbias);
  return launched("conv3x3_wgrad");
}

int qnn_leaky_bwd(int64_t n, const uint16_t* y, const uint16_t* dy, uint16_t* dz, void* hip_stream) {
  if (n < 0 || !y || !dy || !dz) return bad("leaky_bwd: bad size or null pointer");
  if (n % 8 == 0 && a16(y) && a16(dy) && a16(dz)) {
    hipLaunchKernelGGL(leaky_bwd_v8_kernel, dim3(grid_for(n / 8)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n / 8, y, dy, dz);
    return launched("leaky_bwd");
  }
  hipLaunchKernelGGL(leaky_bwd_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, y, dy, dz);
  return launched("leaky_bwd");
}

int qnn_add(int64_t n, const uint16_t* a, const uint16_t* b, uint16_t* y, void* hip_stream) {
  if (n < 0 || !a || !b || !y) return bad("add: bad size or null pointer");
  if (n % 8 == 0 && a16(a) && a16(b) && a16(y)) {
    hipLaunchKernelGGL(add_v8_kernel, dim3(grid_for(n / 8)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n / 8, a, b, y);
    return launched("add");
  }
  hipLaunchKernelGGL(add_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, a, b, y);
  return launched("add");
}

int qnn_avgpool2(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* x, uint16_t* y, void* hip_stream) {
  if (B < 1 || H < 2 || W < 2 || (H | W) & 1 || C < 1 || !x || !y) return bad("avgpool2: bad size or null pointer");
  const int64_t n = static_cast<int64_t>(B) * (H / 2) * (W / 2) * C;
  if (C % 8 == 0 && a16(x) && a16(y)) {
    hipLaunchKernelGGL(avgpool2_v8_kernel, dim3(grid_for(n / 8)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, H, W, C, x, y);
    return launched("avgpool2");
  }
  hipLaunchKernelGGL(avgpool2_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, H, W, C, x, y);
  return launched("avgpool2");
}

int qnn_avgpool2_bwd(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t* dy, uint16_t* dx, int32_t accumulate,
                     void* hip_stream) {
  if (B < 1 || H < 2 || W < 2 || (H | W) & 1 || C < 1 || !dy || !dx) return bad("avgpool2_bwd: bad size or null pointer");
  const int64_t n = static_cast<int64_t>(B) * H * W * C;
  if (C % 8 == 0 && a16(dy) && a16(dx)) {
    hipLaunchKernelGGL(avgpool2_bwd_v8_kernel, dim3(grid_for(n / 32)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, H, W, C, dy, dx, accumulate);
    return launched("avgpool2_bwd");
  }
  hipLaunchKernelGGL(avgpool2_bwd_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, H, W, C, dy, dx, accumulate);
  return launched("avgpool2_bwd");
}

int qnn_upsample2(int32_t B, int32_t h, int32_t w, int32_t C, const uint16_t* x, uint16_t* y, void* hip_stream) {
  if (B < 1 || h < 1 || w < 1 || C < 1 || !x || !y) return bad("upsample2: bad size or null pointer");
  const int64_t n = static_cast<int64_t>(B) * 4 * h * w * C;
  if (C % 8 == 0 && a16(x) && a16(y)) {
    hipLaunchKernelGGL(upsample2_v8_kernel, dim3(grid_for(n / 32)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, h, w, C, x, y);
    return launched("upsample2");
  }
  hipLaunchKernelGGL(upsample2_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, h, w, C, x, y);
  return launched("upsample2");
}

int qnn_upsample2_bwd(int32_t B, int32_t h, int32_t w, int32_t C, const uint16_t* dy, uint16_t* dx, void* hip_stream) {
  if (B < 1 || h < 1 || w < 1 || C < 1 || !dy || !dx) return bad("upsample2_bwd: bad size or null pointer");
  const int64_t n = static_cast<int64_t>(B) * h * w * C;
  if (C % 8 == 0 && a16(dy) && a16(dx)) {
    hipLaunchKernelGGL(upsample2_bwd_v8_kernel, dim3(grid_for(n / 8)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, h, w, C, dy, dx);
    return launched("upsample2_bwd");
  }
  hipLaunchKernelGGL(upsample2_bwd_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, h, w, C, dy, dx);
  return launched("upsample2_bwd");
}

int qnn_absmax(int32_t B, int32_t H, int32_t W, const float* q, const int32_t* idx, float* scale, void* hip_stream) {
  if (B < 1 || H < 1 || W < 1 || !q || !scale) return bad("absmax: bad argument");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int64_t n = 6 * static_cast<int64_t>(H) * W;
  const int nb = static_cast<int>(std::min<int64_t>((n + 255) / 256, 256));
  hipLaunchKernelGGL(absmax_init_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, scale);
  // 16-byte loads when every sample's planes start 16-byte aligned
  if (n % 4 == 0 && a16(q))
    hipLaunchKernelGGL(absmax_kernel<true>, dim3(nb, B), dim3(256), 0, st, H, W, q, idx, scale);
  else
    hipLaunchKernelGGL(absmax_kernel<false>, dim3(nb, B), dim3(256), 0, st, H, W, q, idx, scale);
  hipLaunchKernelGGL(absmax_fix_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, scale);
  return launched("absmax");
}

int qnn_pack_input(int32_t B, int32_t H, int32_t W, const float* q, const int32_t* idx_q, const float* n,
                   const int32_t* idx_n, const float* scale, float n_shift, float n_scale, int32_t shift,
                   uint16_t* x, void* hip_stream) {
  if (B < 1 || H < 1 || W < 1 || !q || !n || !scale || !x || !(n_scale != 0.0f)) return bad("pack_input: bad argument");
  if (!a16(x)) return bad("pack_input: x must be 16-byte aligned");
  if (int64_t{6} * H * W >= (int64_t{1} << 31)) return bad("pack_input: lattice too large");
  const int64_t total = static_cast<int64_t>(B) * H * W;
  const int dx = (shift % W + W) % W, dy = (shift % H + H) % H;
  hipLaunchKernelGGL(pack_input_kernel, dim3(grid_for(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, H, W, q, idx_q, n, idx_n, scale, n_shift, n_scale, dx, dy, x);
  return launched("pack_input");
}

int qnn_unpack_output(int32_t B, int32_t H, int32_t W, const float* y, int32_t y_ld, const float* scale, float* q,
                      void* hip_stream) {
  if (B < 1 || H < 1 || W < 1 || !y || !scale || !q || y_ld < 6) return bad("unpack_output: bad argument");
  const int64_t total = static_cast<int64_t>(B) * H * W;
  hipLaunchKernelGGL(unpack_output_kernel, dim3(grid_for(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), B, H, W, y, y_ld, scale, q);
  return launched("unpack_output");
}

int qnn_rel_l2(int32_t B, int32_t H, int32_t W, const float* pred, int32_t pred_ld, const float* target,
               const int32_t* idx_t, const float* scale, uint16_t* dpred, int32_t d_ld, double* loss_out,
               double* per_sample, double* work, void* hip_stream) {
  if (B < 1 || B > 1024 || H < 1 || W < 1 || !pred || !target || !loss_out || !work || pred_ld < 6)
    return bad("rel_l2: bad argument");
  if (dpred && d_ld < 6) return bad("rel_l2: d_ld < 6");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int nb = 31;   // partial blocks per sample: 2*B*nb + 2*B <= 64*B doubles of work
  hipLaunchKernelGGL(rel_l2_partial_kernel, dim3(nb, B), dim3(256), 0, st, H, W, pred, pred_ld, target, idx_t, scale, work);
  hipLaunchKernelGGL(rel_l2_final_kernel, dim3(1), dim3(256), 0, st, B, nb, work, loss_out, per_sample);
  if (dpred) {
    const int64_t pixels = static_cast<int64_t>(B) * H * W;
    if (d_ld % 8 == 0 && a16(dpred))
      hipLaunchKernelGGL((rel_l2_grad_kernel<true>), dim3(grid_for(pixels)), dim3(256), 0, st, B, H, W, nb, pred, pred_ld, target, idx_t, scale, work, dpred, d_ld);
    else
      hipLaunchKernelGGL((rel_l2_grad_kernel<false>), dim3(grid_for(pixels)), dim3(256), 0, st, B, H, W, nb, pred, pred_ld, target, idx_t, scale, work, dpred, d_ld);
  }
  return launched("rel_l2");
}

int qnn_adam(int64_t n, float* p, float* m, float* v, const float* g, uint16_t* p_bf16, float lr, float b1, float b2,
             float eps, int32_t t, void* hip_stream) {
  if (n < 0 || !p || !m || !v || !g || t < 1) return bad("adam: bad argument");
  const float c1 = 1.0f - powf(b1, static_cast<float>(t));
  const float c2 = 1.0f - powf(b2, static_cast<float>(t));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, p, m, v, g, p_bf16, lr, b1, b2, eps, c1, c2);
  return launched("adam");
}

int64_t qnn_compare_work_doubles(int32_t B) { return B < 1 ? 0 : static_cast<int64_t>(B) * kCompareBlocks * 3; }

int qnn_compare(int32_t B, int64_t m, const float* a, const float* r, double* rel, double* en, double* work,
                void* hip_stream) {
  if (B < 1 || B > 65535 || m < 1 || !a || !r || !rel || !en || !work) return bad("compare: bad argument");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(compare_kernel, dim3(kCompareBlocks, B), dim3(256), 0, st, m, a, r, work);
  hipLaunchKernelGGL(compare_final_kernel, dim3((B + 255) / 256), dim3(256), 0, st, B, work, rel, en);
  return launched("compare");
}

int qnn_to_bf16(int64_t n, const float* x, uint16_t* y, void* hip_stream) {
  if (n < 0 || !x || !y) return bad("to_bf16: bad argument");
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n, x, y);
  return launched("to_bf16");
}

}  // extern "C"
