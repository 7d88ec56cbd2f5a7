// Learned pilot: a six-layer 3x3 convolutional network (2 -> 32 -> ... -> 32
// -> 1 channels, ReLU after the first five, residual output pilot = z - f)
// that stands in for stage 1 as the estimate driving the Wiener stage.
//
// All activations are bfloat16 NHWC with 32 channels (64 B per pixel; the
// two input channels and the single output channel are zero-padded), so every
// layer is the same 32 -> 32 convolution.  A convolution is an implicit GEMM
// on the bf16 matrix cores: for each 16-pixel row segment and each of the 9
// taps, D[out channel][pixel] += W_tap[out][in] * X[in][pixel shifted by the
// tap] with v_mfma_f32_16x16x32_bf16 (K = the 32 input channels of one tap),
// fp32 accumulation, and a fused epilogue (bias + ReLU, or the residual
// output, or the ReLU mask of the backward pass).  The input-gradient pass is
// the same kernel with flipped, transposed weights.  The weight gradient is a
// GEMM over pixels (K = 32 pixels of a tile row per MFMA) into per-workgroup
// partial sums that a second kernel adds in a fixed order.
#include <hip/hip_runtime.h>

#include "common.h"
#include "pilot.h"

namespace gbm3d {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kC = 32;          // channels of every activation tensor
constexpr int kTaps = 9;
constexpr int kTileY = 8, kTileX = 32;
constexpr int kWmat = kTaps * kC * kC;   // one packed weight set per layer

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__host__ __device__ inline int conv_items(int N, int H, int W) {
  return N * ((H + kTileY - 1) / kTileY) * ((W + kTileX - 1) / kTileX);
}

// ---------------------------------------------------------------------------
// convolution 32 -> 32, 3x3, zero "same" padding
// MODE 0: forward, + bias, ReLU, bf16 out
// MODE 1: forward last layer: f = channel 0 + bias; pilot = z - f (fp32 / u16)
// MODE 2: input gradient: out = conv * (mask > 0), bf16 out
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void conv_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wpk,
                                                   const float* __restrict__ bias, const uint16_t* __restrict__ mask,
                                                   uint16_t* __restrict__ out, const uint16_t* __restrict__ noisy,
                                                   float* __restrict__ pilot_f32, uint16_t* __restrict__ pilot_u16,
                                                   int N, int H, int W) {
  __shared__ __align__(16) uint16_t tile[kTileY + 2][kTileX + 2][kC];
  const int tx_n = (W + kTileX - 1) / kTileX, ty_n = (H + kTileY - 1) / kTileY;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;

  // A operands (weights) for all taps, both 16-channel output halves
  bf16x8 A[kTaps][2];
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h)
      A[t][h] = as_bf16x8(*reinterpret_cast<const uint4*>(wpk + (t * kC + h * 16 + col) * kC + 8 * grp));
  float b0[4], b1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    b0[i] = bias ? bias[4 * grp + i] : 0.0f;
    b1[i] = bias ? bias[16 + 4 * grp + i] : 0.0f;
  }

  const int total = conv_items(N, H, W);
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int n = item / (tx_n * ty_n);
    const int rem = item - n * tx_n * ty_n;
    const int y0 = (rem / tx_n) * kTileY, x0 = (rem % tx_n) * kTileX;
    const uint4* src = reinterpret_cast<const uint4*>(in) + static_cast<size_t>(n) * H * W * 4;
    uint4* dst_t = reinterpret_cast<uint4*>(&tile[0][0][0]);
    for (int i = threadIdx.x; i < (kTileY + 2) * (kTileX + 2) * 4; i += blockDim.x) {
      const int pix = i >> 2, part = i & 3;
      const int r = pix / (kTileX + 2), c = pix - r * (kTileX + 2);
      const int y = y0 - 1 + r, x = x0 - 1 + c;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (y >= 0 && y < H && x >= 0 && x < W) v = src[(static_cast<size_t>(y) * W + x) * 4 + part];
      dst_t[i] = v;
    }
    __syncthreads();

#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const int row = 2 * wave + (bi >> 1), xoff = (bi & 1) * 16;
      f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < kTaps; ++t) {
        const int ky = t / 3, kx = t % 3;
        const bf16x8 B = as_bf16x8(*reinterpret_cast<const uint4*>(&tile[row + ky][xoff + col + kx][8 * grp]));
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[t][0], B, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[t][1], B, acc1, 0, 0, 0);
      }
      // lane holds channels 4*grp + i (acc0) and 16 + 4*grp + i (acc1) of pixel (y, x)
      const int y = y0 + row, x = x0 + xoff + col;
      if (y < H && x < W) {
        const size_t p = (static_cast<size_t>(n) * H + y) * W + x;
        if constexpr (MODE == 0 || MODE == 2) {
          float v0[4], v1[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            v0[i] = acc0[i];
            v1[i] = acc1[i];
          }
          if constexpr (MODE == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              v0[i] = fmaxf(v0[i] + b0[i], 0.0f);
              v1[i] = fmaxf(v1[i] + b1[i], 0.0f);
            }
          } else {
            const uint2 m0 = *reinterpret_cast<const uint2*>(mask + p * kC + 4 * grp);
            const uint2 m1 = *reinterpret_cast<const uint2*>(mask + p * kC + 16 + 4 * grp);
            const uint16_t* mm0 = reinterpret_cast<const uint16_t*>(&m0);
            const uint16_t* mm1 = reinterpret_cast<const uint16_t*>(&m1);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              v0[i] = bf2f(mm0[i]) > 0.0f ? v0[i] : 0.0f;
              v1[i] = bf2f(mm1[i]) > 0.0f ? v1[i] : 0.0f;
            }
          }
          uint2 o0, o1;
          o0.x = f2bf(v0[0]) | (static_cast<uint32_t>(f2bf(v0[1])) << 16);
          o0.y = f2bf(v0[2]) | (static_cast<uint32_t>(f2bf(v0[3])) << 16);
          o1.x = f2bf(v1[0]) | (static_cast<uint32_t>(f2bf(v1[1])) << 16);
          o1.y = f2bf(v1[2]) | (static_cast<uint32_t>(f2bf(v1[3])) << 16);
          *reinterpret_cast<uint2*>(out + p * kC + 4 * grp) = o0;
          *reinterpret_cast<uint2*>(out + p * kC + 16 + 4 * grp) = o1;
        } else {
          if (grp == 0) {  // channel 0 sits in acc0[0] of lanes 0..15
            const float f = acc0[0] + b0[0];
            const float pil = static_cast<float>(noisy[p]) * (1.0f / 65535.0f) - f;
            if (pilot_f32) pilot_f32[p] = pil;
            if (pilot_u16) {
              const double d = static_cast<double>(fminf(fmaxf(pil, 0.0f), 1.0f));
              pilot_u16[p] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// fused inference: the six layers of one 16 x 32 output tile in one
// workgroup, every intermediate activation in LDS.  Layer l is evaluated on
// the tile grown by 5 - l pixels on each side (the receptive field of the
// layers after it), so a tile reads only its 28 x 44 window of the noisy
// image and writes only its pilot pixels.  Positions outside the image are
// zero in every layer's output, as the zero "same" padding of the per-layer
// form has them.
//
// One wave per SIMD, each software-pipelining its pixel blocks (the operands
// of the next block are read from LDS and the previous block's results
// written while the current block's products run); the next layer's weights
// are loaded into registers while the current layer computes.
//
// LDS: the input window as (z, sigma) bf16 pairs, and two ping-pong
// activation buffers (layers 0, 2, 4 | 1, 3) of 64 B per pixel.  A pixel's
// 16-byte octet o holds channels 4o .. 4o+3 and 16+4o .. 16+4o+3: exactly
// the eight values one lane holds after the products (output rows 4 grp + i
// of both 16-channel halves), so a lane writes its pixel's results with one
// 16-byte store, and the next layer takes its K dimension in that order (its
// A operands are gathered to match).  Octet o of a pixel in region column x
// sits at slot o ^ ((x >> 1) & 3): the eight consecutive pixels that one
// 128-byte LDS cycle of a 16-byte access serves then hit eight different
// 16-byte bank groups.  A layer's output pixels are taken in raster order,
// 16 per MFMA column block; layer 0 packs its 9 taps x 2 input channels into
// one K = 32 product, and layer 5 computes one 16-channel half (its single
// output channel is row 0).  Bias enters as the initial accumulator.  Lanes
// of a region's last block that fall past its end store into a spare pixel
// at the end of the buffer, so the stores need no branch.
// ---------------------------------------------------------------------------
constexpr int kFY = 16, kFX = 32;                   // output tile
constexpr int kFWaves = 4, kFThreads = 64 * kFWaves;
constexpr int kZY = kFY + 2 * kPilotLayers, kZX = kFX + 2 * kPilotLayers;  // input window
__host__ __device__ constexpr int f_ry(int l) { return kFY + 2 * (kPilotLayers - 1 - l); }
__host__ __device__ constexpr int f_rx(int l) { return kFX + 2 * (kPilotLayers - 1 - l); }
constexpr int kFBufA = f_ry(0) * f_rx(0), kFBufB = f_ry(1) * f_rx(1);  // pixels
static_assert(kFBufA >= f_ry(2) * f_rx(2) && kFBufB >= f_ry(3) * f_rx(3), "ping-pong sizes");
static_assert(kFX % 16 == 0, "output rows are whole 16-pixel blocks");

__host__ __device__ inline int fused_tiles(int N, int H, int W) {
  return N * ((H + kFY - 1) / kFY) * ((W + kFX - 1) / kFX);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));  // round to nearest even
}

// A operands of one layer (HALVES = 1: the first 16 output channels only)
template <int HALVES>
struct FusedW {
  bf16x8 A[kTaps][HALVES];
};

template <int HALVES>
__device__ __forceinline__ void fused_load_w(const uint16_t* __restrict__ wf, int l, int col, int grp,
                                             FusedW<HALVES>& w) {
  // global address space, and opaque to the optimiser, so the loads stay
  // where they are issued instead of being hoisted out of the tile loop (the
  // weights of all layers at once do not fit in the registers)
  typedef const uint16_t __attribute__((address_space(1))) * gptr;
  gptr wl = (gptr)(wf + static_cast<size_t>(l) * kWmat);
  asm volatile("" : "+s"(wl));
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int h = 0; h < HALVES; ++h) {
      // K element 8 grp + e is input channel 4 grp + e (e < 4) or 16 + 4 grp + e - 4
      gptr row = wl + (t * kC + h * 16 + col) * kC;
      typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
      typedef const u32x2 __attribute__((address_space(1))) * gptr2;
      const u32x2 lo = *(gptr2)(row + 4 * grp);
      const u32x2 hi = *(gptr2)(row + 16 + 4 * grp);
      w.A[t][h] = as_bf16x8(make_uint4(lo.x, lo.y, hi.x, hi.y));
    }
}

// ReLU (all zero when keep is false: outside the image), bf16, into octet
// grp of pixel i (region column c).  The ReLU acts on the rounded bf16 pairs
// as signed 16-bit maxima: rounding keeps the sign, so this equals rounding
// the ReLU of the float sums.
__device__ __forceinline__ void fused_store(uint4* __restrict__ out, int i, int c, int grp, f32x4 a0, f32x4 a1,
                                            bool keep) {
  typedef short s16x2 __attribute__((ext_vector_type(2)));
  const s16x2 zero = {0, 0};
  uint32_t q[4] = {pack_bf16(a0[0], a0[1]), pack_bf16(a0[2], a0[3]), pack_bf16(a1[0], a1[1]), pack_bf16(a1[2], a1[3])};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    q[k] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, q[k]), zero));
    q[k] = keep ? q[k] : 0u;
  }
  out[i * 4 + (grp ^ ((c >> 1) & 3))] = make_uint4(q[0], q[1], q[2], q[3]);
}

struct Taps9 {
  bf16x8 v[kTaps];
};

// A 3x3 layer over the NG pixel blocks g = wave, wave + kFWaves, ... of its
// region (row width RX, input row stride RX + 2): after the products of tap
// t of block g are issued, tap t of block g + kFWaves is read into the same
// registers, and the results of block g are stored while the products of
// the next block run.
template <int RX, int NP, int HALVES, class Store>
__device__ __forceinline__ void fused_conv(const uint4* __restrict__ in, const FusedW<HALVES>& w, f32x4 b0, f32x4 b1,
                                           Store&& store) {
  constexpr int S = RX + 2, NG = (NP + 15) / 16;
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  int g = threadIdx.x >> 6;
  if (g >= NG) return;
  auto addr = [&](int gg, int (&e)[3]) {
    const int i = min(gg * 16 + col, NP - 1), r = i / RX, c = i - r * RX, pb = r * S + c;
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) e[kx] = (pb + kx) * 4 + (grp ^ (((c + kx) >> 1) & 3));
  };
  Taps9 B;
  {
    int e[3];
    addr(g, e);
#pragma unroll
    for (int t = 0; t < kTaps; ++t) B.v[t] = as_bf16x8(in[e[t % 3] + (t / 3) * S * 4]);
  }
  f32x4 p0, p1;
  {
    int e[3];
    addr(min(g + kFWaves, NG - 1), e);
    p0 = b0;
    p1 = b1;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      p0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.A[t][0], B.v[t], p0, 0, 0, 0);
      if constexpr (HALVES == 2) p1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.A[t][HALVES - 1], B.v[t], p1, 0, 0, 0);
      B.v[t] = as_bf16x8(in[e[t % 3] + (t / 3) * S * 4]);
    }
    g += kFWaves;
  }
  for (; g + kFWaves < NG; g += kFWaves) {
    int e[3];
    addr(g + kFWaves, e);
    f32x4 a0 = b0, a1 = b1;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.A[t][0], B.v[t], a0, 0, 0, 0);
      if constexpr (HALVES == 2) a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.A[t][HALVES - 1], B.v[t], a1, 0, 0, 0);
      B.v[t] = as_bf16x8(in[e[t % 3] + (t / 3) * S * 4]);
    }
    store(g - kFWaves, p0, p1);
    p0 = a0;
    p1 = a1;
  }
  if (g < NG) {
    f32x4 a0 = b0, a1 = b1;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.A[t][0], B.v[t], a0, 0, 0, 0);
      if constexpr (HALVES == 2) a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.A[t][HALVES - 1], B.v[t], a1, 0, 0, 0);
    }
    store(g - kFWaves, p0, p1);
    store(g, a0, a1);
  } else {
    store(g - kFWaves, p0, p1);
  }
}

// layers 1 .. 4: 32 -> 32, ReLU
template <int L, int DUMMY = (L & 1) ? kFBufB : kFBufA>
__device__ __forceinline__ void fused_mid(const uint4* __restrict__ in, uint4* __restrict__ out,
                                          const FusedW<2>& w, const f32x4* __restrict__ bias4, bool border, int y0,
                                          int x0, int H, int W) {
  constexpr int RX = f_rx(L), NP = f_ry(L) * RX, G = kPilotLayers - 1 - L;
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  fused_conv<RX, NP, 2>(in, w, bias4[L * 8 + grp], bias4[L * 8 + 4 + grp], [&](int g, f32x4 a0, f32x4 a1) {
    const int iv = g * 16 + col, i = min(iv, NP - 1);
    const int r = i / RX, c = i - r * RX;
    bool keep = true;
    if (border) {
      const int y = y0 - G + r, x = x0 - G + c;
      keep = static_cast<unsigned>(y) < static_cast<unsigned>(H) && static_cast<unsigned>(x) < static_cast<unsigned>(W);
    }
    fused_store(out, iv < NP ? i : DUMMY, c, grp, a0, a1, keep);
  });
}

__global__ __launch_bounds__(kFThreads) void fused_infer_kernel(const uint16_t* __restrict__ noisy,
                                                                const float* __restrict__ sigma,
                                                                const uint16_t* __restrict__ wf,
                                                                const float* __restrict__ bias, int N, int H, int W,
                                                                float* __restrict__ pilot_f32,
                                                                uint16_t* __restrict__ pilot_u16) {
  __shared__ __align__(16) uint4 bufA[(kFBufA + 1) * 4];
  __shared__ __align__(16) uint4 bufB[(kFBufB + 1) * 4];
  __shared__ uint32_t zb[kZY * kZX];
  __shared__ uint16_t zc[2][kFY * kFX];  // the tile's own noisy pixels (exact), current / next tile
  __shared__ f32x4 bias4[kPilotLayers * 8];  // [layer][half * 4 + grp]: output channels 16 half + 4 grp + 0..3

  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  const int tx_n = (W + kFX - 1) / kFX, ty_n = (H + kFY - 1) / kFY;
  const int total = fused_tiles(N, H, W);

  if (threadIdx.x < kPilotLayers * kC) {
    const int l = threadIdx.x / kC, ch = threadIdx.x % kC;
    bias4[l * 8 + ch / 4][ch % 4] = bias[l * kC + ch];
  }
  // layer 0 operands: K index 8 grp + e is tap (8 grp + e) / 2, input channel e % 2 (taps past 8 are zero)
  FusedW<2> w0;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int t = (8 * grp + e) >> 1, ci = e & 1;
      w0.A[0][h][e] = t < kTaps ? __builtin_bit_cast(__bf16, wf[(t * kC + h * 16 + col) * kC + ci]) : __bf16(0.0f);
    }
  int zoff[4];  // window offset of the taps this lane's K octet holds (taps past 8: any finite entry)
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int t = 4 * grp + j;
    zoff[j] = t < kTaps ? (t / 3) * kZX + t % 3 : 0;
  }
  // the next layer's operands are loaded while the current layer computes
  FusedW<2> wa, wb;
  FusedW<1> w5;

  // the window of a tile: 28 x 44 (z, sigma) pairs, zero outside the image
  constexpr int kZPer = (kZY * kZX + kFThreads - 1) / kFThreads;
  uint32_t zr[kZPer];
  uint16_t cr[kZPer];
  auto fetch = [&](int item) {
    const int n = item / (tx_n * ty_n), rem = item - n * tx_n * ty_n;
    const int y0 = (rem / tx_n) * kFY - kPilotLayers, x0 = (rem % tx_n) * kFX - kPilotLayers;
    const uint32_t s = f2bf(sigma[n]);
    const uint16_t* src = noisy + static_cast<size_t>(n) * H * W;
#pragma unroll
    for (int k = 0; k < kZPer; ++k) {
      const int pix = threadIdx.x + k * kFThreads;
      const int r = pix / kZX, c = pix - r * kZX, y = y0 + r, x = x0 + c;
      uint16_t v = 0;
      const bool in = pix < kZY * kZX && y >= 0 && y < H && x >= 0 && x < W;
      if (in) v = src[static_cast<size_t>(y) * W + x];
      cr[k] = v;
      zr[k] = in ? (static_cast<uint32_t>(f2bf(static_cast<float>(v) * (1.0f / 65535.0f))) | (s << 16)) : 0u;
    }
  };
  auto park = [&](int buf) {
#pragma unroll
    for (int k = 0; k < kZPer; ++k) {
      const int pix = threadIdx.x + k * kFThreads;
      if (pix < kZY * kZX) {
        zb[pix] = zr[k];
        const int r = pix / kZX - kPilotLayers, c = pix % kZX - kPilotLayers;
        if (r >= 0 && r < kFY && c >= 0 && c < kFX) zc[buf][r * kFX + c] = cr[k];
      }
    }
  };

  int buf = 0;
  if (blockIdx.x < total) {
    fetch(blockIdx.x);
    park(0);
  }
  __syncthreads();
  for (int item = blockIdx.x; item < total; item += gridDim.x, buf ^= 1) {
    const int n = item / (tx_n * ty_n), rem = item - n * tx_n * ty_n;
    const int y0 = (rem / tx_n) * kFY, x0 = (rem % tx_n) * kFX;
    const bool border = y0 < kPilotLayers || x0 < kPilotLayers || y0 + kFY + kPilotLayers > H ||
                        x0 + kFX + kPilotLayers > W;

    fused_load_w(wf, 1, col, grp, wa);
    {  // layer 0: 2 -> 32 from the window, im2col over the K dimension; four blocks per step
      constexpr int RX = f_rx(0), NP = f_ry(0) * RX, NG = (NP + 15) / 16, G = kPilotLayers - 1;
      constexpr int kSteps = (NG + 4 * kFWaves - 1) / (4 * kFWaves);
      const f32x4 b0 = bias4[grp], b1 = bias4[4 + grp];
      const int wave = threadIdx.x >> 6;
      auto read = [&](int g) {
        const int i = min(g * 16 + col, NP - 1), r = i / RX, pb = r * kZX + (i - r * RX);
        return as_bf16x8(make_uint4(zb[pb + zoff[0]], zb[pb + zoff[1]], zb[pb + zoff[2]], zb[pb + zoff[3]]));
      };
      bf16x8 Bz[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) Bz[q] = read(wave + q * kFWaves);
      for (int st = 0; st < kSteps; ++st) {
        const int g0 = st * 4 * kFWaves + wave;
        f32x4 a0[4], a1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a0[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0.A[0][0], Bz[q], b0, 0, 0, 0);
          a1[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0.A[0][1], Bz[q], b1, 0, 0, 0);
          if (st + 1 < kSteps) Bz[q] = read(g0 + (4 + q) * kFWaves);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = (g0 + q * kFWaves) * 16 + col;
          if (i < NP) {
            const int r = i / RX, c = i - r * RX;
            bool keep = true;
            if (border) {
              const int y = y0 - G + r, x = x0 - G + c;
              keep = static_cast<unsigned>(y) < static_cast<unsigned>(H) &&
                     static_cast<unsigned>(x) < static_cast<unsigned>(W);
            }
            fused_store(bufA, i, c, grp, a0[q], a1[q], keep);
          }
        }
      }
    }
    __syncthreads();
    const int next = item + static_cast<int>(gridDim.x);
    if (next < total) fetch(next);  // in flight during layers 1 .. 4
    fused_load_w(wf, 2, col, grp, wb);
    fused_mid<1>(bufA, bufB, wa, bias4, border, y0, x0, H, W);
    __syncthreads();
    fused_load_w(wf, 3, col, grp, wa);
    fused_mid<2>(bufB, bufA, wb, bias4, border, y0, x0, H, W);
    __syncthreads();
    fused_load_w(wf, 4, col, grp, wb);
    fused_mid<3>(bufA, bufB, wa, bias4, border, y0, x0, H, W);
    __syncthreads();
    fused_load_w(wf, 5, col, grp, w5);
    fused_mid<4>(bufB, bufA, wb, bias4, border, y0, x0, H, W);
    if (next < total) park(buf ^ 1);  // the window buffer is free since layer 0
    __syncthreads();

    {  // layer 5: 32 -> 1 (row 0 of the first half), pilot = z - f
      constexpr int RX = f_rx(5), NP = f_ry(5) * RX;
      const uint16_t* zcur = zc[buf];
      fused_conv<RX, NP, 1>(bufA, w5, bias4[5 * 8 + grp], bias4[5 * 8 + grp], [&](int g, f32x4 a0, f32x4) {
        const int i = g * 16 + col, r = i / RX, c = i - r * RX;
        const int y = y0 + r, x = x0 + c;
        if (grp == 0 && y < H && x < W) {
          const size_t p = (static_cast<size_t>(n) * H + y) * W + x;
          const float pil = static_cast<float>(zcur[i]) * (1.0f / 65535.0f) - a0[0];
          if (pilot_f32) pilot_f32[p] = pil;
          if (pilot_u16) {
            const double d = static_cast<double>(fminf(fmaxf(pil, 0.0f), 1.0f));
            pilot_u16[p] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
          }
        }
      });
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[t][ci][co] = sum_p x[p + off_t][ci] g[p][co], db[co] = sum_p g[p][co]
// per-workgroup partials [grid][kWmat + kC]
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wgrad_kernel(const uint16_t* __restrict__ x, const uint16_t* __restrict__ g,
                                                    int N, int H, int W, float* __restrict__ partial) {
  // channel-major tiles; xs[kx] holds x shifted by kx - 1 columns
  __shared__ __align__(16) uint16_t xs[3][kC][kTileY + 2][kTileX];
  __shared__ __align__(16) uint16_t gs[kC][kTileY][kTileX];
  const int tx_n = (W + kTileX - 1) / kTileX, ty_n = (H + kTileY - 1) / kTileY;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int co_t = wave >> 1, ci_t = wave & 1;
  f32x4 acc[kTaps];
#pragma unroll
  for (int t = 0; t < kTaps; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.0f;  // bias-gradient partial of channel tid % 32 over tile rows tid / 32

  const int total = conv_items(N, H, W);
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int n = item / (tx_n * ty_n);
    const int rem = item - n * tx_n * ty_n;
    const int y0 = (rem / tx_n) * kTileY, x0 = (rem % tx_n) * kTileX;
    const uint16_t* xn = x + static_cast<size_t>(n) * H * W * kC;
    const uint16_t* gn = g + static_cast<size_t>(n) * H * W * kC;
    // x: rows y0-1 .. y0+8, columns x0-1 .. x0+32 (34), scattered into the
    // three shifted copies; a thread moves 8 channels of one pixel, consecutive
    // threads take consecutive pixels (conflict-free LDS stores)
    constexpr int kXPix = (kTileY + 2) * (kTileX + 2);
    for (int i = threadIdx.x; i < kXPix * 4; i += blockDim.x) {
      const int c8 = i / kXPix, pix = i - c8 * kXPix;
      const int r = pix / (kTileX + 2), c = pix - r * (kTileX + 2);
      const int y = y0 - 1 + r, xx = x0 - 1 + c;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (y >= 0 && y < H && xx >= 0 && xx < W) v = *reinterpret_cast<const uint4*>(xn + (static_cast<size_t>(y) * W + xx) * kC + 8 * c8);
      const uint16_t* vv = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int cc = c - kx;  // xs[kx][..][cc] = x[column x0 + cc + kx - 1]
        if (cc >= 0 && cc < kTileX) {
#pragma unroll
          for (int j = 0; j < 8; ++j) xs[kx][8 * c8 + j][r][cc] = vv[j];
        }
      }
    }
    constexpr int kGPix = kTileY * kTileX;
    for (int i = threadIdx.x; i < kGPix * 4; i += blockDim.x) {
      const int c8 = i / kGPix, pix = i - c8 * kGPix;
      const int r = pix / kTileX, c = pix - r * kTileX;
      const int y = y0 + r, xx = x0 + c;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (y < H && xx < W) v = *reinterpret_cast<const uint4*>(gn + (static_cast<size_t>(y) * W + xx) * kC + 8 * c8);
      const uint16_t* vv = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) gs[8 * c8 + j][r][c] = vv[j];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      const int ky = t / 3, kx = t % 3;
#pragma unroll
      for (int r = 0; r < kTileY; ++r) {
        const bf16x8 Aop = as_bf16x8(*reinterpret_cast<const uint4*>(&gs[co_t * 16 + col][r][8 * grp]));
        const bf16x8 Bop = as_bf16x8(*reinterpret_cast<const uint4*>(&xs[kx][ci_t * 16 + col][r + ky][8 * grp]));
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop, Bop, acc[t], 0, 0, 0);
      }
    }
    {  // bias gradient: thread (channel tid % 32, row tid / 32) sums one tile row
      const int ch = threadIdx.x & (kC - 1), r = threadIdx.x >> 5;
      float s = 0.0f;
#pragma unroll 8
      for (int c = 0; c < kTileX; ++c) s += bf2f(gs[ch][r][c]);
      db += s;
    }
    __syncthreads();
  }
  // D[co][ci]: lane holds co = co_t*16 + 4*grp + i, ci = ci_t*16 + col; stored as [t][ci][co]
  float* dst = partial + static_cast<size_t>(blockIdx.x) * (kWmat + kC);
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[(t * kC + ci_t * 16 + col) * kC + co_t * 16 + 4 * grp + i] = acc[t][i];
  __shared__ float dbs[256];
  dbs[threadIdx.x] = db;
  __syncthreads();
  if (threadIdx.x < kC) {
    float s = 0.0f;
    for (int r = 0; r < kTileY; ++r) s += dbs[r * kC + threadIdx.x];
    dst[kWmat + threadIdx.x] = s;
  }
}

// grad (canonical layout of one layer) = sum over workgroups of the partials
__global__ void wgrad_reduce_kernel(const float* __restrict__ partial, int n_part, int ci_n, int co_n,
                                    float* __restrict__ grad) {
  const int n_w = kTaps * ci_n * co_n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_w + co_n) return;
  int src;
  if (i < n_w) {
    const int t = i / (ci_n * co_n), rem = i - t * ci_n * co_n;
    const int ci = rem / co_n, co = rem - ci * co_n;
    src = (t * kC + ci) * kC + co;
  } else {
    src = kWmat + (i - n_w);
  }
  double s = 0.0;
  for (int k = 0; k < n_part; ++k) s += partial[static_cast<size_t>(k) * (kWmat + kC) + src];
  grad[i] = static_cast<float>(s);
}

// network input: channel 0 = z, channel 1 = sigma, the rest zero
__global__ void prep_kernel(const uint16_t* __restrict__ noisy, const float* __restrict__ sigma, int N, int HW,
                            uint16_t* __restrict__ x0) {
  const size_t total = static_cast<size_t>(N) * HW;
  for (size_t p = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; p < total;
       p += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int n = static_cast<int>(p / HW);
    uint4* d = reinterpret_cast<uint4*>(x0 + p * kC);
    const uint32_t z = f2bf(static_cast<float>(noisy[p]) * (1.0f / 65535.0f));
    const uint32_t s = f2bf(sigma[n]);
    d[0] = make_uint4(z | (s << 16), 0, 0, 0);
    d[1] = make_uint4(0, 0, 0, 0);
    d[2] = make_uint4(0, 0, 0, 0);
    d[3] = make_uint4(0, 0, 0, 0);
  }
}

// loss gradient of the (per-image weighted) mean squared error:
// dL/df = -2 w_b (pilot - target) / n with w_b = weight[pixel / hw] (1 if no
// weights), written as channel 0 of a 32-channel bf16 tensor; per-block
// partial sums of the weighted squared error in double.
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ pilot, const float* __restrict__ target,
                                                   const float* __restrict__ weight, size_t hw, size_t n,
                                                   uint16_t* __restrict__ g, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = -2.0f / static_cast<float>(n);
  for (size_t p = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; p < n;
       p += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float w = weight ? weight[p / hw] : 1.0f;
    const float d = pilot[p] - target[p];
    s += static_cast<double>(w) * d * d;
    uint4* dst = reinterpret_cast<uint4*>(g + p * kC);
    dst[0] = make_uint4(f2bf(scale * w * d), 0, 0, 0);
    dst[1] = make_uint4(0, 0, 0, 0);
    dst[2] = make_uint4(0, 0, 0, 0);
    dst[3] = make_uint4(0, 0, 0, 0);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void loss_reduce_kernel(const double* __restrict__ part, int n_part, size_t n, float* __restrict__ loss) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n_part; ++i) s += part[i];
  *loss = static_cast<float>(s / static_cast<double>(n));
}

// packed weights from the float32 master vector: forward [l][t][co][ci],
// backward [l][t'][ci][co] = W[8-t'][ci][co], biases [l][32]; zero padded
__global__ void pack_kernel(const float* __restrict__ master, uint16_t* __restrict__ wf, uint16_t* __restrict__ wb,
                            float* __restrict__ bias) {
  const int total = kPilotLayers * kWmat;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total + kPilotLayers * kC; i += gridDim.x * blockDim.x) {
    if (i >= total) {
      const int l = (i - total) / kC, co = (i - total) % kC;
      const int off = pilot_layer_offset(l), ci_n = pilot_cin(l), co_n = pilot_cout(l);
      bias[l * kC + co] = co < co_n ? master[off + kTaps * ci_n * co_n + co] : 0.0f;
      continue;
    }
    const int l = i / kWmat, rem = i % kWmat;
    const int t = rem / (kC * kC), a = (rem / kC) % kC, b = rem % kC;
    const int off = pilot_layer_offset(l), ci_n = pilot_cin(l), co_n = pilot_cout(l);
    // forward: (t, co = a, ci = b)
    wf[i] = (b < ci_n && a < co_n) ? f2bf(master[off + (t * ci_n + b) * co_n + a]) : 0;
    // backward: (t', ci = a, co = b) = W[8 - t'][ci][co]
    wb[i] = (a < ci_n && b < co_n) ? f2bf(master[off + ((8 - t) * ci_n + a) * co_n + b]) : 0;
  }
}

__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace

int pilot_conv_items(int N, int H, int W) { return conv_items(N, H, W); }

size_t pilot_packed_bytes() { return static_cast<size_t>(kPilotLayers) * kWmat * 2 * sizeof(uint16_t); }

size_t pilot_wgrad_partial_floats(int grid) { return static_cast<size_t>(grid) * (kWmat + kC); }

hipError_t launch_pilot_pack(const float* master, uint16_t* wf, uint16_t* wb, float* bias, hipStream_t st) {
  hipLaunchKernelGGL(pack_kernel, dim3(256), dim3(256), 0, st, master, wf, wb, bias);
  return hipGetLastError();
}

hipError_t launch_pilot_prep(const uint16_t* noisy, const float* sigma, int N, int H, int W, uint16_t* x0,
                             hipStream_t st) {
  const size_t total = static_cast<size_t>(N) * H * W;
  const unsigned blocks = static_cast<unsigned>(std::min<size_t>((total + 255) / 256, 16384));
  hipLaunchKernelGGL(prep_kernel, dim3(blocks), dim3(256), 0, st, noisy, sigma, N, H * W, x0);
  return hipGetLastError();
}

int pilot_fused_tiles(int N, int H, int W) { return fused_tiles(N, H, W); }

hipError_t launch_pilot_infer_fused(const uint16_t* noisy, const float* sigma, const uint16_t* wf, const float* bias,
                                    int N, int H, int W, float* pilot_f32, uint16_t* pilot_u16, int grid_cap,
                                    hipStream_t st) {
  const int grid = std::max(1, std::min(fused_tiles(N, H, W), grid_cap));
  hipLaunchKernelGGL(fused_infer_kernel, dim3(grid), dim3(kFThreads), 0, st, noisy, sigma, wf, bias, N, H, W,
                     pilot_f32, pilot_u16);
  return hipGetLastError();
}

hipError_t launch_pilot_conv(int mode, const uint16_t* in, const uint16_t* w, const float* bias, const uint16_t* mask,
                             uint16_t* out, const uint16_t* noisy, float* pilot_f32, uint16_t* pilot_u16, int N,
                             int H, int W, int grid_cap, hipStream_t st) {
  const int items = conv_items(N, H, W);
  const int grid = std::max(1, std::min(items, grid_cap));
  switch (mode) {
    case 0:
      hipLaunchKernelGGL(conv_kernel<0>, dim3(grid), dim3(256), 0, st, in, w, bias, mask, out, noisy, pilot_f32,
                         pilot_u16, N, H, W);
      break;
    case 1:
      hipLaunchKernelGGL(conv_kernel<1>, dim3(grid), dim3(256), 0, st, in, w, bias, mask, out, noisy, pilot_f32,
                         pilot_u16, N, H, W);
      break;
    case 2:
      hipLaunchKernelGGL(conv_kernel<2>, dim3(grid), dim3(256), 0, st, in, w, bias, mask, out, noisy, pilot_f32,
                         pilot_u16, N, H, W);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pilot_loss(const float* pilot, const float* target, const float* weight, size_t hw, size_t n,
                             uint16_t* g, double* part, int n_part, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(loss_kernel, dim3(n_part), dim3(256), 0, st, pilot, target, weight, hw, n, g, part);
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(64), 0, st, part, n_part, n, loss);
  return hipGetLastError();
}

hipError_t launch_pilot_wgrad(const uint16_t* x, const uint16_t* g, int N, int H, int W, int grid, float* partial,
                              int layer, float* grad_layer, hipStream_t st) {
  hipLaunchKernelGGL(wgrad_kernel, dim3(grid), dim3(256), 0, st, x, g, N, H, W, partial);
  const int ci_n = pilot_cin(layer), co_n = pilot_cout(layer);
  const int n_out = kTaps * ci_n * co_n + co_n;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((n_out + 255) / 256), dim3(256), 0, st, partial, grid, ci_n, co_n,
                     grad_layer);
  return hipGetLastError();
}

hipError_t launch_pilot_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
                             float eps, int step, hipStream_t st) {
  const float c1 = 1.0f - powf(b1, static_cast<float>(step));
  const float c2 = 1.0f - powf(b2, static_cast<float>(step));
  hipLaunchKernelGGL(adam_kernel, dim3(64), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace gbm3d
