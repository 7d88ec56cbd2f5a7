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
