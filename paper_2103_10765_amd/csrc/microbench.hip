// Peak-rate probes: the arithmetic units the kernels of this library are
// measured against, run flat out with no memory traffic, so each kernel's
// achieved rate can be read against a measured ceiling as well as the
// published one.
//
//   fp64 vector FMA   every thread runs kChains independent fma chains
//   int8 matrix core  every wave runs kChains independent
//                     v_mfma_i32_16x16x64_i8 accumulations (the matcher's op)
//   bf16 matrix core  the same with v_mfma_f32_16x16x32_bf16 (the pilot's op)
//
// One 32-bit value per thread goes to `sink` so that nothing is dead code.
#include <cstdint>

#include "common.h"
#include "kernels.h"

namespace gbm3d {

namespace {

constexpr int kMbThreads = 256;
constexpr int kChains = 8;

typedef int mb_i32x4 __attribute__((ext_vector_type(4)));
typedef float mb_f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 mb_bf16x8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(kMbThreads) void mb_fp64_kernel(int iters, float* __restrict__ sink) {
  double a[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = 1e-3 * threadIdx.x + c;
  const double m = 0.9999999, b = 1e-9 * blockIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = fma(a[c], m, b);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += a[c];
  sink[static_cast<size_t>(blockIdx.x) * kMbThreads + threadIdx.x] = static_cast<float>(s);
}

__global__ __launch_bounds__(kMbThreads) void mb_mfma_i8_kernel(int iters, float* __restrict__ sink) {
  const int t = static_cast<int>(threadIdx.x);
  const mb_i32x4 x = {t, t ^ 0x01010101, t * 3, 0x7f7f7f7f};
  const mb_i32x4 y = {0x01020304, t, 0x05060708 ^ t, t * 5};
  mb_i32x4 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = mb_i32x4{c, 0, 0, 0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(x, y, acc[c], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[static_cast<size_t>(blockIdx.x) * kMbThreads + threadIdx.x] = static_cast<float>(s);
}

__global__ __launch_bounds__(kMbThreads) void mb_mfma_bf16_kernel(int iters, float* __restrict__ sink) {
  mb_bf16x8 x, y;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    x[j] = static_cast<__bf16>(1e-3f * static_cast<float>(threadIdx.x + j));
    y[j] = static_cast<__bf16>(1e-3f * static_cast<float>(j - static_cast<int>(threadIdx.x & 7)));
  }
  mb_f32x4 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = mb_f32x4{static_cast<float>(c), 0.0f, 0.0f, 0.0f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[static_cast<size_t>(blockIdx.x) * kMbThreads + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_microbench(int kind, int blocks, int iters, float* sink, hipStream_t st) {
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(mb_fp64_kernel, dim3(blocks), dim3(kMbThreads), 0, st, iters, sink);
      break;
    case 1:
      hipLaunchKernelGGL(mb_mfma_i8_kernel, dim3(blocks), dim3(kMbThreads), 0, st, iters, sink);
      break;
    case 2:
      hipLaunchKernelGGL(mb_mfma_bf16_kernel, dim3(blocks), dim3(kMbThreads), 0, st, iters, sink);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

double microbench_ops(int kind, int blocks, int iters) {
  const double threads = static_cast<double>(blocks) * kMbThreads;
  const double waves = threads / kWave;
  switch (kind) {
    case 0:
      return threads * iters * kChains * 2.0;
    case 1:
      return waves * iters * kChains * (16.0 * 16.0 * 64.0 * 2.0);
    case 2:
      return waves * iters * kChains * (16.0 * 16.0 * 32.0 * 2.0);
    default:
      return 0.0;
  }
}

}  // namespace gbm3d
