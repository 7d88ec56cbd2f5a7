// Host-side launchers of the library's kernels (all asynchronous on `st`).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gbm3d {

// idx[n_refs][K]: displacement ranks of the K matched blocks (slot 0 = reference).
// split: parts of the displacement rows per reference row (1, 2, 4; 0 = by size)
hipError_t launch_bm(const uint16_t* img, int H, int W, int R, int K, int16_t* idx, hipStream_t st, int split = 0);

// out[H*W][64]: 2-D transform (kind 0 = bior1.5 Mallat, 1 = DCT) of every block
hipError_t launch_stack(const uint16_t* img, int H, int W, int kind, float* out, hipStream_t st);

// bytes of the per-tile partial-sum buffer (64-bit fixed point) of the group kernels
size_t partials_bytes(int H, int W, int R);

hipError_t launch_group_ht(const float* stack, const int16_t* idx, int H, int W, int R, int K, float sigma,
                           float ht_a, float ht_b, int weight_mode, float eps, int keep_dc, void* partials,
                           hipStream_t st);

hipError_t launch_group_wiener(const float* stack_noisy, const float* stack_pilot, const int16_t* idx, int H,
                               int W, int R, int K, float sigma, void* partials, hipStream_t st);

// out = sum(num) / sum(den) over the overlapping tile footprints; q (optional)
// receives the uint16 quantisation of out
hipError_t launch_reduce(const void* partials, int H, int W, int R, float* out, uint16_t* q, hipStream_t st);

hipError_t launch_quantize(const float* in, uint16_t* out, size_t n, hipStream_t st);

}  // namespace gbm3d
