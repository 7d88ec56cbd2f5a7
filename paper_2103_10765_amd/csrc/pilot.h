// Learned pilot network: layer geometry of the float32 master parameter vector
// and the host-side launchers of its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gbm3d {

constexpr int kPilotLayers = 6;

// input / output channels of layer l (2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1)
__host__ __device__ constexpr int pilot_cin(int l) { return l == 0 ? 2 : 32; }
__host__ __device__ constexpr int pilot_cout(int l) { return l == kPilotLayers - 1 ? 1 : 32; }
// offset of layer l in the master vector: per layer W[ky][kx][ci][co] then bias[co]
__host__ __device__ constexpr int pilot_layer_offset(int l) {
  int o = 0;
  for (int j = 0; j < l; ++j) o += 9 * pilot_cin(j) * pilot_cout(j) + pilot_cout(j);
  return o;
}
constexpr int kPilotParams = pilot_layer_offset(kPilotLayers);
static_assert(kPilotParams == 37889, "parameter count");

int pilot_conv_items(int N, int H, int W);
size_t pilot_packed_bytes();                 // forward + backward bf16 weight sets of all layers
size_t pilot_wgrad_partial_floats(int grid);

hipError_t launch_pilot_pack(const float* master, uint16_t* wf, uint16_t* wb, float* bias, hipStream_t st);
hipError_t launch_pilot_prep(const uint16_t* noisy, const float* sigma, int N, int H, int W, uint16_t* x0,
                             hipStream_t st);
// mode 0: forward + bias + ReLU; 1: last layer -> pilot; 2: input gradient with ReLU mask
hipError_t launch_pilot_conv(int mode, const uint16_t* in, const uint16_t* w, const float* bias, const uint16_t* mask,
                             uint16_t* out, const uint16_t* noisy, float* pilot_f32, uint16_t* pilot_u16, int N,
                             int H, int W, int grid_cap, hipStream_t st);
// inference of all six layers in one launch (one 16 x 32 output tile per
// workgroup at a time, activations in LDS); grid_cap bounds the persistent grid
int pilot_fused_tiles(int N, int H, int W);
hipError_t launch_pilot_infer_fused(const uint16_t* noisy, const float* sigma, const uint16_t* wf, const float* bias,
                                    int N, int H, int W, float* pilot_f32, uint16_t* pilot_u16, int grid_cap,
                                    hipStream_t st);
// loss = sum_p weight[p / hw] (pilot - target)^2 / n (weight NULL: 1), and dL/df
hipError_t launch_pilot_loss(const float* pilot, const float* target, const float* weight, size_t hw, size_t n,
                             uint16_t* g, double* part, int n_part, float* loss, hipStream_t st);
hipError_t launch_pilot_wgrad(const uint16_t* x, const uint16_t* g, int N, int H, int W, int grid, float* partial,
                              int layer, float* grad_layer, hipStream_t st);
hipError_t launch_pilot_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
                             float eps, int step, hipStream_t st);

}  // namespace gbm3d
