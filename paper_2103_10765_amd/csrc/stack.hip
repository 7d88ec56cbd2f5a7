// Transform-domain patch stack: the 2-D transform of the periodic 8x8 block at
// every pixel position, 64 float coefficients per position (256 B, AoS).
//   bior1.5: 3-level periodic Mallat decomposition (Sec. 5), each level
//            applying one analysis step to the rows and columns of the current
//            low-low block;
//   DCT:     orthonormal separable 8x8 DCT-II (Sec. 4).
// A workgroup covers 4 rows x 64 columns of positions.  Each thread
// transforms one block read from an LDS pixel tile; in two halves of 32
// positions, the threads park their 64 coefficients in LDS and the wave
// writes the half's consecutive positions as one contiguous 8 KB run with
// 16-byte stores (half-size staging keeps four workgroups per CU).
#include "common.h"
#include "kernels.h"
#include "norm.h"

namespace gbm3d {

namespace {

constexpr int kRowsPerWg = 4;
constexpr int kStackThreads = kRowsPerWg * kWave;  // one wave per output row
constexpr int kPixRows = kRowsPerWg + kPatch - 1;  // 11
constexpr int kPixCols = kWave + kPatch - 1;       // 71
constexpr int kStagePitch = 65;                    // floats per parked block (odd: conflict-free)
constexpr int kHalf = kWave / 2;                   // positions parked at a time

// one separable level on the leading L x L block: rows (x[a][0..L)), then columns
template <int L, typename F>
__device__ __forceinline__ void rows_cols(float (&x)[8][8], F&& line) {
#pragma unroll
  for (int a = 0; a < L; ++a) {
    float t[8];
    line(x[a], t);
#pragma unroll
    for (int b = 0; b < L; ++b) x[a][b] = t[b];
  }
#pragma unroll
  for (int b = 0; b < L; ++b) {
    float c[8], t[8];
#pragma unroll
    for (int a = 0; a < L; ++a) c[a] = x[a][b];
    line(c, t);
#pragma unroll
    for (int a = 0; a < L; ++a) x[a][b] = t[a];
  }
}

template <int KIND>
__device__ __forceinline__ void forward2d(float (&x)[8][8]) {
  if constexpr (KIND == 0) {
    constexpr Mat8 A8 = bior_analysis(8);
    constexpr Mat8 A4 = bior_analysis(4);
    constexpr Mat8 A2 = bior_analysis(2);
    rows_cols<8>(x, [&](const float* i, float* o) { apply_mat<8>(A8, i, o); });
    rows_cols<4>(x, [&](const float* i, float* o) { apply_mat<4>(A4, i, o); });
    rows_cols<2>(x, [&](const float* i, float* o) { apply_mat<2>(A2, i, o); });
  } else {
    rows_cols<8>(x, [&](const float* i, float* o) { dct8_fwd(i, o); });
  }
}

__host__ __device__ constexpr int stack_items(int H, int W) {
  return ((H + kRowsPerWg - 1) / kRowsPerWg) * ((W + kWave - 1) / kWave);
}

// LOADS_FIRST: every thread's pixel loads are issued before the first is
// used (one memory round trip for the tile); otherwise one item at a time.
template <int KIND, bool LOADS_FIRST>
__device__ __forceinline__ void stack_body(float (*pix)[kPixCols + 1], float (*stage)[kHalf * kStagePitch],
                                           const uint16_t* __restrict__ img_, float* __restrict__ out_,
                                           unsigned long long* __restrict__ block_weights_, int H, int W, int item) {
  const auto img = to_global(img_);
  const auto out = to_global(out_);
  const auto block_weights = to_global(block_weights_);
  const int xt = (W + kWave - 1) / kWave;
  const int y0 = (item / xt) * kRowsPerWg;
  const int x0 = (item % xt) * kWave;
  const float scale = 1.0f / 65535.0f;
  constexpr int kPix = kPixRows * kPixCols;
  if constexpr (LOADS_FIRST) {
    constexpr int kPixIter = (kPix + kStackThreads - 1) / kStackThreads;
    unsigned zv[kPixIter];
#pragma unroll
    for (int it = 0; it < kPixIter; ++it) {
      // (unconditional: threads past the tile's last pixel reload it)
      const int i = min(static_cast<int>(threadIdx.x) + it * kStackThreads, kPix - 1);
      const int r = i / kPixCols, c = i - r * kPixCols;
      const int y = (y0 + r) % H, x = (x0 + c) % W;
      zv[it] = img[static_cast<size_t>(y) * W + x];
    }
#pragma unroll
    for (int it = 0; it < kPixIter; ++it) {
      const int i = static_cast<int>(threadIdx.x) + it * kStackThreads;
      if (i < kPix) {
        const int r = i / kPixCols, c = i - r * kPixCols;
        pix[r][c] = static_cast<float>(zv[it]) * scale;
      }
    }
  } else {
    for (int i = threadIdx.x; i < kPix; i += blockDim.x) {
      const int r = i / kPixCols, c = i - r * kPixCols;
      const int y = (y0 + r) % H, x = (x0 + c) % W;
      pix[r][c] = static_cast<float>(img[static_cast<size_t>(y) * W + x]) * scale;
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  float x[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) x[a][b] = pix[w + a][lane + b];
  forward2d<KIND>(x);
  const int y = y0 + w;
  const int n_pos = min(kWave, W - x0);  // positions of this row in the tile
  // the aggregation that follows adds into the block-start weights and the
  // numerator sums
  if (block_weights && y < H && lane < n_pos) {
    const size_t o = static_cast<size_t>(y) * W + x0 + lane;
    block_weights[o] = 0;
    block_weights[block_weight_entries(H, W) + o] = 0;
  }
  typedef float f32x4v __attribute__((ext_vector_type(4)));
  const auto dst = (global_ptr<f32x4v>)(out + (static_cast<size_t>(y) * W + x0) * 64);
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    wave_lds_sync();  // the previous half's reads are done
    if ((lane / kHalf) == half) {
      float* st = stage[w] + (lane % kHalf) * kStagePitch;
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) st[a * 8 + b] = x[a][b];
    }
    wave_lds_sync();
    if (y < H) {
      // 8 rounds; in round i lane l stores float4 g = i*64 + l of the half's run
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int g = i * kWave + lane;
        const int blk = g >> 4, c = (g & 15) * 4;
        if (half * kHalf + blk < n_pos) {
          const float* s = stage[w] + blk * kStagePitch + c;
          dst[half * kHalf * 16 + g] = f32x4v{s[0], s[1], s[2], s[3]};
        }
      }
    }
  }
  __syncthreads();  // the pixel tile and the staging area are reused
}

// src_sel: 0 = noisy, 1 = pilot; dst_sel: 0 = stack_a, 1 = stack_b; both
// negative: blockIdx.y selects (noisy -> stack_a, pilot -> stack_b)
template <int KIND, bool BATCH>
__global__ __launch_bounds__(kStackThreads) void stack_kernel(ImgRec one, WorkList wl, int src_sel, int dst_sel) {
  __shared__ float pix[kPixRows][kPixCols + 1];
  __shared__ float stage[kRowsPerWg][kHalf * kStagePitch];
  const int src = src_sel < 0 ? static_cast<int>(blockIdx.y) : src_sel;
  const int dst = dst_sel < 0 ? static_cast<int>(blockIdx.y) : dst_sel;
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) {
    stack_body<KIND, false>(pix, stage, src ? r.pilot : r.noisy, dst ? r.stack_b : r.stack_a,
                            dst ? nullptr : r.partials, r.H, r.W, item);
  });
}

// The stacks of a stage beside the correlation matcher's norm table of the
// image it matches, in one launch over one image: grid rows y < gridDim.y - 1
// are stack planes as in stack_kernel, the last row the norm items.  The two
// passes share nothing but the launch: the short, latency-bound norm pass
// runs in the gaps of the write-bound stack items instead of as a launch of
// its own.
// Workgroups (all grid rows) up to which a stack launch counts as short:
// 32 per CU of the 256.
constexpr int kShortLaunchItems = 32 * 256;

struct StackSmem {
  static constexpr int pix_bytes = (kPixRows * (kPixCols + 1) * 4 + 15) / 16 * 16;
  static constexpr int bytes = pix_bytes + kRowsPerWg * kHalf * kStagePitch * 4;
};

template <int KIND, bool LOADS_FIRST>
__global__ __launch_bounds__(kStackThreads) void stack_norm_kernel(ImgRec r, int src_sel, int dst_sel, int R,
                                                                   int norm_src) {
  constexpr int kBytes = StackSmem::bytes > NormSmem::bytes ? StackSmem::bytes : NormSmem::bytes;
  __shared__ __align__(16) unsigned char smem[kBytes];
  static_assert(kStackThreads == 256, "norm items are laid out for 256 threads");
  const int item = static_cast<int>(blockIdx.x);
  if (blockIdx.y == gridDim.y - 1) {
    if (item >= norm_items(r.H, r.W)) return;
    int* zt = reinterpret_cast<int*>(smem);
    double* hs = reinterpret_cast<double*>(smem + NormSmem::zt_bytes);
    norm_body<LOADS_FIRST>(norm_src ? r.pilot : r.noisy, r.norm, r.H, r.W, R, item, zt, hs);
    return;
  }
  if (item >= stack_items(r.H, r.W)) return;
  auto pix = reinterpret_cast<float(*)[kPixCols + 1]>(smem);
  auto stage = reinterpret_cast<float(*)[kHalf * kStagePitch]>(smem + StackSmem::pix_bytes);
  const int src = src_sel < 0 ? static_cast<int>(blockIdx.y) : src_sel;
  const int dst = dst_sel < 0 ? static_cast<int>(blockIdx.y) : dst_sel;
  stack_body<KIND, LOADS_FIRST>(pix, stage, src ? r.pilot : r.noisy, dst ? r.stack_b : r.stack_a,
                                dst ? nullptr : r.partials, r.H, r.W, item);
}

}  // namespace

int stack_items_for(int H, int W) { return stack_items(H, W); }

hipError_t launch_stack(const ImgRec& one, const WorkList* wl, int kind, int src_sel, int dst_sel, int grid_cap,
                        hipStream_t st) {
  if ((src_sel < 0) != (dst_sel < 0)) return hipErrorInvalidValue;
  const unsigned planes = src_sel < 0 ? 2u : 1u;  // both stacks in one launch
  if (!wl) {
    const dim3 grid(static_cast<unsigned>(stack_items(one.H, one.W)), planes);
    if (kind == 0)
      hipLaunchKernelGGL((stack_kernel<0, false>), grid, dim3(kStackThreads), 0, st, one, WorkList{}, src_sel, dst_sel);
    else
      hipLaunchKernelGGL((stack_kernel<1, false>), grid, dim3(kStackThreads), 0, st, one, WorkList{}, src_sel, dst_sel);
  } else {
    if (wl->total <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>(std::min(wl->total, grid_cap)), planes);
    if (kind == 0)
      hipLaunchKernelGGL((stack_kernel<0, true>), grid, dim3(kStackThreads), 0, st, one, *wl, src_sel, dst_sel);
    else
      hipLaunchKernelGGL((stack_kernel<1, true>), grid, dim3(kStackThreads), 0, st, one, *wl, src_sel, dst_sel);
  }
  return hipGetLastError();
}

hipError_t launch_stack_norm(const ImgRec& one, int kind, int src_sel, int dst_sel, int R, int norm_src,
                             hipStream_t st) {
  if ((src_sel < 0) != (dst_sel < 0)) return hipErrorInvalidValue;
  const unsigned rows = (src_sel < 0 ? 2u : 1u) + 1u;  // stack planes, then the norm items
  const int items = std::max(stack_items(one.H, one.W), norm_items(one.H, one.W));
  const dim3 grid(static_cast<unsigned>(items), rows);
  // A launch of a few workgroups per CU is bound by each workgroup's
  // latency: there the pixel loads go out all at once (measured: 512^2
  // faster, 4096^2 slower, where the stack writes bound the launch)
  const bool short_launch = items * static_cast<int>(rows) <= kShortLaunchItems;
  if (kind == 0) {
    if (short_launch)
      hipLaunchKernelGGL((stack_norm_kernel<0, true>), grid, dim3(kStackThreads), 0, st, one, src_sel, dst_sel, R,
                         norm_src);
    else
      hipLaunchKernelGGL((stack_norm_kernel<0, false>), grid, dim3(kStackThreads), 0, st, one, src_sel, dst_sel, R,
                         norm_src);
  } else {
    if (short_launch)
      hipLaunchKernelGGL((stack_norm_kernel<1, true>), grid, dim3(kStackThreads), 0, st, one, src_sel, dst_sel, R,
                         norm_src);
    else
      hipLaunchKernelGGL((stack_norm_kernel<1, false>), grid, dim3(kStackThreads), 0, st, one, src_sel, dst_sel, R,
                         norm_src);
  }
  return hipGetLastError();
}

}  // namespace gbm3d
