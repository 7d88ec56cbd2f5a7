// The block-norm table of the correlation matcher (Theorem 1, Sec. 2): the
// per-position squared norms its keys take from memory.  Shared by the norm
// pass and the launch that forms a stage's patch stacks beside it.
#pragma once

#include "common.h"

namespace gbm3d {

constexpr int kNormPad = 32;                       // periodic border of the norm table
constexpr int kZShift = 32896;

__device__ __forceinline__ int norm_pitch(int W) { return W + 2 * kNormPad; }

// ---------------------------------------------------------------------------
// Norm table: T[ey][ex] = 2048 N + ey S + ex (S = 2R + 1), N the sum over
// the 8 x 8 block at image position ((ey - pad) mod H, (ex - pad) mod W) of
// (Z - 32896)^2, for ey < H + 2 pad, ex < W + 2 pad (exact: 2048 N < 2^47,
// ey S + ex < 2^23).  A candidate's rank (dy + R) S + (dx + R) is the
// difference of the position terms of candidate and reference plus a
// constant, so the matching kernel takes the candidate's whole key term from
// one load and leaves the reference's to a per-reference constant.  Items
// are 8 x 64 output tiles (small tiles: many workgroups in flight for what
// is a short, latency-bound pass).
// ---------------------------------------------------------------------------
constexpr int kNTy = 8, kNTx = 64;

__host__ __device__ constexpr int norm_items(int H, int W) {
  return ((H + 2 * kNormPad + kNTy - 1) / kNTy) * ((W + 2 * kNormPad + kNTx - 1) / kNTx);
}

// LOADS_FIRST: every thread's pixel loads are issued before the first is
// used (one memory round trip for the tile); otherwise one item at a time.
template <bool LOADS_FIRST>
__device__ __forceinline__ void norm_body(const uint16_t* __restrict__ img_, double* __restrict__ norm_, int H, int W,
                                          int R, int item, int* zt, double* hs) {
  const auto img = to_global(img_);
  const auto norm = to_global(norm_);
  const int He = H + 2 * kNormPad, We = norm_pitch(W);
  const int tiles_x = (We + kNTx - 1) / kNTx;
  const int S = 2 * R + 1;
  const int ty0 = (item / tiles_x) * kNTy, tx0 = (item % tiles_x) * kNTx;
  constexpr int ZR = kNTy + 7, ZC = kNTx + 7;
  // table rows and columns lie within one period of the image when it is at
  // least as large as the border plus a tile; else the general modulo
  const bool near = H >= kNormPad + kNTy + 7 && W >= kNormPad + kNTx + 7;
  if constexpr (LOADS_FIRST) {
    constexpr int kZIter = (ZR * ZC + 255) / 256;  // launched with 256 threads
    int zv[kZIter];
#pragma unroll
    for (int it = 0; it < kZIter; ++it) {
      // (unconditional: threads past the tile's last pixel reload it)
      const int i = min(static_cast<int>(threadIdx.x) + it * 256, ZR * ZC - 1);
      const int r = i / ZC, c = i - r * ZC;
      int y = ty0 + r - kNormPad, x = tx0 + c - kNormPad;
      if (near) {
        y += y < 0 ? H : (y >= H ? -H : 0);
        x += x < 0 ? W : (x >= W ? -W : 0);
      } else {
        y = pmod(y, H);
        x = pmod(x, W);
      }
      zv[it] = static_cast<int>(img[static_cast<size_t>(y) * W + x]);
    }
#pragma unroll
    for (int it = 0; it < kZIter; ++it) {
      const int i = static_cast<int>(threadIdx.x) + it * 256;
      if (i < ZR * ZC) zt[i] = zv[it] - kZShift;
    }
  } else {
    for (int i = threadIdx.x; i < ZR * ZC; i += blockDim.x) {
      const int r = i / ZC, c = i - r * ZC;
      int y = ty0 + r - kNormPad, x = tx0 + c - kNormPad;
      if (near) {
        y += y < 0 ? H : (y >= H ? -H : 0);
        x += x < 0 ? W : (x >= W ? -W : 0);
      } else {
        y = pmod(y, H);
        x = pmod(x, W);
      }
      zt[i] = static_cast<int>(img[static_cast<size_t>(y) * W + x]) - kZShift;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ZR * kNTx; i += blockDim.x) {
    const int r = i / kNTx, c = i - r * kNTx;
    double h = 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int v = zt[r * ZC + c + b];
      h += static_cast<double>(v * v);  // |v| <= 32896: v * v < 2^31
    }
    hs[i] = h;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kNTy * kNTx; i += blockDim.x) {
    const int r = i / kNTx, c = i - r * kNTx;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) s += hs[(r + a) * kNTx + c];
    if (ty0 + r < He && tx0 + c < We)
      norm[static_cast<size_t>(ty0 + r) * We + tx0 + c] = fma(s, 2048.0, static_cast<double>((ty0 + r) * S + tx0 + c));
  }
}

// LDS of one norm item: the pixel tile and the row sums
struct NormSmem {
  static constexpr int zt_ints = (kNTy + 7) * (kNTx + 7);
  static constexpr int zt_bytes = (zt_ints * 4 + 15) / 16 * 16;
  static constexpr int bytes = zt_bytes + (kNTy + 7) * kNTx * 8;
};

}  // namespace gbm3d
