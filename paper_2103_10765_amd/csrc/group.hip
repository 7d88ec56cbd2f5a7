// Collaborative filtering of matched groups and their aggregation.
//
// A workgroup owns a tile of TPY x TPX references; each of its four waves
// filters one group at a time with lane = 2-D coefficient index (64 lanes =
// 8x8 coefficients) and the group axis in registers:
//   gather the K spectra from the patch stack (one coalesced 256 B load per
//   block), 1-D Haar along the group, shrink, inverse Haar, inverse 2-D
//   transform of the K blocks through a per-wave LDS scratch (separable rows
//   then columns, level by level), group weight, and accumulation of w*U and
//   w into an LDS image of the tile's footprint (every block a reference of
//   the tile can match lies in it: rows 3p-R .. 3p+7+R).
// The footprint is written once per tile to a partial-sum buffer; a second
// kernel sums the overlapping footprints for every pixel (periodic), divides
// and optionally quantises.  No global atomics are used.
//
// Stage 1 (Sec. 3.1, Sec. 5): bior1.5 stack, hard threshold |C| >= tau_l with
//   tau_l = sigma (a - b l) by Mallat level, 3-D DC kept, weight 1/(TV+eps).
// Stage 2 (Sec. 4): DCT stacks of the noisy image and the pilot, Wiener gain
//   W = b^2 / (b^2 + sigma^2) of the pilot spectrum (W = 1 at the 3-D DC)
//   applied to the noisy spectrum, weight 1 / sum W^2.
#include "common.h"
#include "kernels.h"

namespace gbm3d {

namespace {

constexpr int kScratchPitch = 9;                  // LDS row pitch of a parked 8x8 block
constexpr int kBlockFloats = 8 * kScratchPitch;   // 72

template <int TPY, int TPX>
struct Foot {
  static constexpr int FYmax = kStep * (TPY - 1) + kPatch + 2 * kMaxR;
  static constexpr int FXmax = kStep * (TPX - 1) + kPatch + 2 * kMaxR;
  static constexpr int FXPmax = FXmax + ((8 - FXmax) % 32 + 32) % 32;
  static constexpr int floats = 2 * FYmax * FXPmax;
};

// x[k] (k < K), parked at xw[k*72 + a*9 + b]: inverse of one separable level
// on the leading L x L block of every parked block.
template <int K, int L>
__device__ __forceinline__ void inverse_level(float* xw, const Mat8& S, int lane) {
  constexpr int items = K * L;
  // rows: item = (k, i)
#pragma unroll
  for (int it0 = 0; it0 < items; it0 += kWave) {
    const int it = it0 + lane;
    if (it < items) {
      const int k = it / L, i = it % L;
      float* row = xw + k * kBlockFloats + i * kScratchPitch;
      float x[8], y[8];
#pragma unroll
      for (int j = 0; j < L; ++j) x[j] = row[j];
      apply_mat<L>(S, x, y);
#pragma unroll
      for (int j = 0; j < L; ++j) row[j] = y[j];
    }
  }
  wave_lds_sync();
  // columns: item = (k, j)
#pragma unroll
  for (int it0 = 0; it0 < items; it0 += kWave) {
    const int it = it0 + lane;
    if (it < items) {
      const int k = it / L, j = it % L;
      float* col = xw + k * kBlockFloats + j;
      float x[8], y[8];
#pragma unroll
      for (int i = 0; i < L; ++i) x[i] = col[i * kScratchPitch];
      apply_mat<L>(S, x, y);
#pragma unroll
      for (int i = 0; i < L; ++i) col[i * kScratchPitch] = y[i];
    }
  }
  wave_lds_sync();
}

struct GroupArgs {
  int H, W, R, S, nRy, nRx, nTx;
  int FY, FXP;
};

__device__ __forceinline__ void tile_origin(const GroupArgs& g, int TPY, int TPX, int& fy0, int& fx0) {
  fy0 = kStep * static_cast<int>(blockIdx.y) * TPY - g.R;
  fx0 = kStep * static_cast<int>(blockIdx.x) * TPX - g.R;
}

// Block positions of group `ref` (p, q): tile-local top-left and stack offset.
template <int K>
__device__ __forceinline__ void group_positions(const GroupArgs& g, const int16_t* __restrict__ idx, int p,
                                                int q, int fy0, int fx0, int (&ly)[K], int (&lx)[K],
                                                size_t (&off)[K]) {
  const int16_t* id = idx + (static_cast<size_t>(p) * g.nRx + q) * K;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = id[k];
    const int dyi = r / g.S, dxi = r - dyi * g.S;
    const int y = kStep * p + dyi - g.R, x = kStep * q + dxi - g.R;
    ly[k] = y - fy0;
    lx[k] = x - fx0;
    off[k] = (static_cast<size_t>(pmod(y, g.H)) * g.W + pmod(x, g.W)) * 64;
  }
}

template <int K>
__device__ __forceinline__ void accumulate(float* acc, const GroupArgs& g, const int (&ly)[K], const int (&lx)[K],
                                           const float (&u)[K], float w, int lane) {
  const int a = lane >> 3, b = lane & 7;
  float* num = acc;
  float* den = acc + g.FY * g.FXP;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int o = (ly[k] + a) * g.FXP + lx[k] + b;
    atomicAdd(num + o, w * u[k]);
    atomicAdd(den + o, w);
  }
}

__device__ __forceinline__ void zero_acc(float* acc, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc[i] = 0.0f;
  __syncthreads();
}

__device__ __forceinline__ void flush_acc(const float* acc, int n, float* __restrict__ partials, int nTx) {
  __syncthreads();
  float* dst = partials + (static_cast<size_t>(blockIdx.y) * nTx + blockIdx.x) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = acc[i];
}

template <int K, int TPY, int TPX>
__global__ __launch_bounds__(256) void group_ht_kernel(const float* __restrict__ stack,
                                                       const int16_t* __restrict__ idx, GroupArgs g,
                                                       float sigma, float ht_a, float ht_b, int weight_mode,
                                                       float eps, int keep_dc, float* __restrict__ partials) {
  using F = Foot<TPY, TPX>;
  __shared__ float acc[F::floats];
  __shared__ float scratch[4][K * kBlockFloats];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int n_acc = 2 * g.FY * g.FXP;
  zero_acc(acc, n_acc);
  int fy0, fx0;
  tile_origin(g, TPY, TPX, fy0, fx0);
  float* xw = scratch[wave];
  const int a = lane >> 3, b = lane & 7;
  const float tau = sigma * (ht_a - ht_b * static_cast<float>(bior_level(lane)));
  const bool dc_lane = keep_dc && lane == 0;

  for (int t = wave; t < TPY * TPX; t += 4) {
    const int p = blockIdx.y * TPY + t / TPX, q = blockIdx.x * TPX + t % TPX;
    if (p >= g.nRy || q >= g.nRx) continue;
    int ly[K], lx[K];
    size_t off[K];
    group_positions<K>(g, idx, p, q, fy0, fx0, ly, lx, off);
    float v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = stack[off[k] + lane];
    haar_fwd<K>(v);
    int nnz = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool keep = fabsf(v[k]) >= tau || (k == 0 && dc_lane);
      v[k] = keep ? v[k] : 0.0f;
      nnz += keep ? 1 : 0;
    }
    haar_inv<K>(v);
    wave_lds_sync();  // the previous group's reads of the scratch are done
#pragma unroll
    for (int k = 0; k < K; ++k) xw[k * kBlockFloats + a * kScratchPitch + b] = v[k];
    wave_lds_sync();
    {
      constexpr Mat8 S2 = bior_synthesis(2);
      constexpr Mat8 S4 = bior_synthesis(4);
      constexpr Mat8 S8 = bior_synthesis(8);
      inverse_level<K, 2>(xw, S2, lane);
      inverse_level<K, 4>(xw, S4, lane);
      inverse_level<K, 8>(xw, S8, lane);
    }
    float u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = xw[k * kBlockFloats + a * kScratchPitch + b];
    float w;
    if (weight_mode == 0) {
      float tv = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k + 1 < K) tv += fabsf(u[k + 1] - u[k]);
        if (b < 7) tv += fabsf(xw[k * kBlockFloats + a * kScratchPitch + b + 1] - u[k]);
        if (a < 7) tv += fabsf(xw[k * kBlockFloats + (a + 1) * kScratchPitch + b] - u[k]);
      }
      w = 1.0f / (wave_sum(tv) + eps);
    } else if (weight_mode == 1) {
      w = 1.0f / static_cast<float>(max(wave_sum_int(nnz), 1));
    } else {
      w = 1.0f;
    }
    accumulate<K>(acc, g, ly, lx, u, w, lane);
  }
  flush_acc(acc, n_acc, partials, g.nTx);
}

template <int K, int TPY, int TPX>
__global__ __launch_bounds__(256) void group_wiener_kernel(const float* __restrict__ stack_n,
                                                           const float* __restrict__ stack_p,
                                                           const int16_t* __restrict__ idx, GroupArgs g,
                                                           float sigma, float* __restrict__ partials) {
  using F = Foot<TPY, TPX>;
  __shared__ float acc[F::floats];
  __shared__ float scratch[4][K * kBlockFloats];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int n_acc = 2 * g.FY * g.FXP;
  zero_acc(acc, n_acc);
  int fy0, fx0;
  tile_origin(g, TPY, TPX, fy0, fx0);
  float* xw = scratch[wave];
  const int a = lane >> 3, b = lane & 7;
  const float s2 = sigma * sigma;

  for (int t = wave; t < TPY * TPX; t += 4) {
    const int p = blockIdx.y * TPY + t / TPX, q = blockIdx.x * TPX + t % TPX;
    if (p >= g.nRy || q >= g.nRx) continue;
    int ly[K], lx[K];
    size_t off[K];
    group_positions<K>(g, idx, p, q, fy0, fx0, ly, lx, off);
    float vn[K], vp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      vn[k] = stack_n[off[k] + lane];
      vp[k] = stack_p[off[k] + lane];
    }
    haar_fwd<K>(vn);
    haar_fwd<K>(vp);
    float sw2 = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float b2 = vp[k] * vp[k];
      float wt = b2 / (b2 + s2);
      if (k == 0 && lane == 0) wt = 1.0f;
      vn[k] *= wt;
      sw2 = fmaf(wt, wt, sw2);
    }
    const float w = 1.0f / wave_sum(sw2);
    haar_inv<K>(vn);
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < K; ++k) xw[k * kBlockFloats + a * kScratchPitch + b] = vn[k];
    wave_lds_sync();
    {
      constexpr Mat8 Ct = transpose8(dct8());
      inverse_level<K, 8>(xw, Ct, lane);
    }
    float u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = xw[k * kBlockFloats + a * kScratchPitch + b];
    accumulate<K>(acc, g, ly, lx, u, w, lane);
  }
  flush_acc(acc, n_acc, partials, g.nTx);
}

// floor(a / b) for b > 0
__device__ __forceinline__ int fdiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Sum of the partial footprints covering pixel (y, x), then normalise.
__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ partials, GroupArgs g, int TY,
                                                     int TX, int nTy, int FX, float* __restrict__ out,
                                                     uint16_t* __restrict__ q) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.W) return;
  const int R = g.R;
  // candidate (tile row, local row) pairs for y; footprint of tile row t covers
  // global rows [t*TY - R, t*TY - R + FY) before wrapping
  int cty[16], cly[16], ny = 0;
  {
    const int lo = -R, hi = (nTy - 1) * TY - R + g.FY;  // half-open range of unwrapped rows
    for (int yy = y + fdiv(lo - y + g.H - 1, g.H) * g.H; yy < hi; yy += g.H) {
      const int t0 = max(0, fdiv(yy + R - g.FY, TY) + 1), t1 = min(nTy - 1, fdiv(yy + R, TY));
      for (int t = t0; t <= t1 && ny < 16; ++t) {
        cty[ny] = t;
        cly[ny] = yy - (t * TY - R);
        ++ny;
      }
    }
  }
  int ctx[16], clx[16], nx = 0;
  {
    const int lo = -R, hi = (g.nTx - 1) * TX - R + FX;
    for (int xx = x + fdiv(lo - x + g.W - 1, g.W) * g.W; xx < hi; xx += g.W) {
      const int t0 = max(0, fdiv(xx + R - FX, TX) + 1), t1 = min(g.nTx - 1, fdiv(xx + R, TX));
      for (int t = t0; t <= t1 && nx < 16; ++t) {
        ctx[nx] = t;
        clx[nx] = xx - (t * TX - R);
        ++nx;
      }
    }
  }
  const size_t plane = static_cast<size_t>(g.FY) * g.FXP;
  float num = 0.0f, den = 0.0f;
  for (int i = 0; i < ny; ++i)
    for (int j = 0; j < nx; ++j) {
      const float* t = partials + (static_cast<size_t>(cty[i]) * g.nTx + ctx[j]) * 2 * plane;
      const size_t o = static_cast<size_t>(cly[i]) * g.FXP + clx[j];
      num += t[o];
      den += t[plane + o];
    }
  const float v = num / den;
  const size_t o = static_cast<size_t>(y) * g.W + x;
  out[o] = v;
  if (q) {
    const double d = static_cast<double>(fminf(fmaxf(v, 0.0f), 1.0f));
    q[o] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
  }
}

__global__ void quantize_kernel(const float* __restrict__ in, uint16_t* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const double d = static_cast<double>(fminf(fmaxf(in[i], 0.0f), 1.0f));
    out[i] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
  }
}

constexpr int kTPY = 8, kTPX = 8;

GroupArgs make_args(int H, int W, int R) {
  GroupArgs g;
  g.H = H;
  g.W = W;
  g.R = R;
  g.S = 2 * R + 1;
  g.nRy = (H + kStep - 1) / kStep;
  g.nRx = (W + kStep - 1) / kStep;
  g.nTx = (g.nRx + kTPX - 1) / kTPX;
  g.FY = kStep * (kTPY - 1) + kPatch + 2 * R;
  const int FX = kStep * (kTPX - 1) + kPatch + 2 * R;
  g.FXP = FX + ((8 - FX) % 32 + 32) % 32;
  return g;
}

}  // namespace

size_t partials_floats(int H, int W, int R) {
  const GroupArgs g = make_args(H, W, R);
  const int nTy = (g.nRy + kTPY - 1) / kTPY;
  return static_cast<size_t>(nTy) * g.nTx * 2 * g.FY * g.FXP;
}

template <int K>
static hipError_t launch_ht_k(const float* stack, const int16_t* idx, int H, int W, int R, float sigma,
                              float ht_a, float ht_b, int weight_mode, float eps, int keep_dc, float* partials,
                              hipStream_t st) {
  const GroupArgs g = make_args(H, W, R);
  dim3 grid(g.nTx, (g.nRy + kTPY - 1) / kTPY);
  hipLaunchKernelGGL((group_ht_kernel<K, kTPY, kTPX>), grid, dim3(256), 0, st, stack, idx, g, sigma, ht_a, ht_b,
                     weight_mode, eps, keep_dc, partials);
  return hipGetLastError();
}

hipError_t launch_group_ht(const float* stack, const int16_t* idx, int H, int W, int R, int K, float sigma,
                           float ht_a, float ht_b, int weight_mode, float eps, int keep_dc, float* partials,
                           hipStream_t st) {
  switch (K) {
    case 2: return launch_ht_k<2>(stack, idx, H, W, R, sigma, ht_a, ht_b, weight_mode, eps, keep_dc, partials, st);
    case 4: return launch_ht_k<4>(stack, idx, H, W, R, sigma, ht_a, ht_b, weight_mode, eps, keep_dc, partials, st);
    case 8: return launch_ht_k<8>(stack, idx, H, W, R, sigma, ht_a, ht_b, weight_mode, eps, keep_dc, partials, st);
    case 16: return launch_ht_k<16>(stack, idx, H, W, R, sigma, ht_a, ht_b, weight_mode, eps, keep_dc, partials, st);
    case 32: return launch_ht_k<32>(stack, idx, H, W, R, sigma, ht_a, ht_b, weight_mode, eps, keep_dc, partials, st);
    default: return hipErrorInvalidValue;
  }
}

template <int K>
static hipError_t launch_wiener_k(const float* sn, const float* sp, const int16_t* idx, int H, int W, int R,
                                  float sigma, float* partials, hipStream_t st) {
  const GroupArgs g = make_args(H, W, R);
  dim3 grid(g.nTx, (g.nRy + kTPY - 1) / kTPY);
  hipLaunchKernelGGL((group_wiener_kernel<K, kTPY, kTPX>), grid, dim3(256), 0, st, sn, sp, idx, g, sigma,
                     partials);
  return hipGetLastError();
}

hipError_t launch_group_wiener(const float* sn, const float* sp, const int16_t* idx, int H, int W, int R, int K,
                               float sigma, float* partials, hipStream_t st) {
  switch (K) {
    case 2: return launch_wiener_k<2>(sn, sp, idx, H, W, R, sigma, partials, st);
    case 4: return launch_wiener_k<4>(sn, sp, idx, H, W, R, sigma, partials, st);
    case 8: return launch_wiener_k<8>(sn, sp, idx, H, W, R, sigma, partials, st);
    case 16: return launch_wiener_k<16>(sn, sp, idx, H, W, R, sigma, partials, st);
    case 32: return launch_wiener_k<32>(sn, sp, idx, H, W, R, sigma, partials, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(const float* partials, int H, int W, int R, float* out, uint16_t* q, hipStream_t st) {
  const GroupArgs g = make_args(H, W, R);
  const int nTy = (g.nRy + kTPY - 1) / kTPY;
  const int FX = kStep * (kTPX - 1) + kPatch + 2 * R;
  dim3 grid((W + 255) / 256, H);
  hipLaunchKernelGGL(reduce_kernel, grid, dim3(256), 0, st, partials, g, kStep * kTPY, kStep * kTPX, nTy, FX, out,
                     q);
  return hipGetLastError();
}

hipError_t launch_quantize(const float* in, uint16_t* out, size_t n, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(quantize_kernel, dim3(static_cast<unsigned>(blocks > 0 ? blocks : 1)), dim3(256), 0, st, in,
                     out, n);
  return hipGetLastError();
}

}  // namespace gbm3d
