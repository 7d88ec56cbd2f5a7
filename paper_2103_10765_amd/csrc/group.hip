// Collaborative filtering of matched groups and their aggregation.
//
// A workgroup of sixteen (eight for K = 32) waves owns a tile of 8 x 8 references; each wave
// filters one group at a time with lane = 2-D coefficient index (64 lanes =
// 8x8 coefficients) and the group axis in registers:
//   decode the K block positions (lane k decodes slot k, the values are
//   broadcast as scalars), gather the K spectra from the patch stack (one
//   coalesced 256 B load per block), 1-D Haar along the group, shrink,
//   inverse Haar, inverse 2-D transform of the K blocks through a per-wave LDS
//   scratch (separable rows then columns, level by level), group weight, and
//   accumulation of w*U and w into an LDS image of the tile's footprint
//   (every block a reference of the tile can match lies in it: rows
//   3p-R .. 3p+7+R).
// The sums are 64-bit fixed point (2^-40), so their value does not depend on
// the order in which waves add: results are bit-reproducible.  The footprint
// is written once per tile to a partial-sum buffer; a second kernel adds the
// overlapping footprints of every pixel (periodic), divides and optionally
// quantises.  No global atomics are used.
//
// Stage 1 (Sec. 3.1, Sec. 5): bior1.5 stack, hard threshold |C| >= tau_l with
//   tau_l = sigma (a - b l) by Mallat level, 3-D DC kept, weight 1/(TV+eps)
//   (scaled by eps so that it lies in (0, 1]; the weighted average does not
//   change).
// Stage 2 (Sec. 4): DCT stacks of the noisy image and the pilot, Wiener gain
//   W = b^2 / (b^2 + sigma^2) of the pilot spectrum (W = 1 at the 3-D DC)
//   applied to the noisy spectrum, weight 1 / sum W^2.
#include "common.h"
#include "kernels.h"

namespace gbm3d {

namespace {

constexpr int kScratchPitch = 9;                  // LDS row pitch of a parked 8x8 block
constexpr int kBlockFloats = 8 * kScratchPitch;   // 72
constexpr int kTPY = 8, kTPX = 8;                 // references per tile
constexpr int kReduceThreads = 256;
constexpr int kLdsBytes = 160 * 1024;             // LDS of one workgroup

using acc_t = unsigned long long;

struct Foot {
  static constexpr int FYmax = kStep * (kTPY - 1) + kPatch + 2 * kMaxR;
  static constexpr int FXmax = kStep * (kTPX - 1) + kPatch + 2 * kMaxR;
  static constexpr int FXPmax = FXmax + ((8 - FXmax) % 32 + 32) % 32;
  static constexpr int entries = 2 * FYmax * FXPmax;
};

// Waves per tile: sixteen (four per SIMD, the groups' LDS round trips hide
// each other) where the per-wave transform scratch of K blocks still fits
// beside the footprint accumulator, else eight.
template <int K>
constexpr int group_waves() {
  return Foot::entries * static_cast<int>(sizeof(acc_t)) + 16 * K * kBlockFloats * static_cast<int>(sizeof(float)) <=
                 kLdsBytes
             ? 16
             : 8;
}

struct GroupArgs {
  int H, W, R, S, nRy, nRx, nTx, nTy;
  int FY, FX, FXP;
};

__host__ __device__ inline GroupArgs make_args(int H, int W, int R) {
  GroupArgs g;
  g.H = H;
  g.W = W;
  g.R = R;
  g.S = 2 * R + 1;
  g.nRy = (H + kStep - 1) / kStep;
  g.nRx = (W + kStep - 1) / kStep;
  g.nTx = (g.nRx + kTPX - 1) / kTPX;
  g.nTy = (g.nRy + kTPY - 1) / kTPY;
  g.FY = kStep * (kTPY - 1) + kPatch + 2 * R;
  g.FX = kStep * (kTPX - 1) + kPatch + 2 * R;
  g.FXP = g.FX + ((8 - g.FX) % 32 + 32) % 32;
  return g;
}

__host__ __device__ inline int reduce_items(int H, int W) { return H * ((W + kReduceThreads - 1) / kReduceThreads); }

struct HtParams {
  float ht_a, ht_b;
  int weight_mode, keep_dc;
};

// Inverse of one separable level on the leading L x L block of each of the K
// blocks parked at xw[k*72 + a*9 + b]: rows, then columns.
template <int K, int L, typename F>
__device__ __forceinline__ void inverse_level(float* xw, int lane, F&& line) {
  constexpr int items = K * L;
#pragma unroll
  for (int it0 = 0; it0 < items; it0 += kWave) {
    const int it = it0 + lane;
    if (it < items) {
      const int k = it / L, i = it % L;
      float* row = xw + k * kBlockFloats + i * kScratchPitch;
      float x[8], y[8];
#pragma unroll
      for (int j = 0; j < L; ++j) x[j] = row[j];
      line(x, y);
#pragma unroll
      for (int j = 0; j < L; ++j) row[j] = y[j];
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int it0 = 0; it0 < items; it0 += kWave) {
    const int it = it0 + lane;
    if (it < items) {
      const int k = it / L, j = it % L;
      float* col = xw + k * kBlockFloats + j;
      float x[8], y[8];
#pragma unroll
      for (int i = 0; i < L; ++i) x[i] = col[i * kScratchPitch];
      line(x, y);
#pragma unroll
      for (int i = 0; i < L; ++i) col[i * kScratchPitch] = y[i];
    }
  }
  wave_lds_sync();
}

// Block positions of the group of reference (p, q): lane k < K decodes the
// rank r of slot k into a stack position (pixel index) and the offset of the
// block's top-left in the tile's footprint.
template <int K>
__device__ __forceinline__ void slot_pos(const GroupArgs& g, int r, int p, int q, int fy0, int fx0, int lane, int& pos,
                                         int& fo) {
  pos = 0;
  fo = 0;
  if (lane < K) {
    const int dyi = r / g.S, dxi = r - dyi * g.S;
    const int y = kStep * p + dyi - g.R, x = kStep * q + dxi - g.R;
    pos = pmod(y, g.H) * g.W + pmod(x, g.W);
    fo = (y - fy0) * g.FXP + (x - fx0);
  }
}

template <int K>
__device__ __forceinline__ void accumulate(acc_t* acc, const GroupArgs& g, int fo_v, const float (&u)[K], float w,
                                           int lane) {
  const int ab = (lane >> 3) * g.FXP + (lane & 7);
  acc_t* num = acc;
  acc_t* den = acc + g.FY * g.FXP;
  const acc_t wf = static_cast<acc_t>(to_fixed(w));
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int o = __builtin_amdgcn_readlane(fo_v, k) + ab;
    atomicAdd(num + o, static_cast<acc_t>(to_fixed(w * u[k])));
    atomicAdd(den + o, wf);
  }
}

__device__ __forceinline__ void zero_acc(acc_t* acc, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc[i] = 0;
  __syncthreads();
}

__device__ __forceinline__ void flush_acc(const acc_t* acc, int n, acc_t* __restrict__ dst) {
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = acc[i];
  __syncthreads();  // the accumulator is reused by the next item
}

// The groups a wave filters in a tile: reference t = wave + j * WAVES,
// j < kGroups.  Loads run ahead of the filtering: the ranks of group
// j + 2 and the spectra of group j + 1 are in flight while group j is
// filtered.
template <int WAVES>
struct GroupWalk {
  static constexpr int kGroups = kTPY * kTPX / WAVES;
  const GroupArgs& g;
  const int16_t* __restrict__ idx;
  int tyi, txi, wave, lane, fy0, fx0;

  __device__ __forceinline__ bool ref_of(int j, int& p, int& q) const {
    const int t = wave + j * WAVES;
    p = tyi * kTPY + t / kTPX;
    q = txi * kTPX + t % kTPX;
    return j < kGroups && p < g.nRy && q < g.nRx;
  }
  // rank of slot `lane` of group j (0 where there is none)
  template <int K>
  __device__ __forceinline__ int rank(int j) const {
    int p, q;
    if (!ref_of(j, p, q) || lane >= K) return 0;
    return idx[(static_cast<size_t>(p) * g.nRx + q) * K + lane];
  }
  // stack rows of group j from its ranks: v[k] = stack[pos_k * 64 + lane]
  template <int K, int NS>
  __device__ __forceinline__ bool gather(int j, int r, const float* const (&stacks)[NS], float (&v)[NS][K],
                                         int& fo) const {
    int p, q;
    if (!ref_of(j, p, q)) return false;
    int pos_v;
    slot_pos<K>(g, r, p, q, fy0, fx0, lane, pos_v, fo);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      // the block's base address is uniform: it goes into a buffer resource
      // (scalar arithmetic only), the lane offset into the load itself
      const size_t blk = static_cast<size_t>(__builtin_amdgcn_readlane(pos_v, k)) * 64;
#pragma unroll
      for (int s = 0; s < NS; ++s) v[s][k] = load_block_lane(stacks[s] + blk, lane);
    }
    return true;
  }
};

// One work item = one tile of references: stage-1 groups.
template <int K>
__device__ __forceinline__ void group_ht_body(acc_t* acc, float (*scratch)[K * kBlockFloats], const ImgRec& r, int R,
                                              const HtParams& hp, int item) {
  const GroupArgs g = make_args(r.H, r.W, R);
  const float* __restrict__ stack = r.stack_a;
  const int tyi = item / g.nTx, txi = item % g.nTx;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = wave_id();
  const int n_acc = 2 * g.FY * g.FXP;
  zero_acc(acc, n_acc);
  const int fy0 = kStep * tyi * kTPY - g.R;
  const int fx0 = kStep * txi * kTPX - g.R;
  float* xw = scratch[wave];
  const int a = lane >> 3, b = lane & 7;
  const float tau = r.sigma * (hp.ht_a - hp.ht_b * static_cast<float>(bior_level(lane)));
  const bool dc_lane = hp.keep_dc && lane == 0;

  const GroupWalk<group_waves<K>()> walk{g, r.idx, tyi, txi, wave, lane, fy0, fx0};
  const float* const stacks[1] = {stack};
  int r1 = walk.template rank<K>(1);
  float cur[1][K];
  int fo_c = 0;
  bool ok_c = walk.template gather<K, 1>(0, walk.template rank<K>(0), stacks, cur, fo_c);
  for (int j = 0; j < walk.kGroups; ++j) {
    const int r2 = walk.template rank<K>(j + 2);
    float nxt[1][K];
    int fo_n = 0;
    const bool ok_n = walk.template gather<K, 1>(j + 1, r1, stacks, nxt, fo_n);
    if (ok_c) {
    const int fo_v = fo_c;
    float v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = cur[0][k];
    // unnormalised Haar: coefficient k of the orthonormal transform is
    // haar_gain(k) * v[k]; the kept ones are scaled by haar_gain^2 (a power of
    // two) for the unnormalised inverse
    haar_fwd_raw<K>(v);
    int nnz = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool keep = fabsf(v[k]) * haar_gain<K>(k) >= tau || (k == 0 && dc_lane);
      v[k] = keep ? v[k] * haar_gain2<K>(k) : 0.0f;
      nnz += keep ? 1 : 0;
    }
    haar_inv_raw<K>(v);
    wave_lds_sync();  // the previous group's reads of the scratch are done
#pragma unroll
    for (int k = 0; k < K; ++k) xw[k * kBlockFloats + a * kScratchPitch + b] = v[k];
    wave_lds_sync();
    {
      constexpr Mat8 S2 = bior_synthesis(2);
      constexpr Mat8 S4 = bior_synthesis(4);
      constexpr Mat8 S8 = bior_synthesis(8);
      inverse_level<K, 2>(xw, lane, [&](const float* x, float* y) { apply_mat<2>(S2, x, y); });
      inverse_level<K, 4>(xw, lane, [&](const float* x, float* y) { apply_mat<4>(S4, x, y); });
      inverse_level<K, 8>(xw, lane, [&](const float* x, float* y) { apply_mat<8>(S8, x, y); });
    }
    float u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = xw[k * kBlockFloats + a * kScratchPitch + b];
    float w;
    if (hp.weight_mode == 0) {
      float tv = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (k + 1 < K) tv += fabsf(u[k + 1] - u[k]);
        if (b < 7) tv += fabsf(xw[k * kBlockFloats + a * kScratchPitch + b + 1] - u[k]);
        if (a < 7) tv += fabsf(xw[k * kBlockFloats + (a + 1) * kScratchPitch + b] - u[k]);
      }
      w = r.eps / (wave_sum(tv) + r.eps);
    } else if (hp.weight_mode == 1) {
      w = 1.0f / static_cast<float>(max(wave_sum_int(nnz), 1));
    } else {
      w = 1.0f;
    }
    accumulate<K>(acc, g, fo_v, u, w, lane);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) cur[0][k] = nxt[0][k];
    fo_c = fo_n;
    ok_c = ok_n;
    r1 = r2;
  }
  flush_acc(acc, n_acc, r.partials + static_cast<size_t>(item) * n_acc);
}

// One work item = one tile of references: stage-2 groups.
template <int K>
__device__ __forceinline__ void group_wiener_body(acc_t* acc, float (*scratch)[K * kBlockFloats], const ImgRec& r,
                                                  int R, int item) {
  const GroupArgs g = make_args(r.H, r.W, R);
  const float* __restrict__ stack_n = r.stack_a;
  const float* __restrict__ stack_p = r.stack_b;
  const int tyi = item / g.nTx, txi = item % g.nTx;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = wave_id();
  const int n_acc = 2 * g.FY * g.FXP;
  zero_acc(acc, n_acc);
  const int fy0 = kStep * tyi * kTPY - g.R;
  const int fx0 = kStep * txi * kTPX - g.R;
  float* xw = scratch[wave];
  const int a = lane >> 3, b = lane & 7;
  const float s2 = r.sigma * r.sigma;

  const GroupWalk<group_waves<K>()> walk{g, r.idx, tyi, txi, wave, lane, fy0, fx0};
  const float* const stacks[2] = {stack_n, stack_p};
  int r1 = walk.template rank<K>(1);
  float cur[2][K];
  int fo_c = 0;
  bool ok_c = walk.template gather<K, 2>(0, walk.template rank<K>(0), stacks, cur, fo_c);
  for (int j = 0; j < walk.kGroups; ++j) {
    const int r2 = walk.template rank<K>(j + 2);
    float nxt[2][K];
    int fo_n = 0;
    const bool ok_n = walk.template gather<K, 2>(j + 1, r1, stacks, nxt, fo_n);
    if (ok_c) {
    const int fo_v = fo_c;
    float vn[K], vp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      vn[k] = cur[0][k];
      vp[k] = cur[1][k];
    }
    // unnormalised Haar (orthonormal coefficient k = haar_gain(k) * raw);
    // haar_gain^2 is a power of two, so b^2 and the rescaling are exact
    haar_fwd_raw<K>(vp);
    haar_fwd_raw<K>(vn);
    float sw2 = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float b2 = vp[k] * vp[k] * haar_gain2<K>(k);
      float wt = b2 * __builtin_amdgcn_rcpf(b2 + s2);
      if (k == 0 && lane == 0) wt = 1.0f;
      vn[k] *= wt * haar_gain2<K>(k);
      sw2 = fmaf(wt, wt, sw2);
    }
    const float w = 1.0f / wave_sum(sw2);
    haar_inv_raw<K>(vn);
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < K; ++k) xw[k * kBlockFloats + a * kScratchPitch + b] = vn[k];
    wave_lds_sync();
    inverse_level<K, 8>(xw, lane, [&](const float* x, float* y) { dct8_inv(x, y); });
    float u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = xw[k * kBlockFloats + a * kScratchPitch + b];
    accumulate<K>(acc, g, fo_v, u, w, lane);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      cur[0][k] = nxt[0][k];
      cur[1][k] = nxt[1][k];
    }
    fo_c = fo_n;
    ok_c = ok_n;
    r1 = r2;
  }
  flush_acc(acc, n_acc, r.partials + static_cast<size_t>(item) * n_acc);
}

template <int K, bool BATCH>
__global__ __launch_bounds__(group_waves<K>() * kWave) void group_ht_kernel(ImgRec one, WorkList wl, int R,
                                                                            HtParams hp) {
  __shared__ acc_t acc[Foot::entries];
  __shared__ float scratch[group_waves<K>()][K * kBlockFloats];
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) { group_ht_body<K>(acc, scratch, r, R, hp, item); });
}

template <int K, bool BATCH>
__global__ __launch_bounds__(group_waves<K>() * kWave) void group_wiener_kernel(ImgRec one, WorkList wl, int R) {
  __shared__ acc_t acc[Foot::entries];
  __shared__ float scratch[group_waves<K>()][K * kBlockFloats];
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) { group_wiener_body<K>(acc, scratch, r, R, item); });
}

// floor(a / b) for b > 0
__device__ __forceinline__ int fdiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// One work item = 256 pixels of one row: sum of the partial footprints
// covering each pixel (periodic), then normalise.
__device__ __forceinline__ void reduce_body(const ImgRec& r, int R, int final_stage, int item) {
  const GroupArgs g = make_args(r.H, r.W, R);
  const acc_t* __restrict__ partials = r.partials;
  float* __restrict__ out = final_stage ? r.out : r.basic;
  uint16_t* __restrict__ q = final_stage ? nullptr : r.q;
  const int TY = kStep * kTPY, TX = kStep * kTPX;
  const int xb = (g.W + kReduceThreads - 1) / kReduceThreads;
  const int y = item / xb;
  const int x = (item % xb) * kReduceThreads + static_cast<int>(threadIdx.x);
  if (x >= g.W) return;
  // candidate (tile row, local row) pairs for y; the footprint of tile row t
  // covers unwrapped rows [t*TY - R, t*TY - R + FY)
  int cty[16], cly[16], ny = 0;
  {
    const int lo = -R, hi = (g.nTy - 1) * TY - R + g.FY;
    for (int yy = y + fdiv(lo - y + g.H - 1, g.H) * g.H; yy < hi; yy += g.H) {
      const int t0 = max(0, fdiv(yy + R - g.FY, TY) + 1), t1 = min(g.nTy - 1, fdiv(yy + R, TY));
      for (int t = t0; t <= t1 && ny < 16; ++t) {
        cty[ny] = t;
        cly[ny] = yy - (t * TY - R);
        ++ny;
      }
    }
  }
  int ctx[16], clx[16], nx = 0;
  {
    const int lo = -R, hi = (g.nTx - 1) * TX - R + g.FX;
    for (int xx = x + fdiv(lo - x + g.W - 1, g.W) * g.W; xx < hi; xx += g.W) {
      const int t0 = max(0, fdiv(xx + R - g.FX, TX) + 1), t1 = min(g.nTx - 1, fdiv(xx + R, TX));
      for (int t = t0; t <= t1 && nx < 16; ++t) {
        ctx[nx] = t;
        clx[nx] = xx - (t * TX - R);
        ++nx;
      }
    }
  }
  const size_t plane = static_cast<size_t>(g.FY) * g.FXP;
  auto at = [&](int i, int j) -> const acc_t* {
    return partials + (static_cast<size_t>(cty[i]) * g.nTx + ctx[j]) * 2 * plane +
           static_cast<size_t>(cly[i]) * g.FXP + clx[j];
  };
  acc_t num = 0, den = 0;
  if (ny <= 3 && nx <= 3) {
    // the usual case: at most 3 x 3 footprints; every load is issued before
    // the sums so their latencies overlap
    acc_t vn[3][3], vd[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        vn[i][j] = 0;
        vd[i][j] = 0;
        if (i < ny && j < nx) {
          const acc_t* t = at(i, j);
          vn[i][j] = t[0];
          vd[i][j] = t[plane];
        }
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        num += vn[i][j];
        den += vd[i][j];
      }
  } else {
    // small images whose footprints wrap around more than once
    for (int i = 0; i < ny; ++i)
      for (int j = 0; j < nx; ++j) {
        const acc_t* t = at(i, j);
        num += t[0];
        den += t[plane];
      }
  }
  const float v = static_cast<float>(static_cast<double>(static_cast<long long>(num)) /
                                     static_cast<double>(static_cast<long long>(den)));
  const size_t o = static_cast<size_t>(y) * g.W + x;
  out[o] = v;
  if (q) {
    const double d = static_cast<double>(fminf(fmaxf(v, 0.0f), 1.0f));
    q[o] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
  }
}

template <bool BATCH>
__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(ImgRec one, WorkList wl, int R, int final_stage) {
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) { reduce_body(r, R, final_stage, item); });
}

__global__ void quantize_kernel(const float* __restrict__ in, uint16_t* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const double d = static_cast<double>(fminf(fmaxf(in[i], 0.0f), 1.0f));
    out[i] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
  }
}

}  // namespace

size_t partials_bytes(int H, int W, int R) {
  const GroupArgs g = make_args(H, W, R);
  return static_cast<size_t>(g.nTy) * g.nTx * 2 * g.FY * g.FXP * sizeof(acc_t);
}

int group_items_for(int H, int W, int R) {
  const GroupArgs g = make_args(H, W, R);
  return g.nTy * g.nTx;
}

int reduce_items_for(int H, int W) { return reduce_items(H, W); }

template <int K>
static hipError_t launch_ht_k(const ImgRec& one, const WorkList* wl, int R, const HtParams& hp, int grid_cap,
                              hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((group_ht_kernel<K, false>), dim3(group_items_for(one.H, one.W, R)), dim3(group_waves<K>() * kWave), 0, st,
                       one, WorkList{}, R, hp);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((group_ht_kernel<K, true>), dim3(std::min(wl->total, grid_cap)), dim3(group_waves<K>() * kWave), 0, st, one,
                       *wl, R, hp);
  }
  return hipGetLastError();
}

hipError_t launch_group_ht(const ImgRec& one, const WorkList* wl, int R, int K, float ht_a, float ht_b,
                           int weight_mode, int keep_dc, int grid_cap, hipStream_t st) {
  const HtParams hp{ht_a, ht_b, weight_mode, keep_dc};
  switch (K) {
    case 2: return launch_ht_k<2>(one, wl, R, hp, grid_cap, st);
    case 4: return launch_ht_k<4>(one, wl, R, hp, grid_cap, st);
    case 8: return launch_ht_k<8>(one, wl, R, hp, grid_cap, st);
    case 16: return launch_ht_k<16>(one, wl, R, hp, grid_cap, st);
    case 32: return launch_ht_k<32>(one, wl, R, hp, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

template <int K>
static hipError_t launch_wiener_k(const ImgRec& one, const WorkList* wl, int R, int grid_cap, hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((group_wiener_kernel<K, false>), dim3(group_items_for(one.H, one.W, R)), dim3(group_waves<K>() * kWave), 0,
                       st, one, WorkList{}, R);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((group_wiener_kernel<K, true>), dim3(std::min(wl->total, grid_cap)), dim3(group_waves<K>() * kWave), 0, st,
                       one, *wl, R);
  }
  return hipGetLastError();
}

hipError_t launch_group_wiener(const ImgRec& one, const WorkList* wl, int R, int K, int grid_cap, hipStream_t st) {
  switch (K) {
    case 2: return launch_wiener_k<2>(one, wl, R, grid_cap, st);
    case 4: return launch_wiener_k<4>(one, wl, R, grid_cap, st);
    case 8: return launch_wiener_k<8>(one, wl, R, grid_cap, st);
    case 16: return launch_wiener_k<16>(one, wl, R, grid_cap, st);
    case 32: return launch_wiener_k<32>(one, wl, R, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(const ImgRec& one, const WorkList* wl, int R, int final_stage, int grid_cap,
                         hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((reduce_kernel<false>), dim3(reduce_items(one.H, one.W)), dim3(kReduceThreads), 0, st, one,
                       WorkList{}, R, final_stage);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((reduce_kernel<true>), dim3(std::min(wl->total, grid_cap)), dim3(kReduceThreads), 0, st,
                       one, *wl, R, final_stage);
  }
  return hipGetLastError();
}

hipError_t launch_quantize(const float* in, uint16_t* out, size_t n, hipStream_t st) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(quantize_kernel, dim3(static_cast<unsigned>(blocks > 0 ? blocks : 1)), dim3(256), 0, st, in,
                     out, n);
  return hipGetLastError();
}

}  // namespace gbm3d
