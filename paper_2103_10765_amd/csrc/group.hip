// Collaborative filtering of matched groups and their aggregation.
//
// A workgroup of 8 to 16 waves owns a tile of 8 x 8 references; each wave
// filters one group at a time with lane = 2-D coefficient index (64 lanes =
// 8x8 coefficients) and the group axis in registers:
//   decode the K block positions (lane k decodes slot k, the values are
//   broadcast as scalars), gather the K spectra from the patch stack (one
//   coalesced 256 B load per block), 1-D Haar along the group, shrink,
//   inverse Haar, inverse 2-D transform of the K blocks through a per-wave LDS
//   scratch (separable rows then columns, level by level, at most 16 blocks
//   at a time), group weight, and accumulation of w*U into an LDS image of
//   the tile's footprint (every block a reference of the tile can match lies
//   in it: rows 3p-R .. 3p+7+R).
// The denominator sum of w over the blocks covering a pixel is not spread
// over 64 pixels per block: w is added once per block at the block's
// top-left pixel of an image-sized array (global integer atomics, one
// instruction per group), and the pixel's denominator is the 8 x 8 box sum
// of that array (periodic).
// All sums are 64-bit fixed point (2^-40), so their value does not depend on
// the order in which waves add: results are bit-reproducible.  The footprint
// is written once per tile to a partial-sum buffer; a second kernel adds the
// overlapping footprints of every pixel (periodic), forms the box sum,
// divides and optionally quantises.
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
  static constexpr int entries = FYmax * FXPmax;
};

// Launch shape of a group kernel.  The hard-threshold kernel (K <= 16; the
// WIDE shape, which the autotuner may swap for the one-tile shape below) runs
// two tiles per CU: 12 waves each (six per SIMD), inverse
// transforms 8 blocks at a time through each wave's scratch, no prefetch of
// the next group (the other waves hide the loads).  Otherwise one tile per
// CU: sixteen waves (four per SIMD) where a 16-block scratch per wave fits
// beside the footprint accumulator and the filter's registers fit a quarter
// of the register file, else eight; small groups keep the next group's
// spectra in flight.  The hard-threshold filter holds all K inverse blocks
// until its weight is known, which does not fit sixteen waves for K = 32;
// the batched variant carries more state per wave and keeps one tile per CU.
template <int K, bool HT, bool BATCH, bool WIDE = true>
struct GroupCfg {
  static constexpr bool two_tiles = HT && K <= 16 && WIDE;
  static constexpr int chunk = two_tiles ? (K > 8 ? 8 : K) : (K > 16 ? 16 : K);
  static constexpr int rank_bytes = kTPY * kTPX * K * 2;  // the tile's ranks (int16)
  static constexpr int waves =
      two_tiles ? 12
      : Foot::entries * static_cast<int>(sizeof(acc_t)) +
                      16 * chunk * kBlockFloats * static_cast<int>(sizeof(float)) + rank_bytes <=
                  kLdsBytes &&
              !(HT && K > 16)
          ? 16
          : 8;
  static constexpr int tiles = two_tiles ? 2 : 1;
  static constexpr bool prefetch = !two_tiles && K <= 16;
  static constexpr int threads = waves * kWave;
  static constexpr int min_waves_per_simd = waves * tiles / 4;
  static_assert(tiles * (Foot::entries * static_cast<int>(sizeof(acc_t)) +
                         waves * chunk * kBlockFloats * static_cast<int>(sizeof(float)) + rank_bytes) <=
                    kLdsBytes,
                "LDS of the tiles sharing a CU");
};

struct GroupArgs {
  int H, W, R, S, nRy, nRx, nTx, nTy;
  int FY, FX, FXP;
  float invS;  // 1 / S for the rank decode
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
  g.invS = 1.0f / static_cast<float>(g.S);
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
    // r / S in float: r + 1/2 lies at least 1/(2S) from a multiple of S and
    // r < S^2 <= 1521, far inside float's exact range
    const int dyi = static_cast<int>((static_cast<float>(r) + 0.5f) * g.invS), dxi = r - dyi * g.S;
    const int y = kStep * p + dyi - g.R, x = kStep * q + dxi - g.R;
    // -R <= y < H + R and H >= S > R + 1: at most one period away (same for x)
    const int yw = y < 0 ? y + g.H : (y >= g.H ? y - g.H : y);
    const int xw = x < 0 ? x + g.W : (x >= g.W ? x - g.W : x);
    pos = yw * g.W + xw;
    fo = (y - fy0) * g.FXP + (x - fx0);
  }
}

// w * u[k] into the footprint for blocks k0 .. k0 + N - 1 (u holds their values)
template <int N>
__device__ __forceinline__ void accumulate(acc_t* acc, const GroupArgs& g, int fo_v, int k0, const float (&u)[N],
                                           float w, int lane) {
  const int ab = (lane >> 3) * g.FXP + (lane & 7);
  const float ws = w * kFixScaleF;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int o = __builtin_amdgcn_readlane(fo_v, k0 + k) + ab;
    atomicAdd(acc + o, static_cast<acc_t>(to_fixed_scaled(ws * u[k])));
  }
}

// w at the top-left pixel pos of each of the K blocks (lane k holds slot k's);
// integer addition, so the order of the atomics does not matter
template <int K>
__device__ __forceinline__ void add_block_weights(acc_t* bw, int pos_v, float w, int lane) {
  if (lane < K)
    __hip_atomic_fetch_add(to_global(bw) + pos_v, static_cast<acc_t>(to_fixed(w)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void zero_acc(acc_t* acc, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc[i] = 0;
  __syncthreads();
}

// The tile's footprint (origin fy0, fx0 in unwrapped image coordinates) added
// into the image's numerator sums at the periodic positions it covers, one
// agent-scope integer atomic per nonzero cell: integer addition, so the sums
// do not depend on the order in which tiles arrive.  A wave takes whole
// footprint rows, a lane the same columns of each.
__device__ __forceinline__ void flush_acc(const acc_t* acc, const GroupArgs& g, int fy0, int fx0,
                                          acc_t* __restrict__ num) {
  __syncthreads();
  const auto gnum = to_global(num);
  const int lane = threadIdx.x & (kWave - 1);
  const int waves = static_cast<int>(blockDim.x) / kWave;
  // -R <= fy0 and fy0 + FY <= H + FY - R + 1: with H > FY every footprint row
  // is at most one period away (same for the columns)
  const bool once = g.H > g.FY && g.W > g.FX;
  constexpr int kPasses = (Foot::FXmax + kWave - 1) / kWave;
  int xs[kPasses];
#pragma unroll
  for (int p = 0; p < kPasses; ++p) {
    const int x = fx0 + p * kWave + lane;
    xs[p] = once ? x + (x < 0 ? g.W : (x >= g.W ? -g.W : 0)) : pmod(x, g.W);
  }
  for (int fy = wave_id(); fy < g.FY; fy += waves) {
    int y = fy0 + fy;
    y = once ? y + (y < 0 ? g.H : (y >= g.H ? -g.H : 0)) : pmod(y, g.H);
    const auto row = gnum + static_cast<size_t>(y) * g.W;
    const acc_t* cells = acc + fy * g.FXP;
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      const int fx = p * kWave + lane;
      const acc_t v = fx < g.FX ? cells[fx] : 0;
      if (v != 0) __hip_atomic_fetch_add(row + xs[p], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();  // the accumulator is reused by the next item
}

// The tile's match ranks [reference t][K] into LDS (t = 8 * row + column of
// the tile's 8 x 8 references; references past the image's last row or
// column read a clamped in-bounds entry that no group uses), every thread's
// loads issued before the first is stored: one memory round trip per tile
// instead of one per group.  The caller's next barrier publishes them.
template <int K, int THREADS>
__device__ __forceinline__ void load_ranks(int16_t* ranks, const GroupArgs& g, const int16_t* idx_, int tyi,
                                           int txi) {
  const auto idx = to_global(idx_);
  constexpr int n = kTPY * kTPX * K;
  constexpr int iters = (n + THREADS - 1) / THREADS;
  int v[iters];
#pragma unroll
  for (int it = 0; it < iters; ++it) {
    const int e = min(static_cast<int>(threadIdx.x) + it * THREADS, n - 1);
    const int t = e / K, k = e % K;
    const int p = min(tyi * kTPY + t / kTPX, g.nRy - 1), q = min(txi * kTPX + t % kTPX, g.nRx - 1);
    v[it] = idx[(static_cast<size_t>(p) * g.nRx + q) * K + k];
  }
#pragma unroll
  for (int it = 0; it < iters; ++it) {
    const int e = static_cast<int>(threadIdx.x) + it * THREADS;
    if (e < n) ranks[e] = static_cast<int16_t>(v[it]);
  }
}

// The groups a wave filters in a tile: reference t = wave + j * WAVES,
// j < kGroups.
template <int WAVES>
struct GroupWalk {
  static constexpr int kGroups = (kTPY * kTPX + WAVES - 1) / WAVES;
  const GroupArgs& g;
  const int16_t* ranks;  // the tile's match ranks in LDS [reference t][K]
  int tyi, txi, wave, lane, fy0, fx0;

  __device__ __forceinline__ bool ref_of(int j, int& p, int& q) const {
    const int t = wave + j * WAVES;
    p = tyi * kTPY + t / kTPX;
    q = txi * kTPX + t % kTPX;
    return j < kGroups && t < kTPY * kTPX && p < g.nRy && q < g.nRx;
  }
  // rank of slot `lane` of group j, for lanes below K of a group that exists
  // (gather reads nothing else)
  template <int K>
  __device__ __forceinline__ int rank(int j) const {
    const int t = wave + j * WAVES;
    return t < kTPY * kTPX ? ranks[t * K + (lane & (K - 1))] : 0;
  }
  // stack rows of group j from its ranks: v[k] = stack[pos_k * 64 + lane];
  // lane k < K returns slot k's pixel index and footprint offset
  template <int K, int NS>
  __device__ __forceinline__ bool gather(int j, int r, const float* const (&stacks)[NS], float (&v)[NS][K], int& fo,
                                         int& pos_v) const {
    int p, q;
    if (!ref_of(j, p, q)) return false;
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
  // the pixels of group j's blocks instead of their spectra: v[k] = z at
  // (row lane / 8, column lane % 8) of slot k's block (periodic),
  // z = Z / 65535 as the stack kernel reads it
  template <int K>
  __device__ __forceinline__ bool gather_pixels(int j, int r, const uint16_t* __restrict__ img, float (&v)[1][K],
                                                int& fo, int& pos_v) const {
    int p, q;
    if (!ref_of(j, p, q)) return false;
    slot_pos<K>(g, r, p, q, fy0, fx0, lane, pos_v, fo);
    const int a = lane >> 3, b = lane & 7;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int pos = __builtin_amdgcn_readlane(pos_v, k);
      const int y = pos / g.W, x = pos - y * g.W;
      const int yy = y + a >= g.H ? y + a - g.H : y + a, xx = x + b >= g.W ? x + b - g.W : x + b;
      v[0][k] = static_cast<float>(to_global(img)[static_cast<size_t>(yy) * g.W + xx]) * (1.0f / 65535.0f);
    }
    return true;
  }
};

// The forward 2-D bior1.5 transform (three periodic Mallat levels, rows then
// columns at each, as the stage-1 stack computes it) of K blocks whose
// pixels the lanes hold (lane = pixel a * 8 + b), CH blocks at a time
// through the wave's scratch (the same separable passes as the inverse);
// afterwards v[k] is coefficient `lane` of block k.
template <int K, int CH>
__device__ __forceinline__ void forward_blocks(float* xw, int lane, float (&v)[K]) {
  const int a = lane >> 3, b = lane & 7;
  constexpr Mat8 A8 = bior_analysis(8);
  constexpr Mat8 A4 = bior_analysis(4);
  constexpr Mat8 A2 = bior_analysis(2);
#pragma unroll
  for (int c0 = 0; c0 < K; c0 += CH) {
    wave_lds_sync();  // earlier reads of the scratch are done
#pragma unroll
    for (int k = 0; k < CH; ++k) xw[k * kBlockFloats + a * kScratchPitch + b] = v[c0 + k];
    wave_lds_sync();
    inverse_level<CH, 8>(xw, lane, [&](const float* x, float* y) { apply_mat<8>(A8, x, y); });
    inverse_level<CH, 4>(xw, lane, [&](const float* x, float* y) { apply_mat<4>(A4, x, y); });
    inverse_level<CH, 2>(xw, lane, [&](const float* x, float* y) { apply_mat<2>(A2, x, y); });
#pragma unroll
    for (int k = 0; k < CH; ++k) v[c0 + k] = xw[k * kBlockFloats + a * kScratchPitch + b];
  }
}

// Runs filter(v, fo_v, pos_v) on every group of this wave in the tile, v the
// gathered spectra.  Small groups also keep the next group's spectra in
// flight; large ones leave the registers to the filter (sixteen waves per
// tile hide the loads instead).
template <int K, int NS, bool PREFETCH, int WAVES, typename F>
__device__ __forceinline__ void for_each_group(const GroupWalk<WAVES>& walk, const float* const (&stacks)[NS],
                                               F&& filter) {
  if constexpr (PREFETCH) {
    int r1 = walk.template rank<K>(1);
    float cur[NS][K];
    int fo_c = 0, pos_c = 0;
    bool ok_c = walk.template gather<K, NS>(0, walk.template rank<K>(0), stacks, cur, fo_c, pos_c);
    for (int j = 0; j < walk.kGroups; ++j) {
      const int r2 = walk.template rank<K>(j + 2);
      float nxt[NS][K];
      int fo_n = 0, pos_n = 0;
      const bool ok_n = walk.template gather<K, NS>(j + 1, r1, stacks, nxt, fo_n, pos_n);
      if (ok_c) filter(cur, fo_c, pos_c);
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < K; ++k) cur[s][k] = nxt[s][k];
      fo_c = fo_n;
      pos_c = pos_n;
      ok_c = ok_n;
      r1 = r2;
    }
  } else {
    int r0 = walk.template rank<K>(0);
    for (int j = 0; j < walk.kGroups; ++j) {
      const int r1 = walk.template rank<K>(j + 1);
      float cur[NS][K];
      int fo = 0, pos = 0;
      if (walk.template gather<K, NS>(j, r0, stacks, cur, fo, pos)) filter(cur, fo, pos);
      r0 = r1;
    }
  }
}

// One work item = one tile of references: stage-1 groups.  RECOMPUTE: the
// blocks' spectra are computed here from the image's pixels instead of
// gathered from the bior1.5 stack.
template <int K, bool BATCH, bool RECOMPUTE, bool WIDE>
__device__ __forceinline__ void group_ht_body(acc_t* acc,
                                              float (*scratch)[GroupCfg<K, true, BATCH, WIDE>::chunk * kBlockFloats],
                                              int16_t* ranks, const ImgRec& r, int R, const HtParams& hp, int item) {
  const GroupArgs g = make_args(r.H, r.W, R);
  const int tyi = item / g.nTx, txi = item % g.nTx;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = wave_id();
  const int n_acc = g.FY * g.FXP;
  load_ranks<K, GroupCfg<K, true, BATCH, WIDE>::threads>(ranks, g, r.idx, tyi, txi);
  zero_acc(acc, n_acc);
  const int fy0 = kStep * tyi * kTPY - g.R;
  const int fx0 = kStep * txi * kTPX - g.R;
  float* xw = scratch[wave];
  const int a = lane >> 3, b = lane & 7;
  const float tau = r.sigma * (hp.ht_a - hp.ht_b * static_cast<float>(bior_level(lane)));
  const bool dc_lane = hp.keep_dc && lane == 0;
  acc_t* bw = r.partials;  // block-start weights

  using Cfg = GroupCfg<K, true, BATCH, WIDE>;
  const GroupWalk<Cfg::waves> walk{g, ranks, tyi, txi, wave, lane, fy0, fx0};
  const float* const stacks[1] = {r.stack_a};
  auto filter = [&](const float (&cur)[1][K], int fo_v, int pos_v) {
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
    // inverse 2-D transform, kChunk blocks at a time through the scratch; the
    // spatial total-variation terms are read while a chunk is parked there
    constexpr int CH = Cfg::chunk;
    constexpr Mat8 S2 = bior_synthesis(2);
    constexpr Mat8 S4 = bior_synthesis(4);
    constexpr Mat8 S8 = bior_synthesis(8);
    float u[K];
    float tv = 0.0f;
#pragma unroll
    for (int c0 = 0; c0 < K; c0 += CH) {
      wave_lds_sync();  // earlier reads of the scratch are done
#pragma unroll
      for (int k = 0; k < CH; ++k) xw[k * kBlockFloats + a * kScratchPitch + b] = v[c0 + k];
      wave_lds_sync();
      inverse_level<CH, 2>(xw, lane, [&](const float* x, float* y) { apply_mat<2>(S2, x, y); });
      inverse_level<CH, 4>(xw, lane, [&](const float* x, float* y) { apply_mat<4>(S4, x, y); });
      inverse_level<CH, 8>(xw, lane, [&](const float* x, float* y) { apply_mat<8>(S8, x, y); });
#pragma unroll
      for (int k = 0; k < CH; ++k) u[c0 + k] = xw[k * kBlockFloats + a * kScratchPitch + b];
      if (hp.weight_mode == 0) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
          if (b < 7) tv += fabsf(xw[k * kBlockFloats + a * kScratchPitch + b + 1] - u[c0 + k]);
          if (a < 7) tv += fabsf(xw[k * kBlockFloats + (a + 1) * kScratchPitch + b] - u[c0 + k]);
        }
      }
    }
    float w;
    if (hp.weight_mode == 0) {
#pragma unroll
      for (int k = 0; k + 1 < K; ++k) tv += fabsf(u[k + 1] - u[k]);
      w = r.eps / (wave_sum(tv) + r.eps);
    } else if (hp.weight_mode == 1) {
      w = 1.0f / static_cast<float>(max(wave_sum_int(nnz), 1));
    } else {
      w = 1.0f;
    }
    accumulate<K>(acc, g, fo_v, 0, u, w, lane);
    add_block_weights<K>(bw, pos_v, w, lane);
  };
  if constexpr (RECOMPUTE) {
    int r0 = walk.template rank<K>(0);
    for (int j = 0; j < walk.kGroups; ++j) {
      const int r1 = walk.template rank<K>(j + 1);
      float cur[1][K];
      int fo = 0, pos = 0;
      if (walk.template gather_pixels<K>(j, r0, r.noisy, cur, fo, pos)) {
        forward_blocks<K, Cfg::chunk>(xw, lane, cur[0]);
        filter(cur, fo, pos);
      }
      r0 = r1;
    }
  } else {
    for_each_group<K, 1, Cfg::prefetch>(walk, stacks, filter);
  }
  flush_acc(acc, g, fy0, fx0, numerator_sums(r));
}

// One work item = one tile of references: stage-2 groups.
template <int K, bool BATCH>
__device__ __forceinline__ void group_wiener_body(acc_t* acc,
                                                  float (*scratch)[GroupCfg<K, false, BATCH>::chunk * kBlockFloats],
                                                  int16_t* ranks, const ImgRec& r, int R, int item) {
  const GroupArgs g = make_args(r.H, r.W, R);
  const int tyi = item / g.nTx, txi = item % g.nTx;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = wave_id();
  const int n_acc = g.FY * g.FXP;
  load_ranks<K, GroupCfg<K, false, BATCH>::threads>(ranks, g, r.idx, tyi, txi);
  zero_acc(acc, n_acc);
  const int fy0 = kStep * tyi * kTPY - g.R;
  const int fx0 = kStep * txi * kTPX - g.R;
  float* xw = scratch[wave];
  const int a = lane >> 3, b = lane & 7;
  const float s2 = r.sigma * r.sigma;
  acc_t* bw = r.partials;  // block-start weights

  using Cfg = GroupCfg<K, false, BATCH>;
  const GroupWalk<Cfg::waves> walk{g, ranks, tyi, txi, wave, lane, fy0, fx0};
  // the walk gathers the pilot's spectra; the noisy ones are loaded once the
  // gains are known, so the two groups are never in registers together
  const float* const stacks[1] = {r.stack_b};
  const float* __restrict__ stack_n = r.stack_a;
  for_each_group<K, 1, Cfg::prefetch>(walk, stacks, [&](const float (&cur)[1][K], int fo_v, int pos_v) {
    float vp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) vp[k] = cur[0][k];
    // unnormalised Haar (orthonormal coefficient k = haar_gain(k) * raw);
    // haar_gain^2 is a power of two, so b^2 and the rescaling are exact
    haar_fwd_raw<K>(vp);
    float wt[K];
    float sw2 = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const float b2 = vp[k] * vp[k] * haar_gain2<K>(k);
      wt[k] = b2 * __builtin_amdgcn_rcpf(b2 + s2);
      if (k == 0 && lane == 0) wt[k] = 1.0f;
      sw2 = fmaf(wt[k], wt[k], sw2);
    }
    __builtin_amdgcn_sched_barrier(0);
    float vn[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      vn[k] = load_block_lane(stack_n + static_cast<size_t>(__builtin_amdgcn_readlane(pos_v, k)) * 64, lane);
    haar_fwd_raw<K>(vn);
#pragma unroll
    for (int k = 0; k < K; ++k) vn[k] *= wt[k] * haar_gain2<K>(k);
    const float w = 1.0f / wave_sum(sw2);
    haar_inv_raw<K>(vn);
    // the weight is known: each chunk is aggregated as soon as it is back
    constexpr int CH = Cfg::chunk;
#pragma unroll
    for (int c0 = 0; c0 < K; c0 += CH) {
      wave_lds_sync();  // earlier reads of the scratch are done
#pragma unroll
      for (int k = 0; k < CH; ++k) xw[k * kBlockFloats + a * kScratchPitch + b] = vn[c0 + k];
      wave_lds_sync();
      inverse_level<CH, 8>(xw, lane, [&](const float* x, float* y) { dct8_inv(x, y); });
      float u[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) u[k] = xw[k * kBlockFloats + a * kScratchPitch + b];
      accumulate<CH>(acc, g, fo_v, c0, u, w, lane);
    }
    add_block_weights<K>(bw, pos_v, w, lane);
  });
  flush_acc(acc, g, fy0, fx0, numerator_sums(r));
}

// (the second launch bound is the minimum number of waves per SIMD)
template <int K, bool BATCH, bool RECOMPUTE, bool WIDE>
__global__ __launch_bounds__((GroupCfg<K, true, BATCH, WIDE>::threads),
                             (GroupCfg<K, true, BATCH, WIDE>::min_waves_per_simd)) void group_ht_kernel(ImgRec one,
                                                                                                         WorkList wl,
                                                                                                         int R,
                                                                                                         HtParams hp) {
  using Cfg = GroupCfg<K, true, BATCH, WIDE>;
  __shared__ acc_t acc[Foot::entries];
  __shared__ float scratch[Cfg::waves][Cfg::chunk * kBlockFloats];
  __shared__ int16_t ranks[kTPY * kTPX * K];
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) {
    group_ht_body<K, BATCH, RECOMPUTE, WIDE>(acc, scratch, ranks, r, R, hp, item);
  });
}

// the block-start weights and numerator sums the aggregation adds into (the
// bior1.5 stack launch clears them otherwise)
__global__ void clear_weights_kernel(acc_t* __restrict__ w, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    w[i] = 0;
}

template <int K, bool BATCH>
__global__ __launch_bounds__((GroupCfg<K, false, BATCH>::threads)) void group_wiener_kernel(ImgRec one, WorkList wl,
                                                                                             int R) {
  using Cfg = GroupCfg<K, false, BATCH>;
  __shared__ acc_t acc[Foot::entries];
  __shared__ float scratch[Cfg::waves][Cfg::chunk * kBlockFloats];
  __shared__ int16_t ranks[kTPY * kTPX * K];
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) {
    group_wiener_body<K, BATCH>(acc, scratch, ranks, r, R, item);
  });
}

// One work item = 256 pixels of one row: the numerator sum of each pixel over
// the 8 x 8 box sum of the block-start weights ending at it, then normalise.
__device__ __forceinline__ void reduce_body(acc_t* colsum, const ImgRec& r, int final_stage, int item) {
  const auto bw = to_global(static_cast<const acc_t*>(r.partials));
  const auto nums = to_global(static_cast<const acc_t*>(numerator_sums(r)));
  const auto out = to_global(final_stage ? r.out : r.basic);
  const bool with_q = !final_stage && r.q != nullptr;
  const auto q = to_global(r.q);
  const int H = r.H, W = r.W;
  const int xb = (W + kReduceThreads - 1) / kReduceThreads;
  const int y = item / xb;
  const int xs = (item % xb) * kReduceThreads;
  const int x = xs + static_cast<int>(threadIdx.x);
  const bool active = x < W;
  const size_t o = static_cast<size_t>(y) * W + x;
  // the numerator's load is issued before the weights' column sums below, so
  // the two round trips overlap
  const acc_t num = active ? nums[o] : 0;
  // colsum[c] = sum over rows y-7..y of the weights at column xs - 7 + c
  // (H, W >= 8, so a row index wraps at most once; so does a column index
  // when W covers a chunk and its 7-column margin)
  const bool wide = W >= kReduceThreads + 7;
  constexpr int kCols = kReduceThreads + 7;
  auto column = [&](int c) {
    const int xi = xs - 7 + c;
    return wide ? xi + (xi < 0 ? W : (xi >= W ? -W : 0)) : pmod(xi, W);
  };
  auto rows_of = [&](int xi, acc_t (&v)[8]) {
#pragma unroll
    for (int dy = 0; dy < 8; ++dy) {
      const int yy = y - dy < 0 ? y - dy + H : y - dy;
      v[dy] = bw[static_cast<size_t>(yy) * W + xi];
    }
  };
  auto sum8 = [](const acc_t (&v)[8]) {
    acc_t sum = 0;
#pragma unroll
    for (int dy = 0; dy < 8; ++dy) sum += v[dy];
    return sum;
  };
  // column c = thread, and the last 7 columns in the first wave, whose two
  // sets of loads go out together (one round trip for the block)
  const int c0 = static_cast<int>(threadIdx.x);
  acc_t v0[8];
  rows_of(column(c0), v0);
  if (threadIdx.x < kWave) {
    const int c1 = min(c0 + kReduceThreads, kCols - 1);
    acc_t v1[8];
    rows_of(column(c1), v1);
    if (c0 + kReduceThreads < kCols) colsum[c1] = sum8(v1);
  }
  colsum[c0] = sum8(v0);
  static_assert(kCols - kReduceThreads <= kWave, "the extra columns fit the first wave");
  __syncthreads();
  if (active) {
    acc_t den = 0;
#pragma unroll
    for (int dx = 0; dx < 8; ++dx) den += colsum[threadIdx.x + 7 - dx];
    const float v = static_cast<float>(static_cast<double>(static_cast<long long>(num)) /
                                       static_cast<double>(static_cast<long long>(den)));
    out[o] = v;
    if (with_q) {
      const double d = static_cast<double>(fminf(fmaxf(v, 0.0f), 1.0f));
      q[o] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
    }
  }
}

template <bool BATCH>
__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(ImgRec one, WorkList wl, int final_stage) {
  __shared__ acc_t colsum[kReduceThreads + 8];
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) { reduce_body(colsum, r, final_stage, item); });
}

__global__ void quantize_kernel(const float* __restrict__ in, uint16_t* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const double d = static_cast<double>(fminf(fmaxf(in[i], 0.0f), 1.0f));
    out[i] = static_cast<uint16_t>(floor(d * 65535.0 + 0.5));
  }
}

}  // namespace

size_t partials_bytes(int H, int W) { return aggregation_entries(H, W) * sizeof(acc_t); }

int group_items_for(int H, int W, int R) {
  const GroupArgs g = make_args(H, W, R);
  return g.nTy * g.nTx;
}

int reduce_items_for(int H, int W) { return reduce_items(H, W); }

template <int K, bool WIDE>
static hipError_t launch_ht_shape(const ImgRec& one, const WorkList* wl, int R, const HtParams& hp, int recompute,
                                  int grid_cap, hipStream_t st) {
  using Cfg = GroupCfg<K, true, false, WIDE>;
  if (!wl) {
    if (recompute)
      hipLaunchKernelGGL((group_ht_kernel<K, false, true, WIDE>), dim3(group_items_for(one.H, one.W, R)),
                         dim3(Cfg::threads), 0, st, one, WorkList{}, R, hp);
    else
      hipLaunchKernelGGL((group_ht_kernel<K, false, false, WIDE>), dim3(group_items_for(one.H, one.W, R)),
                         dim3(Cfg::threads), 0, st, one, WorkList{}, R, hp);
  } else {
    if (recompute) return hipErrorInvalidValue;  // batches read the stack
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((group_ht_kernel<K, true, false, WIDE>), dim3(std::min(wl->total, grid_cap)),
                       dim3(GroupCfg<K, true, true, WIDE>::threads), 0, st, one, *wl, R, hp);
  }
  return hipGetLastError();
}

template <int K>
static hipError_t launch_ht_k(const ImgRec& one, const WorkList* wl, int R, const HtParams& hp, int recompute,
                              int shape, int grid_cap, hipStream_t st) {
  if (K <= 16 && shape == 1) return launch_ht_shape<K, false>(one, wl, R, hp, recompute, grid_cap, st);
  return launch_ht_shape<K, true>(one, wl, R, hp, recompute, grid_cap, st);
}

int group_ht_tiles_per_cu(int K, int shape) { return K <= 16 && shape == 0 ? 2 : 1; }

hipError_t launch_group_ht(const ImgRec& one, const WorkList* wl, int R, int K, float ht_a, float ht_b,
                           int weight_mode, int keep_dc, int recompute, int shape, int grid_cap, hipStream_t st) {
  const HtParams hp{ht_a, ht_b, weight_mode, keep_dc};
  switch (K) {
    case 2: return launch_ht_k<2>(one, wl, R, hp, recompute, shape, grid_cap, st);
    case 4: return launch_ht_k<4>(one, wl, R, hp, recompute, shape, grid_cap, st);
    case 8: return launch_ht_k<8>(one, wl, R, hp, recompute, shape, grid_cap, st);
    case 16: return launch_ht_k<16>(one, wl, R, hp, recompute, shape, grid_cap, st);
    case 32: return launch_ht_k<32>(one, wl, R, hp, recompute, shape, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_clear_weights(const ImgRec& one, hipStream_t st) {
  const size_t n = aggregation_entries(one.H, one.W);
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(clear_weights_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, one.partials, n);
  return hipGetLastError();
}

template <int K>
static hipError_t launch_wiener_k(const ImgRec& one, const WorkList* wl, int R, int grid_cap, hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((group_wiener_kernel<K, false>), dim3(group_items_for(one.H, one.W, R)),
                       dim3(GroupCfg<K, false, false>::threads), 0, st, one, WorkList{}, R);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((group_wiener_kernel<K, true>), dim3(std::min(wl->total, grid_cap)),
                       dim3(GroupCfg<K, false, true>::threads), 0, st, one, *wl, R);
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

hipError_t launch_reduce(const ImgRec& one, const WorkList* wl, int final_stage, int grid_cap,
                         hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((reduce_kernel<false>), dim3(reduce_items(one.H, one.W)), dim3(kReduceThreads), 0, st, one,
                       WorkList{}, final_stage);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((reduce_kernel<true>), dim3(std::min(wl->total, grid_cap)), dim3(kReduceThreads), 0, st,
                       one, *wl, final_stage);
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
