// Global stage 1 (Sec. 3): the hard-threshold estimate computed on one volume.
//
// Reference blocks of side N tile the image; each is matched to its K nearest
// blocks (exact distances, same key and tie rule as the grouped path, the
// reference itself in slot 0).  The k-th match of every reference is stacked
// behind the reference's own tile, giving a volume V[k][y][x] with the noisy
// image as its first slice.  The volume is filtered as a whole: a separable
// periodic 3-D Mallat decomposition (bior1.5 along y and x, orthonormal Haar
// along k, three levels), hard thresholding with tau_l = sigma (a - b l) per
// detail level (the final approximation kept), inverse; averaged over cycle
// spins S_h (a circular shift by h along all three axes).  Every filtered
// block returns to its source position with weight 1/TV of its reference's
// N x N x K block (64-bit fixed point, global integer atomics), and the
// normalised estimate is averaged over translations of the image
// (eq. firstEst).
//
// The transform runs one kernel per level for all cycle spins at once: a
// workgroup loads a window of two k-slices of one spin into LDS and does the
// Haar pair along k and the bior1.5 filters along x and y there, writing the
// eight bands of its coefficient tile (thresholded, but for the
// low-low-low band).  Level 0 gathers the spun volume straight from the
// image, so the unfiltered volume is never stored; the aggregation undoes
// the spins and averages them as it loads each tile's blocks.
#include <cstdint>

#include "common.h"
#include "kernels.h"
#include "topk.h"

namespace gbm3d {

namespace {

constexpr int kGlThreads = 256;
constexpr int kMaxSearch = 39;
constexpr double kKeyInfG = __builtin_huge_val();

// The translations of one call, all filtered in the same launches:
// translation ti moves the image by t[ti] along both axes (S_t); its
// translated image is the noisy one when t[ti] = 0, else slice ti of the
// translated-image buffer.  Per-translation buffers are slices ti of theirs.
struct Shifts {
  int n;
  int t[4];
};

__device__ __forceinline__ const uint16_t* translated(const uint16_t* noisy, const uint16_t* shifted, size_t hw,
                                                      const Shifts& sh, int ti) {
  return sh.t[ti] ? shifted + static_cast<size_t>(ti) * hw : noisy;
}

// ---------------------------------------------------------------------------
// Tile matching: one workgroup per reference tile.
// ---------------------------------------------------------------------------
template <int N>
struct TileSmem {
  static constexpr int kRegion = kMaxSearch + N - 1;
  // row pitch: the region plus the columns the last 8-wide displacement
  // group reads past it, made odd so that lanes on consecutive rows fall on
  // different LDS banks
  static constexpr int kPitch = (kRegion + 2) | 1;
  double reg[kRegion * kPitch];          // search region, pixel values
  double keys[kMaxSearch * kMaxSearch];  // dist * 2048 + rank (+inf for the reference)
  double part[kGlThreads / kWave];       // per-wave partial sums of the reference norm
};

template <int N, int K>
// grid: (tiles, translations)
__global__ __launch_bounds__(kGlThreads) void gl_match_kernel(const uint16_t* __restrict__ noisy,
                                                              const uint16_t* __restrict__ shifted, Shifts sh, int H,
                                                              int W, int S, int16_t* __restrict__ idx) {
  using Sm = TileSmem<N>;
  constexpr int P = Sm::kPitch;
  constexpr int L = K - 1;
  __shared__ Sm sm;
  const int tiles_x = W / N;
  const int g = blockIdx.x;
  const int y0 = (g / tiles_x) * N, x0 = (g % tiles_x) * N;
  const int R = S / 2;
  const int side = S + N - 1;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint16_t* img = translated(noisy, shifted, static_cast<size_t>(H) * W, sh, blockIdx.y);
  idx += static_cast<size_t>(blockIdx.y) * gridDim.x * K;
  {
    // the (S + N - 1)^2 search region (rows and columns wrap at most once:
    // R < H, W), all loads issued before any store
    constexpr int kIters = (Sm::kRegion * P + kGlThreads - 1) / kGlThreads;
    uint16_t v[kIters];
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
      const int i = threadIdx.x + it * kGlThreads;
      const int r = i / P, c = i - r * P;
      v[it] = 0;
      if (i < side * P && c < side) {
        int y = y0 - R + r, x = x0 - R + c;
        y = y < 0 ? y + H : (y >= H ? y - H : y);
        x = x < 0 ? x + W : (x >= W ? x - W : x);
        v[it] = img[static_cast<size_t>(y) * W + x];
      }
    }
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
      const int i = threadIdx.x + it * kGlThreads;
      if (i < side * P) sm.reg[i] = v[it];
    }
  }
  __syncthreads();
  // the reference block's squared norm: one pixel per thread (N * N <= 256)
  {
    double v = 0.0;
    if (threadIdx.x < N * N) {
      v = sm.reg[(R + threadIdx.x / N) * P + R + threadIdx.x % N];
      v *= v;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += shfl_xor_double(v, off);
    if (lane == 0) sm.part[wave] = v;
  }
  __syncthreads();
  double ref_norm = 0.0;
#pragma unroll
  for (int w = 0; w < kGlThreads / kWave; ++w) ref_norm += sm.part[w];
  // exact squared distances as |a|^2 + |b|^2 - 2 <a, b>: every term an
  // integer below 2^41, so float64 holds each step exactly and the keys equal
  // those of summed squared differences.  A work item is one displacement
  // row dy and eight consecutive dx: each reference pixel (one LDS word read
  // by the whole wave) serves all eight; the candidates' norms are column
  // sums of squares over the same rows, then sums of N columns.
  const int S2 = S * S;
  constexpr int kDx = 8;
  constexpr int kSeg = N + kDx - 1;
  const int groups = (S + kDx - 1) / kDx;
  for (int item = threadIdx.x; item < S * groups; item += blockDim.x) {
    // consecutive lanes take consecutive rows dy (an odd pitch apart: no
    // two of 32 lanes on one LDS bank)
    const int gi = item / S, dy = item - gi * S, dx0 = gi * kDx;
    double d[kDx];
#pragma unroll
    for (int c = 0; c < kDx; ++c) d[c] = 0.0;
#pragma unroll 1
    for (int a = 0; a < N; ++a) {
      const double* cr = sm.reg + (dy + a) * P + dx0;
      const double* rr = sm.reg + (R + a) * P + R;
      double seg[kSeg];
#pragma unroll
      for (int b = 0; b < kSeg; ++b) seg[b] = cr[b];
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const double rv = rr[b];
#pragma unroll
        for (int c = 0; c < kDx; ++c) d[c] = fma(rv, seg[b + c], d[c]);
      }
    }
    // the candidates' norms: column sums of squares over the same rows
    double col[kSeg];
#pragma unroll
    for (int b = 0; b < kSeg; ++b) col[b] = 0.0;
#pragma unroll 1
    for (int a = 0; a < N; ++a) {
      const double* cr = sm.reg + (dy + a) * P + dx0;
#pragma unroll
      for (int b = 0; b < kSeg; ++b) col[b] = fma(cr[b], cr[b], col[b]);
    }
    double cn = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) cn += col[b];
#pragma unroll
    for (int c = 0; c < kDx; ++c) {
      const int dx = dx0 + c;
      if (c > 0) cn += col[N - 1 + c] - col[c - 1];
      if (dx < S) {
        const int r = dy * S + dx;
        const double dist = (ref_norm + cn) - 2.0 * d[c];
        sm.keys[r] = r == S2 / 2 ? kKeyInfG : fma(dist, 2048.0, static_cast<double>(r));
      }
    }
  }
  __syncthreads();
  // the K-1 smallest keys (keys are unique): each lane sorts its own keys,
  // the lanes of a wave merge their lists pairwise along a butterfly (every
  // lane ends with the wave's K-1 smallest), and wave 0 merges the four
  // waves' lists the same way
  constexpr int kPer = (kMaxSearch * kMaxSearch + kGlThreads - 1) / kGlThreads;
  constexpr int kSort = pow2_ceil(kPer);
  double list[L];
  {
    double mine[kSort];
#pragma unroll
    for (int m = 0; m < kSort; ++m) {
      const int r = threadIdx.x + m * kGlThreads;
      mine[m] = (m < kPer && r < S2) ? sm.keys[r] : kKeyInfG;
    }
    bitonic_sort<kSort>(mine);
#pragma unroll
    for (int i = 0; i < L; ++i) list[i] = i < kSort ? mine[i] : kKeyInfG;
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) merge_sorted<L>(list, [&](int j) { return shfl_xor_double(list[j], off); });
  __syncthreads();  // every key has been read; the key array is reused below
  double* wl = sm.keys;  // [4][L]
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < L; ++i) wl[wave * L + i] = list[i];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int i = 0; i < L; ++i) list[i] = lane < kGlThreads / kWave ? wl[lane * L + i] : kKeyInfG;
#pragma unroll
    for (int off = 1; off < kGlThreads / kWave; off <<= 1)
      merge_sorted<L>(list, [&](int j) { return shfl_xor_double(list[j], off); });
    if (lane == 0) {
      int16_t* out = idx + static_cast<size_t>(g) * K;
      out[0] = static_cast<int16_t>(S2 / 2);
#pragma unroll
      for (int i = 0; i < L; ++i) out[i + 1] = key_rank(list[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// The volume V[k][y][x] and its periodic 3-D Mallat levels.
// ---------------------------------------------------------------------------

// index j (possibly a few periods out of range) folded into [0, L)
__device__ __forceinline__ int wrap(int j, int L) {
  while (j < 0) j += L;
  while (j >= L) j -= L;
  return j;
}

// dst [Hp][Wp]: img extended past its bottom and right edges with mirrored
// values, the edge pixel repeated first (row / column L + i reads L - 1 - i;
// Hp - H <= H and Wp - W <= W)
__global__ void gl_mirror_pad_kernel(const uint16_t* __restrict__ img, int H, int W, uint16_t* __restrict__ dst,
                                     int Hp, int Wp) {
  const size_t n = static_cast<size_t>(Hp) * Wp;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(i / Wp), x = static_cast<int>(i - static_cast<size_t>(y) * Wp);
    const int ys = y < H ? y : 2 * H - 1 - y, xs = x < W ? x : 2 * W - 1 - x;
    dst[i] = img[static_cast<size_t>(ys) * W + xs];
  }
}

// slice ti of shifted: S_t of the image, img[(y - t) mod H][(x - t) mod W],
// for every translation t = sh.t[ti] other than 0; grid (g, translations)
__global__ void gl_roll_kernel(const uint16_t* __restrict__ img, int H, int W, Shifts sh,
                               uint16_t* __restrict__ shifted) {
  const int t = sh.t[blockIdx.y];
  if (t == 0) return;
  const size_t n = static_cast<size_t>(H) * W;
  uint16_t* out = shifted + blockIdx.y * n;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(i / W), x = static_cast<int>(i - static_cast<size_t>(y) * W);
    out[i] = img[static_cast<size_t>(pmod(y - t, H)) * W + pmod(x - t, W)];
  }
}

// bior1.5 analysis low-pass: a[n] = sum_i h_i x[2n + i - 4]; the analysis
// high-pass is the Haar difference d[n] = (x[2n+1] - x[2n]) / sqrt2
__device__ __forceinline__ float bior_lo_tap(int i) {
  constexpr float s = 1.41421356237309505f / 256.0f;
  constexpr float t[10] = {3 * s, -3 * s, -22 * s, 22 * s, 128 * s, 128 * s, 22 * s, -22 * s, -3 * s, 3 * s};
  return t[i];
}
// synthesis: x[n] = a[n >> 1] / sqrt2 + sum_m g_m d[(n - m) / 2] over
// m = -4 .. 5 with n - m even; syn_even(i) = g_{4 - 2i} multiplies
// d[n/2 - 2 + i] for even n, syn_odd(i) = g_{5 - 2i} multiplies
// d[(n-1)/2 - 2 + i] for odd n (i = 0 .. 4)
__device__ __forceinline__ float bior_syn_even(int i) {
  constexpr float s = 1.41421356237309505f / 256.0f;
  constexpr float t[5] = {3 * s, -22 * s, -128 * s, 22 * s, -3 * s};
  return t[i];
}
__device__ __forceinline__ float bior_syn_odd(int i) {
  constexpr float s = 1.41421356237309505f / 256.0f;
  constexpr float t[5] = {3 * s, -22 * s, 128 * s, 22 * s, -3 * s};
  return t[i];
}

__device__ __forceinline__ float hard_threshold(float v, float tau) { return fabsf(v) >= tau ? v : 0.0f; }

// j folded into [0, L) when it lies within one period of it
__device__ __forceinline__ int wrap1(int j, int L) { return j < 0 ? j + L : (j >= L ? j - L : j); }

// Coefficient tiles of a workgroup: TY x TX per band of y and x, one pair of
// slices along k.  The finest level takes 16 x 32; the coarser levels, whose
// regions are 8 and 64 times smaller, take 8 x 16 to keep enough workgroups.
template <int TY, int TX>
struct LevelTile {
  static constexpr int kFwdRows = 2 * TY + 8, kFwdCols = 2 * TX + 8;  // forward input window
  static constexpr int kInvRows = 2 * TY + 4, kInvCols = 2 * TX + 4;  // inverse input window
  static constexpr int kFwdIters = (kFwdRows * kFwdCols + kGlThreads - 1) / kGlThreads;
  static constexpr int kInvIters = (kInvRows * kInvCols + kGlThreads - 1) / kGlThreads;
};

// One forward level over the region [0, Lk) x [0, Ly) x [0, Lx) of a
// K x H x W volume, all three axes in one pass: Haar along k (sums and
// differences over sqrt2), then bior1.5 along x and along y, all periodic
// within the region.  Output bands go to their Mallat positions (low half /
// high half of each axis) in dst; every band but low-low-low is hard
// thresholded with tau.  With GATHER the input is the spun volume V_h,
// gathered from the translated image through its matches, instead of src.
// Every (translation ti, cycle spin h) has its own pair of volumes, volume
// v = ti spins + h at v K H W elements into src and dst.
// grid: (ceil(Lx / 2 / TX), ceil(Ly / 2 / TY), Lk / 2 * volumes), z = v Lk / 2 + kp
template <int N, int K, bool GATHER, int TY, int TX>
__global__ __launch_bounds__(kGlThreads) void gl_forward_kernel(const float* __restrict__ src,
                                                                 const uint16_t* __restrict__ noisy,
                                                                 const uint16_t* __restrict__ shifted, Shifts sh,
                                                                 int spins, const int16_t* __restrict__ idx, int S,
                                                                 float* __restrict__ dst, int H, int W, int Lk, int Ly,
                                                                 int Lx, float tau) {
  using T = LevelTile<TY, TX>;
  // input window: rows 2 cy0 - 4 .. 2 cy0 + 2 TY + 3, the same for columns;
  // columns stored split by parity so the strided filter taps read
  // consecutive LDS words
  constexpr int kRows = T::kFwdRows, kCols = T::kFwdCols, kHalfCols = kCols / 2;
  __shared__ float in_s[2][kRows][2][kHalfCols];
  __shared__ float xs[2][kRows][2 * TX];
  // per window row / column: the volume coordinate (with GATHER: of the
  // unspun volume V, and which of the window's tile rows / columns holds it)
  constexpr int kTileRows = (kRows + 2 * N - 2) / N, kTileCols = (kCols + 2 * N - 2) / N;
  static_assert(kRows + kCols + 2 * kTileRows * kTileCols <= kGlThreads, "one table entry per thread");
  __shared__ int row_at[kRows], col_at[kCols], row_lt[GATHER ? kRows : 1], col_lt[GATHER ? kCols : 1];
  // with GATHER: the match displacement (dy, dx) of slices 2 kp + j of every
  // tile the window touches
  __shared__ int disp_y[GATHER ? 2 : 1][kTileRows][kTileCols], disp_x[GATHER ? 2 : 1][kTileRows][kTileCols];
  const int hy = Ly >> 1, hx = Lx >> 1, hk = Lk >> 1;
  const int v = blockIdx.z / hk, kp = blockIdx.z - v * hk;
  const int ti = v / spins, h = v - ti * spins;
  const int cx0 = blockIdx.x * TX, cy0 = blockIdx.y * TY;
  const size_t hw = static_cast<size_t>(H) * W;
  if constexpr (!GATHER) src += static_cast<size_t>(v) * K * hw;
  dst += static_cast<size_t>(v) * K * hw;
  const uint16_t* img = nullptr;
  if constexpr (GATHER) {
    img = translated(noisy, shifted, hw, sh, ti);
    idx += static_cast<size_t>(ti) * (H / N) * (W / N) * K;
  }
  const float c = 0.70710678118654752f;
  const int tid = threadIdx.x;
  if constexpr (GATHER) {
    // V_h[k][y][x] = V[(k - h) mod K][(y - h) mod H][(x - h) mod W]: the
    // window's rows (columns) are consecutive mod H (W) from ys0 (xs0)
    const int ys0 = wrap1(wrap(2 * cy0 - 4, Ly) - h, H), xs0 = wrap1(wrap(2 * cx0 - 4, Lx) - h, W);
    if (tid < kRows) {
      row_at[tid] = wrap(ys0 + tid, H);
      row_lt[tid] = (ys0 % N + tid) / N;
    } else if (tid < kRows + kCols) {
      const int i = tid - kRows;
      col_at[i] = wrap(xs0 + i, W);
      col_lt[i] = (xs0 % N + i) / N;
    } else if (tid < kRows + kCols + 2 * kTileRows * kTileCols) {
      const int t = tid - kRows - kCols;
      const int j = t / (kTileRows * kTileCols), lr = (t / kTileCols) % kTileRows, lc = t % kTileCols;
      const int TH = H / N, TW = W / N;
      const int trow = (ys0 / N + lr) % TH, tcol = (xs0 / N + lc) % TW;
      const int rank = idx[(static_cast<size_t>(trow) * TW + tcol) * K + wrap1(2 * kp + j - h, K)];
      const int q = rank / S;
      disp_y[j][lr][lc] = q - S / 2;
      disp_x[j][lr][lc] = rank - q * S - S / 2;
    }
  } else {
    if (tid < kRows) {
      row_at[tid] = wrap(2 * cy0 - 4 + tid, Ly);
    } else if (tid < kRows + kCols) {
      col_at[tid - kRows] = wrap(2 * cx0 - 4 + tid - kRows, Lx);
    }
  }
  __syncthreads();
  float v0[T::kFwdIters], v1[T::kFwdIters];
  if constexpr (GATHER) {
    // V[k'][ys][xs] = z at (ys, xs) + the k'-th match displacement of its tile
#pragma unroll
    for (int it = 0; it < T::kFwdIters; ++it) {
      const int e = tid + it * kGlThreads;
      if (e < kRows * kCols) {
        const int r = e / kCols, col = e - r * kCols;
        const int ys = row_at[r], xs = col_at[col], lr = row_lt[r], lc = col_lt[col];
        const size_t o0 = static_cast<size_t>(wrap1(ys + disp_y[0][lr][lc], H)) * W + wrap1(xs + disp_x[0][lr][lc], W);
        const size_t o1 = static_cast<size_t>(wrap1(ys + disp_y[1][lr][lc], H)) * W + wrap1(xs + disp_x[1][lr][lc], W);
        v0[it] = static_cast<float>(img[o0]) * (1.0f / 65535.0f);
        v1[it] = static_cast<float>(img[o1]) * (1.0f / 65535.0f);
      }
    }
  } else {
    const float* s0 = src + static_cast<size_t>(2 * kp) * hw;
    const float* s1 = s0 + hw;
#pragma unroll
    for (int it = 0; it < T::kFwdIters; ++it) {
      const int e = tid + it * kGlThreads;
      if (e < kRows * kCols) {
        const int r = e / kCols, col = e - r * kCols;
        const size_t o = static_cast<size_t>(row_at[r]) * W + col_at[col];
        v0[it] = s0[o];
        v1[it] = s1[o];
      }
    }
  }
#pragma unroll
  for (int it = 0; it < T::kFwdIters; ++it) {
    const int e = tid + it * kGlThreads;
    if (e < kRows * kCols) {
      const int r = e / kCols, col = e - r * kCols;
      in_s[0][r][col & 1][col >> 1] = (v0[it] + v1[it]) * c;
      in_s[1][r][col & 1][col >> 1] = (v0[it] - v1[it]) * c;
    }
  }
  __syncthreads();
  // along x: window column 2 j + i is even[j + i/2] or odd[j + (i-1)/2]
  for (int e = tid; e < 2 * kRows * TX; e += kGlThreads) {
    const int j = e % TX, r = (e / TX) % kRows, kb = e / (TX * kRows);
    const float* ev = in_s[kb][r][0];
    const float* od = in_s[kb][r][1];
    float lo = 0.0f;
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      lo = fmaf(bior_lo_tap(2 * u), ev[j + u], lo);
      lo = fmaf(bior_lo_tap(2 * u + 1), od[j + u], lo);
    }
    xs[kb][r][j] = lo;
    xs[kb][r][TX + j] = (od[j + 2] - ev[j + 2]) * c;
  }
  __syncthreads();
  // along y, then out to the bands
  for (int e = tid; e < 2 * TY * 2 * TX; e += kGlThreads) {
    const int cc = e % (2 * TX), i = (e / (2 * TX)) % TY, kb = e / (2 * TX * TY);
    const int xb = cc >= TX ? 1 : 0;
    const int cy = cy0 + i, cx = cx0 + cc - xb * TX;
    if (cy >= hy || cx >= hx) continue;
    float lo = 0.0f;
#pragma unroll
    for (int t = 0; t < 10; ++t) lo = fmaf(bior_lo_tap(t), xs[kb][2 * i + t][cc], lo);
    const float hi = hard_threshold((xs[kb][2 * i + 5][cc] - xs[kb][2 * i + 4][cc]) * c, tau);
    if (kb | xb) lo = hard_threshold(lo, tau);
    float* o = dst + static_cast<size_t>(kb ? hk + kp : kp) * hw + (xb ? hx + cx : cx);
    o[static_cast<size_t>(cy) * W] = lo;
    o[static_cast<size_t>(hy + cy) * W] = hi;
  }
}

// The inverse of one level: src holds the level's eight bands at their
// Mallat positions in the region; the workgroup rebuilds slices 2 kp, 2 kp + 1,
// rows 2 cy0 .. 2 cy0 + 2 TY - 1 and columns 2 cx0 .. 2 cx0 + 2 TX - 1
// (synthesis along x, then y, then the Haar pair along k) at the same
// positions of dst.  Volumes and grid as in the forward kernel (z = v Lk / 2
// + kp over every volume v).
template <int K, int TY, int TX>
__global__ __launch_bounds__(kGlThreads) void gl_inverse_kernel(const float* __restrict__ src,
                                                                 float* __restrict__ dst, int H, int W, int Lk, int Ly,
                                                                 int Lx) {
  using T = LevelTile<TY, TX>;
  // window rows: low band cy0 .. cy0 + TY - 1, then high band cy0 - 2 ..
  // cy0 + TY + 1 (the synthesis taps reach two coefficients either side);
  // the same for columns
  constexpr int kRows = T::kInvRows, kCols = T::kInvCols;
  __shared__ float in_s[2][kRows][kCols];
  __shared__ float xs[2][kRows][2 * TX];
  __shared__ int row_at[kRows], col_at[kCols];
  const int hy = Ly >> 1, hx = Lx >> 1, hk = Lk >> 1;
  const int h = blockIdx.z / hk, kp = blockIdx.z - h * hk;
  const int cx0 = blockIdx.x * TX, cy0 = blockIdx.y * TY;
  const size_t hw = static_cast<size_t>(H) * W;
  src += static_cast<size_t>(h) * K * hw;
  dst += static_cast<size_t>(h) * K * hw;
  const float c = 0.70710678118654752f;
  const int tid = threadIdx.x;
  if (tid < kRows) {
    row_at[tid] = tid < TY ? wrap(cy0 + tid, hy) : hy + wrap(cy0 - 2 + tid - TY, hy);
  } else if (tid < kRows + kCols) {
    const int col = tid - kRows;
    col_at[col] = col < TX ? wrap(cx0 + col, hx) : hx + wrap(cx0 - 2 + col - TX, hx);
  }
  __syncthreads();
  {
    const float* s0 = src + static_cast<size_t>(kp) * hw;
    const float* s1 = src + static_cast<size_t>(hk + kp) * hw;
    float v0[T::kInvIters], v1[T::kInvIters];
#pragma unroll
    for (int it = 0; it < T::kInvIters; ++it) {
      const int e = tid + it * kGlThreads;
      if (e < kRows * kCols) {
        const int r = e / kCols, col = e - r * kCols;
        const size_t o = static_cast<size_t>(row_at[r]) * W + col_at[col];
        v0[it] = s0[o];
        v1[it] = s1[o];
      }
    }
#pragma unroll
    for (int it = 0; it < T::kInvIters; ++it) {
      const int e = tid + it * kGlThreads;
      if (e < kRows * kCols) {
        const int r = e / kCols, col = e - r * kCols;
        in_s[0][r][col] = v0[it];
        in_s[1][r][col] = v1[it];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < 2 * kRows * TX; e += kGlThreads) {
    const int j = e % TX, r = (e / TX) % kRows, kb = e / (TX * kRows);
    const float* row = in_s[kb][r];
    const float a = c * row[j];
    float ev = a, od = a;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const float d = row[TX + j + i];
      ev = fmaf(bior_syn_even(i), d, ev);
      od = fmaf(bior_syn_odd(i), d, od);
    }
    xs[kb][r][2 * j] = ev;
    xs[kb][r][2 * j + 1] = od;
  }
  __syncthreads();
  for (int e = tid; e < TY * 2 * TX; e += kGlThreads) {
    const int cc = e % (2 * TX), i = e / (2 * TX);
    const int y = 2 * (cy0 + i), x = 2 * cx0 + cc;
    if (y >= Ly || x >= Lx) continue;
    float ev[2], od[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const float a = c * xs[kb][i][cc];
      ev[kb] = a;
      od[kb] = a;
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        const float d = xs[kb][TY + i + u][cc];
        ev[kb] = fmaf(bior_syn_even(u), d, ev[kb]);
        od[kb] = fmaf(bior_syn_odd(u), d, od[kb]);
      }
    }
    const float v[2][2] = {{(ev[0] + ev[1]) * c, (od[0] + od[1]) * c}, {(ev[0] - ev[1]) * c, (od[0] - od[1]) * c}};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int p = 0; p < 2; ++p) dst[static_cast<size_t>(2 * kp + s) * hw + static_cast<size_t>(y + p) * W + x] = v[s][p];
    }
  }
}

__global__ void gl_zero_kernel(unsigned long long* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// One workgroup per tile.  u is the average over the cycle spins h of the
// filtered spun volumes (spin h at vol + h K H W) with each spin undone:
// u[k][y][x] = (1 / spins) sum_h vol_h[(k + h) mod K][(y + h) mod H][(x + h) mod W].
// w = eps / (TV(u) + eps) (the 1 / (TV + eps) weight scaled by eps, which
// cancels in the average), then every filtered block is added at its source
// position: num += w u, den += w (64-bit fixed point).
// The K blocks all lie in the tile's (S + N - 1)^2 search footprint, which
// is summed in LDS first; only its covered cells go to the image with global
// integer atomics.
template <int N, int K>
// grid: (tiles, translations); translation ti reads volumes ti spins ..
// ti spins + spins - 1, its matches and its sums (numerators then
// denominators, 2 H W words per translation).
__global__ __launch_bounds__(kGlThreads) void gl_aggregate_kernel(const float* __restrict__ vol, int spins,
                                                                   const int16_t* __restrict__ idx, int H, int W,
                                                                   int S, float eps,
                                                                   unsigned long long* __restrict__ sums) {
  constexpr int kVals = N * N * K;
  constexpr int kFoot = (kMaxSearch + N - 1) * (kMaxSearch + N - 1);
  __shared__ float blk[kVals];
  __shared__ double part[kGlThreads];
  __shared__ unsigned long long fnum[kFoot], fden[kFoot];
  const size_t hw = static_cast<size_t>(H) * W;
  const int tiles_x = W / N;
  const int g = blockIdx.x;
  const int y0 = (g / tiles_x) * N, x0 = (g % tiles_x) * N;
  const int side = S + N - 1;
  const int ti = blockIdx.y;
  vol += static_cast<size_t>(ti) * spins * K * hw;
  idx += static_cast<size_t>(ti) * gridDim.x * K;
  unsigned long long* num = sums + static_cast<size_t>(ti) * 2 * hw;
  unsigned long long* den = num + hw;
  for (int i = threadIdx.x; i < side * side; i += blockDim.x) {
    fnum[i] = 0;
    fden[i] = 0;
  }
  {
    // all of a spin's loads in flight at once (kVals is a multiple of the
    // block size)
    static_assert(kVals % kGlThreads == 0, "whole rounds of the block");
    constexpr int kIt = kVals / kGlThreads;
    const float scale = 1.0f / static_cast<float>(spins);
    float acc[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) acc[it] = 0.0f;
    for (int h = 0; h < spins; ++h) {
      const float* vh = vol + static_cast<size_t>(h) * K * hw;
      float v[kIt];
#pragma unroll
      for (int it = 0; it < kIt; ++it) {
        const int i = threadIdx.x + it * kGlThreads;
        const int k = i / (N * N), a = (i / N) % N, b = i % N;
        v[it] = vh[static_cast<size_t>(wrap1(k + h, K)) * hw + static_cast<size_t>(wrap1(y0 + a + h, H)) * W +
                   wrap1(x0 + b + h, W)];
      }
#pragma unroll
      for (int it = 0; it < kIt; ++it) acc[it] += scale * v[it];
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) blk[threadIdx.x + it * kGlThreads] = acc[it];
  }
  __syncthreads();
  double tv = 0.0;
  for (int i = threadIdx.x; i < kVals; i += blockDim.x) {
    const int k = i / (N * N), a = (i / N) % N, b = i % N;
    const float v = blk[i];
    float s = 0.0f;
    if (k + 1 < K) s += fabsf(blk[i + N * N] - v);
    if (a + 1 < N) s += fabsf(blk[i + N] - v);
    if (b + 1 < N) s += fabsf(blk[i + 1] - v);
    tv += s;
  }
  part[threadIdx.x] = tv;
  __syncthreads();
  for (int s = kGlThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  const float w = eps / (static_cast<float>(part[0]) + eps);
  const unsigned long long wf = static_cast<unsigned long long>(to_fixed(w));
  for (int i = threadIdx.x; i < kVals; i += blockDim.x) {
    const int k = i / (N * N), a = (i / N) % N, b = i % N;
    const int r = idx[static_cast<size_t>(g) * K + k];
    const int f = (r / S + a) * side + r % S + b;  // footprint cell of (dy + R + a, dx + R + b)
    atomicAdd(fnum + f, static_cast<unsigned long long>(to_fixed(w * blk[i])));
    atomicAdd(fden + f, wf);
  }
  __syncthreads();
  const int R = S / 2;
  for (int i = threadIdx.x; i < side * side; i += blockDim.x) {
    if (fden[i] == 0) continue;
    const int fy = i / side, fx = i - fy * side;
    const size_t o = static_cast<size_t>(wrap(y0 - R + fy, H)) * W + wrap(x0 - R + fx, W);
    __hip_atomic_fetch_add(num + o, fnum[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(den + o, fden[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// out[y][x] = (1 / translations) sum_ti num_ti / den_ti at ((y + t) mod H,
// (x + t) mod W), t = sh.t[ti] (S_{-t} of each translation's estimate),
// summed in translation order
__global__ void gl_normalize_kernel(const unsigned long long* __restrict__ sums, int H, int W, Shifts sh,
                                    float* __restrict__ out) {
  const size_t n = static_cast<size_t>(H) * W;
  const float scale = 1.0f / static_cast<float>(sh.n);
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(i / W), x = static_cast<int>(i - static_cast<size_t>(y) * W);
    float acc = 0.0f;
    for (int ti = 0; ti < sh.n; ++ti) {
      const int t = sh.t[ti];
      const size_t o = static_cast<size_t>(pmod(y + t, H)) * W + pmod(x + t, W);
      const unsigned long long* num = sums + static_cast<size_t>(ti) * 2 * n;
      const float v = scale * static_cast<float>(static_cast<double>(static_cast<long long>(num[o])) /
                                                 static_cast<double>(static_cast<long long>(num[n + o])));
      acc = ti == 0 ? v : acc + v;
    }
    out[i] = acc;
  }
}

dim3 level_grid(int Lk, int Ly, int Lx, int ty, int tx, int volumes) {
  return dim3((Lx / 2 + tx - 1) / tx, (Ly / 2 + ty - 1) / ty, Lk / 2 * volumes);
}

unsigned grid_for(size_t n) {
  const size_t b = (n + kGlThreads - 1) / kGlThreads;
  return static_cast<unsigned>(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

template <int N, int K>
hipError_t global_nk(const GlobalJob& j, hipStream_t st) {
  const int H = j.H, W = j.W;
  const size_t hw = static_cast<size_t>(H) * W;
  const int tiles = (H / N) * (W / N);
  const float eps = j.tv_eps_rel * j.sigma * static_cast<float>(N * N * K);
  Shifts sh{};
  sh.n = j.n_shifts;
  for (int i = 0; i < 4; ++i) sh.t[i] = i < j.n_shifts ? j.shifts[i] : 0;
  const int T = j.n_shifts, C = j.cycles, V = T * C;
  // every translation and cycle spin in the same launches
  hipLaunchKernelGGL(gl_roll_kernel, dim3(grid_for(hw), T), dim3(kGlThreads), 0, st, j.noisy, H, W, sh, j.shifted);
  hipLaunchKernelGGL((gl_match_kernel<N, K>), dim3(tiles, T), dim3(kGlThreads), 0, st, j.noisy, j.shifted, sh, H, W,
                     j.search, j.idx);
  // forward level l writes buf[l & 1]; the next level reads only the
  // low-low-low region of it, so every level's detail bands stay where they
  // were written.  The inverse retraces the same buffers and the finest level
  // leaves the filtered spun volumes in vol_a.
  float* buf[2] = {j.vol_b, j.vol_a};
  for (int l = 0; l < j.levels; ++l) {
    const int Lk = K >> l, Ly = H >> l, Lx = W >> l;
    const float tau = j.sigma * (j.ht_a - j.ht_b * static_cast<float>(l + 1));
    if (l == 0)
      hipLaunchKernelGGL((gl_forward_kernel<N, K, true, 16, 32>), level_grid(Lk, Ly, Lx, 16, 32, V), dim3(kGlThreads),
                         0, st, nullptr, j.noisy, j.shifted, sh, C, j.idx, j.search, buf[0], H, W, Lk, Ly, Lx, tau);
    else
      hipLaunchKernelGGL((gl_forward_kernel<N, K, false, 8, 16>), level_grid(Lk, Ly, Lx, 8, 16, V), dim3(kGlThreads),
                         0, st, buf[(l - 1) & 1], nullptr, nullptr, sh, C, nullptr, j.search, buf[l & 1], H, W, Lk, Ly,
                         Lx, tau);
  }
  for (int l = j.levels - 1; l >= 0; --l) {
    const int Lk = K >> l, Ly = H >> l, Lx = W >> l;
    if (l == 0)
      hipLaunchKernelGGL((gl_inverse_kernel<K, 16, 32>), level_grid(Lk, Ly, Lx, 16, 32, V), dim3(kGlThreads), 0, st,
                         buf[0], j.vol_a, H, W, Lk, Ly, Lx);
    else
      hipLaunchKernelGGL((gl_inverse_kernel<K, 8, 16>), level_grid(Lk, Ly, Lx, 8, 16, V), dim3(kGlThreads), 0, st,
                         buf[l & 1], buf[(l - 1) & 1], H, W, Lk, Ly, Lx);
  }
  hipLaunchKernelGGL(gl_zero_kernel, dim3(grid_for(2 * hw * T)), dim3(kGlThreads), 0, st, j.num, 2 * hw * T);
  hipLaunchKernelGGL((gl_aggregate_kernel<N, K>), dim3(tiles, T), dim3(kGlThreads), 0, st, j.vol_a, C, j.idx, H, W,
                     j.search, eps, j.num);
  hipLaunchKernelGGL(gl_normalize_kernel, dim3(grid_for(hw)), dim3(kGlThreads), 0, st, j.num, H, W, sh, j.out);
  return hipGetLastError();
}

}  // namespace

size_t global_volume_bytes(int H, int W, int K) { return static_cast<size_t>(K) * H * W * sizeof(float); }

template <int N, int K>
static hipError_t match_nk(const uint16_t* img, int H, int W, int search, int16_t* idx, hipStream_t st) {
  const Shifts none{1, {0, 0, 0, 0}};
  hipLaunchKernelGGL((gl_match_kernel<N, K>), dim3((H / N) * (W / N), 1), dim3(kGlThreads), 0, st, img, nullptr, none, H,
                     W, search, idx);
  return hipGetLastError();
}

hipError_t launch_global_match(const uint16_t* img, int H, int W, int patch, int search, int k, int16_t* idx,
                               hipStream_t st) {
  if (patch == 16 && k == 16) return match_nk<16, 16>(img, H, W, search, idx, st);
  if (patch == 16 && k == 8) return match_nk<16, 8>(img, H, W, search, idx, st);
  if (patch == 16 && k == 32) return match_nk<16, 32>(img, H, W, search, idx, st);
  if (patch == 8 && k == 16) return match_nk<8, 16>(img, H, W, search, idx, st);
  if (patch == 8 && k == 8) return match_nk<8, 8>(img, H, W, search, idx, st);
  if (patch == 8 && k == 32) return match_nk<8, 32>(img, H, W, search, idx, st);
  return hipErrorInvalidValue;
}

hipError_t launch_global_pad(const uint16_t* img, int H, int W, uint16_t* dst, int Hp, int Wp, hipStream_t st) {
  hipLaunchKernelGGL(gl_mirror_pad_kernel, dim3(grid_for(static_cast<size_t>(Hp) * Wp)), dim3(kGlThreads), 0, st, img,
                     H, W, dst, Hp, Wp);
  return hipGetLastError();
}

hipError_t launch_global_basic(const GlobalJob& j, hipStream_t st) {
  if (j.patch == 16 && j.k == 16) return global_nk<16, 16>(j, st);
  if (j.patch == 16 && j.k == 8) return global_nk<16, 8>(j, st);
  if (j.patch == 16 && j.k == 32) return global_nk<16, 32>(j, st);
  if (j.patch == 8 && j.k == 16) return global_nk<8, 16>(j, st);
  if (j.patch == 8 && j.k == 8) return global_nk<8, 8>(j, st);
  if (j.patch == 8 && j.k == 32) return global_nk<8, 32>(j, st);
  return hipErrorInvalidValue;
}

}  // namespace gbm3d
