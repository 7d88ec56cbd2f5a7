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
// The transform runs as one kernel per axis and level over the active
// sub-volume, out of place between two volume buffers (each output element
// reads its <= 10 periodic inputs along the axis; consecutive threads take
// consecutive x, so every axis is read and written coalesced).  Three passes
// per level change buffers, so after each coarser level the level's region is
// copied back next to the finer bands.
#include <cstdint>

#include "common.h"
#include "kernels.h"

namespace gbm3d {

namespace {

constexpr int kGlThreads = 256;
constexpr int kMaxSearch = 39;
constexpr double kKeyInfG = __builtin_huge_val();

// ---------------------------------------------------------------------------
// Tile matching: one workgroup per reference tile.
// ---------------------------------------------------------------------------
template <int N>
struct TileSmem {
  static constexpr int kRegion = kMaxSearch + N - 1;
  int reg[kRegion * kRegion];  // search region, pixel values
  double keys[kMaxSearch * kMaxSearch];  // dist * 2048 + rank (+inf for the reference)
};

template <int N, int K>
__global__ __launch_bounds__(kGlThreads) void gl_match_kernel(const uint16_t* __restrict__ img, int H, int W, int S,
                                                              int16_t* __restrict__ idx) {
  __shared__ TileSmem<N> sm;
  const int tiles_x = W / N;
  const int g = blockIdx.x;
  const int y0 = (g / tiles_x) * N, x0 = (g % tiles_x) * N;
  const int R = S / 2;
  const int side = S + N - 1;
  for (int i = threadIdx.x; i < side * side; i += blockDim.x) {
    const int r = i / side, c = i - r * side;
    const int y = pmod(y0 - R + r, H), x = pmod(x0 - R + c, W);
    sm.reg[i] = img[static_cast<size_t>(y) * W + x];
  }
  __syncthreads();
  const int S2 = S * S;
  // exact squared distances, every difference squared and summed in float64
  // (each term < 2^32, the sum < 2^42); a work item is one displacement row
  // dy and four consecutive dx, so each reference pixel read from LDS serves
  // four candidates
  constexpr int kDx = 4;
  const int groups = (S + kDx - 1) / kDx;
  for (int item = threadIdx.x; item < S * groups; item += blockDim.x) {
    const int dy = item / groups, dx0 = (item - dy * groups) * kDx;
    double d[kDx] = {0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < N; ++a) {
      const int* rr = sm.reg + (R + a) * side + R;
      const int* cr = sm.reg + (dy + a) * side + dx0;
      int seg[N + kDx - 1];
#pragma unroll
      for (int b = 0; b < N + kDx - 1; ++b) seg[b] = dx0 + b < side ? cr[b] : 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const int ref = rr[b];
#pragma unroll
        for (int c = 0; c < kDx; ++c) {
          const double t = static_cast<double>(ref - seg[b + c]);
          d[c] = fma(t, t, d[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kDx; ++c) {
      const int dx = dx0 + c;
      if (dx < S) {
        const int r = dy * S + dx;
        sm.keys[r] = r == S2 / 2 ? kKeyInfG : fma(d[c], 2048.0, static_cast<double>(r));
      }
    }
  }
  __syncthreads();
  // the K-1 smallest keys (keys are unique): every wave takes its K-1
  // smallest by repeated wave minima over its lanes' keys, then wave 0 does
  // the same over the four waves' lists
  constexpr int kPer = (kMaxSearch * kMaxSearch + kGlThreads - 1) / kGlThreads;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  double mine[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int r = threadIdx.x + m * kGlThreads;
    mine[m] = r < S2 ? sm.keys[r] : kKeyInfG;
  }
  auto wave_min = [](double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int lo = __shfl_xor(__double2loint(v), off, kWave), hi = __shfl_xor(__double2hiint(v), off, kWave);
      v = fmin(v, __hiloint2double(hi, lo));
    }
    return v;
  };
  auto take_smallest = [&](double (&vals)[kPer], int count, double* dst) {
    for (int s = 0; s < count; ++s) {
      double cur = vals[0];
#pragma unroll
      for (int m = 1; m < kPer; ++m) cur = fmin(cur, vals[m]);
      const double best = wave_min(cur);
      if (lane == 0) dst[s] = best;
#pragma unroll
      for (int m = 0; m < kPer; ++m)
        if (vals[m] == best) vals[m] = kKeyInfG;
    }
  };
  __syncthreads();  // every key has been read; the key array is reused below
  double* wtop = sm.keys;                  // [4][K - 1]
  take_smallest(mine, K - 1, wtop + wave * (K - 1));
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int c = lane + m * kWave;
      mine[m] = c < 4 * (K - 1) ? wtop[c] : kKeyInfG;
    }
    double* top = sm.keys + 4 * (K - 1);   // [K - 1], ascending
    take_smallest(mine, K - 1, top);
    wave_lds_sync();  // lane 0's writes of `top` are visible to the wave
    if (lane < K) {
      int16_t rank;
      if (lane == 0) {
        rank = static_cast<int16_t>(S2 / 2);
      } else {
        const double key = top[lane - 1];
        rank = static_cast<int16_t>(key - 2048.0 * floor(key * (1.0 / 2048.0)));
      }
      idx[static_cast<size_t>(g) * K + lane] = rank;
    }
  }
}

// ---------------------------------------------------------------------------
// Elementwise kernels over the image and the volume V[k][y][x].
// ---------------------------------------------------------------------------

// index j (possibly a few periods out of range) folded into [0, L)
__device__ __forceinline__ int wrap(int j, int L) {
  while (j < 0) j += L;
  while (j >= L) j -= L;
  return j;
}

// out[y][x] = img[(y - t) mod H][(x - t) mod W]  (S_t of the image)
__global__ void gl_roll_kernel(const uint16_t* __restrict__ img, int H, int W, int t, uint16_t* __restrict__ out) {
  const size_t n = static_cast<size_t>(H) * W;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(i / W), x = static_cast<int>(i - static_cast<size_t>(y) * W);
    out[i] = img[static_cast<size_t>(pmod(y - t, H)) * W + pmod(x - t, W)];
  }
}

// V_h[k][y][x] = V[(k - h) mod K][(y - h) mod H][(x - h) mod W] with
// V[k'][y'][x'] = z at the k'-th match of the tile holding (y', x'), offset
// by (y', x') inside the tile.
// grid of the volume kernels: (ceil(W / 256), H, K), thread = element (k, y, x)
template <int N, int K>
__global__ __launch_bounds__(kGlThreads) void gl_volume_kernel(const uint16_t* __restrict__ img,
                                                               const int16_t* __restrict__ idx, int H, int W, int S,
                                                               int h, float* __restrict__ vol) {
  const int x = blockIdx.x * kGlThreads + threadIdx.x;
  if (x >= W) return;
  const int y = blockIdx.y, k = blockIdx.z;
  const size_t i = (static_cast<size_t>(k) * H + y) * W + x;
  const int R = S / 2;
  const int tiles_x = W / N;
  {
    const int ks = wrap(k - h, K), ys = wrap(y - h, H), xs = wrap(x - h, W);
    const int g = (ys / N) * tiles_x + xs / N;
    const int r = idx[static_cast<size_t>(g) * K + ks];
    const int dy = r / S - R, dx = r % S - R;
    const uint16_t v = img[static_cast<size_t>(wrap(ys + dy, H)) * W + wrap(xs + dx, W)];
    vol[i] = static_cast<float>(v) * (1.0f / 65535.0f);
  }
}

// One periodic level along one axis of the region [0, Lk) x [0, Ly) x [0, Lx)
// of a K x H x W volume: analysis (bior1.5 on y / x: low-pass a[n] = sum_i
// h_i x[2n + i - 4], details (x[2n+1] - x[2n]) / sqrt2; Haar on k: sums and
// differences over sqrt2) or its inverse.  Axis 0 = k, 1 = y, 2 = x.
__device__ __forceinline__ float bior_lo_tap(int i) {
  constexpr float s = 1.41421356237309505f / 256.0f;
  constexpr float t[10] = {3 * s, -3 * s, -22 * s, 22 * s, 128 * s, 128 * s, 22 * s, -22 * s, -3 * s, 3 * s};
  return t[i];
}
// coefficient of detail d[n] in x[2n + m], m = -4 .. 5
__device__ __forceinline__ float bior_hi_syn(int m) {
  constexpr float s = 1.41421356237309505f / 256.0f;
  constexpr float t[10] = {-3 * s, -3 * s, 22 * s, 22 * s, -128 * s, 128 * s, -22 * s, -22 * s, 3 * s, 3 * s};
  return t[m + 4];
}

// grid: (ceil(Lx / 256), Ly, Lk); thread = one output element (k, y, x)
__global__ __launch_bounds__(kGlThreads) void gl_axis_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                             int H, int W, int Lk, int Ly, int Lx, int axis,
                                                             int inverse) {
  const int x = blockIdx.x * kGlThreads + threadIdx.x;
  if (x >= Lx) return;
  const int y = blockIdx.y, k = blockIdx.z;
  const size_t hw = static_cast<size_t>(H) * W;
  const size_t base = static_cast<size_t>(k) * hw + static_cast<size_t>(y) * W + x;
  const float c = 0.70710678118654752f;
  int n, L;
  size_t stride;
  if (axis == 0) {
    n = k, L = Lk, stride = hw;
  } else if (axis == 1) {
    n = y, L = Ly, stride = W;
  } else {
    n = x, L = Lx, stride = 1;
  }
  const float* line = in + (base - static_cast<size_t>(n) * stride);  // element 0 of this line
  auto at = [&](int j) { return line[static_cast<size_t>(wrap(j, L)) * stride]; };
  const int half = L / 2;
  float v;
  if (!inverse) {
    if (axis == 0) {
      const int m = n < half ? n : n - half;
      const float e = at(2 * m), o = at(2 * m + 1);
      v = n < half ? (e + o) * c : (e - o) * c;
    } else if (n < half) {
      v = 0.0f;
#pragma unroll
      for (int t = 0; t < 10; ++t) v = fmaf(bior_lo_tap(t), at(2 * n + t - 4), v);
    } else {
      const int m = n - half;
      v = (at(2 * m + 1) - at(2 * m)) * c;
    }
  } else {
    // input: a[0 .. half) then d[0 .. half)
    if (axis == 0) {
      const int m = n >> 1;
      const float a = at(m), d = at(half + m);
      v = (n & 1) ? (a - d) * c : (a + d) * c;
    } else {
      v = c * at(n >> 1);
      // details d[q] with 2q + m = n (mod L), m = -4 .. 5 of the parity of n
#pragma unroll
      for (int m = -4; m <= 5; ++m) {
        if (((n - m) & 1) == 0) v = fmaf(bior_hi_syn(m), at(half + wrap((n - m) / 2, half)), v);
      }
    }
  }
  out[base] = v;
}

__global__ void gl_copy_region_kernel(const float* __restrict__ from, float* __restrict__ to, int H, int W, int Lk,
                                      int Ly, int Lx) {
  const size_t region = static_cast<size_t>(Lk) * Ly * Lx;
  const size_t hw = static_cast<size_t>(H) * W;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < region;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int k = static_cast<int>(i / (static_cast<size_t>(Ly) * Lx));
    const int rem = static_cast<int>(i - static_cast<size_t>(k) * Ly * Lx);
    const size_t o = static_cast<size_t>(k) * hw + static_cast<size_t>(rem / Lx) * W + rem % Lx;
    to[o] = from[o];
  }
}

// hard threshold by band level: level l >= 1 of a detail band is the first
// level whose low-low-low region excludes the coefficient; the final
// approximation (inside the region of every level) is kept
__global__ __launch_bounds__(kGlThreads) void gl_threshold_kernel(float* __restrict__ vol, int K, int H, int W,
                                                                  int levels, float sigma, float a, float b) {
  const int x = blockIdx.x * kGlThreads + threadIdx.x;
  if (x >= W) return;
  const int y = blockIdx.y, k = blockIdx.z;
  const size_t i = (static_cast<size_t>(k) * H + y) * W + x;
  {
    int lev = 0;
    for (int j = 1; j <= levels; ++j)
      if (k >= (K >> j) || y >= (H >> j) || x >= (W >> j)) {
        lev = j;
        break;
      }
    if (lev > 0) {
      const float tau = sigma * (a - b * static_cast<float>(lev));
      if (!(fabsf(vol[i]) >= tau)) vol[i] = 0.0f;
    }
  }
}

// acc (=|+=) scale * src[(k + h) mod K][(y + h) mod H][(x + h) mod W]  (S_{-h})
__global__ __launch_bounds__(kGlThreads) void gl_unspin_kernel(const float* __restrict__ src,
                                                               float* __restrict__ acc, int K, int H, int W, int h,
                                                               int first, float scale) {
  const int x = blockIdx.x * kGlThreads + threadIdx.x;
  if (x >= W) return;
  const int y = blockIdx.y, k = blockIdx.z;
  const size_t i = (static_cast<size_t>(k) * H + y) * W + x;
  {
    const size_t hw = static_cast<size_t>(H) * W;
    const float v = scale * src[static_cast<size_t>(wrap(k + h, K)) * hw + static_cast<size_t>(wrap(y + h, H)) * W +
                                wrap(x + h, W)];
    acc[i] = first ? v : acc[i] + v;
  }
}

__global__ void gl_zero_kernel(unsigned long long* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// One workgroup per tile: w = eps / (TV(u) + eps) (the 1 / (TV + eps) weight
// scaled by eps, which cancels in the average), then every filtered block is
// added at its source position: num += w u, den += w (64-bit fixed point).
// The K blocks all lie in the tile's (S + N - 1)^2 search footprint, which
// is summed in LDS first; only its covered cells go to the image with global
// integer atomics.
template <int N, int K>
__global__ __launch_bounds__(kGlThreads) void gl_aggregate_kernel(const float* __restrict__ u,
                                                                   const int16_t* __restrict__ idx, int H, int W,
                                                                   int S, float eps,
                                                                   unsigned long long* __restrict__ num,
                                                                   unsigned long long* __restrict__ den) {
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
  for (int i = threadIdx.x; i < side * side; i += blockDim.x) {
    fnum[i] = 0;
    fden[i] = 0;
  }
  for (int i = threadIdx.x; i < kVals; i += blockDim.x) {
    const int k = i / (N * N), a = (i / N) % N, b = i % N;
    blk[i] = u[static_cast<size_t>(k) * hw + static_cast<size_t>(y0 + a) * W + x0 + b];
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

// out[(y - t) mod H][(x - t) mod W] (=|+=) scale * num / den  (S_{-t} of the estimate)
__global__ void gl_normalize_kernel(const unsigned long long* __restrict__ num,
                                    const unsigned long long* __restrict__ den, int H, int W, int t, int first,
                                    float scale, float* __restrict__ out) {
  const size_t n = static_cast<size_t>(H) * W;
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(i / W), x = static_cast<int>(i - static_cast<size_t>(y) * W);
    const float v = scale * static_cast<float>(static_cast<double>(static_cast<long long>(num[i])) /
                                               static_cast<double>(static_cast<long long>(den[i])));
    const size_t o = static_cast<size_t>(pmod(y - t, H)) * W + pmod(x - t, W);
    out[o] = first ? v : out[o] + v;
  }
}

unsigned grid_for(size_t n) {
  const size_t b = (n + kGlThreads - 1) / kGlThreads;
  return static_cast<unsigned>(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

template <int N, int K>
hipError_t global_nk(const GlobalJob& j, hipStream_t st) {
  const int H = j.H, W = j.W;
  const size_t hw = static_cast<size_t>(H) * W;
  const dim3 vol_grid((W + kGlThreads - 1) / kGlThreads, H, K);
  const int tiles = (H / N) * (W / N);
  const float eps = j.tv_eps_rel * j.sigma * static_cast<float>(N * N * K);
  for (int ti = 0; ti < j.n_shifts; ++ti) {
    const int t = j.shifts[ti];
    const uint16_t* img = j.noisy;
    if (t != 0) {
      hipLaunchKernelGGL(gl_roll_kernel, dim3(grid_for(hw)), dim3(kGlThreads), 0, st, j.noisy, H, W, t, j.shifted);
      img = j.shifted;
    }
    hipLaunchKernelGGL((gl_match_kernel<N, K>), dim3(tiles), dim3(kGlThreads), 0, st, img, H, W, j.search, j.idx);
    for (int h = 0; h < j.cycles; ++h) {
      float* A = j.vol_a;
      float* B = j.vol_b;
      hipLaunchKernelGGL((gl_volume_kernel<N, K>), vol_grid, dim3(kGlThreads), 0, st, img, j.idx, H, W, j.search, h,
                         A);
      // forward: level 0 ends in B; every coarser level ends in A and its
      // region is copied back into B
      for (int l = 0; l < j.levels; ++l) {
        const int Lk = K >> l, Ly = H >> l, Lx = W >> l;
        const size_t rn = static_cast<size_t>(Lk) * Ly * Lx;
        const dim3 axis_grid((Lx + kGlThreads - 1) / kGlThreads, Ly, Lk);
        float* s0 = l == 0 ? A : B;
        float* s1 = l == 0 ? B : A;
        hipLaunchKernelGGL(gl_axis_kernel, axis_grid, dim3(kGlThreads), 0, st, s0, s1, H, W, Lk, Ly, Lx, 1, 0);
        hipLaunchKernelGGL(gl_axis_kernel, axis_grid, dim3(kGlThreads), 0, st, s1, s0, H, W, Lk, Ly, Lx, 2, 0);
        hipLaunchKernelGGL(gl_axis_kernel, axis_grid, dim3(kGlThreads), 0, st, s0, s1, H, W, Lk, Ly, Lx, 0, 0);
        if (l > 0)
          hipLaunchKernelGGL(gl_copy_region_kernel, dim3(grid_for(rn)), dim3(kGlThreads), 0, st, A, B, H, W, Lk, Ly,
                             Lx);
      }
      hipLaunchKernelGGL(gl_threshold_kernel, vol_grid, dim3(kGlThreads), 0, st, B, K, H, W, j.levels, j.sigma, j.ht_a,
                         j.ht_b);
      // inverse, coarsest level first: each level reads B and ends in A; all
      // but the finest copy their region back into B
      for (int l = j.levels - 1; l >= 0; --l) {
        const int Lk = K >> l, Ly = H >> l, Lx = W >> l;
        const size_t rn = static_cast<size_t>(Lk) * Ly * Lx;
        const dim3 axis_grid((Lx + kGlThreads - 1) / kGlThreads, Ly, Lk);
        hipLaunchKernelGGL(gl_axis_kernel, axis_grid, dim3(kGlThreads), 0, st, B, A, H, W, Lk, Ly, Lx, 0, 1);
        hipLaunchKernelGGL(gl_axis_kernel, axis_grid, dim3(kGlThreads), 0, st, A, B, H, W, Lk, Ly, Lx, 2, 1);
        hipLaunchKernelGGL(gl_axis_kernel, axis_grid, dim3(kGlThreads), 0, st, B, A, H, W, Lk, Ly, Lx, 1, 1);
        if (l > 0)
          hipLaunchKernelGGL(gl_copy_region_kernel, dim3(grid_for(rn)), dim3(kGlThreads), 0, st, A, B, H, W, Lk, Ly,
                             Lx);
      }
      hipLaunchKernelGGL(gl_unspin_kernel, vol_grid, dim3(kGlThreads), 0, st, A, j.vol_u, K, H, W, h, h == 0 ? 1 : 0,
                         1.0f / static_cast<float>(j.cycles));
    }
    hipLaunchKernelGGL(gl_zero_kernel, dim3(grid_for(2 * hw)), dim3(kGlThreads), 0, st, j.num, 2 * hw);
    hipLaunchKernelGGL((gl_aggregate_kernel<N, K>), dim3(tiles), dim3(kGlThreads), 0, st, j.vol_u, j.idx, H, W,
                       j.search, eps, j.num, j.num + hw);
    hipLaunchKernelGGL(gl_normalize_kernel, dim3(grid_for(hw)), dim3(kGlThreads), 0, st, j.num, j.num + hw, H, W, t,
                       ti == 0 ? 1 : 0, 1.0f / static_cast<float>(j.n_shifts), j.out);
  }
  return hipGetLastError();
}

}  // namespace

size_t global_volume_bytes(int H, int W, int K) { return static_cast<size_t>(K) * H * W * sizeof(float); }

template <int N, int K>
static hipError_t match_nk(const uint16_t* img, int H, int W, int search, int16_t* idx, hipStream_t st) {
  hipLaunchKernelGGL((gl_match_kernel<N, K>), dim3((H / N) * (W / N)), dim3(kGlThreads), 0, st, img, H, W, search,
                     idx);
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
