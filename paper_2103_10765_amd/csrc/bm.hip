// Block matching (Sec. 2, eq. dfg; arg_K min of Sec. 3.1), shift-wise.
//
// A wave holds 64 consecutive references of one reference row (62 produce
// output, the last two only contribute columns).  For every displacement
// (dy, dx) of the search window each lane forms the squared differences of its
// own three pixel columns [3q, 3q+3) of the reference block against the
// displaced block, summed over the 8 block rows.  Because references sit 3
// pixels apart, a block's 8 columns are the 3 columns of its own lane, the 3
// of the next lane and the first 2 of the lane after that: the box filter of
// the squared-difference map at the reference position is completed with two
// DPP wave shifts.  Values are integers held in float64, so every distance is
// exact (< 2^38) and keys dist * 2048 + rank order candidates by (distance,
// rank) exactly.
//
// Three consecutive dx are evaluated per iteration as independent chains, with
// the next columns prefetched from LDS while they compute.  Each lane keeps
// the K-1 best keys of its reference in a sorted register list; candidates
// below the current worst key are appended to a per-lane LDS buffer, which is
// sorted and merged into the list as one batch when some lane's buffer is
// nearly full.
//
// A workgroup of four waves covers RPW reference rows x SPLIT parts of the
// displacement rows (RPW * SPLIT = 4) and shares one LDS image tile with the
// search halo.  The tile is held as uint16 in three sub-arrays by column
// residue mod 3, so the 64 lanes of a wave, whose columns are 3 apart, read
// 64 consecutive halfwords (no bank conflicts).  With SPLIT > 1 the waves of a
// row publish their current worst kept key so every wave prunes with the
// row's best bound, and the partial lists are merged at the end by a bitonic
// network in registers.  LDS stays under 40 KB per workgroup, so residency is
// bounded by registers (the float64 reference block, six prefetched columns
// and the sorted list), not by LDS.
#include "common.h"
#include "kernels.h"
#include "topk.h"

namespace gbm3d {

namespace {

constexpr int kLanesOut = 62;
constexpr int kSubCols = 80;  // per residue: columns 3j+m for j < 80 (needs 3*63 + 2*kMaxR + 8)
constexpr double kInf = __builtin_huge_val();

static_assert(3 * kSubCols >= 3 * (kWave - 1) + 2 + (2 * kMaxR + 1 + 5) + 1, "tile too narrow");

template <int RPW>
struct TileShape {
  static constexpr int rows = kStep * (RPW - 1) + kPatch + 2 * kMaxR;
};

// value of lane + 1 (DPP wave shift; lane 63 keeps its own value)
__device__ __forceinline__ double from_next_lane(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int nlo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  const int nhi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __hiloint2double(nhi, nlo);
}

template <int K, int RPW, int SPLIT>
struct BmSmem {
  static constexpr int L = K - 1;
  static constexpr int kBuf = RPW == 1 ? 8 : 7;  // buffered candidates per lane (merged as a batch of 8)
  static constexpr int kFlushAt = kBuf - 3;      // an iteration appends at most 3
  static constexpr size_t kTile = sizeof(uint16_t) * 3 * TileShape<RPW>::rows * kSubCols;
  static constexpr size_t kBufBytes = sizeof(double) * 4 * kBuf * kWave;
  static constexpr size_t kBound = SPLIT > 1 ? sizeof(double) * 4 * kWave : 0;
  static constexpr size_t kScan = kTile + kBufBytes + kBound;
  // merge: SPLIT 4 exchanges two lists at a time, SPLIT 2 one per row (2 rows)
  static constexpr size_t kMerge = SPLIT > 1 ? sizeof(double) * 2 * L * kWave : 0;
  static constexpr size_t bytes = kScan > kMerge ? kScan : kMerge;
  static_assert(bytes <= 40960, "LDS no larger than a quarter of a CU");
};

__host__ __device__ constexpr int bm_segments(int W) { return ((W + kStep - 1) / kStep + kLanesOut - 1) / kLanesOut; }

template <int RPW>
__host__ __device__ constexpr int bm_items(int H, int W) {
  return (((H + kStep - 1) / kStep) + RPW - 1) / RPW * bm_segments(W);
}

// One work item: reference rows [RPW*pb, RPW*pb + RPW) x 62 reference columns.
template <int K, int RPW, int SPLIT>
__device__ __forceinline__ void bm_body(unsigned char* smem, const uint16_t* __restrict__ img_,
                                        int16_t* __restrict__ idx_, int H, int W, int R, int item) {
  const auto img = to_global(img_);
  const auto idx = to_global(idx_);
  static_assert(RPW * SPLIT == 4, "four waves per workgroup");
  using Smem = BmSmem<K, RPW, SPLIT>;
  constexpr int L = K - 1;
  constexpr int kBuf = Smem::kBuf;
  constexpr int rows = TileShape<RPW>::rows;
  // sub[m][r][j] = tile pixel (row r, column 3j + m)
  uint16_t* sub = reinterpret_cast<uint16_t*>(smem);
  double* buf = reinterpret_cast<double*>(smem + Smem::kTile);
  // bound[w][lane]: the worst key of wave w's current list for its reference
  unsigned long long* bound = reinterpret_cast<unsigned long long*>(smem + Smem::kTile + Smem::kBufBytes);

  const int nRy = (H + kStep - 1) / kStep, nRx = (W + kStep - 1) / kStep;
  const int segs = bm_segments(W);
  const int S = 2 * R + 1;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = wave_id();
  const int row_in_wg = wave / SPLIT, part = wave % SPLIT;
  const int p0 = (item / segs) * RPW;
  const int p = p0 + row_in_wg;
  const int q0 = (item % segs) * kLanesOut;

  // LDS image tile, periodic: rows 3p0-R .. 3(p0+RPW-1)+7+R, columns 3q0-R ..
  const int y0 = kStep * p0 - R;
  const int x0 = kStep * q0 - R;
  const int nrows = kStep * (RPW - 1) + kPatch + 2 * R;
  // y0 < H and x0 < W: rows and columns wrap at most once when the image
  // is at least as tall as the tile and as wide as its columns
  const bool near = H >= nrows && W >= 3 * kSubCols;
  for (int i = threadIdx.x; i < nrows * 3 * kSubCols; i += blockDim.x) {
    const int r = i / (3 * kSubCols), c = i - r * (3 * kSubCols);
    int y = y0 + r, x = x0 + c;
    if (near) {
      y += y < 0 ? H : (y >= H ? -H : 0);
      x += x < 0 ? W : (x >= W ? -W : 0);
    } else {
      y = pmod(y, H);
      x = pmod(x, W);
    }
    sub[((c % 3) * rows + r) * kSubCols + c / 3] = img[static_cast<size_t>(y) * W + x];
  }
  if constexpr (SPLIT > 1) bound[threadIdx.x] = __double_as_longlong(kInf);
  __syncthreads();

  // pixel (tile row r, column 3 * lane + c) for c >= 0
  auto px = [&](int r, int c) -> double {
    return static_cast<double>(sub[((c % 3) * rows + r) * kSubCols + lane + c / 3]);
  };
  const int trow = kStep * row_in_wg;  // this wave's first tile row for dy = -R
  double rf[kPatch][3];
#pragma unroll
  for (int a = 0; a < kPatch; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) rf[a][b] = px(trow + R + a, R + b);

  double list[L];
#pragma unroll
  for (int i = 0; i < L; ++i) list[i] = kInf;
  double thr = kInf;
  int cnt = 0;
  double* mybuf = buf + wave * kBuf * kWave + lane;  // entry j at mybuf[j * kWave]

  auto flush = [&]() {
    merge_buffer<L, 8>(list, mybuf, kWave, cnt);
    cnt = 0;
    // Keys are unique, so a key above any wave's current worst kept key has
    // K-1 better keys already and can never enter the merged list: prune
    // with the smallest bound published by the waves of this reference row.
    double t = list[L - 1];
    if constexpr (SPLIT > 1) {
      // relaxed workgroup-scope atomics: another wave's bound may be stale,
      // which only makes it larger (bounds never increase)
      __hip_atomic_store(bound + wave * kWave + lane, static_cast<unsigned long long>(__double_as_longlong(t)),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
      for (int s2 = 0; s2 < SPLIT; ++s2)
        t = fmin(t, __longlong_as_double(static_cast<long long>(__hip_atomic_load(
                        bound + (row_in_wg * SPLIT + s2) * kWave + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))));
    }
    thr = t;
  };

  const int dy_begin = (part * S) / SPLIT, dy_end = ((part + 1) * S) / SPLIT;
  const int nIter = (S + 5) / 6;  // 6 displacements per unrolled iteration (extra ones masked)
  const int r_center = R * S + R;

  for (int dyi = dy_begin; dyi < dy_end; ++dyi) {
    const int rank_row = dyi * S;
    // column 6 * it + 3 * jo + m of the candidate rows (8 tile rows from trow + dyi)
    auto load = [&](double* c, int m, int j) {
      const uint16_t* base = sub + (m * rows + trow + dyi) * kSubCols + lane + j;
#pragma unroll
      for (int a = 0; a < kPatch; ++a) c[a] = static_cast<double>(base[a * kSubCols]);
    };
    // partial sums of one displacement: (cols 0..1, col 2) of this lane
    auto partial = [&](const double* ca, const double* cb, const double* cc, double& a2, double& a1) {
      a2 = 0.0;
      a1 = 0.0;
#pragma unroll
      for (int a = 0; a < kPatch; ++a) {
        const double d0 = rf[a][0] - ca[a];
        const double d1 = rf[a][1] - cb[a];
        const double d2 = rf[a][2] - cc[a];
        a2 = fma(d0, d0, a2);
        a2 = fma(d1, d1, a2);
        a1 = fma(d2, d2, a1);
      }
    };
    auto finish = [&](double a2, double a1, int dxi) {
      const double s3 = a2 + a1;
      // dist(l) = s3(l) + s3(l+1) + a2(l+2) = s3(l) + X(l+1), X = s3 + a2(l+1)
      const double x = s3 + from_next_lane(a2);
      const double dist = s3 + from_next_lane(x);
      const int rank = rank_row + dxi;
      double key = fma(dist, 2048.0, static_cast<double>(rank));
      if (dxi >= S || rank == r_center) key = kInf;
      if (key < thr) {
        mybuf[cnt * kWave] = key;
        ++cnt;
      }
    };
    // displacements dxi, dxi+1, dxi+2 from columns (c0 c1 c2 n0 n1); columns
    // dxi+3 .. dxi+5 (residues 0, 1, 2 at sub-array column j) are prefetched
    auto iter3 = [&](const double* c0, const double* c1, const double* c2, double* n0, double* n1, double* n2,
                     int dxi, int j) {
      load(n0, 0, j);
      load(n1, 1, j);
      load(n2, 2, j);
      double a2a, a1a, a2b, a1b, a2c, a1c;
      partial(c0, c1, c2, a2a, a1a);
      partial(c1, c2, n0, a2b, a1b);
      partial(c2, n0, n1, a2c, a1c);
      finish(a2a, a1a, dxi);
      finish(a2b, a1b, dxi + 1);
      finish(a2c, a1c, dxi + 2);
      if (wave_any(cnt > Smem::kFlushAt)) flush();
    };

    double A0[kPatch], A1[kPatch], A2[kPatch], B0[kPatch], B1[kPatch], B2[kPatch];
    load(A0, 0, 0);
    load(A1, 1, 0);
    load(A2, 2, 0);
    for (int it = 0; it < nIter; ++it) {
      const int dxi = 6 * it;
      iter3(A0, A1, A2, B0, B1, B2, dxi, 2 * it + 1);
      iter3(B0, B1, B2, A0, A1, A2, dxi + 3, 2 * it + 2);
    }
  }
  if (wave_any(cnt > 0)) flush();

  if constexpr (SPLIT > 1) {
    // merge the SPLIT partial lists of each row into its part-0 wave
    __syncthreads();  // tile, buffers and bounds are dead
    double* ml = reinterpret_cast<double*>(smem);
    auto put = [&](int slot) {
#pragma unroll
      for (int i = 0; i < L; ++i) ml[(slot * L + i) * kWave + lane] = list[i];
    };
    auto take = [&](int slot) {
      const double* b = ml + slot * L * kWave + lane;
      merge_sorted<L>(list, [&](int j) { return b[j * kWave]; });
    };
    if constexpr (SPLIT == 2) {
      if (part == 1) put(row_in_wg);
      __syncthreads();
      if (part == 0) take(row_in_wg);
    } else {
      if (part & 1) put(part >> 1);  // parts 1, 3 -> slots 0, 1
      __syncthreads();
      if (!(part & 1)) take(part >> 1);  // part 0 <- 1, part 2 <- 3
      __syncthreads();
      if (part == 2) put(0);
      __syncthreads();
      if (part == 0) take(0);
    }
    if (part != 0) return;
  }

  const int q = q0 + lane;
  if (lane < kLanesOut && q < nRx && p < nRy) {
    const auto out = idx + (static_cast<size_t>(p) * nRx + q) * K;
    out[0] = static_cast<int16_t>(r_center);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      out[1 + i] = key_rank(list[i]);
    }
  }
}

template <int K, int RPW, int SPLIT, bool BATCH>
__global__ __launch_bounds__(256, 2) void bm_kernel(ImgRec one, WorkList wl, int R, int use_pilot) {
  __shared__ __align__(16) unsigned char smem[BmSmem<K, RPW, SPLIT>::bytes];
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) {
    bm_body<K, RPW, SPLIT>(smem, use_pilot ? r.pilot : r.noisy, r.idx, r.H, r.W, R, item);
  });
}

}  // namespace

template <int K, int RPW, int SPLIT>
static hipError_t launch_bm_shape(const ImgRec& one, const WorkList* wl, int R, int use_pilot, int grid_cap,
                                  hipStream_t st) {
  if (!wl) {
    const int items = bm_items<RPW>(one.H, one.W);
    hipLaunchKernelGGL((bm_kernel<K, RPW, SPLIT, false>), dim3(items), dim3(256), 0, st, one, WorkList{}, R,
                       use_pilot);
  } else {
    if (wl->total <= 0) return hipSuccess;
    const int grid = std::min(wl->total, grid_cap);
    hipLaunchKernelGGL((bm_kernel<K, RPW, SPLIT, true>), dim3(grid), dim3(256), 0, st, one, *wl, R, use_pilot);
  }
  return hipGetLastError();
}

int bm_auto_split(long total_waves_unsplit) {
  return total_waves_unsplit >= 2048 ? 1 : (total_waves_unsplit >= 1024 ? 2 : 4);
}

int bm_items_for(int H, int W, int split) {
  switch (split) {
    case 1: return bm_items<4>(H, W);
    case 2: return bm_items<2>(H, W);
    default: return bm_items<1>(H, W);
  }
}

long bm_waves_unsplit(int H, int W) {
  return static_cast<long>((H + kStep - 1) / kStep) * bm_segments(W);
}

template <int K>
static hipError_t launch_bm_k(const ImgRec& one, const WorkList* wl, int R, int split, int use_pilot, int grid_cap,
                              hipStream_t st) {
  switch (split) {
    case 1: return launch_bm_shape<K, 4, 1>(one, wl, R, use_pilot, grid_cap, st);
    case 2: return launch_bm_shape<K, 2, 2>(one, wl, R, use_pilot, grid_cap, st);
    case 4: return launch_bm_shape<K, 1, 4>(one, wl, R, use_pilot, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bm(const ImgRec& one, const WorkList* wl, int R, int K, int split, int use_pilot, int grid_cap,
                     hipStream_t st) {
  if (split <= 0) split = bm_auto_split(bm_waves_unsplit(one.H, one.W));
  switch (K) {
    case 2: return launch_bm_k<2>(one, wl, R, split, use_pilot, grid_cap, st);
    case 4: return launch_bm_k<4>(one, wl, R, split, use_pilot, grid_cap, st);
    case 8: return launch_bm_k<8>(one, wl, R, split, use_pilot, grid_cap, st);
    case 16: return launch_bm_k<16>(one, wl, R, split, use_pilot, grid_cap, st);
    case 32: return launch_bm_k<32>(one, wl, R, split, use_pilot, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbm3d
