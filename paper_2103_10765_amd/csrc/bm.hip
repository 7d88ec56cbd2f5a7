// Block matching (Sec. 2, eq. dfg; arg_K min of Sec. 3.1), shift-wise.
//
// For one reference row p and 62 consecutive reference columns q, a workgroup
// of four waves scans the search window: wave w takes a quarter of the
// displacement rows dy, and for each displacement (dy, dx) every lane forms
// the squared differences of its own three pixel columns [3q, 3q+3) of the
// reference block against the displaced block, summed over the 8 block rows.
// Because references sit 3 pixels apart, a block's 8 columns are the 3
// columns of its own lane, the 3 of the next lane and the first 2 of the lane
// after that: the box filter of the squared-difference map at the reference
// position is completed with two wavefront shuffles.  All arithmetic is on
// integers held in float64, so distances are exact (< 2^38).
//
// Each lane keeps the K-1 best keys (distance * 2048 + rank) of its
// reference in a sorted register list.  Candidates that beat the current
// worst key are appended to a small per-lane LDS buffer; the buffer is merged
// into the list when some lane fills it, so the insertion network runs once
// per batch instead of on almost every displacement.  At the end the four
// waves' lists are merged through LDS and the ranks are written out.
#include "common.h"
#include "kernels.h"

namespace gbm3d {

namespace {

constexpr int kLanesOut = 62;                       // references per workgroup (lanes 62, 63 only help)
constexpr int kTileRows = kPatch + 2 * kMaxR;       // 46
constexpr int kTileCols = 3 * kWave + 2 + 2 * kMaxR + 4;  // 236 (slack for the 3-column unroll)
constexpr int kBuf = 8;                             // buffered candidates per lane
constexpr double kInf = __builtin_huge_val();

template <int L>
__device__ __forceinline__ void insert_sorted(double (&list)[L], double key) {
  // list is ascending; a key not below list[L-1] leaves it unchanged
#pragma unroll
  for (int i = L - 1; i >= 1; --i) list[i] = (key < list[i - 1]) ? list[i - 1] : fmin(key, list[i]);
  list[0] = fmin(key, list[0]);
}

template <int K>
struct BmSmem {
  static constexpr int L = K - 1;
  static constexpr size_t kScan = sizeof(float) * kTileRows * kTileCols + sizeof(double) * 4 * kBuf * kWave;
  static constexpr size_t kMerge = sizeof(double) * 4 * (L > 0 ? L : 1) * kWave;
  static constexpr size_t bytes = kScan > kMerge ? kScan : kMerge;
};

template <int K>
__global__ __launch_bounds__(256, 2) void bm_kernel(const uint16_t* __restrict__ img, int H, int W, int R,
                                                    int nRy, int nRx, int16_t* __restrict__ idx) {
  constexpr int L = K - 1;
  __shared__ __align__(16) unsigned char smem[BmSmem<K>::bytes];
  float(*tile)[kTileCols] = reinterpret_cast<float(*)[kTileCols]>(smem);
  double* buf = reinterpret_cast<double*>(smem + sizeof(float) * kTileRows * kTileCols);

  const int S = 2 * R + 1;
  const int p = blockIdx.y;
  const int q0 = blockIdx.x * kLanesOut;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;

  // Image tile with the search halo, periodic: rows 3p-R .. 3p+7+R,
  // columns 3q0-R .. 3q0+191+R (+ slack).
  const int y0 = kStep * p - R;
  const int x0 = kStep * q0 - R;
  const int rows = kPatch + 2 * R;
  for (int i = threadIdx.x; i < rows * kTileCols; i += blockDim.x) {
    const int r = i / kTileCols, c = i - r * kTileCols;
    const int y = pmod(y0 + r, H), x = pmod(x0 + c, W);
    tile[r][c] = static_cast<float>(img[static_cast<size_t>(y) * W + x]);
  }
  __syncthreads();

  // this lane's three reference columns, all 8 rows
  double rf[kPatch][3];
#pragma unroll
  for (int a = 0; a < kPatch; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) rf[a][b] = static_cast<double>(tile[R + a][R + 3 * lane + b]);

  double list[L];
#pragma unroll
  for (int i = 0; i < L; ++i) list[i] = kInf;
  double thr = kInf;
  int cnt = 0;
  double* mybuf = buf + wave * kBuf * kWave + lane;  // entry j at mybuf[j * kWave]

  auto flush = [&]() {
#pragma unroll 1
    for (int j = 0; j < kBuf; ++j) {
      if (!__any(j < cnt)) break;
      const double k = (j < cnt) ? mybuf[j * kWave] : kInf;
      insert_sorted<L>(list, k);
    }
    cnt = 0;
    thr = list[L - 1];
  };

  const int dy_begin = (wave * S) / 4, dy_end = ((wave + 1) * S) / 4;
  const int S3 = ((S + 2) / 3) * 3;  // dx iterations, a multiple of 3 (extra ones are masked)
  const int r_center = R * S + R;

  for (int dyi = dy_begin; dyi < dy_end; ++dyi) {
    // candidate block rows start at tile row (R + dy) = dyi; columns at 3*lane + dxi
    const float* base = &tile[dyi][3 * lane];
    double c0[kPatch], c1[kPatch], c2[kPatch];
#pragma unroll
    for (int a = 0; a < kPatch; ++a) {
      c0[a] = static_cast<double>(base[a * kTileCols + 0]);
      c1[a] = static_cast<double>(base[a * kTileCols + 1]);
      c2[a] = static_cast<double>(base[a * kTileCols + 2]);
    }
    const int rank_row = dyi * S;

    // one displacement: columns (ca, cb, cc) hold displaced columns dxi, dxi+1, dxi+2
    auto step = [&](const double* ca, const double* cb, const double* cc, int dxi) {
      double a2 = 0.0, a1 = 0.0;
#pragma unroll
      for (int a = 0; a < kPatch; ++a) {
        const double d0 = rf[a][0] - ca[a];
        const double d1 = rf[a][1] - cb[a];
        const double d2 = rf[a][2] - cc[a];
        a2 = fma(d0, d0, a2);
        a2 = fma(d1, d1, a2);
        a1 = fma(d2, d2, a1);
      }
      const double s3 = a2 + a1;
      const double dist = s3 + __shfl_down(s3, 1, kWave) + __shfl_down(a2, 2, kWave);
      const int rank = rank_row + dxi;
      double key = fma(dist, 2048.0, static_cast<double>(rank));
      if (dxi >= S || rank == r_center) key = kInf;
      if (key < thr) {
        mybuf[cnt * kWave] = key;
        ++cnt;
      }
      if (__any(cnt == kBuf)) flush();
    };
    auto reload = [&](double* c, int col) {
#pragma unroll
      for (int a = 0; a < kPatch; ++a) c[a] = static_cast<double>(base[a * kTileCols + col]);
    };

    for (int dxi = 0; dxi < S3; dxi += 3) {
      step(c0, c1, c2, dxi);
      reload(c0, dxi + 3);
      step(c1, c2, c0, dxi + 1);
      reload(c1, dxi + 4);
      step(c2, c0, c1, dxi + 2);
      reload(c2, dxi + 5);
    }
  }
  flush();

  // merge the four waves' lists: lists[w][i][lane]
  __syncthreads();
  double* lists = reinterpret_cast<double*>(smem);
#pragma unroll
  for (int i = 0; i < L; ++i) lists[(wave * L + i) * kWave + lane] = list[i];
  __syncthreads();
  if (wave != 0) return;
  const int q = q0 + lane;
  const bool valid = lane < kLanesOut && q < nRx;
  int16_t* out = idx + (static_cast<size_t>(p) * nRx + q) * K;
  if (valid) out[0] = static_cast<int16_t>(r_center);
  int ptr0 = 0, ptr1 = 0, ptr2 = 0, ptr3 = 0;
  for (int o = 0; o < L; ++o) {
    const double h0 = ptr0 < L ? lists[(0 * L + ptr0) * kWave + lane] : kInf;
    const double h1 = ptr1 < L ? lists[(1 * L + ptr1) * kWave + lane] : kInf;
    const double h2 = ptr2 < L ? lists[(2 * L + ptr2) * kWave + lane] : kInf;
    const double h3 = ptr3 < L ? lists[(3 * L + ptr3) * kWave + lane] : kInf;
    const double m01 = fmin(h0, h1), m23 = fmin(h2, h3);
    const double m = fmin(m01, m23);
    if (m == h0) ++ptr0;
    else if (m == h1) ++ptr1;
    else if (m == h2) ++ptr2;
    else ++ptr3;
    const double rank = m - 2048.0 * floor(m * (1.0 / 2048.0));
    if (valid) out[1 + o] = static_cast<int16_t>(rank);
  }
}

}  // namespace

template <int K>
static hipError_t launch_bm_k(const uint16_t* img, int H, int W, int R, int16_t* idx, hipStream_t st) {
  const int nRy = (H + kStep - 1) / kStep, nRx = (W + kStep - 1) / kStep;
  dim3 grid((nRx + kLanesOut - 1) / kLanesOut, nRy);
  hipLaunchKernelGGL(bm_kernel<K>, grid, dim3(256), 0, st, img, H, W, R, nRy, nRx, idx);
  return hipGetLastError();
}

hipError_t launch_bm(const uint16_t* img, int H, int W, int R, int K, int16_t* idx, hipStream_t st) {
  switch (K) {
    case 2: return launch_bm_k<2>(img, H, W, R, idx, st);
    case 4: return launch_bm_k<4>(img, H, W, R, idx, st);
    case 8: return launch_bm_k<8>(img, H, W, R, idx, st);
    case 16: return launch_bm_k<16>(img, H, W, R, idx, st);
    case 32: return launch_bm_k<32>(img, H, W, R, idx, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbm3d
