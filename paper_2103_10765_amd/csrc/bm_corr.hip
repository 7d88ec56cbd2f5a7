// Block matching in the correlation form of Theorem 1 (Sec. 2), on the
// matrix cores.  Same result as the shift-wise kernel: for every reference
// the K-1 smallest keys dist * 2048 + rank over the search window, the
// reference itself in slot 0.
//
// ||a - b||^2 = N(a) + N(b) - 2 <a, b>, N the block's squared norm.  The
// distance is translation invariant, so pixels are shifted by 32896:
// z = Z - 32896 = 256 h + l with signed bytes h = (Z >> 8) - 128 and
// l = (Z & 255) - 128, and <a, b> = 65536 Phh + 256 (Phl + Plh) + Pll: four
// exact int8 dot products of length 64, one v_mfma_i32_16x16x64_i8 each for
// 16 candidates x 16 references.
//
// A workgroup is four waves over TPW 4 x 4 reference tiles side by side
// (step 3), SPLIT waves per tile, each walking a share of the tile's
// candidate blocks.  Its prologue stages the pixels of the windows' union in
// LDS as byte planes (NC copies shifted by 0..3 bytes, so that every MFMA
// operand is an aligned read) and the exact squared norm of every candidate
// block of the union, split as N = 512 nh + nl (nh in int32, nl < 512).
//
// A tile's windows (39 x 39 each) cover a 48 x 48 square of candidate
// positions, walked in 4 x 4 candidate blocks from the centre outwards.
// Result lane (g, n) holds reference n against candidates (row g, columns
// 0..3) of the block.  With -nh of each candidate as the accumulator input of
// the cross term,
//     s' = 256 Phh + Phl + Plh - nh,     d = N(a) + nl - 2 X,  X = 256 s' + Pll.
// As nl >= 0, a pair with X <= Y = floor((N(a) - ceil(thr / 2048)) / 2) has
// d >= ceil(thr / 2048), so key = 2048 d + rank >= thr, the lane's bound on
// the (K-1)-th best key: it is dropped.  The test runs in 32-bit integers:
// with Y = 65536 Yh + Yl (0 <= Yl < 65536) and -Yh as the accumulator input
// of the high product, X - Y = 256 c + Pll - Yl where
// c = 256 (Phh - Yh) + Phl + Plh - nh; since |Pll - Yl| < 2^21, clamping c
// to [-2^13, 2^13] keeps the sign, so a pair survives iff
// 256 clamp(c) + Pll > Yl.  The few survivors are parked
// raw (c, Pll, position) in the lane's LDS buffer; when some lane's buffer
// is nearly full, every lane forms the exact keys of its parked pairs in
// float64 (integers below 2^51), drops those outside its window and merges
// them into its sorted list.  The first blocks of each wave (those nearest
// the centre) skip the pre-test: their exact keys go straight into the
// lists, whose merged (K-1)-th best then gives a tight first bound.
//
// Every lane keeps the K-1 best keys of its reference among its quarter of
// the candidates; the four quarters, and the SPLIT waves that share a tile,
// share upper bounds on the reference's (K-1)-th best key: the smallest
// worst kept key of any list, the largest m-th best of any list where m
// lists-worth of keys make K-1 (n lists each with m keys at or below a value
// hold n m >= K-1 of them), and after the first blocks the exact (K-1)-th
// best of the wave's four lists.  Keys are unique, so a key at or above a
// bound cannot be among the K-1 best.  The lists merge with bitonic networks
// at the end.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "topk.h"

namespace gbm3d {

namespace {

constexpr int kMaxNb = (2 * kMaxR + 10 + 3) / 4;  // candidate blocks per axis of a tile's union
constexpr int kCand = 4 * kMaxNb;                 // candidate positions per axis of a tile's union
constexpr int kPixRows = kCand + 7;               // pixel rows of the union
constexpr int kZShift = 32896;
constexpr double kInf = __builtin_huge_val();

// Blocks per sorted batch of the first (pre-test free) blocks: four keys
// each, at most the list length + 1; and that phase's length in blocks.
template <int K>
constexpr int kBatchBlocks = K >= 16 ? 4 : (K >= 8 ? 2 : 1);
template <int K>
constexpr int kDenseBlocks = (K >= 32 ? 4 : 2) * kBatchBlocks<K>;

// Workgroup shape: TPW reference tiles side by side, SPLIT waves per tile.
// Eight-wave workgroups (small groups only: their lists fit the registers
// of four waves per SIMD) keep the parked-pair buffers short to stay at two
// workgroups per compute unit; the four-wave ones of four tiles park more.
template <int K, int TPW, int SPLIT>
struct Cfg {
  static constexpr int kWaves = TPW * SPLIT;
  // parked pairs per lane before a merge (a block parks at most four)
  static constexpr int kBuf = kWaves == 8 ? 8 : (K >= 16 ? (TPW == 4 ? 16 : 12) : 8);
  static constexpr int kFlushAt = kBuf - 4;
  // byte-shifted copies of the planes (4: aligned operand reads) where the LDS allows
  static constexpr int kNC = kWaves == 4 && TPW <= 2 ? 4 : 1;
  static_assert(kWaves == 4 || kWaves == 8, "four or eight waves per workgroup");
};

template <int TPW, int NC>
struct Geo {
  static constexpr int kCandCols = kCand + 12 * (TPW - 1);  // candidate columns of the workgroup's union
  static constexpr int kNC = NC;                            // byte-shifted copies of the planes
  // bytes per plane row: with one copy, 25 dwords (mod 32), so that the
  // three-dword reads of the ten rows an operand read touches fall in
  // distinct LDS banks
  static constexpr int kPitch = NC == 4 ? (kCandCols + 8 + 7) / 8 * 8 : ((kCandCols + 8 + 28) / 128 * 128 + 100);
  static constexpr int kZCols = kPitch + 4;                   // pixel columns staged (every copy's bytes)
  static constexpr int kPlane = kPixRows * kPitch;
  // one copy: h plane then l plane, plus a skew that keeps the 16 lanes of
  // an operand read in distinct LDS banks
  static constexpr int kCopy = 2 * kPlane + (TPW == 1 ? 24 : 8);
};

constexpr size_t align16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

template <int K, int TPW, int SPLIT>
struct Smem {
  using C = Cfg<K, TPW, SPLIT>;
  using G = Geo<TPW, C::kNC>;
  static constexpr int L = K - 1;
  static constexpr size_t kNh = align16(static_cast<size_t>(G::kNC) * G::kCopy);  // int32 -nh [kCand][kCandCols]
  static constexpr size_t kNl = kNh + sizeof(int) * kCand * G::kCandCols;        // u16 nl [kCand][kCandCols]
  static constexpr size_t kDyn = align16(kNl + sizeof(uint16_t) * kCand * G::kCandCols);
  // the dynamic region holds the prologue's column sums, then the parked
  // pairs and the shared bounds
  static constexpr size_t kColSums = sizeof(double) * kCand * (G::kCandCols + 7);
  static constexpr size_t kBufBytes = sizeof(unsigned long long) * C::kWaves * C::kBuf * kWave;
  static constexpr size_t kBound = SPLIT > 1 ? sizeof(double) * 2 * C::kWaves * kWave : 0;
  static constexpr size_t kDynBytes = kColSums > kBufBytes + kBound ? kColSums : kBufBytes + kBound;
  // end of the item: lists handed between the SPLIT waves of each tile
  static constexpr size_t kMerge = sizeof(double) * L * kWave * (SPLIT == 1 ? 0 : (SPLIT == 2 ? TPW : 2 * TPW));
  static constexpr size_t bytes = kDyn + kDynBytes > kMerge ? kDyn + kDynBytes : kMerge;
  // the staged pixels (u16 [kPixRows][kZCols]) live in the norm area until the norms are formed
  static_assert(sizeof(uint16_t) * kPixRows * G::kZCols <= sizeof(int) * kCand * G::kCandCols, "pixel stage");
};

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Candidate blocks of an nb x nb grid in rings of growing Chebyshev distance
// from its centre (near displacements first tighten the bounds early), each
// entry the block's (row << 4) | column (the walk does no division by the
// run-time nb, and the position packs into a parked pair).
struct BlockOrder {
  int b[kMaxNb + 1][kMaxNb * kMaxNb];  // 32-bit entries: read with scalar loads
};

constexpr BlockOrder make_block_order() {
  BlockOrder o{};
  for (int nb = 1; nb <= kMaxNb; ++nb) {
    int n = 0;
    for (int ring = 0; ring <= 2 * nb; ++ring)
      for (int b = 0; b < nb * nb; ++b) {
        int dr = 2 * (b / nb) - (nb - 1), dc = 2 * (b % nb) - (nb - 1);
        dr = dr < 0 ? -dr : dr;
        dc = dc < 0 ? -dc : dc;
        if ((dr > dc ? dr : dc) == ring) o.b[nb][n++] = (b / nb) << 4 | (b % nb);
      }
  }
  return o;
}

static_assert(kMaxNb < 16, "block rows and columns pack into 4 bits");

__constant__ BlockOrder kOrder = make_block_order();

template <int TPW>
__host__ __device__ constexpr int corr_col_items(int W) {
  return ((W + kStep - 1) / kStep + 4 * TPW - 1) / (4 * TPW);
}

template <int TPW>
__host__ __device__ constexpr int corr_items(int H, int W) {
  return ((H + kStep - 1) / kStep + 3) / 4 * corr_col_items<TPW>(W);
}

// MFMA operand of the block whose top-left pixel is at plane (row, col):
// rows 2g, 2g + 1 of the block, 8 bytes each, for the h and l planes (byte j
// of the 16 <-> k = 16 g + j, block pixel (2g + j / 8, j % 8); the same map
// for both operands).
template <typename G>
__device__ __forceinline__ void load_operand(const unsigned char* planes, int row, int col, int g, i32x4& oh,
                                             i32x4& ol) {
  if constexpr (G::kNC == 4) {
    // copy c holds pixel column x + c at byte x
    const unsigned char* p = planes + (col & 3) * G::kCopy + (row + 2 * g) * G::kPitch + (col & ~3);
    const unsigned* h0 = reinterpret_cast<const unsigned*>(p);
    const unsigned* l0 = reinterpret_cast<const unsigned*>(p + G::kPlane);
    oh = i32x4{static_cast<int>(h0[0]), static_cast<int>(h0[1]), static_cast<int>(h0[G::kPitch / 4]),
               static_cast<int>(h0[G::kPitch / 4 + 1])};
    ol = i32x4{static_cast<int>(l0[0]), static_cast<int>(l0[1]), static_cast<int>(l0[G::kPitch / 4]),
               static_cast<int>(l0[G::kPitch / 4 + 1])};
  } else {
    // one copy: realign 8 bytes from three dwords
    auto seg8 = [&](const unsigned char* plane, int r, int& w0, int& w1) {
      const unsigned* p = reinterpret_cast<const unsigned*>(plane + r * G::kPitch + (col & ~3));
      const unsigned d0 = p[0], d1 = p[1], d2 = p[2];
      const unsigned sh = static_cast<unsigned>(col & 3);
      w0 = static_cast<int>(__builtin_amdgcn_alignbyte(d1, d0, sh));
      w1 = static_cast<int>(__builtin_amdgcn_alignbyte(d2, d1, sh));
    };
    int a0, a1, a2, a3;
    seg8(planes, row + 2 * g, a0, a1);
    seg8(planes, row + 2 * g + 1, a2, a3);
    oh = i32x4{a0, a1, a2, a3};
    seg8(planes + G::kPlane, row + 2 * g, a0, a1);
    seg8(planes + G::kPlane, row + 2 * g + 1, a2, a3);
    ol = i32x4{a0, a1, a2, a3};
  }
}

// Workgroup prologue: stages the pixels of the union of its tiles' windows,
// rows 3 p0 - R + [0, 4 nb + 7) and columns 3 q0 - R + [0, kZCols)
// (periodic), as byte planes, and the exact block norm of every candidate
// position (y, x) < (4 nb, kCandCols) as -nh (int32) and nl (u16),
// N = 512 nh + nl.  Every loop has a fixed trip count so that its loads are
// all in flight together.
template <int K, int TPW, int SPLIT>
__device__ __forceinline__ void stage_window(unsigned char* smem, const uint16_t* __restrict__ img, int H, int W,
                                             int R, int nb, int p0, int q0) {
  using Sm = Smem<K, TPW, SPLIT>;
  using G = typename Sm::G;
  constexpr int kWaves = TPW * SPLIT;
  constexpr int kZRowsPerWave = (kPixRows + kWaves - 1) / kWaves;
  static_assert(G::kZCols <= 2 * kWave, "two pixel columns per lane");
  const int rows = 4 * nb + 7;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = wave_id();
  uint16_t* zt = reinterpret_cast<uint16_t*>(smem + Sm::kNh);
  // pixels: wave w takes rows w, w + kWaves, ...; lane l columns l and l + 64.
  // Raw buffer loads over the image: the row offset is scalar, the column
  // offset a per-lane constant, and an offset past the image reads 0.
  {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t*>(img), 0, static_cast<int>(static_cast<unsigned>(H) * W * 2u), 0x00020000);
    const int y0 = kStep * p0 - R, x0 = kStep * q0 - R;
    int xo[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) xo[h] = 2 * pmod(x0 + lane + kWave * h, W);
    uint16_t v[kZRowsPerWave][2];
#pragma unroll
    for (int i = 0; i < kZRowsPerWave; ++i) {
      const int r = wave + kWaves * i;
      const int so = 2 * W * pmod(y0 + r, H);  // wave-uniform
#pragma unroll
      for (int h = 0; h < 2; ++h) v[i][h] = __builtin_amdgcn_raw_buffer_load_b16(rs, xo[h], so, 0);
    }
#pragma unroll
    for (int i = 0; i < kZRowsPerWave; ++i) {
      const int r = wave + kWaves * i;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int c = lane + kWave * h;
        if (r < rows && c < G::kZCols) zt[r * G::kZCols + c] = v[i][h];
      }
    }
  }
  __syncthreads();
  // byte planes: copy k, dword w of row r holds the h (l) bytes, xor 0x80,
  // of pixel columns 4 w + k + (0..3), cut out of the 8 pixels 4 w .. 4 w + 7
  constexpr int kWords = G::kPitch / 4;
  for (int i = threadIdx.x; i < rows * kWords; i += blockDim.x) {
    const int r = i / kWords, w = i - r * kWords;
    const uint2* zp = reinterpret_cast<const uint2*>(zt + r * G::kZCols + 4 * w);
    const uint2 e01 = zp[0], e23 = zp[1];
    const unsigned h0 = __builtin_amdgcn_perm(e01.y, e01.x, 0x07050301u) ^ 0x80808080u;
    const unsigned l0 = __builtin_amdgcn_perm(e01.y, e01.x, 0x06040200u) ^ 0x80808080u;
    unsigned char* cp = smem + r * G::kPitch + 4 * w;
    *reinterpret_cast<unsigned*>(cp) = h0;
    *reinterpret_cast<unsigned*>(cp + G::kPlane) = l0;
    if constexpr (G::kNC == 4) {
      const unsigned h1 = __builtin_amdgcn_perm(e23.y, e23.x, 0x07050301u) ^ 0x80808080u;
      const unsigned l1 = __builtin_amdgcn_perm(e23.y, e23.x, 0x06040200u) ^ 0x80808080u;
#pragma unroll
      for (int k = 1; k < 4; ++k) {
        *reinterpret_cast<unsigned*>(cp + k * G::kCopy) = __builtin_amdgcn_alignbyte(h1, h0, k);
        *reinterpret_cast<unsigned*>(cp + k * G::kCopy + G::kPlane) = __builtin_amdgcn_alignbyte(l1, l0, k);
      }
    }
  }
  // column sums of squares over 8 rows, exact in float64: cs[y][c] for
  // y < 4 nb, c < kCandCols + 7, in chunks of 12 rows per work item
  constexpr int kCsCols = G::kCandCols + 7;
  constexpr int kChunk = 12;
  double* cs = reinterpret_cast<double*>(smem + Sm::kDyn);
  const int ny = 4 * nb, nchunk = (ny + kChunk - 1) / kChunk;
  for (int i = threadIdx.x; i < nchunk * kCsCols; i += blockDim.x) {
    const int ch = i / kCsCols, c = i - ch * kCsCols;
    const int ya = kChunk * ch;
    double q[kChunk + 7];
#pragma unroll
    for (int a = 0; a < kChunk + 7; ++a) {
      // rows past the staged ones (a chunk that ends early) read row 0: unused
      const int r = ya + a < rows ? ya + a : 0;
      const double z = static_cast<double>(static_cast<int>(zt[r * G::kZCols + c]) - kZShift);
      q[a] = z * z;  // below 2^31: exact
    }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) s += q[a];
#pragma unroll
    for (int y = 0; y < kChunk; ++y) {
      if (y > 0) s += q[y + 7] - q[y - 1];
      if (ya + y < ny) cs[(ya + y) * kCsCols + c] = s;
    }
  }
  __syncthreads();  // pixels and column sums complete; the pixel stage dies
  // row sums of 8 column sums: the block norms, N < 2^37, exact
  int* nhn = reinterpret_cast<int*>(smem + Sm::kNh);
  uint16_t* nlo = reinterpret_cast<uint16_t*>(smem + Sm::kNl);
  constexpr int nxc = (G::kCandCols + kChunk - 1) / kChunk;
  for (int i = threadIdx.x; i < ny * nxc; i += blockDim.x) {
    const int y = i / nxc, ch = i - y * nxc;
    const int xa = kChunk * ch;
    const double* row = cs + y * kCsCols + xa;
    double q[kChunk + 7];
#pragma unroll
    for (int b = 0; b < kChunk + 7; ++b) q[b] = xa + b < kCsCols ? row[b] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 8; ++b) s += q[b];
#pragma unroll
    for (int x = 0; x < kChunk; ++x) {
      if (x > 0) s += q[x + 7] - q[x - 1];
      if (xa + x < G::kCandCols) {
        const double qq = floor(s * (1.0 / 512.0));
        nhn[y * G::kCandCols + xa + x] = -static_cast<int>(qq);
        nlo[y * G::kCandCols + xa + x] = static_cast<uint16_t>(static_cast<int>(fma(-512.0, qq, s)));
      }
    }
  }
  __syncthreads();  // norms complete; the column sums die
}

// One work item: reference rows [4 pb, 4 pb + 4) x columns [4 TPW qb, 4 TPW (qb + 1)).
template <int K, int TPW, int SPLIT>
__device__ __forceinline__ void corr_body(unsigned char* smem, const uint16_t* __restrict__ img,
                                          int16_t* __restrict__ idx, int H, int W, int R, int item) {
  using Sm = Smem<K, TPW, SPLIT>;
  using G = typename Sm::G;
  using C = Cfg<K, TPW, SPLIT>;
  constexpr int L = K - 1;
  constexpr int KB = C::kBuf;

  const int nRy = (H + kStep - 1) / kStep, nRx = (W + kStep - 1) / kStep;
  const int S = 2 * R + 1;
  const int nb = (2 * R + 10 + 3) / 4;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = wave_id();
  const int t = wave / SPLIT, part = wave % SPLIT;
  const int g = lane >> 4, n = lane & 15;
  const int u = n >> 2, v = n & 3;
  const int segs = corr_col_items<TPW>(W);
  const int p0 = (item / segs) * 4;
  const int q0 = (item % segs) * 4 * TPW;
  const int qt = q0 + 4 * t;  // first reference column of this wave's tile

  stage_window<K, TPW, SPLIT>(smem, img, H, W, R, nb, p0, q0);
  const unsigned char* planes = smem;
  const int* nhn = reinterpret_cast<const int*>(smem + Sm::kNh);
  const uint16_t* nlo = reinterpret_cast<const uint16_t*>(smem + Sm::kNl);
  unsigned long long* buf = reinterpret_cast<unsigned long long*>(smem + Sm::kDyn);
  unsigned long long* bound = buf + C::kWaves * KB * kWave;
  if constexpr (SPLIT > 1) {
    bound[threadIdx.x] = __double_as_longlong(kInf);
    bound[blockDim.x + threadIdx.x] = __double_as_longlong(kInf);
    __syncthreads();
  }

  // this lane's reference (p0 + u, qt + v): operand rows 2g, 2g + 1, and norm
  i32x4 rh, rl;
  load_operand<G>(planes, R + 3 * u, R + 12 * t + 3 * v, g, rh, rl);
  const int ra = (R + 3 * u) * G::kCandCols + R + 12 * t + 3 * v;
  const double na = fma(-512.0, static_cast<double>(nhn[ra]), static_cast<double>(nlo[ra]));  // N(a)
  const double na2048 = 2048.0 * na;

  double list[L];
#pragma unroll
  for (int i = 0; i < L; ++i) list[i] = kInf;
  // pre-test: Y = 65536 yh + yl, the high part as an accumulator input
  i32x4 yhv = {0, 0, 0, 0};
  int yh = 0, yl = 0;
  int cnt = 0;
  unsigned long long* mybuf = buf + wave * KB * kWave + lane;
  const int r_center = R * S + R;

  // the bounds over the 4 SPLIT lists of this reference (a published value
  // may be stale: lists only improve, so it stays a valid bound), and the
  // pre-test threshold they give
  constexpr int M = (L + 4 * SPLIT - 1) / (4 * SPLIT);
  auto publish = [&](auto exact) {
    double b1 = fmin(list[L - 1], shfl_xor_double(list[L - 1], 16));
    b1 = fmin(b1, shfl_xor_double(b1, 32));
    double b2 = fmax(list[M - 1], shfl_xor_double(list[M - 1], 16));
    b2 = fmax(b2, shfl_xor_double(b2, 32));
    if constexpr (decltype(exact)::value) {
      // the (K-1)-th best of the union of the wave's four lists of this reference
      double tmp[L];
#pragma unroll
      for (int i = 0; i < L; ++i) tmp[i] = list[i];
      merge_sorted<L>(tmp, [&](int j) { return shfl_xor_double(tmp[j], 16); });
      merge_sorted<L>(tmp, [&](int j) { return shfl_xor_double(tmp[j], 32); });
      b1 = fmin(b1, tmp[L - 1]);
    }
    if constexpr (SPLIT > 1) {
      unsigned long long* bmax = bound + C::kWaves * kWave;
      __hip_atomic_store(bound + wave * kWave + lane, static_cast<unsigned long long>(__double_as_longlong(b1)),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __hip_atomic_store(bmax + wave * kWave + lane, static_cast<unsigned long long>(__double_as_longlong(b2)),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
      for (int s2 = 0; s2 < SPLIT; ++s2) {
        const int o = (t * SPLIT + s2) * kWave + lane;
        b1 = fmin(b1, __longlong_as_double(static_cast<long long>(
                          __hip_atomic_load(bound + o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))));
        b2 = fmax(b2, __longlong_as_double(static_cast<long long>(
                          __hip_atomic_load(bmax + o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))));
      }
    }
    const double thr = fmin(b1, b2);
    // Y = floor((N(a) - ceil(thr / 2048)) / 2), every term an exact integer
    // in [-2^38, 2^36]; an infinite bound takes Y = -2^38, which passes
    // every pair
    const double dthr = ceil(thr * (1.0 / 2048.0));
    const double y = thr < kInf ? floor((na - dthr) * 0.5) : -274877906944.0;
    const double yhd = floor(fmax(y, -274877906944.0) * (1.0 / 65536.0));
    yh = static_cast<int>(yhd);
    yl = static_cast<int>(fma(-65536.0, yhd, fmax(y, -274877906944.0)));
    yhv = i32x4{-yh, -yh, -yh, -yh};
  };

  if (qt < nRx) {
    const int nblk = nb * nb;
    const int cbase = 12 * t;  // this tile's first candidate column in the workgroup's union
    struct Products {
      i32x4 hh, cc, ll;  // Phh - Yh (Yh of the lane's bound when issued), Phl + Plh - nh, Pll
      int yh;
      int br, bc;
    };
    // per-lane parts of the operand and norm addresses (candidate m = n ->
    // block row n / 4, column n % 4; rows 2g, 2g + 1 of it), so that a block
    // adds only a wave-uniform offset
    const unsigned char* cand_lane =
        planes + (G::kNC == 4 ? (n & 3) * G::kCopy : 0) + ((n >> 2) + 2 * g) * G::kPitch + cbase;
    const int* nh_lane = nhn + g * G::kCandCols + cbase;
    // A block's operand words (read from LDS) and its three products, the
    // cross term started at -nh of each candidate.  The walk below issues a
    // block's products one block before they are tested.
    struct Words {
      unsigned h[G::kNC == 4 ? 4 : 6], l[G::kNC == 4 ? 4 : 6];
      i32x4 nh;
      int br, bc;
    };
    auto words_of = [&](int b) {
      Words w;
      w.br = b >> 4;
      w.bc = b & 15;
      const unsigned char* pc = cand_lane + 4 * w.br * G::kPitch + 4 * w.bc;
      const unsigned* h0 = reinterpret_cast<const unsigned*>(pc);
      const unsigned* l0 = reinterpret_cast<const unsigned*>(pc + G::kPlane);
      if constexpr (G::kNC == 4) {
        // rows 2g and 2g + 1, 8 aligned bytes each
        w.h[0] = h0[0], w.h[1] = h0[1], w.h[2] = h0[G::kPitch / 4], w.h[3] = h0[G::kPitch / 4 + 1];
        w.l[0] = l0[0], w.l[1] = l0[1], w.l[2] = l0[G::kPitch / 4], w.l[3] = l0[G::kPitch / 4 + 1];
      } else {
        // one copy: three dwords per row, realigned when the products are formed
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          w.h[k] = h0[k], w.h[3 + k] = h0[G::kPitch / 4 + k];
          w.l[k] = l0[k], w.l[3 + k] = l0[G::kPitch / 4 + k];
        }
      }
      w.nh = *reinterpret_cast<const i32x4*>(nh_lane + 4 * w.br * G::kCandCols + 4 * w.bc);
      return w;
    };
    auto products_of_words = [&](const Words& w) {
      Products o;
      o.yh = yh;
      o.br = w.br;
      o.bc = w.bc;
      i32x4 ch, cl;
      if constexpr (G::kNC == 4) {
        ch = i32x4{static_cast<int>(w.h[0]), static_cast<int>(w.h[1]), static_cast<int>(w.h[2]),
                   static_cast<int>(w.h[3])};
        cl = i32x4{static_cast<int>(w.l[0]), static_cast<int>(w.l[1]), static_cast<int>(w.l[2]),
                   static_cast<int>(w.l[3])};
      } else {
        // shifted by the candidate's column in its block
        const unsigned sh = static_cast<unsigned>(n & 3);
        auto al = [&](unsigned hi, unsigned lo) { return static_cast<int>(__builtin_amdgcn_alignbyte(hi, lo, sh)); };
        ch = i32x4{al(w.h[1], w.h[0]), al(w.h[2], w.h[1]), al(w.h[4], w.h[3]), al(w.h[5], w.h[4])};
        cl = i32x4{al(w.l[1], w.l[0]), al(w.l[2], w.l[1]), al(w.l[4], w.l[3]), al(w.l[5], w.l[4])};
      }
      const i32x4 zero = {0, 0, 0, 0};
      o.hh = __builtin_amdgcn_mfma_i32_16x16x64_i8(ch, rh, yhv, 0, 0, 0);  // Phh - Yh
      i32x4 cc = __builtin_amdgcn_mfma_i32_16x16x64_i8(ch, rl, w.nh, 0, 0, 0);
      o.cc = __builtin_amdgcn_mfma_i32_16x16x64_i8(cl, rh, cc, 0, 0, 0);
      o.ll = __builtin_amdgcn_mfma_i32_16x16x64_i8(cl, rl, zero, 0, 0, 0);
      return o;
    };
    auto products = [&](int j) { return products_of_words(words_of(kOrder.b[nb][j])); };
    // exact key of reference (u, v) against candidate (cy, cx) of the tile's
    // union, or +inf outside its window or for the reference itself
    auto exact_key = [&](int sp, int ll, int cy, int cx, int nl) {
      const int ey = cy - 3 * u, ex = cx - 3 * v;  // dy + R, dx + R
      const bool ok = (static_cast<unsigned>(ey) <= static_cast<unsigned>(2 * R)) &
                      (static_cast<unsigned>(ex) <= static_cast<unsigned>(2 * R)) & !((ey == R) & (ex == R));
      // 2048 (N(a) + nl) + rank - 2^20 s' - 2^12 Pll
      const double c = na2048 + static_cast<double>(nl * 2048 + ey * S + ex);
      const double key = fma(-1048576.0, static_cast<double>(sp), fma(-4096.0, static_cast<double>(ll), c));
      return ok ? key : kInf;
    };

    // first blocks: exact keys of every pair, sorted in batches into the lists
    constexpr int BB = kBatchBlocks<K>;
    constexpr int kDense = kDenseBlocks<K>;
#pragma unroll 1
    for (int d0 = 0; d0 < kDense; d0 += BB) {
      double keys[4 * BB];
#pragma unroll
      for (int bb = 0; bb < BB; ++bb) {
        const int j = part + SPLIT * (d0 + bb);
        if (j < nblk) {
          const Products o = products(j);
          const int cy = 4 * o.br + g;
          const uint2 nl2 = *reinterpret_cast<const uint2*>(nlo + cy * G::kCandCols + cbase + 4 * o.bc);
          const int nl4[4] = {static_cast<int>(nl2.x & 0xFFFFu), static_cast<int>(nl2.x >> 16),
                              static_cast<int>(nl2.y & 0xFFFFu), static_cast<int>(nl2.y >> 16)};
#pragma unroll
          for (int i = 0; i < 4; ++i)
            keys[4 * bb + i] = exact_key((o.hh[i] + o.yh) * 256 + o.cc[i], o.ll[i], cy, 4 * o.bc + i, nl4[i]);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) keys[4 * bb + i] = kInf;
        }
      }
      bitonic_sort<4 * BB>(keys);
      merge_sorted<L>(list, [&](int j) { return j < 4 * BB ? keys[j] : kInf; });
    }
    publish(std::true_type{});

    // parked pairs -> exact keys -> list; every slot's loads are issued
    // before any is used (a slot this lane has not filled decodes as an
    // in-range position and yields +inf)
    auto flush = [&]() {
      constexpr int P = pow2_ceil(KB);
      unsigned long long w[KB];
#pragma unroll
      for (int e = 0; e < KB; ++e) w[e] = mybuf[e * kWave];
      int nlv[KB];
#pragma unroll
      for (int e = 0; e < KB; ++e) {
        if (e >= cnt) w[e] = 0ull;
        const int w1 = static_cast<int>(w[e] >> 32);
        const int cy = 4 * ((w1 >> 4) & 15) + g, cx = 4 * (w1 & 15) + ((w1 >> 8) & 3);
        nlv[e] = nlo[cy * G::kCandCols + cbase + cx];
      }
      double b[P];
#pragma unroll
      for (int e = 0; e < P; ++e) {
        if (e < KB) {
          const int w0 = static_cast<int>(static_cast<unsigned>(w[e])), w1 = static_cast<int>(w[e] >> 32);
          const int cy = 4 * ((w1 >> 4) & 15) + g, cx = 4 * (w1 & 15) + ((w1 >> 8) & 3);
          const double key = exact_key(w0 + 256 * yh, w1 >> 10, cy, cx, nlv[e]);
          b[e] = e < cnt ? key : kInf;
        } else {
          b[e] = kInf;
        }
      }
      bitonic_sort<P>(b);
      merge_sorted<L>(list, [&](int j) { return j < P ? b[j] : kInf; });
      cnt = 0;
      publish(std::false_type{});
    };

    // the rest: an integer pre-test per pair, raw parking of the survivors;
    // the next block's operand reads and products are issued before this
    // block's tests, and again after a merge, which moves the bound
    auto park = [&](const Products& o) {
      const int ey = 4 * o.br + g - 3 * u;
      // a lane whose window misses the block's row parks nothing (the block's
      // products were issued under the current bound: see the walk below)
      const int ylb = static_cast<unsigned>(ey) <= static_cast<unsigned>(2 * R) ? yl : 2147483647;
      const unsigned pos = static_cast<unsigned>(o.br << 4 | o.bc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = o.hh[i] * 256 + o.cc[i];  // s' - 256 Yh
        const int cl = c < -8192 ? -8192 : (c > 8192 ? 8192 : c);
        if (cl * 256 + o.ll[i] > ylb) {
          // c as is (s' = c + 256 Yh: Yh stays until the next merge), and
          // Pll above the candidate's column in the block and the block's position
          const unsigned hi = (static_cast<unsigned>(o.ll[i]) << 10) | (static_cast<unsigned>(i) << 8) | pos;
          mybuf[cnt * kWave] = (static_cast<unsigned long long>(hi) << 32) | static_cast<unsigned>(c);
          ++cnt;
        }
      }
    };
    // (the order entry of the block after next is read one block early, so
    // that no scalar load latency precedes a block's operand reads)
    int j = part + SPLIT * kDense;
    if (j < nblk) {
      Products cur = products(j);
      int b1 = j + SPLIT < nblk ? kOrder.b[nb][j + SPLIT] : 0;
      for (; j + SPLIT < nblk; j += SPLIT) {
        const int b2 = j + 2 * SPLIT < nblk ? kOrder.b[nb][j + 2 * SPLIT] : 0;
        Products nxt = products_of_words(words_of(b1));
        park(cur);
        if (wave_any(cnt > C::kFlushAt)) {
          flush();
          nxt = products_of_words(words_of(b1));
        }
        cur = nxt;
        b1 = b2;
      }
      park(cur);
    }
    if (wave_any(cnt > 0)) flush();
  }

  // the four quarters of each reference, then the SPLIT waves of the tile
  merge_sorted<L>(list, [&](int j) { return shfl_xor_double(list[j], 16); });
  merge_sorted<L>(list, [&](int j) { return shfl_xor_double(list[j], 32); });
  if constexpr (SPLIT > 1) {
    __syncthreads();  // planes, norms, buffers and bounds are dead
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
      if (part == 1) put(t);
      __syncthreads();
      if (part == 0) take(t);
    } else {
      if (part & 1) put(2 * t + (part >> 1));
      __syncthreads();
      if (!(part & 1)) take(2 * t + (part >> 1));
      __syncthreads();
      if (part == 2) put(t);
      __syncthreads();
      if (part == 0) take(t);
    }
    if (part != 0) return;
  }

  const int p = p0 + u, q = qt + v;
  if (g == 0 && p < nRy && q < nRx) {
    int16_t* out = idx + (static_cast<size_t>(p) * nRx + q) * K;
    out[0] = static_cast<int16_t>(r_center);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      out[1 + i] = key_rank(list[i]);
    }
  }
}

template <int K, int TPW, int SPLIT, bool BATCH>
__global__ __launch_bounds__(TPW * SPLIT * 64, 2) void bm_corr_kernel(ImgRec one, WorkList wl, int R, int use_pilot) {
  __shared__ __align__(16) unsigned char smem[Smem<K, TPW, SPLIT>::bytes];
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) {
    corr_body<K, TPW, SPLIT>(smem, use_pilot ? r.pilot : r.noisy, r.idx, r.H, r.W, R, item);
  });
}

template <int K, int TPW, int SPLIT>
hipError_t launch_corr_shape(const ImgRec& one, const WorkList* wl, int R, int use_pilot, int grid_cap,
                             hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((bm_corr_kernel<K, TPW, SPLIT, false>), dim3(corr_items<TPW>(one.H, one.W)),
                       dim3(64 * TPW * SPLIT), 0, st,
                       one, WorkList{}, R, use_pilot);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((bm_corr_kernel<K, TPW, SPLIT, true>), dim3(std::min(wl->total, grid_cap)),
                       dim3(64 * TPW * SPLIT), 0, st,
                       one, *wl, R, use_pilot);
  }
  return hipGetLastError();
}

// Tiles per workgroup for a split: groups up to 16 share four tiles among
// eight waves when split (their lists are short enough for four waves per
// SIMD); groups of 32 keep four waves per workgroup.
__host__ __device__ constexpr int corr_tpw(int K, int split) {
  return split == 1 ? 4 : (K <= 16 ? 8 / split : 4 / split);
}

template <int K>
hipError_t launch_corr_k(const ImgRec& one, const WorkList* wl, int R, int split, int use_pilot, int grid_cap,
                         hipStream_t st) {
  switch (split) {
    case 1: return launch_corr_shape<K, 4, 1>(one, wl, R, use_pilot, grid_cap, st);
    case 2: return launch_corr_shape<K, corr_tpw(K, 2), 2>(one, wl, R, use_pilot, grid_cap, st);
    case 4: return launch_corr_shape<K, corr_tpw(K, 4), 4>(one, wl, R, use_pilot, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int corr_items_for(int H, int W, int K, int split) {
  switch (corr_tpw(K, split)) {
    case 4: return corr_items<4>(H, W);
    case 2: return corr_items<2>(H, W);
    default: return corr_items<1>(H, W);
  }
}

long corr_tiles(int H, int W) { return static_cast<long>(corr_items<1>(H, W)); }

int corr_auto_split(long tiles) { return tiles >= 4096 ? 1 : (tiles >= 2048 ? 2 : 4); }

hipError_t launch_bm_corr(const ImgRec& one, const WorkList* wl, int R, int K, int split, int use_pilot, int grid_cap,
                          hipStream_t st) {
  if (split <= 0) split = corr_auto_split(corr_tiles(one.H, one.W));
  switch (K) {
    case 2: return launch_corr_k<2>(one, wl, R, split, use_pilot, grid_cap, st);
    case 4: return launch_corr_k<4>(one, wl, R, split, use_pilot, grid_cap, st);
    case 8: return launch_corr_k<8>(one, wl, R, split, use_pilot, grid_cap, st);
    case 16: return launch_corr_k<16>(one, wl, R, split, use_pilot, grid_cap, st);
    case 32: return launch_corr_k<32>(one, wl, R, split, use_pilot, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gbm3d
