// Block matching in the correlation form of Theorem 1 (Sec. 2), on the
// matrix cores.  Same result as the shift-wise kernel: for every reference the
// K-1 smallest keys dist * 2048 + rank over the search window, reference in
// slot 0.
//
// ||a - b||^2 = N(a) + N(b) - 2 <a, b>, with N the block's squared norm.  The
// distance is translation invariant, so pixels are first shifted by 32896:
// z = Z - 32896 = 256 h + l with signed bytes h = (Z >> 8) - 128 and
// l = (Z & 255) - 128.  Then <a, b> = 65536 Phh + 256 (Phl + Plh) + Pll, four
// exact int8 x int8 -> int32 dot products of length 64, which is one
// v_mfma_i32_16x16x64_i8 each for 16 candidates x 16 references.
//
// A wave owns a 4 x 4 tile of references (step 3); the union of their search
// windows is a (2R + 10)^2 square of candidate positions, walked in 4 x 4
// candidate blocks from the centre outwards.  Result lane (g, n) holds
// reference n and candidates (row g, columns 0..3) of the block.  Every pair
// gets its exact key 2048 (N(a) + N(b) - 512 (256 Phh + Phl + Plh) - 2 Pll) +
// rank in float64 (all terms integers below 2^50) with no data-dependent
// branch, held less a constant of its reference (two FMAs on the table
// entry); keys below the lane's bound go to its candidate buffer.  Norms come
// from a table written beforehand (norm.h; float64, exact) by bm_norm_kernel
// or, for a single image, by the stack launch of the same stage.
//
// Every lane keeps the K-1 best keys of its reference among its quarter of
// the candidates; the four quarters, and the SPLIT waves that share a tile,
// share two upper bounds on the (K-1)-th best key seen so far for the
// reference: the smallest worst kept key of any list, and the largest m-th
// best of any list, where m lists-worth of keys make K-1 (n lists each with m
// keys at or below a value hold n m >= K-1 of them).  Keys are unique, so a
// key at or above either bound cannot be among the K-1 best.  The lists merge
// with bitonic networks at the end.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "norm.h"
#include "topk.h"

namespace gbm3d {

namespace {

constexpr int kPitch = 96;                         // bytes per LDS plane row
constexpr int kMaxNb = (2 * kMaxR + 10 + 3) / 4;   // candidate blocks per axis
constexpr int kRows = 4 * kMaxNb + 7;              // LDS plane rows
// Buffered candidates per lane before a merge into the list.  A merge runs
// when any lane of the wave might overflow, so a deeper buffer makes merges
// rarer; the depth is what the LDS allows at the occupancy the registers
// already set (four waves per SIMD for K <= 16, three for K = 32).
template <int K>
constexpr int kBuf = K >= 32 ? 16 : K >= 16 ? 12 : 8;
template <int K>
constexpr int kFlushAt = kBuf<K> - 4;  // a block appends at most 4
constexpr double kInf = __builtin_huge_val();

// an address in LDS, 32 bits wide
typedef __attribute__((address_space(3))) double lds_double;

// Keeps p in its register as it stands (the compiler would otherwise rebuild
// it from the buffer base and an offset at every use).
__device__ __forceinline__ void pin(lds_double*& p) { asm("" : "+v"(p)); }

static_assert(12 * 3 + 4 * kMaxNb + 12 <= kPitch, "plane rows too short");

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Candidate blocks of an nb x nb grid in rings of growing Chebyshev distance
// from its centre (near displacements first tighten the bounds early), each
// entry the block's (row << 8) | column, so no division by the run-time nb is
// left in the walk.
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
        if ((dr > dc ? dr : dc) == ring) o.b[nb][n++] = (b / nb) << 8 | (b % nb);
      }
  }
  return o;
}

__constant__ BlockOrder kOrder = make_block_order();


template <bool BATCH>
__global__ __launch_bounds__(256) void bm_norm_kernel(ImgRec one, WorkList wl, int R, int use_pilot) {
  __shared__ __align__(16) unsigned char smem[NormSmem::bytes];
  int* zt = reinterpret_cast<int*>(smem);
  double* hs = reinterpret_cast<double*>(smem + NormSmem::zt_bytes);
  for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) {
    norm_body<false>(use_pilot ? r.pilot : r.noisy, r.norm, r.H, r.W, R, item, zt, hs);
  });
}

// ---------------------------------------------------------------------------
// matching
// ---------------------------------------------------------------------------

template <int K, int TPW, int SPLIT>
struct CorrSmem {
  static constexpr int L = K - 1;
  static constexpr size_t kPlanes = 2 * kRows * kPitch;
  static constexpr size_t kBufBytes = sizeof(double) * 4 * kBuf<K> * kWave;
  static constexpr size_t kBound = SPLIT > 1 ? sizeof(double) * 2 * 4 * kWave : 0;
  static constexpr size_t kScan = kPlanes + kBufBytes + kBound;
  static constexpr size_t kMerge = SPLIT > 1 ? sizeof(double) * 2 * L * kWave : 0;
  static constexpr size_t bytes = kScan > kMerge ? kScan : kMerge;
};

template <int TPW>
__host__ __device__ constexpr int corr_col_items(int W) {
  return ((W + kStep - 1) / kStep + 4 * TPW - 1) / (4 * TPW);
}

template <int TPW>
__host__ __device__ constexpr int corr_items(int H, int W) {
  return ((H + kStep - 1) / kStep + 3) / 4 * corr_col_items<TPW>(W);
}

// 8 bytes of LDS plane row r from byte column x (any alignment) as 2 dwords
__device__ __forceinline__ void seg8(const unsigned char* plane, int r, int x, int& w0, int& w1) {
  const unsigned* p = reinterpret_cast<const unsigned*>(plane + r * kPitch + (x & ~3));
  const unsigned d0 = p[0], d1 = p[1], d2 = p[2];
  const unsigned sh = static_cast<unsigned>(x & 3);
  w0 = static_cast<int>(__builtin_amdgcn_alignbyte(d1, d0, sh));
  w1 = static_cast<int>(__builtin_amdgcn_alignbyte(d2, d1, sh));
}

// MFMA operand of the block at LDS (row, col): rows 2g, 2g + 1 of the block,
// 8 bytes each, for the h and l planes (byte j of the 16 <-> k = 16 g + j,
// block pixel (2g + j / 8, j % 8); the same map for both operands).
__device__ __forceinline__ void load_operand(const unsigned char* hp, const unsigned char* lp, int row, int col, int g,
                                             i32x4& oh, i32x4& ol) {
  int a0, a1, a2, a3;
  seg8(hp, row + 2 * g, col, a0, a1);
  seg8(hp, row + 2 * g + 1, col, a2, a3);
  oh = i32x4{a0, a1, a2, a3};
  seg8(lp, row + 2 * g, col, a0, a1);
  seg8(lp, row + 2 * g + 1, col, a2, a3);
  ol = i32x4{a0, a1, a2, a3};
}

// One work item: reference rows [4 pb, 4 pb + 4) x columns [4 TPW qb, 4 TPW (qb + 1)).
template <int K, int TPW, int SPLIT>
__device__ __forceinline__ void corr_body(unsigned char* smem, const uint16_t* __restrict__ img_,
                                          const double* __restrict__ norm_, int16_t* __restrict__ idx_, int H, int W,
                                          int R, int item) {
  const auto img = to_global(img_);
  const auto norm = to_global(norm_);
  const auto idx = to_global(idx_);
  static_assert(TPW * SPLIT == 4, "four waves per workgroup");
  using Smem = CorrSmem<K, TPW, SPLIT>;
  constexpr int L = K - 1;
  unsigned char* hp = smem;
  unsigned char* lp = smem + kRows * kPitch;
  double* buf = reinterpret_cast<double*>(smem + Smem::kPlanes);
  unsigned long long* bound = reinterpret_cast<unsigned long long*>(smem + Smem::kPlanes + Smem::kBufBytes);

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

  // LDS planes of the image region rows 3 p0 - R + [0, 4 nb + 7), columns 3 q0 - R + [0, kPitch)
  const int y0 = kStep * p0 - R, x0 = kStep * q0 - R;
  const int rows = 4 * nb + 7;
  // y0 < H and x0 < W: rows and columns wrap at most once when the image
  // is at least as tall as the region and as wide as a plane row
  const bool near = H >= rows && W >= kPitch;
  // the reference's norm-table entry, loaded ahead of the fill (from an
  // in-bounds column also for a tile right of the last reference column,
  // whose value is not used)
  const int We = norm_pitch(W);
  const int cr = kStep * (qt + v) + kNormPad;
  const double nref = norm[static_cast<size_t>(kStep * (p0 + u) + kNormPad) * We + min(cr, We - 1)];
  // every thread's pixel loads are issued before the first is used: one
  // memory round trip for the whole fill instead of one per item
  constexpr int kFillThreads = 256;
  constexpr int kFillIter = (kRows * (kPitch / 4) + kFillThreads - 1) / kFillThreads;
  const int n_fill = rows * (kPitch / 4);
  unsigned zv[kFillIter][4];
#pragma unroll
  for (int it = 0; it < kFillIter; ++it) {
    const int i = static_cast<int>(threadIdx.x) + it * kFillThreads;
    if (i < n_fill) {
      const int r = i / (kPitch / 4), c = (i - r * (kPitch / 4)) * 4;
      int y = y0 + r, xb = x0 + c;
      if (near) {
        y += y < 0 ? H : (y >= H ? -H : 0);
        xb += xb < 0 ? W : (xb >= W ? -W : 0);
      } else {
        y = pmod(y, H);
        xb = pmod(xb, W);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = xb + j < W ? xb + j : xb + j - W;  // W >= 8 > j
        zv[it][j] = img[static_cast<size_t>(y) * W + x];
      }
    }
  }
#pragma unroll
  for (int it = 0; it < kFillIter; ++it) {
    const int i = static_cast<int>(threadIdx.x) + it * kFillThreads;
    if (i < n_fill) {
      const int r = i / (kPitch / 4), c = (i - r * (kPitch / 4)) * 4;
      unsigned wh = 0, wl = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        wh |= ((zv[it][j] >> 8) ^ 0x80u) << (8 * j);
        wl |= ((zv[it][j] & 0xFFu) ^ 0x80u) << (8 * j);
      }
      reinterpret_cast<unsigned*>(hp + r * kPitch)[c / 4] = wh;
      reinterpret_cast<unsigned*>(lp + r * kPitch)[c / 4] = wl;
    }
  }
  if constexpr (SPLIT > 1) {
    bound[threadIdx.x] = __double_as_longlong(kInf);
    bound[blockDim.x + threadIdx.x] = __double_as_longlong(kInf);
  }
  __syncthreads();

  // this lane's reference (p0 + u, qt + v): operand rows 2g, 2g + 1, and norm
  i32x4 rh, rl;
  load_operand(hp, lp, R + 3 * u, R + 12 * t + 3 * v, g, rh, rl);
  // Keys are held less this lane's reference constant A = 2048 N(a) - F(a)
  // + R S + R, with F the position term of the norm table (its entry at the
  // reference is 2048 N(a) + F(a)): a candidate's key is then its table entry
  // less the correlation terms, and the four quarters and SPLIT waves that
  // compare or merge keys share the reference, so A is added only to the
  // final list (a tile right of the last reference column only takes part
  // in the merges)
  const int f_ref = (kStep * (p0 + u) + kNormPad) * S + cr;
  const double key_a = qt < nRx ? nref - static_cast<double>(2 * f_ref - R * S - R) : 0.0;
  // table entries of this lane's result candidates: block (br, bc) row g, columns 0..3
  const auto ncand = norm + static_cast<size_t>(y0 + g + kNormPad) * We + (x0 + 12 * t + kNormPad);

  double list[L];
#pragma unroll
  for (int i = 0; i < L; ++i) list[i] = kInf;
  double thr = kInf;  // no key at or above it can enter the list
  double* mybuf = buf + wave * kBuf<K> * kWave + lane;
  // this lane's next free buffer slot, an LDS address held in a register:
  // an append is one add and a store, and the compiler branches over the
  // appends that no lane makes
  lds_double* const buf0 = (lds_double*)(mybuf);
  lds_double* wp = buf0;
  pin(wp);
  const int r_center = R * S + R;

  // the two bounds over the 4 SPLIT lists of this reference (a published
  // value may be stale: lists only improve, so it stays a valid bound)
  constexpr int M = (L + 4 * SPLIT - 1) / (4 * SPLIT);
  auto publish = [&]() {
    double b1 = fmin(list[L - 1], shfl_xor_double(list[L - 1], 16));
    b1 = fmin(b1, shfl_xor_double(b1, 32));
    double b2 = fmax(list[M - 1], shfl_xor_double(list[M - 1], 16));
    b2 = fmax(b2, shfl_xor_double(b2, 32));
    if constexpr (SPLIT > 1) {
      unsigned long long* bmax = bound + 4 * kWave;
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
    thr = fmin(b1, b2);
  };
  auto flush = [&]() {
    merge_buffer<L, kBuf<K>>(list, mybuf, kWave, static_cast<int>(wp - buf0) / kWave);
    wp = buf0;
    pin(wp);
    publish();
  };

  if (qt < nRx) {
    const int nblk = nb * nb;
    // Block j of the walk: its entry in the walk order (row << 8 | column,
    // a scalar load), this lane's four candidate norms (global loads), its
    // operands (LDS) and its products (matrix cores).  Past the end of the
    // walk the last block's entry is read and what follows from it is never
    // used, so every load is unconditional and the wait before a block's use
    // covers its own loads only.
    auto order = [&](int j) { return kOrder.b[nb][j < nblk ? j : nblk - 1]; };
    auto load_norms = [&](int b, double (&nv)[4]) {
      const auto nc = ncand + static_cast<size_t>(4 * (b >> 8)) * We + 4 * (b & 255);
#pragma unroll
      for (int i = 0; i < 4; ++i) nv[i] = nc[i];
    };
    struct Ops {
      i32x4 ch, cl;
    };
    // operand: candidate m = n -> block row n / 4, column n % 4
    auto operands = [&](int b, Ops& o) {
      load_operand(hp, lp, 4 * (b >> 8) + (n >> 2), 12 * t + 4 * (b & 255) + (n & 3), g, o.ch, o.cl);
    };
    struct Prod {
      i32x4 hh, cc, ll;
    };
    // the block's four exact byte-plane products
    auto products = [&](const Ops& o, Prod& pr) {
      const i32x4 zero = {0, 0, 0, 0};
      pr.hh = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ch, rh, zero, 0, 0, 0);
      pr.cc = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.ch, rl, zero, 0, 0, 0);
      pr.cc = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.cl, rh, pr.cc, 0, 0, 0);
      pr.ll = __builtin_amdgcn_mfma_i32_16x16x64_i8(o.cl, rl, zero, 0, 0, 0);
    };
    // the block's keys from its norms and products
    auto keys_of = [&](int b, const double (&nv)[4], const Prod& pr, auto warm, double (&keys)[4]) {
      const int br = b >> 8, bc = b & 255;
      const i32x4 hh = pr.hh, cc = pr.cc, ll = pr.ll;
      // result lane (g, n): candidates (4 br + g, 4 bc + i) vs reference (3u, 3v), in window units
      const int ey = 4 * br + g - 3 * u;     // dy + R
      const int ex0 = 4 * bc - 3 * v;        // dx + R for i = 0
      const bool row_ok = static_cast<unsigned>(ey) <= static_cast<unsigned>(2 * R);
      // key = 2048 (N(a) + N(b) - 512 s - 2 Pll) + rank, held less A: the
      // table entry 2048 N(b) + F(b) less the correlation terms, every
      // intermediate an integer below 2^50 in magnitude
      // the reference itself (dy = dx = 0) is candidate ic of this block in at most a few lanes
      const int ic = R - ex0;
      const bool center_here = ey == R && static_cast<unsigned>(ic) < 4u;
      auto pairs = [&](auto check_center) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int s = hh[i] * 256 + cc[i];  // 256 Phh + Phl + Plh, |s| < 2^29
          const double key =
              fma(-1048576.0, static_cast<double>(s), fma(-4096.0, static_cast<double>(ll[i]), nv[i]));
          // (bitwise: no short-circuit branches)
          bool ok = row_ok & (static_cast<unsigned>(ex0 + i) <= static_cast<unsigned>(2 * R));
          if constexpr (decltype(check_center)::value) ok = ok & !(center_here & (i == ic));
          if constexpr (decltype(warm)::value) {
            keys[i] = ok ? key : kInf;
          } else if (ok & (key < thr)) {
            *wp = key;
            wp += kWave;
            pin(wp);
          }
        }
      };
      if (wave_any(center_here))
        pairs(std::true_type{});
      else
        pairs(std::false_type{});
      if constexpr (!decltype(warm)::value) {
        if (wave_any(wp > buf0 + kFlushAt<K> * kWave)) flush();
      }
    };
    // Warm start: the first kWarm blocks of this part give each lane four
    // candidates per block; sorted, they are its first list, and the lists
    // hold enough keys for a finite m-th-best bound at once.
    constexpr int kWarm = L < 16 ? 1 : 2;
    {
      double seed[4 * kWarm];
#pragma unroll
      for (int w = 0; w < kWarm; ++w) {
        double k4[4] = {kInf, kInf, kInf, kInf};
        const int jw = part + w * SPLIT;
        if (jw < nblk) {
          const int bw = order(jw);
          double nvw[4];
          Ops ow;
          Prod pw;
          load_norms(bw, nvw);
          operands(bw, ow);
          products(ow, pw);
          keys_of(bw, nvw, pw, std::true_type{}, k4);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) seed[4 * w + i] = k4[i];
      }
      bitonic_sort<4 * kWarm>(seed);
#pragma unroll
      for (int i = 0; i < L && i < 4 * kWarm; ++i) list[i] = seed[i];
      publish();
    }
    double unused[4];
    // Software pipeline over the rest of the walk, in steps of SPLIT blocks:
    // while block j's keys are formed, block j + 2 SPLIT's operands are read
    // from LDS, and its products and norms are issued right after, two steps
    // ahead of their use.  Two register sets of norms and products alternate.
    const int jb = part + kWarm * SPLIT;
    int b0 = order(jb), b1 = order(jb + SPLIT), b2 = order(jb + 2 * SPLIT);
    double nv0[4], nv1[4];
    Prod p0, p1;
    Ops op;
    // (issued in walk order: the waits in the loop count on the older loads
    // landing first)
    load_norms(b0, nv0);
    __builtin_amdgcn_sched_barrier(0);
    load_norms(b1, nv1);
    operands(b0, op);
    products(op, p0);
    operands(b1, op);
    products(op, p1);
    auto step = [&](int j, double (&nvc)[4], Prod& pc) {
      operands(b2, op);
      keys_of(b0, nvc, pc, std::false_type{}, unused);
      products(op, pc);
      load_norms(b2, nvc);
      b0 = b1;
      b1 = b2;
      b2 = order(j + 3 * SPLIT);
    };
    // whole pairs of steps in the loop and an odd last step after it: every
    // path into a step then comes from the step of the other register set,
    // whose loads are the younger ones the wait may leave in flight
    const int steps = jb < nblk ? (nblk - jb + SPLIT - 1) / SPLIT : 0;
    int j = jb;
#pragma unroll 1
    for (int s2 = 0; s2 + 1 < steps; s2 += 2, j += 2 * SPLIT) {
      step(j, nv0, p0);
      step(j + SPLIT, nv1, p1);
    }
    if (steps & 1) step(j, nv0, p0);
  }
  if (wave_any(wp != buf0)) flush();

  // the four quarters of each reference, then the SPLIT waves of the tile
  merge_sorted<L>(list, [&](int j) { return shfl_xor_double(list[j], 16); });
  merge_sorted<L>(list, [&](int j) { return shfl_xor_double(list[j], 32); });
  if constexpr (SPLIT > 1) {
    __syncthreads();  // planes, buffers and bounds are dead
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
      if (part & 1) put(part >> 1);
      __syncthreads();
      if (!(part & 1)) take(part >> 1);
      __syncthreads();
      if (part == 2) put(0);
      __syncthreads();
      if (part == 0) take(0);
    }
    if (part != 0) return;
  }

  const int p = p0 + u, q = qt + v;
  if (g == 0 && p < nRy && q < nRx) {
    const auto out = idx + (static_cast<size_t>(p) * nRx + q) * K;
    out[0] = static_cast<int16_t>(r_center);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      out[1 + i] = key_rank(list[i] + key_a);
    }
  }
}

// The second launch bound is the waves per SIMD that the registers must
// allow: what the LDS of a workgroup allows for K = 16 (four workgroups of
// four waves per CU) and K = 32 (three); smaller groups are held by neither.
template <int K>
constexpr int kCorrWaves = K == 16 ? 4 : K == 32 ? 3 : 2;

template <int K, int TPW, int SPLIT, bool BATCH>
__global__ __launch_bounds__(256, kCorrWaves<K>) void bm_corr_kernel(ImgRec one, WorkList wl, int R, int use_pilot) {
  __shared__ __align__(16) unsigned char smem[CorrSmem<K, TPW, SPLIT>::bytes];
  if constexpr (!BATCH) {
    // Workgroups go to the eight XCDs in turn (g -> XCD g mod 8): XCD x takes
    // the x-th eighth of the items, a band of reference rows, so each XCD's
    // L2 fetches its band's planes and norm-table rows instead of the whole
    // image.  The grid is 8 q; items past the last exit at once.
    const int n = corr_items<TPW>(one.H, one.W), q = (n + 7) / 8;
    const int g = static_cast<int>(blockIdx.x);
    const int item = (g & 7) * q + (g >> 3);
    if (item >= n) return;
    corr_body<K, TPW, SPLIT>(smem, use_pilot ? one.pilot : one.noisy, one.norm, one.idx, one.H, one.W, R, item);
  } else {
    for_each_item<BATCH>(one, wl, [&](const ImgRec& r, int item) {
      corr_body<K, TPW, SPLIT>(smem, use_pilot ? r.pilot : r.noisy, r.norm, r.idx, r.H, r.W, R, item);
    });
  }
}

template <int K, int TPW, int SPLIT>
hipError_t launch_corr_shape(const ImgRec& one, const WorkList* wl, int R, int use_pilot, int grid_cap,
                             hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((bm_corr_kernel<K, TPW, SPLIT, false>), dim3(8 * ((corr_items<TPW>(one.H, one.W) + 7) / 8)), dim3(256), 0, st,
                       one, WorkList{}, R, use_pilot);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((bm_corr_kernel<K, TPW, SPLIT, true>), dim3(std::min(wl->total, grid_cap)), dim3(256), 0, st,
                       one, *wl, R, use_pilot);
  }
  return hipGetLastError();
}

template <int K>
hipError_t launch_corr_k(const ImgRec& one, const WorkList* wl, int R, int split, int use_pilot, int grid_cap,
                         hipStream_t st) {
  switch (split) {
    case 1: return launch_corr_shape<K, 4, 1>(one, wl, R, use_pilot, grid_cap, st);
    case 2: return launch_corr_shape<K, 2, 2>(one, wl, R, use_pilot, grid_cap, st);
    case 4: return launch_corr_shape<K, 1, 4>(one, wl, R, use_pilot, grid_cap, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t norm_bytes(int H, int W) {
  return static_cast<size_t>(H + 2 * kNormPad) * (W + 2 * kNormPad) * sizeof(double);
}

int norm_items_for(int H, int W) { return norm_items(H, W); }

int corr_items_for(int H, int W, int split) {
  switch (split) {
    case 1: return corr_items<4>(H, W);
    case 2: return corr_items<2>(H, W);
    default: return corr_items<1>(H, W);
  }
}

long corr_tiles(int H, int W) { return static_cast<long>(corr_items<1>(H, W)); }

int corr_auto_split(long tiles) { return tiles >= 4096 ? 1 : (tiles >= 2048 ? 2 : 4); }

hipError_t launch_bm_norm(const ImgRec& one, const WorkList* wl, int R, int use_pilot, int grid_cap,
                          hipStream_t st) {
  if (!wl) {
    hipLaunchKernelGGL((bm_norm_kernel<false>), dim3(norm_items(one.H, one.W)), dim3(256), 0, st, one, WorkList{}, R,
                       use_pilot);
  } else {
    if (wl->total <= 0) return hipSuccess;
    hipLaunchKernelGGL((bm_norm_kernel<true>), dim3(std::min(wl->total, grid_cap)), dim3(256), 0, st, one, *wl, R,
                       use_pilot);
  }
  return hipGetLastError();
}

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
