// Device-side building blocks of the G-BM3D library: transform tables built at
// compile time from the filter definitions, and wavefront helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbm3d {

constexpr int kPatch = 8;
constexpr int kStep = 3;
constexpr int kMaxR = 19;  // largest search half-width (39 x 39 window)
constexpr int kWave = 64;

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// bior1.5 (Sec. 5): analysis low-pass taps at offsets -4..5 in units of
// sqrt(2)/256; the synthesis scaling filter is the Haar box.
// ---------------------------------------------------------------------------
constexpr int kBiorTap[10] = {3, -3, -22, 22, 128, 128, 22, -22, -3, 3};

struct Mat8 {
  double m[8][8];
};

constexpr int pmod(int a, int L) { return ((a % L) + L) % L; }

// One periodic analysis level on length L (even): rows 0..L/2-1 give the
// low-pass a[n] = sum_i h_i x[2n+i], rows L/2.. the Haar details
// d[n] = (x[2n+1] - x[2n]) / sqrt(2).
constexpr Mat8 bior_analysis(int L) {
  Mat8 A{};
  for (int n = 0; n < L / 2; ++n) {
    for (int i = 0; i < 10; ++i) A.m[n][pmod(2 * n + i - 4, L)] += kBiorTap[i] * kSqrt2 / 256.0;
    A.m[L / 2 + n][2 * n] += -kInvSqrt2;
    A.m[L / 2 + n][2 * n + 1] += kInvSqrt2;
  }
  return A;
}

// The matching periodic synthesis level (x = S c): a low coefficient spreads
// as the Haar box over (2n, 2n+1); a detail coefficient spreads as the dual
// wavelet psi[m] = (-1)^(m+1) h[1-m], m = -4..5 around 2n.
constexpr Mat8 bior_synthesis(int L) {
  Mat8 S{};
  for (int n = 0; n < L / 2; ++n) {
    S.m[2 * n][n] += kInvSqrt2;
    S.m[2 * n + 1][n] += kInvSqrt2;
    for (int m = -4; m <= 5; ++m) {
      const int t = 1 - m;  // tap offset of h
      if (t < -4 || t > 5) continue;
      const double sign = ((m + 1) & 1) ? -1.0 : 1.0;
      S.m[pmod(2 * n + m, L)][L / 2 + n] += sign * kBiorTap[t + 4] * kSqrt2 / 256.0;
    }
  }
  return S;
}

// ---------------------------------------------------------------------------
// Orthonormal DCT-II of length 8 (Sec. 4): C[k][n] = a_k cos(pi (2n+1) k / 16)
// ---------------------------------------------------------------------------
constexpr double ccos(double x) {
  while (x > kPi) x -= 2 * kPi;
  while (x < -kPi) x += 2 * kPi;
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 40; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}

constexpr Mat8 dct8() {
  Mat8 C{};
  for (int k = 0; k < 8; ++k)
    for (int n = 0; n < 8; ++n)
      C.m[k][n] = (k == 0 ? 0.35355339059327376220 : 0.5) * ccos(kPi * (2 * n + 1) * k / 16.0);
  return C;
}

constexpr Mat8 transpose8(const Mat8& A) {
  Mat8 T{};
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) T.m[i][j] = A.m[j][i];
  return T;
}

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// max |A S - I| over the leading L x L block
constexpr double inverse_error(const Mat8& A, const Mat8& S, int L) {
  double e = 0;
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      double s = 0;
      for (int k = 0; k < L; ++k) s += A.m[i][k] * S.m[k][j];
      const double d = cabs(s - (i == j ? 1.0 : 0.0));
      if (d > e) e = d;
    }
  return e;
}

static_assert(inverse_error(bior_analysis(2), bior_synthesis(2), 2) < 1e-14, "bior L=2");
static_assert(inverse_error(bior_analysis(4), bior_synthesis(4), 4) < 1e-14, "bior L=4");
static_assert(inverse_error(bior_analysis(8), bior_synthesis(8), 8) < 1e-14, "bior L=8");
static_assert(inverse_error(dct8(), transpose8(dct8()), 8) < 1e-14, "dct orthonormal");

// y = M x over the leading L x L block, float arithmetic, zero entries skipped
template <int L>
__device__ __forceinline__ void apply_mat(const Mat8& M, const float* x, float* y) {
#pragma unroll
  for (int i = 0; i < L; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < L; ++j)
      if (M.m[i][j] != 0.0) acc = fmaf(static_cast<float>(M.m[i][j]), x[j], acc);
    y[i] = acc;
  }
}

// 8-point DCT-II and its inverse by the even/odd symmetry of the basis,
// C[k][7-n] = (-1)^k C[k][n]: 40 operations instead of 64.
__device__ __forceinline__ void dct8_fwd(const float* x, float* y) {
  constexpr Mat8 C = dct8();
  float s[4], d[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    s[n] = x[n] + x[7 - n];
    d[n] = x[n] - x[7 - n];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float* v = (k & 1) ? d : s;
    float acc = 0.0f;
#pragma unroll
    for (int n = 0; n < 4; ++n) acc = fmaf(static_cast<float>(C.m[k][n]), v[n], acc);
    y[k] = acc;
  }
}

__device__ __forceinline__ void dct8_inv(const float* X, float* x) {
  constexpr Mat8 C = dct8();
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    float e = 0.0f, o = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; k += 2) e = fmaf(static_cast<float>(C.m[k][n]), X[k], e);
#pragma unroll
    for (int k = 1; k < 8; k += 2) o = fmaf(static_cast<float>(C.m[k][n]), X[k], o);
    x[n] = e + o;
    x[7 - n] = e - o;
  }
}

// Element `lane` of the 64 floats at `blk` (a wave-uniform address) by a raw
// buffer load: the base lives in scalar registers, the offset lane * 4 in
// the instruction, so a gather of whole blocks costs no vector address
// arithmetic.  The resource spans exactly the 256 bytes of the block.
__device__ __forceinline__ float load_block_lane(const float* blk, int lane) {
  constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit dwords on gfx9
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(blk), 0, 64 * sizeof(float), kRsrcWord3);
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4, 0, 0));
}

// round(x * 2^40) as a 64-bit integer, exact for |x| < 2^11: the fixed-point
// format of the aggregation sums (integer addition is order-independent).
// Weights can be small (1/TV), so the format keeps 40 fractional bits.
constexpr double kFixScale = 1099511627776.0;  // 2^40
constexpr float kFixScaleF = 1099511627776.0f;
constexpr double kFixMagic = 6755399441055744.0;  // 1.5 * 2^52: adding it rounds to an integer

__device__ __forceinline__ long long to_fixed(float x) {
  const double y = fma(static_cast<double>(x), kFixScale, kFixMagic);
  return __double_as_longlong(y) - __double_as_longlong(kFixMagic);
}

// The same for xs = x * 2^40 already formed in float (scaling by a power of
// two is exact, so the result is identical); one add instead of an FMA with a
// register copy of the magic constant.
__device__ __forceinline__ long long to_fixed_scaled(float xs) {
  const double y = static_cast<double>(xs) + kFixMagic;
  return __double_as_longlong(y) - __double_as_longlong(kFixMagic);
}

// ---------------------------------------------------------------------------
// Full-depth Haar along a group of K registers (K power of two).  The
// orthonormal forward step turns pairs (2j, 2j+1) of the current sums into the
// sum (x0+x1)/sqrt2 at j and the difference (x0-x1)/sqrt2 at half+j, the
// group DC ending at index 0.  The kernels run it unnormalised:
// ---------------------------------------------------------------------------
// the same butterflies without the 1/sqrt2.  Orthonormal
// coefficient k equals haar_gain<K>(k) times unnormalised coefficient k, with
// haar_gain^2 = h/K for the detail band [h, 2h) that holds k (1/K for the
// DC); the orthonormal inverse of c is haar_inv_raw of haar_gain^2 * c', since
// the unnormalised inverse is the transpose of the unnormalised forward.
template <int K>
__host__ __device__ constexpr float haar_gain2(int k) {
  int h = 1;
  while (2 * h <= k) h *= 2;
  return static_cast<float>(k == 0 ? 1.0 / K : static_cast<double>(h) / K);
}

template <int K>
__host__ __device__ constexpr float haar_gain(int k) {
  // the square root of haar_gain2: one factor 1/sqrt2 per butterfly stage on k's path
  double g = 1.0;
  for (int m = K; m > 1; m /= 2) g *= (k < m) ? kInvSqrt2 : 1.0;
  return static_cast<float>(g);
}

template <int K>
__device__ __forceinline__ void haar_fwd_raw(float* v) {
#pragma unroll
  for (int half = K / 2; half >= 1; half /= 2) {
    float t[K];
#pragma unroll
    for (int j = 0; j < half; ++j) {
      t[j] = v[2 * j] + v[2 * j + 1];
      t[half + j] = v[2 * j] - v[2 * j + 1];
    }
#pragma unroll
    for (int j = 0; j < 2 * half; ++j) v[j] = t[j];
  }
}

template <int K>
__device__ __forceinline__ void haar_inv_raw(float* v) {
#pragma unroll
  for (int half = 1; half <= K / 2; half *= 2) {
    float t[K];
#pragma unroll
    for (int j = 0; j < half; ++j) {
      t[2 * j] = v[j] + v[half + j];
      t[2 * j + 1] = v[j] - v[half + j];
    }
#pragma unroll
    for (int j = 0; j < 2 * half; ++j) v[j] = t[j];
  }
}

// ---------------------------------------------------------------------------
// Per-image descriptor and work lists.  Every kernel is a per-work-item body;
// for one image the grid enumerates its items, for a batch a persistent grid
// walks a work list whose per-image prefix offsets are in `begin`.
// ---------------------------------------------------------------------------
struct ImgRec {
  const uint16_t* noisy;           // u16 [H][W]
  const uint16_t* pilot;           // stage-2 matching input, u16 [H][W]
  float* out;                      // stage-2 output, f32 [H][W]
  float* basic;                    // stage-1 output, f32 [H][W]
  uint16_t* q;                     // optional quantised stage-1 output, u16 [H][W]
  float* stack_a;                  // f32 [H*W][64]
  float* stack_b;                  // f32 [H*W][64]
  int16_t* idx;                    // i16 [n_ref][K]
  unsigned long long* partials;    // 64-bit fixed-point aggregation sums: H*W block-start
                                   // weights, then H*W numerator sums (both cleared by the
                                   // stack launch into stack_a)
  double* norm;                    // block norms with a periodic border (correlation matching)
  int H, W;
  float sigma, eps;
};

// Layout of an image's aggregation buffer (ImgRec::partials): the block-start
// weights [H][W], padded to a multiple of 32 entries, then the numerator sums
// [H][W].
__host__ __device__ inline size_t block_weight_entries(int H, int W) {
  return (static_cast<size_t>(H) * W + 31) / 32 * 32;
}
__host__ __device__ inline size_t aggregation_entries(int H, int W) {
  return block_weight_entries(H, W) + static_cast<size_t>(H) * W;
}
__device__ __forceinline__ unsigned long long* numerator_sums(const ImgRec& r) {
  return r.partials + block_weight_entries(r.H, r.W);
}

struct WorkList {
  const ImgRec* recs;  // device array [n]
  const int* begin;    // device array [n + 1]: first item of each image
  const int* start;    // device array [total / kItemBlock + 1]: the image owning item kItemBlock * b
  int n;
  int total;           // begin[n]
};

// Image buffers in the global address space.  A batch kernel reads each
// image's descriptor from its work list, and the compiler cannot tell that
// pointers loaded from memory address global memory: it would use flat
// instructions, which also count against the LDS wait counter, so that each
// wait for an LDS result would wait for outstanding global loads and stores
// as well.  The kernels cast the descriptor's pointers at their use.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;

// Granularity of a batch work list's item -> image lookup table.
constexpr int kItemBlock = 64;
template <typename T>
__device__ __forceinline__ global_ptr<T> to_global(T* p) {
  return (global_ptr<T>)p;
}

// Runs body(rec, local_item) for this workgroup's items: the single image's
// item blockIdx.x, or every batch item blockIdx.x + k * gridDim.x.  The image
// owning a batch item is found from the image owning the first item of its
// block of kItemBlock items (start) by stepping forward through the
// per-image prefix offsets (begin is non-decreasing, begin[0] = 0,
// begin[n] = total; wave-uniform scalar loads); the descriptor is reloaded
// only when the image changes.
template <bool BATCH, typename F>
__device__ __forceinline__ void for_each_item(const ImgRec& one, const WorkList& wl, F&& body) {
  if constexpr (!BATCH) {
    body(one, static_cast<int>(blockIdx.x));
  } else {
    // the work list is read-only for the launch: through constant-space
    // pointers its uniform loads are scalar loads, which wait on the LDS /
    // scalar counter and not behind the previous item's global stores
    typedef const __attribute__((address_space(4))) int* const_int_ptr;
    typedef const __attribute__((address_space(4))) ImgRec* const_rec_ptr;
    const const_int_ptr begin = (const_int_ptr)wl.begin;
    const const_int_ptr start = (const_int_ptr)wl.start;
    const const_rec_ptr recs = (const_rec_ptr)wl.recs;
    int i = -1, lo = 0, hi = 0;  // image i owns items [lo, hi)
    ImgRec r;
    for (int item = blockIdx.x; item < wl.total; item += gridDim.x) {
      if (item >= hi) {
        i = start[item / kItemBlock];
        while (begin[i + 1] <= item) ++i;
        lo = begin[i];
        hi = begin[i + 1];
        r.noisy = recs[i].noisy;
        r.pilot = recs[i].pilot;
        r.out = recs[i].out;
        r.basic = recs[i].basic;
        r.q = recs[i].q;
        r.stack_a = recs[i].stack_a;
        r.stack_b = recs[i].stack_b;
        r.idx = recs[i].idx;
        r.partials = recs[i].partials;
        r.norm = recs[i].norm;
        r.H = recs[i].H;
        r.W = recs[i].W;
        r.sigma = recs[i].sigma;
        r.eps = recs[i].eps;
      }
      body(r, item - lo);
      __syncthreads();  // LDS is reused by the next item
    }
  }
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64)
// ---------------------------------------------------------------------------

// True if the predicate holds in any active lane (a scalar-mask test).
__device__ __forceinline__ bool wave_any(bool pred) { return __builtin_amdgcn_ballot_w64(pred) != 0; }

// This thread's wave index in the workgroup, as a wave-uniform (scalar) value,
// so that control flow and table lookups keyed on it stay scalar.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave); }

// Orders this wave's LDS accesses: every lane's earlier LDS writes are visible
// to every lane's later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Mallat level of a 2-D bior coefficient c = u*8+v: 1 for the finest
// details, 3 for the coarsest details and the approximation.
__device__ __forceinline__ int bior_level(int c) {
  const int u = c >> 3, v = c & 7;
  const int m = u > v ? u : v;
  return m >= 4 ? 1 : (m >= 2 ? 2 : 3);
}

}  // namespace gbm3d
