// Per-lane selection of the K-1 smallest keys for the block-matching kernels:
// a sorted register list, merged with small sorted batches by bitonic
// networks (no data-dependent control flow, so a wave never diverges here).
#pragma once

#include "common.h"

namespace gbm3d {

constexpr double kKeyInf = __builtin_huge_val();

// Ascending bitonic sort of B (a power of two) values in registers.
template <int B>
__device__ __forceinline__ void bitonic_sort(double (&b)[B]) {
  static_assert((B & (B - 1)) == 0, "B is a power of two");
#pragma unroll
  for (int k = 2; k <= B; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const double lo = fmin(b[i], b[l]), hi = fmax(b[i], b[l]);
          const bool up = (i & k) == 0;
          b[i] = up ? lo : hi;
          b[l] = up ? hi : lo;
        }
      }
}

// list := the L smallest of list (ascending) and the ascending sequence b(0),
// b(1), ... (P = L + 1 a power of two; b(j) for j < L is read).  With
// a = list + [inf], c[i] = min(a[i], b(P-1-i)) is bitonic and holds the P
// smallest of both; a half-cleaner cascade sorts it.
template <int L, typename Bf>
__device__ __forceinline__ void merge_sorted(double (&list)[L], Bf b) {
  constexpr int P = L + 1;
  static_assert((P & (P - 1)) == 0, "K is a power of two");
  // in place: element i < L is list[i], element L is `last`
  double last = b(0);
#pragma unroll
  for (int i = 1; i < L; ++i) list[i] = fmin(list[i], b(L - i));
#pragma unroll
  for (int s = P / 2; s >= 1; s >>= 1)
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (!(i & s)) {
        const int j = i + s;
        if (j < L) {
          const double lo = fmin(list[i], list[j]), hi = fmax(list[i], list[j]);
          list[i] = lo;
          list[j] = hi;
        } else {  // j == L: the largest element is dropped at the end
          const double lo = fmin(list[i], last), hi = fmax(list[i], last);
          list[i] = lo;
          last = hi;
        }
      }
}

constexpr int pow2_ceil(int n) { return n <= 1 ? 1 : 2 * pow2_ceil((n + 1) / 2); }

// Merges this lane's first cnt buffered keys (buf[j * stride], cnt <= B) into
// list: the batch is padded with inf to a power of two, sorted, then merged.
template <int L, int B>
__device__ __forceinline__ void merge_buffer(double (&list)[L], const double* buf, int stride, int cnt) {
  constexpr int P = pow2_ceil(B);
  double b[P];
#pragma unroll
  for (int j = 0; j < P; ++j) b[j] = (j < B && j < cnt) ? buf[j * stride] : kKeyInf;
  bitonic_sort<P>(b);
  merge_sorted<L>(list, [&](int j) { return j < P ? b[j] : kKeyInf; });
}

__device__ __forceinline__ double shfl_xor_double(double v, int mask) {
  const int lo = __shfl_xor(__double2loint(v), mask, kWave);
  const int hi = __shfl_xor(__double2hiint(v), mask, kWave);
  return __hiloint2double(hi, lo);
}

// rank r = (dy + R) * S + (dx + R) of a key dist * 2048 + r
__device__ __forceinline__ int16_t key_rank(double key) {
  return static_cast<int16_t>(key - 2048.0 * floor(key * (1.0 / 2048.0)));
}

}  // namespace gbm3d
