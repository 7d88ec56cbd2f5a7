// Host-side launchers of the library's kernels (all asynchronous on `st`).
//
// Each launcher runs either one image (`wl` == nullptr: the grid enumerates
// the image's work items, the descriptor `one` is passed by value) or a batch
// (`wl` != nullptr: a persistent grid of at most `grid_cap` workgroups walks
// the work list).  The *_items_for functions give an image's item count for
// each kernel, used to build work lists.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace gbm3d {

// Block matching of one image's noisy (use_pilot = 0) or pilot (1) image into
// rec.idx[n_refs][K] (slot 0 = reference).  split: parts of the displacement
// rows per reference row (1, 2, 4; 0 = by image size).
hipError_t launch_bm(const ImgRec& one, const WorkList* wl, int R, int K, int split, int use_pilot, int grid_cap,
                     hipStream_t st);
int bm_auto_split(long total_waves_unsplit);
long bm_waves_unsplit(int H, int W);
int bm_items_for(int H, int W, int split);

// Correlation-form matching (Theorem 1, int8 matrix cores): the same indices.
// launch_bm_norm writes rec.norm (norm_bytes: the block norms of the noisy or
// pilot image with a periodic border, times 2048, plus a position term
// row (2R + 1) + column) and must precede launch_bm_corr with the same R on the
// stream.  split: waves sharing a 4x4 reference tile (1, 2, 4; 0 = by size).
hipError_t launch_bm_norm(const ImgRec& one, const WorkList* wl, int R, int use_pilot, int grid_cap,
                          hipStream_t st);
hipError_t launch_bm_corr(const ImgRec& one, const WorkList* wl, int R, int K, int split, int use_pilot, int grid_cap,
                          hipStream_t st);
size_t norm_bytes(int H, int W);
int norm_items_for(int H, int W);
int corr_items_for(int H, int W, int split);
long corr_tiles(int H, int W);
int corr_auto_split(long tiles);

// 2-D transform (kind 0 = bior1.5 Mallat, 1 = DCT) of every block of noisy
// (src_sel 0) or pilot (1) into stack_a (dst_sel 0) or stack_b (1), [H*W][64];
// src_sel = dst_sel = -1: noisy -> stack_a and pilot -> stack_b in one launch.
// The launch into stack_a clears the aggregation sums of rec.partials (when
// set).
hipError_t launch_stack(const ImgRec& one, const WorkList* wl, int kind, int src_sel, int dst_sel, int grid_cap,
                        hipStream_t st);
int stack_items_for(int H, int W);
// launch_stack of one image and, in the same launch, the correlation
// matcher's norm table (launch_bm_norm) of noisy (norm_src 0) or pilot (1)
// into rec.norm.
hipError_t launch_stack_norm(const ImgRec& one, int kind, int src_sel, int dst_sel, int R, int norm_src,
                             hipStream_t st);

// bytes of the aggregation buffer (64-bit fixed point) of the group kernels:
// block-start weights of the image, then its numerator sums
size_t partials_bytes(int H, int W);
int group_items_for(int H, int W, int R);

// stage-1 groups: stack_a (bior) + idx -> partials (weights scaled by rec.eps);
// recompute (one image only): the blocks' spectra from rec.noisy's pixels
// instead of stack_a.  shape (K <= 16): 0 = two tiles of 12 waves per CU,
// 1 = one tile of 16 waves with the next group's spectra prefetched; the
// same result either way.  group_ht_tiles_per_cu: the persistent-grid
// multiplier of a shape.
hipError_t launch_group_ht(const ImgRec& one, const WorkList* wl, int R, int K, float ht_a, float ht_b,
                           int weight_mode, int keep_dc, int recompute, int shape, int grid_cap, hipStream_t st);
int group_ht_tiles_per_cu(int K, int shape);
// zeroes the block-start weights and numerator sums of rec.partials (what the
// bior1.5 stack launch does when the stage-1 groups read the stack)
hipError_t launch_clear_weights(const ImgRec& one, hipStream_t st);

// stage-2 groups: stack_a (noisy DCT) + stack_b (pilot DCT) + idx -> partials
hipError_t launch_group_wiener(const ImgRec& one, const WorkList* wl, int R, int K, int grid_cap, hipStream_t st);

// numerator sum / 8 x 8 box sum of the block-start weights into rec.basic
// (+ its quantisation into rec.q when set) or, with final_stage, rec.out
hipError_t launch_reduce(const ImgRec& one, const WorkList* wl, int final_stage, int grid_cap,
                         hipStream_t st);
int reduce_items_for(int H, int W);

hipError_t launch_quantize(const float* in, uint16_t* out, size_t n, hipStream_t st);

// Global stage 1 (the volume form of Sec. 3): one image, every buffer on the
// device, every translation and cycle spin filtered in the same launches.
// Per translation (n_shifts of them, slices in this order): vol_a, vol_b:
// cycles * global_volume_bytes each; num: 2 H W 64-bit words (numerators,
// then denominators); idx: (H/patch)(W/patch) k int16; shifted: H W uint16
// (written for the translations that are not 0).
struct GlobalJob {
  const uint16_t* noisy;
  float* out;
  int H, W;
  float sigma;
  int patch, search, k, levels, cycles, n_shifts;
  int shifts[4];
  float ht_a, ht_b, tv_eps_rel;
  float *vol_a, *vol_b;
  unsigned long long* num;
  int16_t* idx;
  uint16_t* shifted;
};
size_t global_volume_bytes(int H, int W, int K);
// the tile matching alone: idx [(H/patch)(W/patch)][k] displacement ranks
hipError_t launch_global_match(const uint16_t* img, int H, int W, int patch, int search, int k, int16_t* idx,
                               hipStream_t st);
hipError_t launch_global_basic(const GlobalJob& job, hipStream_t st);
// dst [Hp][Wp] = img [H][W] mirror-padded at the bottom and right (edge pixel
// repeated first); H <= Hp <= 2 H, W <= Wp <= 2 W
hipError_t launch_global_pad(const uint16_t* img, int H, int W, uint16_t* dst, int Hp, int Wp, hipStream_t st);

// Peak-rate probes (kind 0 = fp64 vector FMA, 1 = int8 MFMA, 2 = bf16 MFMA):
// blocks of 256 threads, iters rounds each, one float per thread to sink.
// microbench_ops gives the arithmetic operations of such a launch (an FMA or
// multiply-accumulate counts 2).
hipError_t launch_microbench(int kind, int blocks, int iters, float* sink, hipStream_t st);
double microbench_ops(int kind, int blocks, int iters);

}  // namespace gbm3d
