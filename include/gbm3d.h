/*
 * gbm3d.h — C ABI of the MI355X (gfx950) G-BM3D hot path.
 *
 * Method: Sanders & Larkin, "New Computational Techniques for a Faster
 * Variation of BM3D Image Denoising".  Denoising takes only the noisy image
 * and the noise level (Sec. 1); stage 1 alone gives the basic estimate
 * (G-BM3D1), both stages give the final estimate (G-BM3D2) (Sec. 1.1).
 *
 * Conventions for every entry point:
 *   - Image pointers are HIP DEVICE pointers to row-major arrays with pitch W
 *     elements.  Pixel value = u16 / 65535 on the [0, 1] scale; sigma is on
 *     the same scale.  Float outputs are unclipped float32.
 *   - Boundary handling is periodic: Z[i, j] = Z[i mod H, j mod W] (Sec. 1.2,
 *     eq. (1)).
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*;
 *     NULL = the null stream).  The caller owns every input and output buffer
 *     and keeps it alive until the stream has passed the work.  A context
 *     owns its device workspace, grows it on demand (hipMalloc, outside any
 *     capture) and frees it in gbm3d_destroy.  A context is not thread-safe;
 *     use one per host thread.  Calls on one context must not overlap on
 *     different streams (they share the workspace).
 *   - Arguments are validated on the host before any launch; an invalid call
 *     returns GBM3D_EINVAL and launches nothing.  Errors from the HIP runtime
 *     return GBM3D_EHIP.  The text of the last error of a context is
 *     available from gbm3d_last_error.  A kernel fault surfaces at the
 *     caller's synchronisation.
 *   - Supported shapes: patch 8, reference step 3, odd search window in
 *     [1, 39], group sizes in {2, 4, 8, 16, 32} not above search^2, and
 *     H, W >= max(8, search) and <= 32768.
 */
#ifndef GBM3D_H
#define GBM3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define GBM3D_OK            0
#define GBM3D_EINVAL       -1
#define GBM3D_EUNSUPPORTED -2
#define GBM3D_ENOMEM       -3
#define GBM3D_EHIP         -4

/* stage-1 aggregation weights (Sec. 3.1 gives 1/TV; a count of retained
 * coefficients and unit weights are the alternatives the paper mentions) */
#define GBM3D_W_TV   0
#define GBM3D_W_NNZ  1
#define GBM3D_W_UNIT 2

/* gbm3d_denoise_batch flags */
#define GBM3D_BATCH_GRAPH      1  /* capture the launches into a hipGraph, replayed
                                     while the batch shape is unchanged            */
#define GBM3D_BATCH_BASIC_ONLY 2  /* stage 1 only: out receives the basic estimate */

/* block-matching kernels; both give the same indices (Sec. 2: eq. dfg
 * summed shift by shift, or the norm/cross-correlation split of Theorem 1) */
#define GBM3D_BM_AUTO  0  /* the autotuned choice for the shape, else CORR  */
#define GBM3D_BM_SHIFT 1  /* per displacement: squared differences, box sums
                             at the reference positions (float64 vector ALU) */
#define GBM3D_BM_CORR  2  /* per 4x4 reference tile: block norms plus int8
                             matrix-core cross-correlations, exact           */

/* patch-stack transforms */
#define GBM3D_STACK_BIOR15 0   /* 3-level periodic Mallat bior1.5 (Sec. 5) */
#define GBM3D_STACK_DCT    1   /* orthonormal 8x8 DCT-II (Sec. 4)           */

typedef struct gbm3d_ctx gbm3d_ctx;

typedef struct {
  uint32_t struct_size; /* = sizeof(gbm3d_params); guards the ABI            */
  int32_t patch;        /* N = 8                                            */
  int32_t step;         /* reference grid step, 3                           */
  int32_t search;       /* S, odd; displacements |dy|,|dx| <= S/2; 39       */
  int32_t k_ht;         /* group size of stage 1, 16                        */
  int32_t k_wiener;     /* group size of stage 2, 32                        */
  float ht_a, ht_b;     /* tau_l = sigma * (ht_a - ht_b * l) (Sec. 5): 3.6, 0.3 */
  int32_t ht_weight;    /* GBM3D_W_TV (default) | GBM3D_W_NNZ | GBM3D_W_UNIT */
  float tv_eps_rel;     /* > 0: w = 1 / (TV + tv_eps_rel * sigma * 64 * k_ht); 1e-3 */
  int32_t keep_dc;      /* 1: the 3-D DC coefficient is never shrunk        */
  /* launch tuning (results do not depend on it) */
  int32_t bm_split;     /* block matching: waves sharing one reference tile,
                           each scanning a part of the search window,
                           1 | 2 | 4; 0 = tuned or chosen by image size      */
  int32_t bm_method;    /* GBM3D_BM_AUTO (tuned or default) | GBM3D_BM_SHIFT |
                           GBM3D_BM_CORR                                     */
  int32_t ht_source;    /* where stage 1 takes each matched block's bior1.5
                           spectrum from: GBM3D_HT_STACK (default: the
                           precomputed stack of every block) |
                           GBM3D_HT_RECOMPUTE (transformed from the block's
                           pixels inside the group kernel; no stack; single
                           images only, batches return GBM3D_EUNSUPPORTED);
                           the same result bit for bit                       */
} gbm3d_params;

#define GBM3D_HT_STACK     0
#define GBM3D_HT_RECOMPUTE 1

/* One image of a batch (see gbm3d_denoise_batch). */
typedef struct {
  const uint16_t* noisy; /* device, H*W                                     */
  const uint16_t* pilot; /* device, H*W, or NULL to run stage 1 as the pilot */
  float* out;            /* device, H*W                                     */
  int32_t H, W;
  float sigma;
} gbm3d_image;

/* Fills *p with the defaults above (sets struct_size). */
void gbm3d_default_params(gbm3d_params* p);

/* Creates a context on HIP device `hip_device` (-1 = the current device).
 * Returns GBM3D_OK and stores the context in *ctx, or an error code. */
int gbm3d_create(gbm3d_ctx** ctx, int hip_device);

/* Frees the context and its workspace (synchronises the device first).
 * NULL is ignored. */
void gbm3d_destroy(gbm3d_ctx* ctx);

/* Static text for a status code. */
const char* gbm3d_status_str(int status);

/* Text of the last error reported on ctx ("" if none); valid until the next
 * call on ctx. */
const char* gbm3d_last_error(const gbm3d_ctx* ctx);

/* Number of references on the periodic grid: ceil(H/step) * ceil(W/step).
 * References are ordered row-major: ref = p * ceil(W/step) + q sits at
 * (step*p, step*q). */
int64_t gbm3d_n_refs(int H, int W, int step);

/* Host-only validation of the arguments of gbm3d_denoise (image shape, noise
 * level, parameters; NULL params = defaults).  Needs no device and launches
 * nothing.  The error text is available from gbm3d_last_error(NULL). */
int gbm3d_check_args(int H, int W, float sigma, const gbm3d_params* params);

/* Library version string. */
const char* gbm3d_version(void);

/* Block matching (Sec. 2 eq. dfg, Theorem 1; arg_K min of Sec. 3.1).
 * img: device u16 [H][W].  idx: device int16 [n_refs][K] receiving, for each
 * reference, the displacement ranks r = (dy + S/2) * S + (dx + S/2) of its K
 * matched blocks: slot 0 is the reference itself, slots 1..K-1 the K-1 other
 * displacements with the smallest (squared distance, rank) keys in ascending
 * order; distances are exact. */
int gbm3d_match(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int K,
                const gbm3d_params* params, int16_t* idx, void* stream);

/* Transform-domain patch stack: for every pixel position (y, x), the 2-D
 * transform of the periodic 8x8 block with top-left (y, x) of img/65535.
 * kind: GBM3D_STACK_BIOR15 (Sec. 5; coefficient (u, v) in Mallat layout) or
 * GBM3D_STACK_DCT (Sec. 4; (u, v) = (row, column) frequency).
 * out: device float [H*W][64], element ((y*W + x)*64 + u*8 + v). */
int gbm3d_stack(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int kind,
                float* out, void* stream);

/* Stage 1 (G-BM3D1): matching with k_ht, bior1.5 x Haar hard thresholding
 * with tau_l, weighted aggregation (Sec. 3.1, Sec. 5).
 * noisy: device u16 [H][W]; basic: device float [H][W]. */
int gbm3d_basic(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma,
                const gbm3d_params* params, float* basic, void* stream);

/* Stage 2 (Sec. 4): matching with k_wiener on `pilot`, DCT x Haar empirical
 * Wiener filter of the noisy groups with the pilot's spectrum, aggregation.
 * noisy, pilot: device u16 [H][W]; out: device float [H][W]. */
int gbm3d_wiener(gbm3d_ctx* ctx, const uint16_t* noisy, const uint16_t* pilot,
                 int H, int W, float sigma, const gbm3d_params* params,
                 float* out, void* stream);

/* Both stages (G-BM3D2): stage 1, pilot Q = floor(clip(basic, 0, 1)*65535
 * + 1/2), stage 2 with Q.  out: device float [H][W].  basic_out and q_out
 * are optional (NULL) device outputs of the intermediate estimate. */
int gbm3d_denoise(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma,
                  const gbm3d_params* params, float* out, float* basic_out,
                  uint16_t* q_out, void* stream);

/* ---------------------------------------------------------------------------
 * Global stage 1 (Sec. 3, the volume form; Sec. 5 parameters): reference
 * blocks of side `patch` tile the image, each is matched to its `k` nearest
 * blocks in the search window (same key and tie rule as gbm3d_match, slot 0
 * the reference), the k-th matches are stacked behind the references into a
 * volume with the noisy image as its first slice, the whole volume is
 * transformed (periodic separable 3-D Mallat decomposition, `levels` levels:
 * bior1.5 along both image axes, orthonormal Haar along the match axis),
 * hard-thresholded with tau_l = sigma (ht_a - ht_b l) per detail level (the
 * final approximation kept) and inverted, averaged over `cycles` cycle spins
 * (circular shifts by h = 0 .. cycles-1 along all three axes); the blocks
 * return to their sources with weight 1 / (TV + eps) of their reference's
 * block (3-D total variation, eps = tv_eps_rel sigma patch^2 k), and the
 * normalised estimate is averaged over the `n_shifts` image translations
 * `shifts` (eq. firstEst).
 * ------------------------------------------------------------------------- */
typedef struct {
  uint32_t struct_size; /* = sizeof(gbm3d_global_params) */
  int32_t patch;        /* 8 or 16 (16 in Sec. 5); H and W multiples of it */
  int32_t search;       /* odd, 3 .. 39 (Sec. 5 states 32; default 33) */
  int32_t k;            /* 8, 16 (default) or 32; k >= 2^levels */
  int32_t levels;       /* 1 .. 3 (default 3) */
  int32_t cycles;       /* 1 .. 4 (default 2) */
  int32_t n_shifts;     /* 1 .. 4 (default 2) */
  int32_t shifts[4];    /* translations, each in [0, patch) (default 0, patch/4) */
  float ht_a, ht_b;     /* 3.6, 0.3 */
  float tv_eps_rel;     /* 1e-3 */
} gbm3d_global_params;

void gbm3d_global_default_params(gbm3d_global_params* p);

/* noisy: device u16 [H][W]; out: device float [H][W].  H, W in
 * [max(search, patch), 32768]; sides that are not multiples of patch are
 * handled as the paper does (Sec. 3.1): the image is extended at the bottom
 * and right with mirrored values (edge pixel repeated first) to the next
 * multiples, filtered, and the estimate cropped back to H x W.  All
 * translations and cycle spins are filtered together, so the context keeps
 * 2 * n_shifts * cycles float volumes of k H W entries (of the padded size)
 * and 2 * n_shifts H W 64-bit sums as workspace; GBM3D_ENOMEM when they
 * cannot be allocated. */
int gbm3d_global_basic(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma,
                       const gbm3d_global_params* params, float* out, void* stream);

/* The tile matching of gbm3d_global_basic alone (S^K_pq of Sec. 3.1 for the
 * reference tiles): idx device int16 [(H/patch)(W/patch)][k], tiles in raster
 * order, displacement ranks r = (dy+R)*search + (dx+R), slot 0 the tile
 * itself, then ascending (distance, rank).  H and W must be multiples of
 * patch here. */
int gbm3d_global_match(gbm3d_ctx* ctx, const uint16_t* img, int H, int W,
                       const gbm3d_global_params* params, int16_t* idx, void* stream);

/* gbm3d_denoise for callers that cannot allocate device memory: code under
 * hipGraph stream capture, tight serving loops, hosts that forbid hipMalloc.
 * Same arguments, validation and result (bit for bit) as gbm3d_denoise, but
 * every intermediate buffer (norm table, two patch stacks, match indices,
 * aggregation sums, and the basic estimate and pilot when basic_out / q_out
 * are NULL) is a slice of one static device array of
 * GBM3D_NOALLOC_SCRATCH_BYTES per device, which the library holds on every
 * device it runs on until the process ends.  The call makes no hipMalloc,
 * hipFree or other allocating call and records no timing events.  It
 * returns GBM3D_EINVAL, launching nothing, when the image needs more scratch
 * than that (with the default parameters square images up to 551 x 551
 * fit, when basic_out and q_out are NULL; the error text gives the bytes
 * needed).  Every call on a device shares that device's
 * array and leaves its contents behind (the kernels clear what must start
 * at zero), so calls that overlap on one device — on two streams, from two
 * contexts or two threads — race and give undefined results; serialise them.
 * The caller owns noisy, out, basic_out and q_out as in gbm3d_denoise. */
#define GBM3D_NOALLOC_SCRATCH_BYTES (160u * 1024u * 1024u)
int gbm3d_denoise_noalloc(gbm3d_ctx* ctx, const uint16_t* noisy, int H, int W, float sigma,
                          const gbm3d_params* params, float* out, float* basic_out,
                          uint16_t* q_out, void* stream);

/* A batch of images of any sizes (the plug-and-play use case of Sec. 1: one
 * denoiser call per iteration, many images).  imgs: HOST array of n
 * descriptors (device pointers inside).  For each image: if pilot == NULL,
 * stage 1, Q and stage 2 as in gbm3d_denoise; otherwise stage 2 with the given
 * pilot.  With GBM3D_BATCH_BASIC_ONLY, stage 1 only (pilot must be NULL) and
 * out receives the basic estimate.  All images run in one sequence of ~9
 * kernel launches over the work items of the whole batch (one workgroup per
 * item, its image found from per-image work lists); with
 * GBM3D_BATCH_GRAPH the sequence is captured once into a hipGraph and replayed
 * while image count, sizes, parameters and flags are unchanged (pointers may
 * change between calls).  Results equal the single-image calls bit for bit.
 * The image array is copied before the call returns. */
int gbm3d_denoise_batch(gbm3d_ctx* ctx, const gbm3d_image* imgs, int n,
                        const gbm3d_params* params, int flags, void* stream);

/* Pilot quantisation: out[i] = floor(clip(in[i], 0, 1) * 65535 + 1/2),
 * evaluated in double from the float input; NaN -> 0.  Device pointers. */
int gbm3d_quantize(gbm3d_ctx* ctx, const float* in, uint16_t* out, size_t n, void* stream);

/* Peak-rate probes, for reading the kernels' achieved rates against measured
 * ceilings: `blocks` workgroups of 256 threads run `iters` rounds of eight
 * independent chains of one operation with no memory traffic, then write one
 * float per thread to the device buffer sink (blocks * 256 floats, owned by
 * the caller; the values carry no meaning).  kind GBM3D_PROBE_FP64: fp64
 * vector FMA (the shift-wise and global matchers' unit); GBM3D_PROBE_MFMA_I8:
 * v_mfma_i32_16x16x64_i8 (the correlation matcher's); GBM3D_PROBE_MFMA_BF16:
 * v_mfma_f32_16x16x32_bf16 (the pilot's).  Asynchronous on stream; time it
 * with events.  blocks and iters in [1, 2^20].  gbm3d_probe_ops returns the
 * arithmetic operations of such a launch (a fused multiply-add counts 2), or
 * 0 for an unknown kind. */
#define GBM3D_PROBE_FP64 0
#define GBM3D_PROBE_MFMA_I8 1
#define GBM3D_PROBE_MFMA_BF16 2
int gbm3d_probe(gbm3d_ctx* ctx, int kind, int blocks, int iters, float* sink, void* stream);
double gbm3d_probe_ops(int kind, int blocks, int iters);

/* ---------------------------------------------------------------------------
 * Learned pilot: a six-layer 3x3 convolutional network (2 -> 32 -> 32 -> 32 ->
 * 32 -> 32 -> 1 channels, ReLU after the first five, zero "same" padding,
 * input (z, sigma plane), output pilot = z - f) that can stand in for stage 1
 * as the first estimate the Wiener stage needs (Sec. 4).  bf16 weights and
 * activations, fp32 accumulation on the matrix cores.  Parameters live in a
 * float32 master vector of gbm3d_pilot_param_count() entries: per layer
 * W[ky][kx][ci][co] (row-major) followed by bias[co].
 * ------------------------------------------------------------------------- */
int gbm3d_pilot_param_count(void);

/* Packs the master vector (device float [P]) into the context's bf16 weights. */
int gbm3d_pilot_load(gbm3d_ctx* ctx, const float* master, void* stream);

/* Pilot of B images noisy [B][H][W] (device u16) with noise levels sigma
 * (device float [B]).  pilot_u16 (device u16 [B][H][W], the quantised pilot
 * floor(clip(p,0,1)*65535 + 1/2)) and/or pilot_f32 (device float) may be NULL.
 * Needs gbm3d_pilot_load first. */
int gbm3d_pilot_infer(gbm3d_ctx* ctx, const uint16_t* noisy, int B, int H, int W,
                      const float* sigma, uint16_t* pilot_u16, float* pilot_f32, void* stream);

/* Training: the mean squared error of the pilot against target (device float
 * [B][H][W]), each image's squared errors scaled by weight[b] (device float
 * [B]; NULL = all 1), written to *loss (device float), and its gradient with
 * respect to the master vector into grad (device float [P]), with the loaded
 * weights.  H and W >= 1. */
int gbm3d_pilot_grad(gbm3d_ctx* ctx, const uint16_t* noisy, const float* target, int B, int H, int W,
                     const float* sigma, const float* weight, float* grad, float* loss, void* stream);

/* One Adam step (bias-corrected, step >= 1) on the master vector with moments
 * m, v (device float [P], zero before the first step), then reloads the
 * packed weights. */
int gbm3d_pilot_adam(gbm3d_ctx* ctx, float* master, float* m, float* v, const float* grad, int step,
                     float lr, float beta1, float beta2, float eps, void* stream);

/* Per-kernel timing for benchmarking.  While enabled, the context brackets
 * every kernel it launches with two HIP events recorded on the launch stream.
 * gbm3d_timing_read synchronises the pending events and returns, for one
 * kernel name ("bm", "bm_norm", "stack_bior", "stack_dct", "group_ht",
 * "group_wiener", "reduce"), the summed elapsed milliseconds and the number of
 * launches since the last reset ("stack_dct" is one launch that forms both
 * stage-2 stacks, of the noisy image and of the pilot).  Off by default. */
int gbm3d_timing_enable(gbm3d_ctx* ctx, int on);
int gbm3d_timing_read(gbm3d_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);
int gbm3d_timing_reset(gbm3d_ctx* ctx);

/* Autotuner of the launch configuration (the paper's method does not depend
 * on it; results are identical for every choice).  With the caller's params
 * (NULL = defaults; search, and for the shape below k_ht and the stage-1
 * options), on the device image img [H][W]:
 *   - times every block-matching variant (GBM3D_BM_SHIFT and GBM3D_BM_CORR,
 *     each with bm_split 1, 2 and 4) with group size K, `reps` runs each
 *     after one warm-up run, and records the fastest;
 *   - when K == params.k_ht <= 16, also times whole stage-1 runs (that
 *     matching, sigma 25/255) with each of the two shapes of the stage-1
 *     group kernel (two tiles of 12 waves per compute unit, or one tile of
 *     16 waves that prefetches the next group) and records the faster.
 * Records are keyed by (K, search, shape class of (H, W): the number of 4x4
 * reference tiles rounded down to a power of two).  Later calls whose params
 * leave bm_method or bm_split at 0 use the record of their class (a batch:
 * the class of all its tiles together); without one, the method recorded for
 * the nearest class of the same K and search, with the split chosen by size;
 * else GBM3D_BM_CORR.  The stage-1 shape likewise (default: two tiles).
 * Timing uses HIP events on `stream` (the call synchronises it).
 * best_method, best_split and best_ms (milliseconds per matching run) may be
 * NULL.  Errors: GBM3D_EINVAL for bad shapes, params, K or reps < 1. */
int gbm3d_autotune(gbm3d_ctx* ctx, const uint16_t* img, int H, int W, int K, const gbm3d_params* params,
                   int reps, int* best_method, int* best_split, float* best_ms, void* stream);

/* The recorded choices as text, one line each: "bm K search class method
 * split ms" or "ht K search class shape ms".  gbm3d_tune_save writes them to
 * `path`, gbm3d_tune_load adds those of `path` to the context (GBM3D_EINVAL,
 * adding nothing, if the file cannot be read or a line parsed). */
int gbm3d_tune_save(const gbm3d_ctx* ctx, const char* path);
int gbm3d_tune_load(gbm3d_ctx* ctx, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* GBM3D_H */
