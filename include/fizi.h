/*
 * fizi.h - C ABI of the MI355X (gfx950) FIZI/Mouse pipeline: the per-frame
 * pixel path of Magoules & Zou, "GPU Accelerated Contactless Human Machine
 * Interface for Driving Car" (arXiv 1907.04393).
 *
 * What the path computes (paper Section 2, "Architecture"; Section 3.1,
 * "Building the Mask of the Hand"; Section 3.2, "Managing Luminosity"):
 *   initialisation: learn the background from user-free frames;
 *   running phase, per frame: correct the brightness, keep the pixels that
 *   are (i) outside the learned background range, (ii) not gray and (iii) of
 *   skin hue, AND the three masks, clean the result with erosion and dilation
 *   (the binary image I_FIZI), pick the hand zone, and reduce it to a pointer
 *   (position sums, area, bounding box and a click state).
 * The readings taken where the paper is silent or garbled are stated at each
 * parameter below.
 *
 * Conventions
 *   - Every d_* pointer is a DEVICE pointer owned by the caller; h_* pointers
 *     are host memory. The library never frees caller memory and never calls
 *     hipMalloc: device state lives in a caller-provided block (d_state).
 *     It allocates a little pinned host memory and a few HIP events at
 *     create time only.
 *   - Frames are H x W x 3 uint8, R,G,B interleaved, row-major, contiguous;
 *     n frames are n consecutive frames. W must be a positive multiple of 64
 *     (so each mask row is a whole number of 64-bit words), H >= 1, and
 *     W * H < 2^31.
 *   - Bit masks are H rows of W/64 uint64 words; bit b of word j of row y is
 *     pixel (x = 64 j + b, y) (LSB first).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked async only enqueue work on it.
 *   - Return value: FIZI_OK (0) or a negative FIZI_E* code; the message of
 *     the last failure on the calling thread is in fizi_last_error(). No C++
 *     exception crosses this boundary, and a failed call leaves its context
 *     usable.
 *   - A context or batch is used from one host thread at a time.
 */
#ifndef FIZI_H
#define FIZI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FIZI_OK = 0,
    FIZI_EINVAL = -1,   /* bad geometry, parameter, pointer or size */
    FIZI_ESTATE = -2,   /* e.g. process_frames before any learn_background */
    FIZI_ENOMEM = -3,   /* state block too small, or pinned host memory */
    FIZI_EHIP = -4,     /* HIP runtime error (message has the HIP string) */
    FIZI_ERANGE = -5    /* frame index not (or no longer) available */
};

typedef struct {
    int32_t width;      /* W: multiple of 64, >= 64 */
    int32_t height;     /* H: >= 1 */
} fizi_geom;

/* Thresholds and readings. fizi_default_params() fills the defaults. */
typedef struct {
    /* Section 3.1 (iii): skin when chroma > 0 and the exact hexcone hue lies
     * in the closed interval [alpha1, alpha2] (centi-degrees, 0..35999),
     * wrapping through 360 when alpha1 > alpha2. Defaults 33000, 7500 (the
     * paper's own values are lost with its Figure 2). */
    int32_t alpha1_cdeg;
    int32_t alpha2_cdeg;
    /* Section 3.1 (ii): gray when max_RGB - min_RGB < S. 0..255, default 20. */
    int32_t gray_S;
    /* Section 3.1 (i): background when every channel lies in
     * [bgmin - delta, bgmax + delta]. 0..255, default 10 (0 = the bare box). */
    int32_t bg_delta;
    /* Section 3.1, last paragraph: opening (erosions then dilations) then
     * closing (dilations then erosions), 3x3 square, out-of-image pixels
     * neutral (1 for erosion, 0 for dilation). 0..3 each, default 1, 1. */
    int32_t open_iters;
    int32_t close_iters;
    /* Section 2, Mouse module: the hand zone is the 8-connected component of
     * largest area (ties: smallest first raster index); present when its
     * area >= min_area (>= 0, default 1). */
    int32_t min_area;
    /* Section 2 "its state (click or not)": click when
     * 1000 * area >= click_fill_permille * bbox_area. 0..1000, default 700. */
    int32_t click_fill_permille;
    /* Section 2 / 3.2 brightness: one global inverse gain per frame, Q16, from
     * the luminance R+2G+B of rows y % gain_row_stride == 0 against the first
     * learning frame, over pixels whose reference is unclipped, whose raw
     * channels are all in 1..254 and whose raw hue is not skin; rounded half
     * up and clamped to [gain_lo_q16, gain_hi_q16]. Each channel becomes
     * min(255, (v * inv + 32768) >> 16). Defaults 8, 32768, 131072. */
    int32_t gain_row_stride;   /* 1..64 */
    int32_t gain_lo_q16;       /* 1..2^20 */
    int32_t gain_hi_q16;       /* gain_lo_q16..2^20 */
    /* Section 3.2 names two ways to follow the brightness: correct the
     * pixels (0, the default, as above) or adapt the thresholds (1): the
     * pixels stay raw, and with the frame's gain g = 2^16 / inv a channel v
     * is inside the box when (bgmin - delta) g <= v <= (bgmax + delta) g and
     * the pixel is gray when max - min < S g (compared exactly, as v * inv
     * against bound * 2^16); the hue is the raw pixel's. The gain itself and
     * the learning (on corrected frames) do not change. */
    int32_t brightness_mode;   /* 0 or 1 */
    /* Section 2, the Mouse module tracks the hand and its state: with
     * temporal tracking on, the reported click changes only once
     * click_debounce consecutive frames show the new state; a frame without
     * a hand reports no click and clears the count. 0..255, default 0
     * (0 and 1 report every frame's own click). No effect without tracking. */
    int32_t click_debounce;
    /* Section 2, the Mouse module tracks the hand zone: with temporal
     * tracking on and a hand in the previous frame, the hand is the
     * component of area >= min_area nearest to the previous centroid pixel
     * (the smallest squared distance from that pixel to one of its pixels,
     * 0 for the component covering it) when that distance is at most
     * track_radius pixels - ties to the larger area, then the smaller first
     * raster index - else the largest component. 0 keeps only a component
     * covering the previous centroid. 0..16384, default 64. */
    int32_t track_radius;
    /* Section 3.2, over-exposure: an over-exposed hand looks white and the
     * gray test removes it, so the Luminosity component is modified in the
     * most obvious cases. With lum_hi in 128..254, a corrected pixel whose
     * HSL lightness (max + min) / 2 exceeds lum_hi has it brought down to
     * lum_hi with hue and HSL saturation kept before the gray test: its
     * chroma becomes (max - min) (510 - 2 lum_hi) / (510 - max - min),
     * compared exactly with S. The box and hue tests are unchanged. 0 (the
     * default) turns it off; it needs brightness_mode 0. */
    int32_t lum_hi;
} fizi_params;

/* One frame's pointer (56 bytes). When `present` is 0 every field except
 * n_components, inv_gain_q16 and frame_index is zero. The centroid is
 * (sum_x / area, sum_y / area); x is the column, y the row. */
typedef struct {
    uint8_t present;
    uint8_t click;
    uint16_t reserved;
    uint32_t area;
    uint64_t sum_x;
    uint64_t sum_y;
    uint32_t x0, y0, x1, y1;     /* inclusive bounding box */
    uint32_t n_components;       /* 8-connected components of I_FIZI */
    uint32_t inv_gain_q16;       /* the frame's inverse gain */
    uint64_t frame_index;        /* running index within the context */
} fizi_pointer;

typedef struct fizi_ctx fizi_ctx;

/* Byte offsets of the learned model inside a context's state block. */
typedef struct {
    uint64_t bgmin;        /* H*W*3 uint8, frame layout */
    uint64_t bgmax;        /* H*W*3 uint8 */
    uint64_t yref;         /* yref_rows * W uint16: reference luminance of the
                              sampled rows, 0xFFFF where a channel was clipped */
    uint64_t yref_rows;    /* ceil(H / gain_row_stride) */
    uint64_t total;        /* == fizi_state_bytes() */
} fizi_layout;

/* Fills *out with the defaults listed above. */
int fizi_default_params(fizi_params *out);

/* Checks geometry and parameters (FIZI_EINVAL with a message, else 0). */
int fizi_validate(const fizi_geom *geom, const fizi_params *params);

/* Device bytes a context needs when it processes up to `chunk_frames`
 * frames per internal batch (1..256). 0 when the arguments are invalid. */
size_t fizi_state_bytes(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames);

/* Offsets of the model arrays inside the state block. */
int fizi_state_layout(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames,
                      fizi_layout *out);

/* Creates a context over the caller's device block d_state (256-byte
 * aligned, >= fizi_state_bytes; kept by the caller until fizi_destroy).
 * Enqueues the block's initialisation on `stream`. */
int fizi_create(const fizi_geom *geom, const fizi_params *params, int32_t chunk_frames,
                void *d_state, size_t state_bytes, void *stream, fizi_ctx **out);

/* Frames everywhere below are H x W x 3 uint8, interleaved RGB, row-major,
 * consecutive frames contiguous, in device memory, 4-byte aligned
 * (FIZI_EINVAL otherwise; 16-byte aligned frames take the faster gain path).
 *
 * Section 2 initialisation ("learns the background without the user") with
 * the model of Section 3.1 (i): with reset != 0 the reference luminance is
 * taken from d_frames[0] and the per-pixel, per-channel [bgmin, bgmax] model
 * starts empty; otherwise learning continues from the current model. Each
 * frame is brightness-corrected (as in process_frames) before it widens the
 * model; the model is read and written once per call. n_frames >= 1. Async. */
int learn_background(fizi_ctx *ctx, const uint8_t *d_frames, int32_t n_frames, int32_t reset,
                     void *stream);

/* Section 3.3 partial re-learning ("dealing with the evolution of the
 * luminosity implies sometimes to re-initiate partly the machine learning"):
 * n_frames >= 1 running frames widen the model exactly as learning frames do
 * (gain-corrected against the unchanged reference luminance, per-channel min
 * and max), but only at the pixels whose bit in that frame's I_FIZI mask
 * (d_fizi_bits: n_frames masks of H rows of W/64 words, as process_frames
 * writes them; 8-byte aligned) is 0, so the hand zone never enters the model.
 * The caller chooses which frames to feed back. FIZI_ESTATE before the first
 * learn_background. Async, ordered after the context's earlier calls. */
int relearn_background(fizi_ctx *ctx, const uint8_t *d_frames, int32_t n_frames,
                       const uint64_t *d_fizi_bits, void *stream);

/* Section 2 running phase for n_frames >= 1 frames: brightness correction,
 * the masks I_R1, I_R2, I_R3 of Section 3.1 and their AND, opening and
 * closing (I_FIZI), the hand zone and its pointer. Frames are independent
 * given the model and are processed in internal batches of chunk_frames.
 * d_fizi_bits (nullable): n_frames bit masks of I_FIZI. d_hand_bits
 * (nullable): n_frames bit masks of the selected hand zone. d_pointers
 * (nullable): n_frames pointers. Frame indices continue from the previous
 * call. FIZI_ESTATE before the first learn_background. Async. */
int process_frames(fizi_ctx *ctx, const uint8_t *d_frames, int32_t n_frames,
                   uint64_t *d_fizi_bits, uint64_t *d_hand_bits, fizi_pointer *d_pointers,
                   void *stream);

/* Temporal tracking of the hand (the Mouse module "tracks" the hand zone,
 * Section 2): with enable != 0, when the previous frame had a hand, the
 * component nearest its centroid pixel (floor of the coordinate sums over the
 * area; the one covering it first) within track_radius keeps the hand if its
 * area reaches min_area (see fizi_params::track_radius); otherwise the
 * largest component is taken, as without tracking. Frames are tracked in
 * order across calls. Waits for the context's work (a pending pipelined
 * call included) and clears the tracking state. */
int fizi_set_tracking(fizi_ctx *ctx, int32_t enable);

/* Pipelined calls, for a stream processed in back-to-back calls: with
 * enable != 0, a call leaves the morphology and components of its last
 * internal batch running on the context's side stream instead of waiting for
 * them before its end, and the next call joins them after its first batch's
 * classify, so that they run beside it. A call's outputs (masks, pointers)
 * are then complete on its stream once the next call, or fizi_flush, has
 * completed there; its input frames may be reused as soon as the call has
 * completed. get_pointer waits on its own. Waits for the context's work;
 * enable == 0 restores calls that complete their outputs themselves. */
int fizi_set_pipelined(fizi_ctx *ctx, int32_t enable);

/* Completes every call's outputs on `stream` (orders it after a pending
 * pipelined call's last batch). Async. */
int fizi_flush(fizi_ctx *ctx, void *stream);

/* Launch shape of the context's morphology. With enable != 0 (the default)
 * a launch too small to fill the device - its frames' morphology in 4-row
 * bands of one wave each needs at most one wave per SIMD, as for one to
 * three 1920x1080 frames - takes that shape: its length is then one wave's
 * chain of rows rather than the work. With 0 every launch keeps 8-row bands
 * (two or four to a wave for frames up to 2048 or 1024 pixels wide).
 * Results do not depend on it; it applies from the next call. */
int fizi_set_short_bands(fizi_ctx *ctx, int32_t enable);

/* Waits for the frame with running index frame_index and copies its pointer
 * to *h_out. The last 65536 frames are kept; older or not yet submitted
 * indices give FIZI_ERANGE. */
int get_pointer(fizi_ctx *ctx, int64_t frame_index, fizi_pointer *h_out);

/* Waits for the context's work (a pending pipelined call included),
 * releases its host resources. Frees nothing the caller owns. */
int fizi_destroy(fizi_ctx *ctx);

/* Measurement hook. With enable != 0 the context records a HIP event pair
 * on the call's stream around each launch of the stages below (at most
 * 16384 launches per stage between two reads); fizi_stage_times() waits for
 * them, returns the summed milliseconds and launch counts per stage, and
 * clears them. Stages: 0 gain, 1 classify, 2 morphology, 3 components and
 * pointer, 4 background learning. */
enum { FIZI_STAGE_GAIN = 0, FIZI_STAGE_CLASSIFY, FIZI_STAGE_MORPH, FIZI_STAGE_RESOLVE,
       FIZI_STAGE_LEARN, FIZI_NSTAGES };
int fizi_stage_timing(fizi_ctx *ctx, int32_t enable);
int fizi_stage_times(fizi_ctx *ctx, double *h_ms /* [FIZI_NSTAGES] */,
                     int64_t *h_launches /* [FIZI_NSTAGES] */);

/* ---- Batched form ---------------------------------------------------------
 * Many camera streams (each its own geometry, thresholds and background
 * model) go through one pipeline pass per frame step: the same per-frame
 * method as process_frames, with the frames of all active streams in one set
 * of launches (or one persistent kernel), optionally replayed from a
 * hipGraph. Streams are independent given their models (Section 2: the
 * running phase treats each camera image on its own). */
typedef struct fizi_batch fizi_batch;

enum {
    FIZI_BATCH_DIRECT = 0,            /* four kernels per step, launched directly */
    FIZI_BATCH_GRAPH = 1,             /* the same, replayed from a hipGraph */
    FIZI_BATCH_PERSISTENT = 2,        /* one persistent kernel per step, fed by an ordered
                                         work queue: gain tiles, row bands (classify, then
                                         morphology of the band above) and components overlap */
    FIZI_BATCH_PERSISTENT_GRAPH = 3,  /* the persistent kernel from a hipGraph */
    FIZI_BATCH_PIPELINED = 4,         /* four kernels, software-pipelined across steps: a
                                         step's gain and classify run on the caller's stream
                                         beside the previous step's morphology, components
                                         and pointers, which run on a second HIP stream
                                         forked from and joined back to the caller's */
    FIZI_BATCH_PIPELINED_GRAPH = 5    /* the same, replayed from hipGraphs */
};

/* Device bytes for n_streams (1..256) streams; geoms and params are arrays of
 * n_streams. 0 when an argument is invalid. */
size_t fizi_batch_state_bytes(int32_t n_streams, const fizi_geom *geoms, const fizi_params *params);

/* Creates a batch over the caller's 256-byte aligned device block. */
int fizi_batch_create(int32_t n_streams, const fizi_geom *geoms, const fizi_params *params,
                      void *d_state, size_t state_bytes, fizi_batch **out);

/* learn_background for one stream of the batch. Async. */
int fizi_batch_learn(fizi_batch *b, int32_t stream_id, const uint8_t *d_frames, int32_t n_frames,
                     int32_t reset, void *stream);

/* fizi_set_tracking for stream stream_id of the batch (one frame per step,
 * so tracked streams keep the batch's parallel component stage). */
int fizi_batch_set_tracking(fizi_batch *b, int32_t stream_id, int32_t enable);

/* relearn_background for stream stream_id of the batch. */
int fizi_batch_relearn(fizi_batch *b, int32_t stream_id, const uint8_t *d_frames, int32_t n_frames,
                       const uint64_t *d_fizi_bits, void *stream);

/* One frame step. h_frames: host array of n_streams device frame pointers,
 * NULL for a stream with no frame this step. h_fizi_bits: NULL, or a host
 * array of n_streams device bit-mask pointers (entries may be NULL).
 * d_pointers: device array of n_streams pointers; entry i is written when
 * stream i has a frame. FIZI_ESTATE if an active stream has no model. Async. */
int fizi_batch_step(fizi_batch *b, const uint8_t *const *h_frames, uint64_t *const *h_fizi_bits,
                    fizi_pointer *d_pointers, void *stream);

/* In the pipelined modes a step's I_FIZI bits and pointers are written by
 * the NEXT call that enqueues work on the batch: its next step (on that
 * step's stream) or fizi_batch_flush. They are complete once that call's
 * work has completed on its stream; until then the caller keeps the step's
 * frame, bit-mask and pointer buffers alive and unread. Results are the same
 * as in every other mode. fizi_batch_flush enqueues the pending half-step on
 * `stream` (nothing to do in the other modes, or when nothing is pending).
 * Learning, re-learning and the calls below that wait for pending steps
 * flush first. Async. */
int fizi_batch_flush(fizi_batch *b, void *stream);

/* Selects how steps are launched (FIZI_BATCH_*); waits for pending steps. */
int fizi_batch_set_mode(fizi_batch *b, int32_t mode);

/* Waits for all steps and returns (and clears) the error word: non-zero when
 * a persistent step gave up one of its bounded waits (its outputs are then
 * not valid). */
int fizi_batch_status(fizi_batch *b, uint32_t *h_flags);

/* Offsets of stream stream_id's model inside the batch state block
 * (`total` is 0). */
int fizi_batch_state_layout(fizi_batch *b, int32_t stream_id, fizi_layout *out);

/* Measurement hook of the batch (see fizi_stage_timing); in the persistent
 * modes the fused kernel is reported as stage 1. */
int fizi_batch_stage_timing(fizi_batch *b, int32_t enable);
int fizi_batch_stage_times(fizi_batch *b, double *h_ms, int64_t *h_launches);

/* Launch shapes of a batch. cls_iters: classify tile = 1024 * cls_iters
 * pixels (1, 2, 4, 8; not used by the persistent kernel, whose classify
 * work comes in bands of 4 * morph_rows rows); morph_rows: morphology band
 * height (8, 16, 32, 64); grid_per_cu: resident blocks per CU for the
 * streaming kernels (1..64); mode: FIZI_BATCH_*; short_bands (0, 1; 1 when
 * the batch is created): a step too small to fill the device - its frames'
 * morphology in 4-row bands of one wave each needs at most one wave per
 * SIMD, as with the few active streams of a serving step - takes that
 * shape instead of morph_rows in the four-kernel modes (its length is then
 * one wave's chain of rows, not the work); 0 keeps morph_rows for every
 * step. Results do not depend on them. */
typedef struct {
    int32_t cls_iters;
    int32_t morph_rows;
    int32_t grid_per_cu;
    int32_t mode;
    int32_t short_bands;
} fizi_tuning;

int fizi_batch_get_tuning(fizi_batch *b, fizi_tuning *out);
/* Waits for pending steps; FIZI_EINVAL for a shape outside the ranges. */
int fizi_batch_set_tuning(fizi_batch *b, const fizi_tuning *t);

/* Autotuner (the paper's Section 3.3 tunes its GPU memory use dynamically;
 * here the launch shapes are tuned on the caller's workload): times `steps`
 * frame steps of h_frames twice (as in fizi_batch_step, after two warm-up
 * steps) for each candidate of a coordinate sweep - mode, then cls_iters,
 * then grid_per_cu, then morph_rows - keeps the fastest by the better of its
 * two times (a candidate replaces the current shape only when at least 1%
 * faster, so that shapes within timing noise of each other leave it where
 * it is; the sweep's pick is then timed against the starting shape three
 * more times, in turn, and kept only if still 1% faster), leaves it set,
 * and returns it with its milliseconds per step. Synchronous. */
int fizi_batch_autotune(fizi_batch *b, const uint8_t *const *h_frames, fizi_pointer *d_pointers,
                        int32_t steps, void *stream, fizi_tuning *best, double *best_ms);

/* Waits for the batch's work and releases its host resources. A pipelined
 * step still pending (not flushed) is dropped. */
int fizi_batch_destroy(fizi_batch *b);

/* ---- Differentiable form (calibration) -------------------------------------
 * A soft, sigmoid-relaxed skin mask and its hand-written adjoint, used to
 * calibrate a chroma skin model from ground-truth masks. Not in the paper,
 * whose skin test is the hard hue interval of Section 3.1 (iii); the hard
 * path above is unchanged by it. For each RGB pixel (uint8, interleaved):
 *   Cb = 128 - 0.168736 R - 0.331264 G + 0.5 B,
 *   Cr = 128 + 0.5 R - 0.418688 G - 0.081312 B       (BT.601 full range),
 *   d  = sqrt(delta^T S^-1 delta), delta = (Cb - mu_b, Cr - mu_r),
 *   m  = sigmoid((theta - d) / T),
 * with params6 = {mu_b, mu_r, s_bb, s_br, s_rr, theta} (host floats; S =
 * [[s_bb, s_br], [s_br, s_rr]] must be positive definite) and T > 0. The
 * per-pixel arithmetic is FP32; sums are FP64 in a fixed order, so results
 * are bitwise reproducible. Where d = 0 the distance contributes no
 * gradient. d_frames is 4-byte aligned, npx >= 1 pixels. */

/* m for npx pixels into d_mask (FP32, 16-byte aligned). Async. */
int fizi_soft_forward(const uint8_t *d_frames, int64_t npx, const float params6[6], float T,
                      float *d_mask, void *stream);

/* Measurement hook of the soft-mask calls (process-wide): with enable != 0
 * each kernel launch records a HIP event pair from its own dispatch (at most
 * 16384 per kernel between two reads); fizi_soft_times() waits for them,
 * returns the summed milliseconds and launch counts per kernel, and clears
 * them. Kernels: 0 the forward mask, 1 the per-block adjoint (or fused BCE)
 * sums, 2 the final fixed-order reduction. */
enum { FIZI_SOFT_STAGE_FORWARD = 0, FIZI_SOFT_STAGE_BACKWARD, FIZI_SOFT_STAGE_FINAL, FIZI_SOFT_NSTAGES };
int fizi_soft_timing(int32_t enable);
int fizi_soft_times(double *h_ms /* [FIZI_SOFT_NSTAGES] */, int64_t *h_launches /* [FIZI_SOFT_NSTAGES] */);

/* Device workspace bytes the two calls below need (caller-owned). */
size_t fizi_soft_workspace_bytes(int64_t npx);

/* Given dL/dm per pixel (FP32), writes dL/dparams6 to d_grad6 (6 doubles,
 * device). Async. */
int fizi_soft_backward(const uint8_t *d_frames, const float *d_dLdm, int64_t npx,
                       const float params6[6], float T, void *d_workspace, size_t workspace_bytes,
                       double *d_grad6, void *stream);

/* Fused loss and gradient against a ground-truth mask d_gt (uint8 0/1 per
 * pixel): L = mean binary cross-entropy of m; d_out7 receives the 6
 * gradients of L followed by L (7 doubles, device). Async. */
int fizi_soft_bce(const uint8_t *d_frames, const uint8_t *d_gt, int64_t npx, const float params6[6],
                  float T, void *d_workspace, size_t workspace_bytes, double *d_out7, void *stream);

/* For callers that cannot allocate device memory (work under hipGraph
 * capture, serving loops or harnesses that forbid hipMalloc): fizi_soft_bce
 * without a workspace argument. Its per-block partial sums go to a
 * 128 KiB array the library holds on each GPU (a static device array, kept
 * until the process ends); the call allocates nothing (no hipMalloc, no
 * library allocation). The array holds one row of 8 partial sums for each
 * of the at most 2048 blocks a launch uses, whatever npx is; a launch that
 * would need more is refused with FIZI_ENOMEM. Same arguments, results (bit
 * for bit) and errors as fizi_soft_bce otherwise. Every call on one GPU uses
 * the same array and it keeps the last call's contents (each block writes
 * its row before the final sum reads it, so nothing needs clearing): calls
 * that overlap on a GPU (on different streams, or from several threads
 * without ordering) race and give undefined results; order them on one
 * stream. Async. */
int fizi_soft_bce_static(const uint8_t *d_frames, const uint8_t *d_gt, int64_t npx, const float params6[6],
                         float T, double *d_out7, void *stream);

/* ---- The pointer's consumers (host) ---------------------------------------
 * A pointer's position is its centroid pixel (floor(sum_x / area),
 * floor(sum_y / area)); a frame without a hand has none. */

/* An inclusive rectangle of image pixels. */
typedef struct {
    int32_t x0, y0, x1, y1;
} fizi_zone;

/* Interface module (Section 2: "the interface zone activated by the
 * pointer"): h_zone[i] = the first zone, in array order, that holds pointer
 * i's position, or -1 (no hand, or no zone holds it). Host arrays owned by
 * the caller (n pointers in, n zone indices out); synchronous, no GPU work.
 * FIZI_EINVAL for a negative count or a null array with a nonzero count. */
int fizi_zone_hit(const fizi_pointer *h_pointers, int32_t n, const fizi_zone *h_zones, int32_t n_zones,
                  int32_t *h_zone);

/* A virtual wheel centred at (cx, cy): positions at a distance in
 * [r_min, r_max] are on it; no steering within +-dead_cdeg of 12 o'clock,
 * full lock at +-full_cdeg (0 <= dead_cdeg < full_cdeg <= 18000). */
typedef struct {
    int32_t cx, cy, r_min, r_max;
    int32_t dead_cdeg, full_cdeg;
} fizi_wheel;

typedef struct {
    int32_t on_wheel;          /* 1 when the position lies on the wheel */
    int32_t angle_cdeg;        /* from 12 o'clock, clockwise > 0, in (-18000, 18000],
                                  rounded half away from zero */
    int32_t steer_permille;    /* 0 in the dead zone, then linear to +-1000 at full lock;
                                  < 0 is left */
    int32_t accelerate;        /* the pointer's click (closed palm) */
} fizi_drive;

/* Driving application (Section 4: the hand turns an imaginary wheel that
 * controls left, right and speed): one fizi_drive per pointer (all zero off
 * the wheel or without a hand). Host arrays owned by the caller; synchronous,
 * no GPU work. FIZI_EINVAL for a negative count, a null argument or a wheel
 * outside the ranges above. */
int fizi_drive_of(const fizi_pointer *h_pointers, int32_t n, const fizi_wheel *wheel, fizi_drive *h_out);

/* Message of the last failed call on this thread ("" if none). */
const char *fizi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FIZI_H */
