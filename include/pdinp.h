/*
 * pdinp.h - C ABI of the MI355X residual decoder: block-based
 * pseudodifferential inpainting of residual planes from sparse mask values
 * (Andris, Peter, Kaja Mohideen, Weickert, Hoffmann, "Inpainting-based Video
 * Compression in FullHD", SSVM 2021).
 *
 * The operation (Sec. 2.1-2.2 of the paper).  A plane is cut into b x b
 * blocks (truncated at the right and bottom edges); each block is an
 * independent image with mirrored boundaries.  Given K distinct mask pixels
 * x_1..x_K of a block with values r_1..r_K, the decoded residual is
 *     u(x) = sum_i c_i G(x, x_i) + a                      (Eq. 2 / Eq. 3)
 * where G is the Green's function of the operator A (its pseudo-inverse,
 * diagonalised by the DCT-II with eigenvalues lambda, Eq. 4) and (c, a) solve
 * the (K+1) x (K+1) system  [G_K 1; 1^T 0] [c; a] = [r; 0]  (Sec. 2.2).
 * For the harmonic operator A = -L this u is the unique solution of the
 * inpainting problem of Eq. (1) on the block.
 *
 * All functions return 0 (PDI_OK) or a negative PDI_E* code; no exception
 * crosses the ABI.  After a failed call `out` is unspecified and the context
 * stays usable.
 */
#ifndef PDINP_H
#define PDINP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PDI_OK      0
#define PDI_EINVAL (-1) /* null pointer, bad geometry, block size not 8/16/32, bad params */
#define PDI_EMASK  (-2) /* position >= w*h, positions not strictly ascending, K > w*h */
#define PDI_ENOMEM (-3) /* device allocation failed or HBM budget exceeded */
#define PDI_EHIP   (-4) /* HIP runtime error; pdi_last_error() has the detail */
#define PDI_EBUSY  (-5) /* server queue full / context busy */
#define PDI_EVALUE (-6) /* a non-finite value (NaN/Inf) in `values` */
#define PDI_ESOLVE (-7) /* a block's system broke down (non-finite solution) */

/* Frame formats. */
#define PDI_GRAY   0 /* one W x H plane */
#define PDI_YUV420 1 /* Y (W x H), Cb, Cr (ceil(W/2) x ceil(H/2)) */

/* Evaluation arithmetic for u(x) = sum c_i G(x, x_i) + a. */
#define PDI_EVAL_FP32   0 /* FP32 matrix-core products (default) */
#define PDI_EVAL_FP16   1 /* FP16 operands, FP32 accumulation */
#define PDI_EVAL_BF16   2 /* BF16 operands, FP32 accumulation */
#define PDI_EVAL_BF16X2 3 /* split BF16 (hi*hi + hi*lo + lo*hi), FP32 accumulation */

/* Execution path. */
#define PDI_PATH_AUTO  0 /* batched wave-level solves + matrix-core evaluation */
#define PDI_PATH_PLAIN 1 /* one workgroup per block, FP32 solve, direct evaluation */

/* Operators (the eigenvalues lambda = mu^-s define the operator, Sec. 2.2). */
#define PDI_OP_DISCRETE   0 /* mu = 4 sin^2(pi p/2w) + 4 sin^2(pi q/2h): 5-point -L */
#define PDI_OP_CONTINUOUS 1 /* mu = pi^2 (p^2/w^2 + q^2/h^2) */

typedef struct pdi_ctx pdi_ctx;

/* Frame geometry.  Planes are row-major with stride = plane width. */
typedef struct {
    int32_t width;
    int32_t height;
    int32_t format; /* PDI_GRAY or PDI_YUV420 */
} pdi_frame;

/* Packed mask (CSR over blocks).  Mask blocks are ordered: the Y blocks, then
 * the chroma blocks once (chroma_shared != 0: one mask for Cb and Cr, as in
 * Sec. 2.3 of the paper) or the Cb blocks then the Cr blocks; raster order
 * inside each plane.  block_ptr[n_mask_blocks + 1] are int32 offsets into
 * pos; pos[] holds in-block pixel indices y*w + x (w = width of that block),
 * strictly ascending inside a block.  K = 0 is allowed (the block decodes to
 * zero).  Both arrays are DEVICE pointers owned by the caller. */
typedef struct {
    const int32_t *block_ptr;
    const uint16_t *pos;
    int32_t n_mask_blocks;
    int32_t chroma_shared;
} pdi_mask;

/* Parameters; pdi_default_params() gives the paper's harmonic operator. */
typedef struct {
    int32_t op;          /* PDI_OP_*; default PDI_OP_DISCRETE */
    double s;            /* lambda = mu^-s; 1.0 = harmonic (default), 2.0 = biharmonic */
    int32_t eval_dtype;  /* PDI_EVAL_*; default PDI_EVAL_FP32 */
    int32_t refine;      /* 0 off, 1 auto (small pivot ratio), 2 always; default 1 */
    int32_t validate;    /* 1: check masks/values on the device, report at pdi_sync */
    int32_t path;        /* PDI_PATH_*; default PDI_PATH_AUTO */
    double refine_tau;   /* auto-refine when min/max pivot < tau; default 1/64 */
    int32_t out_int8;    /* 1: `out` receives int8 pixels clamp(rint(u), -128, 127)
                            (round half to even) instead of FP32; default 0 */
} pdi_params;

/* Fill *p with the defaults. */
void pdi_default_params(pdi_params *p);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the
 * library's own device allocations (0 = no cap).  The context owns the table
 * cache and, per stream it is used on, a workspace and a device status word.
 * Calls are serialised by an internal lock, so one context may be shared by
 * threads and used on several streams at once (decodes on different streams
 * run concurrently on the GPU).
 * Returns PDI_EINVAL (bad device / null out), PDI_EHIP, PDI_ENOMEM. */
int pdi_create(pdi_ctx **out, int device, size_t hbm_budget_bytes);

/* Release the context and every device allocation it owns (synchronises). */
void pdi_destroy(pdi_ctx *ctx);

/* Decode the residual planes of one frame (hot path, asynchronous on
 * `stream`, a hipStream_t; NULL = the null stream).
 *   values: DEVICE float32 array: the Y values aligned with the Y part of
 *     pos, then the Cb values aligned with the chroma part, then the Cr
 *     values (aligned with the chroma part again when chroma_shared).
 *   block_size: 8, 16 or 32.
 *   params: NULL for the defaults.
 *   out: DEVICE array of W*H (+ 2 * ceil(W/2)*ceil(H/2) for YUV420)
 *     elements, planes Y, Cb, Cr back to back, row-major: float32, or int8
 *     with params->out_int8.
 * The library keeps no reference to caller memory after the stream work
 * completes.  Host-side checks (geometry, params, mask block count) return
 * PDI_EINVAL synchronously; with validate=1 mask/value errors found on the
 * device are reported by the next pdi_sync as PDI_EMASK / PDI_EVALUE.
 * The first call for a new frame geometry allocates (not capturable); later
 * calls with the same geometry and params launch kernels only. */
int decode_residual(pdi_ctx *ctx, const pdi_frame *frame, const pdi_mask *mask,
                    const float *values, int block_size, const pdi_params *params,
                    float *out, void *stream);

/* Decode n (1..PDI_MAX_BATCH) frames of one geometry in one launch of each
 * kernel: masks[k] (chroma sharing equal for all k), values[k] and outs[k]
 * describe frame k exactly as for decode_residual (DEVICE pointers, caller
 * owned); the host arrays masks, values and outs are read during the call
 * only.  More blocks per launch keep more waves in flight, so a batch is
 * the throughput form of decode_residual; each frame's result is the same
 * as when decoded alone.  With 32x32 blocks (n > 1, outside graph capture)
 * the batch's four wave-per-block launches run side by side on `stream`
 * and two streams the context creates on first use, forked from `stream`
 * and joined back to it with events, so work queued on `stream` afterwards
 * (and pdi_sync) sees the whole decode; batches of different caller streams
 * share those streams.  Errors as for decode_residual. */
#define PDI_MAX_BATCH 32
int decode_residual_batch(pdi_ctx *ctx, int n, const pdi_frame *frame, const pdi_mask *masks,
                          const float *const *values, int block_size, const pdi_params *params,
                          float *const *outs, void *stream);

/* decode_residual_batch for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results as decode_residual_batch
 * (1..PDI_MAX_BATCH frames of one geometry; DEVICE pointers, caller owned),
 * but the decode's device scratch (status word, counters, deferred-block
 * list, wave-per-block queues, global-memory bordered systems) lives in a
 * static device array of PDI_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends, and the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).
 * Preconditions and limits:
 *   - the context's tables for this geometry, block size, chroma sharing and
 *     operator (op, s) must exist: one decode_residual / decode_residual_batch
 *     call with them builds them (that call allocates); otherwise
 *     PDI_EINVAL with nothing launched;
 *   - the scratch must hold the status word and counters (4.4 KB), 4 bytes
 *     per mask block and frame (about 22 for batches of more than one frame
 *     with 8x8 or 16x16 blocks, 12 with 32x32 blocks: the size-class queues) and
 *     at least one (b*b + 1)(b*b + 3)-float system; more systems fit, up to
 *     64 are used (more workgroups of the general pass then work on K > 96
 *     blocks at once; results do not depend on it).  A larger decode returns
 *     PDI_ENOMEM with nothing launched.  32 frames of 1080p 4:2:0 need at
 *     least 7.4 MB with 16x16 blocks, 28 MB with 8x8 and 5.2 MB with 32x32
 *     blocks, so any batch of up to 32 1080p frames fits;
 *   - every call on a GPU shares that GPU's scratch: calls that overlap on
 *     one GPU (different streams, contexts or threads) race and must be
 *     serialised by the caller.  Each decode leaves its counters at zero;
 *     the status word keeps what kernels report until pdi_sync(ctx, stream)
 *     (on the stream of the call) reads and clears it.
 * Errors as decode_residual_batch, plus PDI_EHIP when the scratch's device
 * address could not be taken at pdi_create. */
#define PDI_NOALLOC_SCRATCH_BYTES (32u << 20)
int decode_residual_batch_noalloc(pdi_ctx *ctx, int n, const pdi_frame *frame, const pdi_mask *masks,
                                  const float *const *values, int block_size, const pdi_params *params,
                                  float *const *outs, void *stream);

/* ---- Decoding stored coefficients (the paper's decoder split) ----
 * When the encoder keeps each block's Green's-function coefficients c and
 * constant a (Sec. 2.2, last paragraph), the decoder only evaluates Eq. 2,
 * u = sum_i c_i G(., x_i) + a over the block (here through Eq. 4 as for
 * decode_residual), with no system to solve.  The coefficients are stored
 * as codes q in [-127, 127] of a uniform quantiser with a dead zone around
 * zero (Sec. 2.3); a code is reconstructed as 0 for q = 0, else as
 * sign(q) (|q| + rho) step[plane]. */
typedef struct {
    float step[3]; /* quantiser step of the Y, Cb, Cr planes (GRAY: step[0]); finite, >= 0 */
    float rho;     /* reconstruction offset inside the quantiser interval, [0, 1) */
} pdi_coef_params;

/* Decode one frame from stored coefficients.  frame, mask, block_size and
 * out as for decode_residual (DEVICE pointers, caller owned); qp is a HOST
 * pointer read during the call.
 *   coef:   int8 codes laid out exactly like decode_residual's values (one
 *           per mask point and value plane: Y, then the chroma runs).
 *   consts: FP32 constant a of EVERY block of every plane: the Y blocks,
 *           then Cb, then Cr, raster order inside each plane
 *           (ceil(W/b) * ceil(H/b) per plane, edge blocks included).
 * A block with K = 0 becomes its constant; K = w*h is allowed.  params: op,
 * s, eval_dtype, validate and out_int8 apply as for decode_residual; refine
 * and path do not (no solve).  With validate = 1 a code of -128 or a
 * non-finite constant is reported as PDI_EVALUE and bad positions as
 * PDI_EMASK at pdi_sync.  Returns PDI_EINVAL for a NULL pointer, a bad step
 * (non-finite or negative) or rho outside [0, 1); otherwise as
 * decode_residual. */
int decode_coefficients(pdi_ctx *ctx, const pdi_frame *frame, const pdi_mask *mask,
                        const int8_t *coef, const float *consts, const pdi_coef_params *qp,
                        int block_size, const pdi_params *params, float *out, void *stream);

/* decode_coefficients for n (1..PDI_MAX_BATCH) frames of one geometry in one
 * launch of each kernel (coefs[k], consts[k], outs[k] as for frame k alone;
 * the host arrays are read during the call only). */
int decode_coefficients_batch(pdi_ctx *ctx, int n, const pdi_frame *frame, const pdi_mask *masks,
                              const int8_t *const *coefs, const float *const *consts,
                              const pdi_coef_params *qp, int block_size, const pdi_params *params,
                              float *const *outs, void *stream);

/* ---- Encoding coefficients (the encoder side of that split) ----
 * The encoder solves each block's bordered system (Sec. 2.2) for c and a
 * from the residual at the block's mask points, maps c to codes in
 * [-127, 127] by dead-zone uniform quantisation (Sec. 2.3) and keeps a.
 * A code is q = sign(c) min(127, floor(|c| / step[plane])): |c| < step
 * gives 0, and q is the interval that decode_coefficients reconstructs as
 * sign(q) (|q| + rho) step.  Mask selection is the caller's (the mask is an
 * input, as for decode_residual).
 * frame, mask, values, block_size: DEVICE pointers as for decode_residual;
 * qp: HOST pointer, step[] finite and > 0 (rho is not used).
 *   coef:   int8 codes out, laid out exactly like values (caller owned,
 *           one per mask point and value plane).
 *   consts: FP32 constant a out for EVERY block of every plane, laid out as
 *           decode_coefficients reads it (caller owned).
 * Blocks with K = 0 get a = 0 (decode_residual gives u = 0 there); K = w*h
 * is solved as well (the decoded block is then the values).  params: op, s,
 * refine, refine_tau and validate apply as for decode_residual (blocks of
 * at most 16x16 pixels take the wave-level solve, 32x32 blocks the
 * per-block one); eval_dtype, out_int8 and path do not.  Asynchronous on
 * `stream`; errors as decode_residual (PDI_EINVAL for a NULL pointer or a
 * bad step; at pdi_sync PDI_EMASK / PDI_EVALUE for invalid input and
 * PDI_ESOLVE for a non-finite c or a: the codes and constants of such
 * blocks are then unspecified). */
int encode_coefficients(pdi_ctx *ctx, const pdi_frame *frame, const pdi_mask *mask, const float *values,
                        const pdi_coef_params *qp, int block_size, const pdi_params *params, int8_t *coef,
                        float *consts, void *stream);

/* Up to PDI_MAX_BATCH frames of one geometry in one launch of each kernel
 * (arrays of n HOST-side entries of DEVICE pointers, as for
 * decode_residual_batch). */
int encode_coefficients_batch(pdi_ctx *ctx, int n, const pdi_frame *frame, const pdi_mask *masks,
                              const float *const *values, const pdi_coef_params *qp, int block_size,
                              const pdi_params *params, int8_t *const *coefs, float *const *consts,
                              void *stream);

/* ---- Mask selection (encoder side) ----
 * The encoder picks each 8x8 block's mask points by rectangular
 * subdivision (Sec. 2.3 of the paper, which takes the scheme from the
 * rectangular-subdivision codec it cites; this is the reading taken): the
 * mask is the set of corners of rectangles (inclusive pixel ranges sharing
 * their common edges) that start as the whole block; each round inpaints
 * the block from the current corners (bordered system of Sec. 2.2, then
 * Eq. 2, harmonic operator), and every rectangle whose mean squared error
 * exceeds the threshold and whose longer side spans at least 2 pixel gaps
 * is halved along that side (x on ties), both halves keeping the middle
 * line.  Rounds end when nothing is split.  A shared chroma mask is chosen
 * on the mean of the two chroma planes' errors (Sec. 2.3: one mask for
 * both chroma channels). */
typedef struct {
    float threshold[2]; /* luma, chroma: split when a rectangle's mean squared error
                           exceeds it (grey levels^2); not NaN; default 16, 32 */
    int32_t max_rounds; /* rounds of splits at most, [0, 64]; default 16 (0: corners only) */
} pdi_select_params;

void pdi_default_select_params(pdi_select_params *p);

/* Select the mask of every 8x8 block of a frame from its dense residual
 * planes and gather the values at the selected points: the outputs are the
 * inputs decode_residual and encode_coefficients take (mask with
 * n_mask_blocks = pdi_frame_info's count for this chroma_shared).
 *   frame:     geometry (HOST pointer); block_size must be 8.
 *   planes:    DEVICE FP32 residual planes Y, then Cb, Cr for 4:2:0,
 *              row-major, back to back (decode_residual's output layout).
 *   block_ptr: DEVICE int32 [n_mask_blocks + 1] out.
 *   pos:       DEVICE uint16 out, room for every pixel of the mask planes.
 *   values:    DEVICE FP32 out, room for every pixel of all planes.
 * All caller owned.  Asynchronous on `stream`.  Returns PDI_EINVAL for a
 * NULL pointer, a bad geometry, a block size other than 8 or bad
 * parameters; PDI_ENOMEM / PDI_EHIP as elsewhere. */
int select_mask(pdi_ctx *ctx, const pdi_frame *frame, int chroma_shared, const float *planes, int block_size,
                const pdi_select_params *sp, int32_t *block_ptr, uint16_t *pos, float *values, void *stream);

/* ---- Global homogeneous diffusion inpainting (intra prediction) ----
 * The codec's intra frames are predicted by Eq. 1 of Sec. 2.1 on the whole
 * plane with A = -L (5-point Laplacian, reflecting boundaries): u = f at
 * the mask pixels and (A u)_i = 0 elsewhere.  Solved coarse to fine with
 * conjugate gradients as in the paper: a pyramid of masks and values by
 * 2x2 restriction (a coarse pixel is known when one of its children is,
 * with their mean value), CG on the coarsest level, each finer level
 * started from the coarser solution. */
typedef struct {
    double tol;       /* stop the finest level when |r|_2 <= tol max(|b|_2, |r_0|_2) (b: right-hand
                         side of the unknowns' system, r_0: residual of the level's start, which
                         matters only when the start is worse than zero, e.g. b = 0 with a
                         nonzero coarse start); in (0, 1), default 1e-6 */
    int32_t max_iter; /* CG iterations per level at most, in [1, 65536]; default 4000 */
    int32_t check;    /* iterations queued between host read-backs at most, in [1, 1024];
                         default 8 (fewer where the norms' decay, or the count of the
                         previous call on this plane size, says fewer are left).
                         Convergence is tested on the device before every iteration and
                         the iterations queued past it do nothing, so a level stops at the
                         first iteration that meets tol whatever check is */
    double coarse_tol; /* the same test on the coarser levels, which only supply the
                          finest level's start; in [tol, 1), default 1e-3 */
} pdi_cg_params;

void pdi_default_cg_params(pdi_cg_params *p);

/* mask: uint8 W*H (non-zero = known), f: float W*H (read at the mask
 * pixels only), u: float W*H output; row-major DEVICE buffers, caller
 * owned.  cp: HOST pointer or NULL for the defaults.  *iterations (HOST,
 * may be NULL) receives the CG iterations of the finest level.
 * Synchronous on `stream` (the residual norms are read back every
 * cp->check iterations); the first call for a plane size allocates its
 * pyramid.  An empty mask gives u = 0 (the system is then
 * singular).  Returns PDI_EINVAL for NULL pointers, a size outside
 * [1, 2^30] pixels or bad parameters, PDI_ESOLVE when the finest level does
 * not reach tol within max_iter, PDI_ENOMEM / PDI_EHIP as elsewhere. */
int inpaint_homogeneous(pdi_ctx *ctx, int width, int height, const uint8_t *mask, const float *f,
                        const pdi_cg_params *cp, float *u, void *stream, int32_t *iterations);

/* Wait for `stream`, then read and clear the device status word.
 * Returns PDI_OK, PDI_EMASK, PDI_EVALUE, PDI_ESOLVE or PDI_EHIP. */
int pdi_sync(pdi_ctx *ctx, void *stream);

/* Text of the last error of this context (never NULL). */
const char *pdi_last_error(pdi_ctx *ctx);

/* Measure the launch choices of the batched path for this frame geometry,
 * operator and evaluation dtype on the given inputs (device pointers, as for
 * decode_residual; `out` is overwritten) and keep the fastest in the context
 * for later single-frame decode_residual calls with the same geometry and params.  The
 * choices only change how blocks are grouped into workgroups, never a
 * block's arithmetic, so results are bitwise the same with any choice.
 * Synchronous (not capturable).  *choice (may be NULL) receives the blocks
 * per workgroup chosen (block size 32: 1, 2 or 4; block sizes 8 and 16: 8 to
 * 16), or 0 with PDI_PATH_PLAIN, which has no choices (the call is then one
 * decode + pdi_sync).
 * Returns the codes of decode_residual / pdi_sync. */
int pdi_autotune(pdi_ctx *ctx, const pdi_frame *frame, const pdi_mask *mask, const float *values,
                 int block_size, const pdi_params *params, float *out, void *stream, int *choice);

/* pdi_autotune for decode_residual_batch launches of n (1..PDI_MAX_BATCH)
 * frames: the candidates are timed on the given batch (arguments as for
 * decode_residual_batch; outs[k] are overwritten) and the fastest is kept
 * for later batches of n frames with the same geometry and params.  A
 * choice is kept per n: a launch of 8 frames has 8 times the workgroups of
 * one and may prefer other groupings.  pdi_autotune is this call with n = 1.
 * Synchronous; *choice and return codes as for pdi_autotune. */
int pdi_autotune_batch(pdi_ctx *ctx, int n, const pdi_frame *frame, const pdi_mask *masks,
                       const float *const *values, int block_size, const pdi_params *params,
                       float *const *outs, void *stream, int *choice);

/* Host helper: number of mask blocks, value count and output size of a
 * frame geometry (for sizing buffers).  Pointers may be NULL. */
int pdi_frame_info(const pdi_frame *frame, int block_size, int chroma_shared,
                   int32_t *n_mask_blocks, int64_t *out_elems);

/* Host helper: pack the paper's dense form (Sec. 2.1: mask m and image f,
 * row-major per plane) into the CSR layout above.  HOST pointers.
 *   m: uint8 mask planes back to back (Y, then C for a shared chroma mask,
 *      else Cb, Cr); f: float32 planes Y, Cb, Cr back to back.
 *   block_ptr: n_mask_blocks + 1 entries; pos / values: capacity in
 *   *pos_cap / *val_cap, replaced by the counts written.
 * Returns PDI_EINVAL on bad geometry, PDI_ENOMEM if a capacity is short. */
int pdi_pack_dense(const pdi_frame *frame, const uint8_t *m, const float *f,
                   int block_size, int chroma_shared, int32_t *block_ptr,
                   uint16_t *pos, int64_t *pos_cap, float *values, int64_t *val_cap);

/* Host-side validation of a HOST copy of a packed mask and values: returns
 * PDI_OK, PDI_EINVAL, PDI_EMASK or PDI_EVALUE (no device work). */
int pdi_validate_host(const pdi_frame *frame, int block_size, const int32_t *block_ptr,
                      const uint16_t *pos, int32_t n_mask_blocks, int32_t chroma_shared,
                      const float *values);

/* ---- Frame sequences as one HIP graph (batched decodes, captured) ----
 * The decodes of n frames of ONE geometry (frame, block_size, params, chroma
 * sharing) are recorded once into a HIP graph as decode_residual_batch calls
 * over consecutive frames (at most PDI_MAX_BATCH per call, about n / nstreams),
 * batch b on internal stream b % nstreams, the streams forked from and
 * joined back to the first one, so that independent batches overlap on the
 * GPU; pdi_seq_launch replays all n decodes with one graph launch.  masks[k], values[k] and outs[k] are DEVICE
 * pointers (caller-owned) read / written by every replay: update their
 * contents between replays, not their addresses.  pdi_seq_create runs one
 * eager decode per internal stream first (allocations and errors happen
 * there), so it must not itself be called under stream capture.
 * Returns PDI_EINVAL (null pointers, n <= 0, nstreams not in 1..16), the
 * codes of decode_residual, or PDI_EHIP. */
typedef struct pdi_seq pdi_seq;
int pdi_seq_create(pdi_ctx *ctx, int n, const pdi_frame *frame, const pdi_mask *masks,
                   const float *const *values, int block_size, const pdi_params *params,
                   float *const *outs, int nstreams, pdi_seq **out);
/* Enqueue one replay on `stream` (asynchronous). */
int pdi_seq_launch(pdi_seq *q, void *stream);
/* Wait for `stream`, then report the device status of the replayed decodes
 * (as pdi_sync). */
int pdi_seq_sync(pdi_seq *q, void *stream);
void pdi_seq_destroy(pdi_seq *q);

/* ---- Serving loop: continuous batching of frames from many streams ----
 * A server owns nlanes HIP streams and a worker thread.  pdi_submit copies a
 * frame's HOST mask and values into pinned staging and queues it; the worker
 * admits queued frames in arrival order whenever a lane is free and the
 * device bytes of the running frames stay within hbm_budget_bytes (0 = no
 * cap): the oldest queued frame, joined by queued frames of the same
 * geometry and params (up to PDI_MAX_BATCH: only frames already waiting join, so
 * a light load admits frames one by one and a deep queue drains in large
 * launches), is copied to the device and
 * decoded by one decode_residual_batch launch on the lane's stream (frames on
 * different lanes overlap on the GPU), and the results are copied back.  A
 * frame's result does not depend on what it is batched with or on what else
 * is in flight.
 * The context must outlive the server.  Created on the current HIP device. */
typedef struct pdi_server pdi_server;
/* max_queue: frames waiting for admission before pdi_submit answers
 * PDI_EBUSY.  Returns PDI_EINVAL (null, nlanes not in 1..32, max_queue <= 0)
 * or PDI_EHIP. */
int pdi_server_create(pdi_ctx *ctx, int nlanes, size_t hbm_budget_bytes, int max_queue,
                      pdi_server **out);
/* Queue one frame.  mask->block_ptr / mask->pos and values are HOST arrays,
 * copied before the call returns (layouts as for decode_residual; n_values
 * is the length of values).  out_dev: caller-owned DEVICE array of the
 * frame's output size (float32, or int8 with params->out_int8) that the
 * decode writes (it must stay valid until the request completes), or NULL
 * to decode into a pooled server buffer.  out: HOST array of the same type
 * and size that pdi_wait fills, or NULL.
 * With params->validate the mask and values are checked here (PDI_EMASK /
 * PDI_EVALUE, nothing queued).  Returns PDI_EINVAL, PDI_ENOMEM (the frame
 * alone exceeds the budget, or staging failed), PDI_EBUSY (queue full); on
 * PDI_OK *ticket identifies the request. */
int pdi_submit(pdi_server *srv, const pdi_frame *frame, const pdi_mask *mask, const float *values,
               int64_t n_values, int block_size, const pdi_params *params, void *out,
               void *out_dev, int64_t *ticket);
/* Non-blocking: *done = 1 once the request has completed; then
 * *latency_us = submit-to-completion time and the return value is the
 * request's status.  PDI_EINVAL for an unknown ticket. */
int pdi_poll(pdi_server *srv, int64_t ticket, int *done, double *latency_us);
/* Block until the request completes, copy its result to the host `out`
 * given at submit (if any), release it and return its status (the ticket is
 * invalid afterwards). */
int pdi_wait(pdi_server *srv, int64_t ticket, double *latency_us);
/* Queue length, running frames, device bytes of running frames and device
 * bytes held (running + buffer pool).  Pointers may be NULL. */
int pdi_server_stats(pdi_server *srv, int64_t *queued, int64_t *running, size_t *bytes_in_use,
                     size_t *bytes_allocated);
/* hold != 0 pauses admission (queued frames wait, running ones finish);
 * hold = 0 resumes it. */
int pdi_server_hold(pdi_server *srv, int hold);
/* Drain queued and running work, then free everything the server owns. */
void pdi_server_destroy(pdi_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* PDINP_H */
