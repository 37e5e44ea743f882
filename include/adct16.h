/*
 * adct16.h - C ABI of the MI355X (gfx950) library for the orthogonal 16-point
 * approximate DCT of da Silveira, Cintra, Bayer, Coelho, Kulasekera,
 * Madanayake and Rajapaksha ("An Orthogonal 16-point Approximate DCT for
 * Image and Video Compression").
 *
 * The method (Section 2): T is a 16x16 matrix with entries in {0, +1, -1};
 * T T^T = diag(n) is diagonal, S = diag(1/sqrt(n)) and C_hat = S T is
 * orthogonal.  Eq. (1) factors T into sparse stages costing 60 additions per
 * 16-point transform (Table 1).  Images are cut into disjoint 16x16 blocks
 * and each block A is transformed as B = C_hat A C_hat^T; coefficients are
 * retained or quantised and the block is rebuilt as A' = C_hat^T B' C_hat;
 * quality is measured by PSNR (Section 4).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All functions have C linkage, never throw and return an adct16_status.
 *   adct16_last_error_string() gives a thread-local description of the last
 *   failure of the calling thread.
 * - Device pointers are plain HIP device addresses owned by the caller.  The
 *   library never frees or retains them beyond the call (a graph keeps the
 *   pointers it was created with, see adct16_graph_create).
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *   is enqueued asynchronously; errors the host can detect are returned
 *   before anything is enqueued, and a failed launch returns
 *   ADCT16_E_LAUNCH.  No compute call allocates memory.
 * - A plan owns workspace (per-image SSE accumulators, task partials) that
 *   its measuring calls use; calls on one plan must not overlap (use one
 *   stream per plan, or one plan per stream).  Every call leaves the
 *   workspace ready for the next, so graph replays need no reset.
 * - Images of a batch live in one packed device buffer.  Image k has
 *   height[k] x width[k] pixels; its row y starts at element
 *   offset[k] + y * pitch[k].  Requirements: pitch >= width rounded up to
 *   a multiple of 16; offset*esize and pitch*esize multiples of 16 bytes;
 *   the buffer base 16-byte aligned.  Reconstructions use the same
 *   offsets and pitches as the input (in elements of their own type).
 *   Performance: with pitches, offsets and buffers that are multiples of
 *   128 bytes, every row segment the matrix-core kernel moves is a whole
 *   cache line and it streams with non-temporal accesses; other layouts
 *   give the same results more slowly (adct16_plan_info reports
 *   "rows_line_aligned").
 * - Blocks are numbered in raster order per image; images follow each other.
 *   Coefficient buffers are block-major: block b occupies 256 consecutive
 *   elements, element u*16+v holding coefficient (u, v), u the vertical and
 *   v the horizontal frequency: Z[u][v] = sum_ab T[u][a] A[a][b] T[v][b].
 *   Image k's first block is the sum of the block counts of images < k.
 * - Sizes that are not multiples of 16 are extended by repeating the last
 *   row / column before the transform; reconstructions are written and PSNR
 *   is measured on the true pixels only.
 */
#ifndef ADCT16_H
#define ADCT16_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum adct16_status {
  ADCT16_OK = 0,
  ADCT16_E_NULL = 1,     /* a required pointer argument is NULL */
  ADCT16_E_SHAPE = 2,    /* non-positive size, pitch too small, batch too large */
  ADCT16_E_DTYPE = 3,    /* unsupported dtype or dtype combination */
  ADCT16_E_MODE = 4,     /* r, q, qmode, backend or precision out of range */
  ADCT16_E_ALIGN = 5,    /* pointer, offset or pitch not 16-byte aligned */
  ADCT16_E_NOMEM = 6,    /* plan-time device or host allocation failed */
  ADCT16_E_DEVICE = 7,   /* no device, or the current device is not gfx950 */
  ADCT16_E_LAUNCH = 8,   /* a kernel launch or graph operation failed */
  ADCT16_E_STATE = 9     /* the call does not apply to this plan */
} adct16_status;

typedef enum adct16_dtype {
  ADCT16_U8 = 1,    /* uint8 pixels 0..255 */
  ADCT16_I16 = 2,   /* int16 (residual samples, centred coefficients, levels) */
  ADCT16_I32 = 3,   /* int32 coefficients or levels */
  ADCT16_F32 = 4,   /* float32 scaled coefficients / unrounded reconstruction */
  ADCT16_BF16 = 5,  /* operand precision of the exact DCT-II comparison */
  ADCT16_F16 = 6
} adct16_dtype;

typedef enum adct16_qmode {
  ADCT16_Q_NONE = 0,     /* keep every coefficient (lossless round trip) */
  ADCT16_Q_ZONAL = 1,    /* keep the top-left r x r coefficients, 1 <= r <= 16 */
  ADCT16_Q_ZIGZAG = 2,   /* keep the first r coefficients of the zig-zag scan, 1 <= r <= 256 (Section 4) */
  ADCT16_Q_UNIFORM = 3,  /* uniform step q >= 1 with S folded into one float32 multiplier */
  ADCT16_Q_DEADZONE = 4  /* deadzone quantiser with a QP-scaled step, q = QP in [0, 63]; a
                            stand-in for the video coder's quantiser of Section 5.3 (see
                            qcoef_dtype below) */
} adct16_qmode;

typedef enum adct16_backend {
  ADCT16_BACKEND_AUTO = 0,  /* autotuned (flag ADCT16_FLAG_AUTOTUNE) or the built-in default */
  ADCT16_BACKEND_VALU = 1,  /* 60-addition butterflies of Eq. (1) on the vector ALUs */
  ADCT16_BACKEND_MFMA = 2   /* T as a dense {0,+1,-1} operand of FP16 matrix-core products,
                               every product and sum exact; used by adct16_forward and by
                               the fused call for U8 input, mask modes, U8 (or no) output,
                               no d_qcoef and every image below 2^31 bytes with rows below
                               2^24 bytes; other cases run the VALU kernels */
} adct16_backend;

enum {
  ADCT16_FLAG_AUTOTUNE = 1,      /* time the candidate launch shapes (and, with
                                    ADCT16_BACKEND_AUTO, both backends) of the fused call at
                                    plan creation on scratch buffers (allocates) */
  ADCT16_FLAG_EXPLICIT_COEF = 2, /* matrix-core fused call: form the coefficients Z of every
                                    block explicitly even for separable masks (by default the
                                    forward column pass, the zonal retention and the inverse
                                    column pass are applied as one exact contraction with
                                    G = T^T diag(w m) T; results are identical) */
  ADCT16_FLAG_MFMA_INT8 = 4,     /* MFMA backend, int8 products with int32 accumulation
                                    instead of FP16 products; results are identical.
                                    adct16_forward: the pixels centred to int8, the column
                                    pass on base-64 hi/lo digit planes of the row-pass
                                    result.  Fused call with a separable mask (none or zonal;
                                    not with ADCT16_FLAG_EXPLICIT_COEF): N = G Xc G with
                                    G = T^T diag(w m) T in int8, the intermediate Xc G on
                                    signed base-256 hi/lo digit planes.  Zig-zag masks keep
                                    the FP16 form (adct16_plan_info "fused_form") */
  ADCT16_FLAG_DEADZONE_INTER = 8, /* deadzone quantiser rounding offset f = 1/6 (inter-coded
                                    residuals) instead of 1/3 (intra) */
  ADCT16_FLAG_RESIDUAL_RANGE = 16 /* I16 input whose samples all lie in [-256, 255] (the
                                    difference of two 8-bit samples, Section 5.3's residual
                                    planes).  With the MFMA backend (or AUTO with
                                    ADCT16_FLAG_AUTOTUNE), a uniform step q >= 8 or a
                                    deadzone QP >= 22, I16 out_dtype, and every image below
                                    2^31 bytes with rows below 2^24 bytes, the fused call
                                    (with or without levels) runs on the matrix cores:
                                    exact FP16 products with FP32 accumulation for the
                                    forward and four integer partial inverses, combined per
                                    pixel in float64; results as the VALU kernel's (levels
                                    bit-exact, reconstructions equal except where the
                                    float64 value lies within 1e-9 of a rounding tie).  The
                                    kernel checks the range: an image with a sample outside
                                    it gets SSE -1 and PSNR NaN, and its levels and
                                    reconstruction are unspecified. */
};

/*
 * Batch descriptor, read by adct16_plan_create (arrays are copied).
 *
 * in_dtype    ADCT16_U8 (8-bit images, Section 4) or ADCT16_I16 (prediction
 *             residuals, Section 5.3).  The MFMA backend runs the fused
 *             call for U8 input, a mask qmode and U8 out_dtype, or for I16
 *             residuals as described at ADCT16_FLAG_RESIDUAL_RANGE, and the
 *             forward transform for U8 input to I32/I16 coefficients or
 *             I16 input to I32 coefficients; a plan with neither form is
 *             rejected (ADCT16_E_MODE).  The VALU backend takes every
 *             combination.
 * coef_dtype  output of adct16_forward:
 *               ADCT16_I32  Z = T A T^T exactly;
 *               ADCT16_I16  (U8 input only) Z of the centred block A - 128,
 *                           i.e. Z with 32768 subtracted at (0,0); fits int16;
 *               ADCT16_F32  B = S Z S, the orthonormal coefficients, as
 *                           fl32(Z) * fl32(1/sqrt(n_u n_v)).
 * qmode, r, q retention / quantiser used by adct16_quantise, adct16_inverse
 *             (uniform only) and the fused calls.
 * qcoef_dtype output of adct16_quantise (input of adct16_inverse):
 *               mask modes: same as coef_dtype (I32 or I16), kept values
 *                           unchanged, the rest zero;
 *               uniform:    levels L_uv = round_half_even(fl32(fl32(Z_uv) *
 *                           M_uv)), M_uv = fl32(1/(sqrt(n_u n_v) q)), stored
 *                           as ADCT16_I16 (saturated) or ADCT16_I32;
 *               deadzone:   L_uv = sign(Z_uv) floor(fl32(fl32(fl32(|Z_uv|) M_uv)
 *                           + f)) with separately rounded multiply and add,
 *                           M_uv = fl32(Q[QP mod 6] / (sqrt(n_u n_v)
 *                           2^(14 + QP/6))), Q = {26214, 23302, 20560, 18396,
 *                           16384, 14564}, f = fl32(1/3) (or 1/6, flag
 *                           ADCT16_FLAG_DEADZONE_INTER); reconstruction
 *                           B' = D[QP mod 6] 2^(QP/6) / 64 L, D = {40, 45, 51,
 *                           57, 64, 72}, then as for the uniform quantiser.
 * out_dtype   reconstruction: ADCT16_U8 (rounded half up, clamped 0..255),
 *             ADCT16_I16 (rounded half up, saturated) or ADCT16_F32 (the
 *             unrounded A').  U8 needs U8 input.
 */
typedef struct adct16_desc {
  int32_t n_images;
  const int32_t *height;
  const int32_t *width;
  const int32_t *pitch;
  const int64_t *offset;
  int32_t in_dtype;
  int32_t coef_dtype;
  int32_t qcoef_dtype;
  int32_t out_dtype;
  int32_t qmode;
  int32_t r;
  int32_t q;
  int32_t backend;
  int32_t flags;
  int32_t matrix;   /* ADCT16_MATRIX_APPROX (or ADCT16_MATRIX_T): the proposed transform,
                       T with S folded into the quantiser; ADCT16_MATRIX_WHT: the same
                       kernels with the Walsh-Hadamard matrix in natural order (S = I/4,
                       all weights 3); ADCT16_E_MODE otherwise */
} adct16_desc;

typedef struct adct16_plan_s *adct16_plan;
typedef struct adct16_graph_s *adct16_graph;

/* Validate `desc`, upload the image table and constant tables to the
 * current device and choose kernels.  Allocates device memory (the only
 * call besides adct16_graph_create that does).  On error *out is NULL. */
adct16_status adct16_plan_create(const adct16_desc *desc, adct16_plan *out);
adct16_status adct16_plan_destroy(adct16_plan plan);

/* Number of 16x16 blocks of the batch; coefficient buffers hold 256 times
 * this many elements. */
adct16_status adct16_plan_num_blocks(adct16_plan plan, int64_t *num_blocks);

/* NUL-terminated JSON describing the chosen kernels: backend of the fused
 * and forward calls, persistent grid (workgroups of 256 threads), the task
 * table of the matrix-core kernels ("task_strips": block rows split into
 * equal runs of at most 1, 2, 3, 4 or 16 strips of 16 x 128 pixels), and how each
 * choice was made.  ADCT16_E_SHAPE when buf_len is too small.
 *
 * Launch shapes without ADCT16_FLAG_AUTOTUNE come from defaults, which
 * these environment variables override at plan creation:
 *   ADCT16_WG_PER_CU    workgroups per CU of the persistent kernels, 1..64;
 *   ADCT16_TASK_STRIPS  1, 2, 3, 4 or 16, the task table of the matrix-core kernels;
 *   ADCT16_TUNE_CACHE   a file where autotuned choices are kept between
 *                       processes (keyed by device, dtypes, modes, the
 *                       batch's strip count and whether its rows are whole
 *                       128-byte lines). */
adct16_status adct16_plan_info(adct16_plan plan, char *buf, int32_t buf_len);

/* Measurement of the hot path (the roofline of the persistent kernel):
 * after adct16_plan_time_fused(plan, n), the next n fused calls on `plan`
 * (adct16_compress_and_measure, adct16_compress_and_measure_static) record a
 * pair of HIP events on the call's stream around their persistent kernel
 * only (not around the SSE / PSNR finishing kernel).  Calls captured into a
 * HIP graph are not timed.  n = 0 stops timing.  Creates 2n events (host
 * objects; E_NOMEM if that fails); n outside 0..65536 is ADCT16_E_SHAPE.
 * adct16_plan_fused_times waits for the recorded calls, writes the first
 * min(cap, recorded) kernel durations in milliseconds to ms, the number of
 * recorded calls to *n_out, and starts a new window of n calls. */
adct16_status adct16_plan_time_fused(adct16_plan plan, int32_t n_calls);
adct16_status adct16_plan_fused_times(adct16_plan plan, float *ms, int32_t cap, int32_t *n_out);

/* Section 4, forward: d_in (in_dtype) -> d_coef (coef_dtype, block-major).
 * Evaluates T by the 60-addition factorisation of Eq. (1) (VALU backend)
 * or as exact matrix-core products (MFMA backend): FP16 products for 8-bit
 * input, int8 products with ADCT16_FLAG_MFMA_INT8, and for 16-bit input
 * (I32 coefficients) int8 products on three base-64 digits per value.
 * Results are identical in every case.  With the MFMA backend, calls
 * without a matrix-core form run on the vector ALUs (adct16_plan_info
 * reports "forward_backend" and "fused_backend"); a plan none of whose
 * calls has one is rejected with ADCT16_E_MODE. */
adct16_status adct16_forward(adct16_plan plan, const void *d_in, void *d_coef, void *stream);

/* Section 4, retention (mask modes) or the uniform quantiser (Section 2: S
 * absorbed into the quantisation step).  d_coef must be I32 or I16
 * coefficients as written by adct16_forward; d_qcoef is qcoef_dtype.
 * d_qcoef may equal d_coef when the dtypes are equal. */
adct16_status adct16_quantise(adct16_plan plan, const void *d_coef, void *d_qcoef, void *stream);

/* Section 4, inverse A' = C_hat^T B' C_hat of every block, reassembled into
 * d_out (out_dtype, same layout as the input batch).
 * Mask modes: d_qcoef holds integer coefficients Z' (coef dtype I32 or
 * I16-centred); A' = T^T (w w^T .* Z') T / 2304 with w = 48/n, evaluated
 * exactly in int32.  Uniform: d_qcoef holds levels L; B' = q L and A' is
 * evaluated in float64. */
adct16_status adct16_inverse(adct16_plan plan, const void *d_qcoef, void *d_out, void *stream);

/* Section 4's comparison: every block through the exact orthonormal DCT-II
 * in float64 (Y = C X C^T), the plan's retention mask (qmode NONE, ZONAL or
 * ZIGZAG, same r), the inverse C^T Y' C in float64, rounding half up and
 * clamping to 0..255; with the per-image SSE and PSNR of that
 * reconstruction (the reference of the APE measure).  U8 input; d_out (U8,
 * the input layout), d_sse and d_psnr optional as in
 * adct16_compress_and_measure.  ADCT16_E_STATE for quantiser plans.
 * Rounded pixels may differ from another float64 evaluation order only
 * where the real value lies within rounding error of a half-integer. */
adct16_status adct16_dct_compress_and_measure(adct16_plan plan, const void *d_in, void *d_out,
                                              int64_t *d_sse, double *d_psnr, void *stream);

/* Section 4, SSIM of d_b against d_a (both U8 in the plan's layout, e.g.
 * an image batch and its reconstruction): per image, the mean over every
 * 11x11 window position inside the image of
 *   ((2 mu_a mu_b + C1)(2 s_ab + C2)) / ((mu_a^2 + mu_b^2 + C1)(s_a + s_b + C2))
 * with Gaussian-weighted moments (sigma 1.5, weights normalised),
 * C1 = (0.01 * 255)^2, C2 = (0.03 * 255)^2, in float64.  d_ssim: n_images
 * doubles (8-byte aligned); NaN for images smaller than 11 x 11.  Needs a
 * plan with U8 input and output dtypes. */
adct16_status adct16_ssim(adct16_plan plan, const void *d_a, const void *d_b, double *d_ssim, void *stream);

/* Rate proxy for the quantisation levels in d_qcoef (qcoef_dtype, block-
 * major, as written by adct16_quantise or the fused call): per image, the
 * total length in bits of the signed Exp-Golomb codes se(v) of its levels
 * (v > 0 -> code number 2v - 1, v <= 0 -> -2v; code number k takes
 * 2 floor(log2(k + 1)) + 1 bits).  d_bits: n_images int64 (overwritten, 8-
 * byte aligned).  ADCT16_E_STATE for plans whose qmode produces no levels. */
adct16_status adct16_rate(adct16_plan plan, const void *d_qcoef, int64_t *d_bits, void *stream);

/* Section 4, quality: per-image SSE over the true pixels and
 * PSNR = 10 log10(255^2 h w / SSE) (+inf when SSE = 0).  d_a is in_dtype,
 * d_b is out_dtype (U8 or I16).  d_sse: n_images int64 (overwritten);
 * d_psnr: n_images doubles, may be NULL. */
adct16_status adct16_measure(adct16_plan plan, const void *d_a, const void *d_b,
                             int64_t *d_sse, double *d_psnr, void *stream);

/* Section 4's compression experiment in one pass over the batch: every
 * 16x16 block A is transformed (B = C_hat A C_hat^T, Section 2 with Eq. (1)),
 * its coefficients retained (zonal / zig-zag) or quantised (uniform step
 * with S absorbed into it, Section 2; the deadzone stand-in of Section 5.3),
 * the block rebuilt as A' = C_hat^T B' C_hat and rounded as adct16_inverse
 * does, and the per-image SSE and PSNR accumulated as adct16_measure
 * computes them.  Results equal those of adct16_forward, adct16_quantise,
 * adct16_inverse and adct16_measure called in turn.  One persistent kernel
 * plus a finalisation kernel.
 * d_in: in_dtype, the batch layout.  d_out (out_dtype U8/I16, the input
 * layout) and d_qcoef (qcoef_dtype, block-major) are optional (NULL = not
 * written).  d_sse: n_images int64, overwritten; NULL uses the plan's
 * workspace.  d_psnr: n_images doubles, may be NULL.  ADCT16_E_NULL for a
 * NULL d_in, ADCT16_E_ALIGN for misaligned pointers, ADCT16_E_STATE for a
 * d_out with an F32 out_dtype, ADCT16_E_LAUNCH if a launch fails. */
adct16_status adct16_compress_and_measure(adct16_plan plan, const void *d_in, void *d_out,
                                          void *d_qcoef, int64_t *d_sse, double *d_psnr,
                                          void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as adct16_compress_and_measure, with the same arguments and
 * identical results, whose scratch memory (the per-task SSE partials of the
 * matrix-core kernel, the per-image accumulators of the vector kernel, and
 * the per-image SSE when d_sse is NULL) comes from a fixed device array of
 * 4 MiB inside the library instead of the plan's workspace.  Each GPU the
 * library runs on holds one such array until the process ends.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * its first use on a device resolves that device's array.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (other streams,
 * other threads) race and give undefined results; calls ordered on one
 * stream do not.  The plan's device must be current (ADCT16_E_DEVICE
 * otherwise).  A batch whose scratch exceeds 4 MiB is ADCT16_E_SHAPE (8
 * bytes per task of the matrix-core kernels, 8 bytes per accumulator slot
 * of the vector kernel: n_images x 64 slots up to 1024 images, x 8 up to
 * 16384).  Other errors as adct16_compress_and_measure. */
adct16_status adct16_compress_and_measure_static(adct16_plan plan, const void *d_in, void *d_out,
                                                 void *d_qcoef, int64_t *d_sse, double *d_psnr,
                                                 void *stream);

/* Comparison transform (Section 3): exact orthonormal DCT-II of every block,
 * Y = C X C^T, on the BF16 or F16 matrix cores with float32 accumulation.
 * X is the block centred to [-128, 127] for U8 input, the raw samples for
 * I16 input (|x| <= 255 is exact in both operand types); C is rounded to
 * the operand type.  d_y: float32, block-major.  Its error against the
 * float64 DCT is a property of the operand precision, not a bug. */
adct16_status adct16_dct_forward(adct16_plan plan, const void *d_in, float *d_y,
                                 int32_t precision, void *stream);

/* Section 2/3: the 16-point 1-D transform y = T x of n vectors (Fig. 4's
 * datapath).  d_x, d_y: n x 16 int32, row-major, 16-byte aligned.
 * Plan-free.  n = 0 is a no-op (pointers may then be NULL); n < 0 is
 * ADCT16_E_SHAPE. */
adct16_status adct16_forward_1d(const int32_t *d_x, int32_t *d_y, int64_t n, void *stream);
/* y = T^T x, the 1-D inverse up to the factor diag(n) (T^T T x / n-weights
 * recover x: x = T^T diag(1/n) T x). */
adct16_status adct16_inverse_1d(const int32_t *d_x, int32_t *d_y, int64_t n, void *stream);

/* Capture adct16_compress_and_measure with fixed pointers into a HIP graph
 * (created with a private capture stream; allocates).  Launching the graph
 * repeats exactly that call on `stream`.  The call is two kernels; on
 * ROCm 7.2, consecutive graph launches of one call each left 12-14 us
 * between calls against 3.6-3.8 us for direct calls, so a stream of small
 * calls (one video frame each) runs faster launched directly. */
adct16_status adct16_graph_create(adct16_plan plan, const void *d_in, void *d_out, void *d_qcoef,
                                  int64_t *d_sse, double *d_psnr, adct16_graph *out);
adct16_status adct16_graph_launch(adct16_graph graph, void *stream);
adct16_status adct16_graph_destroy(adct16_graph graph);

/* ---- Host-side functions (no device involved, synchronous) ------------ */

typedef enum adct16_matrix {
  ADCT16_MATRIX_APPROX = 0,  /* C_hat = S T, the proposed orthogonal approximation (Section 2) */
  ADCT16_MATRIX_T = 1,       /* T itself, entries in {0, +1, -1} (Section 2) */
  ADCT16_MATRIX_WHT = 2,     /* Walsh-Hadamard matrix in natural (Sylvester) order, / 4 */
  ADCT16_MATRIX_DCT = 3      /* orthonormal DCT-II, a_0 = 1/4, a_k = 1/sqrt(8) */
} adct16_matrix;

/* The 16x16 matrix `which` into m (256 doubles, row-major, host memory).
 * ADCT16_E_NULL if m is NULL, ADCT16_E_MODE for an unknown `which`. */
adct16_status adct16_transform_matrix(int32_t which, double *m);

/* Section 3, Table 2: similarity and coding measures of the 16-point
 * transform ct (256 doubles, row-major, host memory, rows = basis vectors)
 * against the orthonormal DCT-II, for the first-order Markov model
 * R_ij = rho^|i-j| (Section 3.2).  out (5 doubles, host memory):
 *   out[0] DCT distortion   d2  = 1 - (1/16) sum_i (C ct^T)_ii^2
 *   out[1] total error energy   = pi ||C - ct||_F^2
 *   out[2] MSE                  = (1/16) tr((C - ct) R (C - ct)^T)
 *   out[3] coding gain (dB)     = 10 log10( mean_i s_ii / (prod_i s_ii ||ct_i||)^(1/16) ),
 *                                  s = ct R ct^T
 *   out[4] transform efficiency (%) = sum_i |s_ii| / sum_ij |s_ij| * 100
 * ADCT16_E_NULL for NULL pointers; ADCT16_E_MODE if rho is outside (0, 1),
 * ct has a non-finite entry or a zero row. */
adct16_status adct16_transform_measures(const double *ct, double rho, double *out);

const char *adct16_status_string(adct16_status status);
const char *adct16_last_error_string(void);

#ifdef __cplusplus
}
#endif

#endif /* ADCT16_H */
