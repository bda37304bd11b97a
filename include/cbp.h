/*
 * cbp.h -- C ABI of the MI355X (gfx950) coprime-blurred-pair deblurring library.
 *
 * Problem (Sec. 4, eq. 1 and eq. 4 of Thorpe et al., "A Co-Prime Blur Scheme
 * for Data Security in Video Surveillance"): two frames B1 = L (x) K1 + N1 and
 * B2 = L (x) K2 + N2 of one latent frame L, blurred by two unknown kernels that
 * are coprime as bivariate polynomials (Sec. 3).  Given B1, B2 and the latent
 * size (Sec. 6: all frames have a known resolution), the library recovers K1,
 * K2 (the cofactors of the GCD) and L.
 *
 * Method (Sec. 4 and Sec. 5), every step on the GPU inside one call:
 *   1. evaluate both frames as polynomials at S roots of unity along one axis
 *      at a time (eq. 3; Sec. 5: the evaluation is an S-point DFT), for both axis orders;
 *   2. at every sample, the 1-D cofactors are the null vector of the stacked
 *      convolution matrix [C(b1) | -C(b2)], taken as the smallest eigenvector
 *      of its Hermitian Gram matrix (Sec. 5: one small factorisation per
 *      sample and direction);
 *   3. the per-sample scales of the two evaluation orders are fixed by one
 *      least-squares problem with 2S unknowns (Sec. 4 last paragraph, Sec. 5);
 *   4. the two scaled kernel spectra are averaged, inverse-DFT'd and
 *      normalised (Sec. 5; abstract);
 *   5. the latent is recovered by Fourier division (Sec. 4; Sec. 5), here over
 *      both channels with a Tikhonov term lambda.
 *
 * Conventions shared by every entry point
 *   - Images are row-major [c][y][x] in DEVICE memory: element (c, y, x) is at
 *     data[c*channel_stride + y*pitch + x] (pitch and channel_stride in
 *     elements).  B_c is H_c x W_c; the latent is m x n; a full convolution
 *     gives H_c = m + k_c - 1 and W_c = n + k_c - 1, so k_c = H_c - m + 1.
 *   - Kernels are FP64, row-major k_c x k_c, in DEVICE memory.
 *   - The caller owns every buffer, including the workspace, whose size comes
 *     from cbp_workspace_size().  The library allocates no device memory for
 *     data; it keeps per device a capture stream, events, a small ring of pinned
 *     host staging buffers (frame descriptors of batched calls), the HIP
 *     graphs of CBP_FLAG_GRAPH calls and the autotuner's choices, until the
 *     process ends.
 *   - Calls are asynchronous on options->stream (a hipStream_t; NULL = the
 *     default stream).  The returned status covers HOST-side validation only;
 *     numerical outcomes are written to options->diag (device, nullable) and
 *     are valid after the stream is synchronised.
 *   - Nothing here is thread-safe for calls that share a workspace.
 *   - No exception crosses this ABI.
 */
#ifndef CBP_H_
#define CBP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CBP_MAX_K 32   /* largest kernel size */
#define CBP_MAX_S 32   /* largest number of samples per axis */
#define CBP_MAX_N 64   /* largest per-sample unknown count k1 + k2 */
#define CBP_MAX_FFT_F32 2048  /* largest FFT grid side, FP32 division */
#define CBP_MAX_FFT_F64 2048  /* largest FFT grid side, FP64 division */

typedef enum {
  CBP_OK = 0,
  CBP_E_INVALID = 1,      /* null pointer, bad option value, S < max k */
  CBP_E_SHAPE = 2,        /* frames not full convolutions of one m x n latent, k outside 1..32, grid too large */
  CBP_E_DEGENERATE = 3,   /* reserved for callers that check diag flags */
  CBP_E_DEVICE = 4,       /* a HIP launch or query failed */
  CBP_E_NOMEM = 5,        /* workspace smaller than cbp_workspace_size() */
  CBP_E_UNSUPPORTED = 6   /* option combination not built */
} cbp_status;

typedef enum { CBP_F32 = 0, CBP_F64 = 1, CBP_U8 = 2 /* 8-bit streams: cbp_quantize / cbp_dequantize only */ } cbp_dtype;

/* Precision form.
 *   FP64   : FP64 frames; evaluation, Gram (double-double accumulated), the
 *            eigen-solves, scale fix and Fourier division all in FP64.
 *   MIXED  : FP32 frames; evaluation accumulated in FP64, Gram double-double,
 *            eigen-solves and scale fix FP64, FFT and division in FP32.
 *   MFMA32 : as MIXED, but the per-sample Gram is A^H A on the matrix cores
 *            from FP32-rounded operands, FP32 accumulation (k1 + k2 <= 32).
 *   BF16   : as MFMA32 with bfloat16 operands (FP32 accumulation).
 *   MFMA64 : as MIXED, but the Gram's correlations come from the FP64 matrix
 *            cores (v_mfma_f64_16x16x4f64) on the FP64 evaluations, FP64
 *            accumulation (k1 + k2 <= 32): an FP64-accurate Gram instead of
 *            a double-double one.
 * MFMA32 and BF16 square the conditioning of the per-sample problems in
 * FP32: their kernel error against the FP64 method is reported, not bounded
 * (see cbp_sample_grams). */
typedef enum { CBP_PREC_FP64 = 0, CBP_PREC_MIXED = 1, CBP_PREC_MFMA32 = 2, CBP_PREC_BF16 = 3,
               CBP_PREC_MFMA64 = 4 } cbp_precision;

typedef struct cbp_image {
  void*     data;            /* device pointer */
  int32_t   dtype;           /* cbp_dtype */
  int32_t   height, width;   /* H x W */
  int32_t   channels;        /* 1 (grayscale) or more; all channels share one kernel pair */
  int64_t   pitch;           /* elements between rows, >= width */
  int64_t   channel_stride;  /* elements between channels, >= height*pitch */
} cbp_image;

typedef struct cbp_options {
  int32_t     precision;        /* cbp_precision */
  int32_t     samples;          /* S per axis; 0 = max(k1, k2); must be >= max(k1, k2) and <= CBP_MAX_S */
  double      lambda;           /* Tikhonov term of the Fourier division, >= 0 */
  double      tau;              /* reserved, must be 0 (the learned form predicts its own) */
  int32_t     learned;          /* 1 = learned form: weights from the network in mlp_blob (k1 + k2 <= 32) */
  int32_t     flags;            /* CBP_FLAG_* bits; 0 = the default method, eager launches, default launch shapes */
  const void* mlp_blob;         /* device network blob (cbp_mlp_export) when learned = 1, else NULL */
  void*       stream;           /* hipStream_t */
  void*       workspace;        /* device scratch owned by the caller */
  size_t      workspace_bytes;  /* its size in bytes */
  void*       diag;             /* device cbp_diag (one per frame for the batch call), or NULL */
} cbp_options;

/* Option flags (cbp_options.flags).
 *   CBP_FLAG_GRAPH    : the call's launches are captured once into a HIP graph
 *                       (keyed by every pointer, size and option the launches
 *                       bake in) and replayed with one hipGraphLaunch on later
 *                       calls with the same key.  Up to 64 graphs are cached
 *                       per device; evicting one synchronises the device.
 *   CBP_FLAG_AUTOTUNE : on the first call of a batch class (dtype, frame count,
 *                       largest frame, kernel and channel count, S, precision)
 *                       the launch shapes -- FFT radix order, rows per fold
 *                       group, columns per column-pass strip, workgroups per
 *                       CU of the streaming launches -- are searched by timing
 *                       the call itself on its stream (the call then blocks
 *                       until the search ends); later calls of that class use
 *                       the choice, with or without the flag. */
#define CBP_FLAG_GRAPH     1
#define CBP_FLAG_AUTOTUNE  2
/* The paper's narrower steps, in place of this library's readings:
 *   CBP_FLAG_DIVIDE_B1 : single-channel division (Sec. 4: B1 divided by K1 in
 *                        the Fourier domain; Sec. 5: one frame of the pair is
 *                        deblurred): Lhat = conj(K1hat) B1hat / (|K1hat|^2 + lambda)
 *                        on the same grid (where K1hat vanishes the quotient is 0);
 *   CBP_FLAG_SCALE_K1  : the scale least squares over kernel 1's equations only
 *                        (Sec. 5: 2t unknowns over the t x t entries of k1's two
 *                        estimates); both kernels use the scales it finds;
 *   CBP_FLAG_ONE_AXIS  : the per-sample scales of pass X alone, fixed by the
 *                        kernels' finite support: with a_j the scale of sample j,
 *                        sum_j a_j X_j[x] w_j^{-y} must vanish for k_c <= y < S
 *                        (smallest eigenvector of those equations' Gram, FP64
 *                        with double-double entries); needs
 *                        k1 (S - k1) + k2 (S - k2) >= S - 1 (so S >= k + 1 when
 *                        k1 = k2 = k; CBP_E_INVALID otherwise).  The kernels are
 *                        the real part of (1/S) sum_j a_j X_j[x] w_j^{-y} on their
 *                        support, divided by its complex sum.
 * SCALE_K1 and ONE_AXIS exclude each other (CBP_E_INVALID) and the learned
 * form (CBP_E_UNSUPPORTED). */
#define CBP_FLAG_DIVIDE_B1 4
#define CBP_FLAG_SCALE_K1  8
#define CBP_FLAG_ONE_AXIS  16

/* Diagnostic flags (cbp_diag.flags). */
#define CBP_DIAG_NONFINITE      1  /* a non-finite value reached the kernels */
#define CBP_DIAG_SAMPLE_WEAK    2  /* some per-sample Gram had no clear null direction */
#define CBP_DIAG_SCALE_WEAK     4  /* the scale system had no clear null direction */
#define CBP_DIAG_KERNEL_ZERO    8  /* a kernel estimate summed to ~0 before normalisation */
#define CBP_DIAG_FALLBACK      16  /* learned form: the plain kernels were kept (a noisy frame, or the learned objective was larger or not a number) */
#define CBP_DIAG_BAD_NETWORK   32  /* learned form: the network blob's header is not this library's (unit weights used) */

/* Per-frame numerical diagnostics, written in device memory when
 * options->diag is not NULL.  Complex values are (re, im) pairs. */
typedef struct cbp_diag {
  int32_t k1, k2, S, n;                      /* sizes used: n = k1 + k2 */
  int32_t flags;                             /* CBP_DIAG_* */
  int32_t refine_sample;                     /* most Newton refinement steps over the per-sample eigen-solves */
  int32_t refine_scale;                      /* Newton refinement steps of the scale-system eigen-solve */
  int32_t reserved;
  double  sample_lambda0[2][CBP_MAX_S];      /* Rayleigh quotient of each null vector (pass X, pass Y) */
  double  sample_lambda1[2][CBP_MAX_S];      /* second smallest eigenvalue of each per-sample Gram */
  double  sample_scale[2][CBP_MAX_S];        /* largest Gram diagonal entry of each sample */
  double  scale_lambda0, scale_lambda1, scale_scale;  /* the same three figures for the scale system */
  double  kernel_imag[2];                    /* ||Im K|| / ||Re K|| after normalisation */
  double  kernel_outside[2];                 /* energy fraction of the S x S inverse DFT outside the k x k support */
  double  sample_vec[2][CBP_MAX_S][CBP_MAX_N][2];  /* unit null vectors x = (u: k2 entries, v: k1 entries) */
  double  scale_vec[2 * CBP_MAX_S][2];             /* unit (a_0..a_{S-1}, b_0..b_{S-1}) */
  double  khat[2][CBP_MAX_S][CBP_MAX_S][2];        /* averaged kernel spectra [kernel][i (x freq)][j (y freq)] */
  float   sample_features[2][CBP_MAX_S][32];         /* the learned form's spectrum features of each sample */
  double  sample_weights[2 * CBP_MAX_S + 1];          /* learned form: wX_0.., wY_0.., tau (unused otherwise) */
  double  judge[2];                                  /* learned form: J of the plain and of the learned kernels */
} cbp_diag;

/* Human-readable name of a status code (static string, never NULL). */
const char* cbp_status_string(cbp_status s);

/* The HIP call behind the last CBP_E_DEVICE returned on this thread and its
 * HIP error string ("" if none); valid until the thread's next failing call. */
const char* cbp_last_error(void);

/* Library version, "major.minor.patch" (static string). */
const char* cbp_version(void);

/* sizeof(cbp_diag), for callers that allocate diag records from another
 * language. */
size_t cbp_diag_size(void);

/* Bytes of workspace needed by one call on frames of at most maxH x maxW
 * pixels with kernels of at most maxk, for `channels` channels and `batch`
 * frames in flight (the batch call).  Returns 0 for invalid sizes.
 * `opts` may be NULL (then precision FP64 and S = maxk are assumed). */
size_t cbp_workspace_size(int32_t maxH, int32_t maxW, int32_t maxk,
                          int32_t channels, int32_t batch, const cbp_options* opts);

/* Unit-circle evaluation of one frame (Sec. 4 eq. 3; Sec. 5): writes
 *   ex[j*W + x] = sum_y B[y][x] w_j^y   (S x W complex, interleaved FP64)
 *   ey[i*H + y] = sum_x B[y][x] w_i^x   (S x H complex, interleaved FP64)
 * with w_j = exp(-2 pi i j / S), accumulated in FP64.  ex, ey are device
 * buffers of 2*S*W and 2*S*H doubles.  Channel 0 only.  Uses the workspace
 * (>= cbp_workspace_size(H, W, S, 1, 1, opts)). */
cbp_status cbp_eval_unit_circle(const cbp_image* b, int32_t S, double* ex, double* ey,
                                const cbp_options* opts);

/* The per-sample Gram matrices of step 2 (Sec. 5: one small factorisation
 * per sample and direction), as the chosen precision form computes them:
 * FP64 / MIXED accumulate the block-Toeplitz correlations in double-double;
 * MFMA32 / BF16 form A^H A on the matrix cores from FP32 / bfloat16 operands
 * with FP32 accumulation.  grams (device) receives 2 * S * N * N complex
 * FP64 values (re, im interleaved), N = k1 + k2, laid out
 * [pass (0: X, 1: Y)][sample][p][q], each the Hermitian
 *   G = A^H A,  A = [C_k2(e1) | -C_k1(e2)]  (unknowns ordered (u: k2, v: k1)),
 * rounded to FP64.  Multi-channel frames: summed over channels. */
cbp_status cbp_sample_grams(const cbp_image* b1, const cbp_image* b2, int32_t m, int32_t n,
                            double* grams, const cbp_options* opts);

/* Kernel recovery (steps 1-4).  b1, b2: the blurred pair (same dtype and
 * channel count); m, n: latent size.  K1 (k1*k1 doubles) and K2 (k2*k2)
 * receive the kernels normalised to sum 1.  Multi-channel frames: the
 * per-sample Gram matrices are summed over channels. */
cbp_status cbp_recover_kernels(const cbp_image* b1, const cbp_image* b2, int32_t m, int32_t n,
                               double* K1, double* K2, const cbp_options* opts);

/* Kernel recovery followed by two-channel regularised Fourier division
 * (steps 1-5).  The latent size m x n and channel count are read from
 * `latent`, whose dtype must equal the inputs'.  K1, K2 may be NULL (then
 * the kernels stay in the workspace). */
cbp_status cbp_deblur(const cbp_image* b1, const cbp_image* b2, cbp_image* latent,
                      double* K1, double* K2, const cbp_options* opts);

/* cbp_deblur over `nframes` independent frames (each with its own kernel
 * pair and sizes; one dtype).  b1s, b2s, latents, K1s, K2s are HOST arrays of
 * nframes entries (K1s / K2s entries may be NULL).  Every phase of the path
 * is ONE launch over the work items of all frames (up to 256 frames per
 * launch; larger batches are split), reading per-frame descriptors that the
 * call stages into the head of the workspace.  per_frame (host, nullable)
 * receives each frame's validation status; invalid frames are skipped, the
 * others run, and the call returns the first failure or CBP_OK.  The
 * workspace must hold `nframes` frames of the largest size
 * (cbp_workspace_size(..., batch = nframes, ...)).  opts->diag, when set,
 * points to nframes cbp_diag records.  With the default launch shapes (no
 * autotuned choice stored for the batch class) per-frame results are
 * identical, bit for bit, to cbp_deblur on that frame alone. */
cbp_status cbp_deblur_batch(int32_t nframes, const cbp_image* b1s, const cbp_image* b2s,
                            cbp_image* latents, double* const* K1s, double* const* K2s,
                            cbp_status* per_frame, const cbp_options* opts);

/* cbp_deblur for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * call uses no caller workspace: options->workspace and workspace_bytes are
 * ignored, and the workspace is a scratch array of
 * cbp_noalloc_scratch_bytes() bytes (48 MiB) that the library holds in every
 * device's memory until the process ends (a grayscale 1080p frame in the
 * MIXED form, or a 720p frame in FP64, fits).  The caller still passes the
 * frames, the latent, the kernels (nullable) and options->diag.  The call
 * makes no hipMalloc, hipFree or pinned-host allocation; the library's
 * per-device set-up (stream, events, the scratch address) happens on the
 * first call of any entry point on that device.
 * Errors: CBP_E_NOMEM when the frame needs more than the scratch holds
 * (cbp_last_error() names both sizes); CBP_E_UNSUPPORTED when
 * options->flags holds CBP_FLAG_GRAPH or CBP_FLAG_AUTOTUNE (graphs and the
 * autotuner allocate); otherwise as cbp_deblur.  Every call on one device shares that device's scratch, which
 * keeps the last call's contents (nothing in it needs to start at zero):
 * calls that overlap on one device -- on two streams, or from two threads --
 * race on it and must be serialised by the caller. */
cbp_status cbp_deblur_noalloc(const cbp_image* b1, const cbp_image* b2, cbp_image* latent,
                              double* K1, double* K2, const cbp_options* opts);

/* Size in bytes of the scratch array that cbp_deblur_noalloc uses. */
size_t cbp_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------
 * Blind kernel-size estimation (Sec. 4: the kernel degree is found first,
 * from the singularity of nested submatrices, after Barnett; Sec. 5 and
 * Table 1: the kernel degree estimation stage, an odd-size search 9..25).
 *
 * With the latent size unknown, only d = H1 - H2 = W1 - W2 = k1 - k2 is
 * known.  For each candidate k (trial sizes k1' = k, k2' = k - d) and each of
 * S unit-circle samples of both passes, the per-sample system
 * [C_{k-d}(e1) | -C_k(e2)] has nullity max(0, k - k1 + 1) (zero below the
 * true size).  The test value is s = lambda_min / lambda_max of its Gram (the
 * Grams of every candidate are principal submatrices of one Gram, built from
 * one set of double-double correlations).  The score of a candidate is the
 * median over the 2S samples of log10(max(s, 1e-13)); the estimate is the
 * candidate whose score drops most below the previous candidate's (0 before
 * the first; the smaller candidate on ties).  A largest drop below 2
 * decades means no candidate made the systems singular: the estimate is then
 * the largest candidate and CBP_SIZE_NONE_SINGULAR is set; a winning first
 * candidate sets CBP_SIZE_FIRST_SINGULAR (the true size may lie below the
 * range).  Noise raises every s toward the noise level; the test separates
 * the sizes when the frames' noise is well below the kernels' conditioning. */
#define CBP_SIZE_NONE_SINGULAR   1
#define CBP_SIZE_FIRST_SINGULAR  2

typedef struct cbp_size_search {
  int32_t kmin, kmax, step;  /* candidates k1' = kmin, kmin + step, ... <= kmax, kept when
                                1 <= k1' - d, both trial sizes <= 32 and k1' <= min(H1, W1) */
  int32_t samples;           /* S per pass (1..32); 0 = the largest trial size of either frame */
} cbp_size_search;

typedef struct cbp_size_result {   /* written in DEVICE memory */
  int32_t k1, k2;                  /* the estimate */
  int32_t flags;                   /* CBP_SIZE_* */
  int32_t ncand;                   /* candidates tested */
  int32_t samples;                 /* S used */
  int32_t reserved;
  int32_t cand[CBP_MAX_K];         /* the candidates k1' (ascending) */
  double  score[CBP_MAX_K];        /* median over samples of log10(max(s, 1e-13)) */
  double  drop[CBP_MAX_K];         /* score[c-1] - score[c] (score[-1] = 0) */
} cbp_size_result;

/* Workspace bytes of cbp_estimate_kernel_sizes for frames of at most
 * maxH x maxW, `channels` channels and the given search (0 when the search
 * has no candidate or S is out of range).  opts may be NULL (FP64). */
size_t cbp_size_workspace_size(int32_t maxH, int32_t maxW, int32_t channels, int32_t d,
                               const cbp_size_search* search, const cbp_options* opts);

/* Estimate (k1, k2) of a blurred pair without the latent size.  b1, b2: the
 * pair (same dtype and channel count; colour frames stack their channels'
 * systems as the recovery does); result: one cbp_size_result in device
 * memory; ratios (device, nullable) receives s for every
 * [candidate][pass][sample] (ncand * 2 * S doubles).  opts: precision FP64
 * (FP64 frames) or MIXED (FP32 frames), the stream and the workspace
 * (cbp_size_workspace_size); the other fields are ignored.  Asynchronous;
 * the caller reads `result` after synchronising the stream.
 * Errors (host side): CBP_E_SHAPE when H1 - H2 != W1 - W2 or no candidate
 * fits; CBP_E_INVALID for a bad search (kmin < 1, kmax < kmin, step < 1, S
 * outside 0..32), NULL pointers or a matrix-core precision; CBP_E_NOMEM when
 * the workspace is too small. */
cbp_status cbp_estimate_kernel_sizes(const cbp_image* b1, const cbp_image* b2, const cbp_size_search* search,
                                     cbp_size_result* result, double* ratios, const cbp_options* opts);

/* ------------------------------------------------------------------------
 * The CBP encoder (Sec. 3, blur kernel selection: large random kernels, a
 * new coprime pair for every frame; Sec. 4 eq. 1 without sensor noise) and
 * the multi-level 8-bit streams (Sec. 3, multi-level security: a level sees
 * the streams without some least significant bits).
 *
 * cbp_draw_kernel_pairs: the kernel pairs of frames frame0 .. frame0 +
 * nframes - 1.  Entry e (row-major) of kernel s in {1, 2} at draw attempt a is
 * u_e = ((w >> 11) + 1/2) 2^-53 with w word e mod 4 of Philox4x64-10
 * (Salmon et al., SC 2011) at counter (e / 4, s, a, 0) and key (seed, frame);
 * the kernel is u / sum(u) (sum in entry order).  A pair is redrawn (a + 1)
 * while, at some sample w_j (j < S; S = samples, 0 = max(k1, k2)) of either
 * evaluation order, the Sylvester system [C_{k2-1}(p) | -C_{k1-1}(q)] of the
 * kernel slices p = k1(w_j, .), q = k2(w_j, .) (or k1(., w_j), k2(., w_j))
 * has lambda_min / lambda_max of its Gram at or below 1e-12 (the slices
 * nearly share a root); at most 64 attempts.  K1s (nframes * k1 * k1 doubles)
 * and K2s receive the pairs, attempts[f] (device int32) the attempt used or
 * -1 when none passed (the last draw is kept), min_ratio[f] (device, nullable)
 * the smallest ratio of the kept pair.  One wave per frame; asynchronous on
 * `stream`.  Errors: CBP_E_INVALID (NULL buffers, nframes < 1, frame0 < 0,
 * S outside 1..32), CBP_E_SHAPE (k outside 1..32). */
cbp_status cbp_draw_kernel_pairs(uint64_t seed, int64_t frame0, int32_t nframes, int32_t k1, int32_t k2,
                                 int32_t samples, double* K1s, double* K2s, int32_t* attempts, double* min_ratio,
                                 void* stream);

/* B1 = L (x) K1 and B2 = L (x) K2 (full linear convolution, every channel):
 * latent m x n, b1 (m + k1 - 1) x (n + k1 - 1), b2 likewise with k2, one
 * dtype and channel count; K1, K2 device FP64 row-major.  FP32 frames
 * accumulate in FP32 (the kernel rounded to FP32), FP64 frames in FP64.
 * Asynchronous on `stream`.  Errors: CBP_E_INVALID, CBP_E_SHAPE. */
cbp_status cbp_encode(const cbp_image* latent, const double* K1, int32_t k1, const double* K2, int32_t k2,
                      cbp_image* b1, cbp_image* b2, void* stream);

/* The 8-bit stream of a level without the drop_bits (0..8) least significant
 * bits: dst = clamp(rint(255 src), 0, 255) & (255 << drop_bits), rint rounding
 * half to even in src's precision.  src: FP32 / FP64 image; dst: a CBP_U8
 * image of the same shape (pitch and channel stride in bytes). */
cbp_status cbp_quantize(const cbp_image* src, cbp_image* dst, int32_t drop_bits, void* stream);

/* The receiver's frame: dst = src / 255 in dst's precision (src CBP_U8). */
cbp_status cbp_dequantize(const cbp_image* src, cbp_image* dst, void* stream);

/* Launch shapes chosen by the last CBP_FLAG_AUTOTUNE search on the current
 * device, with the time of one batch call under them. */
typedef struct cbp_tuning {
  int32_t fold_rows;          /* rows per column-fold group (before rounding up to a multiple of S; 0 = from the frame size) */
  int32_t strip_columns;      /* columns per column-pass strip (0 = automatic) */
  int32_t workgroups_per_cu;  /* persistent-grid cap of the streaming launches (0 = one workgroup per item) */
  int32_t fft_order;          /* radix pass order: 0 = 8,4,2,3,5,7; 1 = 4,8,2,3,5,7; 2 = 7,5,3,8,4,2 */
  double  ms;                 /* measured time of the batch call, ms */
} cbp_tuning;

/* CBP_E_INVALID when no search has run on this device. */
cbp_status cbp_last_tuning(cbp_tuning* out);

/* ------------------------------------------------------------------------
 * The learned form (no counterpart in the paper).  A 32 -> 128 -> 128 -> 2
 * ReLU network reads each sample's Gram spectrum as 32 features
 *   f_i = log10(max(lambda_i, 1e-14 lambda_max) / lambda_max) / 10  (i < k1+k2), +1 after,
 * and predicts w = clip(softplus(o1), 1e-3, 1e3) and tau_j = exp(clip(o2, -30, 5)).
 * The weights enter the scale fix (rows weighted by sqrt(wX_j wY_i)) and the
 * assembly (spectra averaged with weights wX_j, wY_i; the kernel is the
 * separable weighted fit to them with per-axis Tikhonov strength tau =
 * median of tau_j).  Unit weights and tau = 0 reduce it to the plain method.
 * The plain kernels are returned instead (CBP_DIAG_FALLBACK) on a noisy frame
 * -- more than half of the 2S samples with f_0 > -1, i.e. lambda_0 above
 * 1e-10 lambda_max, where the network does not gain -- and when the plain
 * method's per-sample objective sum_j x^H G_j x / x^H x is smaller for them.
 * Layers 1 and 2 run on the matrix cores in bfloat16 with FP32 accumulation;
 * the 2-output head, the biases, the master weights and Adam are FP32.
 *
 * Parameters (FP32, device, packed): W1 [128][32], b1 [128], W2 [128][128],
 * b2 [128], W3 [2][128], b3 [2] -- cbp_mlp_param_count() floats.
 * Training state (device, cbp_mlp_state_size(max_rows) bytes, caller-owned):
 * master weights, Adam moments, bf16 copies and the activations of up to
 * max_rows rows.  Features X: device FP32 [n][32]; targets T: device FP32
 * [n][2] = (log w*, log tau*); loss: device FP32, the mean over rows of
 * (log softplus(o1) - log w*)^2 + (o2 - log tau*)^2.  All calls are
 * asynchronous on `stream`. */
int32_t    cbp_mlp_param_count(void);
size_t     cbp_mlp_blob_size(void);
size_t     cbp_mlp_state_size(int32_t max_rows);
/* Load parameters into a state and reset its Adam moments. */
cbp_status cbp_mlp_set_params(void* state, int32_t max_rows, const float* params, void* stream);
cbp_status cbp_mlp_get_params(const void* state, int32_t max_rows, float* params, void* stream);
/* Checkpoint of a training state (resume): the master weights and both Adam
 * moments, cbp_mlp_checkpoint_size() bytes = 3 x cbp_mlp_param_count() FP32
 * in device memory, caller-owned.  Loading restores them (and the bf16
 * copies) into a state of any max_rows; the caller keeps the step count
 * passed to cbp_mlp_train_step.  CBP_E_INVALID on NULL pointers or
 * max_rows < 1. */
size_t     cbp_mlp_checkpoint_size(void);
cbp_status cbp_mlp_save_state(const void* state, int32_t max_rows, float* out, void* stream);
cbp_status cbp_mlp_load_state(void* state, int32_t max_rows, const float* in, void* stream);
/* Loss and gradient (packed like the parameters; grads may be NULL) of n <= max_rows rows. */
cbp_status cbp_mlp_gradients(void* state, int32_t max_rows, const float* X, const float* T, int32_t n,
                             float* loss, float* grads, void* stream);
/* cbp_mlp_gradients followed by one Adam step (beta 0.9 / 0.999, eps 1e-8; step counts from 1). */
cbp_status cbp_mlp_train_step(void* state, int32_t max_rows, const float* X, const float* T, int32_t n,
                              float lr, int32_t step, float* loss, void* stream);
/* The inference blob (cbp_mlp_blob_size() bytes, device) from a state. */
cbp_status cbp_mlp_export(const void* state, int32_t max_rows, void* blob, void* stream);
/* Network outputs (o1, o2) for n feature rows: out device FP32 [n][2]. */
cbp_status cbp_mlp_forward(const void* blob, const float* X, int32_t n, float* out, void* stream);

/* Phase timing.  While enabled, every call records a HIP event pair around
 * each phase on its stream; cbp_profile_read() waits for the recorded events,
 * adds their elapsed times to per-phase totals and returns the number of
 * phases (at most max_phases are written to ms_total / counts).  Names come
 * from cbp_profile_phase_name().  cbp_profile_reset() clears the totals. */
void        cbp_profile_enable(int32_t on);
void        cbp_profile_reset(void);
int32_t     cbp_profile_read(double* ms_total, int64_t* counts, int32_t max_phases);
const char* cbp_profile_phase_name(int32_t phase);

#ifdef __cplusplus
}
#endif

#endif /* CBP_H_ */
