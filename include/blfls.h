/*
 * blfls.h -- C ABI of the MI355X (gfx950) BLF-LS library.
 *
 * BLF-LS (Liu, Zhang, Chen, Shen, Huang, Yang, "Embedding Bilateral Filter in
 * Least Squares for Efficient Edge-preserving Image Smoothing", arXiv 1812.07122)
 * smooths an image f by solving Eq. (7):
 *
 *     min_u  sum_s (u_s - f_s)^2 + lambda sum_{*=x,y} (d_* u_s - g_{*,s})^2,
 *     g_* = BLF(d_* f)                       (Eq. (1) applied to each gradient field)
 *
 * in two steps (Section III-A): (1) bilateral-filter the forward-difference
 * gradient fields, (2) solve Eq. (8) with Fourier transforms.  Everything runs
 * on the GPU in hand-written HIP kernels; this header is plain C.
 *
 * Conventions shared by every entry point
 *  - Images are planar, row-major FP32 in device memory: channel c, row i,
 *    column j lives at ptr[(c * H + i) * pitch + j].  `pitch` is in elements
 *    (floats), pitch >= W.  W is the width (x, fast axis), H the height.
 *  - Boundaries are circular: the gradients, the filter window and the
 *    Fourier solve all wrap around the image edges (the solve of Eq. (8)
 *    diagonalises circulant difference operators).
 *  - D_x f(i,j) = f(i,j+1) - f(i,j), D_y f(i,j) = f(i+1,j) - f(i,j) (Section II-B).
 *  - Colour channels are processed independently.
 *  - The caller owns every device buffer it passes (f, guide, u, workspace,
 *    arena).  The library never frees caller memory; it owns only plan tables
 *    and host structures.  Buffers must stay valid until the work on the
 *    stream is complete (blfls_smooth) or until blfls_poll reports DONE or
 *    FAILED (server).
 *  - Every call returns a blfls_status; BLFLS_OK is 0 and errors are negative.
 *    The message of the calling thread's last error is in blfls_last_error().
 *    No C++ exception crosses this interface.
 *  - hipStream_t is passed as void* so that this header needs no HIP header.
 */
#ifndef BLFLS_H
#define BLFLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BLFLS_OK = 0,
  BLFLS_E_INVALID = -1,        /* a bad argument: NaN, lambda < 0, sigma <= 0, ... */
  BLFLS_E_UNSUPPORTED = -2,    /* a valid problem this library does not handle (size factors) */
  BLFLS_E_NOMEM = -3,          /* request can never fit in the server arena / allocation failed */
  BLFLS_E_AGAIN = -4,          /* transient: server queue full, try again */
  BLFLS_E_HIP = -5,            /* the HIP runtime reported an error */
  BLFLS_E_UNKNOWN_TICKET = -6  /* blfls_poll on a ticket the server never issued or already retired */
} blfls_status;

/* Storage precision of the two intermediate gradient-residual fields.  The
 * filter weights, its accumulation, the FFTs and the spectral divide run in
 * FP32 in every mode; FP64 is used only for the host-built tables.  FP16
 * fields are stored times a power of two per field: a residual is bounded by
 * the span of its gradient field (the filters output weighted means), and a
 * field whose span exceeds 2^15 is scaled to a span of at most 2^15 (an extra
 * pass reads the image's gradient extrema first), so images of any range stay
 * finite; spans up to 2^15 (e.g. 8- and 15-bit data) are stored unscaled. */
typedef enum {
  BLFLS_FP32 = 0,
  BLFLS_MIXED_BF16 = 1,
  BLFLS_MIXED_FP16 = 2
} blfls_precision;

/* Map each range-source gradient field to [0, 1] before the filter and back
 * after (experiments section of the paper).  The filter weights see only
 * differences, so this equals the raw filter with sigma_r multiplied by the
 * field's (max - min), which is how it is computed. */
#define BLFLS_F_NORMALIZE 0x1u

/* The edge-preserving filter of step 1 (applied to each gradient field). */
typedef enum {
  BLFLS_FILTER_BLF = 0,  /* the bilateral filter of Eq. (1): BLF-LS */
  BLFLS_FILTER_NC = 1,   /* the normalized-convolution filter of the domain transform
                            (Gastal and Oliveira 2011) in its place: NC-LS (Section III-D).
                            Along a row (then a column) the transform advances by
                            1 + (sigma_s / sigma_r) |q(t) - q(t-1)| per pixel, q the range
                            source's gradient field of the same axis; each pass replaces a
                            value by the mean of the values within r_k of it in transformed
                            distance, r_k = 3 sigma_s 2^(N-k) / sqrt(4^N - 1) for round
                            k = 1..N, windows stopping at the image borders.  Window
                            membership is decided in FP32. */
  BLFLS_FILTER_GRID = 2, /* the bilateral-grid approximation of Eq. (1) (Paris and Durand
                            2006), the fast filter of the paper's experiments: p and 1 are
                            splatted into cells of s = floor(sigma_s + 1/2) pixels by one
                            range cell (1/sigma_r, widened so that at most 32 bins span the
                            range source's values), blurred with a Gaussian of sigma_s / s
                            cells across and one range cell deep (taps to +-2 cells), and
                            read back by trilinear interpolation; periodic like the exact
                            filter.  Ignores radius; s at most 32 pixels. */
  BLFLS_FILTER_AMF = 3   /* the adaptive-manifold filter (Gastal and Oliveira 2012) in its
                            place: AMF-LS (Section III-D).  A binary tree of manifolds
                            (images in the range space): the root is a spatial low-pass of q;
                            the two children of a manifold eta are low-passes of q over the
                            pixels with q < eta and q >= eta, weighted by 1 - psi and divided
                            (absent where that weight's low-pass is under 1e-20).  On each
                            manifold, psi = exp(-(eta - q)^2 / sigma_r^2) weights a splat of
                            (psi p, psi), a recursive blur along the manifold and a slice:
                            g = p + max_k psi_k (sum psi_k Bn_k / sum psi_k Bd_k - p).
                            Blur and low-passes are the domain transform's first-order
                            recursive filter y_j = c y_{j-1} + (1 - c) x_j with
                            c = exp(-sqrt(2) d / sigma_s), left to right then right to left,
                            rows then columns, not wrapping; d = 1 + (sqrt(2) sigma_s / sigma_r)
                            |eta_j - eta_{j-1}| on a manifold, 1 for the low-passes.  Full
                            resolution.  Ignores radius.  Needs blfls_workspace_size bytes. */
} blfls_filter;

/* Parameters of Eq. (1) and Eq. (7). */
typedef struct {
  float lambda;      /* weight of the gradient term of Eq. (7); >= 0, finite.
                        The paper's default is 1024 (Section III-C). */
  float sigma_s;     /* spatial Gaussian of Eq. (1), in pixels; > 0, finite */
  float sigma_r;     /* range Gaussian of Eq. (1), in gradient units; > 0, may be
                        +INFINITY (range kernel off: Gaussian-filtered gradients) */
  int32_t radius;    /* half-width of the square window; >= 0, or -1 for ceil(3 sigma_s).
                        At most BLFLS_MAX_RADIUS. */
  int32_t iterations;/* >= 1.  1 is plain BLF-LS (two-step procedure, Section III-A).
                        k > 1 is rolling guidance (Section III-D): iteration k takes its
                        range weights from the gradients of iteration k-1's output. */
  uint32_t flags;    /* BLFLS_F_* bits */
  float sigma_guide; /* >= 0.  > 0 smooths the initial range source (the guidance image,
                        or f itself) with a circular Gaussian of this standard deviation,
                        as the rolling-guidance extension does (Section III-D). 0 = off. */
  int32_t filter;    /* blfls_filter.  BLFLS_FILTER_NC ignores radius; its first box
                        radius r_1 must be at most BLFLS_MAX_RADIUS pixels
                        (sigma_s <= 21 for N = 3), else BLFLS_E_INVALID. */
  int32_t filter_iterations; /* NC: rounds N of a horizontal and a vertical box pass,
                        1..8; 0 selects 3.  AMF: manifold tree height 1..6 (2^h - 1
                        manifolds); 0 selects max(2, ceil(H_s L)), H_s = floor(log2
                        sigma_s) - 1, L = 1 - sigma_r, both clamped at 0, at most 6.
                        Must be 0 for the other filters. */
  float detail_gain; /* finite.  0: the output is u.  m != 0: the output is the
                        detail-enhanced u + m (f - u), the detail layer f - u boosted m
                        times over the smoothed base (the experiments section boosts it
                        5 times).  Applied to the last iteration; since u = f + delta it
                        is folded into the spectral divide (delta scaled by 1 - m), at no
                        extra pass. */
} blfls_params;

#define BLFLS_MAX_RADIUS 32
#define BLFLS_MAX_CHANNELS 4

/* ------------------------------------------------------------------------ */
/* Plans and the synchronous path                                            */
/* ------------------------------------------------------------------------ */

typedef struct blfls_plan_s *blfls_plan_t;

/* Create a plan for H x W images with C channels on the current HIP device.
 * The plan holds the FP32 twiddle and denominator tables (built in FP64 on the
 * host) for the transform sizes: W must be even, and W/2 and H must factor into
 * 2, 3 and 5 only, each at most BLFLS_MAX_FFT (else BLFLS_E_UNSUPPORTED).
 * C in [1, BLFLS_MAX_CHANNELS].  *workspace_bytes (if not NULL) receives the
 * device workspace blfls_smooth needs.  A plan is immutable after creation and
 * may be used from several streams at once, each with its own workspace. */
blfls_status blfls_plan(blfls_plan_t *out, int32_t H, int32_t W, int32_t C,
                        blfls_precision precision, size_t *workspace_bytes);

/* Workspace bytes a plan needs (same value blfls_plan reported).  Enough for
 * every filter except BLFLS_FILTER_AMF. */
blfls_status blfls_plan_workspace_size(blfls_plan_t plan, size_t *workspace_bytes);

/* Workspace bytes blfls_smooth needs for these parameters: the plan's size, plus
 * for BLFLS_FILTER_AMF the manifold arrays ((6 + 2 h) x H x W floats per gradient field
 * and a little more, h the tree height).  Validates params like
 * blfls_smooth (BLFLS_E_INVALID). */
blfls_status blfls_workspace_size(blfls_plan_t plan, const blfls_params *params,
                                  size_t *workspace_bytes);

/* Release a plan's tables.  The caller must ensure no queued work uses it. */
blfls_status blfls_plan_destroy(blfls_plan_t plan);

#define BLFLS_MAX_FFT 4096

/* Smooth f into u (Eq. (7) minimiser, via Eq. (1) then Eq. (8)).
 *   f          device, [C][H][pitch] FP32, read only
 *   guide      device, [C][H][pitch] FP32 or NULL.  Non-NULL: joint filtering
 *              (Section III-D): the range weights of Eq. (1) come from the
 *              gradients of the guide, the filtered values from f's gradients.
 *   u          device, [C][H][pitch] FP32, written.  Must not overlap f, guide
 *              or the workspace (BLFLS_E_INVALID).
 *   workspace  device, at least blfls_workspace_size(plan, params) bytes (the
 *              plan's workspace bytes for every filter but the AMF), 256-byte
 *              aligned; its contents on entry are ignored.
 *   stream     hipStream_t to queue on (NULL = the null stream).
 * All work is queued asynchronously; the call does not synchronise.  Errors
 * found on the host are returned before anything is queued. */
blfls_status blfls_smooth(blfls_plan_t plan, const blfls_params *params, const float *f,
                          const float *guide, float *u, int64_t pitch, void *workspace,
                          void *stream);

/* Static device scratch of blfls_smooth_noalloc, per GPU (192 MiB: the
 * workspace of a 1024 x 1024 RGB plan in FP32 for every filter but the AMF,
 * the pair filter's partial sums included). */
#define BLFLS_NOALLOC_SCRATCH_BYTES (192u << 20)

/* blfls_smooth without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the workspace is a static array of the library, one
 * per GPU, of BLFLS_NOALLOC_SCRATCH_BYTES, held from the library's load on
 * that GPU until the process ends.  The call allocates nothing (no hipMalloc,
 * no hipFree); its device address is looked up once per GPU, on the first call
 * with that GPU current.  Arguments, results and errors as blfls_smooth, plus
 * BLFLS_E_NOMEM when blfls_workspace_size(plan, params) exceeds the scratch.
 * Every call on one GPU uses the same scratch: calls that overlap on a GPU
 * (queued on different streams, or from several threads, without ordering
 * between them) race and give wrong results; calls on one stream are ordered
 * and safe.  The scratch's contents between calls are not part of the result. */
blfls_status blfls_smooth_noalloc(blfls_plan_t plan, const blfls_params *params, const float *f,
                                  const float *guide, float *u, int64_t pitch, void *stream);

/* HDR tone mapping in the log domain (experiments section: the framework of
 * Durand and Dorsey 2002 with BLF-LS as the base/detail decomposition).
 *   I = max((20 R + 40 G + B) / 61, 1e-6), L = log10 I,
 *   base = blfls_smooth(L) with `params` (one channel), detail = L - base,
 *   out_c = c / I * 10^((base - max base) cf + detail),
 *   cf = log10(contrast) / (max base - min base)  (1 if the base is constant):
 * the compressed base spans `contrast` with its maximum at 1, the detail layer
 * and the colour ratios pass unchanged.  Linear in, linear out (no gamma).
 *   plan       a plan with C = 1 for the image's H x W (else BLFLS_E_INVALID)
 *   rgb        device [3][H][pitch] FP32 linear radiance, read only
 *   out        device [3][H][pitch] FP32, written; must not overlap rgb or the workspace
 *              (nor may rgb overlap the workspace)
 *   contrast   target contrast of the compressed base, finite and > 1 (Durand and
 *              Dorsey use 5)
 *   workspace  at least blfls_tonemap_workspace_size(plan, params) bytes, 256-byte aligned
 * Queued on `stream` without synchronising, like blfls_smooth. */
blfls_status blfls_tonemap(blfls_plan_t plan, const blfls_params *params, const float *rgb, float *out,
                           int64_t pitch, float contrast, void *workspace, void *stream);

/* Workspace bytes of blfls_tonemap: blfls_workspace_size plus two H x W planes
 * and the extrema partials. */
blfls_status blfls_tonemap_workspace_size(blfls_plan_t plan, const blfls_params *params,
                                          size_t *workspace_bytes);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent requests                      */
/* ------------------------------------------------------------------------ */

typedef struct blfls_server_s *blfls_server_t;

typedef struct {
  int32_t H, W, C;       /* as for blfls_plan */
  const float *f;        /* device, [C][H][pitch] */
  const float *guide;    /* device or NULL */
  float *u;              /* device, written when the request is DONE */
  int64_t pitch;         /* elements */
  blfls_params params;
} blfls_request;

enum { BLFLS_QUEUED = 0, BLFLS_RUNNING = 1, BLFLS_DONE = 2, BLFLS_FAILED = 3 };

typedef struct {
  uint64_t submitted, admitted, completed, failed;
  uint64_t queued_now, running_now;
  uint64_t steps;               /* device steps launched */
  uint64_t arena_bytes, arena_in_use, arena_peak;
  double step_ms_mean;          /* host-measured wall time per step (launch to retire) */
  uint64_t latency_samples;     /* completed requests with a latency sample */
  double latency_p50_ms;        /* submit -> DONE, host steady clock, over all completed requests */
  double latency_p99_ms;
  double latency_max_ms;
  uint64_t graph_steps;         /* steps replayed from a captured graph of persistent launches */
  uint64_t direct_steps;        /* steps launched kernel by kernel (per-request filters, Fourier
                                   passes holding one transform per wave, or too many groups) */
} blfls_stats;

/* Create a server that runs requests on `stream` (void* hipStream_t).  `arena`
 * is a caller-owned device buffer of arena_bytes (256-byte aligned) from which
 * each admitted request takes its workspace; admission is by these bytes.
 * max_slots bounds the requests in flight at once (>= 1), queue_capacity the
 * requests waiting (>= 1).  A scheduler thread owned by the server launches
 * steps until blfls_server_destroy. */
blfls_status blfls_server_create(blfls_server_t *out, void *arena, size_t arena_bytes,
                                 int32_t max_slots, int32_t queue_capacity,
                                 blfls_precision precision, void *stream);

/* Queue a request.  Validated at once (same errors as blfls_smooth; a request
 * whose workspace exceeds the whole arena gives BLFLS_E_NOMEM).  A full queue
 * gives BLFLS_E_AGAIN.  On success *ticket identifies the request.
 * Ordering: the request's kernels run on the server's stream at some later
 * step and synchronise with nothing else, so f and guide must be fully
 * written, and u no longer in use, as seen from the server's stream, before
 * the call: work still queued on another stream must be made to precede it
 * (hipStreamWaitEvent on the server's stream; the Python binding does this for
 * the caller's current stream).  The buffers stay owned by the caller and must
 * stay valid until blfls_poll reports DONE or FAILED. */
blfls_status blfls_submit(blfls_server_t server, const blfls_request *request, uint64_t *ticket);

/* State of a ticket: *state is BLFLS_QUEUED, _RUNNING, _DONE or _FAILED;
 * *result is the request's status once DONE/FAILED.  Never blocks.  A DONE or
 * FAILED ticket is retired by the poll that reports it. */
blfls_status blfls_poll(blfls_server_t server, uint64_t ticket, int32_t *state,
                        blfls_status *result);

blfls_status blfls_server_stats(blfls_server_t server, blfls_stats *stats);

/* Stop accepting work, finish everything queued or running, join the
 * scheduler and release host state.  The arena is not freed. */
blfls_status blfls_server_destroy(blfls_server_t server);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/* Kernel families of one blfls_smooth call, in queue order. */
enum {
  BLFLS_STAGE_UPLOAD = 0,   /* descriptor upload into the workspace */
  BLFLS_STAGE_GAUSS = 1,    /* Gaussian smoothing of the initial guidance (sigma_guide > 0) */
  BLFLS_STAGE_MINMAX = 2,   /* gradient extrema of the range source (BLFLS_F_NORMALIZE) */
  BLFLS_STAGE_BLF = 3,      /* Eq. (1) on both gradient fields */
  BLFLS_STAGE_ROWS_FWD = 4, /* right-hand side + row real FFTs */
  BLFLS_STAGE_COLS = 5,     /* column FFTs, spectral divide, inverse column FFTs */
  BLFLS_STAGE_ROWS_INV = 6, /* inverse row FFTs, u = f + delta */
  BLFLS_STAGE_COUNT = 7
};

typedef struct {
  double ms[BLFLS_STAGE_COUNT];          /* summed GPU time between the stage's bracketing events */
  uint64_t launches[BLFLS_STAGE_COUNT];  /* bracketed launches summed */
} blfls_profile;

/* Process-wide switch: while enabled, blfls_smooth records a HIP event on its
 * stream before and after each kernel family (no synchronisation).  Meant for
 * benchmarks; it adds two event records per kernel launch. */
blfls_status blfls_profile_enable(int enable);

/* Wait for every recorded event, add the elapsed times per stage into *out,
 * and (reset != 0) drop the records.  Fails with BLFLS_E_HIP if an event
 * reports an error. */
blfls_status blfls_profile_read(blfls_profile *out, int reset);

/* Message of the calling thread's most recent error ("" if none).  The
 * pointer stays valid until the thread's next call into the library. */
const char *blfls_last_error(void);

/* Library version string. */
const char *blfls_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLFLS_H */
