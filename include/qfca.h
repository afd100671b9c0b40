/*
 * qfca.h -- C ABI of libqfca, the MI355X (gfx950) implementation of the
 * Quantized FCA score-map path: "Quantized FCA: Efficient Zero-Shot Texture
 * Anomaly Detection" (Ardelean, Rueckbeil, Weyrich).
 *
 * Problem (Sec. 3, Eq. 1): one C-channel feature map F in R^{C x H x W} in,
 * one per-pixel anomaly map A(x, y) out, zero-shot: every statistic comes
 * from the image itself (Sec. 3.3) or, for served texture classes, from a
 * class exemplar fitted once.
 *
 * Conventions shared by every entry point:
 *   - Array arguments named X, bins, score, amap, w1, achan, resid are DEVICE
 *     pointers owned by the caller (for instance torch tensors on cuda:N).
 *     Arrays passed to qfca_model_create / read by qfca_model_read are HOST
 *     pointers owned by the caller.  The library owns models and scratch.
 *   - Feature maps are float32, channel-planar [C][H][W], row-major, densely
 *     packed.  Bin maps are uint8 [C][H][W].  Score-like maps are float32
 *     [H][W].
 *   - Calls are stream-ordered on the context's HIP stream and return before
 *     the GPU finishes, like HIP itself; outputs are valid once the stream is
 *     synchronised.  qfca_fit_pca and qfca_fit_reference are synchronous.
 *   - Arguments are validated before any launch; no exception or abort
 *     crosses the ABI.  Every call returns a qfca_status; qfca_last_error()
 *     gives a message for the calling thread's last failure.
 *   - A context is used by one host thread at a time; models may be shared
 *     by contexts on the same device.
 *   - Score-side inputs are not checked for non-finite values; NaN or Inf in
 *     X passed to qfca_quantize gives undefined bins.
 */
#ifndef QFCA_H
#define QFCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QFCA_OK = 0,
    QFCA_E_ARG = 1,          /* null pointer or out-of-range parameter */
    QFCA_E_SHAPE = 2,        /* H, W inconsistent with the parameters (e.g. smaller than T) */
    QFCA_E_NOMEM = 3,        /* device or host allocation failed */
    QFCA_E_DEVICE = 4,       /* a HIP call failed; recreate the context */
    QFCA_E_STATE = 5,        /* model not ready for this call (e.g. no reference yet) */
    QFCA_E_NONFINITE = 6,    /* NaN or Inf met where the fit needs finite values */
    QFCA_E_UNSUPPORTED = 7   /* parameters outside what the library implements */
} qfca_status;

enum { QFCA_PRE_NONE = 0,       /* plain QFCA: histogram the features as given */
       QFCA_PRE_RESIDUAL = 1,   /* QFCA+: histogram W - PCA^-1(PCA(W)), Sec. 3.3 */
       QFCA_PRE_COORDS = 2 };   /* histogram the k principal coordinates PCA(W) = V^T (W - mu)
                                   and score each window by its 1-Wasserstein distance to the
                                   reference (Sec. 3.1), box-averaged over the windows holding a
                                   pixel, without per-bin association: bins are [k][H][W] */

enum { QFCA_PREC_FP32 = 0,      /* projection in FP32 */
       QFCA_PREC_BF16 = 1 };    /* projection on BF16 MFMA, FP32 accumulate */

/* How the reference histogram is taken from the full T x T windows of the fit
 * image (Sec. 3.2; the choices of Sec. 4.5.3, Tab. 3). */
enum { QFCA_REF_MEDIAN_QUAN = 0,  /* rank-wise lower median of the sorted windows, then
                                     quantised (the paper's choice; default) */
       QFCA_REF_MEAN_QUAN = 1,    /* rank-wise mean of the sorted windows, then quantised */
       QFCA_REF_QUAN_MEDIAN = 2,  /* bin-wise lower median of the window histograms (mass:
                                     the sum of the medians) */
       QFCA_REF_QUAN_MEAN = 3 };  /* bin-wise mean of the window histograms (fractional) */

/* Method parameters.  Paper defaults: B = 16 bins (Sec. 4.5.1), k = 10
 * principal components (Sec. 4.5.2), sigma_p = infinity (box association),
 * sigma_s = 1 (Sec. 4.5.4), median -> quan reference (Sec. 4.5.3).
 *   C        channels, 1..2048
 *   k        principal components removed, 0..min(64, C-1) (ignored for
 *            PRE_NONE); for PRE_COORDS the histogrammed coordinates, 1..min(64, C)
 *   B        bins N of Sec. 3.1, 1..64
 *   T        patch side, odd, 1..63
 *   q_lo/hi  quantisation range as per-channel quantiles, 0 <= q_lo < q_hi <= 1
 *   sigma_s  final Gaussian blur, 0 (none) .. 5 px
 *   preproc  QFCA_PRE_*
 *   proj_prec QFCA_PREC_*
 *   sigma_p  association weights (Eq. 2, Sec. 4.5.4): the error of a pixel's
 *            bin in the window centred at p is weighted by
 *            exp(-|p - x|^2 / (2 sigma_p^2)) over the T x T windows holding
 *            the pixel (renormalised over those inside the image); INFINITY
 *            (the default) is the plain mean.  > 0.
 *   reference QFCA_REF_* (used by the fit) */
typedef struct {
    int32_t C, k, B, T;
    float q_lo, q_hi, sigma_s;
    int32_t preproc, proj_prec;
    float sigma_p;
    int32_t reference;
} qfca_params;

typedef struct qfca_ctx_s* qfca_ctx;
typedef struct qfca_model_s* qfca_model;

const char* qfca_status_str(qfca_status s);
/* Message describing the calling thread's last failed call ("" if none). */
const char* qfca_last_error(void);
/* Library version, as 10000*major + 100*minor + patch. */
int32_t qfca_version(void);

/* Create a context on HIP device `device`, issuing work on `hip_stream` (a
 * hipStream_t, borrowed; NULL means the default stream).  The context owns a
 * grow-only scratch arena and the tile-configuration cache. */
qfca_status qfca_ctx_create(int32_t device, void* hip_stream, qfca_ctx* out);
qfca_status qfca_ctx_set_stream(qfca_ctx ctx, void* hip_stream);
qfca_status qfca_ctx_destroy(qfca_ctx ctx);

/* Per-kernel timing for benchmarking: the library records a pair of HIP
 * events on the context's stream around every launch of the selected
 * kernels below (a few microseconds of overhead per launch).  enable: 0
 * turns timing off, -1 times every kernel, any other value is a bitmask
 * (bit k selects kernel id k).
 * qfca_ctx_profile_read synchronises on the recorded events and returns the
 * summed duration (ms) and the number of launches of one kernel since the
 * previous read, then resets that kernel's record.  Kernel ids:
 *   0 score (zeroing of the channel sum, window histograms, Alg. 1,
 *   association, channel sum), 1 projection + quantisation, 2 channel mean
 *   and blur. */
qfca_status qfca_ctx_profile(qfca_ctx ctx, int32_t enable);
qfca_status qfca_ctx_profile_read(qfca_ctx ctx, int32_t kernel, double* total_ms,
                                  int64_t* launches);

/* Tile configuration of the score kernel for later qfca_score_map calls on
 * this context: Ws output columns per strip, Hb output rows per band, S
 * channels per wavefront (S * lanes-per-channel <= 64, where lanes per
 * channel is the next power of two >= max(B, 8)) and the kernel variant
 * (0: column walk for any T; 1: block walk, T in 3..31).  The block walk
 * rounds Ws down to a multiple of T (at least T), which places its blocks of
 * T patch columns at the same image columns in every tiling: its maps are
 * then bitwise the same for every (Ws, Hb, S).  Ws == 0 restores the
 * automatic choice.  A tile that does not fit in LDS makes the later score
 * call fail with QFCA_E_UNSUPPORTED. */
qfca_status qfca_ctx_set_tile(qfca_ctx ctx, int32_t Ws, int32_t Hb, int32_t S, int32_t variant);

/* Zero-shot fit on one image (Sec. 3.2, Sec. 3.3).  Synchronous.
 * X: device [C][H][W] float32 with H, W >= T.  Computes, in order:
 *   mean mu and covariance (FP64 on the GPU); the top-k eigenvectors V of the
 *   covariance (host FP64 symmetric eigensolver, since a C x C problem is too
 *   small for the GPU); the residual r = (x - mu) - V V^T (x - mu) with the
 *   projection of params->proj_prec; per-channel type-7 quantiles q_lo, q_hi
 *   of r (exact order statistics on the GPU) giving lo, hi, delta = (hi-lo)/B
 *   and float32 edges lo + m delta; the bins; and the median reference: for
 *   every bin i, cR(i) is the ceil(P/2)-th largest full-window cumulative
 *   count among the P full T x T windows (the rank-wise lower median of the
 *   patches, quantised after the median).
 * On success *out is a new model (free it with qfca_model_destroy). */
qfca_status qfca_fit_pca(qfca_ctx ctx, const qfca_params* params, const float* X,
                         int32_t H, int32_t W, qfca_model* out);

/* Build a model from host arrays, for instance one fitted elsewhere.
 * mu [C], V [C][k] (row-major, column j = j-th principal axis), edges
 * [C][B-1] float32 nondecreasing per channel (a channel of +inf edges is
 * degenerate), delta [C] (bin width, feature units, >= 0), cR [C][B]
 * cumulative reference histogram with cR[c][B-1] == T*T, nondecreasing, or
 * NULL to leave the reference unset (then call qfca_fit_reference).  mu and V
 * may be NULL when preproc == QFCA_PRE_NONE or k == 0. */
qfca_status qfca_model_create(qfca_ctx ctx, const qfca_params* params, const float* mu,
                              const float* V, const float* edges, const double* delta,
                              const int32_t* cR, qfca_model* out);

/* (Re)compute the model's reference from device bins [C][H][W] (H, W >= T)
 * by params->reference: median -> quan exactly in integers (Sec. 3.2),
 * quan -> median and quan -> mean from the count table of the windows' bin
 * counts (Tab. 3).  mean -> quan needs the real values and is computed by
 * qfca_fit_pca only (QFCA_E_UNSUPPORTED here).  Synchronous. */
qfca_status qfca_fit_reference(qfca_ctx ctx, qfca_model model, const uint8_t* bins,
                               int32_t H, int32_t W);

/* Set a general reference: cRw host [C][B] cumulative weights, nonnegative,
 * nondecreasing per channel, finite (any total mass M_R > 0 or 0; Alg. 1
 * accepts arbitrary weights, Sec. 3.1: each window is compared after scaling
 * both histograms to equal mass).  Integer weights of mass T*T take the
 * integer path of a qfca_model_create reference; any other reference is
 * scored by the column-walk kernel in double precision.  Synchronous. */
qfca_status qfca_model_set_reference(qfca_ctx ctx, qfca_model model, const double* cRw);

/* Quantisation (Sec. 3.1, Sec. 3.3).  X: device [C][H][W] float32.
 * bins: device [C][H][W] uint8 out, bins = #{m : r >= edge_m} with r the
 * residual (PRE_RESIDUAL) or the feature (PRE_NONE) in float32, compared
 * against the float32 edges (a value equal to an edge goes to the upper bin).
 * resid: optional device [C][H][W] float32 out (NULL to skip).
 * For PRE_COORDS, bins and resid are [k][H][W]: the principal coordinates
 * z = V^T (x - mu) (FP32 or BF16 MFMA with FP32 accumulation) and their bins. */
qfca_status qfca_quantize(qfca_ctx ctx, qfca_model model, const float* X, int32_t H,
                          int32_t W, uint8_t* bins, float* resid);

/* Patch statistics comparison, association, aggregation and blur
 * (Sec. 3.1, Alg. 1, Sec. 4.5.4).  bins: device [C][H][W] uint8, every value
 * < B.  For every pixel p the T x T window (clipped to the image) is
 * histogrammed and compared with the reference by Algorithm 1 after scaling
 * both to equal mass; each bin's error (bin units) is averaged over the
 * windows that contain a pixel of that bin (sigma_p = infinity) and gathered
 * at the pixel's own bin; channels are averaged with weight delta_c; the map
 * is blurred with sigma_s (renormalised at the border).
 *   score: device [H][W] float32 out (required)
 *   amap:  device [H][W] float32 out, the map before the blur (nullable)
 *   w1:    device [H][W] float32 out, channel mean of delta_c times the window
 *          1-Wasserstein distance sum_k |cP_k - cR_k| / (n_p n_R) (nullable)
 *   achan: device [C][H][W] float32 out, per-channel delta_c-weighted maps
 *          before the channel mean (nullable; an inspection output, the
 *          channel mean does not read it)
 * The channel mean is summed in 64-bit fixed point with integer atomics
 * (each per-channel value rounded once, at 2^-62 of the largest possible
 * sum), so it does not depend on the order of the channel groups; with the
 * block walk (T in 3..31) every output is bitwise independent of the tile.
 * Library scratch: 8 bytes per pixel (16 with w1).
 * PRE_COORDS models (bins [k][H][W]): amap is the mean over the windows
 * holding each pixel of the coordinate-mean window W1 map (w1), score its
 * blur; achan must be NULL.
 * Requires a model with a reference (QFCA_E_STATE otherwise). */
qfca_status qfca_score_map(qfca_ctx ctx, qfca_model model, const uint8_t* bins, int32_t H,
                           int32_t W, float* score, float* amap, float* w1, float* achan);

/* qfca_score_map for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, outputs and arithmetic (bit for bit), but the
 * library's scratch is a fixed device array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends, so the call makes
 * no device allocation.  Limit: H * W <= 4194304 pixels (2048 x 2048);
 * larger maps give QFCA_E_UNSUPPORTED.  The scratch is cleared by the call
 * itself.  Every call on one GPU uses that GPU's single array: calls that
 * overlap on one GPU (on different streams, or from different contexts or
 * threads) race and give wrong maps; order them on one stream. */
qfca_status qfca_score_map_noalloc(qfca_ctx ctx, qfca_model model, const uint8_t* bins, int32_t H,
                                   int32_t W, float* score, float* amap, float* w1, float* achan);

/* Inspection of the integer stages of qfca_score_map (Sec. 3.1, Alg. 1):
 * runs the same score kernel code, built to also store, for every pixel p
 * (window centre) and every bin j < B of every channel c,
 *   cp: device [C][H][W][B] int32 out, cp[c][p][j] = #{q in N(p) : b_c(q) <= j},
 *       the window's cumulative histogram (N(p) the T x T window clipped to
 *       the image, n_p = |N(p)|);
 *   I:  device [C][H][W][B] int32 out, the transport numerator of bin j:
 *       sum_i |i - j| pi_ji over the monotone coupling of the patch masses
 *       P_j T^2 and the reference masses R_i n_p (both of total T^2 n_p),
 *       so that the bin's error is I / (P_j T^2) in bin units.
 * Every value is an exact integer.  Needs the block walk (T in 3..31;
 * QFCA_E_UNSUPPORTED otherwise) and a model with a reference.  Slow (a
 * store per window and bin): for testing.  Stream-ordered. */
qfca_status qfca_inspect_windows(qfca_ctx ctx, qfca_model model, const uint8_t* bins, int32_t H,
                                 int32_t W, int32_t* cp, int32_t* I);

/* One image of a batch. */
typedef struct {
    qfca_model model;  /* fitted model; all jobs of a batch share C, k, B, T, sigma_s,
                          preproc and proj_prec (the values of mu, V, edges and cR may differ) */
    const float* X;    /* device [C][H][W] float32 features */
    int32_t H, W;      /* any size >= 1 */
    float* score;      /* device [H][W] float32 out */
    uint8_t* bins;     /* device [C][H][W] uint8 out, or NULL for library scratch */
    float* amap;       /* device [H][W] float32 out (map before the blur), or NULL */
    float* achan;      /* device [C][H][W] float32 out, per-channel maps as in
                          qfca_score_map (inspection output), or NULL */
} qfca_job;

/* Quantise and score n (1..256) images of different sizes: one persistent
 * kernel drains a device work queue holding the projection tiles of every
 * image followed by their score tiles (a score tile waits for its image's
 * projection tiles), then a batched channel-mean and blur kernel runs; the
 * launch sequence is a HIP graph captured once per context and shape class
 * and replayed.  Stream-ordered like qfca_score_map; the arithmetic is that
 * of qfca_quantize + qfca_score_map with the block walk, so every output is
 * bitwise the one those calls give for the same image, whatever the other
 * images of the batch and the tile.  Requires preproc = QFCA_PRE_RESIDUAL,
 * T odd in 3..31, C <= 512 and k in 1..64 (the kernel is instantiated for
 * channel/component paddings (64, 16), (256, 32), (512, 64) in FP32 and
 * (256, 32), (512, 64) in BF16; a model keeps operand tables padded to the
 * smallest one that holds it); QFCA_E_UNSUPPORTED otherwise. */
qfca_status qfca_score_batch(qfca_ctx ctx, const qfca_job* jobs, int32_t n);

/* Synchronises the context's stream and reports whether a batch on it gave
 * up waiting for its projection tiles (*failed = 1; never expected). */
qfca_status qfca_batch_error(qfca_ctx ctx, int32_t* failed);

/* Tile autotuner: runs the batch `jobs` with candidate score tiles (strip
 * widths n T, band heights 64..256) timed with HIP events, keeps the
 * fastest as this context's tile for later score calls (single image and
 * batch) with the same (T, B), and returns it.  Synchronous; overwrites the
 * jobs' outputs. */
qfca_status qfca_autotune(qfca_ctx ctx, const qfca_job* jobs, int32_t n, int32_t* best_Ws,
                          int32_t* best_Hb, double* best_ms);

/* Model queries.  qfca_model_read copies one field to host memory:
 *   field 0 mu [C] float32, 1 V [C][k] float32, 2 edges [C][B-1] float32,
 *   3 delta [C] float64, 4 cR [C][B] int32 (integer references of mass T*T
 *   only), 5 eigenvalues [C] float64 (descending; fit only), 6 lo [C]
 *   float64, 7 hi [C] float64, 8 reference weights [C][B] float64 (any
 *   reference).
 * bytes must equal the field size; QFCA_E_STATE if the field is not set. */
qfca_status qfca_model_params(qfca_model model, qfca_params* out);
qfca_status qfca_model_read(qfca_model model, int32_t field, void* host_dst, size_t bytes);
/* Frees a model.  No work that uses it may still be queued on any stream.
 * Releasing device memory waits until the device is idle, so this stalls
 * every stream of the device (a live server's included) for as long as its
 * queued work takes: destroy models outside latency-critical loops. */
qfca_status qfca_model_destroy(qfca_model model);

/* Model serialisation, for storing fitted models (for instance one per
 * texture class, Sec. 3.3) and loading them elsewhere.  qfca_model_export
 * writes the model into host memory: with host_buf NULL it only sets
 * *inout_bytes to the size needed; otherwise *inout_bytes is the buffer's
 * size on entry (QFCA_E_ARG if too small, with the size needed set) and the
 * bytes written on return.  The format holds the parameters, mu and V in
 * double precision, the float32 edges, delta, and (when set) the reference
 * cR, the eigenvalues and lo/hi, in host byte order behind a magic and a
 * version.  qfca_model_import builds a new model on ctx's device from such a
 * buffer (bytes must be its exact size), validated like qfca_model_create;
 * the imported model quantises and scores bit for bit like the exported one.
 * Both are synchronous; the caller owns host_buf. */
qfca_status qfca_model_export(qfca_model model, void* host_buf, size_t* inout_bytes);
qfca_status qfca_model_import(qfca_ctx ctx, const void* host_buf, size_t bytes, qfca_model* out);

/* ------------------------------------------------------------------------
 * Serving.  A server scores single images submitted one at a time, each
 * against a resident model (for instance one per texture class), with
 * continuous batching: a dispatcher thread owned by the server admits
 * pending requests into a batch (qfca_score_batch arithmetic: each result is
 * the one that image gets alone) whenever one of its launch slots is free
 * and their device working memory fits in the server's budget, and launches
 * it on that slot's own stream, so batches launched while others run
 * overlap on the device.  Admission is first-come first-served among
 * requests that can share a launch (same C, k, B, T, sigma_s, precision);
 * a request whose memory does not fit waits, and later requests of its kind
 * wait behind it.  Working memory per request is
 * 256-byte-aligned C*H*W (bins) + 8*H*W (fixed-point channel sum) bytes. */
typedef struct qfca_server_s* qfca_server;

typedef struct {
    uint64_t hbm_budget;   /* bytes of device memory for in-flight requests (one allocation) */
    int32_t max_inflight;  /* launch slots (streams), 1..8 */
    int32_t max_batch;     /* requests per launch, 1..256 */
    int32_t Ws, Hb;        /* score tile for every slot (0, 0: automatic) */
} qfca_server_config;

typedef struct {
    uint64_t ticket;      /* as returned by qfca_server_submit */
    int32_t status;       /* QFCA_OK, or the failure of the launch that held it */
    int32_t batch_size;   /* requests in the launch that held it */
    double t_submit;      /* qfca_clock() at submission */
    double t_launch;      /* qfca_clock() when its launch was issued */
    double t_done;        /* qfca_clock() when the dispatcher saw the launch complete */
} qfca_completion;

typedef struct {
    uint64_t submitted, completed, failed, launches;
    uint64_t deferred_memory;     /* launches cut short because memory did not fit */
    int32_t max_inflight_seen;    /* most launches in flight at once */
    int32_t max_batch_seen;       /* largest launch */
    uint64_t arena_bytes, arena_peak;
    double device_busy_s;         /* union of the launches' device intervals (HIP events) */
    double device_span_s;         /* first launch start to last launch end */
    uint64_t overlapped;          /* launches whose device interval met another launch's */
} qfca_server_counters;

/* Seconds of the host's monotonic clock (CLOCK_MONOTONIC), the clock of
 * qfca_completion's times. */
double qfca_clock(void);

/* Creates a server on `device`: allocates the budget, one stream and
 * context per slot, and starts the dispatcher thread.  QFCA_E_NOMEM if the
 * budget cannot be allocated. */
qfca_status qfca_server_create(int32_t device, const qfca_server_config* cfg, qfca_server* out);

/* Queues one request and returns at once with its ticket.  X: device
 * [C][H][W] float32 and score: device [H][W] float32 out, both owned by the
 * caller and left untouched by it until the ticket completes.  model must
 * have a reference and satisfy qfca_score_batch's conditions.
 * QFCA_E_NOMEM if the request alone exceeds the budget. */
qfca_status qfca_server_submit(qfca_server server, qfca_model model, const float* X, int32_t H,
                               int32_t W, float* score, uint64_t* ticket);

/* Moves up to cap completions (in completion order) to out; *n receives how
 * many.  Non-blocking. */
qfca_status qfca_server_poll(qfca_server server, qfca_completion* out, int32_t cap, int32_t* n);

/* Blocks until every submitted request has completed. */
qfca_status qfca_server_drain(qfca_server server);

qfca_status qfca_server_stats(qfca_server server, qfca_server_counters* out);

/* Drains, stops the dispatcher and frees the server. */
qfca_status qfca_server_destroy(qfca_server server);

/* The host FP64 symmetric eigensolver used by qfca_fit_pca (Householder
 * tridiagonalisation, then implicit QL), exposed for testing.  A: host
 * [n][n] row-major symmetric (destroyed); evals: host [n] out, descending;
 * vecs: host [n][n] out, row-major, column j the unit eigenvector of
 * evals[j] with its largest-magnitude entry positive.  Returns 0, or -1 if
 * the iteration fails to converge or n < 1.  Needs no GPU. */
int qfca_host_sym_eig(double* A, int32_t n, double* evals, double* vecs);

/* The variant qfca_fit_pca uses: all eigenvalues (evals [n], descending) but
 * only the k leading eigenvectors (vecs: host [n][k] out, row-major, column
 * j for evals[j], largest-magnitude entry positive), by inverse iteration on
 * the tridiagonal form (close eigenvalues orthogonalised against each other)
 * and the stored Householder reflectors.  0 <= k <= n.  Returns 0, or -1 on
 * failure.  Needs no GPU. */
int qfca_host_sym_eig_top(double* A, int32_t n, int32_t k, double* evals, double* vecs);

#ifdef __cplusplus
}
#endif
#endif /* QFCA_H */
