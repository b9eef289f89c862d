/*
 * libzoomhash: the data-parallel hot path of patch-hashing image zoom
 * (Das Gupta, "Hashing Image Patches for Zooming", arXiv:1004.3980) on
 * AMD Instinct MI355X (gfx950).
 *
 * For every overlapping 5x5 patch of a low-resolution (LR) image the library
 * finds neighbours in a training dictionary of LR/HR patch pairs with p-stable
 * (Cauchy) locality-sensitive hashing, solves the LLE reconstruction weights,
 * synthesises the high-resolution (HR) patches with those weights, blends the
 * overlaps and refines the result by error back-projection with an
 * approximate cross bilateral filter.
 *
 * Conventions
 *  - Every array argument is a HIP device pointer owned by the caller unless
 *    its comment says "host". Images are fp32, row-major, values nominally in
 *    [0, 1] (never clamped).
 *  - A context owns one HIP stream (the caller's, or the null stream) and all
 *    work is enqueued on it asynchronously; device faults surface at a later
 *    call or at zh_sync. Argument and state errors return immediately and
 *    enqueue nothing.
 *  - No call aborts or throws across this boundary. On failure a call
 *    returns a nonzero zh_status and zh_last_error() describes it.
 *  - One context per host thread. Calls on one context are not thread-safe.
 *  - Patch order: patch q of an h x w LR image has top-left corner
 *    (i, j) = (q / (w-4), q % (w-4)); Q = (h-4)(w-4).
 *  - Environment: ZH_MEM_LIMIT (bytes) caps the library's device
 *    allocations; ZH_HASH_FIX_CAP (0..16) overrides the number of entries,
 *    per 16 feature rows, of the list through which codes that the MFMA
 *    projection cannot certify reach the FP64 recomputation (0 sends every
 *    such table through the slower per-row path; results are identical
 *    either way).
 */
#ifndef ZOOMHASH_H
#define ZOOMHASH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t zh_status;
enum {
    ZH_OK = 0,
    ZH_EINVAL = 1,        /* bad argument (size, pointer, parameter range) */
    ZH_ESTATE = 2,        /* call out of order (e.g. zh_reconstruct before zh_lle_weights) */
    ZH_ENOMEM = 3,        /* device allocation failed or exceeded ZH_MEM_LIMIT */
    ZH_EDEVICE = 4,       /* HIP runtime or kernel launch error */
    ZH_EUNSUPPORTED = 5,  /* valid request outside what this build implements */
    ZH_EIO = 6            /* a file could not be read or written, or is damaged */
};

typedef struct zh_ctx zh_ctx;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream). *out receives the context. */
zh_status zh_create(zh_ctx** out, int device, void* hip_stream);
/* Release every device buffer the context owns. NULL is ignored. */
void zh_destroy(zh_ctx* ctx);
zh_status zh_set_stream(zh_ctx* ctx, void* hip_stream);
/* Wait for the context's stream; reports device errors of earlier calls. */
zh_status zh_sync(zh_ctx* ctx);
/* Message of the last failure on this context; owned by the context, valid
 * until the next call on it. Never NULL. */
const char* zh_last_error(const zh_ctx* ctx);

/* ---- training data (Section 2.1: Gaussian blur then decimation) -------- */

/* lr[ceil(H/s), ceil(W/s)] = (g * hr)[s i, s j]: g the normalised Gaussian of
 * `sigma` over offsets -ceil(3 sigma)..ceil(3 sigma) (host libm exp), replicate
 * border; evaluated in FP64 (rows first, taps in ascending order) and rounded
 * once to fp32. hr holds n_img images of H x W. sigma in (0, 5]. */
zh_status zh_degrade(zh_ctx* ctx, const float* hr, int n_img, int H, int W, int scale,
                     float sigma, float* lr);

/* Feature modes (Section 4.1, "Feature representation"). */
enum { ZH_FEAT_MEANREM = 0,   /* D = 25: the patch's pixels minus their mean */
       ZH_FEAT_GRAD4 = 1 };   /* D = 100: 5x5 windows of dx, dy, dxx, dyy maps
                                 (taps [-1,0,1], [-1,0,2,0,-1], replicate border),
                                 channel-major, row-major inside a channel */

/* Cut n training pairs from n_img HR images [n_img, H, W] at LR positions
 * pos[n, 3] = (image, i, j) (int32, device): the LR image is the degradation
 * of the HR image by `sigma` and `scale`; feat[n, D] is the LR patch's
 * feature vector and resid[n, (5s)^2] the HR patch at (s i, s j) minus the
 * mean of the LR patch. Row n is pair ID n (Section 2.1: unique integer IDs).
 * Positions must satisfy 0 <= image < n_img, 0 <= i <= floor(H/s) - 5 and
 * 0 <= j <= floor(W/s) - 5 (the HR patch inside the image): a device kernel
 * checks them before anything is cut, and any position outside returns
 * ZH_EINVAL with feat and resid untouched (the call then synchronises the
 * context's stream). Uses a temporary device buffer of
 * n_img * ceil(H/s) * ceil(W/s) * 5 floats. */
zh_status zh_make_dictionary(zh_ctx* ctx, const float* hr, int n_img, int H, int W,
                             const int32_t* pos, int64_t n, int scale, float sigma,
                             int feat_mode, float* feat, float* resid);

/* Interpolated pairing (Section 2.1: the LR training images are interpolated
 * back to the size of the HR images and both are cut into overlapping
 * patches at the same places). zh_upsample writes that interpolation of an
 * LR image lr[h, w] into out[scale h, scale w]: bicubic, Keys' cubic with
 * a = -0.5, HR pixel X sampling LR coordinate X / scale (phase 0), taps
 * floor - 1 .. floor + 2 with replicate border, in FP64 (along x for each of
 * the four rows, then along y; the weights from the host's libm) and rounded
 * once to fp32. 1 <= scale <= 4.
 * zh_make_dictionary_interp cuts n pairs at HR-grid positions pos[n, 3] =
 * (image, r, c), 0 <= r <= H - 5, 0 <= c <= W - 5 (checked as for
 * zh_make_dictionary): the LR patch is the 5 x 5 patch at (r, c) of the
 * degraded image (sigma, scale) interpolated back by zh_upsample, its
 * features feat[n, D] as for zh_make_dictionary, and resid[n, 25] the 5 x 5
 * HR patch at (r, c) minus the mean of the LR patch. H and W must be
 * multiples of scale. These pairs have 5 x 5 HR patches: build their tables
 * with dictionary scale 1 and query the zh_upsample of the LR image at
 * scale 1; zh_backproject_lr then refines the result against the LR image.
 * Temporary device buffer: n_img (H W (5 + 1 / scale^2)) floats. */
zh_status zh_upsample(zh_ctx* ctx, const float* lr, int h, int w, int scale, float* out);
zh_status zh_make_dictionary_interp(zh_ctx* ctx, const float* hr, int n_img, int H, int W,
                                    const int32_t* pos, int64_t n, int scale, float sigma,
                                    int feat_mode, float* feat, float* resid);

/* Training crops (Section 5, training data generation): draw crop centres
 * from the first-order-gradient distribution of each training image and cut
 * side x side crops around them.
 * imgs[n_img, H, W] fp32 (device); draws[n_img, m] 64-bit integers (device),
 * row i for image i. A pixel weighs q = floor((|dx| + |dy|) 2^20), dx and dy
 * the differences of its right and left (lower and upper) neighbours in FP64,
 * replicate border, q saturated at 2^32 - 1 (also for non-finite values).
 * Draw x picks the first pixel (row-major) whose inclusive cumulative weight
 * exceeds x mod T, T the image's total weight (pixel x mod (H W) if T = 0).
 * corners[n_img, m, 2] (device, int32): top-left (row, col) of each crop, the
 * centre minus side / 2 clamped so the crop lies inside the image.
 * crops[n_img, m, side, side] (device, fp32) or NULL: the crops themselves.
 * 1 <= side <= min(H, W), H W < 2^31, n_img <= 65535, n_img m < 2^31.
 * Scratch: n_img (144 ceil(H W / 1024) + 8) bytes held by the context. */
zh_status zh_sample_crops(zh_ctx* ctx, const float* imgs, int n_img, int H, int W,
                          const uint64_t* draws, int m, int side, int32_t* corners,
                          float* crops);

/* Feature rows of every stride-1 patch of one LR image: feat[Q, D] and the
 * patch means mu[Q] (FP64, may be NULL). */
zh_status zh_features(zh_ctx* ctx, const float* lr, int h, int w, int feat_mode, float* feat,
                      double* mu);

/* ---- hashing and tables (Section 3.2; Section 4.1, Eq. hash_fn, Eq. cauchy) */

typedef struct {
    int64_t n;             /* pairs, 1 <= n < 2^31 */
    int32_t dim;           /* D: 25 or 100 */
    int32_t scale;         /* zoom factor 1 .. 4: HR patch side 5*scale */
    int32_t feat_mode;     /* ZH_FEAT_* that produced `feat` */
    const float* feat;     /* [n, D] fp32; copied at build into the library's own
                              split storage (bf16 high half + low 16 bits) */
    const float* resid;    /* [n, (5 scale)^2] fp32 HR residuals; BORROWED: must
                              stay valid and unchanged while the tables are used */
} zh_dictionary;

/* Build L hash tables of k concatenated Cauchy hashes of bin width w for the
 * dictionary of `scale` (one dictionary per scale; rebuilding replaces it).
 * Hash parameters: per table l an independent SplitMix64 stream with state
 * fmix64(seed + 0x9E3779B97F4A7C15 (l+1)); standard normals by Marsaglia's
 * polar method (first variate of each accepted pair); alpha = a/b with b
 * redrawn while |b| < 1e-3, k*D values in (hash, dim) order; then k values
 * beta = u w, u in [0,1). FP64, rounded to fp32. A bin is the 64-bit key of
 * the k codes c_j = floor((alpha.v + beta)/w) of a table l (Section 4.1:
 * "based on the k integers we form the bins"):
 *   key = fmix64(M[l][63] + sum_j uint32(c_j) M[l][j]  mod 2^64),
 * M[l][j] the SplitMix64 output number 64 l + j + 1 from state 0 (output n is
 * fmix64(n 0x9E3779B97F4A7C15)), fmix64 the SplitMix64 output function; a key
 * equal to 2^64 - 1 becomes 2^64 - 2 (that value marks empty directory slots).
 * Codes equal the FP64 sequential dot-product definition exactly.
 * Limits: 1 <= L <= 64, 1 <= k <= 32, w > 0. */
zh_status zh_build_tables(zh_ctx* ctx, const zh_dictionary* dict, int L, int k, float w,
                          uint64_t seed);

/* Tables on disk (Section 2.1: the training patch pairs are stored on disk
 * and found again through their unique integer IDs). zh_save_tables writes
 * what zh_build_tables built for `scale` to the file `path` (host string):
 * a header (magic, version, n, D, scale, feature mode, L, k, w, seed, the
 * directory size, the error-bound constants, a 64-bit content hash of the
 * dictionary features, the size and content hash of every section, and a
 * hash of the header itself), then the hash parameters, the bucket-key
 * multipliers, the L bin directories with their presence filters, the IDs of
 * the L tables laid out bin by bin, the screen rows and the screen
 * directions: L (16 cap + cap / 2 + 4 n) + 64 n bytes and a few more, cap the
 * power of two with 2 n <= cap < 4 n (2.0 GB for 2M pairs and 24 tables).
 * Synchronises the context's stream.
 * zh_load_tables replaces the tables of dict->scale by those of the file for
 * the dictionary `dict` (as for zh_build_tables: its features are copied, its
 * HR residuals BORROWED); the features must be those the tables were built
 * on (same n, D, scale, mode and content hash, else ZH_EINVAL). A file that
 * is not a table file of this version, is truncated, or whose header or any
 * section does not match its hash gives ZH_EIO and leaves no tables for that
 * scale. The loaded tables are bitwise those that were saved: queries give
 * the results they gave before. */
zh_status zh_save_tables(zh_ctx* ctx, int scale, const char* path);
zh_status zh_load_tables(zh_ctx* ctx, const zh_dictionary* dict, const char* path);

/* Hashing quality (Section 4.1, determining r): the entropy in bits of each
 * table's bucket occupancy, -sum_b p_b log2 p_b with p_b the fraction of the
 * dictionary's rows in bucket b, written to the HOST array entropy[L] (FP64;
 * capacity = its length, at least L). Synchronises the context's stream. */
zh_status zh_table_entropy(zh_ctx* ctx, int scale, double* entropy, int capacity);

/* Copy the hash parameters of `scale` to HOST arrays alpha[L*k*D], beta[L*k]. */
zh_status zh_get_hash_params(zh_ctx* ctx, int scale, float* alpha_host, float* beta_host);

/* Codes (int32 [n, L*k], may be NULL) and bucket keys (uint64 [n, L], may be
 * NULL) of arbitrary feature rows feat[n, D] under the tables of `scale`. */
zh_status zh_hash(zh_ctx* ctx, int scale, const float* feat, int64_t n, int32_t* codes,
                  uint64_t* keys);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): zh_hash
 * with `keys` required, whose kernels take their scratch (the per-row dirty
 * mask and the fix list of the FP64 recomputation) from a fixed device array
 * of the library instead of the context's buffers, so that the call
 * allocates nothing. The array is 8 MiB per GPU, held from the first
 * zh_create on that GPU until the process ends; it bounds n to
 * floor((8 MiB - 512) / (9 + 4 f)) rounded down to a multiple of 16,
 * f = k + 2 rounded up to a multiple of 4 (79,872 rows at k = 20, 94,240 at
 * k = 16, 54,816 at k = 32); a larger n returns ZH_EINVAL and enqueues
 * nothing. Results equal those of zh_hash. Every call on one GPU shares that
 * array: calls that overlap on one GPU (other streams, other contexts, other
 * host threads) race, so order them. Nothing in the array has to start at
 * any value: each call writes what it reads. The count of codes fixed in
 * FP64 (zh_stats) is not updated by this call. */
zh_status zh_hash_noalloc(zh_ctx* ctx, int scale, const float* feat, int64_t n, int32_t* codes,
                          uint64_t* keys);

/* ---- query options ----------------------------------------------------- */
typedef struct {
    int32_t cap;           /* 0: candidates are the union of the L bins; > 0: the
                              early stop of Section 4.2 (tables in order, IDs
                              ascending in a bin, stop at cap distinct IDs),
                              cap <= 256 */
    int32_t rerank;        /* 0: exact ranking (fp32 distances certified against
                              the FP64 distance, exact K nearest by (d, ID));
                              R in [K, 64]: at most R candidates get fp32
                              distances; with cap > 0 those the screen's lower
                              bounds (int8 coordinates in the dictionary's
                              principal directions) do not rule out, smallest
                              bounds first; with cap = 0 the best R by a distance
                              on the bf16 high half of the features */
    int32_t proj;          /* projection on the matrix cores: 0 fp32, 1 split
                              bf16 (three bf16 products); both give exact codes */
    int32_t lle_fp64;      /* 1: Gram and solve in FP64; 0: fp32, FP64 only when
                              the Cholesky diagonal ratio squared exceeds 1e6 */
} zh_query_opts;
/* Defaults: cap 0, rerank 0, proj 1, lle_fp64 1. */
zh_status zh_set_query_opts(zh_ctx* ctx, const zh_query_opts* opts);

/* Distance by which zh_query ranks the candidates (Section 4.1: the Cauchy
 * hash is sensitive to l1 distances; the LLE objective is squared l2).
 * ZH_METRIC_L2 (the default): squared l2, as documented at zh_query.
 * ZH_METRIC_L1: the neighbours are the first min(K, M) early-stop candidates
 * in (l1 distance, ID) order, exactly those of zh_query under ZH_METRIC_L2
 * followed by zh_knn_l1, without the l2 ranking; needs the early stop
 * (query option cap > 0, else zh_query returns ZH_EUNSUPPORTED), the rerank
 * option does not apply, zh_get_results reports l1 distances, and
 * zh_run_batch and zh_tune_batch return
 * ZH_EUNSUPPORTED while it is set. Other values: ZH_EINVAL. Applies to later
 * calls of zh_query. */
enum { ZH_METRIC_L2 = 0, ZH_METRIC_L1 = 1 };
zh_status zh_set_query_metric(zh_ctx* ctx, int metric);

/* ---- the path --------------------------------------------------------- */

/* Section 3.2 and Section 4.2 (query every table, collect the matches, stop
 * early when there are more than a preset number of them), Section 3.1
 * step 1(a) (the K nearest neighbours): features (Section 4.1), codes and
 * bins of every stride-1 patch of the LR image lr[h, w] (copied into the
 * context), then the candidates of each patch (the union of its L bins, or
 * the early stop of the query options) and the K nearest of them by squared
 * l2 distance against the dictionary of `scale`. 1 <= K <= 16, h, w >= 5.
 * Neighbours are ordered by (distance, ID); a patch with fewer than K
 * candidates keeps all of them, one with none contributes no HR patch.
 * Results stay in the context (zh_get_results). */
zh_status zh_query(zh_ctx* ctx, const float* lr, int h, int w, int scale, int K);

/* The t-of-L candidate criterion (Section 4.1: a training patch matches
 * when it shares the query's bucket in at least t of the L tables) over the
 * bins of the last zh_query: counts[Q] (device) the number of such IDs of
 * each patch and ids[Q, cap_per_query] (device) the first cap_per_query of
 * them in table-walk order (bins in table order, IDs ascending in a bin,
 * each ID at the first table that holds it); entries past that are
 * untouched. 1 <= t <= L; t = 1 is the union of zh_candidates without a cap.
 * Leaves the neighbours of the query unchanged. */
zh_status zh_candidates_t(zh_ctx* ctx, int t, int32_t cap_per_query, int32_t* counts,
                          int32_t* ids);

/* Neighbours from the t-of-L candidates (Section 4.1): replace the
 * neighbours of the last zh_query by the first min(K, M_t) of its t-of-L
 * candidates (zh_candidates_t) in (squared l2 distance, ID) order, the
 * distance summed over the coordinates in index order in FP64 from the fp32
 * features; every t-of-L candidate is ranked, however many there are.
 * ncand then reports the t-of-L counts. zh_lle_weights and zh_reconstruct use
 * the new neighbours. 1 <= t <= L. */
zh_status zh_knn_t(zh_ctx* ctx, int t);

/* Re-rank under l1 (Section 4.1: the Cauchy hash is sensitive to l1
 * distances): replace the neighbours of the last zh_query by the first
 * min(K, M) of its early-stop candidates in (l1 distance, ID) order, the
 * distance summed over the coordinates in index order in FP64 from the fp32
 * features. zh_get_results then reports l1 distances (rounded to fp32) in
 * place of squared l2; zh_lle_weights and zh_reconstruct use the new
 * neighbours. Needs the early stop (query option cap > 0, else
 * ZH_EUNSUPPORTED); forms the candidate lists again (the union step of the
 * search alone). The counters of zh_stats then cover this call only (the
 * search's truncation count stays 0). */
zh_status zh_knn_l1(zh_ctx* ctx);

/* LLE weights of every patch (Section 4.2, Eq. LinSys): minimise
 * ||y - sum_m w_m y_m||^2 subject to sum_m w_m = 1, regularised by adding
 * lambda * trace(G) to the diagonal of the Gram matrix G (lambda > 0). */
zh_status zh_lle_weights(zh_ctx* ctx, double lambda);

/* LLE over all M matches (Section 4.2: Eq. LinSys and Eq. HR_Rec with m
 * running over every match the search found, not only the K nearest). Needs
 * the early stop of the last zh_query (query option cap, 1 <= cap <= 80;
 * else ZH_EUNSUPPORTED): the search runs again and lists each patch's M <=
 * cap candidates ascending; the weights minimise ||y - sum_m w_m y_m||^2
 * subject to sum_m w_m = 1 with lambda trace(G) added to the diagonal of the
 * M x M Gram matrix G (FP64: exact differences, Cholesky, two triangular
 * solves; uniform weights when trace(G) = 0). ids[Q, cap] and w[Q, cap]
 * (device, each nullable) receive the lists (-1 past M) and the weights
 * (0 past M). zh_reconstruct then synthesises every HR patch from all of
 * its M matches; zh_backward returns ZH_EUNSUPPORTED until the next
 * zh_lle_weights. */
zh_status zh_lle_all(zh_ctx* ctx, double lambda, int32_t* ids, float* w);

/* HR image hr_out[s h, s w]: each patch x_q = mean(LR patch) + sum_m w_m r_m
 * (Eq. HR_Rec on the residuals), overlaps averaged per pixel (Section 4
 * prior); pixels covered by no patch with a neighbour take the bicubic
 * (Keys a = -0.5) interpolation of the LR image. */
zh_status zh_reconstruct(zh_ctx* ctx, float* hr_out);

/* `iters` error back-projection steps in place on hr_inout[s h, s w]
 * (Section 4 update after Eq. Err_img; Section 4.3 approximate cross
 * bilateral filter, Eq. sx2 and Eq. bl_filter_3): e = I_L - (g * I)
 * decimated, E its bicubic upsampling, F the in-image-normalised Gaussian of
 * sigma_s over a (2R+1)^2 window (R = ceil(3 sigma_s) <= 8) applied to E,
 * S = exp(-(I - mean_window(I))^2 / (2 sigma_r^2)), I += S F. sigma_r may be
 * +inf (plain Gaussian back-projection). Uses the LR image of the last
 * zh_query and the blur sigma of the degradation (1.0). */
zh_status zh_backproject(zh_ctx* ctx, float* hr_inout, int iters, float sigma_s, float sigma_r);

/* The back-projection of zh_backproject on hr_inout[scale h, scale w]
 * against an explicit LR image lr[h, w] (device) and zoom factor (1 .. 4),
 * independent of the last query (the interpolated pairing of Section 2.1
 * queries the upsampled image at zoom factor 1 and is refined against the
 * original LR image). Not recorded for zh_backward: after it, zh_backward on
 * the last zh_reconstruct returns ZH_ESTATE. */
zh_status zh_backproject_lr(zh_ctx* ctx, float* hr_inout, const float* lr, int h, int w, int scale,
                            int iters, float sigma_s, float sigma_r);

/* Gradients of a loss L on the output image of the last zh_reconstruct,
 * or of the zh_backproject call that followed it on that image (one call;
 * after a second one the chain is not recorded and this returns ZH_ESTATE):
 *   g_hr[s h, s w]     (in)  dL/d output image;
 *   g_resid[N, (5s)^2] (out) dL/d the HR residual patches of the dictionary
 *                      used by the query (the same values as dL/d the HR
 *                      patches), overwritten, zero for rows no patch uses;
 *   g_lambda[1]        (out) dL/d lambda of the last zh_lle_weights.
 * Neighbour indices (hash codes, candidates, K nearest) are held at their
 * forward values. Adjoints of the back-projection iterations (Section 4,
 * Section 4.3; the range weight included, from the guides zh_backproject
 * keeps), of the blend, of the synthesis (Eq. HR_Rec) and of the LLE
 * weights through lambda (Eq. LinSys; Gram matrices recomputed and
 * factorised again in FP64). Deterministic: no floating-point atomics.
 * All pointers are device pointers; K <= 16, D <= 128. */
zh_status zh_backward(zh_ctx* ctx, const float* g_hr, float* g_resid, float* g_lambda);

/* ---- batched form ------------------------------------------------------ */

/* Many LR images of uneven size and zoom factor in one launch chain: for
 * each zoom factor present, the patches of all its images form one index
 * space for features, hashing, search, LLE weights and synthesis; the blend
 * and the back-projection run over the images' pixels and tiles (a
 * persistent update kernel takes (image, tile) items from a work counter).
 * The chain is captured once into a HIP graph and replayed while the batch
 * (pointers, sizes, parameters, query options, tuning) stays the same; it
 * runs on a stream of the context ordered after and before the context's
 * stream. Results equal those of zh_query, zh_lle_weights, zh_reconstruct
 * and zh_backproject run image by image. Afterwards the single-image query
 * state is cleared (zh_lle_weights etc. need a new zh_query). */
typedef struct {
    int32_t n_images;
    const float* const* lr;      /* host array [n_images] of device pointers, image i is [h[i], w[i]] */
    float* const* hr_out;        /* host array [n_images] of device pointers, [scale[i] h[i], scale[i] w[i]] */
    const int32_t* h;            /* host arrays [n_images]; h, w >= 5 */
    const int32_t* w;
    const int32_t* scale;        /* each with tables built (zh_build_tables) */
    int32_t K;                   /* neighbours, 1..16 */
    double lambda;               /* LLE regulariser, > 0 */
    int32_t bp_iters;            /* back-projection iterations, >= 0 */
    float sigma_s, sigma_r;      /* as zh_backproject */
} zh_batch;
zh_status zh_run_batch(zh_ctx* ctx, const zh_batch* batch);

/* Autotuner of the batched form (Section 5: the patches are independent
 * sub-problems; the launch shapes are chosen per batch): runs the batch once,
 * then times (HIP events, best of 2) the back-projection update over the
 * batch's tiles for tile sides {16, 32} and persistent grids of {2, 4, 8}
 * workgroups per compute unit, and the fused synthesis and blend of the last
 * zoom factor with tiles of 4 and 8 patch rows; keeps the fastest of each
 * for later zh_run_batch calls and reports them in *out (host, nullable).
 * The tile height is the context's for zh_reconstruct too: it sets how the
 * blend's sum of a pixel is grouped (patch rows of one tile, then tile by
 * tile), so outputs may change in the last bits after tuning, and the
 * batched and single-image results stay bitwise equal. The images' outputs
 * are overwritten. When the environment names a cache file
 * (ZH_TUNE_CACHE), a previous choice for the same device (name and
 * architecture), HIP runtime version and batch (sizes, zoom factors, K,
 * iterations, query options) is taken from it without timing (from_cache =
 * 1, timings 0), and a new choice is appended to it as one JSON object per
 * line. */
typedef struct {
    int32_t bp_tile;             /* chosen tile side */
    int32_t bp_grid_per_cu;      /* chosen workgroups per compute unit */
    float bp_ms[6];              /* per configuration (tile 16: 2, 4, 8; tile 32: 2, 4, 8), ms per iteration */
    int32_t synth_rows;          /* chosen patch rows per tile of the fused synthesis and blend (4 or 8) */
    float synth_ms[2];           /* synthesis and blend of the last zoom factor with tiles of 4 and 8 rows, ms */
    int32_t from_cache;          /* 1: the choice came from the cache file */
} zh_batch_tuning;
zh_status zh_tune_batch(zh_ctx* ctx, const zh_batch* batch, zh_batch_tuning* out);

/* ---- results and diagnostics ------------------------------------------ */

/* Copies of the last query's results (device pointers, each may be NULL):
 * ids[Q, K] int32 (-1 past m), d2[Q, K] squared distances (l1 distances
 * after zh_knn_l1), m[Q] neighbours used, w[Q, K] weights (after
 * zh_lle_weights), ncand[Q] distinct candidates (in early-stop mode at most
 * cap). */
zh_status zh_get_results(zh_ctx* ctx, int32_t* ids, float* d2, int32_t* m, float* w,
                         int32_t* ncand);
/* Candidates of each patch of the last zh_query that reached the exact
 * distance pass (after the screen's lower bounds; equal to the candidate
 * count when the screen did not run) into survivors[Q] (device); after
 * zh_knn_l1, or for a query under ZH_METRIC_L1, those that reached the exact
 * l1 pass (after the l1 screen at D = 100). Early-stop search only
 * (cap > 0); ZH_ESTATE otherwise. */
zh_status zh_survivors(zh_ctx* ctx, int32_t* survivors);
/* Query size of the last zh_query: *Q patches, *D feature dimension. */
zh_status zh_query_shape(zh_ctx* ctx, int64_t* Q, int32_t* D);

/* Re-run the candidate search of the last query and write each patch's
 * candidate IDs ascending into ids[Q, cap_per_query] (device) and their
 * number into counts[Q]; entries past min(count, cap_per_query) are untouched. */
zh_status zh_candidates(zh_ctx* ctx, int32_t cap_per_query, int32_t* counts, int32_t* ids);

typedef struct {
    uint64_t queries;           /* patches of the last zh_query */
    uint64_t codes_fixed;       /* codes decided by the FP64 recomputation */
    uint64_t rank_fallbacks;    /* patches re-ranked by FP64 distances */
    uint64_t deferred;          /* patches sent to the large-union path */
    uint64_t streamed;          /* patches whose bins hold more than 8192 IDs without
                                   a cap: their union is merged from the sorted bins
                                   and ranked by FP64 distances in a streaming pass */
    uint64_t lle_fp64;          /* fp32 solves redone in FP64 */
    uint64_t dict_bytes;        /* device bytes held for dictionaries and tables */
    uint64_t truncated;         /* screened early-stop search (rerank = R): patches
                                   whose candidates that the screen's lower bounds
                                   could not rule out numbered more than R; only
                                   the R with the smallest bounds were ranked, so
                                   their neighbours may differ from the exact ones
                                   (0: the screened neighbours are the exact K
                                   nearest up to fp32 ties) */
} zh_stats_t;
/* Counters of the last zh_query / zh_lle_weights (synchronises the stream). */
zh_status zh_stats(zh_ctx* ctx, zh_stats_t* out);

/* ---- stage timing (HIP events on the context's stream) ----------------- */
enum { ZH_T_FEATURES = 0, ZH_T_HASH = 1, ZH_T_SEARCH = 2, ZH_T_LLE = 3, ZH_T_SYNTH = 4,
       ZH_T_BLEND = 5, ZH_T_BP_ERROR = 6, ZH_T_BP_UPDATE = 7, ZH_T_ROTATE = 8, ZH_T_PROBE = 9,
       ZH_T_COUNT = 10 };
/* ZH_T_HASH times the projection, codes and keys (with their FP64 fixes);
 * ZH_T_PROBE the lookup of the keys' bins; ZH_T_SEARCH the candidate search
 * kernel alone; ZH_T_ROTATE the projection of the queries onto the
 * dictionary's screen directions that precedes it (early-stop search only). */
/* on != 0: bracket every kernel launch of the stages above with a pair of HIP
 * events (at most 256 launches per stage between two zh_get_timing calls;
 * later launches are not timed). on = 0 stops recording. */
zh_status zh_set_timing(zh_ctx* ctx, int on);
/* Times only the stages whose bit (1 << ZH_T_*) is set in mask (0 stops
 * recording). Every pair of events costs a short gap on the stream. */
zh_status zh_set_timing_stages(zh_ctx* ctx, uint32_t mask);
/* Synchronise, then write for each stage the summed milliseconds
 * (ms[ZH_T_COUNT]) and the number of timed launches (launches[ZH_T_COUNT],
 * may be NULL) since the previous
 * call, and start a new period. */
zh_status zh_get_timing(zh_ctx* ctx, double* ms, int32_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* ZOOMHASH_H */
