// Internal launcher interface of libzoomhash (host side). Every launcher
// enqueues on `st` and returns the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zh_device.h"

namespace zh {

constexpr int kPatch = 5;       // LR patch side
constexpr int kMaxScale = 4;    // zoom factors 1 .. 4 (HR patch side 5 s)
constexpr int kMaxPs2 = kPatch * kMaxScale * kPatch * kMaxScale;
constexpr int kMaxTaps = 33;    // longest 1-D Gaussian the kernels accept
constexpr int kMaxK = 16;       // neighbours per patch
constexpr int kMaxL = 64;       // hash tables
constexpr int kMaxKHash = 32;   // hashes per table
constexpr int32_t kCodeUnset = (int32_t)0x80000000;   // MFMA codes lie within +-2^23
constexpr int kFixSlots = 16;                        // fix-list entries per wave of 16 rows

// Device counters of the last query (uint32 each): patches deferred to the
// large-union search, FP64 re-ranks, patches beyond the large-union limit
// (ranked by the streaming merge), codes fixed in FP64, fp32 LLE solves redone
// in FP64, screened patches whose survivors exceeded the exact-row limit.
enum { C_OVERFLOW = 0, C_RANKFB = 1, C_STREAM = 2, C_CODEFIX = 3, C_LLE64 = 4, C_TRUNC = 5, kNumCounters = 8 };

struct Taps {                   // normalised 1-D Gaussian, offsets -R..R
    double g[kMaxTaps];
    int R;
};

// ---- image kernels (k_image.hip) -------------------------------------------
hipError_t launch_degrade(const float* hr, int n_img, int H, int W, int scale, const Taps& t,
                          float* lr, hipStream_t st);
// e = lr_ref - degrade(hr), fp32 [h, w]
hipError_t launch_degrade_residual(const float* hr, int H, int W, int scale, const Taps& t,
                                   const float* lr_ref, float* e, hipStream_t st);
hipError_t launch_gradient_maps(const float* lr, int n_img, int h, int w, float* maps,
                                hipStream_t st);
// features of every stride-1 patch of one LR image (row-major patch order)
hipError_t launch_query_features(const float* lr, const float* maps, int h, int w, int mode,
                                 float* feat, double* mu, hipStream_t st);
// flag[0] set to 1 when a position (image, i, j) of pos[n, 3] is outside
// [0, n_img) x [0, imax] x [0, jmax]
hipError_t launch_check_positions(const int32_t* pos, int64_t n, int n_img, int imax, int jmax, uint32_t* flag,
                                  hipStream_t st);
hipError_t launch_dict_cut(const float* hr, const float* lr, const float* maps, int H, int W,
                           int scale, const int32_t* pos, int64_t n, int mode, float* feat,
                           float* resid, hipStream_t st);
hipError_t launch_split_planes(const float* x, int64_t n, int D, uint16_t* hi, uint16_t* lo,
                               hipStream_t st);
hipError_t launch_bicubic(const float* lr, int h, int w, int scale, float* out, hipStream_t st);
// FP64 bicubic upsampling rounded to fp32 (the interpolated LR images of the
// training pairs); wt[4 r + a]: Keys' weight of tap a at phase r (host table)
hipError_t launch_upsample64(const float* lr, int h, int w, int scale, const double* wt, float* out, hipStream_t st);

// ---- hashing (k_hash.hip) ----------------------------------------------------
struct HashArgs {
    const float* feat;       // [n, D] fp32
    int64_t n;
    int D;
    int L, k;
    const float* alpha;      // [L*k, D] fp32
    const uint16_t* a_hi;    // [L*k, DP] bf16 high parts of fl(alpha / w) (split projection), DP = D rounded to 32
    const uint16_t* a_lo;    // [L*k, DP] bf16 low parts
    const float* beta;       // [L*k]
    const float* beta_w;     // [L*k] fl(beta / w) (split path; its a_hi, a_lo split fl(alpha / w))
    const float* bound_c0;   // [L*k] per-hash constant term of the code error bound
    float bound_c1;          // coefficient of the |alpha|.|v| MFMA value in the bound
    float bound_c2;          // coefficient of |alpha.v| (fp32 path)
    float inv_w;             // fp32 1/w
    float w;
    int prec;                // 0 = fp32 MFMA, 1 = split bf16 MFMA
    const uint64_t* key_mul; // [L, k + 1] multipliers of the key sum, then its start value
    uint64_t* keys;          // [n, L], or [L, n] when keys_tmajor
    int keys_tmajor;         // keys (and bins) stored table by table
    int32_t* codes;          // [n, L*k] or null
    unsigned int* n_fixed;   // count of codes recomputed in FP64 (nullable)
    uint64_t* dirty;         // [n] scratch: per row, bit l set when table l must be recomputed in full
    int32_t* fix_list;       // scratch: per wave of 16 rows, fix_cap entries (row, table, k codes;
                             // kCodeUnset where the FP64 definition must decide)
    int fix_cap;             // entries per wave (<= kFixSlots); tables beyond go to `dirty`
    unsigned int* fix_count; // [ceil(n/16)] entries written by each wave
    const Slot* dir;         // bin directories [L, dir_cap], or null: no lookup
    uint64_t dir_cap;
    const uint32_t* dir_filter;  // [L, dir_cap / 8] presence bits of the keys (dir_filter_bit)
    uint2* bins;             // [L, n] (offset, count) of each key's bin, when dir is set
                             // (needs keys_tmajor)
};
// Presence filter of a table's keys: min(4 dir_cap, 2^32) bits, a key's bit
// taken from its high half (the directory slot comes from the low bits).
// A clear bit proves the key absent; a set bit sends the lookup on to the
// directory.
__host__ __device__ inline uint64_t dir_filter_words(uint64_t cap) {
    const uint64_t w = cap / 8;
    return w < 1 ? 1 : (w > (1ull << 27) ? (1ull << 27) : w);
}
__host__ __device__ inline uint32_t dir_filter_bit(uint64_t key, uint64_t cap) {
    return (uint32_t)(key >> 32) & (uint32_t)(32 * dir_filter_words(cap) - 1);
}
// position of the key of (row, table)
__device__ __forceinline__ int64_t key_pos(const HashArgs& a, int64_t row, int l) {
    return a.keys_tmajor ? (int64_t)l * a.n + row : row * a.L + l;
}
hipError_t launch_hash(const HashArgs& a, hipStream_t st);   // codes and keys, then the bin lookup
hipError_t launch_hash_codes(const HashArgs& a, hipStream_t st);   // codes and keys (with their FP64 fixes)
hipError_t launch_probe(const HashArgs& a, hipStream_t st);        // the bins of the keys (a.bins set)
// bound coefficients for the MFMA projection of precision `prec` (host)
void hash_bound_coeffs(int prec, int D, double w, const float* beta, int m, float* c0, float* c1,
                       float* c2);

// ---- table build (k_table.hip) ----------------------------------------------
hipError_t launch_dir_clear(Slot* dir, uint64_t count, hipStream_t st);
// also sets the key bits of the table's presence filter (cleared beforehand)
hipError_t launch_dir_insert(const uint64_t* keys, int64_t n, int L, int l, Slot* dir,
                             uint64_t cap, uint32_t* filter, uint32_t* slot_of, uint32_t* ids, hipStream_t st);
hipError_t launch_dir_offsets(const uint32_t* sorted_slot, int64_t n, Slot* dir, hipStream_t st);
// stable LSD radix sort of (key, val) pairs on the low `bits` bits of key
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                            int bits, uint32_t* hist, int64_t hist_cap, hipStream_t st,
                            bool* result_in_first);
int64_t radix_hist_size(int64_t n);
// adds the content hash of n_words 32-bit words at p into *out (cleared by
// the caller): sum_i fmix64((i G + salt) ^ word_i) mod 2^64, G = kGolden
hipError_t launch_hash_words(const void* p, int64_t n_words, uint64_t salt, unsigned long long* out,
                             hipStream_t st);

// ---- search (k_search.hip) ---------------------------------------------------
struct SearchArgs {
    int Q, D, L, K, cap, rerank, exact;
    int hsz, cp;             // LDS hash set slots, candidate slots (set by the launcher)
    int hs;                  // row stride of the high plane (halfwords)
    float ce;                // relative error coefficient of the screen's |y_q - y~_x|^2
    const uint8_t* sc;       // [N, kScreenBytes] screen plane (early-stop search)
    const float* xf;         // [N, D] fp32 features: the exact passes of the early-stop search
    const float* qrot;       // [Q, kRotStride] coded rotated queries (k_rotate)
    float inv_s2;            // lower bound of 1 / sigma_max(Phi)^2
    double dist_eps;         // 2 gamma_{D+3}: relative bound of an fp32 distance (set by the launcher)
    void* gram;              // [Q, 36] packed Gram matrices of the neighbours (K <= 8), or null
    int gram_fp64;           // their precision: FP64 or fp32
    const uint2* bins;       // [L, Q] (offset, count) of the query's bin in each table
    const float* qfeat;      // [Q, D]
    const uint32_t* tids;    // [L, N]
    int64_t N;
    const uint16_t* hi;
    const uint16_t* lo;
    int32_t* out_ids;        // [Q, K]
    float* out_d2;           // [Q, K]
    int32_t* out_m;          // [Q]
    int32_t* out_ncand;      // [Q]
    int32_t* out_nsurv;      // [Q] candidates given an exact distance (early-stop search), nullable
    int32_t* dump;           // [Q, dump_cap] or null
    int dump_cap;
    int cand_only;           // early-stop search: candidate counts (and the dump, in the union's order) only, neighbours untouched
    int32_t* overflow;       // [2 Q] deferred queries (uncapped, too many IDs for a wave), then those
                             // beyond the large-union limit
    unsigned int* counters;  // [0] overflow count, [1] FP64 rank fallbacks
};
hipError_t launch_search(const SearchArgs& a, hipStream_t st);
float screen_coeff();        // error coefficient of the search's int8 pre-filter (host)
// Row layout of the high plane: D bf16 values, zero padding to whole 16-byte
// rows with at least 4 halfwords of padding.
__host__ __device__ inline int hi_stride(int D) { return ((((D + 3) & ~3) + 4) + 7) & ~7; }
hipError_t launch_search_overflow(const SearchArgs& a, int n_over, hipStream_t st);

// ---- screen plane and rotated queries (k_screen.hip) --------------------------
// Screen row of a dictionary entry, 64 bytes: the coordinates y = Phi x in the
// m = screen_dims(D) leading principal directions as int8 codes c_j of one
// row scale s_x (bf16), y~ = s_x c, zeros to byte 56; then |y~|^2 (fp32),
// s_x and rho_x >= |Phi x - y~| (bf16, rounded up).
constexpr int kScreenMax = 56;
constexpr int kScreenBytes = 64;
__host__ __device__ inline int screen_dims(int D) { return D < kScreenMax ? D : kScreenMax; }
constexpr int kRotStride = 64;   // floats per coded query row (k_rotate)
// FP64 sum of x x^T over ns rows r_i = floor(i n / ns) (ns <= 65536); part holds
// 128 partial D x D matrices
hipError_t launch_cov(const float* x, int64_t n, int D, int64_t ns, double* part, double* cov, hipStream_t st);
// rows of Phi (m x D fp32) from the covariance; returns a bound on sigma_max(Phi)^2
double screen_basis(const double* C, int D, int m, float* phi);
float rotate_bound_coeff(int D);
// screen rows [n, kScreenBytes] from x [n, D]; phiT is FP64 [D][64]
hipError_t launch_screen_rows(const float* x, int64_t n, int D, int m, const double* phiT, uint8_t* sc,
                              hipStream_t st);
// coded rotated queries [n, kRotStride] from feat [n, D] (int8 codes h, l of
// y_q = Phi q, then s_q, |y^|^2, rho_q); Phi split into bf16 [64][round32(D)] planes
hipError_t launch_rotate(const float* feat, int64_t n, int D, const uint16_t* p_hi, const uint16_t* p_lo, float c1,
                         float* out, hipStream_t st);

// ---- LLE, synthesis, blend (k_lle.hip) --------------------------------------
struct LleArgs {
    int Q, D, K;
    int hs;                  // row stride of the high plane (halfwords)
    const float* qfeat;
    const int32_t* ids;
    const int32_t* m;
    const uint16_t* hi;
    const uint16_t* lo;
    const float* xf;         // [n, D] fp32 copy of the same features (16-byte aligned rows when D % 4 == 0), or null
    double lam;
    int fp64;                // 1: FP64 Gram and solve; 0: FP32, FP64 redo when cond > 1e6
    float* w;                // [Q, K]
    unsigned int* n_fp64;    // FP64 redo count (nullable)
};
hipError_t lle_init();  // once per device, before any launch_lle
// packed Gram matrices [Q, 36] of the <= 8 neighbours (Z = query - rows),
// two patches per wave; then the weights from them, one thread per patch
hipError_t launch_gram(const LleArgs& a, void* gram, int gram_fp64, hipStream_t st);
hipError_t launch_lle_solve(const LleArgs& a, const void* gram, int gram_fp64, hipStream_t st);
hipError_t launch_lle(const LleArgs& a, hipStream_t st);
// LLE over all M <= cap matches of each patch: cand[Q, cap] (IDs, M = ncand
// capped; entries past M set to -1), weights w[Q, cap] (0 past M); Gram and solves in FP64; the LDS of
// a workgroup (packed Gram, rows) stays within 64 KB up to cap 80 at D = 100
constexpr int kAllMax = 80;
hipError_t launch_lle_all(int Q, int D, int cap, double lam, const float* qfeat, const float* xf, int32_t* cand,
                          const int32_t* ncand, float* w, hipStream_t st);
// dictionary-construction tools (k_tools.hip)
int64_t crop_scratch_bytes(int n_img, int H, int W);
hipError_t launch_sample_crops(const float* imgs, int n_img, int H, int W, const uint64_t* draws, int m, int side,
                               int32_t* corners, float* crops, void* scratch, hipStream_t st);
hipError_t launch_knn_rank(int Q, int D, int K, int cap, bool l1, const float* qfeat, const float* xf,
                           const int32_t* cand, const int32_t* ncand, int32_t* ids, float* d, int32_t* m,
                           hipStream_t st);
constexpr int kRankMaxCand = 256;   // candidates a patch the re-rank kernels take
// l1 screen of a dictionary (D = 100): one 128-byte row per entry, the codes
// u_i (one byte each) of x_i on the row's own grid lo + step u, then lo, step
// and eps >= sum_i |x_i - fmaf(step, u_i, lo)| as fp32 at byte kL1sTail
constexpr int kL1sBytes = 128;
constexpr int kL1sDim = 100;
constexpr int kL1sTail = kL1sDim;
hipError_t launch_l1_screen_rows(const float* xf, int64_t n, uint8_t* l1s, hipStream_t st);
// out[i] = min(in[i], cap), i < n
hipError_t launch_min_i32(int n, const int32_t* in, int cap, int32_t* out, hipStream_t st);
// K nearest under l1 of each patch's candidates (D = 100, cap <= 256), the
// screen pruning those whose lower bound exceeds the K-th smallest upper
// bound; outputs as launch_knn_rank's, and (ns non-null) ns[Q] the
// candidates that reached the exact pass
hipError_t launch_knn_l1_screened(int Q, int K, int cap, const float* qfeat, const float* xf, const uint8_t* l1s,
                                  const int32_t* cand, const int32_t* ncand, int32_t* ids, float* d, int32_t* m,
                                  int32_t* ns, hipStream_t st);
// K nearest (squared l2, sequential FP64) of each patch's t-of-L candidates,
// any number of them; counts[Q] the t-of-L counts
hipError_t launch_knn_tofl(int Q, int L, int64_t N, int t, int D, int K, const uint2* bins, const uint32_t* tids,
                           const float* qfeat, const float* xf, int32_t* counts, int32_t* ids, float* d, int32_t* m,
                           hipStream_t st);
hipError_t launch_cand_t(int Q, int L, int64_t N, int t, const uint2* bins, const uint32_t* tids, int cap,
                         int32_t* counts, int32_t* ids, hipStream_t st);
int64_t entropy_scratch_bytes(int L, uint64_t cap);
hipError_t launch_table_entropy(const Slot* dir, int L, uint64_t cap, int64_t n, void* scratch, double* out,
                                hipStream_t st);
// Synthesis fused with the blend (k_lle.hip): tiles of `rows` (4 or 8) patch
// rows x sb_cols(s) patch columns; `part` holds sb_part_floats(s, rows)
// floats for each of the sb_tiles(s, rows, h, w) tiles. which: 1 the tiles,
// 2 the combine into hr, 3 both. m[q] counts the rows of ids/w used for
// patch q (0: the patch is left out of the blend).
__host__ __device__ constexpr int sb_cols(int s) { return s <= 2 ? 40 : 16; }
constexpr int kSbRows = 8;   // tile height of the single-image call
int64_t sb_tiles(int s, int rows, int h, int w);
int64_t sb_part_floats(int s, int rows);
hipError_t launch_synth_blend(int scale, int rows, int K, int h, int w, const int32_t* ids, const int32_t* m,
                              const float* wt, const double* mu, const float* resid, float* part, const float* lr,
                              float* hr, hipStream_t st, int which = 3);

// ---- back-projection (k_bp.hip) ---------------------------------------------
hipError_t launch_bp_update(const float* I, const float* e, int H, int W, int h, int w,
                            int scale, float sigma_s, float sigma_r, float* out,
                            hipStream_t st);
// F, S and a = I - box mean of one iteration into FSa = [F | S | a] (HR each)
hipError_t launch_bp_terms(const float* I, const float* e, int H, int W, int h, int w, int scale,
                           float sigma_s, float sigma_r, float* FSa, hipStream_t st);

// ---- batched form: many LR images of one zoom factor ---------------------------
// One entry per image. Offsets place each image in the concatenated index
// spaces of the batch: LR pixels (gradient maps use 4x, the LR error 1x),
// patches, HR pixels and back-projection tiles.
struct BatchImage {
    const float* lr;         // [h, w]
    float* out;              // [s h, s w] result
    float* scr;              // [s h, s w] back-projection scratch
    int h, w;
    int64_t lr_off, q_off, hr_off, tile_off;
    int64_t fblk_off;             // first workgroup of the image's feature segments
    int64_t sbt_off;              // first tile of the image's fused synthesis and blend
    int64_t dtile_off;            // first tile of the image's LR error (back-projection)
};
// feature segments (64 patches of a patch row) of an h x w LR image
constexpr int kFeatSeg = 64;
__host__ __device__ inline int64_t feature_segments(int h, int w) {
    return h >= kPatch && w >= kPatch ? (int64_t)(h - kPatch + 1) * ((w - kPatch + 1 + kFeatSeg - 1) / kFeatSeg) : 0;
}
// image of a concatenated index: the last entry whose offset field is <= i
template <int64_t BatchImage::*F>
__device__ __forceinline__ int batch_image_of(const BatchImage* im, int n, int64_t i) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (im[mid].*F <= i) lo = mid; else hi = mid;
    }
    return lo;
}
hipError_t launch_b_gradient_maps(const BatchImage* im, int n, int64_t lr_total, float* maps, hipStream_t st);
// one workgroup per feature segment (64 patches of a patch row) of every image
hipError_t launch_b_query_features(const BatchImage* im, int n, int64_t seg_total, int mode, const float* maps,
                                   float* feat, double* mu, hipStream_t st);
// LR error of every image: `tiles` LR tiles in all (degrade_tiles per image)
hipError_t launch_b_degrade_residual(const BatchImage* im, int n, int64_t lr_total, int64_t tiles, int scale,
                                     const Taps& t, int parity, float* e, hipStream_t st);
int64_t degrade_tiles(int h, int w);
// fused synthesis and blend of every image: `tiles` tiles of `rows` patch
// rows (offsets sbt_off), then the combine over the hr_total HR pixels
hipError_t launch_b_synth_blend(const BatchImage* im, int n, int64_t tiles, int64_t hr_total, int scale, int rows,
                                int K, const int32_t* ids, const int32_t* m, const float* wt, const double* mu,
                                const float* resid, float* part, hipStream_t st);
// one back-projection update over all tiles of the batch, persistent: `grid`
// workgroups take tiles from the counter (zeroed here by a fill kernel);
// parity 0 reads out and writes scr, parity 1 the reverse
hipError_t launch_b_bp_update(const BatchImage* im, int n, int64_t n_tiles, int tile, int grid, int scale,
                              float sigma_s, float sigma_r, const float* e, int parity, unsigned int* counter,
                              hipStream_t st);
hipError_t launch_b_copy_scr(const BatchImage* im, int n, int64_t hr_total, int scale, hipStream_t st);
int bp_tiles(int H, int W, int tile);

// ---- adjoint (k_backward.hip) -------------------------------------------------
constexpr int kMaxAdjR = 8;
enum { kAdjGauss = 0, kAdjBox = 1, kAdjUp = 2, kAdjDec = 3 };
struct AxisAdjArgs {
    const float* in;
    const float* mul;        // optional elementwise factor of the input (same layout), nullable
    float* out;
    int rows;                // rows (x pass) or columns (y pass) of the other axis
    int n_in, n_out;         // length of the axis in and out
    int s;                   // zoom factor (bicubic and degradation)
    int R;                   // tap radius (Gaussian, box, blur)
    float taps[2 * kMaxAdjR + 1];   // Gaussian taps (unnormalised) or blur taps
};
// one pass of a transposed separable operator along x (axis 0) or y (axis 1)
hipError_t launch_axis_adj(int op, int axis, const AxisAdjArgs& a, hipStream_t st);
hipError_t launch_bp_adj_z(const float* FSa, const float* g, int64_t n, float sigma_r, float* z, hipStream_t st);
hipError_t launch_bp_adj_combine(float* g, const float* v, const float* z, const float* bz, int64_t n,
                                 hipStream_t st);
hipError_t launch_blend_adj(const float* g, const int32_t* m, int h, int w, int s, float* gp, hipStream_t st);
struct BackwardArgs {
    int Q, D, K, s, w;       // patches, feature dimension, neighbours, zoom, LR width
    int hs;                  // row stride of the high plane
    const float* qfeat;
    const int32_t* ids;
    const int32_t* m;
    const uint16_t* hi;
    const uint16_t* lo;
    const float* resid;      // [N, (5s)^2]
    const float* gp;         // [s h, s w] gradient per covered pixel / its count
    double lam;
    double* c_lam;           // [Q] per-patch contribution to dL/dlambda
};
hipError_t launch_lle_lambda_adj(const BackwardArgs& a, hipStream_t st);
// K <= 8: the same contributions from the packed FP64 Gram matrices [Q, 36];
// gw is scratch [Q, 8] doubles
hipError_t launch_lam_adj8(const BackwardArgs& a, const double* gram, double* gw, hipStream_t st);
hipError_t launch_sum_f64(const double* x, int64_t n, float* out, hipStream_t st);
hipError_t launch_nbr_pairs(const int32_t* ids, const int32_t* m, int Q, int K, uint32_t none, uint32_t* key,
                            uint32_t* val, hipStream_t st);
// part: scratch of 2 (5s)^2 floats per chunk of 64 entries; info: 8 bytes per chunk
hipError_t launch_dict_grad(const uint32_t* key, const uint32_t* val, int64_t n_ent, uint32_t none, const float* wts,
                            const float* gp, int w, int s, int K, float* g_r, float* part, void* info,
                            hipStream_t st);

}  // namespace zh
