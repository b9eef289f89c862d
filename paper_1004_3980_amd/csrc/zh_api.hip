// C-ABI of libzoomhash: context, argument and state checks, device buffer
// management, hash-parameter generation and the orchestration of the
// kernels of the zoom path. Compiled without multiply-add contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zoomhash.h"
#include "zh_internal.h"

using namespace zh;

// Scratch of zh_hash_noalloc: a fixed device array of the library, one copy
// per GPU, held until the process ends (its size is kNoAllocBytes).
static __device__ __align__(256) unsigned char scratch[(size_t)8 << 20];

namespace {

// ---- device buffers ---------------------------------------------------------
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Dict {
    bool valid = false;
    int scale = 0, D = 0, mode = 0;
    int64_t n = 0;
    int L = 0, k = 0;
    float w = 0.f;
    uint64_t seed = 0;
    uint64_t cap = 0;             // directory slots per table
    const float* resid = nullptr; // borrowed
    Buf hi, lo;                   // [n, hi_stride(D)] and [n, D] split planes (64 bytes of slack at the end)
    Buf alpha, beta, bc0[2], ahi, alo;   // ahi, alo: bf16 split of fl(alpha / w)
    Buf bw;                       // [L k] fl(beta / w)
    float bc1[2] = {0.f, 0.f}, bc2[2] = {0.f, 0.f};
    Buf dir;                      // [L, cap] Slot
    Buf dfilt;                    // [L, dir_filter_words(cap)] presence bits of the keys
    Buf tids;                     // [L, n] uint32
    Buf kmul;                     // [L, k] multipliers of the bucket-key sum
    Buf sc;                       // [n, kScreenBytes] screen plane
    Buf xf;                       // [n, D] fp32 copy of the features (exact passes of the search)
    Buf phi_hi, phi_lo;           // [64, round32(D)] bf16 split of the principal directions
    float inv_s2 = 0.f;           // lower bound of 1 / sigma_max(Phi)^2
    float rot_c1 = 0.f;           // error-bound coefficient of the query rotation
    std::vector<float> h_alpha, h_beta;
    uint64_t feat_hash = 0;       // content hash of the features the tables were built on
    Buf l1s;                      // [n, kL1sBytes] l1 screen rows (D = 100), formed at the first zh_knn_l1
    bool l1s_ok = false;          // l1s holds the rows of the current features
};


// ---- fixed scratch of the allocation-free entry point (zh_hash_noalloc) ------
// Host code never uses the array's name `scratch` as an address: each
// device's address is taken once, with that device current, by
// hipGetSymbolAddress (at zh_create) and kept in g_noalloc_ptr.
constexpr size_t kNoAllocBytes = sizeof(scratch);
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocDevices] = {};

}  // namespace

struct zh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    size_t mem_limit = 0, mem_used = 0;
    // bumped whenever a device buffer of the context is allocated, freed or a
    // dictionary is rebuilt: a captured batch graph holds the addresses and
    // the dictionary parameters of the time it was captured
    uint64_t gen = 0;
    Dict dicts[kMaxScale + 1];    // scale 1 .. kMaxScale (index = scale)
    zh_query_opts opts{0, 0, 1, 1};
    int metric = ZH_METRIC_L2;    // distance of zh_query's neighbour ranking
    // last query
    int stage = 0;                // 0 none, 1 queried, 2 weighted, 3 reconstructed
    int qh = 0, qw = 0, qscale = 0, qK = 0;
    bool all_m = false;           // the last weights are over all matches (zh_lle_all)
    int all_cap = 0;              // ... with lists of this many entries a patch
    bool gram_ready = false;      // gram holds the Gram matrices of the last search's neighbours
    int gram_fp64 = 0;            // ... in FP64 (else fp32)
    double lam = 0.0;             // lambda of the last zh_lle_weights
    int sb_rows = kSbRows;        // patch rows per tile of the fused synthesis and blend (4 or 8)
    // batched form: plan of the last batch, its captured graph, tuning
    struct BatchGroup {
        int n = 0;
        int64_t q_total = 0, lr_total = 0, hr_total = 0, tiles = 0;
        int64_t fsegs = 0;              // feature segments of all images
        int64_t sbtiles = 0;            // tiles of the fused synthesis and blend of all images
        int64_t dtiles = 0;             // LR-error tiles of all images
        Buf table;                // device BatchImage[n]
    };
    struct Batch {
        std::vector<uint64_t> sig;
        BatchGroup g[kMaxScale + 1];   // by zoom factor
        hipGraphExec_t exec = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t ev_in = nullptr, ev_out = nullptr;
        int tile = 32, grid_per_cu = 4;
        Buf scr, e, counter;
    } batch;
    // back-projection record for zh_backward: 0 none, 1 one call kept, -1 more than one
    int bp_rec = 0, bp_iters = 0;
    float bp_sigma_s = 0.f, bp_sigma_r = 0.f;
    int64_t Q = 0;
    Buf lr, maps, qfeat, qmu, qkeys, qbins, ids, d2, m, ncand, w, over, sbpart, e, tmp, counters, gram, hmask, fixl, fixc, nsurv, guides, bwd, bwd_k, clam;
    Buf qrot;                     // [Q, 64] rotated queries of the screen
    Buf chk;                      // flag of the training-position check
    Buf bwd_gw;                   // [Q, 8] FP64 scratch of the lambda adjoint
    Buf bwd_part;                 // partial row gradients of the dictionary-gradient passes
    Buf tools;                    // scratch of the training-crop sampler and the entropy diagnostic
    Buf l1cand;                   // [Q, cap] candidate lists of the l1 re-rank and of zh_lle_all
    Buf wall;                     // [Q, cap] weights over all matches (zh_lle_all)
    Buf rs_k1, rs_v1, rs_hist, slot_of, idsort, keys_dict;
    // stage timing
    bool timing = false;
    uint32_t timing_mask = ~0u;   // stages bracketed with events while timing is on
    static constexpr int kEv = 256;
    hipEvent_t ev[ZH_T_COUNT][kEv][2] = {};
    int nev[ZH_T_COUNT] = {0};
};

namespace {

zh_status fail(zh_ctx* c, zh_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIPCHK(c, expr)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail((c), ZH_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

zh_status ensure(zh_ctx* c, Buf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return ZH_OK;
    ++c->gen;
    if (b.p) {
        hipFree(b.p);
        c->mem_used -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    if (c->mem_limit && c->mem_used + bytes > c->mem_limit)
        return fail(c, ZH_ENOMEM, "allocation of %zu bytes exceeds ZH_MEM_LIMIT", bytes);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, ZH_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    c->mem_used += bytes;
    return ZH_OK;
}

void release(zh_ctx* c, Buf& b) {
    if (b.p) {
        hipFree(b.p);
        c->mem_used -= b.bytes;
        ++c->gen;
    }
    b.p = nullptr;
    b.bytes = 0;
}

#define TRY(expr)                      \
    do {                               \
        zh_status s_ = (expr);         \
        if (s_ != ZH_OK) return s_;    \
    } while (0)

template <typename T>
T* P(Buf& b) { return static_cast<T*>(b.p); }

// Brackets one stage's launches with a pair of events when timing is on.
struct StageTimer {
    zh_ctx* c;
    int stage;
    int slot = -1;
    StageTimer(zh_ctx* c_, int s) : c(c_), stage(s) {
        if (!c->timing || !((c->timing_mask >> stage) & 1u) || c->nev[stage] >= zh_ctx::kEv) return;
        slot = c->nev[stage]++;
        hipEvent_t* e = c->ev[stage][slot];
        if (!e[0]) {
            if (hipEventCreate(&e[0]) != hipSuccess || hipEventCreate(&e[1]) != hipSuccess) {
                (void)hipGetLastError();
                slot = -1;
                --c->nev[stage];
                return;
            }
        }
        (void)hipEventRecord(e[0], c->stream);
    }
    ~StageTimer() {
        if (slot >= 0) (void)hipEventRecord(c->ev[stage][slot][1], c->stream);
    }
};

// ---- hash parameters: SplitMix64 + Marsaglia polar normals -------------------
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        s += kGolden;
        return fmix64(s);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    double normal() {
        for (;;) {
            const double u1 = 2.0 * uniform() - 1.0;
            const double u2 = 2.0 * uniform() - 1.0;
            const double s2 = u1 * u1 + u2 * u2;
            if (s2 > 0.0 && s2 < 1.0) return u1 * std::sqrt(-2.0 * std::log(s2) / s2);
        }
    }
};

void hash_params(uint64_t seed, int L, int k, int D, double w, std::vector<float>& alpha,
                 std::vector<float>& beta) {
    alpha.assign((size_t)L * k * D, 0.f);
    beta.assign((size_t)L * k, 0.f);
    const double eps = 1e-3;
    for (int l = 0; l < L; ++l) {
        SplitMix g{fmix64(seed + kGolden * (uint64_t)(l + 1))};
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < D; ++i) {
                const double a = g.normal();
                double b = g.normal();
                while (std::fabs(b) < eps) b = g.normal();
                alpha[((size_t)l * k + j) * D + i] = (float)(a / b);
            }
        for (int j = 0; j < k; ++j) beta[(size_t)l * k + j] = (float)(g.uniform() * w);
    }
}

uint16_t bf16_rne_host(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float bf16_f_host(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

Taps gauss_taps(double sigma) {
    Taps t{};
    t.R = (int)std::ceil(3.0 * sigma);
    std::vector<double> e(2 * t.R + 1);
    double s = 0.0;
    for (int d = -t.R; d <= t.R; ++d) {
        e[d + t.R] = std::exp(-(double)(d * d) / (2.0 * sigma * sigma));
    }
    for (double x : e) s = s + x;
    for (int i = 0; i < 2 * t.R + 1; ++i) t.g[i] = e[i] / s;
    return t;
}

// fl(beta / w) of the host copy of beta, to the device (synchronous)
zh_status upload_beta_w(zh_ctx* c, Dict& d) {
    std::vector<float> bw(d.h_beta.size());
    for (size_t j = 0; j < bw.size(); ++j) bw[j] = d.h_beta[j] / d.w;
    TRY(ensure(c, d.bw, sizeof(float) * std::max<size_t>(bw.size(), 1)));
    HIPCHK(c, hipMemcpyAsync(d.bw.p, bw.data(), sizeof(float) * bw.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ZH_OK;
}

void set_bounds(HashArgs& ha, Dict& d, int prec) {
    ha.bound_c0 = P<float>(d.bc0[prec]);
    ha.bound_c1 = d.bc1[prec];
    ha.bound_c2 = d.bc2[prec];
    ha.inv_w = 1.0f / d.w;
    ha.beta_w = P<float>(d.bw);
}

zh_status set_device(zh_ctx* c) {
    HIPCHK(c, hipSetDevice(c->device));
    return ZH_OK;
}

int dim_of(int mode) { return mode == ZH_FEAT_MEANREM ? 25 : 100; }

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

zh_status clear_counters(zh_ctx* c) {
    TRY(ensure(c, c->counters, kNumCounters * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c->stream, P<uint32_t>(c->counters), kNumCounters, 0u);
    HIPCHK(c, hipGetLastError());
    return ZH_OK;
}

// Scratch of the hash kernels: the per-row dirty mask, and a fix list of
// kFixSlots entries for each wave of 16 rows (384 tables at L = 24; on
// average about 1% of the tables need a fix) with its entry counts.
zh_status hash_scratch(zh_ctx* c, HashArgs& ha) {
    TRY(ensure(c, c->hmask, sizeof(uint64_t) * (size_t)(ha.n > 0 ? ha.n : 1)));
    ha.dirty = P<uint64_t>(c->hmask);
    int cap = kFixSlots;
    if (const char* ev = std::getenv("ZH_HASH_FIX_CAP")) cap = std::min(kFixSlots, std::max(0, std::atoi(ev)));
    const size_t nw = (size_t)((ha.n + 15) / 16);
    TRY(ensure(c, c->fixl, sizeof(int32_t) * nw * cap * (size_t)(((ha.k + 2) + 3) & ~3)));
    TRY(ensure(c, c->fixc, sizeof(uint32_t) * (nw > 0 ? nw : 1)));
    ha.fix_list = P<int32_t>(c->fixl);
    ha.fix_cap = cap;
    ha.fix_count = P<unsigned int>(c->fixc);
    return ZH_OK;
}

// Screen plane of a dictionary: FP64 covariance of up to 65536 evenly spaced
// rows, its leading eigenvectors as Phi (host), the bf16 split of Phi for the
// query rotation and the screen row of every entry.
zh_status build_screen(zh_ctx* c, Dict& d, const float* feat) {
    const int D = d.D, m = screen_dims(D);
    const int64_t n = d.n;
    const int64_t ns = std::min<int64_t>(n, 65536);
    Buf part, cov, phit;
    zh_status st = ZH_OK;
    std::vector<double> C((size_t)D * D), phiT((size_t)D * kRotStride, 0.0);
    std::vector<float> phi((size_t)m * D);
    const int DP = (D + 31) & ~31;
    std::vector<uint16_t> ph((size_t)kRotStride * DP, 0), pl((size_t)kRotStride * DP, 0);
    double s2 = 0.0;
    if ((st = ensure(c, part, sizeof(double) * 128 * (size_t)D * D)) != ZH_OK) goto out;
    if ((st = ensure(c, cov, sizeof(double) * (size_t)D * D)) != ZH_OK) goto out;
    if ((st = ensure(c, phit, sizeof(double) * (size_t)D * kRotStride)) != ZH_OK) goto out;
    if (launch_cov(feat, n, D, ns, P<double>(part), P<double>(cov), c->stream) != hipSuccess ||
        hipMemcpyAsync(C.data(), cov.p, sizeof(double) * (size_t)D * D, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(c, ZH_EDEVICE, "zh_build_tables: covariance of the screen failed");
        goto out;
    }
    s2 = screen_basis(C.data(), D, m, phi.data());
    {
        const double v = (1.0 / s2) * (1.0 - 1e-9);
        float f = (float)v;
        if ((double)f > v) f = std::nextafter(f, 0.0f);
        d.inv_s2 = f;
    }
    d.rot_c1 = rotate_bound_coeff(D);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < D; ++i) {
            const float v = phi[(size_t)j * D + i];
            phiT[(size_t)i * kRotStride + j] = (double)v;
            const uint16_t h = bf16_rne_host(v);
            ph[(size_t)j * DP + i] = h;
            pl[(size_t)j * DP + i] = bf16_rne_host(v - bf16_f_host(h));
        }
    if ((st = ensure(c, d.sc, (size_t)kScreenBytes * (size_t)n)) != ZH_OK) goto out;
    if ((st = ensure(c, d.phi_hi, sizeof(uint16_t) * ph.size())) != ZH_OK) goto out;
    if ((st = ensure(c, d.phi_lo, sizeof(uint16_t) * pl.size())) != ZH_OK) goto out;
    if (hipMemcpyAsync(phit.p, phiT.data(), sizeof(double) * phiT.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(d.phi_hi.p, ph.data(), sizeof(uint16_t) * ph.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(d.phi_lo.p, pl.data(), sizeof(uint16_t) * pl.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        launch_screen_rows(feat, n, D, m, P<double>(phit), P<uint8_t>(d.sc), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(c, ZH_EDEVICE, "zh_build_tables: screen rows failed");
        goto out;
    }
out:
    release(c, part);
    release(c, cov);
    release(c, phit);
    return st;
}

// Content hash of `bytes` bytes of device memory (a multiple of 4), salted by the section.
zh_status device_hash(zh_ctx* c, const void* p, uint64_t bytes, uint64_t salt, uint64_t* out) {
    TRY(ensure(c, c->chk, 16));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c->stream, P<uint32_t>(c->chk), 4, 0u);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, launch_hash_words(p, (int64_t)(bytes / 4), salt, P<unsigned long long>(c->chk), c->stream));
    HIPCHK(c, hipMemcpyAsync(out, c->chk.p, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ZH_OK;
}

// The library's own copies of the dictionary features: the split bf16/low
// planes and the fp32 rows of the exact passes.
zh_status store_features(zh_ctx* c, Dict& d, const float* feat) {
    const int64_t n = d.n;
    const int D = d.D;
    TRY(ensure(c, d.hi, sizeof(uint16_t) * (size_t)n * hi_stride(D) + 64));
    TRY(ensure(c, d.lo, sizeof(uint16_t) * (size_t)n * D + 64));
    HIPCHK(c, hipMemsetAsync(d.hi.p, 0, d.hi.bytes, c->stream));
    HIPCHK(c, hipMemsetAsync(d.lo.p, 0, d.lo.bytes, c->stream));
    HIPCHK(c, launch_split_planes(feat, n, D, P<uint16_t>(d.hi), P<uint16_t>(d.lo), c->stream));
    TRY(ensure(c, d.xf, sizeof(float) * (size_t)n * D + 64));
    HIPCHK(c, hipMemcpyAsync(d.xf.p, feat, sizeof(float) * (size_t)n * D, hipMemcpyDeviceToDevice, c->stream));
    return ZH_OK;
}

// cand_only (early stop): the candidate counts and the dump only; the
// neighbour outputs and the Gram matrices of the last search stay as they are
zh_status run_search(zh_ctx* c, Dict& d, int32_t* dump, int dump_cap, bool cand_only = false) {
    SearchArgs a{};
    a.Q = (int)c->Q;
    a.D = d.D;
    a.L = d.L;
    a.K = c->qK;
    a.cap = c->opts.cap;
    a.rerank = c->opts.rerank;
    a.exact = c->opts.rerank == 0 ? 1 : 0;
    a.bins = P<uint2>(c->qbins);
    a.qfeat = P<float>(c->qfeat);
    a.tids = P<uint32_t>(d.tids);
    a.N = d.n;
    a.hi = P<uint16_t>(d.hi);
    a.lo = P<uint16_t>(d.lo);
    a.hs = hi_stride(d.D);
    a.ce = screen_coeff();
    a.sc = P<uint8_t>(d.sc);
    a.xf = P<float>(d.xf);
    a.inv_s2 = d.inv_s2;
    a.out_ids = P<int32_t>(c->ids);
    a.out_d2 = P<float>(c->d2);
    a.out_m = P<int32_t>(c->m);
    a.out_ncand = P<int32_t>(c->ncand);
    a.cand_only = cand_only && a.cap > 0 ? 1 : 0;
    if (a.cap > 0 && !a.cand_only) {
        TRY(ensure(c, c->nsurv, sizeof(int32_t) * (size_t)(a.Q > 0 ? a.Q : 1)));
        a.out_nsurv = P<int32_t>(c->nsurv);
        TRY(ensure(c, c->qrot, sizeof(float) * kRotStride * (size_t)(a.Q > 0 ? a.Q : 1)));
        a.qrot = P<float>(c->qrot);
        if (a.K <= 8) {
            // the search forms the Gram matrices of the neighbours as well
            a.gram_fp64 = c->opts.lle_fp64;
            TRY(ensure(c, c->gram, (a.gram_fp64 ? 8 : 4) * (size_t)(a.Q > 0 ? a.Q : 1) * 36));
            a.gram = c->gram.p;
        }
        StageTimer t(c, ZH_T_ROTATE);
        HIPCHK(c, launch_rotate(a.qfeat, a.Q, d.D, P<uint16_t>(d.phi_hi), P<uint16_t>(d.phi_lo), d.rot_c1,
                                P<float>(c->qrot), c->stream));
    }
    a.dump = dump;
    a.dump_cap = dump_cap;
    a.overflow = P<int32_t>(c->over);
    a.counters = P<unsigned int>(c->counters);
    if (a.cand_only) {
        StageTimer t(c, ZH_T_SEARCH);
        HIPCHK(c, launch_search(a, c->stream));
        return ZH_OK;
    }
    c->gram_ready = false;
    {
        StageTimer t(c, ZH_T_SEARCH);
        HIPCHK(c, launch_search(a, c->stream));
        if (a.cap == 0) HIPCHK(c, launch_search_overflow(a, 1024, c->stream));
    }
    c->gram_ready = a.gram != nullptr;
    c->gram_fp64 = a.gram_fp64;
    return ZH_OK;
}

}  // namespace

extern "C" {

zh_status zh_create(zh_ctx** out, int device, void* hip_stream) {
    if (!out) return ZH_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return ZH_EDEVICE;
    }
    if (device < 0 || device >= ndev) return ZH_EINVAL;
    zh_ctx* c = new (std::nothrow) zh_ctx();
    if (!c) return ZH_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (const char* lim = std::getenv("ZH_MEM_LIMIT")) c->mem_limit = (size_t)std::strtoull(lim, nullptr, 10);
    if (hipSetDevice(device) != hipSuccess || lle_init() != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return ZH_EDEVICE;
    }
    if (device < kNoAllocDevices) {
        // the device address of this GPU's copy of the fixed scratch, once per device
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (!g_noalloc_ptr[device]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
                (void)hipGetLastError();
                delete c;
                return ZH_EDEVICE;
            }
            g_noalloc_ptr[device] = ptr;
        }
    }
    *out = c;
    return ZH_OK;
}

void zh_destroy(zh_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (Dict& d : c->dicts) {
        release(c, d.hi); release(c, d.lo); release(c, d.alpha); release(c, d.beta); release(c, d.bc0[0]); release(c, d.bc0[1]);
        release(c, d.ahi); release(c, d.alo); release(c, d.bw); release(c, d.dir); release(c, d.dfilt); release(c, d.tids);
        release(c, d.sc); release(c, d.phi_hi); release(c, d.phi_lo); release(c, d.kmul); release(c, d.xf);
        release(c, d.l1s);
    }
    for (int st = 0; st < ZH_T_COUNT; ++st)
        for (int i = 0; i < zh_ctx::kEv; ++i)
            for (int j = 0; j < 2; ++j)
                if (c->ev[st][i][j]) (void)hipEventDestroy(c->ev[st][i][j]);
    if (c->batch.stream) (void)hipStreamSynchronize(c->batch.stream);
    if (c->batch.exec) (void)hipGraphExecDestroy(c->batch.exec);
    if (c->batch.ev_in) (void)hipEventDestroy(c->batch.ev_in);
    if (c->batch.ev_out) (void)hipEventDestroy(c->batch.ev_out);
    if (c->batch.stream) (void)hipStreamDestroy(c->batch.stream);
    for (auto& g : c->batch.g) release(c, g.table);
    release(c, c->batch.scr);
    release(c, c->batch.e);
    release(c, c->batch.counter);
    Buf* bufs[] = {&c->lr, &c->maps, &c->qfeat, &c->qmu, &c->qkeys, &c->qbins, &c->ids, &c->d2, &c->m,
                   &c->ncand, &c->w, &c->over, &c->sbpart, &c->e, &c->tmp, &c->counters, &c->rs_k1,
                   &c->rs_v1, &c->rs_hist, &c->slot_of, &c->idsort, &c->keys_dict, &c->gram, &c->hmask, &c->fixl, &c->fixc, &c->nsurv, &c->guides, &c->bwd, &c->bwd_k, &c->clam, &c->qrot, &c->bwd_gw, &c->bwd_part, &c->tools, &c->l1cand, &c->chk, &c->wall};
    for (Buf* b : bufs) release(c, *b);
    delete c;
}

zh_status zh_set_stream(zh_ctx* c, void* s) {
    if (!c) return ZH_EINVAL;
    c->stream = (hipStream_t)s;
    return ZH_OK;
}

zh_status zh_sync(zh_ctx* c) {
    if (!c) return ZH_EINVAL;
    TRY(set_device(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ZH_OK;
}

const char* zh_last_error(const zh_ctx* c) { return c ? c->err.c_str() : "null context"; }

zh_status zh_degrade(zh_ctx* c, const float* hr, int n_img, int H, int W, int scale, float sigma, float* lr) {
    if (!c) return ZH_EINVAL;
    if (!hr || !lr || n_img < 1 || H < 1 || W < 1 || scale < 1 || scale > 8 || !(sigma > 0.f) || sigma > 5.f)
        return fail(c, ZH_EINVAL, "zh_degrade: bad arguments");
    TRY(set_device(c));
    HIPCHK(c, launch_degrade(hr, n_img, H, W, scale, gauss_taps(sigma), lr, c->stream));
    return ZH_OK;
}

zh_status zh_make_dictionary(zh_ctx* c, const float* hr, int n_img, int H, int W, const int32_t* pos, int64_t n,
                             int scale, float sigma, int mode, float* feat, float* resid) {
    if (!c) return ZH_EINVAL;
    if (!hr || !pos || !feat || !resid || n_img < 1 || n < 1 || n >= (1ll << 31) || scale < 1 || scale > kMaxScale ||
        (mode != ZH_FEAT_MEANREM && mode != ZH_FEAT_GRAD4) || !(sigma > 0.f) || sigma > 5.f)
        return fail(c, ZH_EINVAL, "zh_make_dictionary: bad arguments");
    const int h = (H + scale - 1) / scale, w = (W + scale - 1) / scale;
    if (H / scale < kPatch || W / scale < kPatch) return fail(c, ZH_EINVAL, "zh_make_dictionary: images too small");
    TRY(set_device(c));
    // every position inside its image, checked on the device before any cut
    TRY(ensure(c, c->chk, 16));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c->stream, P<uint32_t>(c->chk), 4, 0u);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, launch_check_positions(pos, n, n_img, H / scale - kPatch, W / scale - kPatch, P<uint32_t>(c->chk),
                                     c->stream));
    {
        uint32_t bad = 0;
        HIPCHK(c, hipMemcpyAsync(&bad, c->chk.p, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (bad) return fail(c, ZH_EINVAL, "zh_make_dictionary: a position lies outside its image");
    }
    TRY(ensure(c, c->tmp, sizeof(float) * (size_t)n_img * h * w * 5));
    float* lrs = P<float>(c->tmp);
    float* maps = lrs + (size_t)n_img * h * w;
    HIPCHK(c, launch_degrade(hr, n_img, H, W, scale, gauss_taps(sigma), lrs, c->stream));
    HIPCHK(c, launch_gradient_maps(lrs, n_img, h, w, maps, c->stream));
    HIPCHK(c, launch_dict_cut(hr, lrs, maps, H, W, scale, pos, n, mode, feat, resid, c->stream));
    return ZH_OK;
}

zh_status zh_sample_crops(zh_ctx* c, const float* imgs, int n_img, int H, int W, const uint64_t* draws, int m,
                          int side, int32_t* corners, float* crops) {
    if (!c) return ZH_EINVAL;
    if (!imgs || n_img < 1 || n_img > 65535 || H < 1 || W < 1 || (int64_t)H * W >= (1ll << 31) || m < 0 ||
        (m > 0 && (!draws || !corners)) || side < 1 || side > H || side > W ||
        (int64_t)n_img * m >= (1ll << 31))
        return fail(c, ZH_EINVAL, "zh_sample_crops: bad arguments");
    if (m == 0) return ZH_OK;
    TRY(set_device(c));
    TRY(ensure(c, c->tools, (size_t)crop_scratch_bytes(n_img, H, W)));
    HIPCHK(c, launch_sample_crops(imgs, n_img, H, W, draws, m, side, corners, crops, c->tools.p, c->stream));
    return ZH_OK;
}

zh_status zh_table_entropy(zh_ctx* c, int scale, double* entropy, int capacity) {
    if (!c) return ZH_EINVAL;
    if (scale < 1 || scale > kMaxScale || !c->dicts[scale].valid)
        return fail(c, ZH_ESTATE, "zh_table_entropy: no tables for scale %d", scale);
    Dict& d = c->dicts[scale];
    if (!entropy || capacity < d.L) return fail(c, ZH_EINVAL, "zh_table_entropy: room for %d tables needed", d.L);
    TRY(set_device(c));
    TRY(ensure(c, c->tools, (size_t)entropy_scratch_bytes(d.L, d.cap)));
    double* out = reinterpret_cast<double*>(static_cast<char*>(c->tools.p) + entropy_scratch_bytes(d.L, d.cap)) - d.L;
    HIPCHK(c, launch_table_entropy(P<Slot>(d.dir), d.L, d.cap, d.n, c->tools.p, out, c->stream));
    HIPCHK(c, hipMemcpyAsync(entropy, out, sizeof(double) * d.L, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ZH_OK;
}

zh_status zh_features(zh_ctx* c, const float* lr, int h, int w, int mode, float* feat, double* mu) {
    if (!c) return ZH_EINVAL;
    if (!lr || !feat || h < kPatch || w < kPatch || (mode != ZH_FEAT_MEANREM && mode != ZH_FEAT_GRAD4))
        return fail(c, ZH_EINVAL, "zh_features: bad arguments");
    TRY(set_device(c));
    const int64_t Q = (int64_t)(h - 4) * (w - 4);
    TRY(ensure(c, c->maps, sizeof(float) * 4 * (size_t)h * w));
    double* mup = mu;
    if (!mup) {
        TRY(ensure(c, c->qmu, sizeof(double) * (size_t)Q));
        mup = P<double>(c->qmu);
    }
    if (mode == ZH_FEAT_GRAD4) HIPCHK(c, launch_gradient_maps(lr, 1, h, w, P<float>(c->maps), c->stream));
    HIPCHK(c, launch_query_features(lr, P<float>(c->maps), h, w, mode, feat, mup, c->stream));
    return ZH_OK;
}

zh_status zh_build_tables(zh_ctx* c, const zh_dictionary* dict, int L, int k, float w, uint64_t seed) {
    if (!c) return ZH_EINVAL;
    if (!dict || !dict->feat || !dict->resid || dict->n < 1 || dict->n >= (1ll << 31) ||
        (dict->scale < 1 || dict->scale > kMaxScale) ||
        (dict->feat_mode != ZH_FEAT_MEANREM && dict->feat_mode != ZH_FEAT_GRAD4) ||
        dict->dim != dim_of(dict->feat_mode))
        return fail(c, ZH_EINVAL, "zh_build_tables: bad dictionary");
    if (L < 1 || L > kMaxL || k < 1 || k > kMaxKHash || !(w > 0.f) || !std::isfinite(w))
        return fail(c, ZH_EINVAL, "zh_build_tables: need 1 <= L <= %d, 1 <= k <= %d, w > 0", kMaxL, kMaxKHash);
    TRY(set_device(c));
    Dict& d = c->dicts[dict->scale];
    d.valid = false;
    d.l1s_ok = false;
    c->stage = 0;
    ++c->gen;   // the tables and parameters a captured batch graph baked in change
    const int64_t n = dict->n;
    const int D = dict->dim;
    d.scale = dict->scale;
    d.D = D;
    d.mode = dict->feat_mode;
    d.n = n;
    d.L = L;
    d.k = k;
    d.w = w;
    d.seed = seed;
    d.resid = dict->resid;
    uint64_t cap = 1;
    while (cap < 2 * (uint64_t)n) cap <<= 1;
    d.cap = cap;
    TRY(store_features(c, d, dict->feat));
    TRY(device_hash(c, dict->feat, sizeof(float) * (uint64_t)n * D, 0, &d.feat_hash));
    TRY(build_screen(c, d, dict->feat));
    // hash parameters
    hash_params(seed, L, k, D, (double)w, d.h_alpha, d.h_beta);
    const int m = L * k;
    const int DP = (D + 31) & ~31;
    std::vector<uint16_t> ahi((size_t)m * DP, 0), alo((size_t)m * DP, 0);
    for (int j = 0; j < m; ++j) {
        for (int i = 0; i < D; ++i) {
            const float a = d.h_alpha[(size_t)j * D + i] / w;
            const uint16_t h = bf16_rne_host(a);
            ahi[(size_t)j * DP + i] = h;
            alo[(size_t)j * DP + i] = bf16_rne_host(a - bf16_f_host(h));
        }
    }
    std::vector<float> bc0[2] = {std::vector<float>(m), std::vector<float>(m)};
    for (int pr = 0; pr < 2; ++pr)
        hash_bound_coeffs(pr, D, (double)w, d.h_beta.data(), m, bc0[pr].data(), &d.bc1[pr], &d.bc2[pr]);
    {
        std::vector<uint64_t> km((size_t)L * (k + 1));
        for (int l = 0; l < L; ++l) {
            for (int j = 0; j < k; ++j) km[(size_t)l * (k + 1) + j] = key_mul(l, j);
            km[(size_t)l * (k + 1) + k] = key_mul(l, 63);
        }
        TRY(ensure(c, d.kmul, sizeof(uint64_t) * km.size()));
        HIPCHK(c, hipMemcpyAsync(d.kmul.p, km.data(), sizeof(uint64_t) * km.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    TRY(ensure(c, d.alpha, sizeof(float) * (size_t)m * D));
    TRY(ensure(c, d.beta, sizeof(float) * (size_t)m));
    TRY(ensure(c, d.bc0[0], sizeof(float) * (size_t)m));
    TRY(ensure(c, d.bc0[1], sizeof(float) * (size_t)m));
    TRY(ensure(c, d.ahi, sizeof(uint16_t) * (size_t)m * DP));
    TRY(ensure(c, d.alo, sizeof(uint16_t) * (size_t)m * DP));
    HIPCHK(c, hipMemcpyAsync(d.alpha.p, d.h_alpha.data(), sizeof(float) * (size_t)m * D, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.beta.p, d.h_beta.data(), sizeof(float) * (size_t)m, hipMemcpyHostToDevice, c->stream));
    TRY(upload_beta_w(c, d));
    for (int pr = 0; pr < 2; ++pr)
        HIPCHK(c, hipMemcpyAsync(d.bc0[pr].p, bc0[pr].data(), sizeof(float) * (size_t)m, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpyAsync(d.ahi.p, ahi.data(), sizeof(uint16_t) * (size_t)m * DP, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.alo.p, alo.data(), sizeof(uint16_t) * (size_t)m * DP, hipMemcpyHostToDevice, c->stream));
    // keys of every pair in every table
    TRY(ensure(c, c->keys_dict, sizeof(uint64_t) * (size_t)n * L));
    TRY(clear_counters(c));
    HashArgs ha{};
    ha.feat = dict->feat;
    ha.n = n;
    ha.D = D;
    ha.L = L;
    ha.k = k;
    ha.alpha = P<float>(d.alpha);
    ha.a_hi = P<uint16_t>(d.ahi);
    ha.a_lo = P<uint16_t>(d.alo);
    ha.beta = P<float>(d.beta);
    ha.key_mul = P<uint64_t>(d.kmul);
    set_bounds(ha, d, c->opts.proj);
    ha.w = w;
    ha.prec = c->opts.proj;
    ha.keys = P<uint64_t>(c->keys_dict);
    ha.codes = nullptr;
    ha.n_fixed = P<unsigned int>(c->counters) + C_CODEFIX;
    TRY(hash_scratch(c, ha));
    HIPCHK(c, launch_hash(ha, c->stream));
    // directory and bins, table by table
    TRY(ensure(c, d.dir, sizeof(Slot) * (size_t)L * cap));
    const uint64_t fw = dir_filter_words(cap);
    TRY(ensure(c, d.dfilt, sizeof(uint32_t) * (size_t)L * fw));
    HIPCHK(c, hipMemsetAsync(d.dfilt.p, 0, sizeof(uint32_t) * (size_t)L * fw, c->stream));
    TRY(ensure(c, d.tids, sizeof(uint32_t) * (size_t)L * n));
    TRY(ensure(c, c->slot_of, sizeof(uint32_t) * (size_t)n));
    TRY(ensure(c, c->idsort, sizeof(uint32_t) * (size_t)n));
    TRY(ensure(c, c->rs_k1, sizeof(uint32_t) * (size_t)n));
    TRY(ensure(c, c->rs_v1, sizeof(uint32_t) * (size_t)n));
    const int64_t hs = radix_hist_size(n);
    TRY(ensure(c, c->rs_hist, sizeof(uint32_t) * (size_t)hs));
    int bits = 0;
    while ((1ull << bits) < cap) ++bits;
    HIPCHK(c, launch_dir_clear(P<Slot>(d.dir), (uint64_t)L * cap, c->stream));
    for (int l = 0; l < L; ++l) {
        Slot* dl = P<Slot>(d.dir) + (size_t)l * cap;
        HIPCHK(c, launch_dir_insert(P<uint64_t>(c->keys_dict), n, L, l, dl, cap,
                                    P<uint32_t>(d.dfilt) + (size_t)l * fw, P<uint32_t>(c->slot_of),
                                    P<uint32_t>(c->idsort), c->stream));
        bool in_first = true;
        HIPCHK(c, radix_sort_pairs(P<uint32_t>(c->slot_of), P<uint32_t>(c->idsort), P<uint32_t>(c->rs_k1),
                                   P<uint32_t>(c->rs_v1), n, bits, P<uint32_t>(c->rs_hist), hs, c->stream, &in_first));
        const uint32_t* sk = in_first ? P<uint32_t>(c->slot_of) : P<uint32_t>(c->rs_k1);
        const uint32_t* sv = in_first ? P<uint32_t>(c->idsort) : P<uint32_t>(c->rs_v1);
        HIPCHK(c, launch_dir_offsets(sk, n, dl, c->stream));
        HIPCHK(c, hipMemcpyAsync(P<uint32_t>(d.tids) + (size_t)l * n, sv, sizeof(uint32_t) * (size_t)n,
                                 hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    release(c, c->keys_dict);
    d.valid = true;
    return ZH_OK;
}

}  // extern "C"

// ---- tables on disk ------------------------------------------------------------
namespace {

constexpr int kTabSections = 13;
constexpr uint32_t kTabVersion = 2;
constexpr size_t kTabStage = (size_t)32 << 20;   // pinned staging buffer of the file I/O

// File header: everything zh_build_tables decided, the size and content hash
// of each section, and a hash of the header itself (every byte before
// header_hash, padding zeroed).
struct TabHeader {
    char magic[8];
    uint32_t version, header_bytes;
    int64_t n;
    int32_t D, scale, mode, L, k, nsec;
    float w, inv_s2, rot_c1, bc1[2], bc2[2];
    uint64_t seed, cap, feat_hash;
    uint64_t sec_bytes[kTabSections], sec_hash[kTabSections];
    uint64_t header_hash;
};

uint64_t fnv64(const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

// The device buffers of a dictionary's tables in file order, with the bytes
// each holds for the parameters in d.
void tab_sections(Dict& d, Buf* (&buf)[kTabSections], uint64_t (&bytes)[kTabSections]) {
    const uint64_t m = (uint64_t)d.L * d.k, DP = (uint64_t)((d.D + 31) & ~31);
    Buf* b[kTabSections] = {&d.alpha, &d.beta, &d.bc0[0], &d.bc0[1], &d.ahi, &d.alo, &d.kmul, &d.dir, &d.dfilt,
                            &d.tids, &d.sc, &d.phi_hi, &d.phi_lo};
    const uint64_t z[kTabSections] = {4 * m * d.D, 4 * m, 4 * m, 4 * m, 2 * m * DP, 2 * m * DP,
                                      8 * (uint64_t)d.L * (d.k + 1), sizeof(Slot) * (uint64_t)d.L * d.cap,
                                      4 * (uint64_t)d.L * dir_filter_words(d.cap), 4 * (uint64_t)d.L * d.n,
                                      (uint64_t)kScreenBytes * d.n, 2 * (uint64_t)kRotStride * DP,
                                      2 * (uint64_t)kRotStride * DP};
    for (int i = 0; i < kTabSections; ++i) {
        buf[i] = b[i];
        bytes[i] = z[i];
    }
}

struct PinnedStage {
    void* p = nullptr;
    ~PinnedStage() {
        if (p) (void)hipHostFree(p);
    }
};

struct File {
    FILE* f = nullptr;
    ~File() {
        if (f) fclose(f);
    }
};

}  // namespace

extern "C" {

zh_status zh_save_tables(zh_ctx* c, int scale, const char* path) {
    if (!c) return ZH_EINVAL;
    if (!path) return fail(c, ZH_EINVAL, "zh_save_tables: null path");
    if (scale < 1 || scale > kMaxScale || !c->dicts[scale].valid)
        return fail(c, ZH_ESTATE, "zh_save_tables: no tables for scale %d", scale);
    TRY(set_device(c));
    Dict& d = c->dicts[scale];
    TabHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, "ZHTABLE", 8);
    h.version = kTabVersion;
    h.header_bytes = sizeof(TabHeader);
    h.n = d.n;
    h.D = d.D;
    h.scale = d.scale;
    h.mode = d.mode;
    h.L = d.L;
    h.k = d.k;
    h.nsec = kTabSections;
    h.w = d.w;
    h.inv_s2 = d.inv_s2;
    h.rot_c1 = d.rot_c1;
    for (int i = 0; i < 2; ++i) {
        h.bc1[i] = d.bc1[i];
        h.bc2[i] = d.bc2[i];
    }
    h.seed = d.seed;
    h.cap = d.cap;
    h.feat_hash = d.feat_hash;
    Buf* buf[kTabSections];
    uint64_t bytes[kTabSections];
    tab_sections(d, buf, bytes);
    for (int i = 0; i < kTabSections; ++i) {
        h.sec_bytes[i] = bytes[i];
        TRY(device_hash(c, buf[i]->p, bytes[i], (uint64_t)i + 1, &h.sec_hash[i]));
    }
    h.header_hash = fnv64(&h, offsetof(TabHeader, header_hash));
    File f;
    f.f = std::fopen(path, "wb");
    if (!f.f) return fail(c, ZH_EIO, "zh_save_tables: cannot open %s for writing", path);
    if (std::fwrite(&h, sizeof(h), 1, f.f) != 1) return fail(c, ZH_EIO, "zh_save_tables: write failed");
    PinnedStage stage;
    HIPCHK(c, hipHostMalloc(&stage.p, kTabStage, hipHostMallocDefault));
    for (int i = 0; i < kTabSections; ++i) {
        for (uint64_t off = 0; off < bytes[i]; off += kTabStage) {
            const size_t len = (size_t)std::min<uint64_t>(kTabStage, bytes[i] - off);
            HIPCHK(c, hipMemcpyAsync(stage.p, static_cast<char*>(buf[i]->p) + off, len, hipMemcpyDeviceToHost,
                                     c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (std::fwrite(stage.p, 1, len, f.f) != len) return fail(c, ZH_EIO, "zh_save_tables: write failed");
        }
    }
    if (std::fclose(f.f) != 0) {
        f.f = nullptr;
        return fail(c, ZH_EIO, "zh_save_tables: close failed");
    }
    f.f = nullptr;
    return ZH_OK;
}

zh_status zh_load_tables(zh_ctx* c, const zh_dictionary* dict, const char* path) {
    if (!c) return ZH_EINVAL;
    if (!path) return fail(c, ZH_EINVAL, "zh_load_tables: null path");
    if (!dict || !dict->feat || !dict->resid || dict->n < 1 || dict->n >= (1ll << 31) ||
        (dict->scale < 1 || dict->scale > kMaxScale) ||
        (dict->feat_mode != ZH_FEAT_MEANREM && dict->feat_mode != ZH_FEAT_GRAD4) ||
        dict->dim != dim_of(dict->feat_mode))
        return fail(c, ZH_EINVAL, "zh_load_tables: bad dictionary");
    TRY(set_device(c));
    File f;
    f.f = std::fopen(path, "rb");
    if (!f.f) return fail(c, ZH_EIO, "zh_load_tables: cannot open %s", path);
    TabHeader h;
    if (std::fread(&h, sizeof(h), 1, f.f) != 1 || std::memcmp(h.magic, "ZHTABLE", 8) != 0 ||
        h.version != kTabVersion || h.header_bytes != sizeof(TabHeader) || h.nsec != kTabSections ||
        h.header_hash != fnv64(&h, offsetof(TabHeader, header_hash)))
        return fail(c, ZH_EIO, "zh_load_tables: %s is not a table file of this version (or its header is damaged)", path);
    if (h.n != dict->n || h.D != dict->dim || h.scale != dict->scale || h.mode != dict->feat_mode)
        return fail(c, ZH_EINVAL, "zh_load_tables: the file holds tables of another dictionary shape");
    if (h.L < 1 || h.L > kMaxL || h.k < 1 || h.k > kMaxKHash || !(h.w > 0.f))
        return fail(c, ZH_EIO, "zh_load_tables: bad parameters in %s", path);
    uint64_t fh = 0;
    TRY(device_hash(c, dict->feat, sizeof(float) * (uint64_t)dict->n * dict->dim, 0, &fh));
    if (fh != h.feat_hash)
        return fail(c, ZH_EINVAL, "zh_load_tables: the dictionary features differ from those the tables were built on");
    Dict& d = c->dicts[dict->scale];
    d.valid = false;
    d.l1s_ok = false;
    c->stage = 0;
    ++c->gen;
    d.scale = h.scale;
    d.D = h.D;
    d.mode = h.mode;
    d.n = h.n;
    d.L = h.L;
    d.k = h.k;
    d.w = h.w;
    d.seed = h.seed;
    d.cap = h.cap;
    d.inv_s2 = h.inv_s2;
    d.rot_c1 = h.rot_c1;
    for (int i = 0; i < 2; ++i) {
        d.bc1[i] = h.bc1[i];
        d.bc2[i] = h.bc2[i];
    }
    d.feat_hash = fh;
    d.resid = dict->resid;
    {
        uint64_t cap = 1;
        while (cap < 2 * (uint64_t)d.n) cap <<= 1;
        if (cap != d.cap) return fail(c, ZH_EIO, "zh_load_tables: directory size in %s does not match", path);
    }
    Buf* buf[kTabSections];
    uint64_t bytes[kTabSections];
    tab_sections(d, buf, bytes);
    for (int i = 0; i < kTabSections; ++i)
        if (bytes[i] != h.sec_bytes[i]) return fail(c, ZH_EIO, "zh_load_tables: section %d of %s has the wrong size", i, path);
    TRY(store_features(c, d, dict->feat));
    PinnedStage stage;
    HIPCHK(c, hipHostMalloc(&stage.p, kTabStage, hipHostMallocDefault));
    for (int i = 0; i < kTabSections; ++i) {
        TRY(ensure(c, *buf[i], bytes[i]));
        for (uint64_t off = 0; off < bytes[i]; off += kTabStage) {
            const size_t len = (size_t)std::min<uint64_t>(kTabStage, bytes[i] - off);
            HIPCHK(c, hipStreamSynchronize(c->stream));   // the stage is free again
            if (std::fread(stage.p, 1, len, f.f) != len) return fail(c, ZH_EIO, "zh_load_tables: %s is truncated", path);
            HIPCHK(c, hipMemcpyAsync(static_cast<char*>(buf[i]->p) + off, stage.p, len, hipMemcpyHostToDevice,
                                     c->stream));
        }
        uint64_t sh = 0;
        TRY(device_hash(c, buf[i]->p, bytes[i], (uint64_t)i + 1, &sh));
        if (sh != h.sec_hash[i]) return fail(c, ZH_EIO, "zh_load_tables: section %d of %s is damaged", i, path);
    }
    // host copies of the hash parameters (zh_get_hash_params)
    const size_t m = (size_t)d.L * d.k;
    d.h_alpha.resize(m * d.D);
    d.h_beta.resize(m);
    HIPCHK(c, hipMemcpyAsync(d.h_alpha.data(), d.alpha.p, sizeof(float) * m * d.D, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.h_beta.data(), d.beta.p, sizeof(float) * m, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TRY(upload_beta_w(c, d));
    d.valid = true;
    return ZH_OK;
}

zh_status zh_get_hash_params(zh_ctx* c, int scale, float* alpha, float* beta) {
    if (!c) return ZH_EINVAL;
    if (scale < 1 || scale > kMaxScale || !c->dicts[scale].valid) return fail(c, ZH_ESTATE, "no tables for scale %d", scale);
    const Dict& d = c->dicts[scale];
    if (alpha) std::memcpy(alpha, d.h_alpha.data(), sizeof(float) * d.h_alpha.size());
    if (beta) std::memcpy(beta, d.h_beta.data(), sizeof(float) * d.h_beta.size());
    return ZH_OK;
}

zh_status zh_hash(zh_ctx* c, int scale, const float* feat, int64_t n, int32_t* codes, uint64_t* keys) {
    if (!c) return ZH_EINVAL;
    if (scale < 1 || scale > kMaxScale || !c->dicts[scale].valid) return fail(c, ZH_ESTATE, "no tables for scale %d", scale);
    if (!feat || n < 0) return fail(c, ZH_EINVAL, "zh_hash: bad arguments");
    TRY(set_device(c));
    Dict& d = c->dicts[scale];
    uint64_t* kp = keys;
    if (!kp) {
        TRY(ensure(c, c->tmp, sizeof(uint64_t) * (size_t)(n > 0 ? n : 1) * d.L));
        kp = P<uint64_t>(c->tmp);
    }
    TRY(clear_counters(c));
    HashArgs ha{};
    ha.feat = feat;
    ha.n = n;
    ha.D = d.D;
    ha.L = d.L;
    ha.k = d.k;
    ha.alpha = P<float>(d.alpha);
    ha.a_hi = P<uint16_t>(d.ahi);
    ha.a_lo = P<uint16_t>(d.alo);
    ha.beta = P<float>(d.beta);
    ha.key_mul = P<uint64_t>(d.kmul);
    set_bounds(ha, d, c->opts.proj);
    ha.w = d.w;
    ha.prec = c->opts.proj;
    ha.keys = kp;
    ha.codes = codes;
    ha.n_fixed = P<unsigned int>(c->counters) + C_CODEFIX;
    TRY(hash_scratch(c, ha));
    HIPCHK(c, launch_hash(ha, c->stream));
    return ZH_OK;
}

// Per feature row of zh_hash_noalloc: the dirty mask (8 bytes) and its share of
// the fix list (kFixSlots entries per 16 rows) and of the list's counts.
static size_t noalloc_row_bytes(int k) {
    return 8 + (size_t)kFixSlots * sizeof(int32_t) * (size_t)(((k + 2) + 3) & ~3) / 16 + 1;
}
static int64_t noalloc_max_rows(int k) {
    return (int64_t)((kNoAllocBytes - 512) / noalloc_row_bytes(k)) & ~(int64_t)15;
}

zh_status zh_hash_noalloc(zh_ctx* c, int scale, const float* feat, int64_t n, int32_t* codes, uint64_t* keys) {
    if (!c) return ZH_EINVAL;
    if (scale < 1 || scale > kMaxScale || !c->dicts[scale].valid) return fail(c, ZH_ESTATE, "no tables for scale %d", scale);
    Dict& d = c->dicts[scale];
    if (!feat || !keys || n < 0) return fail(c, ZH_EINVAL, "zh_hash_noalloc: need feat and keys, n >= 0");
    const int64_t nmax = noalloc_max_rows(d.k);
    if (n > nmax)
        return fail(c, ZH_EINVAL, "zh_hash_noalloc: %lld rows exceed the fixed scratch (%zu bytes: at most %lld rows at k = %d)",
                    (long long)n, kNoAllocBytes, (long long)nmax, d.k);
    if (c->device >= kNoAllocDevices || !g_noalloc_ptr[c->device])
        return fail(c, ZH_EDEVICE, "zh_hash_noalloc: no fixed scratch on device %d", c->device);
    if (n == 0) return ZH_OK;
    TRY(set_device(c));
    // carve the scratch: dirty mask [n] u64, fix list, fix counts [ceil(n/16)]
    // (every entry the kernels read is written by them first in the same
    // call, so nothing needs clearing)
    unsigned char* base = static_cast<unsigned char*>(g_noalloc_ptr[c->device]);
    const size_t nw = (size_t)((n + 15) / 16);
    const size_t fe = (size_t)(((d.k + 2) + 3) & ~3);
    HashArgs ha{};
    ha.feat = feat;
    ha.n = n;
    ha.D = d.D;
    ha.L = d.L;
    ha.k = d.k;
    ha.alpha = P<float>(d.alpha);
    ha.a_hi = P<uint16_t>(d.ahi);
    ha.a_lo = P<uint16_t>(d.alo);
    ha.beta = P<float>(d.beta);
    ha.key_mul = P<uint64_t>(d.kmul);
    set_bounds(ha, d, c->opts.proj);
    ha.w = d.w;
    ha.prec = c->opts.proj;
    ha.keys = keys;
    ha.codes = codes;
    ha.n_fixed = nullptr;
    ha.dirty = reinterpret_cast<uint64_t*>(base);
    ha.fix_cap = kFixSlots;
    ha.fix_list = reinterpret_cast<int32_t*>(base + ((8 * (size_t)n + 255) & ~(size_t)255));
    ha.fix_count = reinterpret_cast<unsigned int*>(reinterpret_cast<unsigned char*>(ha.fix_list) +
                                                  ((nw * kFixSlots * fe * sizeof(int32_t) + 255) & ~(size_t)255));
    HIPCHK(c, launch_hash(ha, c->stream));
    return ZH_OK;
}

zh_status zh_set_query_opts(zh_ctx* c, const zh_query_opts* o) {
    if (!c) return ZH_EINVAL;
    if (!o || o->cap < 0 || o->cap > 256 || o->rerank < 0 || o->rerank > 64 || (o->proj != 0 && o->proj != 1) ||
        (o->lle_fp64 != 0 && o->lle_fp64 != 1))
        return fail(c, ZH_EINVAL, "zh_set_query_opts: cap in [0,256], rerank in [0,64], proj and lle_fp64 in {0,1}");
    c->opts = *o;
    return ZH_OK;
}

zh_status zh_set_query_metric(zh_ctx* c, int metric) {
    if (!c) return ZH_EINVAL;
    if (metric != ZH_METRIC_L2 && metric != ZH_METRIC_L1)
        return fail(c, ZH_EINVAL, "zh_set_query_metric: ZH_METRIC_L2 or ZH_METRIC_L1");
    c->metric = metric;
    return ZH_OK;
}

// The K nearest of every patch of the current query under l1 (Section 4.1):
// the early-stop candidate lists (the union step of the search alone), then
// the ranking, through the l1 screen when D = 100. Needs opts.cap > 0.
zh_status rank_l1(zh_ctx* c, Dict& d) {
    const int cap = c->opts.cap;
    TRY(ensure(c, c->l1cand, sizeof(int32_t) * (size_t)(c->Q > 0 ? c->Q : 1) * cap));
    // the l1 screen of the dictionary (D = 100), once per set of features
    const bool screened = d.D == kL1sDim && cap <= kRankMaxCand;
    if (screened && !d.l1s_ok) {
        TRY(ensure(c, d.l1s, (size_t)kL1sBytes * (size_t)d.n));
        HIPCHK(c, launch_l1_screen_rows(P<float>(d.xf), d.n, P<uint8_t>(d.l1s), c->stream));
        d.l1s_ok = true;
    }
    TRY(ensure(c, c->nsurv, sizeof(int32_t) * (size_t)(c->Q > 0 ? c->Q : 1)));
    TRY(run_search(c, d, P<int32_t>(c->l1cand), cap, true));
    StageTimer t(c, ZH_T_SEARCH);
    if (screened) {
        HIPCHK(c, launch_knn_l1_screened((int)c->Q, c->qK, cap, P<float>(c->qfeat), P<float>(d.xf), P<uint8_t>(d.l1s),
                                         P<int32_t>(c->l1cand), P<int32_t>(c->ncand), P<int32_t>(c->ids),
                                         P<float>(c->d2), P<int32_t>(c->m), P<int32_t>(c->nsurv), c->stream));
    } else {
        HIPCHK(c, launch_knn_rank((int)c->Q, d.D, c->qK, cap, true, P<float>(c->qfeat), P<float>(d.xf),
                                  P<int32_t>(c->l1cand), P<int32_t>(c->ncand), P<int32_t>(c->ids), P<float>(c->d2),
                                  P<int32_t>(c->m), c->stream));
        // every candidate reaches the exact pass: survivors = min(ncand, cap)
        HIPCHK(c, launch_min_i32((int)c->Q, P<int32_t>(c->ncand), cap, P<int32_t>(c->nsurv), c->stream));
    }
    return ZH_OK;
}

zh_status zh_query(zh_ctx* c, const float* lr, int h, int w, int scale, int K) {
    if (!c) return ZH_EINVAL;
    if (!lr || h < kPatch || w < kPatch || K < 1 || K > kMaxK)
        return fail(c, ZH_EINVAL, "zh_query: need lr, h, w >= 5 and 1 <= K <= %d", kMaxK);
    if (scale < 1 || scale > kMaxScale || !c->dicts[scale].valid)
        return fail(c, ZH_ESTATE, "zh_query: no tables built for scale %d", scale);
    if (c->opts.rerank > 0 && c->opts.rerank < K)
        return fail(c, ZH_EINVAL, "zh_query: rerank %d below K %d", c->opts.rerank, K);
    if (c->metric == ZH_METRIC_L1 && c->opts.cap < 1)
        return fail(c, ZH_EUNSUPPORTED, "zh_query: the l1 metric needs the early stop (query option cap > 0)");
    const int64_t Q = (int64_t)(h - 4) * (w - 4);
    if (Q >= (1ll << 31) / kMaxK) return fail(c, ZH_EINVAL, "zh_query: image too large");
    TRY(set_device(c));
    Dict& d = c->dicts[scale];
    c->stage = 0;
    const int ps2 = (kPatch * scale) * (kPatch * scale);
    TRY(ensure(c, c->lr, sizeof(float) * (size_t)h * w));
    TRY(ensure(c, c->maps, sizeof(float) * 4 * (size_t)h * w));
    TRY(ensure(c, c->qfeat, sizeof(float) * (size_t)Q * d.D));
    TRY(ensure(c, c->qmu, sizeof(double) * (size_t)Q));
    TRY(ensure(c, c->qkeys, sizeof(uint64_t) * (size_t)Q * d.L));
    TRY(ensure(c, c->qbins, sizeof(uint2) * (size_t)Q * d.L));
    TRY(ensure(c, c->ids, sizeof(int32_t) * (size_t)Q * K));
    TRY(ensure(c, c->d2, sizeof(float) * (size_t)Q * K));
    TRY(ensure(c, c->w, sizeof(float) * (size_t)Q * K));
    TRY(ensure(c, c->m, sizeof(int32_t) * (size_t)Q));
    TRY(ensure(c, c->ncand, sizeof(int32_t) * (size_t)Q));
    TRY(ensure(c, c->over, 2 * sizeof(int32_t) * (size_t)Q));
    HIPCHK(c, hipMemcpyAsync(c->lr.p, lr, sizeof(float) * (size_t)h * w, hipMemcpyDeviceToDevice, c->stream));
    c->qh = h;
    c->qw = w;
    c->qscale = scale;
    c->qK = K;
    c->Q = Q;
    c->all_m = false;
    TRY(clear_counters(c));
    {
        StageTimer t(c, ZH_T_FEATURES);
        if (d.mode == ZH_FEAT_GRAD4) HIPCHK(c, launch_gradient_maps(P<float>(c->lr), 1, h, w, P<float>(c->maps), c->stream));
        HIPCHK(c, launch_query_features(P<float>(c->lr), P<float>(c->maps), h, w, d.mode, P<float>(c->qfeat),
                                        P<double>(c->qmu), c->stream));
    }
    HashArgs ha{};
    ha.feat = P<float>(c->qfeat);
    ha.n = Q;
    ha.D = d.D;
    ha.L = d.L;
    ha.k = d.k;
    ha.alpha = P<float>(d.alpha);
    ha.a_hi = P<uint16_t>(d.ahi);
    ha.a_lo = P<uint16_t>(d.alo);
    ha.beta = P<float>(d.beta);
    ha.key_mul = P<uint64_t>(d.kmul);
    set_bounds(ha, d, c->opts.proj);
    ha.w = d.w;
    ha.prec = c->opts.proj;
    ha.keys = P<uint64_t>(c->qkeys);
    ha.codes = nullptr;
    ha.n_fixed = P<unsigned int>(c->counters) + C_CODEFIX;
    TRY(hash_scratch(c, ha));
    ha.dir = P<Slot>(d.dir);
    ha.dir_cap = d.cap;
    ha.dir_filter = P<uint32_t>(d.dfilt);
    ha.bins = P<uint2>(c->qbins);
    ha.keys_tmajor = 1;
    {
        StageTimer t(c, ZH_T_HASH);
        HIPCHK(c, launch_hash_codes(ha, c->stream));
    }
    {
        StageTimer t(c, ZH_T_PROBE);
        HIPCHK(c, launch_probe(ha, c->stream));
    }
    if (c->metric == ZH_METRIC_L1) {
        TRY(rank_l1(c, d));
        c->gram_ready = false;   // no search formed Gram matrices; zh_lle_weights forms them
    } else {
        TRY(run_search(c, d, nullptr, 0));
    }
    c->stage = 1;
    return ZH_OK;
}

zh_status zh_lle_weights(zh_ctx* c, double lambda) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_lle_weights before zh_query");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, ZH_EINVAL, "zh_lle_weights: lambda must be > 0");
    TRY(set_device(c));
    Dict& d = c->dicts[c->qscale];
    LleArgs a{};
    a.Q = (int)c->Q;
    a.D = d.D;
    a.K = c->qK;
    a.qfeat = P<float>(c->qfeat);
    a.ids = P<int32_t>(c->ids);
    a.m = P<int32_t>(c->m);
    a.hi = P<uint16_t>(d.hi);
    a.lo = P<uint16_t>(d.lo);
    a.hs = hi_stride(d.D);
    a.xf = P<float>(d.xf);
    a.lam = lambda;
    a.fp64 = c->opts.lle_fp64;
    a.w = P<float>(c->w);
    a.n_fp64 = P<unsigned int>(c->counters) + C_LLE64;
    if (c->qK <= 8) {
        // packed Gram matrices, then one thread per patch solves its system
        const int f64 = c->opts.lle_fp64;
        TRY(ensure(c, c->gram, (f64 ? 8 : 4) * (size_t)c->Q * 36));
        StageTimer t(c, ZH_T_LLE);
        if (!(c->gram_ready && c->gram_fp64 == f64)) HIPCHK(c, launch_gram(a, c->gram.p, f64, c->stream));
        HIPCHK(c, launch_lle_solve(a, c->gram.p, f64, c->stream));
    } else {
        StageTimer t(c, ZH_T_LLE);
        HIPCHK(c, launch_lle(a, c->stream));
    }
    c->lam = lambda;
    c->all_m = false;
    c->stage = 2;
    return ZH_OK;
}

zh_status zh_lle_all(zh_ctx* c, double lambda, int32_t* ids, float* w) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_lle_all before zh_query");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(c, ZH_EINVAL, "zh_lle_all: lambda must be > 0");
    const int cap = c->opts.cap;
    if (cap < 1 || cap > kAllMax)
        return fail(c, ZH_EUNSUPPORTED, "zh_lle_all needs the early stop with cap <= %d (query option cap)", kAllMax);
    TRY(set_device(c));
    Dict& d = c->dicts[c->qscale];
    const size_t Qn = (size_t)(c->Q > 0 ? c->Q : 1);
    TRY(ensure(c, c->l1cand, sizeof(int32_t) * Qn * cap));
    TRY(ensure(c, c->wall, sizeof(float) * Qn * cap));
    TRY(clear_counters(c));
    // the candidate lists of the last query, ascending (the search runs again and dumps them)
    TRY(run_search(c, d, P<int32_t>(c->l1cand), cap));
    {
        StageTimer t(c, ZH_T_LLE);
        HIPCHK(c, launch_lle_all((int)c->Q, d.D, cap, lambda, P<float>(c->qfeat), P<float>(d.xf), P<int32_t>(c->l1cand),
                                 P<int32_t>(c->ncand), P<float>(c->wall), c->stream));
    }
    if (ids) HIPCHK(c, hipMemcpyAsync(ids, c->l1cand.p, sizeof(int32_t) * (size_t)c->Q * cap, hipMemcpyDeviceToDevice, c->stream));
    if (w) HIPCHK(c, hipMemcpyAsync(w, c->wall.p, sizeof(float) * (size_t)c->Q * cap, hipMemcpyDeviceToDevice, c->stream));
    c->lam = lambda;
    c->all_m = true;
    c->all_cap = cap;
    c->stage = 2;
    return ZH_OK;
}

zh_status zh_reconstruct(zh_ctx* c, float* hr_out) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 2) return fail(c, ZH_ESTATE, "zh_reconstruct before zh_lle_weights");
    if (!hr_out) return fail(c, ZH_EINVAL, "zh_reconstruct: null output");
    TRY(set_device(c));
    Dict& d = c->dicts[c->qscale];
    const int s = c->qscale, ps2 = (kPatch * s) * (kPatch * s);
    // every match (zh_lle_all): ncand rows of the dumped lists; else the m
    // nearest
    const int32_t* ids = P<int32_t>(c->all_m ? c->l1cand : c->ids);
    const int32_t* cnt = P<int32_t>(c->all_m ? c->ncand : c->m);
    const float* wt = P<float>(c->all_m ? c->wall : c->w);
    const int K = c->all_m ? c->all_cap : c->qK;
    TRY(ensure(c, c->sbpart,
               sizeof(float) *
                   (size_t)std::max<int64_t>(sb_tiles(s, c->sb_rows, c->qh, c->qw) * sb_part_floats(s, c->sb_rows), 1)));
    {
        StageTimer t(c, ZH_T_SYNTH);
        HIPCHK(c, launch_synth_blend(s, c->sb_rows, K, c->qh, c->qw, ids, cnt, wt, P<double>(c->qmu), d.resid,
                                     P<float>(c->sbpart), P<float>(c->lr), hr_out, c->stream, 1));
    }
    {
        StageTimer t(c, ZH_T_BLEND);
        HIPCHK(c, launch_synth_blend(s, c->sb_rows, K, c->qh, c->qw, ids, cnt, wt, P<double>(c->qmu), d.resid,
                                     P<float>(c->sbpart), P<float>(c->lr), hr_out, c->stream, 2));
    }
    c->stage = 3;
    c->bp_rec = 0;
    return ZH_OK;
}

}  // extern "C"

namespace {

// `iters` back-projection steps of hr [s h, s w] against the LR image lr [h, w];
// record: keep the guides of the steps for zh_backward.
zh_status backproject_steps(zh_ctx* c, float* hr, const float* lr, int h, int w, int s, int iters, float sigma_s,
                            float sigma_r, bool record) {
    const int H = s * h, W = s * w;
    TRY(ensure(c, c->e, sizeof(float) * (size_t)h * w));
    TRY(ensure(c, c->tmp, sizeof(float) * (size_t)H * W));
    const Taps g = gauss_taps(1.0);
    float* a = hr;
    float* b = P<float>(c->tmp);
    if (record) {
        TRY(ensure(c, c->guides, sizeof(float) * (size_t)H * W * (size_t)(iters > 0 ? iters : 1)));
        c->bp_rec = 1;
        c->bp_iters = iters;
        c->bp_sigma_s = sigma_s;
        c->bp_sigma_r = sigma_r;
    }
    for (int t = 0; t < iters; ++t) {
        if (record)
            HIPCHK(c, hipMemcpyAsync(P<float>(c->guides) + (size_t)t * H * W, a, sizeof(float) * (size_t)H * W,
                                     hipMemcpyDeviceToDevice, c->stream));
        {
            StageTimer t1(c, ZH_T_BP_ERROR);
            HIPCHK(c, launch_degrade_residual(a, H, W, s, g, lr, P<float>(c->e), c->stream));
        }
        {
            StageTimer t2(c, ZH_T_BP_UPDATE);
            HIPCHK(c, launch_bp_update(a, P<float>(c->e), H, W, h, w, s, sigma_s, sigma_r, b, c->stream));
        }
        float* t2 = a; a = b; b = t2;
    }
    if (a != hr)
        HIPCHK(c, hipMemcpyAsync(hr, a, sizeof(float) * (size_t)H * W, hipMemcpyDeviceToDevice, c->stream));
    return ZH_OK;
}

// Keys' cubic (a = -0.5) at distance x, written as the oracle's expression
// (host libm pow), so that the weight tables agree bit for bit.
double keys_cubic_host(double x) {
    const double a = -0.5;
    x = std::fabs(x);
    if (x <= 1.0) return (a + 2.0) * std::pow(x, 3.0) - (a + 3.0) * std::pow(x, 2.0) + 1.0;
    if (x < 2.0) return a * std::pow(x, 3.0) - 5.0 * a * std::pow(x, 2.0) + 8.0 * a * x - 4.0 * a;
    return 0.0;
}

// wt[4 r + a] = weight of tap a (offset a - 1) at phase t = r / s
void upsample_weights(int s, double* wt) {
    for (int r = 0; r < s; ++r) {
        const double t = (double)r / (double)s;
        for (int a = 0; a < 4; ++a) wt[4 * r + a] = keys_cubic_host(t - (double)(a - 1));
    }
}

}  // namespace

extern "C" {

zh_status zh_backproject(zh_ctx* c, float* hr, int iters, float sigma_s, float sigma_r) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_backproject needs the LR image of a zh_query");
    if (!hr || iters < 0 || !(sigma_s > 0.f) || std::ceil(3.0 * sigma_s) > 8.0 || !(sigma_r > 0.f))
        return fail(c, ZH_EINVAL, "zh_backproject: need iters >= 0, 0 < sigma_s <= 8/3, sigma_r > 0");
    TRY(set_device(c));
    // keep the guides I^0 .. I^{iters-1} of the first call after zh_reconstruct
    const bool record = c->stage == 3 && c->bp_rec == 0;
    if (c->stage == 3 && c->bp_rec != 0) c->bp_rec = -1;
    return backproject_steps(c, hr, P<float>(c->lr), c->qh, c->qw, c->qscale, iters, sigma_s, sigma_r, record);
}

zh_status zh_backproject_lr(zh_ctx* c, float* hr, const float* lr, int h, int w, int scale, int iters, float sigma_s,
                            float sigma_r) {
    if (!c) return ZH_EINVAL;
    if (!hr || !lr || h < 1 || w < 1 || scale < 1 || scale > kMaxScale || iters < 0 || !(sigma_s > 0.f) ||
        std::ceil(3.0 * sigma_s) > 8.0 || !(sigma_r > 0.f))
        return fail(c, ZH_EINVAL, "zh_backproject_lr: need h, w >= 1, 1 <= scale <= %d, iters >= 0, "
                                  "0 < sigma_s <= 8/3, sigma_r > 0", kMaxScale);
    TRY(set_device(c));
    if (c->stage == 3) c->bp_rec = -1;   // the output of zh_reconstruct is no longer the recorded chain
    return backproject_steps(c, hr, lr, h, w, scale, iters, sigma_s, sigma_r, false);
}

zh_status zh_upsample(zh_ctx* c, const float* lr, int h, int w, int scale, float* out) {
    if (!c) return ZH_EINVAL;
    if (!lr || !out || h < 1 || w < 1 || scale < 1 || scale > kMaxScale || (int64_t)scale * h * scale * w >= (1ll << 31))
        return fail(c, ZH_EINVAL, "zh_upsample: bad arguments");
    TRY(set_device(c));
    double wt[4 * kMaxScale];
    upsample_weights(scale, wt);
    HIPCHK(c, launch_upsample64(lr, h, w, scale, wt, out, c->stream));
    return ZH_OK;
}

zh_status zh_make_dictionary_interp(zh_ctx* c, const float* hr, int n_img, int H, int W, const int32_t* pos, int64_t n,
                                    int scale, float sigma, int mode, float* feat, float* resid) {
    if (!c) return ZH_EINVAL;
    if (!hr || !pos || !feat || !resid || n_img < 1 || n < 1 || n >= (1ll << 31) || scale < 1 || scale > kMaxScale ||
        (mode != ZH_FEAT_MEANREM && mode != ZH_FEAT_GRAD4) || !(sigma > 0.f) || sigma > 5.f)
        return fail(c, ZH_EINVAL, "zh_make_dictionary_interp: bad arguments");
    if (H % scale || W % scale || H < kPatch || W < kPatch || (int64_t)n_img * H * W >= (1ll << 31))
        return fail(c, ZH_EINVAL, "zh_make_dictionary_interp: H and W must be multiples of scale and >= 5");
    TRY(set_device(c));
    TRY(ensure(c, c->chk, 16));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c->stream, P<uint32_t>(c->chk), 4, 0u);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, launch_check_positions(pos, n, n_img, H - kPatch, W - kPatch, P<uint32_t>(c->chk), c->stream));
    {
        uint32_t bad = 0;
        HIPCHK(c, hipMemcpyAsync(&bad, c->chk.p, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (bad) return fail(c, ZH_EINVAL, "zh_make_dictionary_interp: a position lies outside its image");
    }
    const int h = H / scale, w = W / scale;
    const size_t hw = (size_t)h * w, HW = (size_t)H * W;
    TRY(ensure(c, c->tmp, sizeof(float) * ((size_t)n_img * hw + 5 * (size_t)n_img * HW)));
    float* lrs = P<float>(c->tmp);
    float* up = lrs + (size_t)n_img * hw;
    float* maps = up + (size_t)n_img * HW;
    double wt[4 * kMaxScale];
    upsample_weights(scale, wt);
    HIPCHK(c, launch_degrade(hr, n_img, H, W, scale, gauss_taps(sigma), lrs, c->stream));
    for (int i = 0; i < n_img; ++i)
        HIPCHK(c, launch_upsample64(lrs + (size_t)i * hw, h, w, scale, wt, up + (size_t)i * HW, c->stream));
    HIPCHK(c, launch_gradient_maps(up, n_img, H, W, maps, c->stream));
    HIPCHK(c, launch_dict_cut(hr, up, maps, H, W, 1, pos, n, mode, feat, resid, c->stream));
    return ZH_OK;
}

zh_status zh_backward(zh_ctx* c, const float* g_hr, float* g_resid, float* g_lambda) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 3) return fail(c, ZH_ESTATE, "zh_backward needs zh_reconstruct first");
    if (c->bp_rec < 0)
        return fail(c, ZH_ESTATE, "zh_backward: more than one zh_backproject after zh_reconstruct");
    if (!g_hr || !g_resid || !g_lambda) return fail(c, ZH_EINVAL, "zh_backward: null pointer");
    if (c->all_m) return fail(c, ZH_EUNSUPPORTED, "zh_backward: weights over all matches (zh_lle_all) have no adjoint here");
    Dict& d = c->dicts[c->qscale];
    if (!d.resid) return fail(c, ZH_ESTATE, "zh_backward: the dictionary has no HR residuals");
    const int s = c->qscale, h = c->qh, w = c->qw, H = s * h, W = s * w, K = c->qK;
    const int ps2 = (kPatch * s) * (kPatch * s);
    if (K > kMaxK || d.D > 128) return fail(c, ZH_EUNSUPPORTED, "zh_backward: K <= 16, D <= 128");
    TRY(set_device(c));
    const int64_t HW = (int64_t)H * W, Q = c->Q;
    // workspace: gamma, F|S|a, four HR temporaries, H x w, h x w, h x W
    TRY(ensure(c, c->bwd, sizeof(float) * (size_t)(8 * HW + (int64_t)H * w + (int64_t)h * w + (int64_t)h * W)));
    float* gam = P<float>(c->bwd);
    float* FSa = gam + HW;
    float* tA = FSa + 3 * HW;
    float* tB = tA + HW;
    float* tC = tB + HW;
    float* tD = tC + HW;
    float* tHw = tD + HW;
    float* thw = tHw + (int64_t)H * w;
    float* thW = thw + (int64_t)h * w;
    TRY(ensure(c, c->e, sizeof(float) * (size_t)h * w));
    HIPCHK(c, hipMemcpyAsync(gam, g_hr, sizeof(float) * (size_t)HW, hipMemcpyDeviceToDevice, c->stream));
    const int T = c->bp_rec == 1 ? c->bp_iters : 0;
    if (T > 0) {
        const Taps g = gauss_taps(1.0);
        const float ss = c->bp_sigma_s, sr = c->bp_sigma_r;
        const int Rs = (int)std::ceil(3.0 * (double)ss);
        AxisAdjArgs gx{}, bx{}, ux{}, dx{};
        for (int dd = -Rs; dd <= Rs; ++dd) gx.taps[dd + Rs] = (float)std::exp(-(double)(dd * dd) / (2.0 * ss * ss));
        gx.R = Rs;
        bx.R = Rs;
        ux.s = s;
        dx.s = s;
        dx.R = g.R;
        for (int t = -g.R; t <= g.R; ++t) dx.taps[t + g.R] = (float)g.g[t + g.R];
        const bool range = std::isfinite(sr);
        for (int t = T - 1; t >= 0; --t) {
            const float* I = P<float>(c->guides) + (size_t)t * HW;
            HIPCHK(c, launch_degrade_residual(I, H, W, s, g, P<float>(c->lr), P<float>(c->e), c->stream));
            HIPCHK(c, launch_bp_terms(I, P<float>(c->e), H, W, h, w, s, ss, sr, FSa, c->stream));
            // v = Blur^T Dec^T Up^T N^T (S gamma)
            AxisAdjArgs a = gx;
            a.in = gam; a.mul = FSa + HW; a.out = tA; a.rows = H; a.n_in = W; a.n_out = W;
            HIPCHK(c, launch_axis_adj(kAdjGauss, 0, a, c->stream));
            a = gx;
            a.in = tA; a.out = tB; a.rows = W; a.n_in = H; a.n_out = H;
            HIPCHK(c, launch_axis_adj(kAdjGauss, 1, a, c->stream));
            a = ux;
            a.in = tB; a.out = tHw; a.rows = H; a.n_in = W; a.n_out = w;
            HIPCHK(c, launch_axis_adj(kAdjUp, 0, a, c->stream));
            a = ux;
            a.in = tHw; a.out = thw; a.rows = w; a.n_in = H; a.n_out = h;
            HIPCHK(c, launch_axis_adj(kAdjUp, 1, a, c->stream));
            a = dx;
            a.in = thw; a.out = thW; a.rows = h; a.n_in = w; a.n_out = W;
            HIPCHK(c, launch_axis_adj(kAdjDec, 0, a, c->stream));
            a = dx;
            a.in = thW; a.out = tA; a.rows = W; a.n_in = h; a.n_out = H;
            HIPCHK(c, launch_axis_adj(kAdjDec, 1, a, c->stream));
            if (range) {
                // z = -(a / sigma_r^2) S F gamma, then Box^T z
                HIPCHK(c, launch_bp_adj_z(FSa, gam, HW, sr, tC, c->stream));
                a = bx;
                a.in = tC; a.out = tB; a.rows = H; a.n_in = W; a.n_out = W;
                HIPCHK(c, launch_axis_adj(kAdjBox, 0, a, c->stream));
                a = bx;
                a.in = tB; a.out = tD; a.rows = W; a.n_in = H; a.n_out = H;
                HIPCHK(c, launch_axis_adj(kAdjBox, 1, a, c->stream));
                HIPCHK(c, launch_bp_adj_combine(gam, tA, tC, tD, HW, c->stream));
            } else {
                HIPCHK(c, launch_bp_adj_combine(gam, tA, nullptr, nullptr, HW, c->stream));
            }
        }
    }
    // blend: gradient per covered pixel over its count
    float* gp = tB;
    HIPCHK(c, launch_blend_adj(gam, P<int32_t>(c->m), h, w, s, gp, c->stream));
    // lambda
    TRY(ensure(c, c->clam, sizeof(double) * (size_t)(Q > 0 ? Q : 1)));
    BackwardArgs ba{};
    ba.Q = (int)Q;
    ba.D = d.D;
    ba.K = K;
    ba.s = s;
    ba.w = w;
    ba.hs = hi_stride(d.D);
    ba.qfeat = P<float>(c->qfeat);
    ba.ids = P<int32_t>(c->ids);
    ba.m = P<int32_t>(c->m);
    ba.hi = P<uint16_t>(d.hi);
    ba.lo = P<uint16_t>(d.lo);
    ba.resid = d.resid;
    ba.gp = gp;
    ba.lam = c->lam;
    ba.c_lam = P<double>(c->clam);
    if (K <= 8) {
        // FP64 Gram matrices of the neighbours: those of the search when it
        // formed them in FP64, else formed here
        if (!(c->gram_ready && c->gram_fp64)) {
            LleArgs la{};
            la.Q = (int)Q;
            la.D = d.D;
            la.K = K;
            la.qfeat = P<float>(c->qfeat);
            la.ids = P<int32_t>(c->ids);
            la.m = P<int32_t>(c->m);
            la.hi = P<uint16_t>(d.hi);
            la.lo = P<uint16_t>(d.lo);
            la.hs = hi_stride(d.D);
            la.xf = P<float>(d.xf);
            TRY(ensure(c, c->gram, sizeof(double) * (size_t)(Q > 0 ? Q : 1) * 36));
            HIPCHK(c, launch_gram(la, c->gram.p, 1, c->stream));
            c->gram_ready = true;
            c->gram_fp64 = 1;
        }
        TRY(ensure(c, c->bwd_gw, sizeof(double) * 8 * (size_t)(Q > 0 ? Q : 1)));
        HIPCHK(c, launch_lam_adj8(ba, P<double>(c->gram), P<double>(c->bwd_gw), c->stream));
    } else {
        HIPCHK(c, launch_lle_lambda_adj(ba, c->stream));
    }
    HIPCHK(c, launch_sum_f64(P<double>(c->clam), Q, g_lambda, c->stream));
    // dictionary rows: the neighbour lists sorted by row (stable), one wave per row
    const int64_t E = Q * K;
    const uint32_t none = (uint32_t)d.n;
    int bits = 1;
    while (bits < 32 && (1ull << bits) <= (uint64_t)d.n) ++bits;
    const int64_t hsz = radix_hist_size(E > 0 ? E : 1);
    TRY(ensure(c, c->bwd_k, sizeof(uint32_t) * (size_t)(4 * (E > 0 ? E : 1) + hsz)));
    uint32_t* k0 = P<uint32_t>(c->bwd_k);
    uint32_t* v0 = k0 + E;
    uint32_t* k1 = v0 + E;
    uint32_t* v1 = k1 + E;
    uint32_t* hist = v1 + E;
    HIPCHK(c, hipMemsetAsync(g_resid, 0, sizeof(float) * (size_t)d.n * ps2, c->stream));
    if (E > 0) {
        HIPCHK(c, launch_nbr_pairs(P<int32_t>(c->ids), P<int32_t>(c->m), (int)Q, K, none, k0, v0, c->stream));
        bool first = true;
        HIPCHK(c, radix_sort_pairs(k0, v0, k1, v1, E, bits, hist, hsz, c->stream, &first));
        const int64_t nchunk = (E + 63) / 64;
        TRY(ensure(c, c->bwd_part, sizeof(float) * 2 * (size_t)ps2 * nchunk + 8 * (size_t)nchunk));
        float* part = P<float>(c->bwd_part);
        void* info = part + 2 * (size_t)ps2 * nchunk;
        HIPCHK(c, launch_dict_grad(first ? k0 : k1, first ? v0 : v1, E, none, P<float>(c->w), gp, w, s, K, g_resid,
                                   part, info, c->stream));
    }
    return ZH_OK;
}

// ---- batched form -------------------------------------------------------------
namespace {

zh_status batch_check(zh_ctx* c, const zh_batch* b) {
    if (!b || b->n_images < 1 || !b->lr || !b->hr_out || !b->h || !b->w || !b->scale)
        return fail(c, ZH_EINVAL, "zh_run_batch: empty or incomplete batch");
    if (b->K < 1 || b->K > kMaxK || !(b->lambda > 0.0) || !std::isfinite(b->lambda) || b->bp_iters < 0 ||
        !(b->sigma_s > 0.f) || std::ceil(3.0 * b->sigma_s) > 8.0 || !(b->sigma_r > 0.f))
        return fail(c, ZH_EINVAL, "zh_run_batch: bad K, lambda or back-projection parameters");
    if (c->opts.rerank > 0 && c->opts.rerank < b->K) return fail(c, ZH_EINVAL, "zh_run_batch: rerank below K");
    if (c->metric != ZH_METRIC_L2)
        return fail(c, ZH_EUNSUPPORTED, "zh_run_batch: the batched form ranks by squared l2 (query metric l1 set)");
    for (int i = 0; i < b->n_images; ++i) {
        const int s = b->scale[i];
        if (!b->lr[i] || !b->hr_out[i] || b->h[i] < kPatch || b->w[i] < kPatch)
            return fail(c, ZH_EINVAL, "zh_run_batch: image %d: null pointer or side < 5", i);
        if (s < 1 || s > kMaxScale || !c->dicts[s].valid) return fail(c, ZH_ESTATE, "zh_run_batch: no tables for scale %d", s);
    }
    return ZH_OK;
}

std::vector<uint64_t> batch_signature(zh_ctx* c, const zh_batch* b) {
    std::vector<uint64_t> v;
    uint64_t lb;
    std::memcpy(&lb, &b->lambda, 8);
    uint32_t ss, sr;
    std::memcpy(&ss, &b->sigma_s, 4);
    std::memcpy(&sr, &b->sigma_r, 4);
    v.insert(v.end(), {(uint64_t)b->n_images, (uint64_t)b->K, lb, (uint64_t)b->bp_iters, ss, sr,
                       (uint64_t)c->opts.cap, (uint64_t)c->opts.rerank, (uint64_t)c->opts.proj,
                       (uint64_t)c->opts.lle_fp64, (uint64_t)c->batch.tile, (uint64_t)c->batch.grid_per_cu,
                       (uint64_t)c->sb_rows, (uint64_t)(uintptr_t)c->stream, c->gen});
    for (int s = 1; s <= kMaxScale; ++s) {
        v.push_back((uint64_t)(uintptr_t)c->dicts[s].dir.p);
        v.push_back((uint64_t)(uintptr_t)c->dicts[s].dfilt.p);
    }
    for (int i = 0; i < b->n_images; ++i)
        v.insert(v.end(), {(uint64_t)(uintptr_t)b->lr[i], (uint64_t)(uintptr_t)b->hr_out[i], (uint64_t)b->h[i],
                           (uint64_t)b->w[i], (uint64_t)b->scale[i]});
    return v;
}

// Image tables and every buffer the chain needs, sized before any capture.
zh_status batch_plan(zh_ctx* c, const zh_batch* b) {
    auto& B = c->batch;
    int64_t q_max = 0, lr_max = 0, hr_max = 0, part_max = 0, L_max = 0, k_max = 0, D_max = 0;
    std::vector<BatchImage> tabs[kMaxScale + 1];
    for (int s = 1; s <= kMaxScale; ++s) {
        auto& g = B.g[s];
        int64_t q = 0, lr = 0, hr = 0, tiles = 0, fsegs = 0, sbt = 0, dt = 0;
        for (int i = 0; i < b->n_images; ++i) {
            if (b->scale[i] != s) continue;
            BatchImage im{};
            im.lr = b->lr[i];
            im.out = b->hr_out[i];
            im.h = b->h[i];
            im.w = b->w[i];
            im.lr_off = lr;
            im.q_off = q;
            im.hr_off = hr;
            im.tile_off = tiles;
            im.fblk_off = fsegs;
            im.sbt_off = sbt;
            im.dtile_off = dt;
            tabs[s].push_back(im);
            lr += (int64_t)im.h * im.w;
            q += (int64_t)(im.h - 4) * (im.w - 4);
            hr += (int64_t)s * im.h * s * im.w;
            tiles += bp_tiles(s * im.h, s * im.w, B.tile);
            fsegs += feature_segments(im.h, im.w);
            sbt += sb_tiles(s, c->sb_rows, im.h, im.w);
            dt += degrade_tiles(im.h, im.w);
        }
        g.n = (int)tabs[s].size();
        g.q_total = q;
        g.lr_total = lr;
        g.hr_total = hr;
        g.tiles = tiles;
        g.fsegs = fsegs;
        g.sbtiles = sbt;
        g.dtiles = dt;
        if (!g.n) continue;
        if (q * kMaxK >= (1ll << 31)) return fail(c, ZH_EINVAL, "zh_run_batch: too many patches at scale %d", s);
        const Dict& d = c->dicts[s];
        q_max = std::max(q_max, q);
        lr_max = std::max(lr_max, lr);
        hr_max = std::max(hr_max, hr);
        part_max = std::max<int64_t>(part_max, g.sbtiles * sb_part_floats(s, c->sb_rows));
        L_max = std::max<int64_t>(L_max, d.L);
        k_max = std::max<int64_t>(k_max, d.k);
        D_max = std::max<int64_t>(D_max, d.D);
    }
    // the groups run one after another and share the scratch
    TRY(ensure(c, B.scr, sizeof(float) * (size_t)std::max<int64_t>(hr_max, 1)));
    for (int s = 1; s <= kMaxScale; ++s) {
        auto& g = B.g[s];
        if (!g.n) continue;
        for (auto& im : tabs[s]) im.scr = P<float>(B.scr) + im.hr_off;
        TRY(ensure(c, g.table, sizeof(BatchImage) * tabs[s].size()));
        HIPCHK(c, hipMemcpy(g.table.p, tabs[s].data(), sizeof(BatchImage) * tabs[s].size(), hipMemcpyHostToDevice));
    }
    const int64_t K = b->K;
    TRY(ensure(c, B.e, sizeof(float) * (size_t)std::max<int64_t>(lr_max, 1)));
    TRY(ensure(c, B.counter, 16));
    TRY(ensure(c, c->maps, sizeof(float) * 4 * (size_t)std::max<int64_t>(lr_max, 1)));
    TRY(ensure(c, c->qfeat, sizeof(float) * (size_t)q_max * D_max));
    TRY(ensure(c, c->qmu, sizeof(double) * (size_t)q_max));
    TRY(ensure(c, c->qkeys, sizeof(uint64_t) * (size_t)q_max * L_max));
    TRY(ensure(c, c->qbins, sizeof(uint2) * (size_t)q_max * L_max));
    TRY(ensure(c, c->ids, sizeof(int32_t) * (size_t)q_max * K));
    TRY(ensure(c, c->d2, sizeof(float) * (size_t)q_max * K));
    TRY(ensure(c, c->w, sizeof(float) * (size_t)q_max * K));
    TRY(ensure(c, c->m, sizeof(int32_t) * (size_t)q_max));
    TRY(ensure(c, c->ncand, sizeof(int32_t) * (size_t)q_max));
    TRY(ensure(c, c->nsurv, sizeof(int32_t) * (size_t)std::max<int64_t>(q_max, 1)));
    TRY(ensure(c, c->qrot, sizeof(float) * kRotStride * (size_t)std::max<int64_t>(q_max, 1)));
    TRY(ensure(c, c->over, 2 * sizeof(int32_t) * (size_t)q_max));
    TRY(ensure(c, c->sbpart, sizeof(float) * (size_t)std::max<int64_t>(part_max, 1)));
    TRY(ensure(c, c->counters, kNumCounters * sizeof(uint32_t)));
    if (K <= 8) TRY(ensure(c, c->gram, (c->opts.lle_fp64 ? 8 : 4) * (size_t)q_max * 36));
    HashArgs ha{};
    ha.n = q_max;
    ha.L = (int)L_max;
    ha.k = (int)k_max;
    TRY(hash_scratch(c, ha));
    return ZH_OK;
}

// The launch chain of a planned batch on stream st: nothing allocates.
zh_status batch_chain(zh_ctx* c, const zh_batch* b, hipStream_t st) {
    auto& B = c->batch;
    hipStream_t saved = c->stream;
    const bool timing = c->timing;
    c->stream = st;
    c->timing = false;
    zh_status rc = ZH_OK;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || ncu < 1) ncu = 256;
    for (int s = 1; s <= kMaxScale && rc == ZH_OK; ++s) {
        auto& g = B.g[s];
        if (!g.n) continue;
        Dict& d = c->dicts[s];
        const BatchImage* tab = P<BatchImage>(g.table);
        const int K = b->K;
        rc = [&]() -> zh_status {
            c->Q = g.q_total;
            c->qK = K;
            c->qscale = s;
            TRY(clear_counters(c));
            if (d.mode == ZH_FEAT_GRAD4) HIPCHK(c, launch_b_gradient_maps(tab, g.n, g.lr_total, P<float>(c->maps), st));
            HIPCHK(c, launch_b_query_features(tab, g.n, g.fsegs, d.mode, P<float>(c->maps), P<float>(c->qfeat),
                                              P<double>(c->qmu), st));
            HashArgs ha{};
            ha.feat = P<float>(c->qfeat);
            ha.n = g.q_total;
            ha.D = d.D;
            ha.L = d.L;
            ha.k = d.k;
            ha.alpha = P<float>(d.alpha);
            ha.a_hi = P<uint16_t>(d.ahi);
            ha.a_lo = P<uint16_t>(d.alo);
            ha.beta = P<float>(d.beta);
            ha.key_mul = P<uint64_t>(d.kmul);
            set_bounds(ha, d, c->opts.proj);
            ha.w = d.w;
            ha.prec = c->opts.proj;
            ha.keys = P<uint64_t>(c->qkeys);
            ha.n_fixed = P<unsigned int>(c->counters) + C_CODEFIX;
            TRY(hash_scratch(c, ha));
            ha.dir = P<Slot>(d.dir);
            ha.dir_cap = d.cap;
            ha.dir_filter = P<uint32_t>(d.dfilt);
            ha.bins = P<uint2>(c->qbins);
            ha.keys_tmajor = 1;
            HIPCHK(c, launch_hash(ha, st));
            TRY(run_search(c, d, nullptr, 0));
            LleArgs la{};
            la.Q = (int)g.q_total;
            la.D = d.D;
            la.K = K;
            la.qfeat = P<float>(c->qfeat);
            la.ids = P<int32_t>(c->ids);
            la.m = P<int32_t>(c->m);
            la.hi = P<uint16_t>(d.hi);
            la.lo = P<uint16_t>(d.lo);
            la.hs = hi_stride(d.D);
            la.xf = P<float>(d.xf);
            la.lam = b->lambda;
            la.fp64 = c->opts.lle_fp64;
            la.w = P<float>(c->w);
            la.n_fp64 = P<unsigned int>(c->counters) + C_LLE64;
            if (K <= 8) {
                if (!c->gram_ready) HIPCHK(c, launch_gram(la, c->gram.p, c->opts.lle_fp64, st));
                HIPCHK(c, launch_lle_solve(la, c->gram.p, c->opts.lle_fp64, st));
            } else {
                HIPCHK(c, launch_lle(la, st));
            }
            HIPCHK(c, launch_b_synth_blend(tab, g.n, g.sbtiles, g.hr_total, s, c->sb_rows, K, P<int32_t>(c->ids),
                                           P<int32_t>(c->m), P<float>(c->w), P<double>(c->qmu), d.resid,
                                           P<float>(c->sbpart), st));
            const Taps tg = gauss_taps(1.0);
            for (int t = 0; t < b->bp_iters; ++t) {
                HIPCHK(c, launch_b_degrade_residual(tab, g.n, g.lr_total, g.dtiles, s, tg, t & 1, P<float>(B.e), st));
                HIPCHK(c, launch_b_bp_update(tab, g.n, g.tiles, B.tile, B.grid_per_cu * ncu, s, b->sigma_s, b->sigma_r,
                                             P<float>(B.e), t & 1, P<unsigned int>(B.counter), st));
            }
            if (b->bp_iters & 1) HIPCHK(c, launch_b_copy_scr(tab, g.n, g.hr_total, s, st));
            return ZH_OK;
        }();
    }
    c->stream = saved;
    c->timing = timing;
    return rc;
}

zh_status batch_stream(zh_ctx* c) {
    auto& B = c->batch;
    if (!B.stream) {
        HIPCHK(c, hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&B.ev_in, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&B.ev_out, hipEventDisableTiming));
    }
    return ZH_OK;
}

}  // namespace

zh_status zh_run_batch(zh_ctx* c, const zh_batch* b) {
    if (!c) return ZH_EINVAL;
    TRY(batch_check(c, b));
    TRY(set_device(c));
    TRY(batch_stream(c));
    auto& B = c->batch;
    c->stage = 0;
    std::vector<uint64_t> sig = batch_signature(c, b);
    if (sig != B.sig || !B.exec) {
        if (B.exec) {
            HIPCHK(c, hipStreamSynchronize(B.stream));
            HIPCHK(c, hipGraphExecDestroy(B.exec));
            B.exec = nullptr;
        }
        B.sig.clear();
        HIPCHK(c, hipStreamSynchronize(c->stream));
        TRY(batch_plan(c, b));
        hipGraph_t graph = nullptr;
        HIPCHK(c, hipStreamBeginCapture(B.stream, hipStreamCaptureModeRelaxed));
        const zh_status rc = batch_chain(c, b, B.stream);
        const hipError_t ec = hipStreamEndCapture(B.stream, &graph);
        if (rc != ZH_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        HIPCHK(c, ec);
        const hipError_t ei = hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(c, ei);
        // planning sizes (and may reallocate) buffers: the signature is that
        // of the state the graph was captured against
        B.sig = batch_signature(c, b);
    }
    HIPCHK(c, hipEventRecord(B.ev_in, c->stream));
    HIPCHK(c, hipStreamWaitEvent(B.stream, B.ev_in, 0));
    HIPCHK(c, hipGraphLaunch(B.exec, B.stream));
    HIPCHK(c, hipEventRecord(B.ev_out, B.stream));
    HIPCHK(c, hipStreamWaitEvent(c->stream, B.ev_out, 0));
    return ZH_OK;
}

}  // extern "C"

namespace {

// Key of a batch for the tuning cache: device, HIP runtime, and everything
// that shapes the launches (sizes, zoom factors, K, iterations, query options).
uint64_t tune_key(zh_ctx* c, const zh_batch* b, std::string& dev, std::string& arch, int& rt) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) (void)hipGetLastError();
    dev = prop.name;
    arch = prop.gcnArchName;
    rt = 0;
    if (hipRuntimeGetVersion(&rt) != hipSuccess) (void)hipGetLastError();
    uint64_t h = fmix64(0x5A17ull + (uint64_t)rt);
    auto mix = [&](uint64_t v) { h = fmix64(h ^ (v + kGolden)); };
    for (char ch : dev) mix((uint64_t)(unsigned char)ch);
    for (char ch : arch) mix((uint64_t)(unsigned char)ch);
    mix((uint64_t)b->n_images);
    for (int i = 0; i < b->n_images; ++i) {
        mix((uint64_t)b->h[i]);
        mix((uint64_t)b->w[i]);
        mix((uint64_t)b->scale[i]);
    }
    mix((uint64_t)b->K);
    mix((uint64_t)b->bp_iters);
    mix((uint64_t)c->opts.cap);
    mix((uint64_t)c->opts.rerank);
    mix((uint64_t)c->opts.proj);
    mix((uint64_t)c->opts.lle_fp64);
    return h;
}

// An earlier choice for `key` in the cache file (one JSON object per line).
bool tune_lookup(const char* path, uint64_t key, int& tile, int& mult, int& rows) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[2048];
    char want[64];
    std::snprintf(want, sizeof(want), "\"key\": \"%016llx\"", (unsigned long long)key);
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, want)) continue;
        const char* a = std::strstr(line, "\"bp_tile\": ");
        const char* g = std::strstr(line, "\"bp_grid_per_cu\": ");
        const char* y = std::strstr(line, "\"synth_rows\": ");
        int t = 0, m = 0, sg = 0;
        if (a && g && y && std::sscanf(a + 11, "%d", &t) == 1 && std::sscanf(g + 18, "%d", &m) == 1 &&
            std::sscanf(y + 14, "%d", &sg) == 1 && (t == 16 || t == 32) && (m == 2 || m == 4 || m == 8) &&
            (sg == 4 || sg == 8)) {
            tile = t;
            mult = m;
            rows = sg;
            found = true;   // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const char* path, uint64_t key, const std::string& dev, const std::string& arch, int rt,
                const zh_batch_tuning& t) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::string d;
    for (char ch : dev) d += (ch == '"' || ch == '\\') ? '_' : ch;
    std::string a;
    for (char ch : arch) a += (ch == '"' || ch == '\\') ? '_' : ch;
    std::fprintf(f, "{\"key\": \"%016llx\", \"device\": \"%s\", \"arch\": \"%s\", \"hip_runtime\": %d, "
                    "\"bp_tile\": %d, \"bp_grid_per_cu\": %d, \"synth_rows\": %d, \"bp_ms\": [%.4f, %.4f, %.4f, "
                    "%.4f, %.4f, %.4f], \"synth_ms\": [%.4f, %.4f]}\n",
                 (unsigned long long)key, d.c_str(), a.c_str(), rt, t.bp_tile, t.bp_grid_per_cu, t.synth_rows,
                 t.bp_ms[0], t.bp_ms[1], t.bp_ms[2], t.bp_ms[3], t.bp_ms[4], t.bp_ms[5], t.synth_ms[0],
                 t.synth_ms[1]);
    std::fclose(f);
}

}  // namespace

extern "C" {

zh_status zh_tune_batch(zh_ctx* c, const zh_batch* b, zh_batch_tuning* out) {
    if (!c) return ZH_EINVAL;
    TRY(batch_check(c, b));
    TRY(set_device(c));
    auto& B = c->batch;
    const char* cache = std::getenv("ZH_TUNE_CACHE");
    std::string dev, arch;
    int rt = 0;
    const uint64_t key = tune_key(c, b, dev, arch, rt);
    if (cache && cache[0]) {
        int t = 0, m = 0, g = 0;
        if (tune_lookup(cache, key, t, m, g)) {
            B.tile = t;
            B.grid_per_cu = m;
            c->sb_rows = g;
            B.sig.clear();
            if (out) {
                std::memset(out, 0, sizeof(*out));
                out->bp_tile = t;
                out->bp_grid_per_cu = m;
                out->synth_rows = g;
                out->from_cache = 1;
            }
            return zh_run_batch(c, b);
        }
    }
    TRY(zh_run_batch(c, b));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int tiles[2] = {16, 32}, mults[3] = {2, 4, 8};
    float ms[6];
    int best = -1;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || ncu < 1) ncu = 256;
    const int keep_tile = B.tile, keep_mult = B.grid_per_cu, keep_rows = c->sb_rows;
    zh_status rc = ZH_OK;
    auto time_once = [&](auto&& launch, float& best_ms) {
        best_ms = 1e30f;
        for (int rep = 0; rep < 2 && rc == ZH_OK; ++rep) {
            if (hipEventRecord(e0, B.stream) != hipSuccess) { rc = fail(c, ZH_EDEVICE, "event"); return; }
            if (!launch()) { rc = fail(c, ZH_EDEVICE, "zh_tune_batch: launch failed"); return; }
            (void)hipEventRecord(e1, B.stream);
            (void)hipEventSynchronize(e1);
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            best_ms = std::min(best_ms, t);
        }
    };
    for (int ti = 0; ti < 2 && rc == ZH_OK; ++ti) {
        B.tile = tiles[ti];
        B.sig.clear();
        rc = batch_plan(c, b);   // tile offsets of this tile size
        for (int mi = 0; mi < 3 && rc == ZH_OK; ++mi) {
            time_once([&]() {
                for (int s = 1; s <= kMaxScale; ++s) {
                    auto& g = B.g[s];
                    if (!g.n) continue;
                    const BatchImage* tab = P<BatchImage>(g.table);
                    if (launch_b_degrade_residual(tab, g.n, g.lr_total, g.dtiles, s, gauss_taps(1.0), 0, P<float>(B.e),
                                                  B.stream) !=
                            hipSuccess ||
                        launch_b_bp_update(tab, g.n, g.tiles, tiles[ti], mults[mi] * ncu, s, b->sigma_s, b->sigma_r,
                                           P<float>(B.e), 0, P<unsigned int>(B.counter), B.stream) != hipSuccess)
                        return false;
                }
                return true;
            }, ms[ti * 3 + mi]);
            if (best < 0 || ms[ti * 3 + mi] < ms[best]) best = ti * 3 + mi;
        }
    }
    // fused synthesis and blend of the last zoom factor of the batch (its
    // neighbours and weights are the context's) with tiles of 4 and 8 patch
    // rows
    float sms[2] = {0.f, 0.f};
    int sbest = kSbRows;
    int last = 0;
    for (int s = 1; s <= kMaxScale; ++s)
        if (B.g[s].n) last = s;
    if (rc == ZH_OK && last > 0) {
        const Dict& d = c->dicts[last];
        for (int ri = 0; ri < 2 && rc == ZH_OK; ++ri) {
            c->sb_rows = ri ? 8 : 4;
            B.sig.clear();
            rc = batch_plan(c, b);   // tile offsets of this tile height
            if (rc != ZH_OK) break;
            auto& g = B.g[last];
            time_once([&]() {
                return launch_b_synth_blend(P<BatchImage>(g.table), g.n, g.sbtiles, g.hr_total, last, c->sb_rows,
                                            b->K, P<int32_t>(c->ids), P<int32_t>(c->m), P<float>(c->w),
                                            P<double>(c->qmu), d.resid, P<float>(c->sbpart), B.stream) == hipSuccess;
            }, sms[ri]);
        }
        sbest = sms[0] < sms[1] ? 4 : 8;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ZH_OK || best < 0) {
        B.tile = keep_tile;
        B.grid_per_cu = keep_mult;
        c->sb_rows = keep_rows;
        B.sig.clear();
        return rc != ZH_OK ? rc : fail(c, ZH_EDEVICE, "zh_tune_batch: nothing timed");
    }
    B.tile = tiles[best / 3];
    B.grid_per_cu = mults[best % 3];
    c->sb_rows = sbest;
    B.sig.clear();   // re-plan and capture again with the chosen tuning
    zh_batch_tuning t{};
    t.bp_tile = B.tile;
    t.bp_grid_per_cu = B.grid_per_cu;
    for (int i = 0; i < 6; ++i) t.bp_ms[i] = ms[i];
    t.synth_rows = sbest;
    t.synth_ms[0] = sms[0];
    t.synth_ms[1] = sms[1];
    t.from_cache = 0;
    if (cache && cache[0]) tune_store(cache, key, dev, arch, rt, t);
    if (out) *out = t;
    return ZH_OK;
}

zh_status zh_get_results(zh_ctx* c, int32_t* ids, float* d2, int32_t* m, float* w, int32_t* ncand) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_get_results before zh_query");
    if (w && (c->stage < 2 || c->all_m))
        return fail(c, ZH_ESTATE, "weights of the K nearest requested before zh_lle_weights (or after zh_lle_all)");
    TRY(set_device(c));
    const size_t QK = (size_t)c->Q * c->qK, Q = (size_t)c->Q;
    if (ids) HIPCHK(c, hipMemcpyAsync(ids, c->ids.p, QK * 4, hipMemcpyDeviceToDevice, c->stream));
    if (d2) HIPCHK(c, hipMemcpyAsync(d2, c->d2.p, QK * 4, hipMemcpyDeviceToDevice, c->stream));
    if (m) HIPCHK(c, hipMemcpyAsync(m, c->m.p, Q * 4, hipMemcpyDeviceToDevice, c->stream));
    if (w) HIPCHK(c, hipMemcpyAsync(w, c->w.p, QK * 4, hipMemcpyDeviceToDevice, c->stream));
    if (ncand) HIPCHK(c, hipMemcpyAsync(ncand, c->ncand.p, Q * 4, hipMemcpyDeviceToDevice, c->stream));
    return ZH_OK;
}

zh_status zh_survivors(zh_ctx* c, int32_t* survivors) {
    if (!c || !survivors) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_survivors before zh_query");
    if (c->opts.cap <= 0 || !c->nsurv.p) return fail(c, ZH_ESTATE, "zh_survivors: the last query had no early stop");
    TRY(set_device(c));
    HIPCHK(c, hipMemcpyAsync(survivors, c->nsurv.p, (size_t)c->Q * 4, hipMemcpyDeviceToDevice, c->stream));
    return ZH_OK;
}

zh_status zh_query_shape(zh_ctx* c, int64_t* Q, int32_t* D) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "no query");
    if (Q) *Q = c->Q;
    if (D) *D = c->dicts[c->qscale].D;
    return ZH_OK;
}

zh_status zh_candidates(zh_ctx* c, int32_t cap_per_query, int32_t* counts, int32_t* ids) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_candidates before zh_query");
    if (cap_per_query < 1 || !counts || !ids) return fail(c, ZH_EINVAL, "zh_candidates: bad arguments");
    TRY(set_device(c));
    TRY(clear_counters(c));
    TRY(run_search(c, c->dicts[c->qscale], ids, cap_per_query));
    HIPCHK(c, hipMemcpyAsync(counts, c->ncand.p, (size_t)c->Q * 4, hipMemcpyDeviceToDevice, c->stream));
    if (c->stage > 1) c->stage = 1;
    return ZH_OK;
}

zh_status zh_candidates_t(zh_ctx* c, int t, int32_t cap_per_query, int32_t* counts, int32_t* ids) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_candidates_t before zh_query");
    Dict& d = c->dicts[c->qscale];
    if (t < 1 || t > d.L || cap_per_query < 1 || !counts || !ids)
        return fail(c, ZH_EINVAL, "zh_candidates_t: need 1 <= t <= L = %d, cap_per_query >= 1", d.L);
    TRY(set_device(c));
    HIPCHK(c, launch_cand_t((int)c->Q, d.L, d.n, t, P<uint2>(c->qbins), P<uint32_t>(d.tids), cap_per_query, counts,
                            ids, c->stream));
    return ZH_OK;
}

zh_status zh_knn_t(zh_ctx* c, int t) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_knn_t before zh_query");
    Dict& d = c->dicts[c->qscale];
    if (t < 1 || t > d.L) return fail(c, ZH_EINVAL, "zh_knn_t: need 1 <= t <= L = %d", d.L);
    TRY(set_device(c));
    {
        StageTimer tm(c, ZH_T_SEARCH);
        HIPCHK(c, launch_knn_tofl((int)c->Q, d.L, d.n, t, d.D, c->qK, P<uint2>(c->qbins), P<uint32_t>(d.tids),
                                  P<float>(c->qfeat), P<float>(d.xf), P<int32_t>(c->ncand), P<int32_t>(c->ids),
                                  P<float>(c->d2), P<int32_t>(c->m), c->stream));
    }
    c->gram_ready = false;   // the Gram matrices of the new neighbours are formed by zh_lle_weights
    c->stage = 1;
    return ZH_OK;
}

zh_status zh_knn_l1(zh_ctx* c) {
    if (!c) return ZH_EINVAL;
    if (c->stage < 1) return fail(c, ZH_ESTATE, "zh_knn_l1 before zh_query");
    if (c->opts.cap < 1) return fail(c, ZH_EUNSUPPORTED, "zh_knn_l1 needs the early stop (query option cap > 0)");
    TRY(set_device(c));
    TRY(clear_counters(c));
    TRY(rank_l1(c, c->dicts[c->qscale]));
    c->gram_ready = false;   // the Gram matrices of the new neighbours are formed by zh_lle_weights
    c->stage = 1;
    return ZH_OK;
}

zh_status zh_stats(zh_ctx* c, zh_stats_t* out) {
    if (!c) return ZH_EINVAL;
    if (!out) return fail(c, ZH_EINVAL, "zh_stats: null output");
    TRY(set_device(c));
    std::memset(out, 0, sizeof(*out));
    uint32_t h[kNumCounters] = {0};
    if (c->counters.p) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipMemcpy(h, c->counters.p, sizeof(h), hipMemcpyDeviceToHost));
    }
    out->queries = (uint64_t)c->Q;
    out->codes_fixed = h[C_CODEFIX];
    out->rank_fallbacks = h[C_RANKFB];
    out->deferred = h[C_OVERFLOW];
    out->streamed = h[C_STREAM];
    out->lle_fp64 = h[C_LLE64];
    out->truncated = h[C_TRUNC];
    uint64_t db = 0;
    for (const Dict& d : c->dicts)
        db += d.hi.bytes + d.lo.bytes + d.dir.bytes + d.dfilt.bytes + d.tids.bytes + d.alpha.bytes + d.ahi.bytes + d.alo.bytes +
              d.l1s.bytes;
    out->dict_bytes = db;
    return ZH_OK;
}

zh_status zh_set_timing(zh_ctx* c, int on) {
    if (!c) return ZH_EINVAL;
    c->timing = on != 0;
    c->timing_mask = ~0u;
    return ZH_OK;
}

zh_status zh_set_timing_stages(zh_ctx* c, uint32_t mask) {
    if (!c) return ZH_EINVAL;
    c->timing = mask != 0;
    c->timing_mask = mask;
    return ZH_OK;
}

zh_status zh_get_timing(zh_ctx* c, double* ms, int32_t* launches) {
    if (!c) return ZH_EINVAL;
    if (!ms) return fail(c, ZH_EINVAL, "zh_get_timing: null output");
    TRY(set_device(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int st = 0; st < ZH_T_COUNT; ++st) {
        double sum = 0.0;
        for (int i = 0; i < c->nev[st]; ++i) {
            float t = 0.f;
            HIPCHK(c, hipEventElapsedTime(&t, c->ev[st][i][0], c->ev[st][i][1]));
            sum += t;
        }
        ms[st] = sum;
        if (launches) launches[st] = c->nev[st];
        c->nev[st] = 0;
    }
    return ZH_OK;
}

}  // extern "C"
