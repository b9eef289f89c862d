// Candidate search for every LR patch (Section 3.2, Section 4.2):
// given the patch's bin in each of the L tables, collect the union of the
// IDs found (t = 1), optionally with the early stop of Section 4.2 (tables in
// order, IDs ascending inside a bin, stop at `cap` distinct IDs), then keep
// the K nearest by squared l2 distance, ties broken by the lower ID.
//
// One wave per patch. Dictionary features are stored as two 16-bit planes of
// the fp32 value (bf16 high half, low half). Exact mode: every candidate's
// distance is computed in fp32 from both planes; a forward error bound on
// each fp32 distance certifies the selected set and its order against the
// FP64 sequential distance, and when it cannot, the ambiguous candidates are
// re-ranked by that FP64 distance, so the result equals the FP64 definition.
// Screened mode (rerank = R): the high plane alone (a bf16 feature) ranks the
// candidates, the best R are re-ranked exactly in fp32.
#include <type_traits>

#include "zh_internal.h"

namespace zh {

// candidate ordering key: distance bits, then a "not exactly equal" bit, then
// the ID (IDs < 2^31). Exactly equal rows have distance 0 in every precision.
__device__ __forceinline__ uint64_t cand_key(uint32_t dbits, uint32_t id) {
    return ((uint64_t)(dbits & 0x7FFFFFFFu) << 32) | ((uint64_t)(dbits >> 31 ^ 1u) << 31) | id;
}
__device__ __forceinline__ bool key_exact(uint64_t key) { return ((key >> 31) & 1u) == 0; }
__device__ __forceinline__ uint32_t key_id(uint64_t key) { return (uint32_t)(key & 0x7FFFFFFFu); }
__device__ __forceinline__ float key_dist(uint64_t key) { return __uint_as_float((uint32_t)(key >> 32)); }

// Bitonic sort of s[0..n) ascending by one wave (n padded to a power of two
// with 0xFFFFFFFF; s must have room for the padding).
__device__ void wave_sort_u32(uint32_t* s, int n) {
    const int lane = threadIdx.x;
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    for (int i = n + lane; i < p2; i += 64) s[i] = 0xFFFFFFFFu;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < p2; i += 64) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint32_t x = s[i], y = s[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        s[i] = y;
                        s[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Bitonic sort of NS*64 keys held NS per lane (element s*64 + lane) in
// registers, ascending.
template <int NS>
__device__ __forceinline__ void wave_sort_keys(uint64_t (&key)[NS]) {
    const int lane = threadIdx.x & 63;
    constexpr int N = NS * 64;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                const int js = j >> 6;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int t = s ^ js;
                    if (t > s) {
                        const bool up = ((s * 64 + lane) & k) == 0;
                        const uint64_t x = key[s], y = key[t];
                        if ((x > y) == up) {
                            key[s] = y;
                            key[t] = x;
                        }
                    }
                }
            } else {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const uint64_t x = key[s];
                    const uint64_t y = __shfl_xor(x, j);
                    const bool up = ((s * 64 + lane) & k) == 0;
                    const bool lower = (lane & j) == 0;
                    const uint64_t mn = x < y ? x : y, mx = x < y ? y : x;
                    key[s] = (lower == up) ? mn : mx;
                }
            }
        }
    }
}

// Squared distances of the query to candidates cids[0..c1) into cdist[c]
// (fp32 bits; bit 31 set when the row equals the query exactly). Half a wave
// per row: lane l of a half holds coordinates [VEC l, VEC l + VEC); U row
// pairs are loaded before any is used.
template <int VEC, bool HI_ONLY>
__device__ void cand_distances(const float (&qv)[VEC], int D, const uint16_t* __restrict__ hi,
                               const uint16_t* __restrict__ lo, const uint32_t* cids, uint32_t* cdist,
                               int c1) {
    // VEC == 4: 8 bytes of each plane per lane; VEC == 1: 2 bytes
    typedef typename std::conditional<VEC == 4, uint2, uint32_t>::type raw_t;
    const int lane = threadIdx.x, hl = lane & 31, half = lane >> 5;
    const bool dl = hl * VEC < D;
    constexpr int U = HI_ONLY ? 16 : 8;
    for (int cb = 0; cb < c1; cb += 2 * U) {
        raw_t hr[U], lr[U];
        bool cv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = cb + 2 * u + half;
            cv[u] = c < c1;
            const uint32_t id = cv[u] ? cids[c] : 0u;
            // N * D < 2^31 elements: 32-bit offsets from the plane bases
            const uint32_t base = id * (uint32_t)D + (uint32_t)(hl * VEC);
            hr[u] = raw_t{};
            lr[u] = raw_t{};
            if (cv[u] && dl) {
                const uint32_t bo = base * 2u;  // byte offset, < 2^32
                if constexpr (VEC == 4) {
                    hr[u] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(hi) + bo);
                    if (!HI_ONLY) lr[u] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(lo) + bo);
                } else {
                    hr[u] = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(hi) + bo);
                    if (!HI_ONLY) lr[u] = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(lo) + bo);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t hv[VEC], lv[VEC];
            if constexpr (VEC == 4) {
                hv[0] = hr[u].x & 0xFFFFu; hv[1] = hr[u].x >> 16; hv[2] = hr[u].y & 0xFFFFu; hv[3] = hr[u].y >> 16;
                lv[0] = lr[u].x & 0xFFFFu; lv[1] = lr[u].x >> 16; lv[2] = lr[u].y & 0xFFFFu; lv[3] = lr[u].y >> 16;
            } else {
                hv[0] = hr[u];
                lv[0] = lr[u];
            }
            float p = 0.0f;
            bool eq = true;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float y = __uint_as_float((hv[e] << 16) | lv[e]);
                const float d = qv[e] - y;
                p = fmaf(d, d, p);
                eq = eq && (!dl || __float_as_uint(qv[e]) == __float_as_uint(y));
            }
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) p += __shfl_xor(p, o);
            const uint64_t em = __ballot(eq);
            const uint32_t hm = (uint32_t)(em >> (32 * half));
            const int c = cb + 2 * u + half;
            if (hl == 0 && cv[u]) cdist[c] = __float_as_uint(p) | (hm == 0xFFFFFFFFu ? 0x80000000u : 0u);
        }
    }
    __syncthreads();
}

// K' rounds of wave argmin over the candidates' keys; lane r receives the
// r-th smallest key. (Used when the candidates exceed the register sort.)
__device__ uint64_t select_topk(const uint32_t* cids, const uint32_t* cdist, int M, int Kp) {
    const int lane = threadIdx.x;
    uint64_t mine = ~0ull, last = 0;
    for (int r = 0; r < Kp; ++r) {
        uint64_t best = ~0ull;
        for (int c = lane; c < M; c += 64) {
            const uint64_t key = cand_key(cdist[c], cids[c]);
            if ((r == 0 || key > last) && key < best) best = key;
        }
        best = wave_min_u64(best);
        if (lane == r) mine = best;
        last = best;
    }
    return mine;
}

// Sorted selection for M <= 256 candidates: lane r < min(M, 64) receives the
// r-th smallest key.
__device__ uint64_t sort_select(const uint32_t* cids, const uint32_t* cdist, int M) {
    const int lane = threadIdx.x;
    if (M <= 64) {
        uint64_t k[1] = {lane < M ? cand_key(cdist[lane], cids[lane]) : ~0ull};
        wave_sort_keys<1>(k);
        return k[0];
    }
    if (M <= 128) {
        uint64_t k[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c = s * 64 + lane;
            k[s] = c < M ? cand_key(cdist[c], cids[c]) : ~0ull;
        }
        wave_sort_keys<2>(k);
        return k[0];
    }
    uint64_t k[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = s * 64 + lane;
        k[s] = c < M ? cand_key(cdist[c], cids[c]) : ~0ull;
    }
    wave_sort_keys<4>(k);
    return k[0];
}

// FP64 sequential squared distance: the definition.
__device__ double exact_dist64(const float* __restrict__ qrow, int D, const uint16_t* __restrict__ hi,
                               const uint16_t* __restrict__ lo, uint32_t id) {
    const int64_t b = (int64_t)id * D;
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
        const double d = (double)qrow[i] - (double)join_planes(hi[b + i], lo[b + i]);
        s = s + d * d;
    }
    return s;
}

struct Bounds {
    double eps, abs_;
};

__device__ __forceinline__ void dist_interval(uint32_t dbits, const Bounds& bd, double& lo, double& hi) {
    if (dbits & 0x80000000u) { lo = 0.0; hi = 0.0; return; }
    const double d = (double)__uint_as_float(dbits);
    hi = d * (1.0 + bd.eps) + bd.abs_;
    lo = d * (1.0 - bd.eps) - bd.abs_;
    if (lo < 0.0) lo = 0.0;
}

// Certify the fp32 selection; on failure re-rank the ambiguous candidates by
// the FP64 distance. Lane r < Kp holds the r-th key on entry; on exit lane r
// holds (id, d2) of the r-th neighbour of the exact ranking.
__device__ void certify_or_fix(const SearchArgs& a, int q, const uint32_t* cids, const uint32_t* cdist,
                               int M, int Kp, uint64_t mykey, uint32_t& out_id, float& out_d) {
    const int lane = threadIdx.x;
    const Bounds bd{2.0 * gamma_n(a.D + 3, 1.0 / 16777216.0), (double)a.D * 1.2e-38};
    const bool ex = key_exact(mykey);
    double lo, hi;
    dist_interval(ex ? 0x80000000u : (uint32_t)(mykey >> 32), bd, lo, hi);
    const bool ex_n = __shfl_down(ex ? 1 : 0, 1) != 0;
    const double lo_n = __shfl_down(lo, 1);
    bool ok = true;
    if (lane + 1 < Kp) {
        if (!ex && ex_n) ok = false;
        else if (!ex && !ex_n) ok = hi < lo_n;
    }
    bool certified = __ballot(!ok) == 0;
    const uint64_t lastkey = __shfl(mykey, Kp - 1);
    const bool last_ex = key_exact(lastkey);
    double tlo, thi;
    dist_interval(last_ex ? 0x80000000u : (uint32_t)(lastkey >> 32), bd, tlo, thi);
    if (certified && Kp < M && !last_ex) {
        int cnt = 0;
        for (int c = lane; c < M; c += 64) {
            const uint32_t db = cdist[c];
            if (db & 0x80000000u) continue;
            double l2, h2;
            dist_interval(db, bd, l2, h2);
            if (l2 <= thi) ++cnt;
        }
        cnt = wave_sum_i32(cnt);
        const int nsel_nonex = __popcll(__ballot(lane < Kp && !ex));
        certified = cnt == nsel_nonex;
    }
    if (certified) {
        out_id = key_id(mykey);
        out_d = key_dist(mykey);
        return;
    }
    if (lane == 0) atomicAdd(&a.counters[1], 1u);
    const float* qrow = a.qfeat + (int64_t)q * a.D;
    const bool bounded = Kp < M && !last_ex;
    double lastd = 0.0;
    uint32_t lastid = 0;
    for (int r = 0; r < Kp; ++r) {
        double bestd = 1.0e300;
        uint32_t bestid = 0xFFFFFFFFu;
        for (int c = lane; c < M; c += 64) {
            const uint32_t db = cdist[c];
            const bool cex = (db & 0x80000000u) != 0;
            if (bounded && !cex) {
                double l2, h2;
                dist_interval(db, bd, l2, h2);
                if (l2 > thi) continue;
            }
            const uint32_t id = cids[c];
            const double d = cex ? 0.0 : exact_dist64(qrow, a.D, a.hi, a.lo, id);
            const bool after = r == 0 || d > lastd || (d == lastd && id > lastid);
            if (after && (d < bestd || (d == bestd && id < bestid))) {
                bestd = d;
                bestid = id;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(bestd, o);
            const uint32_t oi = __shfl_xor(bestid, o);
            if (od < bestd || (od == bestd && oi < bestid)) {
                bestd = od;
                bestid = oi;
            }
        }
        if (lane == r) {
            out_id = bestid;
            out_d = (float)bestd;
        }
        lastd = bestd;
        lastid = bestid;
    }
}

__device__ __forceinline__ void write_result(const SearchArgs& a, int q, int Kp, uint32_t oid, float od) {
    const int lane = threadIdx.x;
    if (lane < a.K) {
        a.out_ids[(int64_t)q * a.K + lane] = lane < Kp ? (int32_t)oid : -1;
        a.out_d2[(int64_t)q * a.K + lane] = lane < Kp ? od : 0.0f;
    }
    if (lane == 0) a.out_m[q] = Kp;
}

template <int VEC>
__device__ __forceinline__ void load_query(const SearchArgs& a, int q, float (&qv)[VEC]) {
    const int hl = threadIdx.x & 31;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        qv[e] = (hl * VEC + e < a.D) ? a.qfeat[(int64_t)q * a.D + hl * VEC + e] : 0.0f;
}

// Early-stop search (cap <= 256): the concatenation of the L bins is read in
// parallel 128 positions at a time; first occurrences are kept in order.
template <int VEC, bool EXACT>
__global__ __launch_bounds__(64) void k_search_cap(SearchArgs a) {
    __shared__ uint32_t cids[256];
    __shared__ uint32_t cdist[256];
    __shared__ uint32_t chunk[64];
    __shared__ uint32_t sstart[kMaxL + 1];
    __shared__ uint32_t soff[kMaxL];
    const int lane = threadIdx.x;
    const int L = a.L;

    for (int q = blockIdx.x; q < a.Q; q += gridDim.x) {
        uint32_t off = 0, cnt = 0;
        if (lane < L) {
            const uint2 b = a.bins[(int64_t)q * L + lane];
            off = b.x;
            cnt = b.y;
        }
        const int T = wave_sum_i32((int)cnt);
        const int incl = wave_incl_scan((int)cnt);
        if (lane < L) {
            sstart[lane] = (uint32_t)(incl - (int)cnt);
            soff[lane] = off;
        }
        if (lane == 0) sstart[L] = (uint32_t)T;
        __syncthreads();
        int M = 0;
        for (int base = 0; base < T && M < a.cap; base += 128) {
            uint32_t idv[2];
            int tabv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int i = base + 64 * u + lane;
                idv[u] = 0xFFFFFFFFu;
                tabv[u] = -1;
                if (i < T) {
                    int lo = 0, hi = L;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (sstart[mid] <= (uint32_t)i) lo = mid; else hi = mid;
                    }
                    tabv[u] = lo;
                    idv[u] = a.tids[(int64_t)lo * a.N + soff[lo] + (i - sstart[lo])];
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int cb = base + 64 * u;
                if (cb >= T || M >= a.cap) break;
                const bool valid = cb + lane < T;
                const uint32_t id = idv[u];
                bool dup = false;
                for (int i = 0; i < M; ++i) dup |= cids[i] == id;
                // IDs inside one bin are distinct: only a chunk that spans
                // several tables can repeat an ID within itself
                const int tfirst = __shfl(tabv[u], 0);
                const int tlast = __shfl(tabv[u], min(63, T - 1 - cb));
                if (tfirst != tlast) {
                    chunk[lane] = id;
                    __syncthreads();
                    for (int j = 0; j < 64; ++j) dup |= (j < lane) && chunk[j] == id;
                }
                const bool nw = valid && !dup;
                const uint64_t bal = __ballot(nw);
                const int rank = __popcll(bal & lanemask_lt());
                if (nw && M + rank < a.cap) cids[M + rank] = id;
                M = min(a.cap, M + (int)__popcll(bal));
                __syncthreads();
            }
        }
        if (a.dump) {
            wave_sort_u32(cids, M);
            for (int i = lane; i < M && i < a.dump_cap; i += 64) a.dump[(int64_t)q * a.dump_cap + i] = (int32_t)cids[i];
        }
        if (lane == 0) a.out_ncand[q] = M;
        float qv[VEC];
        load_query<VEC>(a, q, qv);
        int Mr = M;
        if (!EXACT && M > a.rerank) {
            cand_distances<VEC, true>(qv, a.D, a.hi, a.lo, cids, cdist, M);
            const uint64_t k2 = sort_select(cids, cdist, M);
            __syncthreads();
            if (lane < a.rerank) cids[lane] = key_id(k2);
            __syncthreads();
            Mr = a.rerank;
        }
        cand_distances<VEC, false>(qv, a.D, a.hi, a.lo, cids, cdist, Mr);
        const int Kp = min(a.K, Mr);
        const uint64_t mykey = sort_select(cids, cdist, Mr);
        uint32_t oid = 0xFFFFFFFFu;
        float od = 0.0f;
        if (EXACT && Kp > 0) {
            certify_or_fix(a, q, cids, cdist, Mr, Kp, mykey, oid, od);
        } else if (lane < Kp) {
            oid = key_id(mykey);
            od = key_dist(mykey);
        }
        write_result(a, q, Kp, oid, od);
        __syncthreads();
    }
}

// Union search without early stop: all IDs of the L bins are gathered,
// sorted and deduplicated in LDS (T <= CMAX), else the patch is deferred.
template <int VEC, int CMAX, bool BIG>
__global__ __launch_bounds__(64) void k_search_union(SearchArgs a) {
    __shared__ uint32_t cids[CMAX];
    __shared__ uint32_t cdist[CMAX];
    __shared__ uint32_t sstart[kMaxL + 1];
    __shared__ uint32_t soff[kMaxL];
    const int lane = threadIdx.x;
    const int L = a.L;
    const int nq = BIG ? (int)a.counters[0] : a.Q;

    for (int t = blockIdx.x; t < nq; t += gridDim.x) {
        const int q = BIG ? a.overflow[t] : t;
        uint32_t off = 0, cnt = 0;
        if (lane < L) {
            const uint2 b = a.bins[(int64_t)q * L + lane];
            off = b.x;
            cnt = b.y;
        }
        const int T = wave_sum_i32((int)cnt);
        if (T > CMAX) {
            if (!BIG) {
                if (lane == 0) {
                    const unsigned int pos = atomicAdd(&a.counters[0], 1u);
                    a.overflow[pos] = q;
                }
            } else {
                if (lane == 0) {
                    a.out_m[q] = -1;
                    a.out_ncand[q] = T;
                    atomicAdd(&a.counters[2], 1u);
                }
                if (lane < a.K) a.out_ids[(int64_t)q * a.K + lane] = -1;
            }
            continue;
        }
        const int incl = wave_incl_scan((int)cnt);
        if (lane < L) {
            sstart[lane] = (uint32_t)(incl - (int)cnt);
            soff[lane] = off;
        }
        if (lane == 0) sstart[L] = (uint32_t)T;
        __syncthreads();
        for (int i = lane; i < T; i += 64) {
            int lo = 0, hi = L;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sstart[mid] <= (uint32_t)i) lo = mid; else hi = mid;
            }
            cids[i] = a.tids[(int64_t)lo * a.N + soff[lo] + (i - sstart[lo])];
        }
        __syncthreads();
        if (T > 0) wave_sort_u32(cids, T);
        int M = 0;
        for (int b = 0; b < T; b += 64) {
            const int i = b + lane;
            const bool valid = i < T;
            const uint32_t v = valid ? cids[i] : 0u;
            const uint32_t prev = (valid && i > 0) ? cids[i - 1] : 0xFFFFFFFFu;
            __syncthreads();
            const bool keep = valid && (i == 0 || v != prev);
            const uint64_t bal = __ballot(keep);
            if (keep) cids[M + __popcll(bal & lanemask_lt())] = v;
            M += __popcll(bal);
            __syncthreads();
        }
        if (a.dump) {
            for (int i = lane; i < M && i < a.dump_cap; i += 64) a.dump[(int64_t)q * a.dump_cap + i] = (int32_t)cids[i];
        }
        if (lane == 0) a.out_ncand[q] = M;
        float qv[VEC];
        load_query<VEC>(a, q, qv);
        int Mr = M;
        if (a.rerank > 0 && M > a.rerank) {
            cand_distances<VEC, true>(qv, a.D, a.hi, a.lo, cids, cdist, M);
            const uint64_t k2 = M <= 256 ? sort_select(cids, cdist, M) : select_topk(cids, cdist, M, a.rerank);
            __syncthreads();
            if (lane < a.rerank) cids[lane] = key_id(k2);
            __syncthreads();
            Mr = a.rerank;
        }
        cand_distances<VEC, false>(qv, a.D, a.hi, a.lo, cids, cdist, Mr);
        const int Kp = min(a.K, Mr);
        const uint64_t mykey = Mr <= 256 ? sort_select(cids, cdist, Mr) : select_topk(cids, cdist, Mr, Kp);
        uint32_t oid = 0xFFFFFFFFu;
        float od = 0.0f;
        if (a.exact && Kp > 0) {
            certify_or_fix(a, q, cids, cdist, Mr, Kp, mykey, oid, od);
        } else if (lane < Kp) {
            oid = key_id(mykey);
            od = key_dist(mykey);
        }
        write_result(a, q, Kp, oid, od);
        __syncthreads();
    }
}

constexpr int kCapMax = 256;      // early-stop limit a wave can hold
constexpr int kUnionMax = 2048;   // uncapped: IDs per wave before deferring
constexpr int kUnionBig = 8192;   // uncapped, deferred patches

template <int VEC>
static void launch_search_t(const SearchArgs& a, int grid, hipStream_t st) {
    if (a.cap > 0) {
        if (a.exact) hipLaunchKernelGGL((k_search_cap<VEC, true>), dim3(grid), dim3(64), 0, st, a);
        else hipLaunchKernelGGL((k_search_cap<VEC, false>), dim3(grid), dim3(64), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_search_union<VEC, kUnionMax, false>), dim3(grid), dim3(64), 0, st, a);
    }
}

hipError_t launch_search(const SearchArgs& a, hipStream_t st) {
    if (a.Q == 0) return hipSuccess;
    const int grid = a.Q < 32768 ? a.Q : 32768;
    const bool v4 = a.D % 4 == 0 && a.D <= 128;
    if (!v4 && a.D > 32) return hipErrorInvalidValue;
    if (a.cap > kCapMax) return hipErrorInvalidValue;
    if (!a.exact && (a.rerank < 1 || a.rerank > 64)) return hipErrorInvalidValue;
    if (v4) launch_search_t<4>(a, grid, st);
    else launch_search_t<1>(a, grid, st);
    return hipGetLastError();
}

hipError_t launch_search_overflow(const SearchArgs& a, int grid, hipStream_t st) {
    const bool v4 = a.D % 4 == 0 && a.D <= 128;
    if (v4) hipLaunchKernelGGL((k_search_union<4, kUnionBig, true>), dim3(grid), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_search_union<1, kUnionBig, true>), dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace zh
