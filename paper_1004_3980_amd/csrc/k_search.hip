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
// Screened mode (rerank = R): with the early stop, lower bounds from int8
// coordinates in the dictionary's principal directions rule candidates out and
// at most R of the others get exact fp32 distances (patches where more than R
// survive are counted); without it, a distance on the high plane alone (a
// bf16 feature) ranks the candidates and the best R are re-ranked in fp32.
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
// registers, ascending. With NS == 1 and N < 64, each aligned group of N lanes
// is sorted on its own: ascending where (lane & N) == 0, descending in the
// other groups.
template <int NS, int N = NS * 64>
__device__ __forceinline__ void wave_sort_keys(uint64_t (&key)[NS]) {
    const int lane = threadIdx.x & 63;
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
__device__ void cand_distances(const float (&qv)[VEC], int D, int HS, const uint16_t* __restrict__ hi,
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
            const uint32_t hbase = id * (uint32_t)HS + (uint32_t)(hl * VEC);
            hr[u] = raw_t{};
            lr[u] = raw_t{};
            if (cv[u] && dl) {
                const uint32_t bo = base * 2u, bh = hbase * 2u;  // byte offsets, < 2^32
                if constexpr (VEC == 4) {
                    hr[u] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(hi) + bh);
                    if (!HI_ONLY) lr[u] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(lo) + bo);
                } else {
                    hr[u] = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(hi) + bh);
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

// Sorted selection for M <= 64 NSL candidates: lane r < min(M, 64) receives
// the r-th smallest key. Up to 16 candidates: each lane counts the keys below
// its own (the keys are distinct: they carry the ID) and places its key at
// that rank in `rk` (16 slots of LDS).
// slot (optional): on the ranking path, lane r < M also receives the
// candidate index (into cids) of its key; elsewhere -1.
template <int NSL = 4>
__device__ __forceinline__ uint64_t sort_select(const uint32_t* cids, const uint32_t* cdist, int M,
                                                uint64_t* rk = nullptr, int* slot = nullptr) {
    const int lane = threadIdx.x;
    if (slot) *slot = -1;
    if (rk && M <= 16) {
        const uint64_t mine = lane < M ? cand_key(cdist[lane], cids[lane]) : ~0ull;
        const uint32_t mlo = (uint32_t)mine, mhi = (uint32_t)(mine >> 32);
        int rank = 0;
        for (int c = 0; c < M; ++c) {
            const uint32_t lo = __builtin_amdgcn_readlane(mlo, c), hi = __builtin_amdgcn_readlane(mhi, c);
            rank += ((((uint64_t)hi << 32) | lo) < mine) ? 1 : 0;
        }
        // rk[0..16): the keys by rank; the candidate index of each in the
        // upper half of its slot's neighbour (rk + 16)
        if (lane < M) {
            rk[rank] = mine;
            if (slot) reinterpret_cast<int*>(rk + 16)[rank] = lane;
        }
        __syncthreads();
        const uint64_t out = lane < M ? rk[lane] : ~0ull;
        if (slot && lane < M) *slot = reinterpret_cast<const int*>(rk + 16)[lane];
        __syncthreads();
        return out;
    }
    if (M <= 64) {
        uint64_t k[1] = {lane < M ? cand_key(cdist[lane], cids[lane]) : ~0ull};
        if (M <= 16)
            wave_sort_keys<1, 16>(k);
        else if (M <= 32)
            wave_sort_keys<1, 32>(k);
        else
            wave_sort_keys<1>(k);
        return k[0];
    }
    if (NSL <= 2 || M <= 128) {
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
__device__ double exact_dist64(const float* __restrict__ qrow, int D, int HS, const uint16_t* __restrict__ hi,
                               const uint16_t* __restrict__ lo, uint32_t id) {
    const int64_t b = (int64_t)id * D, bh = (int64_t)id * HS;
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
        const double d = (double)qrow[i] - (double)join_planes(hi[bh + i], lo[b + i]);
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
    const Bounds bd{a.dist_eps, (double)a.D * 1.2e-38};
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
    if (lane == 0) atomicAdd(&a.counters[C_RANKFB], 1u);
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
            const double d = cex ? 0.0 : exact_dist64(qrow, a.D, a.hs, a.hi, a.lo, id);
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

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// order-preserving map of a finite float to uint32
__device__ __forceinline__ uint32_t ord_u32(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
// 16 bytes from an 8-byte aligned address
__device__ __forceinline__ uint4 ld16(const char* p) {
    const uint2 x = *reinterpret_cast<const uint2*>(p);
    const uint2 y = *reinterpret_cast<const uint2*>(p + 8);
    return make_uint4(x.x, x.y, y.x, y.y);
}

// R-th smallest (R >= 1) of the M keys held NSL per lane (element s*64 + lane):
// a 32-step radix search with wave ballots.
template <int NSL>
__device__ uint32_t radix_kth(const uint32_t (&kv)[NSL], int M, int R) {
    // keys past M are 0xFFFFFFFF, which no trial value exceeds
    (void)M;
    uint32_t tau = 0;
    for (int b = 31; b >= 0; --b) {
        const uint32_t trial = tau + (1u << b);
        int n = 0;
#pragma unroll
        for (int s = 0; s < NSL; ++s) n += __popcll(__ballot(kv[s] < trial));
        if (n < R) tau = trial;
    }
    return tau;
}

// Marks n (1 <= n <= number of keys below 0xFFFFFFFF) of the keys held NSL per
// lane that are among the smallest up to the top 16 bits: all keys whose top
// 16 bits lie below the n-th smallest key's, and the rest from those equal to
// it in that prefix, in slot order.
template <int NSL>
__device__ void mark_lowest16(const uint32_t (&kv)[NSL], int n, bool (&keep)[NSL]) {
    uint32_t k16[NSL];
#pragma unroll
    for (int s = 0; s < NSL; ++s) k16[s] = kv[s] >> 16;
    uint32_t hk = 0;
    for (int b = 15; b >= 0; --b) {
        const uint32_t trial = hk | (1u << b);
        int c = 0;
#pragma unroll
        for (int s = 0; s < NSL; ++s) c += __popcll(__ballot(k16[s] < trial));
        if (c < n) hk = trial;
    }
    int nlt = 0;
#pragma unroll
    for (int s = 0; s < NSL; ++s) nlt += __popcll(__ballot(k16[s] < hk));
    int need = n - nlt;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        const uint64_t eq = __ballot(k16[s] == hk);
        const int rank = __popcll(eq & lanemask_lt());
        keep[s] = k16[s] < hk || (k16[s] == hk && rank < need);
        need -= __popcll(eq);
    }
}

// Relative error coefficient c of the screen value a2 = |y^|^2 + |y~|^2 -
// 2 y^.y~ against |y^ - y~|^2, y^ = s_q (h + l / 128) the coded query and
// y~ = s_x c the screen row: the error is at most c (|y^|^2 + |y~|^2). The
// integer products h.c and l.c are exact; the terms are the fp32 roundings
// of |y^|^2 and |y~|^2 (u each), of (128 h.c + l.c) / 128 and its two scale
// factors (3 u of |y^.y~| <= (|y^|^2 + |y~|^2) / 2, doubled in a2), of the sum
// |y^|^2 + |y~|^2 (u) and of the difference (u |a2| <= 2 u (|y^|^2 + |y~|^2)):
// 7 u in all, doubled, rounded up to 16 u.
float screen_coeff() { return (float)(16.0 / 16777216.0); }

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Gram matrix G[i][j] = sum_c z_i[c] z_j[c] of the eight rows of one exact
// pass (lane = 8 row + group g, z = the lane's 16 coordinates 16 g + e), on
// the matrix cores: 16 steps of a 16x16x4 product whose operand rows 0..7
// carry the eight rows' first 64 coordinates and rows 8..15 their last 64,
// each value fetched from the lane that holds it; A and B are the same
// register, and the two diagonal 8x8 blocks of the product add up to G.
// Writes sG[8][8].
template <typename T>
__device__ __forceinline__ void gram_mfma(const T (&z)[16], T* sG) {
    const int lane = threadIdx.x;
    const int col = lane & 15, kk = lane >> 4;
    // operand lane (row r = l % 16, k = l / 16) of step t: coordinate 16 g + t
    // of neighbour r % 8, with g = 4 (r / 8) + k: rows 0..7 take the first 64
    // coordinates, rows 8..15 the last 64
    const int src = (col & 7) * 8 + 4 * (col >> 3) + kk;
    typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type acc = {};
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const T v = __shfl(z[t], src);
        if constexpr (sizeof(T) == 4)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v, v, acc, 0, 0, 0);
        else
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
    }
    // G = C[0..7][0..7] + C[8..15][8..15] (the other quadrants mix the halves)
    if constexpr (sizeof(T) == 4) {
        // fp32: lane l holds C[4 (l / 16) + i][l % 16]
        T o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = __shfl(acc[i], (lane + 40) & 63);
        if (kk < 2 && col < 8) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sG[(4 * kk + i) * 8 + col] = acc[i] + o[i];
        }
    } else {
        // FP64: lane l holds C[4 i + l / 16][l % 16]
        T o[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) o[i] = __shfl(acc[i + 2], (lane + 8) & 63);
        if (col < 8) {
#pragma unroll
            for (int i = 0; i < 2; ++i) sG[(4 * i + kk) * 8 + col] = acc[i] + o[i];
        }
    }
}

// Exact fp32 distances |q - x|^2 of the candidates cids[cb..min(cb+8, c1))
// from both planes, eight lanes per row (16 coordinates each), into cdist; a
// row whose fp32 distance is 0 is checked for exact equality with the query
// (flag bit). GT float or double: also the Gram matrix of the pass's rows in
// that precision, into sG[8][8] (rows past c1 zero); GT int: none.
template <typename GT>
__device__ __forceinline__ void exact_pass(const SearchArgs& a, const float* sq, const uint32_t* cids,
                                           uint32_t* cdist, int cb, int c1, GT* sG) {
    const int lane = threadIdx.x;
    const int D = a.D;
    const int rg = lane >> 3, g = lane & 7;
    const int c = cb + rg;
    const bool cv = c < c1;
    const uint32_t id = cv ? cids[c] : 0u;
    // the row's fp32 values 16 g .. 16 g + 15 (zero past D)
    const float* xr = a.xf + (size_t)id * (uint32_t)D;
    float x[16];
    if ((D & 3) == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c0 = 16 * g + 4 * u;
            float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
            if (cv && c0 < D) t = *reinterpret_cast<const float4*>(xr + c0);
            x[4 * u] = t.x;
            x[4 * u + 1] = t.y;
            x[4 * u + 2] = t.z;
            x[4 * u + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = (cv && 16 * g + e < D) ? xr[16 * g + e] : 0.0f;
    }
    float z[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) z[e] = sq[16 * g + e] - x[e];
    float p = 0.0f;
#pragma unroll
    for (int e = 0; e < 16; ++e) p = fmaf(z[e], z[e], p);
    p += __shfl_xor(p, 1);
    p += __shfl_xor(p, 2);
    p += __shfl_xor(p, 4);
    bool exact_row = false;
    if (__ballot(cv && p == 0.0f) != 0) {
        bool eq = true;
#pragma unroll
        for (int e = 0; e < 16; ++e) eq = eq && __float_as_uint(x[e]) == __float_as_uint(sq[16 * g + e]);
        const uint32_t grp = (uint32_t)(__ballot(eq) >> (8 * rg)) & 0xFFu;
        exact_row = grp == 0xFFu;
    }
    if (g == 0 && cv) cdist[c] = __float_as_uint(p) | (exact_row ? 0x80000000u : 0u);
    if constexpr (std::is_same<GT, float>::value) {
#pragma unroll
        for (int e = 0; e < 16; ++e) z[e] = cv ? z[e] : 0.0f;
        gram_mfma<float>(z, sG);
    } else if constexpr (std::is_same<GT, double>::value) {
        // exact differences: q - x in FP64 from the fp32 values
        double zd[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) zd[e] = cv ? (double)sq[16 * g + e] - (double)x[e] : 0.0;
        gram_mfma<double>(zd, sG);
    }
}

__device__ __forceinline__ void exact_rows(const SearchArgs& a, const float* sq, const uint32_t* cids,
                                           uint32_t* cdist, int c0, int c1) {
    for (int cb = c0; cb < c1; cb += 8) exact_pass<int>(a, sq, cids, cdist, cb, c1, nullptr);
}

// Packed lower triangle (p = i (i + 1) / 2 + j, 36 entries) of the Gram
// matrix of the Kp final neighbours into gram[q]: lane r < Kp holds the r-th
// neighbour's id. When every neighbour is one of the nA rows whose Gram
// matrix sG was formed in the first exact pass (cids[0..nA)), the entries are
// taken from it; otherwise the rows of the neighbours are read again.
template <typename GT>
__device__ void write_gram(const SearchArgs& a, int q, const float* sq, uint32_t* cids, uint32_t* cdist, int nA,
                           int Kp, uint32_t oid, GT* sG, int slot) {
    const int lane = threadIdx.x;
    // index of the neighbour among the first pass's rows: the ranking's
    // candidate index when known, else a search of cids[0..nA)
    int pi = -1;
    if (__ballot(lane < Kp && slot < 0) == 0) {
        pi = slot < nA ? slot : -1;
    } else {
        for (int s = 0; s < nA; ++s)
            if (cids[s] == oid) pi = s;
    }
    const bool all = __ballot(lane < Kp && pi < 0) == 0;
    if (!all) {
        // rare: a neighbour outside the first pass; its rows in final order
        __syncthreads();
        if (lane < Kp) cids[lane] = oid;
        __syncthreads();
        exact_pass<GT>(a, sq, cids, cdist, 0, Kp, sG);
        pi = lane;
    }
    __syncthreads();
    GT* out = reinterpret_cast<GT*>(a.gram) + (int64_t)q * 36;
    if (lane < 36) {
        // row i of packed entry `lane` (i (i + 1) / 2 <= lane < (i + 1) (i + 2) / 2)
        int i = (int)((__builtin_amdgcn_sqrtf((float)(8 * lane + 1)) - 1.0f) * 0.5f);
        if ((i + 1) * (i + 2) / 2 <= lane) ++i;
        if (i * (i + 1) / 2 > lane) --i;
        const int j = lane - i * (i + 1) / 2;
        const int pa = __shfl(pi, i), pb = __shfl(pi, j);
        out[lane] = i < Kp ? sG[pa * 8 + pb] : (GT)0;
    }
}

// Of the M keys held NSL per lane (element s*64 + lane) with flag `in`, mark
// the n smallest (n <= number flagged); equal keys by lower `tie` value.
template <int NSL>
__device__ void mark_smallest(const uint32_t (&kv)[NSL], const uint32_t (&tie)[NSL], const bool (&in)[NSL], int M,
                              int n, bool (&keep)[NSL]) {
    const int lane = threadIdx.x & 63;
    uint32_t k2[NSL];
#pragma unroll
    for (int s = 0; s < NSL; ++s) k2[s] = in[s] ? kv[s] : 0xFFFFFFFFu;
    const uint32_t tau = radix_kth(k2, M, n);
    int nlt = 0, neq = 0;
#pragma unroll
    for (int s = 0; s < NSL; ++s) {
        nlt += __popcll(__ballot(in[s] && k2[s] < tau));
        neq += __popcll(__ballot(in[s] && k2[s] == tau));
    }
#pragma unroll
    for (int s = 0; s < NSL; ++s) keep[s] = in[s] && k2[s] < tau;
    const int need = n - nlt;
    if (neq == need) {
#pragma unroll
        for (int s = 0; s < NSL; ++s) keep[s] = keep[s] || (in[s] && k2[s] == tau);
    } else {
        uint32_t last = 0;
        for (int r = 0; r < need; ++r) {
            uint32_t best = 0xFFFFFFFFu;
#pragma unroll
            for (int s = 0; s < NSL; ++s)
                if (in[s] && k2[s] == tau && (r == 0 || tie[s] > last) && tie[s] < best) best = tie[s];
            best = wave_min_u32(best);
#pragma unroll
            for (int s = 0; s < NSL; ++s)
                if (in[s] && k2[s] == tau && tie[s] == best) keep[s] = true;
            last = best;
        }
    }
    (void)lane;
}

// The early stop's candidates of patch q (step 1 of the search below):
// the concatenation of its L bins read 64 positions at a time; an LDS hash
// set of the IDs seen so far (open addressing, atomic compare-and-swap
// inserts, an atomic minimum keeping the earliest lane of a chunk) keeps
// first occurrences in order, up to cap. Leaves them in cids[0..M) and
// returns M; hset holds hsz slots. Ends with the workgroup synchronised.
__device__ __forceinline__ int cap_union(const SearchArgs& a, int q, uint64_t* hset, uint32_t* cids, int64_t* sbase,
                                         int32_t* smark) {
    const int lane = threadIdx.x;
    const int L = a.L;
    const int hsz = a.hsz;
    const uint32_t hmask = (uint32_t)hsz - 1u;
    const int hshift = 32 - __builtin_ctz((unsigned)hsz);
    uint32_t off = 0, cnt = 0;
    if (lane < L) {
        const uint2 b = a.bins[(int64_t)lane * a.Q + q];
        off = b.x;
        cnt = b.y;
    }
    const int T = wave_sum_i32((int)cnt);
    // bins concatenated in table order: position i of bin l is entry
    // i - start_l of that bin
    const int start = wave_incl_scan((int)cnt) - (int)cnt;
    if (lane < L) sbase[lane] = (int64_t)lane * a.N + off - start;
    for (int i = lane; i < hsz; i += 64) hset[i] = ~0ull;
    __syncthreads();
    int M = 0;
    int carry = 0;   // table of the position before the chunk
    for (int base = 0; base < T && M < a.cap; base += 64) {
        const int i = base + lane;
        const bool valid = i < T;
        // the table of each position: the last nonempty bin starting at
        // or before it (the bins starting inside the chunk mark their
        // first position)
        smark[lane] = -1;
        __syncthreads();
        const int ps = start - base;
        if (lane < L && cnt > 0 && ps >= 0 && ps < 64) smark[ps] = lane;
        __syncthreads();
        const uint64_t starts = __ballot(smark[lane] >= 0);
        const uint64_t below = starts & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
        const int tbl = below ? smark[63 - __builtin_clzll(below)] : carry;
        carry = __builtin_amdgcn_readlane(tbl, 63);
        uint32_t id = 0xFFFFFFFFu;
        if (valid) id = a.tids[sbase[tbl] + i];
        uint32_t slot = (id * 0x9E3779B1u) >> hshift;
        bool found = false;
        if (valid) {
            for (;;) {
                const uint64_t v = hset[slot];
                if ((uint32_t)(v >> 32) == id) {
                    found = true;
                    break;
                }
                if (v == ~0ull) break;
                slot = (slot + 1u) & hmask;
            }
        }
        const bool ins = valid && !found;
        const uint64_t mine = ((uint64_t)id << 32) | (uint32_t)lane;
        if (ins) {
            for (;;) {
                const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(&hset[slot]), ~0ull, mine);
                if (old == ~0ull) break;
                if ((uint32_t)(old >> 32) == id) {
                    atomicMin(reinterpret_cast<unsigned long long*>(&hset[slot]), mine);
                    break;
                }
                slot = (slot + 1u) & hmask;
            }
        }
        __syncthreads();
        const bool nw = ins && hset[slot] == mine;
        const uint64_t bal = __ballot(nw);
        const int rank = __popcll(bal & lanemask_lt());
        if (nw && M + rank < a.cap) cids[M + rank] = id;
        M = min(a.cap, M + (int)__popcll(bal));
    }
    __syncthreads();
    return M;
}

// Early-stop search (cap <= 256), one wave per patch.
//  1. Candidates: the concatenation of the L bins is read 64 positions at a
//     time; an LDS hash set of the IDs seen so far (open addressing, atomic
//     compare-and-swap inserts, an atomic minimum keeping the earliest lane
//     of a chunk) keeps first occurrences in order, up to `cap`.
//  2. Screen, when more than K candidates: each candidate's 64-byte screen
//     row (its coordinates y~ = s_x c in the dictionary's leading principal
//     directions as int8 codes c, with |y~|^2, s_x and rho_x) gives
//     |y^_q - y~|^2 = |y^_q|^2 + |y~|^2 - 2 y^_q.y~ from one int8 product on
//     the matrix cores (the rotated query coded as s_q (h + l / 128), its
//     int8 codes h and l as two rows of A, the screen rows as the columns of
//     B, so that one lane receives both products of a candidate), and
//     with the error bounds a lower bound L <= |q - x|^2. The K
//     candidates of smallest L get exact distances; the largest upper bound
//     U_K of those bounds the K-th smallest distance, so only candidates with
//     L <= U_K can be among the K nearest. Those get exact distances too (the
//     screened form keeps at most R in all, by smallest L).
//  3. Exact fp32 distances from both planes of the full features.
//  4. Sorted selection of the K best, certification (exact form), output.
// Seven waves per SIMD (72 registers, a few bytes of spill) hide more of the
// dependent memory round trips than six without spill, and spill less than
// eight. GT float or double: the Gram matrix of the neighbours is formed too
// (K <= 8).
template <bool EXACT, int NSL, typename GT>
__global__ __launch_bounds__(64, 7) void k_search_cap(SearchArgs a) {
    // dynamic LDS: hash set [hsz] of (id << 32 | first lane), empty = ~0, then
    // the candidate IDs and values [cp] each, cp = max(64, next_pow2(cap));
    // after the union the hash set holds the screen tails (float2 per candidate)
    extern __shared__ uint64_t hset[];
    uint32_t* cids = reinterpret_cast<uint32_t*>(hset + a.hsz);
    uint32_t* cdist = cids + a.cp;
    float2* stl = reinterpret_cast<float2*>(hset);
    __shared__ __align__(16) float sq[128];
    __shared__ int64_t sbase[kMaxL];       // per table: bin offset in tids minus the bin's first position
    __shared__ int32_t smark[64];          // table whose bin starts at a position of the current chunk, or -1
    __shared__ uint64_t srank[24];        // ranked keys, then their candidate indices
    const int lane = threadIdx.x;
    const int D = a.D;
    const int ri = lane & 15, kb = lane >> 4;   // MFMA layout

    {
        const int q = xcd_block();
        if (q >= a.Q) return;
        for (int i = lane; i < 128; i += 64) sq[i] = i < D ? a.qfeat[(int64_t)q * D + i] : 0.0f;

        // ---- 1. candidates, first occurrences in order, up to cap
        const int M = cap_union(a, q, hset, cids, sbase, smark);
        // the coded query y^ = s_q (h + l / 128): int8 codes h and l, then
        // s_q, |y^|^2 and rho_q >= |y^ - Phi q|
        const float* qr = a.qrot + (int64_t)q * kRotStride;
        const float s_q = qr[32], qn2 = qr[33], rho_q = qr[34];
        if (a.dump) {
            wave_sort_u32(cids, M);
            for (int i = lane; i < M && i < a.dump_cap; i += 64) a.dump[(int64_t)q * a.dump_cap + i] = (int32_t)cids[i];
        }
        if (lane == 0) a.out_ncand[q] = M;

        // ---- 2. screen lower bounds, exact distances of the K lowest, U_K
        int Mr = M;
        int nA = 0;   // rows of the first exact pass (cids[0..nA)), whose Gram matrix is in hset
        if (M > a.K) {
            const int K = a.K;
            // A operand: row 0 the high codes of y_q, row 1 the low codes,
            // lane (ri, kb) coordinates 16 kb .. 16 kb + 15
            const i32x4 qa = ri < 2 ? *reinterpret_cast<const i32x4*>(qr + 16 * ri + 4 * kb) : i32x4{0, 0, 0, 0};
            // B operand, the screen rows of 16 candidates as columns: lane
            // (ri, kb) holds bytes 16 kb .. 16 kb + 15 of candidate t + ri's
            // row (columns past M read row 0: column j of the product
            // depends on column j of B only, and is not used); the tail
            // (bytes 56 .. 63) goes to stl, and meets the query's zero codes
            // past the 56 screen coordinates in the product
            auto load_chunk = [&](int t, i32x4& v) {
                const int c = t + ri;
                const uint32_t id = c < M ? cids[c] : 0u;
                v = *reinterpret_cast<const i32x4*>(a.sc + (size_t)id * kScreenBytes + 16 * kb);
            };
            auto screen_chunk = [&](int t, const i32x4& v) {
                const int c = t + ri;
                if (kb == 3 && c < M) stl[c] = make_float2(__int_as_float(v[2]), __int_as_float(v[3]));
                const i32x4 acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(qa, v, i32x4{0, 0, 0, 0}, 0, 0, 0);
                // lane j < 16 holds rows 0 and 1 of column j: h.c and l.c of
                // candidate t + j, both exact; (128 h.c + l.c) / 128 is rounded once
                if (lane < 16 && c < M) cdist[c] = __float_as_uint((float)(128 * acc[0] + acc[1]) * (1.0f / 128.0f));
            };
            // four chunks (64 rows) in flight per step
            for (int t = 0; t < M; t += 64) {
                i32x4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) load_chunk(t + 16 * u, v[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (t + 16 * u < M) screen_chunk(t + 16 * u, v[u]);
            }
            __syncthreads();
            // |y^_q - y~| >= a_lo from the screen value and its error bound c (|y^_q|^2 + |y~|^2);
            // |q - x| >= (a_lo - rho_q - rho_x) / sigma; every fp32 step moves outward
            uint32_t lv[NSL], iv[NSL];
            bool valid[NSL];
#pragma unroll
            for (int s = 0; s < NSL; ++s) {
                const int c = s * 64 + lane;
                lv[s] = iv[s] = 0xFFFFFFFFu;
                valid[s] = c < M;
                if (c < M) {
                    const float2 tl = stl[c];
                    const uint32_t sr = __float_as_uint(tl.y);
                    const float dot = __uint_as_float(cdist[c]) * s_q * bf16_to_f((uint16_t)(sr & 0xFFFFu));
                    const float rho_x = bf16_to_f((uint16_t)(sr >> 16));
                    const float nn = qn2 + tl.x;
                    const float a2 = nn - 2.0f * dot;
                    const float E = fmaf(a.ce, nn, 1e-30f);
                    // the hardware square root (within 1 ulp; a flushed tiny
                    // argument gives 0), then 1e-6 down
                    const float alo = __builtin_amdgcn_sqrtf(fmaxf((a2 - E) * (1.0f - 1e-6f), 0.0f)) * (1.0f - 1e-6f);
                    const float l = fmaxf(alo * (1.0f - 1e-6f) - (rho_q + rho_x) * (1.0f + 1e-6f), 0.0f);
                    lv[s] = __float_as_uint(l * l * a.inv_s2 * (1.0f - 1e-5f));
                    iv[s] = cids[c];
                }
            }
            bool inA[NSL];
            mark_lowest16<NSL>(lv, K, inA);
            __syncthreads();
            int pos = 0;
#pragma unroll
            for (int s = 0; s < NSL; ++s) {
                const uint64_t bal = __ballot(inA[s]);
                if (inA[s]) cids[pos + __popcll(bal & lanemask_lt())] = iv[s];
                pos += __popcll(bal);
            }
            __syncthreads();
            if constexpr (std::is_same<GT, int>::value) {
                exact_rows(a, sq, cids, cdist, 0, K);
            } else {
                exact_pass<GT>(a, sq, cids, cdist, 0, K, reinterpret_cast<GT*>(hset));
                nA = K;
            }
            __syncthreads();
            // U_K: the largest upper bound of the K exact distances
            const Bounds bd{a.dist_eps, (double)D * 1.2e-38};
            double uk = 0.0;
            if (lane < K) {
                double dlo, dhi;
                dist_interval(cdist[lane], bd, dlo, dhi);
                uk = dhi;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) uk = fmax(uk, __shfl_xor(uk, o));
            bool sel[NSL];
            int S = 0;
#pragma unroll
            for (int s = 0; s < NSL; ++s) {
                sel[s] = valid[s] && !inA[s] && (double)__uint_as_float(lv[s]) <= uk;
                S += __popcll(__ballot(sel[s]));
            }
            if (!EXACT && K + S > a.rerank) {
                // screened form: at most R survivors in all, by lower bound, equal bounds by lower ID;
                // the cut is counted (the neighbours may then differ from the exact ones)
                if (lane == 0) atomicAdd(&a.counters[C_TRUNC], 1u);
                bool keep[NSL];
                mark_smallest<NSL>(lv, iv, sel, M, a.rerank - K, keep);
#pragma unroll
                for (int s = 0; s < NSL; ++s) sel[s] = keep[s];
                S = a.rerank - K;
            }
            pos = K;
#pragma unroll
            for (int s = 0; s < NSL; ++s) {
                const uint64_t bal = __ballot(sel[s]);
                if (sel[s]) cids[pos + __popcll(bal & lanemask_lt())] = iv[s];
                pos += __popcll(bal);
            }
            __syncthreads();
            Mr = K + S;
            // ---- 3. exact distances of the remaining survivors
            if (S > 0) exact_rows(a, sq, cids, cdist, K, Mr);
        } else if (!std::is_same<GT, int>::value && M <= 8) {
            // ---- 3. exact distances of all candidates, and their Gram matrix
            exact_pass<GT>(a, sq, cids, cdist, 0, M, reinterpret_cast<GT*>(hset));
            nA = M;
        } else {
            // ---- 3. exact distances of all candidates
            exact_rows(a, sq, cids, cdist, 0, M);
        }
        if (lane == 0 && a.out_nsurv) a.out_nsurv[q] = Mr;
        __syncthreads();

        // ---- 4. K best, certification, output
        const int Kp = min(a.K, Mr);
        int slot = -1;
        const uint64_t mykey = sort_select<NSL>(cids, cdist, Mr, srank, &slot);
        uint32_t oid = 0xFFFFFFFFu;
        float od = 0.0f;
        if (EXACT && Kp > 0) {
            // the certification may re-rank: the slots no longer apply
            certify_or_fix(a, q, cids, cdist, Mr, Kp, mykey, oid, od);
            slot = -1;
        } else if (lane < Kp) {
            oid = key_id(mykey);
            od = key_dist(mykey);
        }
        write_result(a, q, Kp, oid, od);
        if constexpr (!std::is_same<GT, int>::value)
            write_gram<GT>(a, q, sq, cids, cdist, nA, Kp, oid, reinterpret_cast<GT*>(hset), slot);
        __syncthreads();
    }
}

// Step 1 of the early-stop search alone (the candidates-only form): M into
// out_ncand and, when asked, the dump of the M IDs in the order the union
// met them (its only reader, the l1 ranking, does not depend on the order,
// so no sort). Few registers, so more waves per SIMD hide the dependent
// reads of the bins.
__global__ __launch_bounds__(64, 12) void k_union_cap(SearchArgs a) {
    extern __shared__ uint64_t hset[];
    uint32_t* cids = reinterpret_cast<uint32_t*>(hset + a.hsz);
    __shared__ int64_t sbase[kMaxL];
    __shared__ int32_t smark[64];
    const int lane = threadIdx.x;
    const int q = xcd_block();
    if (q >= a.Q) return;
    const int M = cap_union(a, q, hset, cids, sbase, smark);
    if (a.dump)
        for (int i = lane; i < M && i < a.dump_cap; i += 64) a.dump[(int64_t)q * a.dump_cap + i] = (int32_t)cids[i];
    if (lane == 0) a.out_ncand[q] = M;
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
    const int nq = BIG ? (int)a.counters[C_OVERFLOW] : a.Q;

    for (int t = xcd_block(); t < nq; t += gridDim.x) {
        const int q = BIG ? a.overflow[t] : t;
        uint32_t off = 0, cnt = 0;
        if (lane < L) {
            const uint2 b = a.bins[(int64_t)lane * a.Q + q];
            off = b.x;
            cnt = b.y;
        }
        const int T = wave_sum_i32((int)cnt);
        if (T > CMAX) {
            if (!BIG) {
                if (lane == 0) {
                    const unsigned int pos = atomicAdd(&a.counters[C_OVERFLOW], 1u);
                    a.overflow[pos] = q;
                }
            } else if (lane == 0) {
                // too many for LDS: the streaming pass ranks it (second half of the list)
                const unsigned int pos = atomicAdd(&a.counters[C_STREAM], 1u);
                a.overflow[(int64_t)a.Q + pos] = q;
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
            cand_distances<VEC, true>(qv, a.D, a.hs, a.hi, a.lo, cids, cdist, M);
            const uint64_t k2 = M <= 256 ? sort_select(cids, cdist, M) : select_topk(cids, cdist, M, a.rerank);
            __syncthreads();
            if (lane < a.rerank) cids[lane] = key_id(k2);
            __syncthreads();
            Mr = a.rerank;
        }
        cand_distances<VEC, false>(qv, a.D, a.hs, a.hi, a.lo, cids, cdist, Mr);
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

// Union search for patches whose bins hold more IDs than LDS takes (any
// number): one wave per listed patch merges the L bins (each sorted by ID)
// into the ascending sequence of distinct IDs, lane l streaming bin l from a
// register buffer of its next eight IDs; every step takes the wave minimum of
// the heads and advances every bin that holds it. Chunks of 64 distinct IDs
// get their squared distances as the FP64 sequential sum over the
// coordinates (the definition, so no certification is needed) and are merged
// into a running top K held by lanes 0..K-1 (K rounds of a wave minimum over
// (distance, ID)). Writes the neighbours, their distances rounded to fp32,
// the distinct-ID count and, when asked, the first dump_cap IDs ascending.
__global__ __launch_bounds__(64) void k_union_stream(SearchArgs a) {
    __shared__ uint32_t chunk[64];
    __shared__ double sq[128];
    const int lane = threadIdx.x;
    const int n = (int)a.counters[C_STREAM];
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const int q = a.overflow[(int64_t)a.Q + t];
        const int D = a.D;
        for (int i = lane; i < 128; i += 64) sq[i] = i < D ? (double)a.qfeat[(int64_t)q * D + i] : 0.0;
        uint32_t off = 0, cnt = 0;
        if (lane < a.L) {
            const uint2 b = a.bins[(int64_t)lane * a.Q + q];
            off = b.x;
            cnt = b.y;
        }
        const uint32_t* src = a.tids + (int64_t)lane * a.N + off;
        uint32_t buf[8];
        uint32_t pos = 0;   // next position of this lane's bin to load into buf
        int have = 0, at = 0;
        auto refill = [&]() {
#pragma unroll
            for (int e = 0; e < 8; ++e) buf[e] = (lane < a.L && pos + e < cnt) ? src[pos + e] : 0xFFFFFFFFu;
            have = (lane < a.L && pos < cnt) ? (int)min(8u, cnt - pos) : 0;
            pos += 8;
            at = 0;
        };
        refill();
        double bd = INFINITY;
        int bi = 0x7FFFFFFF;
        int nd = 0;
        __syncthreads();
        for (;;) {
            // the next chunk of up to 64 distinct IDs, ascending
            int nc = 0;
            for (; nc < 64; ++nc) {
                uint32_t head = 0xFFFFFFFFu;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (e == at) head = at < have ? buf[e] : 0xFFFFFFFFu;
                const uint32_t mn = wave_min_u32(head);
                if (mn == 0xFFFFFFFFu) break;
                if (head == mn) {
                    if (++at == have) {
                        if (pos < cnt) refill();
                        else have = 0, at = 0;
                    }
                }
                if (lane == 0) chunk[nc] = mn;
            }
            __syncthreads();
            if (nc == 0) break;
            if (a.dump && lane < nc && nd + lane < a.dump_cap)
                a.dump[(int64_t)q * a.dump_cap + nd + lane] = (int32_t)chunk[lane];
            double nd2 = INFINITY;
            int ni = 0x7FFFFFFF;
            if (lane < nc) {
                const float* row = a.xf + (int64_t)chunk[lane] * D;
                double acc = 0.0;
                for (int i = 0; i < D; ++i) {
                    const double z = sq[i] - (double)row[i];
                    acc = acc + z * z;
                }
                nd2 = acc;
                ni = (int)chunk[lane];
            }
            double rd = INFINITY;
            int rI = 0x7FFFFFFF;
            for (int k = 0; k < a.K; ++k) {
                const bool bfirst = bd < nd2 || (bd == nd2 && bi < ni);
                double md = bfirst ? bd : nd2;
                int mi = bfirst ? bi : ni;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const double od = __shfl_xor(md, o);
                    const int oi = __shfl_xor(mi, o);
                    if (od < md || (od == md && oi < mi)) {
                        md = od;
                        mi = oi;
                    }
                }
                if (bi == mi && bd == md) {
                    bd = INFINITY;
                    bi = 0x7FFFFFFF;
                } else if (ni == mi && nd2 == md) {
                    nd2 = INFINITY;
                    ni = 0x7FFFFFFF;
                }
                if (lane == k) {
                    rd = md;
                    rI = mi;
                }
            }
            bd = rd;
            bi = rI;
            nd += nc;
            __syncthreads();
            if (nc < 64) break;
        }
        const int m = min(a.K, nd);
        if (lane < a.K) {
            a.out_ids[(int64_t)q * a.K + lane] = lane < m ? bi : -1;
            a.out_d2[(int64_t)q * a.K + lane] = lane < m ? (float)bd : 0.0f;
        }
        if (lane == 0) {
            a.out_m[q] = m;
            a.out_ncand[q] = nd;
        }
        __syncthreads();
    }
}

constexpr int kCapMax = 256;      // early-stop limit a wave can hold
constexpr int kUnionMax = 2048;   // uncapped: IDs per wave before deferring
constexpr int kUnionBig = 8192;   // uncapped, deferred patches

static int cap_hash_slots_min(int cap) { return (5 * (cap + 63) + 2) / 3; }

template <int NSL, typename GT>
static void launch_cap_g(const SearchArgs& a, int grid, size_t lds, hipStream_t st) {
    if (a.exact) hipLaunchKernelGGL((k_search_cap<true, NSL, GT>), dim3(grid), dim3(64), lds, st, a);
    else hipLaunchKernelGGL((k_search_cap<false, NSL, GT>), dim3(grid), dim3(64), lds, st, a);
}
template <int NSL>
static void launch_cap_n(const SearchArgs& a, int grid, size_t lds, hipStream_t st) {
    if (!a.gram) launch_cap_g<NSL, int>(a, grid, lds, st);
    else if (a.gram_fp64) launch_cap_g<NSL, double>(a, grid, lds, st);
    else launch_cap_g<NSL, float>(a, grid, lds, st);
}
// one wave (workgroup) per patch: no loop over patches, so that nothing is
// held in registers from one patch to the next
static void launch_cap(const SearchArgs& a, hipStream_t st) {
    const int grid = round_grid8(a.Q);
    if (a.cand_only) {
        const size_t lu = (size_t)a.hsz * sizeof(uint64_t) + (size_t)a.cp * sizeof(uint32_t);
        hipLaunchKernelGGL(k_union_cap, dim3(grid), dim3(64), lu, st, a);
        return;
    }
    const size_t lds = (size_t)a.hsz * sizeof(uint64_t) + 2 * (size_t)a.cp * sizeof(uint32_t);
    if (a.cap <= 128) launch_cap_n<2>(a, grid, lds, st);
    else launch_cap_n<4>(a, grid, lds, st);
}

hipError_t launch_search(const SearchArgs& a_in, hipStream_t st) {
    if (a_in.Q == 0) return hipSuccess;
    SearchArgs a = a_in;
    a.dist_eps = 2.0 * gamma_n(a.D + 3, 1.0 / 16777216.0);
    const int grid = round_grid8(a.Q < 32768 ? a.Q : 32768);
    if (a.D < 1 || a.D > 128) return hipErrorInvalidValue;
    if (a.cap > kCapMax) return hipErrorInvalidValue;
    if (!a.exact && (a.rerank < 1 || a.rerank > 64)) return hipErrorInvalidValue;
    if (a.cap > 0) {
        // hash set of at most cap + 63 IDs at load <= 0.6
        int h = 64;
        while (h < cap_hash_slots_min(a.cap)) h <<= 1;
        a.hsz = h;
        int cp = 64;
        while (cp < a.cap) cp <<= 1;
        a.cp = cp;
        if (a.gram && a.K > 8) return hipErrorInvalidValue;
        launch_cap(a, st);
        return hipGetLastError();
    }
    const bool v4 = a.D % 4 == 0;
    if (!v4 && a.D > 32) return hipErrorInvalidValue;
    if (v4) hipLaunchKernelGGL((k_search_union<4, kUnionMax, false>), dim3(grid), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_search_union<1, kUnionMax, false>), dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_search_overflow(const SearchArgs& a_in, int grid, hipStream_t st) {
    SearchArgs a = a_in;
    a.dist_eps = 2.0 * gamma_n(a.D + 3, 1.0 / 16777216.0);
    const bool v4 = a.D % 4 == 0 && a.D <= 128;
    if (v4) hipLaunchKernelGGL((k_search_union<4, kUnionBig, true>), dim3(grid), dim3(64), 0, st, a);
    else hipLaunchKernelGGL((k_search_union<1, kUnionBig, true>), dim3(grid), dim3(64), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_union_stream, dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace zh
