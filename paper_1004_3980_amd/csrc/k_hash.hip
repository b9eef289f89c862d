// Projection, p-stable codes, bucket keys and bin lookup (Section 4.1,
// Eq. hash_fn; Section 3.2: k concatenated hashes per table, L tables).
//
//   code_j(v) = floor((alpha_j . v + beta_j) / w)
//
// A wave owns 16 or 32 feature rows and runs over all tables. The dot
// products of its rows with the k hashes of a table run on the matrix cores,
// either as fp32 MFMA (P = (alpha.v + beta) / w evaluated as written) or as
// three bf16 MFMAs over a high/low split of both operands, with alpha / w
// and beta / w rounded to fp32 beforehand (a' = alpha / w = a_hi + a_lo,
// v = v_hi + v_lo; a_hi v_hi + a_hi v_lo + a_lo v_hi accumulate in fp32 and
// P = S + beta / w); the split of the wave's rows stays in registers for all
// tables. A fourth product of the absolute values bounds
// sum_i |a'_i v_i|, which gives a rigorous bound B on |P_mfma - P_exact|;
// when [P - B, P + B] holds no integer the MFMA floor is the exact code,
// otherwise the code is recomputed by the FP64 sequential dot product that
// defines it (in a second kernel, for the few tables that need it). The
// codes therefore equal the FP64 definition bit for bit.
//
// The k codes of a table become a 64-bit key
//   key = fmix64( M_l63 + sum_j uint32(c_j) * M_lj  mod 2^64 ),
// M_lj = SplitMix64 output 64 l + j + 1 from state 0 (table a.key_mul: k
// multipliers and the start value M_l63 per table), and,
// when a directory is given, a third kernel looks up each key's bin
// (offset, count).
#include <cmath>

#include "zh_internal.h"

namespace zh {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kRowsPerWave = 16;


__device__ __forceinline__ int32_t floor_sat(double t) {
    const double f = floor(t);
    if (f >= 2147483647.0) return 2147483647;
    if (f <= -2147483648.0) return (int32_t)0x80000000;
    return (int32_t)f;
}

// floor(x) as int32 in one instruction (x of magnitude below 2^31)
__device__ __forceinline__ int32_t cvt_floor(float x) {
    int32_t r;
    asm volatile("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// |x| of eight bf16 values: the sign bits cleared, one 32-bit AND per pair
__device__ __forceinline__ u16x8 abs8(u16x8 x) {
    uint4 w = __builtin_bit_cast(uint4, x);
    w.x &= 0x7FFF7FFFu;
    w.y &= 0x7FFF7FFFu;
    w.z &= 0x7FFF7FFFu;
    w.w &= 0x7FFF7FFFu;
    return __builtin_bit_cast(u16x8, w);
}

// Walk the directory from slot s on (linear probing) to the key or an empty
// slot; (off, cnt) stay 0 for an absent key.
__device__ __forceinline__ void probe_bin_from(const Slot* __restrict__ dir, uint64_t cap, uint64_t key, uint64_t s,
                                               uint32_t& off, uint32_t& cnt) {
    const uint64_t mask = cap - 1;
    off = 0;
    cnt = 0;
    for (uint64_t step = 0; step < cap; ++step) {
        const uint4 e = *reinterpret_cast<const uint4*>(dir + s);
        const uint64_t k = ((uint64_t)e.y << 32) | e.x;
        if (k == key) {
            cnt = e.z;
            off = e.w;
            return;
        }
        if (k == kEmptyKey) return;
        s = (s + 1) & mask;
    }
}

constexpr int kWaves = 4;         // waves per workgroup, 16 feature rows each
constexpr int kStage = 2;         // tables whose alpha is staged in LDS together

// Staged hash rows of a pair of tables, padded to whole 16-row MFMA tiles.
__host__ __device__ inline int stage_rows(int k) { return (kStage * k + 15) & ~15; }
// LDS row stride of the staged alpha. Split path: halfwords, the 32*NS
// coordinates of the MFMA steps plus one 16-byte chunk, so that a row holds
// an odd number of chunks and the 16-byte reads of eight consecutive rows
// fall on distinct banks. fp32 path: an odd number of words.
__host__ __device__ inline int stage_stride(int prec, int D) {
    if (prec == 0) return (D & 1) ? D : D + 1;
    return ((D + 31) & ~31) + 8;
}
__host__ __device__ inline int fold_tables(int k) { return k <= 24 ? 4 : 2; }
// fix-list entry: row, table, k codes, padded to 16 bytes
__host__ __device__ inline int fix_entry_ints(int k) { return (k + 2 + 3) & ~3; }
// bytes of the staged alpha, then beta and the bound constant of each staged row
// (split path: the high plane, then the low plane)
__host__ __device__ inline int stage_alpha_bytes(int prec, int k, int D) {
    const int R = stage_rows(k);
    return prec == 0 ? R * stage_stride(0, D) * 4 : 2 * R * stage_stride(1, D) * 2;
}
__host__ __device__ inline int stage_bytes(int prec, int k, int D) {
    return ((stage_alpha_bytes(prec, k, D) + 15) & ~15) + 2 * stage_rows(k) * 4;
}

// PREC 0: fp32 MFMA (4 coordinates per step); PREC 1: split bf16 (32 per
// step, NS steps). The alpha of two tables at a time is staged in LDS with
// its beta and bound constants and shared by the four waves (the split path
// stages alpha / w and beta / w);
// on the split path the next pair is fetched into registers while the
// current one is in use. The 2k hash rows of a pair are packed into ceil(2k/16) MFMA tiles.
// A wave owns RT tiles of 16 feature rows: every A fragment read from LDS
// feeds the products of all RT tiles (RT = 2 halves the LDS reads and the
// staging per row).
// A code whose interval [P - B, P + B] holds an integer is left to the FP64
// definition: the table's k codes go to a compact list (the uncertain ones
// marked kCodeUnset) for k_hash_fixlist, or, when the list is full, the
// table's bit is set in the row's dirty mask for k_hash_fix; the key written
// here is replaced there. The list has a region of fix_cap entries per 16
// feature rows.
// Three waves per SIMD (at most 168 registers) for one tile a wave, two for two.
template <int PREC, int NS, int NPRE, int RT>
__global__ __launch_bounds__(256, RT == 1 ? 3 : 2) void k_hash(HashArgs a) {
    constexpr int RPW = kRowsPerWave * RT;   // feature rows of a wave
    const int D = a.D, k = a.k, L = a.L, m = L * k;
    const int GK = kStage * k;
    const int R = stage_rows(k);
    const int ntile = R >> 4;
    const int nsteps = PREC == 0 ? (D + 3) / 4 : NS;
    const int DP = (D + 31) & ~31;
    const int DS = stage_stride(PREC, D);
    const int fold = fold_tables(k) / RT;   // tables folded together: fold * RPW = 64 lanes
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ri = lane & 15, kb = lane >> 4;
    const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * RPW;

    extern __shared__ __align__(16) unsigned char smem[];
    uint16_t* sA16 = reinterpret_cast<uint16_t*>(smem);
    float* sAf = reinterpret_cast<float*>(smem);
    float* sBeta = reinterpret_cast<float*>(smem + ((stage_alpha_bytes(PREC, k, D) + 15) & ~15));
    float* sBc0 = sBeta + R;
    // per wave codes of `fold` tables: [fold*k][RPW rows], then per wave a
    // flag per (table of the fold group, row) with an uncertain code
    int32_t* sC = reinterpret_cast<int32_t*>(smem + stage_bytes(PREC, k, D)) + wave * (fold * k * RPW);
    uint8_t* sU = reinterpret_cast<uint8_t*>(reinterpret_cast<int32_t*>(smem + stage_bytes(PREC, k, D)) +
                                             kWaves * fold * k * RPW) + wave * 64;
    sU[lane] = 0;
    // key multipliers of every table, [L][k + 1]
    uint64_t* smul = reinterpret_cast<uint64_t*>(reinterpret_cast<unsigned char*>(sU - wave * 64) + kWaves * 64);
    for (int e = threadIdx.x; e < L * (k + 1); e += 256) smul[e] = a.key_mul[e];

    // B operand of this lane for every k-step and row tile rt: feature row
    // r0 + 16 rt + ri, coordinates 32 s + 8 kb + e (e < 8) as bf16 high/low
    // parts (PREC 1), or 4 s + kb as fp32 (PREC 0)
    u16x8 bh[RT][PREC == 1 ? NS : 1], bl[RT][PREC == 1 ? NS : 1];
    float bf[PREC == 0 ? 32 : 1];
    bool rowok[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) rowok[rt] = r0 + 16 * rt + ri < a.n;
    if (PREC == 1) {
        // rows on 16-byte boundaries: two 16-byte loads per step
        const bool vec = (D & 3) == 0 && (reinterpret_cast<uintptr_t>(a.feat) & 15) == 0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int64_t row = r0 + 16 * rt + ri;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int d0 = 32 * s + 8 * kb;
                float x[8];
                if (vec) {
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const float4 v = (rowok[rt] && d0 + 4 * j < D)
                                             ? *reinterpret_cast<const float4*>(a.feat + row * D + d0 + 4 * j)
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
                        x[4 * j] = v.x;
                        x[4 * j + 1] = v.y;
                        x[4 * j + 2] = v.z;
                        x[4 * j + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) x[e] = (rowok[rt] && d0 + e < D) ? a.feat[row * D + d0 + e] : 0.0f;
                }
                // high part: x rounded to bf16 (nearest even); low part: the
                // exact remainder rounded likewise
                bf16x8 hv, lv;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    hv[e] = (__bf16)x[e];
                    lv[e] = (__bf16)(x[e] - (float)hv[e]);
                }
                bh[rt][s] = __builtin_bit_cast(u16x8, hv);
                bl[rt][s] = __builtin_bit_cast(u16x8, lv);
            }
        }
    } else {
        const int64_t row = r0 + ri;
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            const int d = 4 * s + kb;
            bf[s] = (rowok[0] && d < D) ? a.feat[row * D + d] : 0.0f;
        }
    }
    const float c1 = a.bound_c1, c2 = a.bound_c2;

    // split path: 16-byte chunks [plane][row][chunk], CH chunks a row (the
    // zero-padded DP coordinates of the host copy); rows past the last table
    // are zero
    constexpr int CH = 4 * NS;
    const int NC = 2 * GK * CH;
    u16x8 pre[NPRE];
    float pbc = 0.0f;
    // per chunk of this thread, fixed over the groups: bits 0..15 its offset
    // r DP + 8 ch in the pair's rows (halfwords), bits 16..30 its LDS offset,
    // bit 31 the low plane; 0x7FFFFFFF when the thread has no such chunk
    // (offsets below 2^15: GK <= 64 rows of DP <= 128, 2 R DS < 2^15)
    uint32_t cdesc[NPRE];
#pragma unroll
    for (int c = 0; c < NPRE; ++c) {
        const int ci = threadIdx.x + 256 * c;
        const int plane = ci >= GK * CH;
        const int r2 = ci - plane * GK * CH;
        const int r = r2 / CH, ch = r2 - r * CH;
        cdesc[c] = ci < NC ? (uint32_t)(r * DP + 8 * ch) | ((uint32_t)((plane * R + r) * DS + 8 * ch) << 16) |
                                 ((uint32_t)plane << 31)
                           : 0x7FFFFFFFu;
    }
    auto fetch = [&](int g) {
        const int l0 = g * kStage;
        // chunks of rows l0 k + r < m only
        const uint32_t lim = (uint32_t)((m - l0 * k) * DP);
        const uint16_t* bhi = a.a_hi + (int64_t)l0 * k * DP;
        const uint16_t* blo = a.a_lo + (int64_t)l0 * k * DP;
#pragma unroll
        for (int c = 0; c < NPRE; ++c) {
            const uint32_t off = cdesc[c] & 0xFFFFu;
            u16x8 v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (cdesc[c] != 0x7FFFFFFFu && off < lim)
                v = *reinterpret_cast<const u16x8*>(((cdesc[c] >> 31) ? blo : bhi) + off);
            pre[c] = v;
        }
        // beta and the bound constant: thread t < 2 GK takes one value
        const int t = threadIdx.x;
        const int r = t < GK ? t : t - GK;
        pbc = 0.0f;
        if (t < 2 * GK && l0 * k + r < m) pbc = (t < GK ? a.beta_w : a.bound_c0)[l0 * k + r];
    };
    auto stash = [&]() {
#pragma unroll
        for (int c = 0; c < NPRE; ++c)
            if (cdesc[c] != 0x7FFFFFFFu) *reinterpret_cast<u16x8*>(sA16 + ((cdesc[c] >> 16) & 0x7FFFu)) = pre[c];
        const int t = threadIdx.x;
        if (t < 2 * GK) (t < GK ? sBeta[t] : sBc0[t - GK]) = pbc;
    };
    auto copy_f32 = [&](int g) {
        const int l0 = g * kStage;
        const int tot = GK * D;
        for (int e = threadIdx.x; e < tot; e += 256) {
            const int r = e / D, c = e - r * D;
            sAf[r * DS + c] = l0 * k + r < m ? a.alpha[(int64_t)l0 * k * D + e] : 0.0f;
        }
        for (int t = threadIdx.x; t < 2 * GK; t += 256) {
            const int r = t < GK ? t : t - GK;
            const float v = l0 * k + r < m ? (t < GK ? a.beta : a.bound_c0)[l0 * k + r] : 0.0f;
            (t < GK ? sBeta[r] : sBc0[r]) = v;
        }
    };

    // rows GK..R-1 of the stage are never written by the staging: zero them
    if (PREC == 1) {
        const int padrows = R - GK;
        for (int e = threadIdx.x; e < 2 * padrows * (DS / 8); e += 256) {
            const int plane = e / (padrows * (DS / 8));
            const int e2 = e - plane * padrows * (DS / 8);
            const int r = GK + e2 / (DS / 8), ch = e2 % (DS / 8);
            *reinterpret_cast<u16x8*>(sA16 + (plane * R + r) * DS + 8 * ch) = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        }
    } else {
        for (int e = threadIdx.x; e < (R - GK) * DS; e += 256) sAf[GK * DS + e] = 0.0f;
    }
    for (int e = threadIdx.x; e < R - GK; e += 256) sBeta[GK + e] = sBc0[GK + e] = 0.0f;

    const int ngroups = (L + kStage - 1) / kStage;
    if (PREC == 1) {
        fetch(0);
        stash();
    } else {
        copy_f32(0);
    }
    __syncthreads();

    // fix-list regions of the wave: one per 16 rows (region of lane (t, rr)
    // in the fold stage: rr / 16)
    const int64_t w16 = r0 / kRowsPerWave;
    uint64_t dirty = 0;
    unsigned nflag = 0;
    unsigned wcnt[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) wcnt[rt] = 0;
    for (int g = 0; g < ngroups; ++g) {
        const int l0 = g * kStage;
        const int GKa = (L - l0 < kStage ? L - l0 : kStage) * k;
        if (PREC == 1 && g + 1 < ngroups) fetch(g + 1);
        for (int tt = 0; tt < ntile; ++tt) {
            const int ar = tt * 16 + ri;
            f32x4 cs[RT], cab[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) cs[rt] = cab[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (PREC == 1) {
                // the three split products share one fp32 accumulator: the
                // bound covers any order of the 3 DP additions
                const uint16_t* Ah = sA16 + ar * DS + 8 * kb;
                const uint16_t* Al = Ah + R * DS;
                u16x8 ah[NS], al[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    ah[s] = *reinterpret_cast<const u16x8*>(Ah + 32 * s);
                    al[s] = *reinterpret_cast<const u16x8*>(Al + 32 * s);
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const bf16x8 ahb = __builtin_bit_cast(bf16x8, ah[s]);
                    const bf16x8 alb = __builtin_bit_cast(bf16x8, al[s]);
                    const bf16x8 aab8 = __builtin_bit_cast(bf16x8, abs8(ah[s]));
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        const bf16x8 vhb = __builtin_bit_cast(bf16x8, bh[rt][s]);
                        const bf16x8 vlb = __builtin_bit_cast(bf16x8, bl[rt][s]);
                        const bf16x8 vab = __builtin_bit_cast(bf16x8, abs8(bh[rt][s]));
                        cs[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahb, vhb, cs[rt], 0, 0, 0);
                        cab[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aab8, vab, cab[rt], 0, 0, 0);
                        cs[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahb, vlb, cs[rt], 0, 0, 0);
                        cs[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alb, vhb, cs[rt], 0, 0, 0);
                    }
                }
            } else {
                const float* Af = sAf + ar * DS;
                for (int s = 0; s < nsteps; ++s) {
                    const int d = 4 * s + kb;
                    const float av = d < D ? Af[d] : 0.0f;
                    cs[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bf[s < 32 ? s : 0], cs[0], 0, 0, 0);
                    cab[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fabsf(av), fabsf(bf[s < 32 ? s : 0]), cab[0], 0, 0,
                                                                  0);
                }
            }
            // 16x16 tile: lane holds hash rows 4*kb+i of the tile, feature row ri
            const float4 be = *reinterpret_cast<const float4*>(sBeta + tt * 16 + 4 * kb);
            const float4 b0 = *reinterpret_cast<const float4*>(sBc0 + tt * 16 + 4 * kb);
            const float bev[4] = {be.x, be.y, be.z, be.w};
            const float b0v[4] = {b0.x, b0.y, b0.z, b0.w};
            // codes of rows past the table count stay out of the stage (their
            // slots belong to other tables); codes of feature rows past n are
            // written but never read
            const bool full = tt * 16 + 16 <= GKa;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                int32_t* cdst = sC + ((l0 % fold) * k + tt * 16 + 4 * kb) * RPW + 16 * rt + ri;
                unsigned fl = 0;
                int32_t cv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float S = cs[rt][i];
                    // split path: alpha and beta came divided by w
                    const float P = PREC == 1 ? S + bev[i] : (S + bev[i]) * a.inv_w;
                    const float B = PREC == 1 ? fmaf(c1, cab[rt][i], b0v[i])
                                              : fmaf(c1, cab[rt][i], fmaf(c2, fabsf(S), b0v[i]));
                    // uncertain when an integer lies within B of P; every P of
                    // magnitude >= 2^23 is an integer, so each certain code has
                    // |floor(P)| <= 2^23 (a NaN P or B is uncertain as well)
                    const bool flag = !(fabsf(P - rintf(P)) > B);
                    fl |= (flag ? 1u : 0u) << i;
                    const int32_t c = cvt_floor(P);
                    cv[i] = flag ? kCodeUnset : c;
                }
                if (full) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) cdst[i * RPW] = cv[i];
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (tt * 16 + 4 * kb + i < GKa) cdst[i * RPW] = cv[i];
                }
                if (fl != 0 && rowok[rt]) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int hr = tt * 16 + 4 * kb + i;
                        if (((fl >> i) & 1u) && hr < GKa) {
                            ++nflag;
                            sU[((l0 % fold) + (hr >= k ? 1 : 0)) * RPW + 16 * rt + ri] = 1;
                        }
                    }
                }
            }
        }
        __syncthreads();   // the staged pair is no longer read; codes visible to the wave
        if (g + 1 < ngroups) {
            if (PREC == 1)
                stash();
            else
                copy_f32(g + 1);
        }
        if ((l0 + kStage) % fold == 0 || g + 1 == ngroups) {
            // fold codes into keys: lane = (table of the fold group, feature row)
            const int fl0 = (l0 / fold) * fold;
            const int t = lane / RPW, rr = lane - t * RPW;
            const int lt = fl0 + t;
            const int64_t row = r0 + rr;
            const bool act = t < fold && lt < L && row < a.n;
            const bool unset = act && sU[t * RPW + rr] != 0;
            // a table with an uncertain code goes to the fix-list region of
            // its row's 16 with its codes (or, when the region is full, to the
            // row's dirty mask)
            const uint64_t bal = __ballot(unset);
            const int reg = rr >> 4;
            // lanes of region reg: rr in [16 reg, 16 reg + 16) of every table slot
            const uint64_t regmask = RT == 1 ? ~0ull : (reg ? 0xFFFF0000FFFF0000ull : 0x0000FFFF0000FFFFull);
            const int idx = (int)wcnt[RT == 1 ? 0 : reg] + __popcll(bal & regmask & lanemask_lt());
            int32_t* ent = nullptr;
            if (unset) {
                if (idx < a.fix_cap) {
                    ent = a.fix_list + ((w16 + reg) * a.fix_cap + idx) * fix_entry_ints(k);
                    ent[0] = (int32_t)row;
                    ent[1] = lt;
                } else {
                    dirty |= 1ull << lt;
                }
            }
            if (RT == 1) {
                wcnt[0] += (unsigned)__popcll(bal);
            } else {
                wcnt[0] += (unsigned)__popcll(bal & 0x0000FFFF0000FFFFull);
                wcnt[RT - 1] += (unsigned)__popcll(bal & 0xFFFF0000FFFF0000ull);
            }
            if (act) {
                const uint64_t* mul = smul + lt * (k + 1);
                const int32_t* cp = sC + t * k * RPW + rr;
                uint64_t h = mul[k];
#pragma unroll 10
                for (int j = 0; j < k; ++j) h += key_term(cp[j * RPW], mul[j]);
                a.keys[key_pos(a, row, lt)] = key_final(h);
                if (a.codes)
                    for (int j = 0; j < k; ++j) a.codes[row * m + lt * k + j] = cp[j * RPW];
                if (ent)
                    for (int j = 0; j < k; ++j) ent[2 + j] = cp[j * RPW];
            }
            sU[lane] = 0;
        }
        __syncthreads();
    }
    // tables of the fold lanes (t, row) that did not fit in the list
    for (int o = RPW; o < 64; o <<= 1) dirty |= __shfl_xor(dirty, o);
    if (lane < RPW && r0 + lane < a.n) a.dirty[r0 + lane] = dirty;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
        if (lane == 0 && r0 + 16 * rt < a.n)
            a.fix_count[w16 + rt] = wcnt[rt] < (unsigned)a.fix_cap ? wcnt[rt] : (unsigned)a.fix_cap;
    if (nflag && a.n_fixed) atomicAdd(a.n_fixed, nflag);
}

// FP64 sequential dot product of an alpha row and a feature row (coordinates
// in index order; each product is exact in FP64), 16-byte loads when the rows
// allow it.
__device__ __forceinline__ double dot_fp64(const float* __restrict__ ar, const float* __restrict__ vr, int D) {
    double s = 0.0;
    int i = 0;
    if ((D & 3) == 0 && ((reinterpret_cast<uintptr_t>(ar) | reinterpret_cast<uintptr_t>(vr)) & 15) == 0) {
        const float4* a4 = reinterpret_cast<const float4*>(ar);
        const float4* v4 = reinterpret_cast<const float4*>(vr);
#pragma unroll 5
        for (int c = 0; c < D / 4; ++c) {
            const float4 x = a4[c], y = v4[c];
            s = s + (double)x.x * (double)y.x;
            s = s + (double)x.y * (double)y.y;
            s = s + (double)x.z * (double)y.z;
            s = s + (double)x.w * (double)y.w;
        }
        i = D;
    }
    for (; i < D; ++i) s = s + (double)ar[i] * (double)vr[i];
    return s;
}

// Entries of the fix list, one thread per entry slot: the uncertain codes of
// the (row, table) pair are computed by the FP64 sequential dot product that
// defines them, and the table's key is folded again from all k codes. The
// entry is read into registers with 16-byte loads first.
__global__ __launch_bounds__(256) void k_hash_fixlist(HashArgs a) {
    const int64_t nw = (a.n + kRowsPerWave - 1) / kRowsPerWave;
    const int cap = a.fix_cap;
    const int64_t total = nw * cap;
    const int k = a.k, D = a.D, L = a.L, m = L * k;
    const int es4 = fix_entry_ints(k) / 4;
    const double wd = (double)a.w;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t w = (uint64_t)i / (uint32_t)cap;
        if ((int)(i - w * cap) >= (int)a.fix_count[w]) continue;
        const int4* e4 = reinterpret_cast<const int4*>(a.fix_list + i * fix_entry_ints(k));
        int32_t ev[(kMaxKHash + 2 + 3) & ~3];
#pragma unroll
        for (int c = 0; c < (kMaxKHash + 2 + 3) / 4; ++c) {
            int4 v = make_int4(0, 0, 0, 0);
            if (c < es4) v = e4[c];
            ev[4 * c] = v.x;
            ev[4 * c + 1] = v.y;
            ev[4 * c + 2] = v.z;
            ev[4 * c + 3] = v.w;
        }
        const int64_t row = (uint32_t)ev[0];
        const int l = ev[1];
        const float* vr = a.feat + row * D;
        uint32_t um = 0;
#pragma unroll
        for (int j = 0; j < kMaxKHash; ++j)
            if (j < k && ev[2 + j] == kCodeUnset) um |= 1u << j;
        while (um) {
            const int j = __builtin_ctz(um);
            um &= um - 1;
            const int hrow = l * k + j;
            const int32_t c = floor_sat((dot_fp64(a.alpha + (int64_t)hrow * D, vr, D) + (double)a.beta[hrow]) / wd);
#pragma unroll
            for (int jj = 0; jj < kMaxKHash; ++jj)
                if (jj == j) ev[2 + jj] = c;
        }
        uint64_t h = a.key_mul[l * (k + 1) + k];
#pragma unroll
        for (int j = 0; j < kMaxKHash; ++j) {
            if (j < k) {
                if (a.codes) a.codes[row * m + l * k + j] = ev[2 + j];
                h += key_term(ev[2 + j], a.key_mul[l * (k + 1) + j]);
            }
        }
        a.keys[key_pos(a, row, l)] = key_final(h);
    }
}

// Keys of the (row, table) pairs whose codes were not certain: every code of
// the table is recomputed by the FP64 sequential dot product that defines it
// (coordinates in index order), and the key is folded again. One wave (one
// workgroup) takes 64 rows; its lanes form G = min(4, 64/k) groups, each
// group one (row, table) pair with a lane per hash. The k alpha rows of the
// table (contiguous in memory) and the feature row are first copied to LDS
// with coalesced loads; each lane then runs its dot product from LDS.
__host__ __device__ inline int fix_groups(int k) { return 64 / k < 4 ? 64 / k : 4; }

__global__ __launch_bounds__(64) void k_hash_fix(HashArgs a) {
    extern __shared__ float sfix[];   // [G][k*D alpha | D feature]
    const int lane = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int k = a.k, D = a.D, L = a.L, m = L * k;
    const int G = fix_groups(k);
    const int per = (k + 1) * D;
    const int grp = lane / k, jj = lane - grp * k;
    const double wd = (double)a.w;
    uint64_t mk = r0 + lane < a.n ? a.dirty[r0 + lane] : 0;
    for (;;) {
        int src_mine = 0, l_mine = 0, got = 0;
        for (int g = 0; g < G; ++g) {
            const uint64_t any = __ballot(mk != 0);
            if (!any) break;
            const int src = __builtin_ctzll(any);
            const uint64_t bits = __shfl(mk, src);
            const int l = __builtin_ctzll(bits);
            if (lane == src) mk &= mk - 1;
            // stage alpha rows l*k .. l*k+k-1 and the feature row of row r0+src
            float* dst = sfix + g * per;
            const float* asrc = a.alpha + (int64_t)l * k * D;
#pragma unroll 8
            for (int e = lane; e < k * D; e += 64) dst[e] = asrc[e];
            const float* vsrc = a.feat + (r0 + src) * D;
            for (int e = lane; e < D; e += 64) dst[k * D + e] = vsrc[e];
            if (grp == g) {
                src_mine = src;
                l_mine = l;
            }
            ++got;
        }
        if (got == 0) break;
        __syncthreads();
        const bool act = grp < got;
        const int64_t row = r0 + src_mine;
        int32_t c = 0;
        if (act) {
            const int hrow = l_mine * k + jj;
            const float* ar = sfix + grp * per + jj * D;
            const float* vr = sfix + grp * per + k * D;
            double s = 0.0;
#pragma unroll 4
            for (int i = 0; i < D; ++i) s = s + (double)ar[i] * (double)vr[i];
            c = floor_sat((s + (double)a.beta[hrow]) / wd);
            if (a.codes) a.codes[row * m + hrow] = c;
        }
        uint64_t h = a.key_mul[l_mine * (k + 1) + k];
        const int base = act ? grp * k : 0;
        for (int j = 0; j < k; ++j) h += key_term(__shfl(c, base + j), a.key_mul[l_mine * (k + 1) + j]);
        if (act && jj == 0) a.keys[key_pos(a, row, l_mine)] = key_final(h);
        __syncthreads();
    }
}

// Bin (offset, count) of every key, keys and bins table by table: blocks of
// one table run together, so the lookups of the whole chip go to one
// table's directory at a time (it stays in the last-level cache). A thread
// takes kProbeRows rows of a block's kProbeRows * 256 and keeps their
// lookups in flight together: keys, then filter words, then the first
// directory slot of each key the filter lets through; a key that meets
// neither itself nor an empty slot there walks on alone.
constexpr int kProbeRows = 4;
__global__ __launch_bounds__(256) void k_probe(const uint64_t* __restrict__ keys, int64_t n, int L,
                                               const Slot* __restrict__ dir, uint64_t cap,
                                               const uint32_t* __restrict__ filter, uint2* __restrict__ bins) {
    const uint64_t fw = dir_filter_words(cap);
    const uint64_t mask = cap - 1;
    const int64_t span = 256 * kProbeRows;
    const int64_t bpt = (n + span - 1) / span;   // blocks per table
    for (int64_t b = blockIdx.x; b < bpt * L; b += gridDim.x) {
        const int l = (int)(b / bpt);
        const int64_t row0 = (b - l * bpt) * span + threadIdx.x;
        const Slot* dl = dir + (uint64_t)l * cap;
        const uint32_t* fl = filter + (uint64_t)l * fw;
        uint64_t key[kProbeRows];
        uint32_t fword[kProbeRows];
        uint4 e[kProbeRows];
#pragma unroll
        for (int j = 0; j < kProbeRows; ++j) {
            const int64_t row = row0 + 256 * j;
            key[j] = row < n ? keys[(int64_t)l * n + row] : kEmptyKey;
        }
#pragma unroll
        for (int j = 0; j < kProbeRows; ++j) fword[j] = key[j] != kEmptyKey ? fl[dir_filter_bit(key[j], cap) >> 5] : 0u;
#pragma unroll
        for (int j = 0; j < kProbeRows; ++j) {
            e[j] = make_uint4(0u, 0u, 0u, 0u);
            if ((fword[j] >> (dir_filter_bit(key[j], cap) & 31)) & 1u)
                e[j] = *reinterpret_cast<const uint4*>(dl + (key[j] & mask));
        }
#pragma unroll
        for (int j = 0; j < kProbeRows; ++j) {
            const int64_t row = row0 + 256 * j;
            if (row >= n) continue;
            uint32_t off = 0, cnt = 0;
            if ((fword[j] >> (dir_filter_bit(key[j], cap) & 31)) & 1u) {
                const uint64_t k0 = ((uint64_t)e[j].y << 32) | e[j].x;
                if (k0 == key[j]) {
                    cnt = e[j].z;
                    off = e[j].w;
                } else if (k0 != kEmptyKey) {
                    probe_bin_from(dl, cap, key[j], ((key[j] & mask) + 1) & mask, off, cnt);
                }
            }
            bins[(int64_t)l * n + row] = make_uint2(off, cnt);
        }
    }
}

// Error bound of the fp32 code value P against the exact (S + beta) / w,
// S = sum_i alpha_i v_i, from the MFMA sums S~ and S_abs (the MFMA value of
// sum |a_i||v_i| over the operands' high parts). u = 2^-24, n the fp32
// additions of one dot product (counted twice for safety).
//   fp32 path, P = fl(fl(S~ + beta) * fl(1/w)): |S~ - S| <= gamma_n
//     sum|alpha_i v_i|, sum <= S_abs / (1 - gamma); the add, the reciprocal
//     and the multiply add 3.1 u (|S~| + |beta|) / w.
//   split path, P = fl(S~ + beta'), alpha' = fl(alpha / w), beta' =
//     fl(beta / w): |S~ - sum alpha'_i v_i| <= (gamma_n 1.016 + 3.5 2^-16)
//     sum|alpha'_i v_i| (the dropped low x low and rounding-residual
//     products contribute at most 3.1 2^-16), the rounding of alpha / w adds
//     u (1 + u) of the same sum and that of beta / w u / (1 - u) |beta'|;
//     the final add u / (1 - u) |P| with |P| <= (1 + u) ((1 + E) sum + |beta'|);
//     sum|alpha'_i v_i| <= S_abs / ((1 - 2^-8)^2 (1 - gamma)). All of it is
//     c1 S_abs + c0_j (c2 = 0): one fused multiply-add a code.
// Every term is doubled, and the FP64 sequential sum of the definition is
// within ~1e-13 of the exact value, far inside the margin.
void hash_bound_coeffs(int prec, int D, double w, const float* beta, int m, float* c0, float* c1,
                       float* c2) {
    const double u = 1.0 / 16777216.0;
    const int DP = prec == 0 ? ((D + 3) & ~3) : ((D + 31) & ~31);
    const int nadd = prec == 0 ? 2 * DP : 2 * 3 * DP;
    const double g = gamma_n(nadd, u);
    const double up = 1.0 + 1e-6;
    if (prec == 0) {
        const double c_abs = 1.0 / (1.0 - gamma_n(2 * DP, u));
        *c1 = (float)(2.0 * g * c_abs / w * up);
        *c2 = (float)(2.0 * 3.1 * u / w * up);
        for (int j = 0; j < m; ++j) c0[j] = (float)((2.0 * 3.1 * u * std::fabs((double)beta[j]) / w + 1e-30) * up);
        return;
    }
    const double t = 1.0 - 1.0 / 256.0;
    const double c_abs = 1.0 / (t * t * (1.0 - gamma_n(2 * DP, u)));
    const double E = g * 1.016 + 3.5 / 65536.0 + u * (1.0 + u);
    const double e2 = u / (1.0 - u);
    *c1 = (float)(2.0 * c_abs * (E + e2 * (1.0 + u) * (1.0 + E)) * up);
    *c2 = 0.0f;
    for (int j = 0; j < m; ++j) {
        const double bw = std::fabs((double)(beta[j] / (float)w));
        c0[j] = (float)((2.0 * (e2 + e2 * (1.0 + u)) * bw + 1e-30) * up);
    }
}

// Split path: two 16-row tiles per wave when the fold group of four tables
// splits into two (k <= 24), else one.
template <int NS>
static void launch_split(const HashArgs& a, size_t lds, hipStream_t st) {
    const int nc = 2 * kStage * a.k * 4 * NS;
    const int rt = fold_tables(a.k) == 4 ? 2 : 1;
    const int rows = kWaves * kRowsPerWave * rt;
    const dim3 grid((unsigned)((a.n + rows - 1) / rows));
    if (rt == 2) {
        if (nc <= 5 * 256)
            hipLaunchKernelGGL((k_hash<1, NS, 5, 2>), grid, dim3(256), lds, st, a);
        else
            hipLaunchKernelGGL((k_hash<1, NS, 8, 2>), grid, dim3(256), lds, st, a);
    } else {
        if (nc <= 5 * 256)
            hipLaunchKernelGGL((k_hash<1, NS, 5, 1>), grid, dim3(256), lds, st, a);
        else
            hipLaunchKernelGGL((k_hash<1, NS, 8, 1>), grid, dim3(256), lds, st, a);
    }
}

hipError_t launch_hash(const HashArgs& a, hipStream_t st) {
    const hipError_t e = launch_hash_codes(a, st);
    if (e != hipSuccess || !a.bins) return e;
    return launch_probe(a, st);
}

hipError_t launch_probe(const HashArgs& a, hipStream_t st) {
    if (a.n == 0 || !a.bins) return hipSuccess;
    if (!a.keys_tmajor || !a.dir || !a.dir_filter) return hipErrorInvalidValue;
    const int64_t total = a.n * a.L;
    int64_t g = (total + 256 * kProbeRows - 1) / (256 * kProbeRows);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_probe, dim3((unsigned)g), dim3(256), 0, st, a.keys, a.n, a.L, a.dir, a.dir_cap,
                       a.dir_filter, a.bins);
    return hipGetLastError();
}

hipError_t launch_hash_codes(const HashArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    if (a.D < 1 || a.D > 128 || a.k < 1 || a.k > 32 || a.L < 1 || a.L > 64 || !a.dirty || !a.fix_count || !a.key_mul ||
        a.fix_cap < 0 || a.fix_cap > kFixSlots || (a.fix_cap > 0 && !a.fix_list) ||
        (a.bins && (!a.keys_tmajor || !a.dir || !a.dir_filter)))
        return hipErrorInvalidValue;
    const size_t lds = (size_t)stage_bytes(a.prec, a.k, a.D) +
                       (size_t)kWaves * fold_tables(a.k) * a.k * kRowsPerWave * 4 + kWaves * 4 * kRowsPerWave +
                       sizeof(uint64_t) * (size_t)a.L * (a.k + 1);
    if (a.prec == 0) {
        const int rows = kWaves * kRowsPerWave;
        const dim3 grid((unsigned)((a.n + rows - 1) / rows));
        hipLaunchKernelGGL((k_hash<0, 1, 1, 1>), grid, dim3(256), lds, st, a);
    } else {
        switch ((a.D + 31) / 32) {
            case 1: launch_split<1>(a, lds, st); break;
            case 2: launch_split<2>(a, lds, st); break;
            case 3: launch_split<3>(a, lds, st); break;
            default: launch_split<4>(a, lds, st); break;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t slots = (a.n + kRowsPerWave - 1) / kRowsPerWave * a.fix_cap;
    if (slots > 0) {
        const int64_t gl = (slots + 255) / 256;
        hipLaunchKernelGGL(k_hash_fixlist, dim3((unsigned)(gl < 8192 ? gl : 8192)), dim3(256), 0, st, a);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 gfix((unsigned)((a.n + 63) / 64));
    const size_t lfix = (size_t)fix_groups(a.k) * (a.k + 1) * a.D * sizeof(float);
    hipLaunchKernelGGL(k_hash_fix, gfix, dim3(64), lfix, st, a);
    return hipGetLastError();
}

}  // namespace zh
