// Projection, p-stable codes and bucket keys (Section 4.1, Eq. hash_fn;
// Section 3.2: k concatenated hashes per table, L tables).
//
//   code_j(v) = floor((alpha_j . v + beta_j) / w)
//
// The dot products of a tile of 64 feature rows with the k hashes of one
// table run on the matrix cores, either as fp32 MFMA or as three bf16 MFMAs
// over a high/low split of both operands (alpha = a_hi + a_lo, v = v_hi +
// v_lo; the products a_hi v_hi + a_hi v_lo + a_lo v_hi accumulate in fp32).
// A fourth product of the absolute values bounds sum_i |alpha_i v_i|, which
// gives a rigorous bound B on |P_mfma - P_exact|; when [P - B, P + B] holds
// no integer the MFMA floor is the exact code, otherwise the code is
// recomputed by the FP64 sequential dot product that defines it (all lanes of
// a wave re-evaluate the flagged codes together). The codes therefore equal
// the FP64 definition bit for bit.
//
// The k codes of a table are folded into a 64-bit key in index order:
//   h = fmix64(GOLDEN*(l+1)); h = fmix64(h ^ uint32(c_j)) for j = 0..k-1.
#include <cmath>

#include "zh_internal.h"

namespace zh {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kHashBQ = 64;   // feature rows per workgroup
constexpr int kHashWaves = 4;

__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int32_t floor_sat(double t) {
    const double f = floor(t);
    if (f >= 2147483647.0) return 2147483647;
    if (f <= -2147483648.0) return (int32_t)0x80000000;
    return (int32_t)f;
}

__device__ __forceinline__ u16x8 abs8(u16x8 x) {
    const u16x8 m = {0x7FFF, 0x7FFF, 0x7FFF, 0x7FFF, 0x7FFF, 0x7FFF, 0x7FFF, 0x7FFF};
    return x & m;
}

// Bound coefficients, per hash: B = c1 * S_abs + c2 * |S| + c0[j] with
// S_abs the MFMA value of sum |alpha_hi_i| |v_hi_i| (or of sum |alpha_i||v_i|
// on the fp32 path). Computed on the host, rounded up.
template <int PREC>
__global__ __launch_bounds__(256) void k_hash(HashArgs a) {
    const int D = a.D;
    const int DP = PREC == 0 ? ((D + 3) & ~3) : ((D + 31) & ~31);
    const int KP = a.k <= 16 ? 16 : 32;
    const int m = a.L * a.k;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * kHashBQ;

    extern __shared__ float smem[];
    // fp32 path: sfeat [64][DP+1] floats; split path: vh, vl [64][DP] bf16
    float* sfeat = smem;
    uint16_t* vh = reinterpret_cast<uint16_t*>(smem);
    uint16_t* vl = vh + kHashBQ * DP;
    const int feat_words = PREC == 0 ? kHashBQ * (DP + 1) : kHashBQ * DP;  // 32-bit words
    int32_t* sC = reinterpret_cast<int32_t*>(smem + feat_words) + wave * (a.k * kHashBQ);  // per wave [k][64]
    uint16_t* flist = reinterpret_cast<uint16_t*>(smem + feat_words + kHashWaves * a.k * kHashBQ) +
                      wave * (a.k * kHashBQ);

    for (int t = threadIdx.x; t < kHashBQ * DP; t += blockDim.x) {
        const int r = t / DP, c = t % DP;
        const int64_t q = q0 + r;
        const float x = (q < a.n && c < D) ? a.feat[q * D + c] : 0.0f;
        if (PREC == 0) {
            sfeat[r * (DP + 1) + c] = x;
        } else {
            const uint16_t h = bf16_rne(x);
            vh[r * DP + c] = h;
            vl[r * DP + c] = bf16_rne(x - bf16_to_f(h));
        }
    }
    __syncthreads();

    const int iters = (a.L + kHashWaves - 1) / kHashWaves;
    const int ri = lane & 15, kb = lane >> 4;
    const float c1 = a.bound_c1, c2 = a.bound_c2;
    const double wd = (double)a.w;

    for (int it = 0; it < iters; ++it) {
        const int l = it * kHashWaves + wave;
        int nflag = 0;
        if (l < a.L) {
            f32x4 acc[2][4], aab[2][4];
#pragma unroll
            for (int ht = 0; ht < 2; ++ht)
#pragma unroll
                for (int qt = 0; qt < 4; ++qt) {
                    acc[ht][qt] = f32x4{0.f, 0.f, 0.f, 0.f};
                    aab[ht][qt] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
            const int nht = KP / 16;
            if (PREC == 0) {
                for (int d0 = 0; d0 < DP; d0 += 4) {
                    const int d = d0 + kb;
                    float bv[4];
#pragma unroll
                    for (int qt = 0; qt < 4; ++qt) bv[qt] = sfeat[(qt * 16 + ri) * (DP + 1) + d];
#pragma unroll
                    for (int ht = 0; ht < 2; ++ht) {
                        if (ht >= nht) break;
                        const int j = ht * 16 + ri;
                        const float av = (j < a.k && d < D) ? a.alpha[(int64_t)(l * a.k + j) * D + d] : 0.0f;
#pragma unroll
                        for (int qt = 0; qt < 4; ++qt) {
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[qt], acc[ht][qt], 0, 0, 0);
                            aab[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fabsf(av), fabsf(bv[qt]), aab[ht][qt], 0, 0, 0);
                        }
                    }
                }
            } else {
                for (int d0 = 0; d0 < DP; d0 += 32) {
                    const int d = d0 + 8 * kb;
                    u16x8 xh[4], xl[4];
#pragma unroll
                    for (int qt = 0; qt < 4; ++qt) {
                        xh[qt] = *reinterpret_cast<const u16x8*>(vh + (qt * 16 + ri) * DP + d);
                        xl[qt] = *reinterpret_cast<const u16x8*>(vl + (qt * 16 + ri) * DP + d);
                    }
#pragma unroll
                    for (int ht = 0; ht < 2; ++ht) {
                        if (ht >= nht) break;
                        const int j = ht * 16 + ri;
                        u16x8 ah = u16x8{0, 0, 0, 0, 0, 0, 0, 0}, al = ah;
                        if (j < a.k) {
                            const int64_t off = (int64_t)(l * a.k + j) * DP + d;
                            ah = *reinterpret_cast<const u16x8*>(a.a_hi + off);
                            al = *reinterpret_cast<const u16x8*>(a.a_lo + off);
                        }
                        const bf16x8 ahb = __builtin_bit_cast(bf16x8, ah);
                        const bf16x8 alb = __builtin_bit_cast(bf16x8, al);
                        const bf16x8 aab8 = __builtin_bit_cast(bf16x8, abs8(ah));
#pragma unroll
                        for (int qt = 0; qt < 4; ++qt) {
                            const bf16x8 vhb = __builtin_bit_cast(bf16x8, xh[qt]);
                            const bf16x8 vlb = __builtin_bit_cast(bf16x8, xl[qt]);
                            const bf16x8 vab = __builtin_bit_cast(bf16x8, abs8(xh[qt]));
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahb, vhb, acc[ht][qt], 0, 0, 0);
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahb, vlb, acc[ht][qt], 0, 0, 0);
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alb, vhb, acc[ht][qt], 0, 0, 0);
                            aab[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aab8, vab, aab[ht][qt], 0, 0, 0);
                        }
                    }
                }
            }
            // D layout of a 16x16 MFMA tile: lane holds rows 4*(lane/16)+i, column
            // lane%16. Decide every code whose bin is certain; list the others.
#pragma unroll
            for (int ht = 0; ht < 2; ++ht) {
                if (ht >= nht) break;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = ht * 16 + 4 * kb + i;
                    const int row = l * a.k + (j < a.k ? j : 0);
                    const float bj = a.beta[row], c0 = a.bound_c0[row];
#pragma unroll
                    for (int qt = 0; qt < 4; ++qt) {
                        const int qi = qt * 16 + ri;
                        const bool valid = j < a.k && q0 + qi < a.n;
                        const float S = acc[ht][qt][i];
                        const float P = (S + bj) * a.inv_w;
                        const float B = fmaf(c1, aab[ht][qt][i], fmaf(c2, fabsf(S), c0));
                        const float n = rintf(P);
                        const bool flag = !(fabsf(P - n) > B) || !(fabsf(P) < 4194304.0f);
                        const uint64_t fm = __ballot(flag && valid);
                        if (flag && valid) flist[nflag + __popcll(fm & lanemask_lt())] = (uint16_t)((j << 6) | qi);
                        nflag += __popcll(fm);
                        if (valid) sC[j * kHashBQ + qi] = flag ? 0 : (int32_t)floorf(P);
                    }
                }
            }
        }
        __syncthreads();
        if (l < a.L) {
            // FP64 sequential dot products of the flagged codes, one per lane
            for (int f = lane; f < nflag; f += 64) {
                const int e = flist[f];
                const int j = e >> 6, qi = e & 63;
                const int row = l * a.k + j;
                const float* ar = a.alpha + (int64_t)row * D;
                const float* vr = a.feat + (q0 + qi) * D;
                double s = 0.0;
#pragma unroll 10
                for (int i = 0; i < D; ++i) s = s + (double)ar[i] * (double)vr[i];
                sC[j * kHashBQ + qi] = floor_sat((s + (double)a.beta[row]) / wd);
            }
            if (lane == 0 && nflag && a.n_fixed) atomicAdd(a.n_fixed, (unsigned)nflag);
        }
        __syncthreads();
        if (l < a.L) {
            const int qi = lane;
            const int64_t q = q0 + qi;
            if (q < a.n) {
                uint64_t h = key_seed(l);
                for (int j = 0; j < a.k; ++j) {
                    const int32_t c = sC[j * kHashBQ + qi];
                    if (a.codes) a.codes[q * m + l * a.k + j] = c;
                    h = key_step(h, c);
                }
                a.keys[q * a.L + l] = key_final(h);
            }
        }
        __syncthreads();
    }
}

// Error bound of the fp32 code value P = fl(fl(S~ + beta) * fl(1/w)) against
// the exact (S + beta)/w, S = sum_i alpha_i v_i, from the MFMA sums S~ and
// S_abs (the MFMA value of sum |alpha_i||v_i|, from the bf16 high parts on
// the split path). With u = 2^-24 and n the fp32 additions of one dot
// product (counted twice for safety):
//   split bf16: |S~ - S| <= (gamma_n 1.016 + 3.5 2^-16) sum|alpha_i v_i|,
//     the dropped low x low and rounding-residual products contributing at
//     most 3.1 2^-16 relative; sum|alpha_i||v_i| <= S_abs / ((1-2^-8)^2 (1-gamma))
//   fp32: |S~ - S| <= gamma_n sum|alpha_i v_i|, sum <= S_abs / (1 - gamma)
//   the add, the reciprocal and the multiply add 3.1 u (|S~| + |beta|) / w.
// Every term is doubled, and the FP64 sequential sum of the definition is
// within ~1e-13 of the exact value, far inside the margin.
void hash_bound_coeffs(int prec, int D, double w, const float* beta, int m, float* c0, float* c1,
                       float* c2) {
    const double u = 1.0 / 16777216.0;
    const int DP = prec == 0 ? ((D + 3) & ~3) : ((D + 31) & ~31);
    const int nadd = prec == 0 ? 2 * DP : 2 * 3 * DP;
    const double g = gamma_n(nadd, u);
    double e_rel, c_abs;
    if (prec == 0) {
        e_rel = g;
        c_abs = 1.0 / (1.0 - gamma_n(2 * DP, u));
    } else {
        e_rel = g * 1.016 + 3.5 / 65536.0;
        const double t = 1.0 - 1.0 / 256.0;
        c_abs = 1.0 / (t * t * (1.0 - gamma_n(2 * DP, u)));
    }
    const double up = 1.0 + 1e-6;
    *c1 = (float)(2.0 * e_rel * c_abs / w * up);
    *c2 = (float)(2.0 * 3.1 * u / w * up);
    for (int j = 0; j < m; ++j) c0[j] = (float)((2.0 * 3.1 * u * std::fabs((double)beta[j]) / w + 1e-30) * up);
}

size_t hash_lds_bytes(int prec, int D, int k) {
    const int DP = prec == 0 ? ((D + 3) & ~3) : ((D + 31) & ~31);
    const size_t feat_words = prec == 0 ? (size_t)kHashBQ * (DP + 1) : (size_t)kHashBQ * DP;
    return 4 * (feat_words + (size_t)kHashWaves * k * kHashBQ) + 2 * (size_t)kHashWaves * k * kHashBQ;
}

hipError_t launch_hash(const HashArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    const size_t lds = hash_lds_bytes(a.prec, a.D, a.k);
    const dim3 grid((unsigned)((a.n + kHashBQ - 1) / kHashBQ));
    if (a.prec == 0)
        hipLaunchKernelGGL(k_hash<0>, grid, dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL(k_hash<1>, grid, dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace zh
