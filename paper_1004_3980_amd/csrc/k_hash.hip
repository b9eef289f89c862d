// Projection, p-stable codes and bucket keys (Section 4.1, Eq. hash_fn;
// Section 3.2: k concatenated hashes per table, L tables).
//
//   code_j(v) = floor((alpha_j . v + beta_j) / w)
//
// The dot products of a tile of 64 feature rows with the k hashes of one
// table run on the matrix cores, either as fp32 MFMA or as three bf16 MFMAs
// over a high/low split of both operands (alpha = a_hi + a_lo, v = v_hi +
// v_lo; the products a_hi v_hi + a_hi v_lo + a_lo v_hi accumulate in fp32).
// A rigorous bound B on |P_mfma - P_exact| decides each floor: when the
// interval [P - B, P + B] holds no integer the MFMA code is the exact code;
// otherwise the code is recomputed by the FP64 sequential dot product that
// defines it. The result therefore equals the FP64 definition bit for bit.
//
// The k codes of a table are folded into a 64-bit key in index order:
//   h = fmix64(GOLDEN*(l+1)); h = fmix64(h ^ uint32(c_j)) for j = 0..k-1.
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

template <int PREC>
__global__ __launch_bounds__(256) void k_hash(HashArgs a) {
    const int D = a.D;
    const int DP = PREC == 0 ? ((D + 3) & ~3) : ((D + 31) & ~31);
    const int DPS = DP + 1;                 // padded LDS row stride
    const int KP = a.k <= 16 ? 16 : 32;     // hashes per table rounded to MFMA tiles
    const int m = a.L * a.k;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * kHashBQ;

    extern __shared__ float smem[];
    float* sfeat = smem;                                  // [64][DPS]
    float* snorm = sfeat + kHashBQ * DPS;                 // [64]
    float* sP = snorm + kHashBQ + wave * (a.k * kHashBQ);  // per wave [k][64]

    for (int t = threadIdx.x; t < kHashBQ * DP; t += blockDim.x) {
        const int r = t / DP, c = t % DP;
        const int64_t q = q0 + r;
        sfeat[r * DPS + c] = (q < a.n && c < D) ? a.feat[q * D + c] : 0.0f;
    }
    __syncthreads();
    if (threadIdx.x < kHashBQ) {
        float s = 0.0f;
        for (int c = 0; c < D; ++c) s = fmaf(sfeat[threadIdx.x * DPS + c], sfeat[threadIdx.x * DPS + c], s);
        snorm[threadIdx.x] = sqrtf(s);
    }
    __syncthreads();

    const double u32 = 1.0 / 16777216.0;
    const double cb = PREC == 0 ? 2.0 * gamma_n(DP + 2, u32)
                                : 2.0 * (gamma_n(3 * DP + 2, u32) + 3.5 / 65536.0);
    const double wd = (double)a.w;
    const int iters = (a.L + kHashWaves - 1) / kHashWaves;
    const int ri = lane & 15, kb = lane >> 4;

    for (int it = 0; it < iters; ++it) {
        const int l = it * kHashWaves + wave;
        if (l < a.L) {
            f32x4 acc[2][4];
#pragma unroll
            for (int ht = 0; ht < 2; ++ht)
#pragma unroll
                for (int qt = 0; qt < 4; ++qt) acc[ht][qt] = f32x4{0.f, 0.f, 0.f, 0.f};
            const int nht = KP / 16;
            if (PREC == 0) {
                for (int d0 = 0; d0 < DP; d0 += 4) {
                    const int d = d0 + kb;
                    float bv[4];
#pragma unroll
                    for (int qt = 0; qt < 4; ++qt) bv[qt] = sfeat[(qt * 16 + ri) * DPS + d];
#pragma unroll
                    for (int ht = 0; ht < 2; ++ht) {
                        if (ht >= nht) break;
                        const int j = ht * 16 + ri;
                        const float av = (j < a.k && d < D) ? a.alpha[(int64_t)(l * a.k + j) * D + d] : 0.0f;
#pragma unroll
                        for (int qt = 0; qt < 4; ++qt)
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[qt], acc[ht][qt], 0, 0, 0);
                    }
                }
            } else {
                for (int d0 = 0; d0 < DP; d0 += 32) {
                    const int d = d0 + 8 * kb;
                    u16x8 vh[4], vl[4];
#pragma unroll
                    for (int qt = 0; qt < 4; ++qt) {
                        const float* src = sfeat + (qt * 16 + ri) * DPS + d;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const float x = src[e];
                            const uint16_t h = bf16_rne(x);
                            vh[qt][e] = h;
                            vl[qt][e] = bf16_rne(x - bf16_to_f(h));
                        }
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
#pragma unroll
                        for (int qt = 0; qt < 4; ++qt) {
                            const bf16x8 vhb = __builtin_bit_cast(bf16x8, vh[qt]);
                            const bf16x8 vlb = __builtin_bit_cast(bf16x8, vl[qt]);
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahb, vhb, acc[ht][qt], 0, 0, 0);
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahb, vlb, acc[ht][qt], 0, 0, 0);
                            acc[ht][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alb, vhb, acc[ht][qt], 0, 0, 0);
                        }
                    }
                }
            }
            // D layout of a 16x16 MFMA tile: lane holds rows 4*(lane/16)+i, column lane%16
#pragma unroll
            for (int ht = 0; ht < 2; ++ht) {
                if (ht >= nht) break;
#pragma unroll
                for (int qt = 0; qt < 4; ++qt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int j = ht * 16 + 4 * kb + i;
                        if (j < a.k) sP[j * kHashBQ + qt * 16 + ri] = acc[ht][qt][i];
                    }
            }
        }
        __syncthreads();
        if (l < a.L) {
            const int qi = lane;
            const int64_t q = q0 + qi;
            if (q < a.n) {
                const double vn = (double)snorm[qi] * (1.0 + 1e-6);
                uint64_t h = key_seed(l);
                for (int j = 0; j < a.k; ++j) {
                    const int row = l * a.k + j;
                    const float S = sP[j * kHashBQ + qi];
                    const float bj = a.beta[row];
                    const float P = (S + bj) / a.w;
                    const double B = cb * ((double)a.anorm[row] * vn + fabs((double)bj)) / wd + 1e-35;
                    const double lo = floor((double)P - B), hi = floor((double)P + B);
                    int32_t c;
                    if (lo == hi) {
                        c = floor_sat((double)P);
                    } else {
                        // FP64 sequential dot product, index order (the definition)
                        const float* ar = a.alpha + (int64_t)row * D;
                        double s = 0.0;
                        for (int i = 0; i < D; ++i) s = s + (double)ar[i] * (double)sfeat[qi * DPS + i];
                        c = floor_sat((s + (double)bj) / wd);
                        if (a.n_fixed) atomicAdd(a.n_fixed, 1u);
                    }
                    if (a.codes) a.codes[q * m + row] = c;
                    h = key_step(h, c);
                }
                a.keys[q * a.L + l] = key_final(h);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_hash(const HashArgs& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    const int DP = a.prec == 0 ? ((a.D + 3) & ~3) : ((a.D + 31) & ~31);
    const size_t lds = sizeof(float) * ((size_t)kHashBQ * (DP + 1) + kHashBQ + (size_t)kHashWaves * a.k * kHashBQ);
    const dim3 grid((unsigned)((a.n + kHashBQ - 1) / kHashBQ));
    if (a.prec == 0)
        hipLaunchKernelGGL(k_hash<0>, grid, dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL(k_hash<1>, grid, dim3(256), lds, st, a);
    return hipGetLastError();
}

}  // namespace zh
