// Dictionary-construction tools, off the per-image path.
//
// Training crops (Section 5, training data generation): every pixel of a
// training image weighs its first-order gradient (taps [-1, 0, 1] along each
// axis, replicate border), |dx| + |dy| in FP64 from the fp32 pixels,
// quantised to q = floor(g 2^20) (saturated at 2^32 - 1, also for non-finite
// g), so the cumulative distribution is an exact integer sum in any order.
// A 64-bit draw x picks the first pixel (row-major) whose inclusive
// cumulative weight exceeds x mod T (T the image's total; x mod (H W) when
// T = 0); the crop of side S around it has its top-left corner at the centre
// minus S / 2, clamped inside the image.
//
// Hashing quality (Section 4.1, determining r): the entropy in bits of each
// table's bucket occupancy, -sum_b p_b log2 p_b, p_b = (rows in bucket b) / N,
// read from the bin directory.
#include <cmath>

#include "zh_internal.h"

namespace zh {

constexpr int kCdfBlock = 1024;   // pixels per block of cumulative weights
constexpr int kCdfSub = kCdfBlock / 64;   // sub-blocks of 64 pixels per block

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline unsigned long long wave_incl_scan_u64(unsigned long long v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ inline uint32_t grad_weight(const float* __restrict__ img, int H, int W, int r, int c) {
    const double dx = (double)img[(int64_t)r * W + min(c + 1, W - 1)] - (double)img[(int64_t)r * W + max(c - 1, 0)];
    const double dy = (double)img[(int64_t)min(r + 1, H - 1) * W + c] - (double)img[(int64_t)max(r - 1, 0) * W + c];
    const double s = (fabs(dx) + fabs(dy)) * 1048576.0;
    return s < 4294967295.0 ? (uint32_t)floor(s) : 0xFFFFFFFFu;
}

// Sum of the weights of block blockIdx.x of image blockIdx.y (bsum) and of
// each of its 16 sub-blocks of 64 pixels (ssum). The weights themselves are
// not stored: the sampler recomputes the 64 of the sub-block it lands in.
__global__ __launch_bounds__(256) void k_cdf_weights(const float* __restrict__ imgs, int H, int W, int nb,
                                                     unsigned long long* __restrict__ bsum,
                                                     unsigned long long* __restrict__ ssum) {
    __shared__ unsigned long long ws[4];
    const int HW = H * W;
    const float* img = imgs + (int64_t)blockIdx.y * HW;
    const int p0 = blockIdx.x * kCdfBlock;
    unsigned long long acc = 0;
    unsigned long long* sub = ssum + ((int64_t)blockIdx.y * nb + blockIdx.x) * kCdfSub;
#pragma unroll
    for (int u = 0; u < kCdfBlock / 256; ++u) {
        const int p = p0 + (int)threadIdx.x + 256 * u;
        unsigned long long v = 0;
        if (p < HW) {
            const int r = p / W;
            v = grad_weight(img, H, W, r, p - r * W);
        }
        // the wave's 64 lanes hold one sub-block (pixels 256 u + 64 w ..)
        v = wave_sum_u64(v);
        if (__lane_id() == 0) sub[4 * u + (threadIdx.x >> 6)] = v;
        acc += v;
    }
    if (__lane_id() == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) bsum[(int64_t)blockIdx.y * nb + blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive prefix of the block sums of image blockIdx.x: bpre[0 .. nb], the
// last entry the image's total. One workgroup per image, 256 sums a pass.
__global__ __launch_bounds__(256) void k_cdf_scan(const unsigned long long* __restrict__ bsum, int nb,
                                                  unsigned long long* __restrict__ bpre) {
    __shared__ unsigned long long wt[4];
    const unsigned long long* in = bsum + (int64_t)blockIdx.x * nb;
    unsigned long long* out = bpre + (int64_t)blockIdx.x * (nb + 1);
    unsigned long long carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const unsigned long long v = b < nb ? in[b] : 0ull;
        const unsigned long long incl = wave_incl_scan_u64(v);
        if (__lane_id() == 63) wt[threadIdx.x >> 6] = incl;
        __syncthreads();
        unsigned long long before = carry;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) before += wt[w];
        if (b < nb) out[b] = before + incl - v;
        carry += wt[0] + wt[1] + wt[2] + wt[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[nb] = carry;
}

// One wave per draw: the centre pixel, then the clamped crop corner.
__global__ __launch_bounds__(256) void k_cdf_sample(const float* __restrict__ imgs,
                                                    const unsigned long long* __restrict__ bpre,
                                                    const unsigned long long* __restrict__ ssum, int H, int W, int nb,
                                                    const unsigned long long* __restrict__ draws, int64_t n_draws,
                                                    int m, int side, int32_t* __restrict__ corners) {
    const int lane = __lane_id();
    const int64_t d = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (d >= n_draws) return;
    const int64_t img = d / m;
    const int HW = H * W;
    const unsigned long long* pre = bpre + img * (nb + 1);
    const unsigned long long T = pre[nb], x = draws[d];
    int64_t centre = -1;
    if (T == 0) {
        centre = (int64_t)(x % (unsigned long long)HW);
    } else {
        const unsigned long long t = x % T;
        // last block whose exclusive prefix is <= t (pre[0] = 0)
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        unsigned long long tl = t - pre[lo];
        // the sub-block of 64 pixels holding tl, then the pixel inside it
        const unsigned long long sv = lane < kCdfSub ? ssum[(img * nb + lo) * kCdfSub + lane] : 0ull;
        const unsigned long long sincl = wave_incl_scan_u64(sv);
        const uint64_t shit = __ballot(sincl > tl);
        const int sb = shit ? __builtin_ctzll(shit) : kCdfSub - 1;
        tl -= __shfl(sincl - sv, sb);
        const int p = lo * kCdfBlock + sb * 64 + lane;
        const float* im = imgs + img * HW;
        unsigned long long q = 0;
        if (p < HW) {
            const int r = p / W;
            q = grad_weight(im, H, W, r, p - r * W);
        }
        const unsigned long long incl = wave_incl_scan_u64(q);
        const uint64_t hit = __ballot(incl > tl);
        const int src = hit ? __builtin_ctzll(hit) : 63;
        centre = (int64_t)lo * kCdfBlock + sb * 64 + src;
    }
    if (lane == 0) {
        const int r = (int)(centre / W), c = (int)(centre - (int64_t)(centre / W) * W);
        corners[2 * d] = min(max(r - side / 2, 0), H - side);
        corners[2 * d + 1] = min(max(c - side / 2, 0), W - side);
    }
}

// One workgroup per crop.
__global__ __launch_bounds__(256) void k_crop_cut(const float* __restrict__ imgs, int H, int W, int m, int side,
                                                  const int32_t* __restrict__ corners, float* __restrict__ crops) {
    const int64_t d = blockIdx.x;
    const int ss = side * side;
    const float* src = imgs + (d / m) * ((int64_t)H * W) + (int64_t)corners[2 * d] * W + corners[2 * d + 1];
    float* dst = crops + d * ss;
    for (int e = threadIdx.x; e < ss; e += 256) {
        const int r = e / side;
        dst[e] = src[(int64_t)r * W + (e - r * side)];
    }
}

int64_t crop_scratch_bytes(int n_img, int H, int W) {
    const int64_t HW = (int64_t)H * W, nb = (HW + kCdfBlock - 1) / kCdfBlock;
    return (int64_t)n_img * (8 * nb + 8 * (nb + 1) + 8 * kCdfSub * nb);
}

hipError_t launch_sample_crops(const float* imgs, int n_img, int H, int W, const uint64_t* draws, int m, int side,
                               int32_t* corners, float* crops, void* scratch, hipStream_t st) {
    const int64_t HW = (int64_t)H * W;
    const int nb = (int)((HW + kCdfBlock - 1) / kCdfBlock);
    if (n_img < 1 || n_img > 65535 || side < 1 || side > H || side > W || m < 0) return hipErrorInvalidValue;
    unsigned long long* bsum = static_cast<unsigned long long*>(scratch);
    unsigned long long* bpre = bsum + (int64_t)n_img * nb;
    unsigned long long* ssum = bpre + (int64_t)n_img * (nb + 1);
    hipLaunchKernelGGL(k_cdf_weights, dim3(nb, n_img), dim3(256), 0, st, imgs, H, W, nb, bsum, ssum);
    hipLaunchKernelGGL(k_cdf_scan, dim3(n_img), dim3(256), 0, st, bsum, nb, bpre);
    const int64_t nd = (int64_t)n_img * m;
    if (nd == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_cdf_sample, dim3((unsigned)((nd + 3) / 4)), dim3(256), 0, st, imgs, bpre, ssum, H, W, nb,
                       reinterpret_cast<const unsigned long long*>(draws), nd, m, side, corners);
    if (crops)
        hipLaunchKernelGGL(k_crop_cut, dim3((unsigned)nd), dim3(256), 0, st, imgs, H, W, m, side, corners, crops);
    return hipGetLastError();
}

// Entropy partial sums: block blockIdx.x of table blockIdx.y, 256 x 16 slots.
constexpr int kEntSlots = 4096;

__global__ __launch_bounds__(256) void k_dir_entropy(const Slot* __restrict__ dir, uint64_t cap, double n,
                                                     int nblk, double* __restrict__ part) {
    __shared__ double ws[4];
    const Slot* tab = dir + (uint64_t)blockIdx.y * cap;
    const uint64_t s0 = (uint64_t)blockIdx.x * kEntSlots;
    double acc = 0.0;
    for (int u = 0; u < kEntSlots / 256; ++u) {
        const uint64_t s = s0 + threadIdx.x + 256 * u;
        if (s < cap) {
            const Slot e = tab[s];
            if (e.key != kEmptyKey && e.count > 0) {
                const double p = (double)e.count / n;
                acc -= p * log2(p);
            }
        }
    }
    acc = wave_sum_f64(acc);
    if (__lane_id() == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * nblk + blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// Table blockIdx.x's partials: lane i adds blocks i, i + 64, ... in order,
// then a fixed-order wave sum.
__global__ __launch_bounds__(64) void k_entropy_sum(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += part[(int64_t)blockIdx.x * nblk + b];
    s = wave_sum_f64(s);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

int64_t entropy_scratch_bytes(int L, uint64_t cap) {
    const int64_t nblk = (int64_t)((cap + kEntSlots - 1) / kEntSlots);
    return 8 * ((int64_t)L * nblk + L);
}

hipError_t launch_table_entropy(const Slot* dir, int L, uint64_t cap, int64_t n, void* scratch, double* out,
                                hipStream_t st) {
    const int nblk = (int)((cap + kEntSlots - 1) / kEntSlots);
    if (L < 1 || n < 1 || nblk < 1) return hipErrorInvalidValue;
    double* part = static_cast<double*>(scratch);
    hipLaunchKernelGGL(k_dir_entropy, dim3(nblk, L), dim3(256), 0, st, dir, cap, (double)n, nblk, part);
    hipLaunchKernelGGL(k_entropy_sum, dim3(L), dim3(64), 0, st, part, nblk, out);
    return hipGetLastError();
}

}  // namespace zh

namespace zh {

// K nearest candidates under l1 (Section 4.1: the Cauchy hash is sensitive to
// l1 distances) or squared l2 (for candidate sets other than the search's,
// such as the t-of-L sets). One wave (one workgroup) per patch. Candidates go in chunks
// of 16: the wave stages their feature rows in LDS (the chunk's rows
// flattened over the lanes, 16-byte loads when D is a multiple of 4; odd row
// stride in LDS: no bank conflicts), then lane j sums the terms of candidate j
// over the coordinates in index order in FP64, so every distance is the
// oracle's to the bit. Then K rounds of a wave minimum over (distance, ID)
// pick the neighbours in order.
constexpr int kL1Chunk = 16;    // candidates staged at a time (6.5 KB of LDS at D = 100)
constexpr int kL1PerLane = 16;  // chunks: at most 256 candidates a patch
constexpr int kL1MaxD = 128;

// DT: the feature dimension at compile time (0: D at run time, up to 128).
// L1: l1 distances; otherwise squared l2, each term (q_i - x_i)^2 rounded
// before it is added, in index order, as the oracle's FP64 loop does.
template <int DT, bool L1>
__global__ __launch_bounds__(64) void k_knn_rank(int Q, int Drt, int K, int cap, const float* __restrict__ qfeat,
                                               const float* __restrict__ xf, const int32_t* __restrict__ cand,
                                               const int32_t* __restrict__ ncand, int32_t* __restrict__ out_ids,
                                               float* __restrict__ out_d, int32_t* __restrict__ out_m) {
    constexpr int kSt = (DT ? DT : kL1MaxD) | 1;
    __shared__ double sq[DT ? DT : kL1MaxD];
    __shared__ float sx[kL1Chunk * kSt];
    __shared__ int sid[kL1Chunk];
    const int D = DT ? DT : Drt;
    const int lane = threadIdx.x;
    const int q = xcd_block();
    if (q >= Q) return;
    const int M = min(ncand[q], cap);
    const int st = DT ? kSt : (D | 1);
    for (int i = lane; i < D; i += 64) sq[i] = (double)qfeat[(int64_t)q * D + i];
    double d[kL1PerLane];
    int id[kL1PerLane];
#pragma unroll
    for (int u = 0; u < kL1PerLane; ++u) {
        d[u] = INFINITY;
        id[u] = 0x7FFFFFFF;
        const int c0 = kL1Chunk * u;
        if (c0 < M) {
            const int nc = min(kL1Chunk, M - c0);
            const int myid = lane < nc ? cand[(int64_t)q * cap + c0 + lane] : 0;
            __syncthreads();
            if (lane < kL1Chunk) sid[lane] = myid;
            __syncthreads();
            // the chunk's rows, flattened over the wave, eight loads in flight a lane
            if ((D & 3) == 0) {
                const int D4 = D >> 2, n4 = nc * D4;
                const float4* x4 = reinterpret_cast<const float4*>(xf);
                for (int e0 = 0; e0 < n4; e0 += 64 * 8) {
                    float4 v[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int e = e0 + lane + 64 * t;
                        if (e < n4) {
                            const int c = e / D4;
                            v[t] = x4[(int64_t)sid[c] * D4 + (e - c * D4)];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int e = e0 + lane + 64 * t;
                        if (e < n4) {
                            const int c = e / D4;
                            float* dst = sx + c * st + 4 * (e - c * D4);
                            dst[0] = v[t].x;
                            dst[1] = v[t].y;
                            dst[2] = v[t].z;
                            dst[3] = v[t].w;
                        }
                    }
                }
            } else {
                const int n1 = nc * D;
                for (int e0 = 0; e0 < n1; e0 += 64 * 8) {
                    float v[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int e = e0 + lane + 64 * t;
                        if (e < n1) {
                            const int c = e / D;
                            v[t] = xf[(int64_t)sid[c] * D + (e - c * D)];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const int e = e0 + lane + 64 * t;
                        if (e < n1) {
                            const int c = e / D;
                            sx[c * st + (e - c * D)] = v[t];
                        }
                    }
                }
            }
            __syncthreads();
            if (lane < nc) {
                double acc = 0.0;
#pragma unroll 20
                for (int i = 0; i < D; ++i) {
                    const double t = sq[i] - (double)sx[lane * st + i];
                    acc = acc + (L1 ? fabs(t) : t * t);
                }
                d[u] = acc;
                id[u] = myid;
            }
        }
    }
    const int m = min(K, M);
    for (int k = 0; k < m; ++k) {
        // this lane's smallest (distance, ID), then the wave's
        double bd = d[0];
        int bi = id[0];
#pragma unroll
        for (int u = 1; u < kL1PerLane; ++u)
            if (d[u] < bd || (d[u] == bd && id[u] < bi)) {
                bd = d[u];
                bi = id[u];
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(bd, o);
            const int oi = __shfl_xor(bi, o);
            if (od < bd || (od == bd && oi < bi)) {
                bd = od;
                bi = oi;
            }
        }
#pragma unroll
        for (int u = 0; u < kL1PerLane; ++u)
            if (id[u] == bi) {
                d[u] = INFINITY;
                id[u] = 0x7FFFFFFF;
            }
        if (lane == 0) {
            out_ids[(int64_t)q * K + k] = bi;
            out_d[(int64_t)q * K + k] = (float)bd;
        }
    }
    if (lane >= m && lane < K) {
        out_ids[(int64_t)q * K + lane] = -1;   // past m, as the search leaves them
        out_d[(int64_t)q * K + lane] = 0.0f;
    }
    if (lane == 0) out_m[q] = m;
}

// The same ranking when D is a multiple of 4 (D = 100): lane j takes
// candidate j of each chunk of 64, reads its whole row into registers with
// 16-byte loads (all in flight at once) and sums its terms in index order in
// FP64, the same operations as above; the K rounds of wave minimum follow.
template <int DT, bool L1>
__global__ __launch_bounds__(64) void k_knn_rank_rows(int Q, int K, int cap, const float* __restrict__ qfeat,
                                                    const float* __restrict__ xf, const int32_t* __restrict__ cand,
                                                    const int32_t* __restrict__ ncand, int32_t* __restrict__ out_ids,
                                                    float* __restrict__ out_d, int32_t* __restrict__ out_m) {
    static_assert(DT % 4 == 0 && DT <= kL1MaxD, "rows of whole 16-byte chunks");
    constexpr int D4 = DT / 4;
    constexpr int NCH = kL1Chunk * kL1PerLane / 64;
    __shared__ double sq[DT];
    const int lane = threadIdx.x;
    const int q = xcd_block();
    if (q >= Q) return;
    const int M = min(ncand[q], cap);
    for (int i = lane; i < DT; i += 64) sq[i] = (double)qfeat[(int64_t)q * DT + i];
    __syncthreads();
    double d[NCH];
    int id[NCH];
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
        d[u] = INFINITY;
        id[u] = 0x7FFFFFFF;
        const int c = 64 * u + lane;
        if (c < M) {
            const int myid = cand[(int64_t)q * cap + c];
            const float4* row = reinterpret_cast<const float4*>(xf) + (int64_t)myid * D4;
            float4 x[D4];
#pragma unroll
            for (int t = 0; t < D4; ++t) x[t] = row[t];
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < D4; ++t) {
                const float xv[4] = {x[t].x, x[t].y, x[t].z, x[t].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double dv = sq[4 * t + e] - (double)xv[e];
                    acc = acc + (L1 ? fabs(dv) : dv * dv);
                }
            }
            d[u] = acc;
            id[u] = myid;
        }
    }
    const int m = min(K, M);
    for (int k = 0; k < m; ++k) {
        double bd = d[0];
        int bi = id[0];
#pragma unroll
        for (int u = 1; u < NCH; ++u)
            if (d[u] < bd || (d[u] == bd && id[u] < bi)) {
                bd = d[u];
                bi = id[u];
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double od = __shfl_xor(bd, o);
            const int oi = __shfl_xor(bi, o);
            if (od < bd || (od == bd && oi < bi)) {
                bd = od;
                bi = oi;
            }
        }
#pragma unroll
        for (int u = 0; u < NCH; ++u)
            if (id[u] == bi) {
                d[u] = INFINITY;
                id[u] = 0x7FFFFFFF;
            }
        if (lane == 0) {
            out_ids[(int64_t)q * K + k] = bi;
            out_d[(int64_t)q * K + k] = (float)bd;
        }
    }
    if (lane >= m && lane < K) {
        out_ids[(int64_t)q * K + lane] = -1;
        out_d[(int64_t)q * K + lane] = 0.0f;
    }
    if (lane == 0) out_m[q] = m;
}

// The l1 screen rows, one thread an entry. Any lo and step give valid
// bounds, since eps is measured against the very values fmaf(step, u, lo)
// the ranking forms; the row's minimum and range / 255 keep eps small. eps is
// summed in FP64 and rounded up with a margin of 2^-20 relative, which covers
// that sum's own rounding and the fp32 rounding of the bounds formed from it.
__global__ __launch_bounds__(256) void k_l1_screen_rows(const float* __restrict__ xf, int64_t n,
                                                      uint8_t* __restrict__ l1s) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float4* x4 = reinterpret_cast<const float4*>(xf + r * kL1sDim);
    float x[kL1sDim];
#pragma unroll
    for (int t = 0; t < kL1sDim / 4; ++t) {
        const float4 v = x4[t];
        x[4 * t] = v.x;
        x[4 * t + 1] = v.y;
        x[4 * t + 2] = v.z;
        x[4 * t + 3] = v.w;
    }
    float lo = x[0], hi = x[0];
#pragma unroll
    for (int i = 1; i < kL1sDim; ++i) {
        lo = fminf(lo, x[i]);
        hi = fmaxf(hi, x[i]);
    }
    float step = (hi - lo) * (1.0f / 255.0f);
    if (!(step > 0.0f) || !(step < INFINITY)) step = 0.0f;
    uint32_t w[kL1sBytes / 4];
#pragma unroll
    for (int i = 0; i < kL1sBytes / 4; ++i) w[i] = 0u;
    double eps = 0.0;
#pragma unroll
    for (int i = 0; i < kL1sDim; ++i) {
        float u = step > 0.0f ? rintf((x[i] - lo) / step) : 0.0f;
        u = fminf(fmaxf(u, 0.0f), 255.0f);
        eps += fabs((double)x[i] - (double)fmaf(step, u, lo));
        w[i >> 2] |= (uint32_t)u << (8 * (i & 3));
    }
    const double eu = eps * (1.0 + 0x1p-20);
    float ef = (float)eu;
    if ((double)ef < eu) ef = nextafterf(ef, INFINITY);
    if (!(ef >= 0.0f)) ef = INFINITY;   // a non-finite feature: bounds that prune nothing
    constexpr int t0 = kL1sTail / 4;
    w[t0] = __float_as_uint(lo);
    w[t0 + 1] = __float_as_uint(step);
    w[t0 + 2] = __float_as_uint(ef);
    uint4* out = reinterpret_cast<uint4*>(l1s + r * kL1sBytes);
#pragma unroll
    for (int t = 0; t < kL1sBytes / 16; ++t) out[t] = make_uint4(w[4 * t], w[4 * t + 1], w[4 * t + 2], w[4 * t + 3]);
}

__global__ void k_min_i32(int n, const int32_t* __restrict__ in, int cap, int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = min(in[i], cap);
}

hipError_t launch_min_i32(int n, const int32_t* in, int cap, int32_t* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_min_i32, dim3((n + 255) / 256), dim3(256), 0, st, n, in, cap, out);
    return hipGetLastError();
}

hipError_t launch_l1_screen_rows(const float* xf, int64_t n, uint8_t* l1s, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(xf) & 15) || (reinterpret_cast<uintptr_t>(l1s) & 15)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_l1_screen_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xf, n, l1s);
    return hipGetLastError();
}

// K nearest under l1 with the screen (D = 100). One wave a patch:
//  1. A = sum_i |q_i - fmaf(step, u_i, lo)| in fp32 from the candidate's
//     128-byte screen row; with eps = ||x - x~||_1 the triangle inequality
//     puts its l1 distance in [A - eps, A + eps]. An fp32 sum of 100
//     non-negative terms, in any order, is within 101 u A of its exact value,
//     so the bounds widen A by 2^-15 relative: lb = fmaf(A, 1 - 2^-15, -eps),
//     ub = fmaf(A, 1 + 2^-15, eps), each rounded once. Lane j takes candidate
//     j of a chunk of 64; a last chunk of at most 8 candidates is spread over
//     8 lanes each, one 16-byte segment of the row a lane.
//  2. tau = the K-th smallest ub, by binary search over the bit patterns of
//     the (non-negative) bounds with ballot counts: K candidates lie within
//     tau.
//  3. A candidate with lb > tau (1 + 2^-20) is farther than those K even
//     after the FP64 rounding of every distance, so it cannot be among the K
//     nearest in (distance, ID) order; the others survive, compacted in LDS.
//  4. The survivors' exact distances, summed in index order in FP64 as the
//     unscreened kernels do; with at most 64 survivors each one's rank in
//     (distance, ID) order is counted against all the others (IDs are
//     distinct), else K rounds of wave minimum pick them.
// With M <= K candidates nothing is screened.
__global__ __launch_bounds__(64) void k_knn_l1_screened(int Q, int K, int cap, const float* __restrict__ qfeat,
                                                      const float* __restrict__ xf, const uint8_t* __restrict__ l1s,
                                                      const int32_t* __restrict__ cand,
                                                      const int32_t* __restrict__ ncand, int32_t* __restrict__ out_ids,
                                                      float* __restrict__ out_d, int32_t* __restrict__ out_m,
                                                      int32_t* __restrict__ out_ns) {
    constexpr int DT = kL1sDim, D4 = DT / 4, NCH = kRankMaxCand / 64;
    constexpr int kSeg = (kL1sTail + 12 + 15) / 16;   // 16-byte loads that hold the codes and the tail
    static_assert(kSeg <= 8 && kL1sTail % 16 == 4, "codes, then lo, step, eps in the last 16-byte load");
    __shared__ double sq[DT];
    __shared__ float4 sqf[D4];
    __shared__ int sid[kRankMaxCand];
    const int lane = threadIdx.x;
    const int q = xcd_block();
    if (q >= Q) return;
    const int M = min(ncand[q], cap);
    const int32_t* cq = cand + (int64_t)q * cap;
    for (int i = lane; i < DT; i += 64) {
        const float v = qfeat[(int64_t)q * DT + i];
        sq[i] = (double)v;
        reinterpret_cast<float*>(sqf)[i] = v;
    }
    int ns = 0;
    if (M > K) {
        __syncthreads();
        uint32_t ubb[NCH];   // bit patterns of the upper bounds; 0xFFFFFFFF: no candidate
        float lb[NCH];
        int idc[NCH];
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
            ubb[u] = 0xFFFFFFFFu;
            lb[u] = INFINITY;
            idc[u] = 0;
            const int base = 64 * u;
            if (base >= M) continue;
            const int r = M - base;
            float A = 0.0f, lo = 0.0f, st = 0.0f, e = 0.0f;
            bool own = false;   // this lane reports the chunk's candidate
            int id = 0;
            if (r > 8) {
                if (lane < r) {
                    id = cq[base + lane];
                    own = true;
                    const uint4* row = reinterpret_cast<const uint4*>(l1s + (size_t)id * kL1sBytes);
                    uint4 v[kSeg];
#pragma unroll
                    for (int t = 0; t < kSeg; ++t) v[t] = row[t];
                    const uint32_t* wv = reinterpret_cast<const uint32_t*>(v);
                    lo = __uint_as_float(wv[kL1sTail / 4]);
                    st = __uint_as_float(wv[kL1sTail / 4 + 1]);
                    e = __uint_as_float(wv[kL1sTail / 4 + 2]);
#pragma unroll
                    for (int t = 0; t < D4; ++t) {
                        const float4 qv = sqf[t];
                        const uint32_t cw = wv[t];
                        A += fabsf(qv.x - fmaf(st, (float)(cw & 255u), lo));
                        A += fabsf(qv.y - fmaf(st, (float)((cw >> 8) & 255u), lo));
                        A += fabsf(qv.z - fmaf(st, (float)((cw >> 16) & 255u), lo));
                        A += fabsf(qv.w - fmaf(st, (float)(cw >> 24), lo));
                    }
                }
            } else {
                // 8 lanes a candidate, lane seg of the group on codes 16 seg .. 16 seg + 15
                const int g = lane >> 3, seg = lane & 7;
                if (g < r) {
                    id = cq[base + g];
                    own = seg == 0;
                    const uint4* row = reinterpret_cast<const uint4*>(l1s + (size_t)id * kL1sBytes);
                    const uint4 tl = row[kSeg - 1];
                    lo = __uint_as_float(tl.y);
                    st = __uint_as_float(tl.z);
                    e = __uint_as_float(tl.w);
                    if (seg < kSeg) {
                        const uint4 v = row[seg];
                        const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            if (4 * seg + t >= D4) break;
                            const float4 qv = sqf[4 * seg + t];
                            const uint32_t cw = wv[t];
                            A += fabsf(qv.x - fmaf(st, (float)(cw & 255u), lo));
                            A += fabsf(qv.y - fmaf(st, (float)((cw >> 8) & 255u), lo));
                            A += fabsf(qv.z - fmaf(st, (float)((cw >> 16) & 255u), lo));
                            A += fabsf(qv.w - fmaf(st, (float)(cw >> 24), lo));
                        }
                    }
                }
                A += __shfl_xor(A, 1);
                A += __shfl_xor(A, 2);
                A += __shfl_xor(A, 4);
            }
            if (own) {
                float l = fmaf(A, 1.0f - 0x1p-15f, -e);
                float h = fmaf(A, 1.0f + 0x1p-15f, e);
                if (!(h >= 0.0f)) {   // non-finite: keep the candidate, set no threshold by it
                    l = 0.0f;
                    h = INFINITY;
                }
                lb[u] = l;
                ubb[u] = __float_as_uint(h);
                idc[u] = id;
            }
        }
        // 2. tau: the smallest bit pattern with at least K upper bounds at or below it
        uint32_t blo = 0u, bhi = 0x7F800000u;
        while (blo < bhi) {
            const uint32_t mid = blo + ((bhi - blo) >> 1);
            int cnt = 0;
#pragma unroll
            for (int u = 0; u < NCH; ++u) {
                if (64 * u >= M) break;
                cnt += __popcll(__ballot(ubb[u] <= mid));
            }
            if (cnt >= K) bhi = mid;
            else blo = mid + 1u;
        }
        const float thr = __uint_as_float(blo) * (1.0f + 0x1p-20f);
        // 3. survivors, compacted in candidate order
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
            if (64 * u >= M) break;
            const bool keep = ubb[u] != 0xFFFFFFFFu && !(lb[u] > thr);
            const uint64_t bm = __ballot(keep);
            if (keep) sid[ns + __popcll(bm & ((1ull << lane) - 1ull))] = idc[u];
            ns += __popcll(bm);
        }
    } else {
        for (int j = lane; j < M; j += 64) sid[j] = cq[j];
        ns = M;
    }
    __syncthreads();
    if (out_ns && lane == 0) out_ns[q] = ns;
    // 4. exact distances of the survivors
    double d[NCH];
    int id[NCH];
#pragma unroll
    for (int u = 0; u < NCH; ++u) {
        d[u] = INFINITY;
        id[u] = 0x7FFFFFFF;
        const int j = 64 * u + lane;
        if (64 * u < ns && j < ns) {
            const int myid = sid[j];
            const float4* row = reinterpret_cast<const float4*>(xf) + (int64_t)myid * D4;
            double acc = 0.0;
            constexpr int H = (D4 + 1) / 2;   // the row in two halves of loads in flight
#pragma unroll
            for (int h0 = 0; h0 < D4; h0 += H) {
                float4 x[H];
#pragma unroll
                for (int t = 0; t < H; ++t)
                    if (h0 + t < D4) x[t] = row[h0 + t];
#pragma unroll
                for (int t = 0; t < H; ++t) {
                    if (h0 + t >= D4) break;
                    const float xv[4] = {x[t].x, x[t].y, x[t].z, x[t].w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc = acc + fabs(sq[4 * (h0 + t) + e] - (double)xv[e]);
                }
            }
            d[u] = acc;
            id[u] = myid;
        }
    }
    const int m = min(K, M);
    if (ns <= 64) {
        // rank of survivor lane among all survivors in (distance, ID) order
        const int64_t dbits = __double_as_longlong(d[0]);
        const int dlo = (int)(dbits & 0xFFFFFFFF), dhi = (int)(dbits >> 32);
        int rank = 0;
        for (int t = 0; t < ns; ++t) {
            const int tlo = __builtin_amdgcn_readlane(dlo, t), thi = __builtin_amdgcn_readlane(dhi, t);
            const int tid = __builtin_amdgcn_readlane(id[0], t);
            const double dt = __longlong_as_double(((int64_t)thi << 32) | (int64_t)(uint32_t)tlo);
            rank += (dt < d[0] || (dt == d[0] && tid < id[0])) ? 1 : 0;
        }
        if (lane < ns && rank < m) {
            out_ids[(int64_t)q * K + rank] = id[0];
            out_d[(int64_t)q * K + rank] = (float)d[0];
        }
    } else {
        for (int k = 0; k < m; ++k) {
            double bd = d[0];
            int bi = id[0];
#pragma unroll
            for (int u = 1; u < NCH; ++u)
                if (d[u] < bd || (d[u] == bd && id[u] < bi)) {
                    bd = d[u];
                    bi = id[u];
                }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double od = __shfl_xor(bd, o);
                const int oi = __shfl_xor(bi, o);
                if (od < bd || (od == bd && oi < bi)) {
                    bd = od;
                    bi = oi;
                }
            }
#pragma unroll
            for (int u = 0; u < NCH; ++u)
                if (id[u] == bi) {
                    d[u] = INFINITY;
                    id[u] = 0x7FFFFFFF;
                }
            if (lane == 0) {
                out_ids[(int64_t)q * K + k] = bi;
                out_d[(int64_t)q * K + k] = (float)bd;
            }
        }
    }
    if (lane >= m && lane < K) {
        out_ids[(int64_t)q * K + lane] = -1;
        out_d[(int64_t)q * K + lane] = 0.0f;
    }
    if (lane == 0) out_m[q] = m;
}

hipError_t launch_knn_l1_screened(int Q, int K, int cap, const float* qfeat, const float* xf, const uint8_t* l1s,
                                  const int32_t* cand, const int32_t* ncand, int32_t* ids, float* d, int32_t* m,
                                  int32_t* ns, hipStream_t st) {
    if (Q == 0) return hipSuccess;
    if (cap < 1 || cap > kRankMaxCand || K < 1 || K > kMaxK) return hipErrorInvalidValue;
    if ((reinterpret_cast<uintptr_t>(xf) & 15) || (reinterpret_cast<uintptr_t>(l1s) & 15)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_knn_l1_screened, dim3(round_grid8(Q)), dim3(64), 0, st, Q, K, cap, qfeat, xf, l1s, cand,
                       ncand, ids, d, m, ns);
    return hipGetLastError();
}

hipError_t launch_knn_rank(int Q, int D, int K, int cap, bool l1, const float* qfeat, const float* xf,
                           const int32_t* cand, const int32_t* ncand, int32_t* ids, float* d, int32_t* m,
                           hipStream_t st) {
    if (Q == 0) return hipSuccess;
    if (cap < 1 || cap > kL1Chunk * kL1PerLane || K < 1 || K > kMaxK || D < 1 || D > kL1MaxD) return hipErrorInvalidValue;
    const int grid = round_grid8(Q);   // patches in contiguous runs per XCD: neighbours share candidates in L2
#define ZH_RANK(DT, M1) \
    hipLaunchKernelGGL((k_knn_rank<DT, M1>), dim3(grid), dim3(64), 0, st, Q, D, K, cap, qfeat, xf, cand, ncand, ids, d, m)
    if (D == 100) {
        const bool al = (reinterpret_cast<uintptr_t>(xf) & 15) == 0;
        if (al && l1)
            hipLaunchKernelGGL((k_knn_rank_rows<100, true>), dim3(grid), dim3(64), 0, st, Q, K, cap, qfeat, xf, cand, ncand,
                               ids, d, m);
        else if (al)
            hipLaunchKernelGGL((k_knn_rank_rows<100, false>), dim3(grid), dim3(64), 0, st, Q, K, cap, qfeat, xf, cand,
                               ncand, ids, d, m);
        if (al) return hipGetLastError();
    }
    if (l1) {
        if (D == 100) ZH_RANK(100, true);
        else if (D == 25) ZH_RANK(25, true);
        else ZH_RANK(0, true);
    } else {
        if (D == 100) ZH_RANK(100, false);
        else if (D == 25) ZH_RANK(25, false);
        else ZH_RANK(0, false);
    }
#undef ZH_RANK
    return hipGetLastError();
}

}  // namespace zh

namespace zh {

// t-of-L candidates (Section 4.1: a training patch matches when it shares the
// query's bucket in at least t of the L tables). One wave per patch; the
// patch's L bins (sorted by ID) are walked in table order, 64 entries at a
// time. An entry x of bin l is kept at its first table only (no earlier bin
// holds it) and counted in the later ones, both by binary search; IDs with
// at least t hits are written in walk order (the set is what is defined).
__global__ __launch_bounds__(256) void k_cand_t(int Q, int L, int64_t N, int t, const uint2* __restrict__ bins,
                                                const uint32_t* __restrict__ tids, int cap,
                                                int32_t* __restrict__ counts, int32_t* __restrict__ ids) {
    __shared__ uint32_t s_off[4][64], s_cnt[4][64];
    __shared__ int64_t s_st[4][64];
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    const int q = blockIdx.x * 4 + wv;
    if (q >= Q) return;
    const uint2 b = lane < L ? bins[(int64_t)lane * Q + q] : make_uint2(0u, 0u);
    int64_t incl = b.y;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    s_off[wv][lane] = b.x;
    s_cnt[wv][lane] = b.y;
    s_st[wv][lane] = incl - b.y;
    const int64_t S = __shfl(incl, 63);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    auto in_bin = [&](int l, uint32_t x) {
        const uint32_t* p = tids + (int64_t)l * N + s_off[wv][l];
        uint32_t lo = 0, hi = s_cnt[wv][l];
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (p[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        return lo < s_cnt[wv][l] && p[lo] == x;
    };
    int64_t kept = 0;
    for (int64_t e0 = 0; e0 < S; e0 += 64) {
        const int64_t e = e0 + lane;
        bool keep = false;
        uint32_t x = 0;
        if (e < S) {
            int l = 0;
            while (l + 1 < L && s_st[wv][l + 1] <= e) ++l;
            x = tids[(int64_t)l * N + s_off[wv][l] + (e - s_st[wv][l])];
            bool first = true;
            for (int j = 0; j < l && first; ++j) first = !in_bin(j, x);
            if (first) {
                int hits = 1;
                for (int j = l + 1; j < L && hits < t; ++j) hits += in_bin(j, x) ? 1 : 0;
                keep = hits >= t;
            }
        }
        const uint64_t mask = __ballot(keep);
        const int64_t pos = kept + __popcll(mask & lanemask_lt());
        if (keep && pos < cap) ids[(int64_t)q * cap + pos] = (int32_t)x;
        kept += __popcll(mask);
    }
    if (lane == 0) counts[q] = (int32_t)kept;
}

// K nearest of the t-of-L candidates, however many there are. One wave per
// patch walks its bins as k_cand_t does (an ID kept at its first table when
// it has at least t hits); each lane with a kept ID sums its squared l2
// distance over the coordinates in index order in FP64 (each term rounded
// before it is added, as the oracle's loop), and the wave merges the chunk's
// (distance, ID) pairs into a running top K held by lanes 0..K-1: K rounds
// of a wave minimum over both sets. IDs are distinct across chunks (first
// occurrences only), so no pair is seen twice.
template <int DT>
__global__ __launch_bounds__(256) void k_knn_tofl(int Q, int L, int64_t N, int t, int Drt, int K,
                                                  const uint2* __restrict__ bins, const uint32_t* __restrict__ tids,
                                                  const float* __restrict__ qfeat, const float* __restrict__ xf,
                                                  int32_t* __restrict__ counts, int32_t* __restrict__ out_ids,
                                                  float* __restrict__ out_d, int32_t* __restrict__ out_m) {
    __shared__ uint32_t s_off[4][64], s_cnt[4][64];
    __shared__ int64_t s_st[4][64];
    __shared__ double s_q[4][kL1MaxD];
    const int D = DT ? DT : Drt;
    const int lane = __lane_id(), wv = threadIdx.x >> 6;
    const int q = blockIdx.x * 4 + wv;
    if (q >= Q) return;
    const uint2 b = lane < L ? bins[(int64_t)lane * Q + q] : make_uint2(0u, 0u);
    int64_t incl = b.y;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    s_off[wv][lane] = b.x;
    s_cnt[wv][lane] = b.y;
    s_st[wv][lane] = incl - b.y;
    for (int i = lane; i < D; i += 64) s_q[wv][i] = (double)qfeat[(int64_t)q * D + i];
    const int64_t S = __shfl(incl, 63);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    auto in_bin = [&](int l, uint32_t x) {
        const uint32_t* p = tids + (int64_t)l * N + s_off[wv][l];
        uint32_t lo = 0, hi = s_cnt[wv][l];
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (p[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        return lo < s_cnt[wv][l] && p[lo] == x;
    };
    // running top K: lane k < K holds the k-th smallest (distance, ID) so far
    double bd = INFINITY;
    int bi = 0x7FFFFFFF;
    int64_t kept = 0;
    for (int64_t e0 = 0; e0 < S; e0 += 64) {
        const int64_t e = e0 + lane;
        bool keep = false;
        uint32_t x = 0;
        if (e < S) {
            int l = 0;
            while (l + 1 < L && s_st[wv][l + 1] <= e) ++l;
            x = tids[(int64_t)l * N + s_off[wv][l] + (e - s_st[wv][l])];
            bool first = true;
            for (int j = 0; j < l && first; ++j) first = !in_bin(j, x);
            if (first) {
                int hits = 1;
                for (int j = l + 1; j < L && hits < t; ++j) hits += in_bin(j, x) ? 1 : 0;
                keep = hits >= t;
            }
        }
        const uint64_t mask = __ballot(keep);
        kept += __popcll(mask);
        if (!mask) continue;
        double nd = INFINITY;
        int ni = 0x7FFFFFFF;
        if (keep) {
            const float* row = xf + (int64_t)x * D;
            double acc = 0.0;
            if ((D & 3) == 0) {
                const float4* r4 = reinterpret_cast<const float4*>(row);
                for (int i = 0; i < D; i += 4) {
                    const float4 v = r4[i >> 2];
                    const double t0 = s_q[wv][i] - (double)v.x;
                    acc = acc + t0 * t0;
                    const double t1 = s_q[wv][i + 1] - (double)v.y;
                    acc = acc + t1 * t1;
                    const double t2 = s_q[wv][i + 2] - (double)v.z;
                    acc = acc + t2 * t2;
                    const double t3 = s_q[wv][i + 3] - (double)v.w;
                    acc = acc + t3 * t3;
                }
            } else {
                for (int i = 0; i < D; ++i) {
                    const double t0 = s_q[wv][i] - (double)row[i];
                    acc = acc + t0 * t0;
                }
            }
            nd = acc;
            ni = (int)x;
        }
        // K rounds: the smallest of the running top K and the chunk's pairs
        double rd = INFINITY;
        int ri = 0x7FFFFFFF;
        for (int k = 0; k < K; ++k) {
            const bool bfirst = bd < nd || (bd == nd && bi < ni);
            double md = bfirst ? bd : nd;
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
            } else if (ni == mi && nd == md) {
                nd = INFINITY;
                ni = 0x7FFFFFFF;
            }
            if (lane == k) {
                rd = md;
                ri = mi;
            }
        }
        bd = rd;
        bi = ri;
    }
    const int m = (int)(kept < K ? kept : K);
    if (lane < m) {
        out_ids[(int64_t)q * K + lane] = bi;
        out_d[(int64_t)q * K + lane] = (float)bd;
    } else if (lane < K) {
        out_ids[(int64_t)q * K + lane] = -1;
        out_d[(int64_t)q * K + lane] = 0.0f;
    }
    if (lane == 0) {
        counts[q] = (int32_t)kept;
        out_m[q] = m;
    }
}

hipError_t launch_knn_tofl(int Q, int L, int64_t N, int t, int D, int K, const uint2* bins, const uint32_t* tids,
                           const float* qfeat, const float* xf, int32_t* counts, int32_t* ids, float* d, int32_t* m,
                           hipStream_t st) {
    if (Q == 0) return hipSuccess;
    if (L < 1 || L > 64 || t < 1 || t > L || K < 1 || K > kMaxK || D < 1 || D > kL1MaxD) return hipErrorInvalidValue;
    const dim3 grid((Q + 3) / 4);
    if (D == 100) hipLaunchKernelGGL(k_knn_tofl<100>, grid, dim3(256), 0, st, Q, L, N, t, D, K, bins, tids, qfeat, xf, counts, ids, d, m);
    else if (D == 25) hipLaunchKernelGGL(k_knn_tofl<25>, grid, dim3(256), 0, st, Q, L, N, t, D, K, bins, tids, qfeat, xf, counts, ids, d, m);
    else hipLaunchKernelGGL(k_knn_tofl<0>, grid, dim3(256), 0, st, Q, L, N, t, D, K, bins, tids, qfeat, xf, counts, ids, d, m);
    return hipGetLastError();
}

hipError_t launch_cand_t(int Q, int L, int64_t N, int t, const uint2* bins, const uint32_t* tids, int cap,
                         int32_t* counts, int32_t* ids, hipStream_t st) {
    if (Q == 0) return hipSuccess;
    if (L < 1 || L > 64 || t < 1 || t > L || cap < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cand_t, dim3((Q + 3) / 4), dim3(256), 0, st, Q, L, N, t, bins, tids, cap, counts, ids);
    return hipGetLastError();
}

}  // namespace zh
