// LLE weights (Section 4.2, Eq. LinSys), HR synthesis (Eq. HR_Rec) and the
// overlap blend (Section 4: quadratic prior on the overlaps, whose equal-
// weight minimiser is the per-pixel mean of the covering patches).
//
// Weights: Z = y - Y (the K neighbour rows), G = Z Z^T, A = G + lam tr(G) I,
// A w~ = 1 by Cholesky, w = w~ / sum(w~); uniform weights when tr(G) = 0.
// A workgroup (one wave) forms the Gram matrices of QPW patches one after
// the other, every lane owning one (a, b) entry; then each lane solves one
// patch's system.
#include <algorithm>
#include <type_traits>

#include "zh_internal.h"

namespace zh {

// (a, b) with a >= b for packed lower index p = a (a + 1) / 2 + b
__constant__ uint8_t c_pa[136];
__constant__ uint8_t c_pb[136];
static bool g_pair_table_ready[64] = {false};

template <typename T, int KMAX, int QPW>
__global__ __launch_bounds__(64) void k_lle(LleArgs a) {
    constexpr int NPM = KMAX * (KMAX + 1) / 2;
    constexpr int GST = NPM + 1;                      // padded per-patch stride
    __shared__ T sG[QPW * GST];
    __shared__ T sZ[128 * KMAX];                      // Z transposed: [dim][neighbour]
    const int lane = threadIdx.x;
    const int D = a.D, K = a.K;
    const int q0 = blockIdx.x * QPW;

    for (int qi = 0; qi < QPW; ++qi) {
        const int q = q0 + qi;
        if (q >= a.Q) break;
        const int m = a.m[q];
        if (m <= 0) continue;
        const float* qrow = a.qfeat + (int64_t)q * D;
        for (int r = 0; r < m; ++r) {
            const int64_t id = a.ids[(int64_t)q * K + r];
            const int64_t b = id * D, bh = id * a.hs;
            for (int t = lane; t < D; t += 64)
                sZ[t * KMAX + r] = (T)qrow[t] - (T)join_planes(a.hi[bh + t], a.lo[b + t]);
        }
        __syncthreads();
        const int np = m * (m + 1) / 2;
        for (int p = lane; p < np; p += 64) {
            const int ia = c_pa[p], ib = c_pb[p];
            T g = (T)0;
            for (int t = 0; t < D; ++t) g += sZ[t * KMAX + ia] * sZ[t * KMAX + ib];
            sG[qi * GST + p] = g;
        }
        __syncthreads();
    }

    if (lane < QPW && q0 + lane < a.Q) {
        const int q = q0 + lane;
        const int m = a.m[q];
        float* wout = a.w + (int64_t)q * K;
        if (m <= 0) {
            for (int r = 0; r < K; ++r) wout[r] = 0.0f;
            return;
        }
        T* G = sG + lane * GST;
        auto at = [&](int i, int j) -> T& { return G[i * (i + 1) / 2 + j]; };  // i >= j
        T tau = (T)0;
        for (int i = 0; i < m; ++i) tau += at(i, i);
        T wv[KMAX];
        bool redo64 = false;
        if (tau == (T)0) {
            for (int i = 0; i < m; ++i) wv[i] = (T)1 / (T)m;
        } else {
            const T reg = (T)a.lam * tau;
            for (int i = 0; i < m; ++i) at(i, i) += reg;
            // Cholesky A = L L^T in place (packed lower)
            T dmin = (T)1e300, dmax = (T)0;
            for (int j = 0; j < m; ++j) {
                T s = at(j, j);
                for (int k = 0; k < j; ++k) s -= at(j, k) * at(j, k);
                const T d = sqrt(s);
                at(j, j) = d;
                dmin = d < dmin ? d : dmin;
                dmax = d > dmax ? d : dmax;
                for (int i = j + 1; i < m; ++i) {
                    T t = at(i, j);
                    for (int k = 0; k < j; ++k) t -= at(i, k) * at(j, k);
                    at(i, j) = t / d;
                }
            }
            // condition estimate from the Cholesky diagonal
            if (sizeof(T) == 4 && (double)dmax * (double)dmax > 1e6 * (double)dmin * (double)dmin) redo64 = true;
            T y[KMAX];
            for (int i = 0; i < m; ++i) {
                T s = (T)1;
                for (int k = 0; k < i; ++k) s -= at(i, k) * y[k];
                y[i] = s / at(i, i);
            }
            T sum = (T)0;
            for (int i = m - 1; i >= 0; --i) {
                T s = y[i];
                for (int k = i + 1; k < m; ++k) s -= at(k, i) * wv[k];
                wv[i] = s / at(i, i);
            }
            for (int i = 0; i < m; ++i) sum += wv[i];
            for (int i = 0; i < m; ++i) wv[i] /= sum;
        }
        if (redo64) {
            // ill-conditioned in fp32: the whole solve again in FP64
            if (a.n_fp64) atomicAdd(a.n_fp64, 1u);
            double Gd[KMAX * (KMAX + 1) / 2];
            const float* qrow = a.qfeat + (int64_t)q * D;
            for (int i = 0; i < m; ++i)
                for (int j = 0; j <= i; ++j) {
                    const int64_t ii = a.ids[(int64_t)q * K + i], ij = a.ids[(int64_t)q * K + j];
                    const int64_t bi = ii * D, bj = ij * D, hi_i = ii * a.hs, hi_j = ij * a.hs;
                    double g = 0.0;
                    for (int t = 0; t < D; ++t) {
                        const double zi = (double)qrow[t] - (double)join_planes(a.hi[hi_i + t], a.lo[bi + t]);
                        const double zj = (double)qrow[t] - (double)join_planes(a.hi[hi_j + t], a.lo[bj + t]);
                        g += zi * zj;
                    }
                    Gd[i * (i + 1) / 2 + j] = g;
                }
            double td = 0.0;
            for (int i = 0; i < m; ++i) td += Gd[i * (i + 1) / 2 + i];
            for (int i = 0; i < m; ++i) Gd[i * (i + 1) / 2 + i] += (double)a.lam * td;
            for (int j = 0; j < m; ++j) {
                double s = Gd[j * (j + 1) / 2 + j];
                for (int k = 0; k < j; ++k) s -= Gd[j * (j + 1) / 2 + k] * Gd[j * (j + 1) / 2 + k];
                const double d = sqrt(s);
                Gd[j * (j + 1) / 2 + j] = d;
                for (int i = j + 1; i < m; ++i) {
                    double t = Gd[i * (i + 1) / 2 + j];
                    for (int k = 0; k < j; ++k) t -= Gd[i * (i + 1) / 2 + k] * Gd[j * (j + 1) / 2 + k];
                    Gd[i * (i + 1) / 2 + j] = t / d;
                }
            }
            double yd[KMAX], xd[KMAX], sd = 0.0;
            for (int i = 0; i < m; ++i) {
                double s = 1.0;
                for (int k = 0; k < i; ++k) s -= Gd[i * (i + 1) / 2 + k] * yd[k];
                yd[i] = s / Gd[i * (i + 1) / 2 + i];
            }
            for (int i = m - 1; i >= 0; --i) {
                double s = yd[i];
                for (int k = i + 1; k < m; ++k) s -= Gd[k * (k + 1) / 2 + i] * xd[k];
                xd[i] = s / Gd[i * (i + 1) / 2 + i];
            }
            for (int i = 0; i < m; ++i) sd += xd[i];
            for (int i = 0; i < m; ++i) wv[i] = (T)(xd[i] / sd);
        }
        for (int r = 0; r < K; ++r) wout[r] = r < m ? (float)wv[r] : 0.0f;
    }
}

// One halving step of a reduce-scatter over the lanes of a half wave: lanes
// whose bit O is clear keep the first half of their N values, the others the
// second half, each adding its partner's partial sums; (base, cnt) track the
// index range the lane holds.
template <typename T, int N, int O, int NMAX>
__device__ __forceinline__ void rs_step(T (&v)[NMAX], int& base, int& cnt) {
    constexpr int NK = (N + 1) / 2;
    const bool hb = (threadIdx.x & O) != 0;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
        const T lo_v = v[i];
        const T hi_v = (NK + i < N) ? v[NK + i] : (T)0;
        const T send = hb ? lo_v : hi_v;
        const T keep = hb ? hi_v : lo_v;
        v[i] = keep + __shfl_xor(send, O);
    }
    if (hb) {
        base += NK;
        cnt -= NK;
    } else {
        cnt = cnt < NK ? cnt : NK;
    }
}

// Packed Gram matrix (lower triangle, p = i(i+1)/2 + j, 36 entries) of the
// m <= 8 neighbours of each patch, Z_r = q - y_r, in T precision. Two patches
// per wave: half h of the wave owns one patch and lane l of the half holds
// coordinates [VEC l, VEC l + VEC); the 8 neighbour rows are loaded before
// use, partial products are reduce-scattered over the half in two groups of
// 18 entries.
template <typename T, int VEC>
__global__ __launch_bounds__(256) void k_gram(LleArgs a, T* __restrict__ gram) {
    typedef typename std::conditional<VEC == 4, uint2, uint32_t>::type raw_t;
    constexpr int PI[36] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 4, 5, 5, 5,
                            5, 5, 5, 6, 6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7};
    constexpr int PJ[36] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4, 0, 1, 2,
                            3, 4, 5, 0, 1, 2, 3, 4, 5, 6, 0, 1, 2, 3, 4, 5, 6, 7};
    const int lane = threadIdx.x & 63, hl = lane & 31, half = lane >> 5;
    const int wpb = blockDim.x >> 6;
    const int D = a.D;
    const bool dl = hl * VEC < D;
    for (int pr = xcd_block() * wpb + (threadIdx.x >> 6); 2 * pr < a.Q; pr += gridDim.x * wpb) {
        const int q = 2 * pr + half;
        const bool qv = q < a.Q;
        const int m = qv ? a.m[q] : 0;
        float qf[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) qf[e] = (qv && dl) ? a.qfeat[(int64_t)q * D + hl * VEC + e] : 0.0f;
        T z[8][VEC];
        if (VEC == 4 && a.xf) {
            // the fp32 copy: one 16-byte load of a contiguous 400-byte row
            float4 xr[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                xr[r] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (r < m && dl) {
                    const int64_t id = a.ids[(int64_t)q * a.K + r];
                    xr[r] = *reinterpret_cast<const float4*>(a.xf + id * D + hl * VEC);
                }
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const float xv[4] = {xr[r].x, xr[r].y, xr[r].z, xr[r].w};
#pragma unroll
                for (int e = 0; e < VEC; ++e) z[r][e] = (r < m && dl) ? (T)qf[e] - (T)xv[e % 4] : (T)0;
            }
        } else {
            raw_t hr[8], lr[8];
    #pragma unroll
            for (int r = 0; r < 8; ++r) {
                hr[r] = raw_t{};
                lr[r] = raw_t{};
                if (r < m && dl) {
                    const uint32_t id = (uint32_t)a.ids[(int64_t)q * a.K + r];
                    const uint32_t bo = (id * (uint32_t)D + (uint32_t)(hl * VEC)) * 2u;
                    const uint32_t bh = (id * (uint32_t)a.hs + (uint32_t)(hl * VEC)) * 2u;
                    if constexpr (VEC == 4) {
                        hr[r] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(a.hi) + bh);
                        lr[r] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(a.lo) + bo);
                    } else {
                        hr[r] = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(a.hi) + bh);
                        lr[r] = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(a.lo) + bo);
                    }
                }
            }
    #pragma unroll
            for (int r = 0; r < 8; ++r) {
                uint32_t hv[VEC], lv[VEC];
                if constexpr (VEC == 4) {
                    hv[0] = hr[r].x & 0xFFFFu; hv[1] = hr[r].x >> 16; hv[2] = hr[r].y & 0xFFFFu; hv[3] = hr[r].y >> 16;
                    lv[0] = lr[r].x & 0xFFFFu; lv[1] = lr[r].x >> 16; lv[2] = lr[r].y & 0xFFFFu; lv[3] = lr[r].y >> 16;
                } else {
                    hv[0] = hr[r];
                    lv[0] = lr[r];
                }
    #pragma unroll
                for (int e = 0; e < VEC; ++e)
                    z[r][e] = (r < m && dl) ? (T)qf[e] - (T)__uint_as_float((hv[e] << 16) | lv[e]) : (T)0;
            }
        }
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            T v[18];
#pragma unroll
            for (int p = 0; p < 18; ++p) {
                T acc = (T)0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc += z[PI[18 * g + p]][e] * z[PJ[18 * g + p]][e];
                v[p] = acc;
            }
            int base = 0, cnt = 18;
            rs_step<T, 18, 16>(v, base, cnt);
            rs_step<T, 9, 8>(v, base, cnt);
            rs_step<T, 5, 4>(v, base, cnt);
            rs_step<T, 3, 2>(v, base, cnt);
            rs_step<T, 2, 1>(v, base, cnt);
            if (m > 0 && cnt >= 1) gram[(int64_t)q * 36 + 18 * g + base] = v[0];
        }
    }
}

hipError_t launch_gram(const LleArgs& a, void* gram, int gram_fp64, hipStream_t st) {
    if (a.Q == 0) return hipSuccess;
    if (a.K > 8 || a.D > 128) return hipErrorInvalidValue;
    const bool v4 = a.D % 4 == 0;
    if (!v4 && a.D > 32) return hipErrorInvalidValue;
    int grid = (a.Q + 7) / 8;
    if (grid > 65536) grid = 65536;
    grid = round_grid8(grid);
    if (gram_fp64) {
        if (v4) hipLaunchKernelGGL((k_gram<double, 4>), dim3(grid), dim3(256), 0, st, a, static_cast<double*>(gram));
        else hipLaunchKernelGGL((k_gram<double, 1>), dim3(grid), dim3(256), 0, st, a, static_cast<double*>(gram));
    } else {
        if (v4) hipLaunchKernelGGL((k_gram<float, 4>), dim3(grid), dim3(256), 0, st, a, static_cast<float*>(gram));
        else hipLaunchKernelGGL((k_gram<float, 1>), dim3(grid), dim3(256), 0, st, a, static_cast<float*>(gram));
    }
    return hipGetLastError();
}

// FP64 Gram of patch q's m neighbours straight from the rows (the slow path of
// the fp32 solve when its condition estimate exceeds 1e6).
__device__ void gram_fp64_rows(const LleArgs& a, int q, int m, double* Gd) {
    const int D = a.D;
    const float* qrow = a.qfeat + (int64_t)q * D;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j <= i; ++j) {
            const int64_t ii = a.ids[(int64_t)q * a.K + i], ij = a.ids[(int64_t)q * a.K + j];
            const int64_t bi = ii * D, bj = ij * D, hi_i = ii * a.hs, hi_j = ij * a.hs;
            double g = 0.0;
            for (int t = 0; t < D; ++t) {
                const double zi = (double)qrow[t] - (double)join_planes(a.hi[hi_i + t], a.lo[bi + t]);
                const double zj = (double)qrow[t] - (double)join_planes(a.hi[hi_j + t], a.lo[bj + t]);
                g += zi * zj;
            }
            Gd[i * (i + 1) / 2 + j] = g;
        }
}

// Solve (G + lam tr(G) I) w~ = 1 on the first m rows (rows m..7 are set to
// the identity with a zero right-hand side), w = w~ / sum(w~). Returns the
// squared ratio of the largest to the smallest Cholesky diagonal.
template <typename T>
__device__ __forceinline__ double solve8(T (&A)[36], int m, double lam, T (&w)[8]) {
    T tau = (T)0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (i < m) tau += A[i * (i + 1) / 2 + i];
    if (tau == (T)0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = i < m ? (T)1 / (T)m : (T)0;
        return 1.0;
    }
    const T reg = (T)lam * tau;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            T& x = A[i * (i + 1) / 2 + j];
            if (i >= m || j >= m) x = (i == j) ? (T)1 : (T)0;
            else if (i == j) x += reg;
        }
    T dmin = (T)0, dmax = (T)0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        T s = A[j * (j + 1) / 2 + j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= A[j * (j + 1) / 2 + k] * A[j * (j + 1) / 2 + k];
        const T d = sqrt(s);
        A[j * (j + 1) / 2 + j] = d;
        if (j < m) {
            dmin = (j == 0 || d < dmin) ? d : dmin;
            dmax = d > dmax ? d : dmax;
        }
        const T inv = (T)1 / d;
#pragma unroll
        for (int i = j + 1; i < 8; ++i) {
            T t = A[i * (i + 1) / 2 + j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= A[i * (i + 1) / 2 + k] * A[j * (j + 1) / 2 + k];
            A[i * (i + 1) / 2 + j] = t * inv;
        }
    }
    T y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        T s = i < m ? (T)1 : (T)0;
#pragma unroll
        for (int k = 0; k < i; ++k) s -= A[i * (i + 1) / 2 + k] * y[k];
        y[i] = s / A[i * (i + 1) / 2 + i];
    }
    T sum = (T)0;
#pragma unroll
    for (int i = 7; i >= 0; --i) {
        T s = y[i];
#pragma unroll
        for (int k = i + 1; k < 8; ++k) s -= A[k * (k + 1) / 2 + i] * w[k];
        w[i] = s / A[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (i < m) sum += w[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = i < m ? w[i] / sum : (T)0;
    const double r = (double)dmax / (double)dmin;
    return r * r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_lle_solve(LleArgs a, const T* __restrict__ gram) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.Q) return;
    const int m = a.m[q];
    float* wout = a.w + (int64_t)q * a.K;
    if (m <= 0) {
        for (int r = 0; r < a.K; ++r) wout[r] = 0.0f;
        return;
    }
    T A[36];
#pragma unroll
    for (int p = 0; p < 36; ++p) A[p] = gram[(int64_t)q * 36 + p];
    T w[8];
    const double cond = solve8<T>(A, m, a.lam, w);
    if (sizeof(T) == 4 && cond > 1e6) {
        if (a.n_fp64) atomicAdd(a.n_fp64, 1u);
        double Ad[36], wd[8];
#pragma unroll
        for (int p = 0; p < 36; ++p) Ad[p] = 0.0;
        gram_fp64_rows(a, q, m, Ad);
        solve8<double>(Ad, m, a.lam, wd);
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = (T)wd[i];
    }
    for (int r = 0; r < a.K; ++r) wout[r] = r < m && r < 8 ? (float)w[r] : 0.0f;
}

hipError_t launch_lle_solve(const LleArgs& a, const void* gram, int gram_fp64, hipStream_t st) {
    if (a.Q == 0) return hipSuccess;
    if (a.K > 8) return hipErrorInvalidValue;
    const int grid = (a.Q + 255) / 256;
    if (gram_fp64)
        hipLaunchKernelGGL(k_lle_solve<double>, dim3(grid), dim3(256), 0, st, a, static_cast<const double*>(gram));
    else
        hipLaunchKernelGGL(k_lle_solve<float>, dim3(grid), dim3(256), 0, st, a, static_cast<const float*>(gram));
    return hipGetLastError();
}

// LLE over all M matches of each patch (Section 4.2: Eq. LinSys with m
// running over every match found, M <= kAllMax): one wave per patch. The M
// candidate rows sit in LDS (fp32, odd stride); the packed lower triangle of
// G = Z Z^T, z_m = q - y_m, is formed in FP64 from exact differences (sums in
// coordinate order), tau = tr G is added times lambda to the diagonal, the
// Cholesky factor overwrites it (column by column, lanes over rows), and two
// triangular solves give w~ = A^-1 1, w = w~ / sum w~. tau = 0 (every
// candidate equals the query) gives uniform weights. Weights past M are 0 and
// list entries past M are set to -1.
__global__ __launch_bounds__(64) void k_lle_all(int Q, int D, int cap, double lam, const float* __restrict__ qfeat,
                                                const float* __restrict__ xf, int32_t* __restrict__ cand,
                                                const int32_t* __restrict__ ncand, float* __restrict__ w) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int q = blockIdx.x;
    const int M = min(ncand[q], cap);
    const int st = D | 1;
    double* A = reinterpret_cast<double*>(smem);                        // [cap (cap + 1) / 2]
    double* y = A + (size_t)cap * (cap + 1) / 2;                         // [cap]
    double* sq = y + cap;                                               // [D]
    float* rows = reinterpret_cast<float*>(sq + D);                     // [cap][st]
    for (int i = lane; i < D; i += 64) sq[i] = (double)qfeat[(int64_t)q * D + i];
    for (int e = lane; e < M * D; e += 64) {
        const int r = e / D, c = e - r * D;
        rows[r * st + c] = xf[(int64_t)cand[(int64_t)q * cap + r] * D + c];
    }
    for (int i = M + lane; i < cap; i += 64) cand[(int64_t)q * cap + i] = -1;   // list entries past M
    __syncthreads();
    // G, packed: entry (i, j <= i) at i (i + 1) / 2 + j
    const int np = M * (M + 1) / 2;
    for (int e = lane; e < np; e += 64) {
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (i * (i + 1) / 2 > e) --i;
        while ((i + 1) * (i + 2) / 2 <= e) ++i;
        const int j = e - i * (i + 1) / 2;
        const float* ri = rows + i * st;
        const float* rj = rows + j * st;
        double g = 0.0;
        for (int c = 0; c < D; ++c) {
            const double zi = sq[c] - (double)ri[c];
            const double zj = sq[c] - (double)rj[c];
            g = g + zi * zj;
        }
        A[e] = g;
    }
    __syncthreads();
    double tau = 0.0;
    for (int i = lane; i < M; i += 64) tau += A[i * (i + 1) / 2 + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tau += __shfl_xor(tau, o);
    if (M > 0 && tau == 0.0) {
        for (int i = lane; i < cap; i += 64) w[(int64_t)q * cap + i] = i < M ? (float)(1.0 / M) : 0.0f;
        return;
    }
    for (int i = lane; i < M; i += 64) A[i * (i + 1) / 2 + i] += lam * tau;
    __syncthreads();
    // Cholesky, right-looking: column j, then the trailing rows of later columns
    for (int j = 0; j < M; ++j) {
        const int dj = j * (j + 1) / 2 + j;
        const double d = sqrt(A[dj]);
        __syncthreads();
        for (int i = j + 1 + lane; i < M; i += 64) A[i * (i + 1) / 2 + j] /= d;
        if (lane == 0) A[dj] = d;
        __syncthreads();
        for (int i = j + 1 + lane; i < M; i += 64) {
            const int ri = i * (i + 1) / 2;
            const double lij = A[ri + j];
            for (int k = j + 1; k <= i; ++k) A[ri + k] -= lij * A[k * (k + 1) / 2 + j];
        }
        __syncthreads();
    }
    // L y = 1, then L^T w~ = y (columns in turn, lanes over the other rows)
    for (int i = lane; i < M; i += 64) y[i] = 1.0;
    __syncthreads();
    for (int j = 0; j < M; ++j) {
        const double yj = y[j] / A[j * (j + 1) / 2 + j];
        __syncthreads();
        if (lane == 0) y[j] = yj;
        for (int i = j + 1 + lane; i < M; i += 64) y[i] -= A[i * (i + 1) / 2 + j] * yj;
        __syncthreads();
    }
    for (int j = M - 1; j >= 0; --j) {
        const int rj = j * (j + 1) / 2;
        const double xj = y[j] / A[rj + j];
        __syncthreads();
        if (lane == 0) y[j] = xj;
        for (int i = lane; i < j; i += 64) y[i] -= A[rj + i] * xj;
        __syncthreads();
    }
    double sum = 0.0;
    for (int i = lane; i < M; i += 64) sum += y[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    for (int i = lane; i < cap; i += 64) w[(int64_t)q * cap + i] = i < M ? (float)(y[i] / sum) : 0.0f;
}

size_t lle_all_lds(int cap, int D) {
    return sizeof(double) * ((size_t)cap * (cap + 1) / 2 + cap + D) + sizeof(float) * (size_t)cap * (D | 1);
}

hipError_t launch_lle_all(int Q, int D, int cap, double lam, const float* qfeat, const float* xf, int32_t* cand,
                          const int32_t* ncand, float* w, hipStream_t st) {
    if (Q == 0) return hipSuccess;
    if (cap < 1 || cap > kAllMax || D < 1 || D > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lle_all, dim3(Q), dim3(64), lle_all_lds(cap, D), st, Q, D, cap, lam, qfeat, xf, cand, ncand, w);
    return hipGetLastError();
}

// ---- synthesis fused with the blend -------------------------------------------
// The synthesised patches are never written out. The patch origins are cut
// into tiles of TI patch rows x sb_cols(s) patch columns; a workgroup takes a
// tile, forms x_q = mu_q + sum_m w_m r_{n_m} of one patch row at a time in
// LDS (the K residual rows read once, in chunks of eight neighbours; each
// value is a fused multiply-add over the neighbours in order from zero, then
// mu_q is added) and adds each
// pixel's values of the row's patches, in ascending column order, to the
// tile's region: the (TI + 4) s x (TJ + 4) s HR pixels its patches cover,
// together with the count of covering patches of every LR cell. Regions go
// to a partial buffer; k_sb_combine then gives each HR pixel the sum of the
// (at most four) regions that hold it, in tile order, divided by the summed
// count, or the bicubic of the LR image where no patch covers it. The sum
// of a pixel is therefore taken patch row by patch row in row-major order
// inside a tile and tile by tile across tiles.
template <int s, int TI>
struct SbGeom {
    static constexpr int ps = kPatch * s, ps2 = ps * ps;
    static constexpr int VEC = (ps2 & 3) == 0 ? 4 : 1;    // floats per load
    static constexpr int NCH = ps2 / VEC;                  // loads per residual row
    static constexpr int TJ = sb_cols(s);
    static constexpr int CY = TI + kPatch - 1, CX = TJ + kPatch - 1;   // LR cells of a region
    static constexpr int RY = CY * s, RX = CX * s;                       // HR pixels of a region
    static constexpr int64_t PART = (int64_t)RY * RX + CY * CX;         // floats + counts per tile
};

template <int s, int TI>
__device__ __forceinline__ void sb_tile(const int32_t* __restrict__ ids, const int32_t* __restrict__ m,
                                        const float* __restrict__ wt, const double* __restrict__ mu,
                                        const float* __restrict__ resid, int K, int h, int w, int64_t tile,
                                        float* __restrict__ part) {
    using G = SbGeom<s, TI>;
    constexpr int ps = G::ps, ps2 = G::ps2, VEC = G::VEC, NCH = G::NCH, TJ = G::TJ;
    constexpr int CX = G::CX, RY = G::RY, RX = G::RX, CY = G::CY;
    __shared__ __align__(16) float sx[TJ * ps2];   // the synthesised patches of one patch row
    __shared__ float sacc[RY * RX];
    __shared__ int scnt[CY * CX];
    __shared__ int64_t sbase[TJ * 8];              // residual row offsets of a chunk (-1: none)
    __shared__ float swt[TJ * 8];
    __shared__ int sflag[TJ];
    __shared__ float smu[TJ];
    const int tid = threadIdx.x;
    const int npi = h - kPatch + 1, npj = w - kPatch + 1;
    const int ntj = (npj + TJ - 1) / TJ;
    // the grid is rounded up to a multiple of 8: workgroups past the last
    // tile have no region
    if (npi <= 0 || npj <= 0 || tile >= (int64_t)((npi + TI - 1) / TI) * ntj) return;
    const int ti = (int)(tile / ntj), tj = (int)(tile - (int64_t)ti * ntj);
    const int i0 = ti * TI, j0 = tj * TJ;
    for (int e = tid; e < RY * RX; e += 256) sacc[e] = 0.0f;
    for (int e = tid; e < CY * CX; e += 256) scnt[e] = 0;
    for (int ii = 0; ii < TI && i0 + ii < npi; ++ii) {
        const int64_t qrow = (int64_t)(i0 + ii) * npj;
        // ---- the patches of this row
        for (int r0 = 0; r0 < K; r0 += 8) {
            __syncthreads();   // the previous chunk, row or the zeroing is done
            for (int e = tid; e < TJ * 8; e += 256) {
                const int jj = e >> 3, r = e & 7, j = j0 + jj;
                const int64_t q = qrow + j;
                const int mq = j < npj ? m[q] : 0;
                const bool ok = r0 + r < mq;
                sbase[e] = ok ? (int64_t)ids[q * K + r0 + r] * ps2 : -1;
                swt[e] = ok ? wt[q * K + r0 + r] : 0.0f;
                if (r0 == 0 && r == 0) {
                    sflag[jj] = mq > 0;
                    smu[jj] = mq > 0 ? (float)mu[q] : 0.0f;
                }
            }
            __syncthreads();
            const bool last = r0 + 8 >= K;
            for (int it = tid; it < TJ * NCH; it += 256) {
                const int jj = it / NCH, c = it - jj * NCH;
                float* dst = sx + jj * ps2 + c * VEC;
                float acc[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = r0 == 0 ? 0.0f : dst[e];
                float v[8][VEC];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int64_t b = sbase[jj * 8 + r];
                    if constexpr (VEC == 4) {
                        const float4 x = b >= 0 ? *reinterpret_cast<const float4*>(resid + b + 4 * c)
                                                : make_float4(0.f, 0.f, 0.f, 0.f);
                        v[r][0] = x.x;
                        v[r][1] = x.y;
                        v[r][2] = x.z;
                        v[r][3] = x.w;
                    } else {
                        v[r][0] = b >= 0 ? resid[b + c] : 0.0f;
                    }
                }
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const float wr = swt[jj * 8 + r];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] = fmaf(wr, v[r][e], acc[e]);
                }
                const float mf = last ? smu[jj] : 0.0f;
#pragma unroll
                for (int e = 0; e < VEC; ++e) dst[e] = last ? mf + acc[e] : acc[e];
            }
        }
        __syncthreads();
        // ---- their values added to the region rows s ii .. s ii + 5 s
        for (int it = tid; it < ps * RX; it += 256) {
            const int u = it / RX, X = it - u * RX;
            const int cl = X / s;
            const int jlo = cl - (kPatch - 1) > 0 ? cl - (kPatch - 1) : 0, jhi = cl < TJ - 1 ? cl : TJ - 1;
            float* a = sacc + (s * ii + u) * RX + X;
            float acc = *a;
            for (int jj = jlo; jj <= jhi; ++jj)
                if (sflag[jj]) acc += sx[jj * ps2 + u * ps + X - s * jj];
            *a = acc;
        }
        for (int it = tid; it < kPatch * CX; it += 256) {
            const int cu = it / CX, cl = it - cu * CX;
            const int jlo = cl - (kPatch - 1) > 0 ? cl - (kPatch - 1) : 0, jhi = cl < TJ - 1 ? cl : TJ - 1;
            int n = 0;
            for (int jj = jlo; jj <= jhi; ++jj) n += sflag[jj];
            scnt[(ii + cu) * CX + cl] += n;
        }
    }
    __syncthreads();
    float* pa = part + tile * G::PART;
    int* pc = reinterpret_cast<int*>(pa + RY * RX);
    for (int e = tid; e < RY * RX; e += 256) pa[e] = sacc[e];
    for (int e = tid; e < CY * CX; e += 256) pc[e] = scnt[e];
}

template <int s, int TI>
__device__ __forceinline__ float sb_pixel(const float* __restrict__ part, const float* __restrict__ lr, int h, int w,
                                          int Y, int X) {
    using G = SbGeom<s, TI>;
    constexpr int TJ = G::TJ, CX = G::CX, RX = G::RX, RY = G::RY;
    const int npi = h - kPatch + 1, npj = w - kPatch + 1;
    float acc = 0.0f;
    int cnt = 0;
    if (npi > 0 && npj > 0) {
        const int ntj = (npj + TJ - 1) / TJ, nti = (npi + TI - 1) / TI;
        const int cy = Y / s, cx = X / s;
        // tiles holding a patch origin in [cy - 4, cy] x [cx - 4, cx]
        const int tilo = cy >= kPatch - 1 ? (cy - (kPatch - 1)) / TI : 0, tihi = min(nti - 1, cy / TI);
        const int tjlo = cx >= kPatch - 1 ? (cx - (kPatch - 1)) / TJ : 0, tjhi = min(ntj - 1, cx / TJ);
        for (int ti = tilo; ti <= tihi; ++ti)
            for (int tj = tjlo; tj <= tjhi; ++tj) {
                const float* pa = part + ((int64_t)ti * ntj + tj) * G::PART;
                const int ly = Y - s * TI * ti, lx = X - s * TJ * tj;
                acc += pa[ly * RX + lx];
                cnt += reinterpret_cast<const int*>(pa + RY * RX)[(cy - TI * ti) * CX + (cx - TJ * tj)];
            }
    }
    return cnt > 0 ? acc / (float)cnt : bicubic_at(lr, h, w, s, Y, X);
}

template <int s, int TI>
__global__ __launch_bounds__(256) void k_sb_tile(int K, int h, int w, const int32_t* __restrict__ ids,
                                                 const int32_t* __restrict__ m, const float* __restrict__ wt,
                                                 const double* __restrict__ mu, const float* __restrict__ resid,
                                                 float* __restrict__ part) {
    sb_tile<s, TI>(ids, m, wt, mu, resid, K, h, w, xcd_block(), part);
}

template <int s, int TI>
__global__ __launch_bounds__(256) void k_sb_combine(const float* __restrict__ part, const float* __restrict__ lr,
                                                    int h, int w, float* __restrict__ hr) {
    const int W = s * w;
    const int64_t total = (int64_t)s * h * W;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int Y = (int)(p / W), X = (int)(p - (int64_t)Y * W);
        hr[p] = sb_pixel<s, TI>(part, lr, h, w, Y, X);
    }
}

// Batched: the tiles and HR pixels of every image of the batch, the image
// found from its first tile (sbt_off) or HR pixel (hr_off); partial regions
// at the image's first tile.
template <int s, int TI>
__global__ __launch_bounds__(256) void k_b_sb_tile(const BatchImage* __restrict__ im, int n, int64_t tiles, int K,
                                                   const int32_t* __restrict__ ids, const int32_t* __restrict__ m,
                                                   const float* __restrict__ wt, const double* __restrict__ mu,
                                                   const float* __restrict__ resid, float* __restrict__ part) {
    const int64_t t = xcd_block();
    if (t >= tiles) return;   // the grid is rounded up to a multiple of 8
    const BatchImage& b = im[batch_image_of<&BatchImage::sbt_off>(im, n, t)];
    sb_tile<s, TI>(ids + b.q_off * K, m + b.q_off, wt + b.q_off * K, mu + b.q_off, resid, K, b.h, b.w,
                   t - b.sbt_off, part + b.sbt_off * SbGeom<s, TI>::PART);
}

template <int s, int TI>
__global__ __launch_bounds__(256) void k_b_sb_combine(const BatchImage* __restrict__ im, int n, int64_t total,
                                                      const float* __restrict__ part) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const BatchImage& b = im[batch_image_of<&BatchImage::hr_off>(im, n, p)];
        const int W = s * b.w;
        const int64_t lp = p - b.hr_off;
        const int Y = (int)(lp / W), X = (int)(lp - (int64_t)Y * W);
        b.out[lp] = sb_pixel<s, TI>(part + b.sbt_off * SbGeom<s, TI>::PART, b.lr, b.h, b.w, Y, X);
    }
}

int64_t sb_tiles(int s, int rows, int h, int w) {
    if (h < kPatch || w < kPatch) return 0;
    const int64_t npi = h - kPatch + 1, npj = w - kPatch + 1;
    return ((npi + rows - 1) / rows) * ((npj + sb_cols(s) - 1) / sb_cols(s));
}

int64_t sb_part_floats(int s, int rows) {
    const int64_t cy = rows + kPatch - 1, cx = sb_cols(s) + kPatch - 1;
    return cy * s * cx * s + cy * cx;
}

template <int s, int TI>
static hipError_t sb_launch(int K, int h, int w, const int32_t* ids, const int32_t* m, const float* wt,
                            const double* mu, const float* resid, float* part, const float* lr, float* hr,
                            hipStream_t st, int which) {
    const int64_t nt = sb_tiles(s, TI, h, w);
    if (which & 1 && nt > 0) {
        if (nt > 0x7FFFFFFF) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_sb_tile<s, TI>), dim3((unsigned)round_grid8((int)nt)), dim3(256), 0, st, K, h, w, ids, m,
                           wt, mu, resid, part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (which & 2) {
        const int64_t total = (int64_t)s * h * s * w;
        if (total > 0)
            hipLaunchKernelGGL((k_sb_combine<s, TI>), dim3((unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20)),
                               dim3(256), 0, st, part, lr, h, w, hr);
    }
    return hipGetLastError();
}

hipError_t launch_synth_blend(int scale, int rows, int K, int h, int w, const int32_t* ids, const int32_t* m,
                              const float* wt, const double* mu, const float* resid, float* part, const float* lr,
                              float* hr, hipStream_t st, int which) {
    if (K < 1 || (rows != 4 && rows != 8)) return hipErrorInvalidValue;
    switch (scale * 10 + rows) {
        case 14: return sb_launch<1, 4>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        case 18: return sb_launch<1, 8>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        case 24: return sb_launch<2, 4>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        case 28: return sb_launch<2, 8>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        case 34: return sb_launch<3, 4>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        case 38: return sb_launch<3, 8>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        case 44: return sb_launch<4, 4>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        case 48: return sb_launch<4, 8>(K, h, w, ids, m, wt, mu, resid, part, lr, hr, st, which);
        default: return hipErrorInvalidValue;
    }
}

template <int s, int TI>
static hipError_t b_sb_launch(const BatchImage* im, int n, int64_t tiles, int64_t hr_total, int K, const int32_t* ids,
                              const int32_t* m, const float* wt, const double* mu, const float* resid, float* part,
                              hipStream_t st) {
    if (tiles > 0) {
        if (tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_b_sb_tile<s, TI>), dim3((unsigned)round_grid8((int)tiles)), dim3(256), 0, st, im, n, tiles,
                           K, ids, m, wt, mu, resid, part);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (hr_total > 0)
        hipLaunchKernelGGL((k_b_sb_combine<s, TI>), dim3((unsigned)std::min<int64_t>((hr_total + 255) / 256, 1 << 20)),
                           dim3(256), 0, st, im, n, hr_total, part);
    return hipGetLastError();
}

hipError_t launch_b_synth_blend(const BatchImage* im, int n, int64_t tiles, int64_t hr_total, int scale, int rows,
                                int K, const int32_t* ids, const int32_t* m, const float* wt, const double* mu,
                                const float* resid, float* part, hipStream_t st) {
    if (K < 1 || (rows != 4 && rows != 8)) return hipErrorInvalidValue;
    switch (scale * 10 + rows) {
        case 14: return b_sb_launch<1, 4>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        case 18: return b_sb_launch<1, 8>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        case 24: return b_sb_launch<2, 4>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        case 28: return b_sb_launch<2, 8>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        case 34: return b_sb_launch<3, 4>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        case 38: return b_sb_launch<3, 8>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        case 44: return b_sb_launch<4, 4>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        case 48: return b_sb_launch<4, 8>(im, n, tiles, hr_total, K, ids, m, wt, mu, resid, part, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t lle_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 64 && g_pair_table_ready[dev]) return hipSuccess;
    uint8_t pa[136], pb[136];
    int p = 0;
    for (int i = 0; i < 16; ++i)
        for (int j = 0; j <= i; ++j) {
            pa[p] = (uint8_t)i;
            pb[p] = (uint8_t)j;
            ++p;
        }
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_pa), pa, sizeof(pa));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_pb), pb, sizeof(pb));
    if (e == hipSuccess && dev < 64) g_pair_table_ready[dev] = true;
    return e;
}

hipError_t launch_lle(const LleArgs& a, hipStream_t st) {
    if (a.Q == 0) return hipSuccess;
    if (a.D > 128 || a.K > kMaxK) return hipErrorInvalidValue;
    if (a.K <= 8) {
        const int grid = (a.Q + 63) / 64;
        if (a.fp64) hipLaunchKernelGGL((k_lle<double, 8, 64>), dim3(grid), dim3(64), 0, st, a);
        else hipLaunchKernelGGL((k_lle<float, 8, 64>), dim3(grid), dim3(64), 0, st, a);
    } else {
        const int grid = (a.Q + 15) / 16;
        if (a.fp64) hipLaunchKernelGGL((k_lle<double, 16, 16>), dim3(grid), dim3(64), 0, st, a);
        else hipLaunchKernelGGL((k_lle<float, 16, 16>), dim3(grid), dim3(64), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace zh
