// Adjoint of the zoom: gradients of a loss on the output image with respect
// to the dictionary's HR residual patches and the LLE regulariser lambda.
// Neighbour indices (hash codes, candidates, top-K) are discrete and stay at
// their forward values.
//
// Back-projection (Section 4, the update after Eq. Err_img; Section 4.3,
// Eq. sx2 and Eq. bl_filter_3), one iteration I' = I + S(I) F(I) with
// F = N Up (I_L - Dec Blur I) and S = exp(-(I - Box I)^2 / (2 sigma_r^2)):
//
//   g <- g - Blur^T Dec^T Up^T N^T (S g) + (Id - Box)^T [-(a / sigma_r^2) S F g],
//
// a = I - Box I. Every operator is separable (a matrix per axis with
// replicate or in-image-normalised borders), so each transpose is two
// one-axis gathers (k_axis_adj) whose weights are rebuilt from the forward
// definitions: normalised Gaussian (taps inside the image, divided by their
// sum), box mean (in-image count), Keys' cubic (a = -0.5, replicate border),
// Gaussian blur with replicate border followed by phase-0 decimation.
//
// Blend (per-pixel mean of the covering patches): each patch pixel receives
// g(X) / cnt(X). Synthesis x_q = mu_q + sum_m w_qm r_{n_qm} (Eq. HR_Rec):
// dL/dr_n = sum over the (q, m) with n_qm = n of w_qm g_q, gathered per
// dictionary row over a stable sort of the neighbour lists (no float
// atomics, fixed order); dL/dw_qm = <g_q, r_{n_qm}>. LLE weights (Eq. LinSys)
// with A = G + lambda tr(G) I: the Gram matrix is recomputed in FP64 and
// factorised again, dw~/dlambda = -tr(G) A^-1 w~, dw/dlambda =
// (dw~/dlambda - w 1^T dw~/dlambda) / 1^T w~; dL/dlambda is a fixed-order
// FP64 reduction over the patches.
#include <cmath>

#include "zh_internal.h"

namespace zh {

// HR patch values per lane, in chunks of 64, at the largest zoom factor
constexpr int kPixChunks = (kMaxPs2 + 63) / 64;

// ---- one-axis transposed operators ------------------------------------------
// Along x (AXIS 0) the array is [rows][n] and the pass maps rows of n_in to
// rows of n_out; along y (AXIS 1) it is [n][cols], cols = a.rows.
template <int OP, int AXIS>
__global__ __launch_bounds__(256) void k_axis_adj(AxisAdjArgs a) {
    const int64_t total = (int64_t)a.rows * a.n_out;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int c, o;
        if (AXIS == 0) {
            c = (int)(idx / a.n_out);
            o = (int)(idx - (int64_t)c * a.n_out);
        } else {
            o = (int)(idx / a.rows);
            c = (int)(idx - (int64_t)o * a.rows);
        }
        auto in = [&](int x) -> float {
            const int64_t p = AXIS == 0 ? (int64_t)c * a.n_in + x : (int64_t)x * a.rows + c;
            return a.mul ? a.in[p] * a.mul[p] : a.in[p];
        };
        const int n = a.n_in, R = a.R;
        float acc = 0.0f;
        if (OP == kAdjGauss) {
            // out[o] = sum_x c(o - x) in[x] / nrm(x), nrm(x) = sum of the in-image taps at x
            for (int x = max(0, o - R); x <= min(n - 1, o + R); ++x) {
                float nrm = 0.0f;
                for (int d = -R; d <= R; ++d)
                    if (x + d >= 0 && x + d < n) nrm += a.taps[d + R];
                acc = fmaf(a.taps[o - x + R] / nrm, in(x), acc);
            }
        } else if (OP == kAdjBox) {
            for (int x = max(0, o - R); x <= min(n - 1, o + R); ++x) {
                const int cnt = min(n - 1, x + R) - max(0, x - R) + 1;
                acc += in(x) / (float)cnt;
            }
        } else if (OP == kAdjUp) {
            // HR n_in -> LR n_out: HR sample x reads LR floor(x/s) - 1 + t, t = 0..3
            const int s = a.s;
            for (int x = max(0, s * (o - 2)); x < min(n, s * (o + 3)); ++x) {
                const int i0 = x / s;
                const float tx = (float)(x - i0 * s) / (float)s;
                float wsum = 0.0f;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (clampi(i0 - 1 + t, 0, a.n_out - 1) == o) wsum += keys_w(tx - (float)(t - 1));
                acc = fmaf(wsum, in(x), acc);
            }
        } else {
            // LR n_in -> HR n_out: LR sample i reads HR clamp(s i + t), |t| <= R
            const int s = a.s;
            const int ilo = max(0, (o - R) / s - 1), ihi = min(n - 1, (o + R) / s + 1);
            for (int i = ilo; i <= ihi; ++i) {
                float wsum = 0.0f;
                for (int t = -R; t <= R; ++t)
                    if (clampi(s * i + t, 0, a.n_out - 1) == o) wsum += a.taps[t + R];
                acc = fmaf(wsum, in(i), acc);
            }
        }
        const int64_t po = AXIS == 0 ? (int64_t)c * a.n_out + o : (int64_t)o * a.rows + c;
        a.out[po] = acc;
    }
}

template <int OP>
static hipError_t axis_pass(AxisAdjArgs a, int axis, hipStream_t st) {
    const int64_t total = (int64_t)a.rows * a.n_out;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (axis == 0)
        hipLaunchKernelGGL((k_axis_adj<OP, 0>), dim3((unsigned)g), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_axis_adj<OP, 1>), dim3((unsigned)g), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_axis_adj(int op, int axis, const AxisAdjArgs& a, hipStream_t st) {
    if (a.R > kMaxAdjR) return hipErrorInvalidValue;
    switch (op) {
        case kAdjGauss: return axis_pass<kAdjGauss>(a, axis, st);
        case kAdjBox: return axis_pass<kAdjBox>(a, axis, st);
        case kAdjUp: return axis_pass<kAdjUp>(a, axis, st);
        default: return axis_pass<kAdjDec>(a, axis, st);
    }
}

// ---- elementwise pieces of one iteration's adjoint --------------------------
// z = -(a / sigma_r^2) S F g   (FSa = [F | S | a])
__global__ void k_bp_adj_z(const float* __restrict__ FSa, const float* __restrict__ g, int64_t n, float inv_sr2,
                           float* __restrict__ z) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = -(FSa[2 * n + i] * inv_sr2) * FSa[n + i] * FSa[i] * g[i];
}
// g <- g - v + z - bz  (z, bz null when the range weight is constant)
__global__ void k_bp_adj_combine(float* __restrict__ g, const float* __restrict__ v, const float* __restrict__ z,
                                 const float* __restrict__ bz, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float r = g[i] - v[i];
        if (z) r += z[i] - bz[i];
        g[i] = r;
    }
}

static dim3 grid1(int64_t n) {
    int64_t g = (n + 255) / 256;
    return dim3((unsigned)(g > 65536 ? 65536 : (g < 1 ? 1 : g)));
}

hipError_t launch_bp_adj_z(const float* FSa, const float* g, int64_t n, float sigma_r, float* z, hipStream_t st) {
    hipLaunchKernelGGL(k_bp_adj_z, grid1(n), dim3(256), 0, st, FSa, g, n, 1.0f / (sigma_r * sigma_r), z);
    return hipGetLastError();
}
hipError_t launch_bp_adj_combine(float* g, const float* v, const float* z, const float* bz, int64_t n,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_bp_adj_combine, grid1(n), dim3(256), 0, st, g, v, z, bz, n);
    return hipGetLastError();
}

// ---- blend adjoint: gradient per covered pixel divided by its count ---------
__global__ void k_blend_adj(const float* __restrict__ g, const int32_t* __restrict__ m, int h, int w, int s,
                            float* __restrict__ gp) {
    const int H = s * h, W = s * w, ps = kPatch * s;
    const int npi = h - kPatch + 1, npj = w - kPatch + 1;
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int Y = (int)(idx / W), X = (int)(idx % W);
        const int ilo = Y - ps + 1 <= 0 ? 0 : (Y - ps + s) / s;
        const int ihi = min(npi - 1, Y / s);
        const int jlo = X - ps + 1 <= 0 ? 0 : (X - ps + s) / s;
        const int jhi = min(npj - 1, X / s);
        int cnt = 0;
        for (int i = ilo; i <= ihi; ++i)
            for (int j = jlo; j <= jhi; ++j) cnt += m[i * npj + j] > 0 ? 1 : 0;
        gp[idx] = cnt > 0 ? g[idx] / (float)cnt : 0.0f;
    }
}

hipError_t launch_blend_adj(const float* g, const int32_t* m, int h, int w, int s, float* gp, hipStream_t st) {
    hipLaunchKernelGGL(k_blend_adj, grid1((int64_t)s * h * s * w), dim3(256), 0, st, g, m, h, w, s, gp);
    return hipGetLastError();
}

// ---- LLE adjoint through lambda: one wave per patch --------------------------
// dL/dw_m = <g_q, r_{n_m}> over the patch's HR pixels; the Gram matrix of
// Z = q - X_N in FP64 (coordinates over the lanes, wave sums), then on lane
// 0: A = G + lambda tau I, Cholesky, w~ = A^-1 1, d = -tau A^-1 w~,
// contribution [g_w . d - (g_w . w)(1 . d)] / (1 . w~).
template <int U>
__global__ __launch_bounds__(256) void k_lle_lambda_adj(BackwardArgs a) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int D = a.D, K = a.K, s = a.s, ps = kPatch * s, ps2 = ps * ps;
    const int npj = a.w - kPatch + 1;
    const int W = s * a.w;
    for (int q = blockIdx.x * wpb + (threadIdx.x >> 6); q < a.Q; q += gridDim.x * wpb) {
        const int mq = a.m[q];
        if (mq <= 0) {
            if (lane == 0) a.c_lam[q] = 0.0;
            continue;
        }
        const int pi = q / npj, pj = q % npj;
        // patch gradient values of this lane: pixels lane + 64 u
        float gq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int P = lane + 64 * u;
            gq[u] = 0.0f;
            if (P < ps2) {
                const int py = P / ps, px = P % ps;
                gq[u] = a.gp[(int64_t)(s * pi + py) * W + s * pj + px];
            }
        }
        double gw[kMaxK];
        for (int mi = 0; mi < K; ++mi) {
            double acc = 0.0;
            if (mi < mq) {
                const float* r = a.resid + (int64_t)a.ids[(int64_t)q * K + mi] * ps2;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int P = lane + 64 * u;
                    if (P < ps2) acc += (double)gq[u] * (double)r[P];
                }
            }
            gw[mi] = wave_sum_f64(acc);
        }
        // Gram of Z = q - x_n (FP64), coordinates lane and lane + 64
        double z0[kMaxK], z1[kMaxK];
        const float* qf = a.qfeat + (int64_t)q * D;
        for (int mi = 0; mi < K; ++mi) {
            z0[mi] = z1[mi] = 0.0;
            if (mi < mq) {
                const int64_t id = a.ids[(int64_t)q * K + mi];
                if (lane < D)
                    z0[mi] = (double)qf[lane] - (double)join_planes(a.hi[id * a.hs + lane], a.lo[id * D + lane]);
                if (lane + 64 < D)
                    z1[mi] = (double)qf[lane + 64] -
                             (double)join_planes(a.hi[id * a.hs + lane + 64], a.lo[id * D + lane + 64]);
            }
        }
        double G[kMaxK * (kMaxK + 1) / 2];
        for (int i = 0; i < mq; ++i)
            for (int j = 0; j <= i; ++j) G[i * (i + 1) / 2 + j] = wave_sum_f64(z0[i] * z0[j] + z1[i] * z1[j]);
        if (lane == 0) {
            double tau = 0.0;
            for (int i = 0; i < mq; ++i) tau += G[i * (i + 1) / 2 + i];
            double contrib = 0.0;
            if (tau > 0.0) {
                // Cholesky of A = G + lambda tau I (lower, packed)
                double Lc[kMaxK * (kMaxK + 1) / 2];
                for (int i = 0; i < mq; ++i) {
                    for (int j = 0; j <= i; ++j) {
                        double v = G[i * (i + 1) / 2 + j] + (i == j ? a.lam * tau : 0.0);
                        for (int t = 0; t < j; ++t) v -= Lc[i * (i + 1) / 2 + t] * Lc[j * (j + 1) / 2 + t];
                        Lc[i * (i + 1) / 2 + j] = i == j ? sqrt(v) : v / Lc[j * (j + 1) / 2 + j];
                    }
                }
                auto solve = [&](const double* b, double* x) {
                    for (int i = 0; i < mq; ++i) {
                        double v = b[i];
                        for (int t = 0; t < i; ++t) v -= Lc[i * (i + 1) / 2 + t] * x[t];
                        x[i] = v / Lc[i * (i + 1) / 2 + i];
                    }
                    for (int i = mq - 1; i >= 0; --i) {
                        double v = x[i];
                        for (int t = i + 1; t < mq; ++t) v -= Lc[t * (t + 1) / 2 + i] * x[t];
                        x[i] = v / Lc[i * (i + 1) / 2 + i];
                    }
                };
                double one[kMaxK], wt[kMaxK], d[kMaxK];
                for (int i = 0; i < mq; ++i) one[i] = 1.0;
                solve(one, wt);
                double sig = 0.0;
                for (int i = 0; i < mq; ++i) sig += wt[i];
                solve(wt, d);
                double dsum = 0.0, gd = 0.0, gww = 0.0;
                for (int i = 0; i < mq; ++i) {
                    d[i] *= -tau;
                    dsum += d[i];
                    gd += gw[i] * d[i];
                    gww += gw[i] * wt[i] / sig;
                }
                contrib = (gd - gww * dsum) / sig;
            }
            a.c_lam[q] = contrib;
        }
    }
}

// dL/dw_m = <g_q, r_{n_m}> for K <= 8, one wave per patch (pixels lane + 64 u),
// into gw[q][8] (FP64, zero past m_q).
template <int U>
__global__ __launch_bounds__(256) void k_lam_gw(BackwardArgs a, double* __restrict__ gw) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int K = a.K, s = a.s, ps = kPatch * s, ps2 = ps * ps;
    const int npj = a.w - kPatch + 1;
    const int W = s * a.w;
    for (int q = blockIdx.x * wpb + (threadIdx.x >> 6); q < a.Q; q += gridDim.x * wpb) {
        const int mq = a.m[q];
        const int pi = q / npj, pj = q - (q / npj) * npj;
        float gq[U];
        int P4[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int P = lane + 64 * u;
            P4[u] = P;
            gq[u] = 0.0f;
            if (P < ps2 && mq > 0) {
                const int py = P / ps, px = P - py * ps;
                gq[u] = a.gp[(int64_t)(s * pi + py) * W + s * pj + px];
            }
        }
#pragma unroll
        for (int mi = 0; mi < 8; ++mi) {
            double acc = 0.0;
            if (mi < mq) {
                const float* r = a.resid + (int64_t)a.ids[(int64_t)q * K + mi] * ps2;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (P4[u] < ps2) acc += (double)gq[u] * (double)r[P4[u]];
            }
            acc = wave_sum_f64(acc);
            if (lane == mi) gw[(int64_t)q * 8 + mi] = acc;
        }
    }
}

// Contribution of each patch to dL/dlambda (K <= 8), one thread per patch,
// from its packed FP64 Gram matrix G and gw: with tau = tr(G) and
// A = G + lambda tau I factored again here (Cholesky),
//   w~ = A^-1 1, sigma = sum w~, d = -tau A^-1 w~,
//   dL/dlambda_q = (gw.d - (gw.w~ / sigma) sum d) / sigma.
__global__ __launch_bounds__(256) void k_lam_solve(BackwardArgs a, const double* __restrict__ gram,
                                                   const double* __restrict__ gw) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.Q) return;
    const int m = a.m[q];
    double A[36], g[8];
#pragma unroll
    for (int p = 0; p < 36; ++p) A[p] = gram[(int64_t)q * 36 + p];
#pragma unroll
    for (int i = 0; i < 8; ++i) g[i] = i < m ? gw[(int64_t)q * 8 + i] : 0.0;
    double tau = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (i < m) tau += A[i * (i + 1) / 2 + i];
    if (m <= 0 || !(tau > 0.0)) {
        a.c_lam[q] = 0.0;
        return;
    }
    // rows m..7: identity, so that the unrolled factorisation stays valid
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double& x = A[i * (i + 1) / 2 + j];
            if (i >= m || j >= m) x = i == j ? 1.0 : 0.0;
            else if (i == j) x += a.lam * tau;
        }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        double v = A[j * (j + 1) / 2 + j];
#pragma unroll
        for (int t = 0; t < j; ++t) v -= A[j * (j + 1) / 2 + t] * A[j * (j + 1) / 2 + t];
        A[j * (j + 1) / 2 + j] = sqrt(v);
#pragma unroll
        for (int i = j + 1; i < 8; ++i) {
            double t2 = A[i * (i + 1) / 2 + j];
#pragma unroll
            for (int t = 0; t < j; ++t) t2 -= A[i * (i + 1) / 2 + t] * A[j * (j + 1) / 2 + t];
            A[i * (i + 1) / 2 + j] = t2 / A[j * (j + 1) / 2 + j];
        }
    }
    auto solve = [&](const double (&b)[8], double (&x)[8]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double v = b[i];
#pragma unroll
            for (int t = 0; t < i; ++t) v -= A[i * (i + 1) / 2 + t] * x[t];
            x[i] = v / A[i * (i + 1) / 2 + i];
        }
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            double v = x[i];
#pragma unroll
            for (int t = i + 1; t < 8; ++t) v -= A[t * (t + 1) / 2 + i] * x[t];
            x[i] = v / A[i * (i + 1) / 2 + i];
        }
    };
    double one[8], wt[8], d[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) one[i] = i < m ? 1.0 : 0.0;
    solve(one, wt);
    double sig = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) sig += i < m ? wt[i] : 0.0;
    solve(wt, d);
    double dsum = 0.0, gd = 0.0, gww = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (i < m) {
            const double di = -tau * d[i];
            dsum += di;
            gd += g[i] * di;
            gww += g[i] * wt[i] / sig;
        }
    }
    a.c_lam[q] = (gd - gww * dsum) / sig;
}

hipError_t launch_lam_adj8(const BackwardArgs& a, const double* gram, double* gw, hipStream_t st) {
    if (a.Q == 0) return hipSuccess;
    if (a.K > 8 || a.s < 1 || a.s > kMaxScale) return hipErrorInvalidValue;
    int g = (a.Q + 3) / 4;
    if (g > 65536) g = 65536;
    if (kPatch * a.s * kPatch * a.s <= 256) hipLaunchKernelGGL(k_lam_gw<4>, dim3(g), dim3(256), 0, st, a, gw);
    else hipLaunchKernelGGL(k_lam_gw<kPixChunks>, dim3(g), dim3(256), 0, st, a, gw);
    hipLaunchKernelGGL(k_lam_solve, dim3((a.Q + 255) / 256), dim3(256), 0, st, a, gram, gw);
    return hipGetLastError();
}

hipError_t launch_lle_lambda_adj(const BackwardArgs& a, hipStream_t st) {
    if (a.K > kMaxK || a.D > 128 || a.s < 1 || a.s > kMaxScale) return hipErrorInvalidValue;
    int g = (a.Q + 3) / 4;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    if (kPatch * a.s * kPatch * a.s <= 256) hipLaunchKernelGGL(k_lle_lambda_adj<4>, dim3(g), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_lle_lambda_adj<kPixChunks>, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Fixed-order FP64 sum of n values: one workgroup, thread t adds t, t + 1024,
// ... in order, then a tree over the threads; the result is rounded to fp32.
__global__ __launch_bounds__(1024) void k_sum_f64(const double* __restrict__ x, int64_t n, float* __restrict__ out) {
    __shared__ double s[1024];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc += x[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)s[0];
}

hipError_t launch_sum_f64(const double* x, int64_t n, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(1024), 0, st, x, n, out);
    return hipGetLastError();
}

// ---- dictionary gradient ----------------------------------------------------
// Neighbour list entries e = q K + m as (key = dictionary row, value = e);
// entries past m_q get the key `none` and sort last.
__global__ void k_nbr_pairs(const int32_t* __restrict__ ids, const int32_t* __restrict__ m, int Q, int K,
                            uint32_t none, uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
    const int64_t total = (int64_t)Q * K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / K), mi = (int)(e % K);
        key[e] = mi < m[q] ? (uint32_t)ids[e] : none;
        val[e] = (uint32_t)e;
    }
}

hipError_t launch_nbr_pairs(const int32_t* ids, const int32_t* m, int Q, int K, uint32_t none, uint32_t* key,
                            uint32_t* val, hipStream_t st) {
    hipLaunchKernelGGL(k_nbr_pairs, grid1((int64_t)Q * K), dim3(256), 0, st, ids, m, Q, K, none, key, val);
    return hipGetLastError();
}

// Gradient of each dictionary row that some patch uses: the sum over its
// entries (q, m) of w_qm g_q, with the pairs sorted stably by row. Pass 1:
// a wave per chunk of 64 consecutive entries (one per lane) sums each run of
// equal rows inside the chunk in entry order (lane = pixel); a run that lies
// wholly in the chunk is written, while a run that crosses a chunk border
// leaves its partial sum in the chunk's first or last slot. Pass 2: a wave
// per run that starts in a chunk and continues into the next adds the
// partial sums in chunk order. The result depends only on the sorted pairs:
// equal calls give equal gradients.
struct DictGradChunk {
    uint32_t key_last;   // row of the chunk's last run
    uint8_t nseg;        // runs (of used rows) starting or continuing in the chunk
    uint8_t first_cont;  // the first run continues from the previous chunk
    uint8_t last_cont;   // the last run continues into the next chunk
    uint8_t last_start;  // the last run starts in this chunk
};

template <int U>
__global__ __launch_bounds__(256) void k_dict_grad(const uint32_t* __restrict__ key, const uint32_t* __restrict__ val,
                                                   int64_t n_ent, uint32_t none, const float* __restrict__ wts,
                                                   const float* __restrict__ gp, int w, int s, int K,
                                                   float* __restrict__ g_r, float* __restrict__ part,
                                                   DictGradChunk* __restrict__ info) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int ps = kPatch * s, ps2 = ps * ps;
    const int npj = w - kPatch + 1, W = s * w;
    int off[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int P = lane + 64 * u;
        off[u] = P < ps2 ? (P / ps) * W + P % ps : 0;
    }
    const int64_t nchunk = (n_ent + 63) / 64;
    for (int64_t c = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); c < nchunk; c += (int64_t)gridDim.x * wpb) {
        const int64_t base = c * 64;
        const int64_t e = base + lane;
        const bool in = e < n_ent;
        const uint32_t k = in ? key[e] : none;
        const uint32_t kprev = (in && e > 0) ? key[e - 1] : none;
        const uint32_t knext = (e + 1 < n_ent) ? key[e + 1] : none;
        const uint32_t v = in ? val[e] : 0u;
        const float wv = (in && k != none) ? wts[v] : 0.0f;
        // segment starts inside the chunk: first lane, or a change of row
        const uint64_t seg = __ballot(in && k != none && (lane == 0 || k != kprev));
        const uint64_t ends = __ballot(in && k != none && (lane == 63 || e + 1 == n_ent || knext != k));
        uint64_t todo = seg;
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int stop = __builtin_ctzll(ends & (~0ull << src));   // last entry of the segment
            const uint32_t kk = __shfl(k, src);
            float acc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) acc[u] = 0.0f;
            for (int j = src; j <= stop; ++j) {
                const uint32_t vv = __shfl(v, j);
                const float ww = __shfl(wv, j);
                const int q = (int)(vv / (uint32_t)K);
                const int pi = q / npj, pj = q - pi * npj;
                const float* g = gp + (int64_t)s * pi * W + (int64_t)s * pj;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (lane + 64 * u < ps2) acc[u] = fmaf(ww, g[off[u]], acc[u]);
            }
            const bool from_prev = src == 0 && __shfl(kprev, 0) == kk;
            const bool into_next = stop == 63 && __shfl(knext, 63) == kk;
            float* dst = g_r + (int64_t)kk * ps2;
            if (from_prev) dst = part + (c * 2) * ps2;
            else if (into_next) dst = part + (c * 2 + 1) * ps2;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int P = lane + 64 * u;
                if (P < ps2) dst[P] = acc[u];
            }
        }
        const int last = seg ? 63 - __builtin_clzll(seg) : 0;
        const uint32_t kl = __shfl(k, last);
        const uint32_t k0 = __shfl(k, 0), kp0 = __shfl(kprev, 0);
        const uint32_t k63 = __shfl(k, 63), kn63 = __shfl(knext, 63);
        if (lane == 0) {
            DictGradChunk ci;
            ci.key_last = seg ? kl : none;
            ci.nseg = (uint8_t)__popcll(seg);
            ci.first_cont = (uint8_t)(k0 != none && kp0 == k0);
            ci.last_cont = (uint8_t)(seg && k63 == kl && kn63 == kl);
            ci.last_start = (uint8_t)(seg && !(last == 0 && kp0 == kl));
            info[c] = ci;
        }
    }
}

// Pass 2: runs that cross chunk borders, from the chunk where they start.
template <int U>
__global__ __launch_bounds__(256) void k_dict_grad_join(int64_t n_ent, int s, const float* __restrict__ part,
                                                        const DictGradChunk* __restrict__ info, float* __restrict__ g_r) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int ps = kPatch * s, ps2 = ps * ps;
    const int64_t nchunk = (n_ent + 63) / 64;
    for (int64_t c = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); c < nchunk; c += (int64_t)gridDim.x * wpb) {
        const DictGradChunk ci = info[c];
        if (!ci.last_cont || !ci.last_start) continue;
        // the run starts in chunk c and continues: its partial is in slot 1,
        // and in slot 0 of every later chunk it reaches
        const float* p0 = part + (c * 2 + 1) * ps2;
        float acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = lane + 64 * u < ps2 ? p0[lane + 64 * u] : 0.0f;
        for (int64_t cc = c + 1; cc < nchunk; ++cc) {
            const DictGradChunk cn = info[cc];
            const float* pp = part + (cc * 2) * ps2;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (lane + 64 * u < ps2) acc[u] += pp[lane + 64 * u];
            if (!(cn.nseg == 1 && cn.last_cont)) break;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int P = lane + 64 * u;
            if (P < ps2) g_r[(int64_t)ci.key_last * ps2 + P] = acc[u];
        }
    }
}

hipError_t launch_dict_grad(const uint32_t* key, const uint32_t* val, int64_t n_ent, uint32_t none, const float* wts,
                            const float* gp, int w, int s, int K, float* g_r, float* part, void* info,
                            hipStream_t st) {
    if (s < 1 || s > kMaxScale) return hipErrorInvalidValue;
    if (n_ent == 0) return hipSuccess;
    const int64_t nchunk = (n_ent + 63) / 64;
    int64_t g = (nchunk + 3) / 4;
    if (g > 65536) g = 65536;
    DictGradChunk* ci = static_cast<DictGradChunk*>(info);
    if (kPatch * s * kPatch * s <= 256) {
        hipLaunchKernelGGL(k_dict_grad<4>, dim3((unsigned)g), dim3(256), 0, st, key, val, n_ent, none, wts, gp, w, s, K,
                           g_r, part, ci);
        hipLaunchKernelGGL(k_dict_grad_join<4>, dim3((unsigned)g), dim3(256), 0, st, n_ent, s, part, ci, g_r);
    } else {
        hipLaunchKernelGGL(k_dict_grad<kPixChunks>, dim3((unsigned)g), dim3(256), 0, st, key, val, n_ent, none, wts, gp,
                           w, s, K, g_r, part, ci);
        hipLaunchKernelGGL(k_dict_grad_join<kPixChunks>, dim3((unsigned)g), dim3(256), 0, st, n_ent, s, part, ci, g_r);
    }
    return hipGetLastError();
}

}  // namespace zh
