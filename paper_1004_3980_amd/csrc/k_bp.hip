// Back-projection update with the approximate cross bilateral filter
// (Section 4, the update after Eq. Err_img; Section 4.3, Eq. sx2 and
// Eq. bl_filter_3):
//
//   E  = bicubic upsampling of the LR error e = I_L - (g * I) decimated
//   F  = C * E, C a Gaussian of sigma_s over (2R+1)^2, R = ceil(3 sigma_s),
//        normalised over the taps inside the image (separable)
//   mu = mean of I over the in-image pixels of the same window
//   S  = exp(-(I - mu)^2 / (2 sigma_r^2))
//   I' = I + S * F
//
// One workgroup per 32x32 output tile; I and E are staged with an R-pixel
// halo in LDS and both separable passes (Gaussian of E, box sum of I) run
// from LDS. The LR error itself comes from the FP64 degradation kernel.
#include <cmath>

#include "zh_internal.h"

namespace zh {

constexpr int kBpTile = 32;
constexpr int kBpMaxR = 8;
constexpr int kBpReg = kBpTile + 2 * kBpMaxR;

// TERMS: instead of the update, write F, S and a = I - mu (the pieces the
// adjoint of the iteration needs) to out, out + H W and out + 2 H W.
template <bool TERMS>
__global__ __launch_bounds__(256) void k_bp_update(const float* __restrict__ I, const float* __restrict__ e,
                                                   int H, int W, int h, int w, int s, int R, float sigma_s,
                                                   float inv2sr2, float* __restrict__ out) {
    __shared__ float sI[kBpReg][kBpReg];
    __shared__ float sE[kBpReg][kBpReg];
    __shared__ float sHE[kBpReg][kBpTile];
    __shared__ float sHB[kBpReg][kBpTile];
    __shared__ float sg[2 * kBpMaxR + 1];
    const int Y0 = blockIdx.y * kBpTile, X0 = blockIdx.x * kBpTile;
    const int reg = kBpTile + 2 * R;
    if (threadIdx.x < 2 * R + 1) {
        const float d = (float)((int)threadIdx.x - R);
        sg[threadIdx.x] = expf(-(d * d) / (2.0f * sigma_s * sigma_s));
    }
    for (int t = threadIdx.x; t < reg * reg; t += blockDim.x) {
        const int r = t / reg, c = t % reg;
        const int Y = Y0 - R + r, X = X0 - R + c;
        const bool in = Y >= 0 && Y < H && X >= 0 && X < W;
        sI[r][c] = in ? I[(int64_t)Y * W + X] : 0.0f;
        sE[r][c] = in ? bicubic_at(e, h, w, s, Y, X) : 0.0f;
    }
    __syncthreads();
    // horizontal passes over every staged row, the tile's columns
    for (int t = threadIdx.x; t < reg * kBpTile; t += blockDim.x) {
        const int r = t / kBpTile, c = t % kBpTile;
        const int X = X0 + c;
        float ge = 0.0f, gn = 0.0f, bs = 0.0f;
        for (int d = -R; d <= R; ++d) {
            const int x = X + d;
            if (x < 0 || x >= W) continue;
            const float g = sg[d + R];
            ge = fmaf(g, sE[r][c + R + d], ge);
            gn += g;
            bs += sI[r][c + R + d];
        }
        sHE[r][c] = gn > 0.0f ? ge / gn : 0.0f;
        sHB[r][c] = bs;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kBpTile * kBpTile; t += blockDim.x) {
        const int r = t / kBpTile, c = t % kBpTile;
        const int Y = Y0 + r, X = X0 + c;
        if (Y >= H || X >= W) continue;
        float ge = 0.0f, gn = 0.0f, bs = 0.0f;
        for (int d = -R; d <= R; ++d) {
            const int y = Y + d;
            if (y < 0 || y >= H) continue;
            const float g = sg[d + R];
            ge = fmaf(g, sHE[r + R + d][c], ge);
            gn += g;
            bs += sHB[r + R + d][c];
        }
        const int ny = min(H - 1, Y + R) - max(0, Y - R) + 1;
        const int nx = min(W - 1, X + R) - max(0, X - R) + 1;
        const float Ixy = sI[r + R][c + R];
        const float mu = bs / (float)(ny * nx);
        const float dd = Ixy - mu;
        const float S = expf(-dd * dd * inv2sr2);
        if (TERMS) {
            const int64_t hw = (int64_t)H * W, o = (int64_t)Y * W + X;
            out[o] = ge / gn;
            out[hw + o] = S;
            out[2 * hw + o] = dd;
        } else {
            out[(int64_t)Y * W + X] = fmaf(S, ge / gn, Ixy);
        }
    }
}

hipError_t launch_bp_update(const float* I, const float* e, int H, int W, int h, int w, int scale,
                            float sigma_s, float sigma_r, float* out, hipStream_t st) {
    const int R = (int)std::ceil(3.0 * (double)sigma_s);
    if (R > kBpMaxR || R < 0) return hipErrorInvalidValue;
    const float inv2sr2 = sigma_r > 0.0f && std::isfinite(sigma_r) ? 1.0f / (2.0f * sigma_r * sigma_r) : 0.0f;
    dim3 grid((W + kBpTile - 1) / kBpTile, (H + kBpTile - 1) / kBpTile);
    hipLaunchKernelGGL((k_bp_update<false>), grid, dim3(256), 0, st, I, e, H, W, h, w, scale, R, sigma_s, inv2sr2,
                       out);
    return hipGetLastError();
}

hipError_t launch_bp_terms(const float* I, const float* e, int H, int W, int h, int w, int scale,
                           float sigma_s, float sigma_r, float* FSa, hipStream_t st) {
    const int R = (int)std::ceil(3.0 * (double)sigma_s);
    if (R > kBpMaxR || R < 0) return hipErrorInvalidValue;
    const float inv2sr2 = sigma_r > 0.0f && std::isfinite(sigma_r) ? 1.0f / (2.0f * sigma_r * sigma_r) : 0.0f;
    dim3 grid((W + kBpTile - 1) / kBpTile, (H + kBpTile - 1) / kBpTile);
    hipLaunchKernelGGL((k_bp_update<true>), grid, dim3(256), 0, st, I, e, H, W, h, w, scale, R, sigma_s, inv2sr2,
                       FSa);
    return hipGetLastError();
}

}  // namespace zh
