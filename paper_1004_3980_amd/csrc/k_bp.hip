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

// One T x T output tile with origin (Y0, X0). TERMS: instead of the update,
// write F, S and a = I - mu (the pieces the adjoint of the iteration needs)
// to out, out + H W and out + 2 H W.
//
// E on the staged region comes from the LR error patch under it: the patch
// (clamped indices, so the border replicates) is staged in LDS, upsampled
// along x for each of its rows, then along y, with the same fused
// multiply-adds in the same order as bicubic_at (bitwise its values). Tiles
// whose halo lies inside the image take the Gaussian and box sums without
// per-tap border tests (the same operations in the same order).
template <int T, bool TERMS>
__device__ __forceinline__ void bp_tile(const float* __restrict__ I, const float* __restrict__ e, int H, int W, int h,
                                        int w, int s, int R, float sigma_s, float inv2sr2, float* __restrict__ out,
                                        int Y0, int X0) {
    constexpr int REG = T + 2 * kBpMaxR;
    // LR rows / columns under REG HR pixels at zoom >= 2: REG / 2 + 4
    constexpr int LREG = REG / 2 + 5;
    __shared__ float sI[REG][REG];
    __shared__ float sE[REG][REG];          // first the staged LR error patch [LREG][LREG]
    __shared__ float sH[2][REG][T];         // the passes' sums; first the x pass of the upsampling [LREG][REG]
    __shared__ float sg[2 * kBpMaxR + 1];
    __shared__ float sw[kMaxScale][4];      // Keys' weights of each phase
    static_assert(LREG * LREG <= REG * REG && LREG * REG <= 2 * REG * T, "LDS aliases");
    float (*sHE)[T] = sH[0];
    float (*sHB)[T] = sH[1];
    float* eL = &sE[0][0];
    float* xU = &sH[0][0][0];
    const int reg = T + 2 * R;
    if ((int)threadIdx.x < 2 * R + 1) {
        const float d = (float)((int)threadIdx.x - R);
        sg[threadIdx.x] = expf(-(d * d) / (2.0f * sigma_s * sigma_s));
    }
    if ((int)threadIdx.x < 4 * s && s <= kMaxScale) {
        const int ph = threadIdx.x >> 2, a = threadIdx.x & 3;
        sw[ph][a] = keys_w((float)ph / (float)s - (float)(a - 1));
    }
    for (int t = threadIdx.x; t < reg * reg; t += blockDim.x) {
        const int r = t / reg, c = t % reg;
        const int Y = Y0 - R + r, X = X0 - R + c;
        const bool in = Y >= 0 && Y < H && X >= 0 && X < W;
        sI[r][c] = in ? I[(int64_t)Y * W + X] : 0.0f;
    }
    // the staged region's in-image HR rows [ya, yb] and columns [xa, xb]
    const int ya = max(0, Y0 - R), yb = min(H - 1, Y0 - R + reg - 1);
    const int xa = max(0, X0 - R), xb = min(W - 1, X0 - R + reg - 1);
    const bool sep = s >= 2 && s <= kMaxScale;
    const int la = ya / s - 1, lc = xa / s - 1;          // first staged LR row / column
    const int nlr = yb / s + 2 - la + 1, nlc = xb / s + 2 - lc + 1;
    if (sep) {
        for (int t = threadIdx.x; t < nlr * nlc; t += blockDim.x) {
            const int r = t / nlc, c = t % nlc;
            eL[r * LREG + c] = e[(int64_t)clampi(la + r, 0, h - 1) * w + clampi(lc + c, 0, w - 1)];
        }
    }
    __syncthreads();
    if (sep) {
        // along x: every staged LR row at the region's columns
        for (int t = threadIdx.x; t < nlr * reg; t += blockDim.x) {
            const int r = t / reg, c = t % reg;
            const int X = X0 - R + c;
            if (X < xa || X > xb) continue;
            const int j0 = X / s;
            const float* wx = sw[X - j0 * s];
            const float* row = eL + r * LREG + (j0 - 1 - lc);
            float v = 0.0f;
#pragma unroll
            for (int b = 0; b < 4; ++b) v = fmaf(wx[b], row[b], v);
            xU[r * REG + c] = v;
        }
        __syncthreads();
        // along y
        for (int t = threadIdx.x; t < reg * reg; t += blockDim.x) {
            const int r = t / reg, c = t % reg;
            const int Y = Y0 - R + r, X = X0 - R + c;
            float v = 0.0f;
            if (Y >= 0 && Y < H && X >= 0 && X < W) {
                const int i0 = Y / s;
                const float* wy = sw[Y - i0 * s];
                const int r0 = i0 - 1 - la;
#pragma unroll
                for (int a = 0; a < 4; ++a) v = fmaf(wy[a], xU[(r0 + a) * REG + c], v);
            }
            sE[r][c] = v;
        }
    } else {
        for (int t = threadIdx.x; t < reg * reg; t += blockDim.x) {
            const int r = t / reg, c = t % reg;
            const int Y = Y0 - R + r, X = X0 - R + c;
            const bool in = Y >= 0 && Y < H && X >= 0 && X < W;
            sE[r][c] = in ? bicubic_at(e, h, w, s, Y, X) : 0.0f;
        }
    }
    __syncthreads();
    const bool inner = Y0 - R >= 0 && X0 - R >= 0 && Y0 + T + R <= H && X0 + T + R <= W;
    // horizontal passes over every staged row, the tile's columns
    for (int t = threadIdx.x; t < reg * T; t += blockDim.x) {
        const int r = t / T, c = t % T;
        const int X = X0 + c;
        float ge = 0.0f, gn = 0.0f, bs = 0.0f;
        if (inner) {
            for (int d = -R; d <= R; ++d) {
                const float g = sg[d + R];
                ge = fmaf(g, sE[r][c + R + d], ge);
                gn += g;
                bs += sI[r][c + R + d];
            }
        } else {
            for (int d = -R; d <= R; ++d) {
                const int x = X + d;
                if (x < 0 || x >= W) continue;
                const float g = sg[d + R];
                ge = fmaf(g, sE[r][c + R + d], ge);
                gn += g;
                bs += sI[r][c + R + d];
            }
        }
        sHE[r][c] = gn > 0.0f ? ge / gn : 0.0f;
        sHB[r][c] = bs;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < T * T; t += blockDim.x) {
        const int r = t / T, c = t % T;
        const int Y = Y0 + r, X = X0 + c;
        if (Y >= H || X >= W) continue;
        float ge = 0.0f, gn = 0.0f, bs = 0.0f;
        if (inner) {
            for (int d = -R; d <= R; ++d) {
                const float g = sg[d + R];
                ge = fmaf(g, sHE[r + R + d][c], ge);
                gn += g;
                bs += sHB[r + R + d][c];
            }
        } else {
            for (int d = -R; d <= R; ++d) {
                const int y = Y + d;
                if (y < 0 || y >= H) continue;
                const float g = sg[d + R];
                ge = fmaf(g, sHE[r + R + d][c], ge);
                gn += g;
                bs += sHB[r + R + d][c];
            }
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

template <bool TERMS>
__global__ __launch_bounds__(256) void k_bp_update(const float* __restrict__ I, const float* __restrict__ e,
                                                   int H, int W, int h, int w, int s, int R, float sigma_s,
                                                   float inv2sr2, float* __restrict__ out) {
    bp_tile<kBpTile, TERMS>(I, e, H, W, h, w, s, R, sigma_s, inv2sr2, out, blockIdx.y * kBpTile,
                            blockIdx.x * kBpTile);
}

int bp_tiles(int H, int W, int tile) { return ((H + tile - 1) / tile) * ((W + tile - 1) / tile); }

// Batched update: persistent workgroups take (image, tile) items from the
// counter until none is left; every workgroup exits after one failed take.
template <int T>
__global__ __launch_bounds__(256) void k_b_bp_update(const BatchImage* __restrict__ im, int n, int64_t n_tiles, int s,
                                                     int R, float sigma_s, float inv2sr2, const float* __restrict__ e,
                                                     int parity, unsigned int* __restrict__ counter) {
    __shared__ int64_t item;
    for (;;) {
        if (threadIdx.x == 0) item = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t it = item;
        __syncthreads();
        if (it >= n_tiles) break;
        const BatchImage& b = im[batch_image_of<&BatchImage::tile_off>(im, n, it)];
        const int H = s * b.h, W = s * b.w;
        const int tx = (W + T - 1) / T;
        const int local = (int)(it - b.tile_off);
        const float* I = parity ? b.scr : b.out;
        float* out = parity ? b.out : b.scr;
        bp_tile<T, false>(I, e + b.lr_off, H, W, b.h, b.w, s, R, sigma_s, inv2sr2, out, (local / tx) * T,
                          (local % tx) * T);
        __syncthreads();
    }
}

__global__ void k_b_zero_u32(unsigned int* p) { *p = 0u; }

// Results of an odd number of iterations are in scr: copy them to out.
__global__ void k_b_copy_scr(const BatchImage* __restrict__ im, int n, int64_t total, int s) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const BatchImage& b = im[batch_image_of<&BatchImage::hr_off>(im, n, idx)];
        const int64_t r = idx - b.hr_off;
        b.out[r] = b.scr[r];
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

hipError_t launch_b_bp_update(const BatchImage* im, int n, int64_t n_tiles, int tile, int grid, int scale,
                              float sigma_s, float sigma_r, const float* e, int parity, unsigned int* counter,
                              hipStream_t st) {
    const int R = (int)std::ceil(3.0 * (double)sigma_s);
    if (R > kBpMaxR || R < 0 || (tile != 16 && tile != 32) || grid < 1) return hipErrorInvalidValue;
    if (n_tiles == 0) return hipSuccess;
    const float inv2sr2 = sigma_r > 0.0f && std::isfinite(sigma_r) ? 1.0f / (2.0f * sigma_r * sigma_r) : 0.0f;
    hipLaunchKernelGGL(k_b_zero_u32, dim3(1), dim3(1), 0, st, counter);
    if (tile == 16)
        hipLaunchKernelGGL((k_b_bp_update<16>), dim3(grid), dim3(256), 0, st, im, n, n_tiles, scale, R, sigma_s, inv2sr2,
                           e, parity, counter);
    else
        hipLaunchKernelGGL((k_b_bp_update<32>), dim3(grid), dim3(256), 0, st, im, n, n_tiles, scale, R, sigma_s, inv2sr2,
                           e, parity, counter);
    return hipGetLastError();
}

hipError_t launch_b_copy_scr(const BatchImage* im, int n, int64_t hr_total, int scale, hipStream_t st) {
    if (hr_total == 0) return hipSuccess;
    int64_t g = (hr_total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_b_copy_scr, dim3((unsigned)g), dim3(256), 0, st, im, n, hr_total, scale);
    return hipGetLastError();
}

}  // namespace zh
