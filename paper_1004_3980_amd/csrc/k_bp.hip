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
    constexpr int NT = 2 * kBpMaxR + 1;
    __shared__ float sI[REG][REG];
    __shared__ float sE[REG][REG];          // first the staged LR error patch [LREG][LREG]
    __shared__ float sH[2][REG][T];         // the passes' sums; first the x pass of the upsampling [LREG][REG]
    __shared__ float sg[NT];
    __shared__ float sw[kMaxScale][4];      // Keys' weights of each phase
    // per staged row / column in the image: the first of its four LR taps
    // relative to the staged LR patch (<< 8) and its phase; -1 outside the image
    __shared__ int srow[REG], scol[REG];
    static_assert(LREG * LREG <= REG * REG && LREG * REG <= 2 * REG * T, "LDS aliases");
    float (*sHE)[T] = sH[0];
    float (*sHB)[T] = sH[1];
    float* eL = &sE[0][0];
    float* xU = &sH[0][0][0];
    const int reg = T + 2 * R;
    const int tid = threadIdx.x;
    if (tid < 2 * R + 1) {
        const float d = (float)(tid - R);
        sg[tid] = expf(-(d * d) / (2.0f * sigma_s * sigma_s));
    }
    if (tid < 4 * s && s <= kMaxScale) {
        const int ph = tid >> 2, a = tid & 3;
        sw[ph][a] = keys_w((float)ph / (float)s - (float)(a - 1));
    }
    // loops over the staged region run over REG x REG (a constant divisor)
    // and skip what lies past reg
    for (int t = tid; t < REG * REG; t += blockDim.x) {
        const int r = t / REG, c = t - r * REG;
        if (r >= reg || c >= reg) continue;
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
        for (int t = tid; t < LREG * LREG; t += blockDim.x) {
            const int r = t / LREG, c = t - r * LREG;
            if (r >= nlr || c >= nlc) continue;
            eL[r * LREG + c] = e[(int64_t)clampi(la + r, 0, h - 1) * w + clampi(lc + c, 0, w - 1)];
        }
        if (tid < reg) {
            const int Y = Y0 - R + tid;
            const int i0 = Y / s;
            srow[tid] = Y < ya || Y > yb ? -1 : ((i0 - 1 - la) << 8) | (Y - i0 * s);
        } else if (tid >= 64 && tid < 64 + reg) {
            const int c = tid - 64;
            const int X = X0 - R + c;
            const int j0 = X / s;
            scol[c] = X < xa || X > xb ? -1 : ((j0 - 1 - lc) << 8) | (X - j0 * s);
        }
    }
    __syncthreads();
    if (sep) {
        // along x: every staged LR row at the region's columns
        for (int t = tid; t < LREG * REG; t += blockDim.x) {
            const int r = t / REG, c = t - r * REG;
            if (r >= nlr || c >= reg) continue;
            const int sc = scol[c];
            if (sc < 0) continue;
            const float* wx = sw[sc & 0xFF];
            const float* row = eL + r * LREG + (sc >> 8);
            float v = 0.0f;
#pragma unroll
            for (int b = 0; b < 4; ++b) v = fmaf(wx[b], row[b], v);
            xU[r * REG + c] = v;
        }
        __syncthreads();
        // along y
        for (int t = tid; t < REG * REG; t += blockDim.x) {
            const int r = t / REG, c = t - r * REG;
            if (r >= reg || c >= reg) continue;
            const int sr = srow[r];
            float v = 0.0f;
            if (sr >= 0 && scol[c] >= 0) {
                const float* wy = sw[sr & 0xFF];
                const int r0 = sr >> 8;
#pragma unroll
                for (int a = 0; a < 4; ++a) v = fmaf(wy[a], xU[(r0 + a) * REG + c], v);
            }
            sE[r][c] = v;
        }
    } else {
        for (int t = tid; t < REG * REG; t += blockDim.x) {
            const int r = t / REG, c = t - r * REG;
            if (r >= reg || c >= reg) continue;
            const int Y = Y0 - R + r, X = X0 - R + c;
            const bool in = Y >= 0 && Y < H && X >= 0 && X < W;
            sE[r][c] = in ? bicubic_at(e, h, w, s, Y, X) : 0.0f;
        }
    }
    __syncthreads();
    const bool inner = Y0 - R >= 0 && X0 - R >= 0 && Y0 + T + R <= H && X0 + T + R <= W;
    const int nt = 2 * R + 1;
    // the output of pixel (r, c) of the tile from its vertical sums
    auto emit = [&](int r, int c, float ge, float gn, float bs) {
        const int Y = Y0 + r, X = X0 + c;
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
    };
    if (inner) {
        // no tap leaves the image: four adjacent outputs a thread, their
        // taps d = -R .. R in order from registers (the same operations as
        // the one-output loops below)
        for (int t = tid; t < reg * (T / 4); t += blockDim.x) {
            const int r = t / (T / 4), c = 4 * (t % (T / 4));
            // columns past the last tap (c + q >= reg) are read and not used
            float ev[NT + 3], iv[NT + 3];
#pragma unroll
            for (int q = 0; q < (NT + 3) / 4; ++q) {
                const float4 x = *reinterpret_cast<const float4*>(&sE[r][c + 4 * q]);
                const float4 y = *reinterpret_cast<const float4*>(&sI[r][c + 4 * q]);
                ev[4 * q] = x.x, ev[4 * q + 1] = x.y, ev[4 * q + 2] = x.z, ev[4 * q + 3] = x.w;
                iv[4 * q] = y.x, iv[4 * q + 1] = y.y, iv[4 * q + 2] = y.z, iv[4 * q + 3] = y.w;
            }
            float ge[4] = {0.0f, 0.0f, 0.0f, 0.0f}, bs[4] = {0.0f, 0.0f, 0.0f, 0.0f}, gn = 0.0f;
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                if (u >= nt) break;
                const float g = sg[u];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    ge[j] = fmaf(g, ev[j + u], ge[j]);
                    bs[j] += iv[j + u];
                }
                gn += g;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sHE[r][c + j] = gn > 0.0f ? ge[j] / gn : 0.0f;
                sHB[r][c + j] = bs[j];
            }
        }
        __syncthreads();
        for (int t = tid; t < (T / 4) * T; t += blockDim.x) {
            const int r = 4 * (t / T), c = t % T;
            float hv[NT + 3], bv[NT + 3];
            // rows past the last tap (r + q >= reg) are read and not used
#pragma unroll
            for (int q = 0; q < NT + 3; ++q) {
                hv[q] = sHE[r + q][c];
                bv[q] = sHB[r + q][c];
            }
            float ge[4] = {0.0f, 0.0f, 0.0f, 0.0f}, bs[4] = {0.0f, 0.0f, 0.0f, 0.0f}, gn = 0.0f;
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                if (u >= nt) break;
                const float g = sg[u];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    ge[j] = fmaf(g, hv[j + u], ge[j]);
                    bs[j] += bv[j + u];
                }
                gn += g;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) emit(r + j, c, ge[j], gn, bs[j]);
        }
        return;
    }
    // horizontal passes over every staged row, the tile's columns; the taps
    // d = -R .. R in order, those outside the image left out
    for (int t = tid; t < reg * T; t += blockDim.x) {
        const int r = t / T, c = t % T;
        const int X = X0 + c;
        float ge = 0.0f, gn = 0.0f, bs = 0.0f;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            if (u >= nt) break;
            const int x = X + u - R;
            if (x < 0 || x >= W) continue;
            const float g = sg[u];
            ge = fmaf(g, sE[r][c + u], ge);
            gn += g;
            bs += sI[r][c + u];
        }
        sHE[r][c] = gn > 0.0f ? ge / gn : 0.0f;
        sHB[r][c] = bs;
    }
    __syncthreads();
    for (int t = tid; t < T * T; t += blockDim.x) {
        const int r = t / T, c = t % T;
        const int Y = Y0 + r, X = X0 + c;
        if (Y >= H || X >= W) continue;
        float ge = 0.0f, gn = 0.0f, bs = 0.0f;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            if (u >= nt) break;
            const int y = Y + u - R;
            if (y < 0 || y >= H) continue;
            const float g = sg[u];
            ge = fmaf(g, sHE[r + u][c], ge);
            gn += g;
            bs += sHB[r + u][c];
        }
        emit(r, c, ge, gn, bs);
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
