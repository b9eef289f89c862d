// Image-side kernels: degradation (Section 2.1: Gaussian blur then
// decimation), the gradient maps and patch features of Section 4.1, cutting
// of the LR/HR training pairs, and bicubic upsampling.
//
// The degradation and the features are evaluated in FP64 in a fixed order
// and rounded once to fp32, so the stored LR images and features are
// reproducible bit for bit by any implementation that follows the same
// order (the file is compiled without multiply-add contraction).
#include "zh_internal.h"

namespace zh {

// (g * hr)[s i, s j] in FP64: horizontal pass along each needed row, then the
// vertical combination, both accumulating taps in ascending offset order.
__device__ __forceinline__ double blur_at(const float* __restrict__ hr, int H, int W, int y, int x,
                                          const Taps& t) {
    double acc = 0.0;
    for (int a = -t.R; a <= t.R; ++a) {
        const float* row = hr + (int64_t)clampi(y + a, 0, H - 1) * W;
        double hrow = 0.0;
        for (int b = -t.R; b <= t.R; ++b) hrow = hrow + t.g[b + t.R] * (double)row[clampi(x + b, 0, W - 1)];
        acc = acc + t.g[a + t.R] * hrow;
    }
    return acc;
}

__global__ void k_degrade(const float* __restrict__ hr, int n_img, int H, int W, int scale, Taps t,
                          float* __restrict__ lr) {
    const int h = (H + scale - 1) / scale, w = (W + scale - 1) / scale;
    const int64_t total = (int64_t)n_img * h * w;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t im = idx / ((int64_t)h * w);
        const int r = (int)(idx % ((int64_t)h * w));
        const int i = r / w, j = r % w;
        lr[idx] = (float)blur_at(hr + im * (int64_t)H * W, H, W, scale * i, scale * j, t);
    }
}

__global__ void k_degrade_residual(const float* __restrict__ hr, int H, int W, int scale, Taps t,
                                   const float* __restrict__ lr_ref, float* __restrict__ e) {
    const int h = (H + scale - 1) / scale, w = (W + scale - 1) / scale;
    const int64_t total = (int64_t)h * w;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / w), j = (int)(idx % w);
        e[idx] = (float)((double)lr_ref[idx] - blur_at(hr, H, W, scale * i, scale * j, t));
    }
}

// The same LR error by LR tiles of kDrI x kDrJ: the HR rows and columns under
// a tile (clamped indices: replicate border) are staged in LDS, the
// horizontal FP64 sums are formed once per (HR row, LR column) and shared by
// the LR rows that use them, then the vertical sums; each value is the
// blur_at sum to the bit (same products, same order).
constexpr int kDrI = 8, kDrJ = 32;
// The LR tile with origin (i0, j0) of an h x w LR error (h, w from H, W).
__device__ __forceinline__ void degrade_tile(const float* __restrict__ hr, int H, int W, int scale, const Taps& t,
                                             const float* __restrict__ lr_ref, float* __restrict__ e, int i0, int j0,
                                             unsigned char* smem) {
    const int h = (H + scale - 1) / scale, w = (W + scale - 1) / scale;
    const int R = t.R;
    const int ny = scale * (kDrI - 1) + 2 * R + 1, nx = scale * (kDrJ - 1) + 2 * R + 1;
    double* hrow = reinterpret_cast<double*>(smem);                       // [ny][kDrJ]
    float* sh = reinterpret_cast<float*>(smem + sizeof(double) * ny * kDrJ);   // [ny][nx]
    const int y0 = scale * i0 - R, x0 = scale * j0 - R;
    for (int q = threadIdx.x; q < ny * nx; q += blockDim.x) {
        const int r = q / nx, c = q % nx;
        sh[q] = hr[(int64_t)clampi(y0 + r, 0, H - 1) * W + clampi(x0 + c, 0, W - 1)];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < ny * kDrJ; q += blockDim.x) {
        const int r = q / kDrJ, jj = q % kDrJ;
        const float* row = sh + r * nx + scale * jj;
        double v = 0.0;
        for (int b = 0; b <= 2 * R; ++b) v = v + t.g[b] * (double)row[b];
        hrow[q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kDrI * kDrJ; q += blockDim.x) {
        const int ii = q / kDrJ, jj = q % kDrJ;
        const int i = i0 + ii, j = j0 + jj;
        if (i >= h || j >= w) continue;
        double acc = 0.0;
        for (int a = 0; a <= 2 * R; ++a) acc = acc + t.g[a] * hrow[(scale * ii + a) * kDrJ + jj];
        e[(int64_t)i * w + j] = (float)((double)lr_ref[(int64_t)i * w + j] - acc);
    }
}

__global__ __launch_bounds__(256) void k_degrade_residual_t(const float* __restrict__ hr, int H, int W, int scale,
                                                            Taps t, const float* __restrict__ lr_ref,
                                                            float* __restrict__ e) {
    extern __shared__ __align__(16) unsigned char smem[];
    degrade_tile(hr, H, W, scale, t, lr_ref, e, blockIdx.y * kDrI, blockIdx.x * kDrJ, smem);
}

// Batched, by tiles: workgroup b takes tile b of the concatenated tile lists
// of the images (the current estimate in out for parity 0, scr for parity 1;
// image b's error at e + lr_off); the grid may be rounded up past the last tile.
__global__ __launch_bounds__(256) void k_b_degrade_residual_t(const BatchImage* __restrict__ im, int n, int64_t tiles,
                                                              int scale, Taps t, int parity, float* __restrict__ e) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t tile = blockIdx.x;
    if (tile >= tiles) return;
    const BatchImage& b = im[batch_image_of<&BatchImage::dtile_off>(im, n, tile)];
    const int local = (int)(tile - b.dtile_off);
    const int tx = (b.w + kDrJ - 1) / kDrJ;
    const float* hr = parity ? b.scr : b.out;
    degrade_tile(hr, scale * b.h, scale * b.w, scale, t, b.lr, e + b.lr_off, (local / tx) * kDrI, (local % tx) * kDrJ,
                 smem);
}

int64_t degrade_tiles(int h, int w) { return (int64_t)((h + kDrI - 1) / kDrI) * ((w + kDrJ - 1) / kDrJ); }

// Batched: LR error of every image, the current estimate in out (parity 0)
// or scr (parity 1); image b's error at e + lr_off.
__global__ void k_b_degrade_residual(const BatchImage* __restrict__ im, int n, int64_t total, int scale, Taps t,
                                     int parity, float* __restrict__ e) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const BatchImage& b = im[batch_image_of<&BatchImage::lr_off>(im, n, idx)];
        const int r = (int)(idx - b.lr_off);
        const int i = r / b.w, j = r % b.w;
        const float* hr = parity ? b.scr : b.out;
        e[idx] = (float)((double)b.lr[r] - blur_at(hr, scale * b.h, scale * b.w, scale * i, scale * j, t));
    }
}

// Four gradient maps per image, fp32 [n_img, 4, h, w]:
//   dx = I(c+1) - I(c-1), dy likewise along rows,
//   dxx = (2 I(c) - I(c-2)) - I(c+2), dyy likewise; replicate border.
__device__ __forceinline__ void gradient_maps_at(const float* __restrict__ I, int h, int w, int rc,
                                                 float* __restrict__ M) {
    const int r = rc / w, c = rc % w;
    auto at = [&](int rr, int cc) -> double {
        return (double)I[(int64_t)clampi(rr, 0, h - 1) * w + clampi(cc, 0, w - 1)];
    };
    const double x0 = at(r, c);
    const double dx = at(r, c + 1) - at(r, c - 1);
    const double dy = at(r + 1, c) - at(r - 1, c);
    const double dxx = (2.0 * x0 - at(r, c - 2)) - at(r, c + 2);
    const double dyy = (2.0 * x0 - at(r - 2, c)) - at(r + 2, c);
    const int64_t plane = (int64_t)h * w;
    M[rc] = (float)dx;
    M[plane + rc] = (float)dy;
    M[2 * plane + rc] = (float)dxx;
    M[3 * plane + rc] = (float)dyy;
}

__global__ void k_gradient_maps(const float* __restrict__ lr, int n_img, int h, int w,
                                float* __restrict__ maps) {
    const int64_t total = (int64_t)n_img * h * w;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t im = idx / ((int64_t)h * w);
        const int rc = (int)(idx % ((int64_t)h * w));
        gradient_maps_at(lr + im * (int64_t)h * w, h, w, rc, maps + im * 4 * (int64_t)h * w);
    }
}

// Batched: every LR pixel of every image; maps of image b at 4 lr_off.
__global__ void k_b_gradient_maps(const BatchImage* __restrict__ im, int n, int64_t total, float* __restrict__ maps) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const BatchImage& b = im[batch_image_of<&BatchImage::lr_off>(im, n, idx)];
        gradient_maps_at(b.lr, b.h, b.w, (int)(idx - b.lr_off), maps + 4 * b.lr_off);
    }
}

// Patch mean: FP64 sum over the 25 pixels in row-major order, then / 25.
__device__ __forceinline__ double patch_mean(const float* __restrict__ I, int w, int i, int j) {
    double s = 0.0;
    for (int a = 0; a < kPatch; ++a)
        for (int b = 0; b < kPatch; ++b) s = s + (double)I[(int64_t)(i + a) * w + j + b];
    return s / (double)(kPatch * kPatch);
}

// One workgroup per segment of up to 64 consecutive patches of one patch row:
// the first threads form the segment's patch means (patch_mean), the rows
// under the segment are staged in LDS, then the threads write the
// segment's features in memory order (coalesced): the map values (gradient
// mode) or the pixels minus the FP64 mean, rounded to fp32.
template <int MODE>
__device__ __forceinline__ void query_features_seg(const float* __restrict__ lr, const float* __restrict__ maps,
                                                   int h, int w, int i, int j0, float* __restrict__ feat,
                                                   double* __restrict__ mu) {
    constexpr int D = MODE == 0 ? 25 : 100;
    constexpr int NCH = MODE == 0 ? 1 : 4;        // image, or the four gradient maps
    constexpr int SW = kFeatSeg + kPatch - 1;     // columns under a segment of patches
    __shared__ double smu[kFeatSeg];
    __shared__ float stile[NCH * kPatch * SW];    // the 5 rows of each channel under the segment
    const int nj = w - kPatch + 1;
    const int np = nj - j0 < kFeatSeg ? nj - j0 : kFeatSeg;
    const int64_t q0 = (int64_t)i * nj + j0;
    const int t = threadIdx.x;
    if (t < np) {
        const double m = patch_mean(lr, w, i, j0 + t);
        smu[t] = m;
        mu[q0 + t] = m;
    }
    const int64_t plane = (int64_t)h * w;
    const int ncols = np + kPatch - 1;
    // coalesced reads of the rows i .. i + 4 of every channel, columns j0 ..
    for (int e = t; e < NCH * kPatch * SW; e += 256) {
        const int ca = e / SW, c = e - ca * SW;
        const int ch = ca / kPatch, a = ca - ch * kPatch;
        if (c < ncols) stile[e] = (MODE == 0 ? lr : maps + ch * plane)[(int64_t)(i + a) * w + j0 + c];
    }
    __syncthreads();
    if (MODE == 0) {
#pragma unroll 5
        for (int l = t; l < np * D; l += 256) {
            const int p = l / D, e = l - p * D;
            const int a = e / kPatch, b = e - a * kPatch;
            feat[q0 * D + l] = (float)((double)stile[a * SW + p + b] - smu[p]);
        }
    } else {
        // 16-byte stores: D = 100 keeps a group of four inside one patch row
        float4* f4 = reinterpret_cast<float4*>(feat + q0 * D);
#pragma unroll 2
        for (int l4 = t; l4 < np * (D / 4); l4 += 256) {
            const int p = l4 / (D / 4), e0 = 4 * (l4 - p * (D / 4));
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u;
                const int ch = e / 25, r = e - ch * 25, a = r / kPatch, b = r - a * kPatch;
                v[u] = stile[(ch * kPatch + a) * SW + p + b];
            }
            f4[l4] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_query_features(const float* __restrict__ lr, const float* __restrict__ maps,
                                                        int h, int w, float* __restrict__ feat,
                                                        double* __restrict__ mu) {
    const int nseg = (w - kPatch + 1 + kFeatSeg - 1) / kFeatSeg;
    const int i = blockIdx.x / nseg, j0 = (blockIdx.x - i * nseg) * kFeatSeg;
    query_features_seg<MODE>(lr, maps, h, w, i, j0, feat, mu);
}

// Batched: one workgroup per segment of every image (the image from the
// table's segment offsets), the single-image code on the image's arrays.
template <int MODE>
__global__ __launch_bounds__(256) void k_b_query_features(const BatchImage* __restrict__ im, int n,
                                                          const float* __restrict__ maps, float* __restrict__ feat,
                                                          double* __restrict__ mu) {
    constexpr int D = MODE == 0 ? 25 : 100;
    const BatchImage& b = im[batch_image_of<&BatchImage::fblk_off>(im, n, blockIdx.x)];
    const int64_t lb = blockIdx.x - b.fblk_off;
    const int nseg = (b.w - kPatch + 1 + kFeatSeg - 1) / kFeatSeg;
    const int i = (int)(lb / nseg), j0 = (int)(lb - (int64_t)i * nseg) * kFeatSeg;
    query_features_seg<MODE>(b.lr, maps + 4 * b.lr_off, b.h, b.w, i, j0, feat + b.q_off * D, mu + b.q_off);
}

// Training pairs at positions (image, i, j): features, and the HR patch
// (5s x 5s at (s i, s j)) minus the mean of the LR patch, in FP64 rounded to
// fp32. One thread per (pair, element) over D + (5s)^2 elements.
__global__ void k_dict_cut(const float* __restrict__ hr, const float* __restrict__ lr,
                           const float* __restrict__ maps, int H, int W, int scale,
                           const int32_t* __restrict__ pos, int64_t n, int mode,
                           float* __restrict__ feat, float* __restrict__ resid) {
    const int h = (H + scale - 1) / scale, w = (W + scale - 1) / scale;
    const int D = mode == 0 ? 25 : 100;
    const int ps = kPatch * scale, ps2 = ps * ps;
    const int per = D + ps2;
    const int64_t total = n * per;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = idx / per;
        const int e = (int)(idx % per);
        const int im = pos[3 * p], i = pos[3 * p + 1], j = pos[3 * p + 2];
        const float* L = lr + (int64_t)im * h * w;
        if (e < D) {
            float v;
            if (mode == 0) {
                const double m = patch_mean(L, w, i, j);
                v = (float)((double)L[(int64_t)(i + e / kPatch) * w + j + e % kPatch] - m);
            } else {
                const int ch = e / 25, a = (e % 25) / kPatch, b = e % kPatch;
                v = maps[((int64_t)im * 4 + ch) * h * w + (int64_t)(i + a) * w + j + b];
            }
            feat[p * D + e] = v;
        } else {
            const int t = e - D, a = t / ps, b = t % ps;
            const double m = patch_mean(L, w, i, j);
            const float x = hr[(int64_t)im * H * W + (int64_t)(scale * i + a) * W + scale * j + b];
            resid[p * ps2 + t] = (float)((double)x - m);
        }
    }
}

// Split storage of the dictionary features: the high plane holds the upper
// 16 bits of each fp32 value (a bf16 truncation) in rows of hi_stride(D)
// halfwords, the low plane the lower 16 bits in rows of D.
__global__ void k_split_planes(const float* __restrict__ x, int64_t n, int D, uint16_t* __restrict__ hi,
                               uint16_t* __restrict__ lo) {
    const int hs = hi_stride(D);
    const int64_t count = n * D;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < count;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / D;
        const int c = (int)(idx - r * D);
        const uint32_t b = __float_as_uint(x[idx]);
        hi[r * hs + c] = (uint16_t)(b >> 16);
        lo[idx] = (uint16_t)(b & 0xFFFFu);
    }
}


__global__ void k_bicubic(const float* __restrict__ lr, int h, int w, int s, float* __restrict__ out) {
    const int H = s * h, W = s * w;
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x)
        out[idx] = bicubic_at(lr, h, w, s, (int)(idx / W), (int)(idx % W));
}

// The LR image interpolated back to the HR grid (Section 2.1, the paired
// LR images of the training set have the HR images' size): bicubic with
// Keys' weights (a = -0.5) taken from the host table wt[r][tap] for the
// phase r = X mod s, taps floor - 1 .. floor + 2, replicate border; FP64,
// along x first (for each of the four rows), then along y, every sum started
// at 0 and taken in tap order; rounded once to fp32.
struct UpWeights {
    double w[kMaxScale * 2][4];
};
__global__ void k_upsample64(const float* __restrict__ lr, int h, int w, int s, UpWeights uw,
                             float* __restrict__ out) {
    const int H = s * h, W = s * w;
    const int64_t total = (int64_t)H * W;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int Y = (int)(idx / W), X = (int)(idx % W);
        const int i0 = Y / s, j0 = X / s;
        const double* wy = uw.w[Y - i0 * s];
        const double* wx = uw.w[X - j0 * s];
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const float* row = lr + (int64_t)clampi(i0 - 1 + a, 0, h - 1) * w;
            double r = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) r = r + wx[b] * (double)row[clampi(j0 - 1 + b, 0, w - 1)];
            acc = acc + wy[a] * r;
        }
        out[idx] = (float)acc;
    }
}

static inline int grid_for(int64_t total, int block) {
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_degrade(const float* hr, int n_img, int H, int W, int scale, const Taps& t,
                          float* lr, hipStream_t st) {
    const int64_t total = (int64_t)n_img * ((H + scale - 1) / scale) * ((W + scale - 1) / scale);
    hipLaunchKernelGGL(k_degrade, dim3(grid_for(total, 256)), dim3(256), 0, st, hr, n_img, H, W,
                       scale, t, lr);
    return hipGetLastError();
}

hipError_t launch_degrade_residual(const float* hr, int H, int W, int scale, const Taps& t,
                                   const float* lr_ref, float* e, hipStream_t st) {
    const int h = (H + scale - 1) / scale, w = (W + scale - 1) / scale;
    const size_t lds = sizeof(double) * (size_t)(scale * (kDrI - 1) + 2 * t.R + 1) * kDrJ +
                       sizeof(float) * (size_t)(scale * (kDrI - 1) + 2 * t.R + 1) * (scale * (kDrJ - 1) + 2 * t.R + 1);
    if (lds <= 48 * 1024 && h > 0 && w > 0) {
        const dim3 grid((unsigned)((w + kDrJ - 1) / kDrJ), (unsigned)((h + kDrI - 1) / kDrI));
        hipLaunchKernelGGL(k_degrade_residual_t, grid, dim3(256), lds, st, hr, H, W, scale, t, lr_ref, e);
        return hipGetLastError();
    }
    const int64_t total = (int64_t)h * w;
    hipLaunchKernelGGL(k_degrade_residual, dim3(grid_for(total, 256)), dim3(256), 0, st, hr, H, W,
                       scale, t, lr_ref, e);
    return hipGetLastError();
}

hipError_t launch_gradient_maps(const float* lr, int n_img, int h, int w, float* maps,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_gradient_maps, dim3(grid_for((int64_t)n_img * h * w, 256)), dim3(256), 0,
                       st, lr, n_img, h, w, maps);
    return hipGetLastError();
}

hipError_t launch_query_features(const float* lr, const float* maps, int h, int w, int mode,
                                 float* feat, double* mu, hipStream_t st) {
    const int ni = h - kPatch + 1, nj = w - kPatch + 1;
    if (ni < 1 || nj < 1) return hipSuccess;
    const int64_t blocks = feature_segments(h, w);
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    if (mode == 0)
        hipLaunchKernelGGL(k_query_features<0>, grid, dim3(256), 0, st, lr, maps, h, w, feat, mu);
    else
        hipLaunchKernelGGL(k_query_features<1>, grid, dim3(256), 0, st, lr, maps, h, w, feat, mu);
    return hipGetLastError();
}

hipError_t launch_b_gradient_maps(const BatchImage* im, int n, int64_t lr_total, float* maps, hipStream_t st) {
    if (lr_total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_b_gradient_maps, dim3(grid_for(lr_total, 256)), dim3(256), 0, st, im, n, lr_total, maps);
    return hipGetLastError();
}

hipError_t launch_b_query_features(const BatchImage* im, int n, int64_t seg_total, int mode, const float* maps,
                                   float* feat, double* mu, hipStream_t st) {
    if (seg_total == 0) return hipSuccess;
    if (seg_total > 0x7FFFFFFF) return hipErrorInvalidValue;
    if (mode == 0)
        hipLaunchKernelGGL(k_b_query_features<0>, dim3((unsigned)seg_total), dim3(256), 0, st, im, n, maps, feat, mu);
    else
        hipLaunchKernelGGL(k_b_query_features<1>, dim3((unsigned)seg_total), dim3(256), 0, st, im, n, maps, feat, mu);
    return hipGetLastError();
}

hipError_t launch_b_degrade_residual(const BatchImage* im, int n, int64_t lr_total, int64_t tiles, int scale,
                                     const Taps& t, int parity, float* e, hipStream_t st) {
    if (lr_total == 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)(scale * (kDrI - 1) + 2 * t.R + 1) * kDrJ +
                       sizeof(float) * (size_t)(scale * (kDrI - 1) + 2 * t.R + 1) * (scale * (kDrJ - 1) + 2 * t.R + 1);
    if (lds <= 48 * 1024 && tiles > 0 && tiles <= 0x7FFFFFFF) {
        hipLaunchKernelGGL(k_b_degrade_residual_t, dim3((unsigned)tiles), dim3(256), lds, st, im, n, tiles, scale, t,
                           parity, e);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_b_degrade_residual, dim3(grid_for(lr_total, 256)), dim3(256), 0, st, im, n, lr_total, scale,
                       t, parity, e);
    return hipGetLastError();
}

// flag[0] = 1 when any training position (image, i, j) lies outside
// [0, n_img) x [0, imax] x [0, jmax]; flag is cleared by the caller
__global__ __launch_bounds__(256) void k_check_positions(const int32_t* __restrict__ pos, int64_t n, int n_img,
                                                         int imax, int jmax, uint32_t* __restrict__ flag) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int im = pos[3 * r], i = pos[3 * r + 1], j = pos[3 * r + 2];
    if (im < 0 || im >= n_img || i < 0 || i > imax || j < 0 || j > jmax) flag[0] = 1u;
}

hipError_t launch_check_positions(const int32_t* pos, int64_t n, int n_img, int imax, int jmax, uint32_t* flag,
                                  hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_positions, dim3(grid_for(n, 256)), dim3(256), 0, st, pos, n, n_img, imax, jmax, flag);
    return hipGetLastError();
}

hipError_t launch_dict_cut(const float* hr, const float* lr, const float* maps, int H, int W,
                           int scale, const int32_t* pos, int64_t n, int mode, float* feat,
                           float* resid, hipStream_t st) {
    const int per = (mode == 0 ? 25 : 100) + kPatch * scale * kPatch * scale;
    hipLaunchKernelGGL(k_dict_cut, dim3(grid_for(n * per, 256)), dim3(256), 0, st, hr, lr, maps,
                       H, W, scale, pos, n, mode, feat, resid);
    return hipGetLastError();
}

hipError_t launch_split_planes(const float* x, int64_t n, int D, uint16_t* hi, uint16_t* lo,
                               hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_planes, dim3(grid_for(n * D, 256)), dim3(256), 0, st, x, n, D, hi, lo);
    return hipGetLastError();
}


hipError_t launch_upsample64(const float* lr, int h, int w, int scale, const double* wt, float* out, hipStream_t st) {
    if (scale < 1 || scale > 2 * kMaxScale) return hipErrorInvalidValue;
    UpWeights uw{};
    for (int r = 0; r < scale; ++r)
        for (int a = 0; a < 4; ++a) uw.w[r][a] = wt[4 * r + a];
    hipLaunchKernelGGL(k_upsample64, dim3(grid_for((int64_t)scale * h * scale * w, 256)), dim3(256), 0, st, lr, h, w,
                       scale, uw, out);
    return hipGetLastError();
}

hipError_t launch_bicubic(const float* lr, int h, int w, int scale, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_bicubic, dim3(grid_for((int64_t)scale * h * scale * w, 256)), dim3(256),
                       0, st, lr, h, w, scale, out);
    return hipGetLastError();
}

}  // namespace zh
