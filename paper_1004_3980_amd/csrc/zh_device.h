// Device-side helpers shared by the libzoomhash kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ZH_WAVE 64

namespace zh {

// SplitMix64 output function (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t fmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kEmptyKey = ~0ull;

// Multiplier of code j of table l in the bucket key (j = 63: the start value
// of the sum): SplitMix64 output number 64 l + j + 1 from state 0.
__host__ __device__ inline uint64_t key_mul(int l, int j) {
    return fmix64(kGolden * (uint64_t)(64 * l + j + 1));
}
// One term of the key sum: uint32(c) times the 64-bit multiplier, mod 2^64.
__host__ __device__ inline uint64_t key_term(int32_t c, uint64_t mul) {
    return (uint64_t)(uint32_t)c * mul;
}
// Bucket key from the wrapped sum of the terms; the empty-slot marker is
// never a key.
__host__ __device__ inline uint64_t key_final(uint64_t sum) {
    const uint64_t h = fmix64(sum);
    return h == kEmptyKey ? kEmptyKey - 1 : h;
}

// Bucket directory entry of one hash table (open addressing, linear probing).
struct Slot {
    unsigned long long key;  // kEmptyKey when free
    uint32_t count;          // number of IDs in the bin
    uint32_t offset;         // first ID of the bin inside the table's ID array
};

// fp32 value from its split storage: bf16 high half (round toward zero) and
// the low 16 bits.
__device__ inline float join_planes(uint16_t hi, uint16_t lo) {
    return __uint_as_float(((uint32_t)hi << 16) | (uint32_t)lo);
}
__device__ inline float hi_plane(uint16_t hi) { return __uint_as_float((uint32_t)hi << 16); }

// Wave reductions (64 lanes).
__device__ inline unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return v;
}
__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return v;
}
__device__ inline int wave_sum_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double wave_max_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_max_f32(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_sum_f32(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// inclusive prefix sum over the 64 lanes
__device__ inline int wave_incl_scan(int v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}
__device__ inline uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// bf16 of an fp32 value, round to nearest even; and back (exact)
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Block index for XCD-aware launches. Workgroups are handed to the eight
// XCDs in turn (block b runs on XCD b % 8) and every XCD has its own L2.
// Renumbering so that XCD x owns the x-th contiguous eighth of the blocks puts
// blocks that run at the same time on one XCD on neighbouring work items
// (neighbouring patches share most of their dictionary candidates). Grids
// whose size is not a multiple of 8 keep the plain numbering.
__device__ inline int xcd_block() {
    const int G = gridDim.x;
    if (G & 7) return blockIdx.x;
    return (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
}
__host__ __device__ inline int round_grid8(int g) { return g >= 8 ? (g + 7) & ~7 : g; }

// Higham's gamma_n = n u / (1 - n u) for unit roundoff u.
__host__ __device__ inline double gamma_n(int n, double u) { return n * u / (1.0 - n * u); }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Keys' cubic kernel, a = -0.5.
__device__ __forceinline__ float keys_w(float x) {
    x = fabsf(x);
    if (x <= 1.0f) return (1.5f * x - 2.5f) * x * x + 1.0f;
    if (x < 2.0f) return ((-0.5f * x + 2.5f) * x - 4.0f) * x + 2.0f;
    return 0.0f;
}

// Bicubic value at HR pixel (Y, X): LR coordinate (Y/s, X/s), taps at
// floor-1 .. floor+2 with replicate border; along x first, then y.
__device__ __forceinline__ float bicubic_at(const float* __restrict__ lr, int h, int w, int s, int Y,
                                            int X) {
    const int i0 = Y / s, j0 = X / s;
    const float ty = (float)(Y - i0 * s) / (float)s, tx = (float)(X - j0 * s) / (float)s;
    float wy[4], wx[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        wy[a] = keys_w(ty - (float)(a - 1));
        wx[a] = keys_w(tx - (float)(a - 1));
    }
    float acc = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const float* row = lr + (int64_t)clampi(i0 - 1 + a, 0, h - 1) * w;
        float r = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b) r = fmaf(wx[b], row[clampi(j0 - 1 + b, 0, w - 1)], r);
        acc = fmaf(wy[a], r, acc);
    }
    return acc;
}

}  // namespace zh
