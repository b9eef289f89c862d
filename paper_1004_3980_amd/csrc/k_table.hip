// Hash-table build (Section 3.2 and Section 4.1: the IDs of the training
// patches are stored in the bins of L tables, a bin being one k-tuple of
// codes, identified here by its 64-bit key).
//
// Per table: every key is inserted into an open-addressing directory with
// linear probing (64-bit compare-and-swap), which gives each ID the slot of
// its bin and counts the bin. A stable LSD radix sort of (slot, ID) pairs,
// taken in ID order, lays the IDs out bin by bin with IDs ascending inside
// each bin; the first position of each slot in the sorted order is its bin's
// offset. Slot placement depends on insertion order, the bins' contents and
// their order do not.
#include "zh_internal.h"

namespace zh {

static inline int grid_for(int64_t total, int block) {
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

__global__ void k_dir_clear(Slot* __restrict__ dir, uint64_t count) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        Slot s;
        s.key = kEmptyKey;
        s.count = 0;
        s.offset = 0;
        dir[i] = s;
    }
}

__global__ void k_dir_insert(const uint64_t* __restrict__ keys, int64_t n, int L, int l,
                             Slot* __restrict__ dir, uint64_t cap, uint32_t* __restrict__ filter,
                             uint32_t* __restrict__ slot_of, uint32_t* __restrict__ ids) {
    const uint64_t mask = cap - 1;
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < n;
         id += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long key = keys[id * L + l];
        uint64_t s = key & mask;
        // the directory holds at most n distinct keys in cap >= 2n slots, so
        // the probe ends within cap steps
        for (uint64_t step = 0; step < cap; ++step) {
            const unsigned long long old = atomicCAS(&dir[s].key, (unsigned long long)kEmptyKey, key);
            if (old == kEmptyKey || old == key) {
                if (old == kEmptyKey) {
                    const uint32_t fb = dir_filter_bit(key, cap);
                    atomicOr(&filter[fb >> 5], 1u << (fb & 31));
                }
                atomicAdd(&dir[s].count, 1u);
                slot_of[id] = (uint32_t)s;
                ids[id] = (uint32_t)id;
                break;
            }
            s = (s + 1) & mask;
        }
    }
}

__global__ void k_dir_offsets(const uint32_t* __restrict__ sorted_slot, int64_t n, Slot* __restrict__ dir) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = sorted_slot[i];
        if (i == 0 || sorted_slot[i - 1] != s) dir[s].offset = (uint32_t)i;
    }
}

hipError_t launch_dir_clear(Slot* dir, uint64_t count, hipStream_t st) {
    hipLaunchKernelGGL(k_dir_clear, dim3(grid_for((int64_t)count, 256)), dim3(256), 0, st, dir, count);
    return hipGetLastError();
}

hipError_t launch_dir_insert(const uint64_t* keys, int64_t n, int L, int l, Slot* dir, uint64_t cap,
                             uint32_t* filter, uint32_t* slot_of, uint32_t* ids, hipStream_t st) {
    hipLaunchKernelGGL(k_dir_insert, dim3(grid_for(n, 256)), dim3(256), 0, st, keys, n, L, l, dir,
                       cap, filter, slot_of, ids);
    return hipGetLastError();
}

hipError_t launch_dir_offsets(const uint32_t* sorted_slot, int64_t n, Slot* dir, hipStream_t st) {
    hipLaunchKernelGGL(k_dir_offsets, dim3(grid_for(n, 256)), dim3(256), 0, st, sorted_slot, n, dir);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits. A tile is 4096 consecutive elements;
// each of the 4 waves of a tile owns 1024 consecutive elements, walked in 16
// chunks of 64 in order, so ranks follow the input order (stability).
// ---------------------------------------------------------------------------
constexpr int kRsTile = 4096;
constexpr int kRsChunks = 16;

int64_t radix_hist_size(int64_t n) { return 256 * ((n + kRsTile - 1) / kRsTile); }

// lanes of the wave holding the same 8-bit digit (valid lanes only)
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

__global__ __launch_bounds__(256) void k_rs_hist(const uint32_t* __restrict__ key, int64_t n, int shift,
                                                 uint32_t* __restrict__ hist, int ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int t = threadIdx.x; t < kRsTile; t += 256) {
        const int64_t i = base + t;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of `count` values in place by one workgroup of 1024 threads:
// chunks of 4096 values, four consecutive values per thread, wave scans of
// the thread sums and a scan of the 16 wave sums, a running carry between
// chunks
__global__ __launch_bounds__(1024) void k_scan_1wg(uint32_t* __restrict__ v, int64_t count) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t wtot;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t carry = 0;
    for (int64_t base = 0; base < count; base += 4096) {
        const int64_t i0 = base + 4 * (int64_t)t;
        uint32_t x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = i0 + j < count ? v[i0 + j] : 0u;
        const uint32_t loc = x[0] + x[1] + x[2] + x[3];
        const uint32_t incl = (uint32_t)wave_incl_scan((int)loc);
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        if (wv == 0) {
            const uint32_t ws = lane < 16 ? wsum[lane] : 0u;
            const uint32_t wi = (uint32_t)wave_incl_scan((int)ws);
            if (lane < 16) wsum[lane] = wi - ws;
            if (lane == 15) wtot = wi;
        }
        __syncthreads();
        uint32_t run = carry + wsum[wv] + incl - loc;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < count) v[i0 + j] = run;
            run += x[j];
        }
        carry += wtot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin, int64_t n,
                                                    int shift, const uint32_t* __restrict__ hist,
                                                    int ntiles, uint32_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout) {
    __shared__ uint32_t cnt[4][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < 4 * 256; t += 256) (&cnt[0][0])[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)wave * (kRsChunks * 64);
    // pass 1: per-wave digit counts
    for (int c = 0; c < kRsChunks; ++c) {
        const int64_t i = base + c * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = valid ? (kin[i] >> shift) & 255u : 0u;
        const uint64_t peers = match_digit(d, valid);
        if (valid && (peers & lanemask_lt()) == 0) cnt[wave][d] += (uint32_t)__popcll(peers);
        __syncthreads();
    }
    // running start of each wave's run of every digit
    {
        const int d = threadIdx.x;
        uint32_t run = hist[(int64_t)d * ntiles + blockIdx.x];
        for (int w = 0; w < 4; ++w) {
            const uint32_t c = cnt[w][d];
            cnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
    // pass 2: stable scatter
    for (int c = 0; c < kRsChunks; ++c) {
        const int64_t i = base + c * 64 + lane;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u;
        const uint32_t d = (k >> shift) & 255u;
        const uint64_t peers = match_digit(d, valid);
        if (valid) {
            const uint32_t pos = cnt[wave][d] + (uint32_t)__popcll(peers & lanemask_lt());
            kout[pos] = k;
            vout[pos] = vin[i];
        }
        __syncthreads();
        if (valid && (peers & lanemask_lt()) == 0) cnt[wave][d] += (uint32_t)__popcll(peers);
        __syncthreads();
    }
}

hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int bits,
                            uint32_t* hist, int64_t hist_cap, hipStream_t st, bool* result_in_first) {
    const int ntiles = (int)((n + kRsTile - 1) / kRsTile);
    if ((int64_t)ntiles * 256 > hist_cap) return hipErrorInvalidValue;
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
    bool first = true;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(256), 0, st, ka, n, shift, hist, ntiles);
        hipLaunchKernelGGL(k_scan_1wg, dim3(1), dim3(1024), 0, st, hist, (int64_t)ntiles * 256);
        hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(256), 0, st, ka, va, n, shift, hist, ntiles,
                           kb, vb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint32_t* t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
        first = !first;
    }
    *result_in_first = first;
    return hipSuccess;
}

// Content hash of n 32-bit words for the table files: the sum over i of
// fmix64((i G + salt) ^ w_i) mod 2^64, G the SplitMix64 increment. Integer sums do not depend on their
// order, so the value is the same for every launch shape; it changes with any
// word and with its position.
__global__ __launch_bounds__(256) void k_hash_words(const uint32_t* __restrict__ p, int64_t n, uint64_t salt,
                                                    unsigned long long* __restrict__ out) {
    uint64_t acc = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += fmix64(((uint64_t)i * kGolden + salt) ^ (uint64_t)p[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)acc);
}

hipError_t launch_hash_words(const void* p, int64_t n_words, uint64_t salt, unsigned long long* out,
                             hipStream_t st) {
    if (n_words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hash_words, dim3(grid_for(n_words, 256)), dim3(256), 0, st,
                       static_cast<const uint32_t*>(p), n_words, salt, out);
    return hipGetLastError();
}

}  // namespace zh
