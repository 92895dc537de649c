// Device helpers shared by the gj kernels (CDNA4 / gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace gj {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup for the partition and join kernels
constexpr int kWaves = kBlock / kWave;
constexpr int kRadix = 256;  // at most 8 bits per partition pass
constexpr int kMaxCols = 10; // 8 payload columns + generated row id + spare

enum DigitMode : int { kDigitBits = 0, kDigitHash = 1, kDigitOrdered = 2 };

// MurmurHash3 32-bit finalizer (Appleby); used to partition on hashed keys.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

struct DigitFn {
    int mode;       // DigitMode
    int shift;      // first bit of the digit
    uint32_t mask;  // (1 << bits) - 1
};

template <typename K>
__device__ __forceinline__ uint64_t digit_source(K key, int mode) {
    if constexpr (sizeof(K) == 4) {
        uint32_t u = (uint32_t)key;
        if (mode == kDigitHash) return fmix32(u);
        if (mode == kDigitOrdered) return u ^ 0x80000000u;
        return u;
    } else {
        uint64_t u = (uint64_t)key;
        if (mode == kDigitHash) return fmix32((uint32_t)u ^ (uint32_t)(u >> 32));
        if (mode == kDigitOrdered) return u ^ 0x8000000000000000ull;
        return u;
    }
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, const DigitFn &f) {
    return (uint32_t)(digit_source(key, f.mode) >> f.shift) & f.mask;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Lanes of the wave whose `bits`-bit value equals this lane's (only lanes with
// valid = true take part). All 64 lanes must execute this call.
__device__ __forceinline__ uint64_t match_peers(uint32_t v, int bits, bool valid) {
    uint64_t m = __ballot(valid);
    for (int k = 0; k < bits; ++k) {
        const bool b = (v >> k) & 1u;
        const uint64_t bk = __ballot(b);
        m &= b ? bk : ~bk;
    }
    return valid ? m : 0ull;
}

// Inclusive prefix sum over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive prefix sum over a workgroup of W waves (kBlock threads by default).
// `s_tmp` holds W values; returns the exclusive prefix and writes the total to *total.
template <typename T, int W = kWaves>
__device__ __forceinline__ T block_exclusive_sum(T v, T *s_tmp, T *total) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    T inc = wave_inclusive_sum(v);
    if (lane == kWave - 1) s_tmp[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        T x = s_tmp[i];
        if (i < w) before += x;
        all += x;
    }
    __syncthreads();
    if (total) *total = all;
    return before + inc - v;
}

// Multiplicative (Fibonacci) hash of a key's bits above the partition digit,
// giving `log2b` bits; keys of one partition share their low digit bits.
template <typename K>
__device__ __forceinline__ uint32_t bucket_of(K key, int skip_bits, int log2b) {
    uint64_t u = (uint64_t)key;
    if constexpr (sizeof(K) == 4) u &= 0xFFFFFFFFull;
    u >>= skip_bits;
    const uint32_t x = (uint32_t)u ^ (uint32_t)(u >> 32);
    return log2b == 0 ? 0u : (uint32_t)(x * 0x9E3779B1u) >> (32 - log2b);
}

__host__ __device__ constexpr uint32_t ceil_div_u32(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// A thread's run of IT consecutive values of T at p (16-byte aligned), moved in
// 16-byte accesses. Where each lane of a wave owns a run, plain element accesses
// would touch one line per lane and instruction; these touch each line once.
template <typename T, int IT>
__device__ __forceinline__ void load_run16(const T *__restrict__ p, T (&out)[IT]) {
    constexpr int PER = 16 / (int)sizeof(T);  // values per 16-byte access
    static_assert(IT % PER == 0, "whole 16-byte accesses");
    const uint4 *__restrict__ q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int l = 0; l < IT / PER; ++l) {
        const uint4 v = q[l];
        const T *t = reinterpret_cast<const T *>(&v);
#pragma unroll
        for (int e = 0; e < PER; ++e) out[l * PER + e] = t[e];
    }
}
template <typename T, int IT>
__device__ __forceinline__ void store_run16(T *__restrict__ p, const T (&in)[IT]) {
    constexpr int PER = 16 / (int)sizeof(T);
    static_assert(IT % PER == 0, "whole 16-byte accesses");
    uint4 *__restrict__ q = reinterpret_cast<uint4 *>(p);
#pragma unroll
    for (int l = 0; l < IT / PER; ++l) {
        uint4 v;
        T *t = reinterpret_cast<T *>(&v);
#pragma unroll
        for (int e = 0; e < PER; ++e) t[e] = in[l * PER + e];
        q[l] = v;
    }
}

}  // namespace gj
