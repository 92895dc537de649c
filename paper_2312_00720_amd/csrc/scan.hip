// Device-wide exclusive prefix sums (reduce, scan of block totals, downsweep)
// and fill kernels. The scans give the stable scatter offsets and partition
// boundaries of the radix partition (Section 4.1.4: a histogram plus a prefix
// sum locate every partition) and the output offsets of the join and group-by.
// Deterministic: no atomics decide any order.
#include "internal.hpp"

namespace gj {
namespace {

constexpr int kItems = 16;
constexpr uint32_t kTile = kBlock * kItems;

// Element count: nmax, or min(nmax, *n_dev * mult) when the count lives in device
// memory (launches sized for nmax; blocks past the count do nothing).
__device__ __forceinline__ uint64_t scan_len(uint64_t nmax, const uint32_t *n_dev, uint32_t mult) {
    return n_dev ? min(nmax, (uint64_t)(*n_dev) * mult) : nmax;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T *__restrict__ in, uint64_t nmax,
                                                        const uint32_t *n_dev, uint32_t mult,
                                                        T *__restrict__ partial) {
    __shared__ T s_tmp[kWaves];
    const uint64_t n = scan_len(nmax, n_dev, mult);
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    T acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t i = base + (uint64_t)k * kBlock + threadIdx.x;
        if (i < n) acc += in[i];
    }
    T total;
    block_exclusive_sum<T>(acc, s_tmp, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// One workgroup scans the block totals in place, carrying across tiles.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_partials(T *__restrict__ partial, uint64_t nmax,
                                                          const uint32_t *n_dev, uint32_t mult,
                                                          T *__restrict__ total_out) {
    __shared__ T s_tmp[kWaves];
    const uint64_t n = (scan_len(nmax * kTile, n_dev, mult) + kTile - 1) / kTile;  // block totals in use
    T carry = 0;
    for (uint64_t base = 0; base < n; base += kTile) {
        T v[kItems];
        T sum = 0;
        const uint64_t first = base + (uint64_t)threadIdx.x * kItems;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t i = first + k;
            v[k] = i < n ? partial[i] : T(0);
            sum += v[k];
        }
        T tile_total;
        T run = carry + block_exclusive_sum<T>(sum, s_tmp, &tile_total);
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t i = first + k;
            if (i < n) partial[i] = run;
            run += v[k];
        }
        carry += tile_total;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_down(const T *in, T *out, uint64_t nmax,
                                                      const uint32_t *n_dev, uint32_t mult,
                                                      const T *__restrict__ partial) {
    __shared__ T s_tmp[kWaves];
    const uint64_t n = scan_len(nmax, n_dev, mult);
    if ((uint64_t)blockIdx.x * kTile >= n) return;
    const uint64_t first = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
    // a whole run of this thread's items at 16-byte aligned addresses moves in
    // 16-byte accesses
    const bool vec = first + kItems <= n && (((uintptr_t)in | (uintptr_t)out) & 15u) == 0;
    T v[kItems];
    T sum = 0;
    if (vec) {
        load_run16<T>(in + first, v);
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t i = first + k;
            v[k] = i < n ? in[i] : T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) sum += v[k];
    T run = partial[blockIdx.x] + block_exclusive_sum<T>(sum, s_tmp, (T *)nullptr);
    if (vec) {
        T o[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            o[k] = run;
            run += v[k];
        }
        store_run16<T>(out + first, o);
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint64_t i = first + k;
            if (i < n) out[i] = run;
            run += v[k];
        }
    }
}

template <typename T>
__global__ void k_fill(T *p, T v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
void scan_exclusive(Ctx &ctx, const T *in, T *out, uint64_t n, T *total, const uint32_t *n_dev = nullptr,
                    uint32_t mult = 1) {
    hipStream_t s = ctx.stream;
    if (n == 0) {
        if (total) {
            GJ_LAUNCH("k_fill", sizeof(T), k_fill<T>, dim3(1), dim3(64), 0, s, total, T(0), (uint64_t)1);
        }
        return;
    }
    const uint64_t blocks = (n + kTile - 1) / kTile;
    T *partial = ctx.scratch_n<T>(blocks);
    const double nb = (double)n * sizeof(T);
    GJ_LAUNCH("k_scan_reduce", nb, k_scan_reduce<T>, dim3((uint32_t)blocks), dim3(kBlock), 0, s, in, n, n_dev,
              mult, partial);
    GJ_LAUNCH("k_scan_partials", 2.0 * blocks * sizeof(T), k_scan_partials<T>, dim3(1), dim3(kBlock), 0, s,
              partial, blocks, n_dev, mult, total);
    GJ_LAUNCH("k_scan_down", 2.0 * nb, k_scan_down<T>, dim3((uint32_t)blocks), dim3(kBlock), 0, s, in, out,
              n, n_dev, mult, (const T *)partial);
}

template <typename T>
void fill(hipStream_t s, T *p, T v, uint64_t n) {
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    GJ_LAUNCH("k_fill", (double)n * sizeof(T), k_fill<T>, dim3((uint32_t)blocks), dim3(256), 0, s, p, v, n);
}

}  // namespace

void scan_exclusive_u32(Ctx &ctx, const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total) {
    scan_exclusive<uint32_t>(ctx, in, out, n, total);
}
void scan_exclusive_u64(Ctx &ctx, const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *total) {
    scan_exclusive<uint64_t>(ctx, in, out, n, total);
}
void scan_exclusive_u64_dev(Ctx &ctx, const uint64_t *in, uint64_t *out, uint64_t nmax, const uint32_t *n_dev,
                            uint32_t mult, uint64_t *total) {
    scan_exclusive<uint64_t>(ctx, in, out, nmax, total, n_dev, mult);
}
void fill_u32(hipStream_t s, uint32_t *p, uint32_t v, uint64_t n) { fill<uint32_t>(s, p, v, n); }
void fill_u64(hipStream_t s, uint64_t *p, uint64_t v, uint64_t n) { fill<uint64_t>(s, p, v, n); }

}  // namespace gj
