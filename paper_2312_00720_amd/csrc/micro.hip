// Machine measurements behind the cost model (Section 4.1.1, Table 1): a plain
// stream copy, which bounds what any pass over HBM can reach, and the gather
// T[i] = V[M[i]] of 4-byte values whose map M is either clustered (the rows of
// V it reads are partition-local, as after radix partitioning) or unclustered
// (a random permutation). The ratio of the two gathers gives the penalty of
// random access, B_G / B_R, the way the paper derives it from its profile.
#include "internal.hpp"

namespace gj {
namespace {

// Copy of 16-byte words: every thread moves kU words per round, all loads of a
// round issued before its stores; a tail of fewer than 16 bytes goes byte-wise.
constexpr int kCopyU = 4;

__global__ __launch_bounds__(kBlock) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                        uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * kCopyU;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock * kCopyU + threadIdx.x; base < n16; base += stride) {
        uint4 v[kCopyU];
#pragma unroll
        for (int u = 0; u < kCopyU; ++u) {
            const uint64_t i = base + (uint64_t)u * kBlock;
            if (i < n16) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < kCopyU; ++u) {
            const uint64_t i = base + (uint64_t)u * kBlock;
            if (i < n16) dst[i] = v[u];
        }
    }
}

__global__ void k_copy_tail(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst, uint64_t n) {
    if (threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

// T[i] = V[M[i]]: M and T are streamed, V is read where M points.
constexpr int kGatherU = 8;

__global__ __launch_bounds__(kBlock) void k_gather(const int32_t *__restrict__ map, const int32_t *__restrict__ v,
                                                   uint32_t nv, int32_t *__restrict__ out, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * kGatherU;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock * kGatherU + threadIdx.x; base < n; base += stride) {
        int32_t m[kGatherU];
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            const uint64_t i = base + (uint64_t)u * kBlock;
            m[u] = i < n ? map[i] : 0;
        }
        int32_t x[kGatherU];
#pragma unroll
        for (int u = 0; u < kGatherU; ++u)
            x[u] = (base + (uint64_t)u * kBlock < n && (uint32_t)m[u] < nv) ? v[m[u]] : 0;
#pragma unroll
        for (int u = 0; u < kGatherU; ++u) {
            const uint64_t i = base + (uint64_t)u * kBlock;
            if (i < n) out[i] = x[u];
        }
    }
}

// Enough workgroups for about 8 per compute unit of the 256.
constexpr uint32_t kStreamGrid = 2048;

}  // namespace
}  // namespace gj

extern "C" {

int gj_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    try {
        gj::clear_error();
        gj::require(bytes == 0 || (src && dst), "null buffer");
        gj::require(((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0, "buffers must be 16-byte aligned");
        hipStream_t st = (hipStream_t)stream;
        const uint64_t n16 = bytes / 16, tail = bytes % 16;
        if (n16) {
            const uint32_t grid = (uint32_t)std::min<uint64_t>(gj::kStreamGrid,
                                                               (n16 + gj::kBlock * gj::kCopyU - 1) / (gj::kBlock * gj::kCopyU));
            GJ_LAUNCH("k_stream_copy", 2.0 * 16.0 * n16, gj::k_stream_copy, dim3(grid), dim3(gj::kBlock), 0, st,
                      static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
        }
        if (tail)
            GJ_LAUNCH("k_copy_tail", 2.0 * tail, gj::k_copy_tail, dim3(1), dim3(64), 0, st,
                      static_cast<const uint8_t *>(src) + 16 * n16, static_cast<uint8_t *>(dst) + 16 * n16, tail);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return gj::fail(e.code, e.what());
    } catch (const std::exception &e) {
        return gj::fail(GJ_EHIP, e.what());
    }
}

int gj_gather_i32(const int32_t *map, const int32_t *values, int64_t n_values, int32_t *out, int64_t n,
                  void *stream) {
    try {
        gj::clear_error();
        gj::require(n >= 0 && n_values >= 0, "negative size");
        gj::require(n_values <= 2147483647LL, "more than 2^31-1 values", GJ_EOVERFLOW);
        gj::require(n == 0 || (map && values && out), "null buffer");
        if (n == 0) return GJ_OK;
        const uint32_t grid = (uint32_t)std::min<uint64_t>(
            gj::kStreamGrid, ((uint64_t)n + gj::kBlock * gj::kGatherU - 1) / (gj::kBlock * gj::kGatherU));
        GJ_LAUNCH("k_gather", 12.0 * n, gj::k_gather, dim3(grid), dim3(gj::kBlock), 0, (hipStream_t)stream, map,
                  values, (uint32_t)n_values, out, (uint64_t)n);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return gj::fail(e.code, e.what());
    } catch (const std::exception &e) {
        return gj::fail(GJ_EHIP, e.what());
    }
}

}  // extern "C"
