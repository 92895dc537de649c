// The radix-partition primitive (Section 2.3) without any device allocation.
//
// gj_partition takes the scratch of a pass (the chunk table, the per-chunk
// digit histograms and the partial sums of their scan) from the caller's
// allocator. gj_partition_noalloc runs the same kernels over one statically
// allocated device array instead, for callers that cannot allocate device
// memory: code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc. It is restricted to one pass (at most 8 digit bits),
// whose scratch does not grow with the row count: at most 4097 chunks x 256
// digits of 4-byte counts plus a few small tables, about 4.2 MB.
//
// The array is a file-scope __device__ symbol. In host code its name stands
// for a host-side shadow, not a device address, so the library looks up the
// device address once per device (hipGetSymbolAddress, with that device
// current) and passes only that address to kernels. Every call on a device
// shares the device's array: calls that overlap on one device race and give
// wrong results. Every scratch word a call reads is first written by a kernel
// of the same call (fills are kernels, no memset), so the previous call's
// contents never leak into a result.
#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device

// Device address of the current device's array (looked up on first use).
char *device_scratch() {
    int dev = -1;
    GJ_HIP(hipGetDevice(&dev));
    gj::require(dev >= 0 && dev < kMaxDevices, "device ordinal out of range", GJ_EHIP);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        GJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        gj::require(p != nullptr, "no device address for the scratch array", GJ_EHIP);
        g_scratch_dev[dev] = p;
    }
    return static_cast<char *>(g_scratch_dev[dev]);
}

int dtype_bytes(int32_t dt) { return dt == GJ_I32 ? 4 : (dt == GJ_I64 ? 8 : 0); }

// Keeps launches off for a scope (scratch measurement).
struct NoLaunch {
    NoLaunch() {
        gj::g_dry_run = true;
        gj::g_dry_launches = 0;
    }
    ~NoLaunch() { gj::g_dry_run = false; }
};

}  // namespace

extern "C" {

size_t gj_partition_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int gj_partition_noalloc(gj_col key, const gj_col *cols, int32_t n_cols, int64_t n_rows, int32_t bit_lo,
                         int32_t bits, int32_t mode, void *out_key, void *const *out_cols, void *out_rowid,
                         int32_t *out_offsets, void *stream) {
    try {
        gj::clear_error();
        gj::require(n_rows >= 0, "negative row count");
        gj::require(n_rows <= 2147483647LL, "more than 2^31-1 rows", GJ_EOVERFLOW);
        gj::require(n_cols >= 0 && n_cols <= 8, "0..8 columns");
        gj::require(n_cols == 0 || (cols && out_cols), "null column arrays");
        gj::require(bits >= 1 && bits <= 8, "bits must be 1..8 (one pass) without allocation");
        gj::require(mode >= 0 && mode <= 2, "bad digit mode");
        const int kb = dtype_bytes(key.dtype);
        gj::require(kb != 0, "key dtype must be GJ_I32 or GJ_I64");
        gj::require(n_rows == 0 || key.data != nullptr, "null key data");
        gj::require(bit_lo >= 0 && bit_lo + bits <= 8 * kb, "digit bits outside the key");
        gj::require(n_rows == 0 || out_key, "null output key");
        gj::require(out_offsets != nullptr, "null output offsets (2^bits + 1 int32, device)");
        gj::PartCols pc;
        pc.n = n_cols;
        for (int i = 0; i < n_cols; ++i) {
            gj::require(dtype_bytes(cols[i].dtype) != 0, "column dtype must be GJ_I32 or GJ_I64");
            gj::require(n_rows == 0 || cols[i].data != nullptr, "null column data");
            gj::require(n_rows == 0 || out_cols[i], "null output column");
            pc.in[i] = cols[i].data;
            pc.out[i] = out_cols[i];
            pc.width[i] = dtype_bytes(cols[i].dtype);
        }
        pc.gen_rowid = out_rowid != nullptr;
        pc.rowid_out = out_rowid;
        uint32_t *poff = reinterpret_cast<uint32_t *>(out_offsets);
        const uint32_t n = (uint32_t)n_rows;
        hipStream_t st = (hipStream_t)stream;

        // The scratch of this call, measured with launches off.
        gj::Arena measure;
        {
            NoLaunch off;
            gj::Ctx ctx(&measure, st);
            gj::partition_run(ctx, kb, key.data, out_key, pc, n, bit_lo, bits, 1, mode, poff);
        }
        if (measure.peak > kNoAllocScratchBytes)
            return gj::fail(GJ_ECAPACITY, "needs " + std::to_string(measure.peak) +
                                              " bytes of scratch; the static array holds " +
                                              std::to_string(kNoAllocScratchBytes));

        gj::Arena arena;
        arena.base = device_scratch();
        arena.size = kNoAllocScratchBytes;
        gj::Ctx ctx(&arena, st);
        gj::partition_run(ctx, kb, key.data, out_key, pc, n, bit_lo, bits, 1, mode, poff);
        return GJ_OK;
    } catch (const gj::Error &e) {
        return gj::fail(e.code, e.what());
    } catch (const std::exception &e) {
        return gj::fail(GJ_EHIP, e.what());
    }
}

}  // extern "C"
