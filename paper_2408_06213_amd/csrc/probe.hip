// Diagnostics for the roofline: the rate at which the device runs the
// Theorem 1 chain step (two 32x32+64 -> 64-bit multiply-adds per die),
// the vector-ALU ceiling of a dice stream whose words are free; and the rate
// of a bare copy that reads and writes as many bytes as a dice stream, its
// memory ceiling.
#include <hip/hip_runtime.h>

#include "brr.h"
#include "internal.hpp"

using namespace brr;

namespace {

constexpr int kChains = 8; // independent chains per thread

__global__ __launch_bounds__(256) void k_chain_rate(uint64_t *out, uint32_t iters, uint32_t b0)
{
    uint64_t r[kChains];
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        r[c] = ((uint64_t)(blockIdx.x * 256u + threadIdx.x) << 32) ^ (0x9E3779B97F4A7C15ull * (c + 1));
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc += mul_roll(b0 + (uint32_t)c, r[c]);
    }
    uint64_t x = acc;
#pragma unroll
    for (int c = 0; c < kChains; ++c) x ^= r[c];
    out[blockIdx.x * 256u + threadIdx.x] = x; // keeps the chains live
}

constexpr uint32_t kCopyThreads = 256;
constexpr uint32_t kCopyVec = 1; // 16-byte vectors per thread

// Each block copies one contiguous tile of kCopyThreads * kCopyVec 16-byte
// vectors, lane-consecutive so every load/store instruction covers one span;
// nontemporal both ways. Of the shapes measured on MI355X over 1 GiB (4-,
// 8- and 16-byte elements, 1 to 8 per lane, nontemporal or not: 3.8 to
// 6.5 TB/s read + written), one 16-byte vector per lane was the fastest.
__global__ __launch_bounds__(kCopyThreads) void k_copy_rate(const u32x4 *src, u32x4 *dst,
                                                            uint64_t nvec)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kCopyThreads * kCopyVec) + threadIdx.x;
    u32x4 v[kCopyVec];
#pragma unroll
    for (uint32_t u = 0; u < kCopyVec; ++u) {
        const uint64_t i = base + (uint64_t)u * kCopyThreads;
        if (i < nvec) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (uint32_t u = 0; u < kCopyVec; ++u) {
        const uint64_t i = base + (uint64_t)u * kCopyThreads;
        if (i < nvec) __builtin_nontemporal_store(v[u], dst + i);
    }
}

} // namespace

extern "C" {

brr_status brr_probe_copy_rate(const void *src, void *dst, uint64_t bytes, uint32_t reps,
                               void *stream_, double *bytes_per_s)
{
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (!src || !dst || !bytes_per_s || reps == 0 || bytes == 0 || bytes % 16 != 0 ||
        reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return BRR_EINVAL;
    const uint64_t nvec = bytes / 16, tile = kCopyThreads * kCopyVec;
    const uint64_t blocks = (nvec + tile - 1) / tile;
    if (blocks > 0x7FFFFFFFull) return BRR_EINVAL;
    brr_status st = ensure_device();
    if (st != BRR_OK) return st;
    const u32x4 *s4 = static_cast<const u32x4 *>(src);
    u32x4 *d4 = static_cast<u32x4 *>(dst);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0;
    if (e == hipSuccess) {
        k_copy_rate<<<(uint32_t)blocks, kCopyThreads, 0, stream>>>(s4, d4, nvec); // warm-up
        e = hipEventRecord(e0, stream);
    }
    for (uint32_t r = 0; e == hipSuccess && r < reps; ++r) {
        k_copy_rate<<<(uint32_t)blocks, kCopyThreads, 0, stream>>>(s4, d4, nvec);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess || ms <= 0) return BRR_EHIP;
    *bytes_per_s = 2.0 * (double)bytes * reps / (ms * 1e-3);
    return BRR_OK;
}

brr_status brr_probe_chain_rate(uint32_t iters, double *dice_per_s)
{
    if (!dice_per_s || iters == 0) return BRR_EINVAL;
    brr_status st = ensure_device();
    if (st != BRR_OK) return st;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return BRR_EHIP;
    const uint32_t blocks = (uint32_t)cus * 16u; // 16 wavefronts of work per CU
    uint64_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&out), (size_t)blocks * 256 * 8) != hipSuccess)
        return BRR_ENOMEM;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0;
    if (e == hipSuccess) {
        k_chain_rate<<<blocks, 256>>>(out, iters, 65521u); // warm-up
        e = hipEventRecord(e0, nullptr);
    }
    if (e == hipSuccess) {
        k_chain_rate<<<blocks, 256>>>(out, iters, 65521u);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (e != hipSuccess || ms <= 0) return BRR_EHIP;
    *dice_per_s = (double)blocks * 256.0 * kChains * iters / (ms * 1e-3);
    return BRR_OK;
}

} // extern "C"
