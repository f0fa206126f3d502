// Dice streams: groups of K bounds rolled from one 64-bit word each by the
// Theorem 1 chain (Sec. 4), accepted by Algorithm 3 (Sec. 5): the exact
// bound product P is formed, and only when the leftover r is below P is the
// threshold 2^64 mod P computed and the group rerolled while r stays below
// it. The constant-bound form uses Algorithm 2 with t precomputed.
//
// Work mapping: one lane owns a "quad" of 4 consecutive groups = 4K rolls,
// read and written as K 16-byte vectors, and draws its 4 words from two
// Philox blocks (block = 2 words, and group g's first word is word g). The
// at most 4 groups past the last full quad (including a short last group)
// go to the lanes after the last quad, one group each.
#include "device.hpp"
#include "internal.hpp"

namespace brr {

namespace {

constexpr uint64_t kMaxAttempts = 1024;

template <int K>
__device__ __forceinline__ void check_group(const uint32_t *b, int kk, uint64_t r, bool &need,
                                            uint64_t &t, uint32_t &err)
{
    BoundProduct P;
    P.init(b[0]);
#pragma unroll
    for (int i = 1; i < K; ++i)
        if (i < kk) P.mul(b[i]);
    need = false;
    t = 0;
    if (P.zero) {
        err |= kDevZeroBound;
    } else if (P.over) {
        err |= kDevOverflow;
    } else if (!P.e64 && r < P.p) {
        t = group_threshold(P);
        need = (r < t);
    }
}

// Rolls group `g` again from attempt 1 on until accepted.
template <int K>
__device__ __forceinline__ void reroll_group(const uint32_t *b, int kk, uint32_t *a, uint64_t t,
                                          uint64_t S, uint64_t g, StreamKey key)
{
    // each attempt is rejected with probability t / 2^64 < 1/2; the cap only
    // bounds the loop against corrupted inputs
    uint64_t r;
    uint64_t attempt = 1;
    do {
        r = word_at(attempt * S + g, key);
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < kk) a[i] = mul_roll(b[i], r);
        ++attempt;
    } while (r < t && attempt <= kMaxAttempts);
}

template <int K, bool VEC>
__global__ __launch_bounds__(256) void dice_kernel(const uint32_t *__restrict__ bounds,
                                                   uint32_t *__restrict__ out, uint64_t count,
                                                   uint64_t S, uint64_t nquads, StreamKey key,
                                                   uint32_t *status)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t err = 0;
    if (tid < nquads) {
        uint32_t b[4 * K], a[4 * K];
        const uint64_t base = tid * 4 * K;
        if (VEC) {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(bounds + base);
#pragma unroll
            for (int v = 0; v < K; ++v) {
                const u32x4 x = __builtin_nontemporal_load(src + v);
                b[4 * v + 0] = x.x;
                b[4 * v + 1] = x.y;
                b[4 * v + 2] = x.z;
                b[4 * v + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4 * K; ++i) b[i] = bounds[base + i];
        }
        uint64_t r[4];
        word_pair(2 * tid, key, r[0], r[1]);
        word_pair(2 * tid + 1, key, r[2], r[3]);
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int i = 0; i < K; ++i) a[g * K + i] = mul_roll(b[g * K + i], r[g]);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            bool need;
            uint64_t t;
            check_group<K>(b + g * K, K, r[g], need, t, err);
            if (need) reroll_group<K>(b + g * K, K, a + g * K, t, S, 4 * tid + g, key);
        }
        if (VEC) {
            u32x4 *dst = reinterpret_cast<u32x4 *>(out + base);
#pragma unroll
            for (int v = 0; v < K; ++v) {
                const u32x4 o = {a[4 * v + 0], a[4 * v + 1], a[4 * v + 2], a[4 * v + 3]};
                __builtin_nontemporal_store(o, dst + v);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4 * K; ++i) out[base + i] = a[i];
        }
    } else {
        const uint64_t g = 4 * nquads + (tid - nquads);
        if (g < S) {
            const uint64_t first = g * K;
            const int kk = (int)((count - first < (uint64_t)K) ? count - first : K);
            uint32_t b[K], a[K];
#pragma unroll
            for (int i = 0; i < K; ++i) b[i] = (i < kk) ? bounds[first + i] : 1u;
            uint64_t r = word_at(g, key);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) a[i] = mul_roll(b[i], r);
            bool need;
            uint64_t t;
            check_group<K>(b, kk, r, need, t, err);
            if (need) reroll_group<K>(b, kk, a, t, S, g, key);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) out[first + i] = a[i];
        }
    }
    if (err) atomicOr(status, err);
}

// Constant bound (Algorithm 2): t_full is 2^64 mod bound^K, t_last the same
// for the short last group of k_last dice.
template <int K, bool VEC>
__global__ __launch_bounds__(256) void dice_const_kernel(uint32_t bound, uint32_t *__restrict__ out,
                                                         uint64_t count, uint64_t S,
                                                         uint64_t nquads, StreamKey key,
                                                         uint64_t t_full, uint64_t t_last)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < nquads) {
        uint32_t a[4 * K];
        uint64_t r[4];
        word_pair(2 * tid, key, r[0], r[1]);
        word_pair(2 * tid + 1, key, r[2], r[3]);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            uint64_t rr = r[g];
#pragma unroll
            for (int i = 0; i < K; ++i) a[g * K + i] = mul_roll(bound, rr);
            const uint64_t G = 4 * tid + g;
            const uint64_t t = (G + 1 == S) ? t_last : t_full;
            for (uint64_t attempt = 1; rr < t && attempt <= kMaxAttempts; ++attempt) {
                rr = word_at(attempt * S + G, key);
#pragma unroll
                for (int i = 0; i < K; ++i) a[g * K + i] = mul_roll(bound, rr);
            }
        }
        const uint64_t base = tid * 4 * K;
        if (VEC) {
            u32x4 *dst = reinterpret_cast<u32x4 *>(out + base);
#pragma unroll
            for (int v = 0; v < K; ++v) {
                const u32x4 o = {a[4 * v + 0], a[4 * v + 1], a[4 * v + 2], a[4 * v + 3]};
                __builtin_nontemporal_store(o, dst + v);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4 * K; ++i) out[base + i] = a[i];
        }
    } else {
        const uint64_t g = 4 * nquads + (tid - nquads);
        if (g < S) {
            const uint64_t first = g * K;
            const int kk = (int)((count - first < (uint64_t)K) ? count - first : K);
            const uint64_t t = (g + 1 == S) ? t_last : t_full;
            uint32_t a[K];
            uint64_t attempt = 0, r;
            do {
                r = word_at(attempt * S + g, key);
#pragma unroll
                for (int i = 0; i < K; ++i)
                    if (i < kk) a[i] = mul_roll(bound, r);
                ++attempt;
            } while (r < t && attempt <= kMaxAttempts);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) out[first + i] = a[i];
        }
    }
}

template <int K>
hipError_t launch_dice_k(const uint32_t *bounds, uint32_t *out, uint64_t count, StreamKey key,
                         uint32_t *status, hipStream_t stream)
{
    const uint64_t S = (count + K - 1) / K;
    const uint64_t nquads = (count / K) / 4;
    const uint64_t lanes = nquads + (S - 4 * nquads);
    const uint64_t blocks = (lanes + 255) / 256;
    const bool vec = ((((uintptr_t)bounds) | ((uintptr_t)out)) & 15) == 0;
    if (vec)
        dice_kernel<K, true><<<dim3((uint32_t)blocks), dim3(256), 0, stream>>>(bounds, out, count, S,
                                                                              nquads, key, status);
    else
        dice_kernel<K, false><<<dim3((uint32_t)blocks), dim3(256), 0, stream>>>(
            bounds, out, count, S, nquads, key, status);
    return hipGetLastError();
}

template <int K>
hipError_t launch_dice_const_k(uint32_t bound, uint32_t *out, uint64_t count, StreamKey key,
                               uint64_t t_full, uint64_t t_last, hipStream_t stream)
{
    const uint64_t S = (count + K - 1) / K;
    const uint64_t nquads = (count / K) / 4;
    const uint64_t lanes = nquads + (S - 4 * nquads);
    const uint64_t blocks = (lanes + 255) / 256;
    const bool vec = (((uintptr_t)out) & 15) == 0;
    if (vec)
        dice_const_kernel<K, true><<<dim3((uint32_t)blocks), dim3(256), 0, stream>>>(
            bound, out, count, S, nquads, key, t_full, t_last);
    else
        dice_const_kernel<K, false><<<dim3((uint32_t)blocks), dim3(256), 0, stream>>>(
            bound, out, count, S, nquads, key, t_full, t_last);
    return hipGetLastError();
}

} // namespace

hipError_t launch_dice(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                       StreamKey key, uint32_t *status, hipStream_t stream)
{
    switch (k) {
    case 1: return launch_dice_k<1>(bounds, out, count, key, status, stream);
    case 2: return launch_dice_k<2>(bounds, out, count, key, status, stream);
    case 3: return launch_dice_k<3>(bounds, out, count, key, status, stream);
    case 4: return launch_dice_k<4>(bounds, out, count, key, status, stream);
    case 5: return launch_dice_k<5>(bounds, out, count, key, status, stream);
    case 6: return launch_dice_k<6>(bounds, out, count, key, status, stream);
    case 7: return launch_dice_k<7>(bounds, out, count, key, status, stream);
    case 8: return launch_dice_k<8>(bounds, out, count, key, status, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dice_const(uint32_t bound, uint32_t *out, uint64_t count, uint32_t k,
                             StreamKey key, uint64_t t_full, uint64_t t_last, hipStream_t stream)
{
    switch (k) {
    case 1: return launch_dice_const_k<1>(bound, out, count, key, t_full, t_last, stream);
    case 2: return launch_dice_const_k<2>(bound, out, count, key, t_full, t_last, stream);
    case 3: return launch_dice_const_k<3>(bound, out, count, key, t_full, t_last, stream);
    case 4: return launch_dice_const_k<4>(bound, out, count, key, t_full, t_last, stream);
    case 5: return launch_dice_const_k<5>(bound, out, count, key, t_full, t_last, stream);
    case 6: return launch_dice_const_k<6>(bound, out, count, key, t_full, t_last, stream);
    case 7: return launch_dice_const_k<7>(bound, out, count, key, t_full, t_last, stream);
    case 8: return launch_dice_const_k<8>(bound, out, count, key, t_full, t_last, stream);
    default: return hipErrorInvalidValue;
    }
}

} // namespace brr
