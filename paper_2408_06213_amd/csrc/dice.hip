// Dice streams: groups of K bounds rolled from one 64-bit word each by the
// Theorem 1 chain (Sec. 4), accepted by Algorithm 3 (Sec. 5): the exact
// bound product P is formed, and only when the leftover r is below P is the
// threshold 2^64 mod P computed and the group rerolled while r stays below
// it. The constant-bound form uses Algorithm 2 with t precomputed.
//
// Work mapping: a wavefront owns a tile of 64*G consecutive groups; lane L
// takes groups g0 + 64j + L (j < G), so every load and store instruction of
// the wave covers one contiguous span of 64*K*4 bytes. Group g reads word g
// on its first attempt; words 2m and 2m+1 are the two halves of Philox block
// m, so lanes L and L^1 each compute one block per pair of their groups and
// swap the half the other one needs (a DPP lane swap). Rerolls read word
// a*S + g on attempt a.
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace brr {

namespace {

constexpr uint64_t kMaxAttempts = 1024;
constexpr int kGroupsPerLane = 4;
constexpr uint32_t kUndecided = 64;

// Value of lane L^1 (swap within lane pairs, quad_perm [1,0,3,2]).
__device__ __forceinline__ uint64_t swap_lane_pair(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, 0xB1, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), 0xB1, 0xF, 0xF, false);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// First-attempt words of this lane's G groups g0 + 64j + lane.
template <int G>
__device__ __forceinline__ void tile_words(uint64_t g0, uint32_t lane, const StreamKey &key,
                                           uint64_t *r)
{
#pragma unroll
    for (int t = 0; t < G / 2; ++t) {
        // even lanes: block of their group 2t (and the next lane's);
        // odd lanes: block of the previous lane's group 2t+1 (and theirs)
        const uint64_t gb = g0 + 64 * (2 * t + (lane & 1)) + (lane & ~1u);
        uint64_t we, wo;
        word_pair(gb >> 1, key, we, wo);
        const uint64_t recv = swap_lane_pair((lane & 1) ? we : wo);
        r[2 * t] = (lane & 1) ? recv : we;
        r[2 * t + 1] = (lane & 1) ? wo : recv;
    }
}

template <int K, bool VEC>
__device__ __forceinline__ void load_group(const uint32_t *__restrict__ p, uint32_t *b)
{
    if (VEC && K == 4) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        b[0] = v.x;
        b[1] = v.y;
        b[2] = v.z;
        b[3] = v.w;
    } else if (VEC && K == 2) {
        const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
        b[0] = v.x;
        b[1] = v.y;
    } else if (K == 3) { // one 12-byte access (4-byte alignment suffices)
        const u32x3 v = __builtin_nontemporal_load(reinterpret_cast<const u32x3 *>(p));
        b[0] = v.x;
        b[1] = v.y;
        b[2] = v.z;
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) b[i] = __builtin_nontemporal_load(p + i);
    }
}

template <int K, bool VEC>
__device__ __forceinline__ void store_group(uint32_t *__restrict__ p, const uint32_t *a)
{
    if (VEC && K == 4) {
        const u32x4 v = {a[0], a[1], a[2], a[3]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
    } else if (VEC && K == 2) {
        const u32x2 v = {a[0], a[1]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(p));
    } else if (K == 3) {
        const u32x3 v = {a[0], a[1], a[2]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x3 *>(p));
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) __builtin_nontemporal_store(a[i], p + i);
    }
}

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

// The group's product when its threshold decides (r below it), else 0:
// accepted at once (r >= P > t, or P = 2^64), or a bad group, flagged in
// err.
template <int K>
__device__ __forceinline__ uint64_t undecided_product(const uint32_t *b, uint64_t r, uint32_t &err)
{
    const BoundProduct P = bound_product<K>(b);
    if (P.zero) {
        err |= kDevZeroBound;
        return 0;
    }
    if (P.over) {
        err |= kDevOverflow;
        return 0;
    }
    return (P.e64 || r >= P.p) ? 0 : P.p; // P >= 1 here
}

// Rolls group g again from attempt 1 on until accepted.
template <int K>
__device__ __forceinline__ void reroll_group(const uint32_t *b, int kk, uint32_t *a, uint64_t t,
                                             uint64_t S, uint64_t g, const StreamKey &key)
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

template <int K, int G, bool VEC>
__global__ __launch_bounds__(256) void dice_kernel(const uint32_t *__restrict__ bounds,
                                                   uint32_t *__restrict__ out, uint64_t count,
                                                   uint64_t S, uint64_t full, StreamKey key,
                                                   uint32_t *status)
{
    // Groups whose threshold decides (r < P: one in 16 at k = 4 with 16-bit
    // bounds) are set aside (up to kUndecided per wave) and decided after
    // the checks, one per lane in one pass, instead of in the check of
    // every j, where nearly every j has such a lane and the whole wave runs
    // the threshold's steps.
    __shared__ uint64_t und_p[4][kUndecided], und_r[4][kUndecided];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t g0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * G);
    if (g0 >= S) return; // the whole wavefront leaves together
    uint64_t r[G];
    tile_words<G>(g0, lane, key, r);
    uint32_t b[G][K], a[G][K];
    uint32_t err = 0;
    if (g0 + 64 * G <= full) { // every group of the tile has K dice
        const uint64_t lt_mask = (1ull << lane) - 1;
#pragma unroll
        for (int j = 0; j < G; ++j) load_group<K, VEC>(bounds + K * (g0 + 64 * j + lane), b[j]);
#pragma unroll
        for (int j = 0; j < G; ++j)
#pragma unroll
            for (int i = 0; i < K; ++i) a[j][i] = mul_roll(b[j][i], r[j]);
        uint32_t at[G], nu = 0; // slot of each set-aside group (kUndecided: none)
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t ps = undecided_product<K>(b[j], r[j], err);
            const uint64_t um = __ballot(ps != 0);
            const uint32_t slot = nu + (uint32_t)__builtin_popcountll(um & lt_mask);
            nu += (uint32_t)__builtin_popcountll(um);
            at[j] = kUndecided;
            if (ps != 0) {
                if (slot < kUndecided) {
                    und_p[w][slot] = ps;
                    und_r[w][slot] = r[j];
                    at[j] = slot;
                } else {
                    const uint64_t t = pow2_64_mod(ps);
                    if (r[j] < t) reroll_group<K>(b[j], K, a[j], t, S, g0 + 64 * j + lane, key);
                }
            }
        }
        if (nu != 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // the threshold of each set-aside group, or 0 once its word is accepted
            if (lane < std::min(nu, kUndecided)) {
                const uint64_t t = pow2_64_mod(und_p[w][lane]);
                und_p[w][lane] = und_r[w][lane] < t ? t : 0;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const uint64_t t = at[j] < kUndecided ? und_p[w][at[j]] : 0;
                if (t != 0) reroll_group<K>(b[j], K, a[j], t, S, g0 + 64 * j + lane, key);
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) store_group<K, VEC>(out + K * (g0 + 64 * j + lane), a[j]);
    } else { // last tile: short or missing groups
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t g = g0 + 64 * j + lane;
            const int kk = (g < full) ? K : (g < S ? (int)(count - K * g) : 0);
            if (kk == 0) continue;
#pragma unroll
            for (int i = 0; i < K; ++i) b[j][i] = (i < kk) ? bounds[K * g + i] : 1u;
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) a[j][i] = mul_roll(b[j][i], r[j]);
            bool need;
            uint64_t t;
            check_group<K>(b[j], kk, r[j], need, t, err);
            if (need) reroll_group<K>(b[j], kk, a[j], t, S, g, key);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) out[K * g + i] = a[j][i];
        }
    }
    if (err) atomicOr(status, err);
}

// The division form (Sec. 2.1), the comparison for the kernel above: group
// g rolls one value V below the product P of its bounds by Lemire's method
// (Sec. 2) on the same words (attempt a reads word a*S + g), accepting when
// the low half of P*r is at least 2^64 mod P, and splits V into dice by
// successive division: a_1 = V mod b_1, V <- V div b_1, ... (the last die is
// what remains). Same tiling and word sharing as dice_kernel.
template <int K>
__device__ __forceinline__ void div_group(const uint32_t *b, int kk, uint32_t *a, uint64_t r,
                                          uint64_t S, uint64_t g, const StreamKey &key,
                                          uint32_t &err)
{
    BoundProduct P;
    P.init(b[0]);
#pragma unroll
    for (int i = 1; i < K; ++i)
        if (i < kk) P.mul(b[i]);
    if (P.zero) {
        err |= kDevZeroBound;
        return;
    }
    if (P.over) {
        err |= kDevOverflow;
        return;
    }
    uint64_t V = r; // P = 2^64: every word is accepted and V is the word
    if (!P.e64) {
        V = __umul64hi(P.p, r);
        uint64_t y = P.p * r;
        if (y < P.p) {
            const uint64_t t = pow2_64_mod(P.p);
            // each attempt is rejected with probability t / 2^64 < 1/2; the
            // cap only bounds the loop against corrupted inputs
            for (uint64_t attempt = 1; y < t && attempt <= kMaxAttempts; ++attempt) {
                const uint64_t w = word_at(attempt * S + g, key);
                V = __umul64hi(P.p, w);
                y = P.p * w;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i < kk) a[i] = (i + 1 < kk) ? div_digit(b[i], V) : (uint32_t)V;
}

template <int K, int G, bool VEC>
__global__ __launch_bounds__(256) void dice_div_kernel(const uint32_t *__restrict__ bounds,
                                                       uint32_t *__restrict__ out, uint64_t count,
                                                       uint64_t S, uint64_t full, StreamKey key,
                                                       uint32_t *status)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t g0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * G);
    if (g0 >= S) return;
    uint64_t r[G];
    tile_words<G>(g0, lane, key, r);
    uint32_t b[G][K], a[G][K];
    uint32_t err = 0;
    if (g0 + 64 * G <= full) {
#pragma unroll
        for (int j = 0; j < G; ++j) load_group<K, VEC>(bounds + K * (g0 + 64 * j + lane), b[j]);
#pragma unroll
        for (int j = 0; j < G; ++j)
            div_group<K>(b[j], K, a[j], r[j], S, g0 + 64 * j + lane, key, err);
#pragma unroll
        for (int j = 0; j < G; ++j) store_group<K, VEC>(out + K * (g0 + 64 * j + lane), a[j]);
    } else {
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t g = g0 + 64 * j + lane;
            const int kk = (g < full) ? K : (g < S ? (int)(count - K * g) : 0);
            if (kk == 0) continue;
#pragma unroll
            for (int i = 0; i < K; ++i) b[j][i] = (i < kk) ? bounds[K * g + i] : 1u;
            div_group<K>(b[j], kk, a[j], r[j], S, g, key, err);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) out[K * g + i] = a[j][i];
        }
    }
    if (err) atomicOr(status, err);
}

// Known bounds (Algorithm 2): every group rolls the same tuple tb.b[0..K),
// t_full is 2^64 mod their product, t_last the same for the short last group
// (the tuple's first count mod K bounds). A constant bound is the tuple of K
// equal bounds.
template <int K, int G, bool VEC>
__global__ __launch_bounds__(256) void dice_const_kernel(BoundTuple tb, uint32_t *__restrict__ out,
                                                         uint64_t count, uint64_t S, uint64_t full,
                                                         StreamKey key, uint64_t t_full,
                                                         uint64_t t_last)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t g0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * G);
    if (g0 >= S) return;
    uint64_t r[G];
    tile_words<G>(g0, lane, key, r);
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const uint64_t g = g0 + 64 * j + lane;
        const int kk = (g < full) ? K : (g < S ? (int)(count - K * g) : 0);
        if (kk == 0) continue;
        const uint64_t t = (kk == K) ? t_full : t_last;
        uint32_t a[K];
        uint64_t rr = r[j];
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < kk) a[i] = mul_roll(tb.b[i], rr);
        for (uint64_t attempt = 1; rr < t && attempt <= kMaxAttempts; ++attempt) {
            rr = word_at(attempt * S + g, key);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) a[i] = mul_roll(tb.b[i], rr);
        }
        if (kk == K)
            store_group<K, VEC>(out + K * g, a);
        else
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) out[K * g + i] = a[i];
    }
}

uint32_t tile_blocks(uint64_t S)
{
    const uint64_t waves = (S + 64 * kGroupsPerLane - 1) / (64 * kGroupsPerLane);
    return (uint32_t)((waves + 3) / 4); // 4 wavefronts per 256-thread block
}

template <int K>
hipError_t launch_dice_k(const uint32_t *bounds, uint32_t *out, uint64_t count, StreamKey key,
                         uint32_t *status, hipStream_t stream)
{
    const uint64_t S = (count + K - 1) / K;
    const uint64_t full = count / K;
    const bool vec = ((((uintptr_t)bounds) | ((uintptr_t)out)) & 15) == 0;
    if (vec)
        dice_kernel<K, kGroupsPerLane, true><<<tile_blocks(S), 256, 0, stream>>>(
            bounds, out, count, S, full, key, status);
    else
        dice_kernel<K, kGroupsPerLane, false><<<tile_blocks(S), 256, 0, stream>>>(
            bounds, out, count, S, full, key, status);
    return hipGetLastError();
}

template <int K>
hipError_t launch_dice_div_k(const uint32_t *bounds, uint32_t *out, uint64_t count, StreamKey key,
                             uint32_t *status, hipStream_t stream)
{
    const uint64_t S = (count + K - 1) / K;
    const uint64_t full = count / K;
    const bool vec = ((((uintptr_t)bounds) | ((uintptr_t)out)) & 15) == 0;
    if (vec)
        dice_div_kernel<K, kGroupsPerLane, true><<<tile_blocks(S), 256, 0, stream>>>(
            bounds, out, count, S, full, key, status);
    else
        dice_div_kernel<K, kGroupsPerLane, false><<<tile_blocks(S), 256, 0, stream>>>(
            bounds, out, count, S, full, key, status);
    return hipGetLastError();
}

template <int K>
hipError_t launch_dice_const_k(const BoundTuple &tb, uint32_t *out, uint64_t count, StreamKey key,
                               uint64_t t_full, uint64_t t_last, hipStream_t stream)
{
    const uint64_t S = (count + K - 1) / K;
    const uint64_t full = count / K;
    const bool vec = (((uintptr_t)out) & 15) == 0;
    if (vec)
        dice_const_kernel<K, kGroupsPerLane, true><<<tile_blocks(S), 256, 0, stream>>>(
            tb, out, count, S, full, key, t_full, t_last);
    else
        dice_const_kernel<K, kGroupsPerLane, false><<<tile_blocks(S), 256, 0, stream>>>(
            tb, out, count, S, full, key, t_full, t_last);
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

hipError_t launch_dice_div(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                           StreamKey key, uint32_t *status, hipStream_t stream)
{
    switch (k) {
    case 1: return launch_dice_div_k<1>(bounds, out, count, key, status, stream);
    case 2: return launch_dice_div_k<2>(bounds, out, count, key, status, stream);
    case 3: return launch_dice_div_k<3>(bounds, out, count, key, status, stream);
    case 4: return launch_dice_div_k<4>(bounds, out, count, key, status, stream);
    case 5: return launch_dice_div_k<5>(bounds, out, count, key, status, stream);
    case 6: return launch_dice_div_k<6>(bounds, out, count, key, status, stream);
    case 7: return launch_dice_div_k<7>(bounds, out, count, key, status, stream);
    case 8: return launch_dice_div_k<8>(bounds, out, count, key, status, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dice_const(const BoundTuple &tb, uint32_t *out, uint64_t count, uint32_t k,
                             StreamKey key, uint64_t t_full, uint64_t t_last, hipStream_t stream)
{
    switch (k) {
    case 1: return launch_dice_const_k<1>(tb, out, count, key, t_full, t_last, stream);
    case 2: return launch_dice_const_k<2>(tb, out, count, key, t_full, t_last, stream);
    case 3: return launch_dice_const_k<3>(tb, out, count, key, t_full, t_last, stream);
    case 4: return launch_dice_const_k<4>(tb, out, count, key, t_full, t_last, stream);
    case 5: return launch_dice_const_k<5>(tb, out, count, key, t_full, t_last, stream);
    case 6: return launch_dice_const_k<6>(tb, out, count, key, t_full, t_last, stream);
    case 7: return launch_dice_const_k<7>(tb, out, count, key, t_full, t_last, stream);
    case 8: return launch_dice_const_k<8>(tb, out, count, key, t_full, t_last, stream);
    default: return hipErrorInvalidValue;
    }
}

} // namespace brr
