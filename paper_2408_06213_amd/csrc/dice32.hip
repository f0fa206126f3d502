// Dice streams at word width L = 32 (Theorem 1 at L = 32, Sec. 4;
// Algorithm 3, Sec. 5): each group of K bounds is rolled from one 32-bit
// word, the chain taking the high and low 32 bits of b_i * r (one 32x32 ->
// 64-bit multiply per die), accepted when the leftover is at least
// 2^32 mod P for the bound product P <= 2^32.
//
// Word c of the 32-bit stream is the 32-bit half c mod 2 (low half first)
// of 64-bit word c/2, i.e. x[c mod 4] of Philox block c/4. Attempt a of
// group g reads word a*S + g, as at L = 64.
//
// Work mapping as at L = 64: lane L takes groups g0 + 64j + L (j < 4), so
// each load and store instruction covers one contiguous span. The four
// lanes of a quad hold consecutive groups, which share one Philox block per
// j; each lane computes the block of one j and a quad transpose (DPP) hands
// every lane its word of all four blocks.
#include "device.hpp"
#include "internal.hpp"

namespace brr {

namespace {

constexpr uint64_t kMaxAttempts32 = 1024;
constexpr int kGroups32 = 4; // groups per lane = lanes per quad

// Value of lane L ^ M within this lane's quad (M = 1: quad_perm [1,0,3,2];
// M = 2: quad_perm [2,3,0,1]).
template <int M> __device__ __forceinline__ uint32_t from_quad_xor(uint32_t v)
{
    constexpr int ctrl = (M == 1) ? 0xB1 : 0x4E;
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xF, 0xF, false);
}

// First-attempt words of this lane's groups g0 + 64j + lane, j = 0..3.
//
// Lane q of a quad (q = lane mod 4) computes the Philox block of slot j = q,
// i.e. the words of the quad's four groups g0 + 64q + (lane & ~3) + m; word
// m belongs to quad lane m. As a matrix M[row = computing lane][column =
// receiving lane] this is a 4x4 transpose, done as two exchange stages
// (partner q ^ 1, then q ^ 2) with selects on the lane bits only: no
// dynamically indexed register array, which the compiler would put in
// scratch memory.
__device__ __forceinline__ void tile_words32(uint64_t g0, uint32_t lane, const StreamKey &key,
                                             uint32_t (&r)[4])
{
    const bool o1 = lane & 1, o2 = lane & 2;
    uint64_t we, wo;
    word_pair((g0 + 64 * (lane & 3) + (lane & ~3u)) >> 2, key, we, wo);
    const uint32_t x0 = (uint32_t)we, x1 = (uint32_t)(we >> 32), x2 = (uint32_t)wo,
                   x3 = (uint32_t)(wo >> 32);
    // stage 1: keep the columns of this lane's parity, swap the others with
    // lane q ^ 1; afterwards this lane holds rows q and q ^ 1 of columns
    // c0 = q & 1 and c1 = c0 + 2
    const uint32_t k0 = o1 ? x1 : x0, k1 = o1 ? x3 : x2;
    const uint32_t r0 = from_quad_xor<1>(o1 ? x0 : x1);
    const uint32_t r1 = from_quad_xor<1>(o1 ? x2 : x3);
    // stage 2: keep column q, swap the other with lane q ^ 2
    const uint32_t u0 = o2 ? k1 : k0; // M[q][q]
    const uint32_t u1 = o2 ? r1 : r0; // M[q ^ 1][q]
    const uint32_t w0 = from_quad_xor<2>(o2 ? k0 : k1); // M[q ^ 2][q]
    const uint32_t w1 = from_quad_xor<2>(o2 ? r0 : r1); // M[q ^ 3][q]
    // order by row: rows q, q ^ 1 share bit 1 with q, rows q ^ 2, q ^ 3 not
    const uint32_t ue = o1 ? u1 : u0, uo = o1 ? u0 : u1; // even, odd row of {q, q ^ 1}
    const uint32_t we_ = o1 ? w1 : w0, wo_ = o1 ? w0 : w1;
    r[0] = o2 ? we_ : ue;
    r[1] = o2 ? wo_ : uo;
    r[2] = o2 ? ue : we_;
    r[3] = o2 ? uo : wo_;
}

__device__ __forceinline__ uint32_t word32_at(uint64_t c, const StreamKey &key)
{
    const uint64_t w = word_at(c >> 1, key);
    return (c & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
}

// (a, r) <- b (x) r at L = 32.
__device__ __forceinline__ uint32_t mul_roll32(uint32_t b, uint32_t &r)
{
    const uint64_t x = (uint64_t)b * r;
    r = (uint32_t)x;
    return (uint32_t)(x >> 32);
}

template <int K>
__device__ __forceinline__ void roll_group32(const uint32_t *b, int kk, uint32_t *a, uint32_t r,
                                             uint64_t S, uint64_t g, const StreamKey &key,
                                             uint32_t &err)
{
    uint64_t P = 1;
    bool zero = false, over = false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (i < kk) {
            zero |= b[i] == 0;
            P *= b[i];
            over |= P > (1ull << 32); // once above 2^32 it stays above (factors >= 1)
            if (P > (1ull << 32)) P = (1ull << 32) + 1;
        }
    }
    uint32_t rr = r;
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i < kk) a[i] = mul_roll32(b[i], rr);
    if (zero) {
        err |= kDevZeroBound;
        return;
    }
    if (over) {
        err |= kDevOverflow;
        return;
    }
    if (P == (1ull << 32) || (uint64_t)rr >= P) return; // threshold 0, or r >= P > t
    const uint32_t p32 = (uint32_t)P;
    const uint32_t t = (0u - p32) % p32; // 2^32 mod P
    // each attempt is rejected with probability t / 2^32 < 1/2; the cap only
    // bounds the loop against corrupted inputs
    for (uint64_t attempt = 1; rr < t && attempt <= kMaxAttempts32; ++attempt) {
        rr = word32_at(attempt * S + g, key);
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < kk) a[i] = mul_roll32(b[i], rr);
    }
}

template <int K, bool VEC>
__device__ __forceinline__ void load_group32(const uint32_t *__restrict__ p, uint32_t *b)
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
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) b[i] = __builtin_nontemporal_load(p + i);
    }
}

template <int K, bool VEC>
__device__ __forceinline__ void store_group32(uint32_t *__restrict__ p, const uint32_t *a)
{
    if (VEC && K == 4) {
        const u32x4 v = {a[0], a[1], a[2], a[3]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
    } else if (VEC && K == 2) {
        const u32x2 v = {a[0], a[1]};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(p));
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) __builtin_nontemporal_store(a[i], p + i);
    }
}

template <int K, bool VEC>
__global__ __launch_bounds__(256) void dice32_kernel(const uint32_t *__restrict__ bounds,
                                                     uint32_t *__restrict__ out, uint64_t count,
                                                     uint64_t S, uint64_t full, StreamKey key,
                                                     uint32_t *status)
{
    constexpr int G = kGroups32;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t g0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * G);
    if (g0 >= S) return; // the whole wavefront leaves together
    uint32_t r[G];
    tile_words32(g0, lane, key, r);
    uint32_t b[G][K], a[G][K];
    uint32_t err = 0;
    if (g0 + 64 * G <= full) { // every group of the tile has K dice
#pragma unroll
        for (int j = 0; j < G; ++j) load_group32<K, VEC>(bounds + K * (g0 + 64 * j + lane), b[j]);
#pragma unroll
        for (int j = 0; j < G; ++j)
            roll_group32<K>(b[j], K, a[j], r[j], S, g0 + 64 * j + lane, key, err);
#pragma unroll
        for (int j = 0; j < G; ++j) store_group32<K, VEC>(out + K * (g0 + 64 * j + lane), a[j]);
    } else { // last tile: short or missing groups
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t g = g0 + 64 * j + lane;
            const int kk = (g < full) ? K : (g < S ? (int)(count - K * g) : 0);
            if (kk == 0) continue;
#pragma unroll
            for (int i = 0; i < K; ++i) b[j][i] = (i < kk) ? bounds[K * g + i] : 1u;
            roll_group32<K>(b[j], kk, a[j], r[j], S, g, key, err);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < kk) out[K * g + i] = a[j][i];
        }
    }
    if (err) atomicOr(status, err);
}

template <int K>
hipError_t launch_dice32_k(const uint32_t *bounds, uint32_t *out, uint64_t count, StreamKey key,
                           uint32_t *status, hipStream_t stream)
{
    const uint64_t S = (count + K - 1) / K;
    const uint64_t full = count / K;
    const uint64_t waves = (S + 64 * kGroups32 - 1) / (64 * kGroups32);
    const uint32_t blocks = (uint32_t)((waves + 3) / 4); // 4 wavefronts per block
    const bool vec = ((((uintptr_t)bounds) | ((uintptr_t)out)) & 15) == 0;
    if (vec)
        dice32_kernel<K, true><<<blocks, 256, 0, stream>>>(bounds, out, count, S, full, key,
                                                           status);
    else
        dice32_kernel<K, false><<<blocks, 256, 0, stream>>>(bounds, out, count, S, full, key,
                                                            status);
    return hipGetLastError();
}

} // namespace

hipError_t launch_dice32(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                         StreamKey key, uint32_t *status, hipStream_t stream)
{
    switch (k) {
    case 1: return launch_dice32_k<1>(bounds, out, count, key, status, stream);
    case 2: return launch_dice32_k<2>(bounds, out, count, key, status, stream);
    case 3: return launch_dice32_k<3>(bounds, out, count, key, status, stream);
    case 4: return launch_dice32_k<4>(bounds, out, count, key, status, stream);
    case 5: return launch_dice32_k<5>(bounds, out, count, key, status, stream);
    case 6: return launch_dice32_k<6>(bounds, out, count, key, status, stream);
    case 7: return launch_dice32_k<7>(bounds, out, count, key, status, stream);
    case 8: return launch_dice32_k<8>(bounds, out, count, key, status, stream);
    default: return hipErrorInvalidValue;
    }
}

} // namespace brr
