// Device-side building blocks shared by the dice and shuffle kernels of
// libbrr (gfx950, wave64). Everything here is exact integer arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace brr {

// Native 4 x u32 vector (16-byte global loads/stores, nontemporal builtins).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// three dwords at 4-byte alignment: one 12-byte load or store
typedef uint32_t u32x3 __attribute__((ext_vector_type(3), aligned(4)));

// Bits of the per-device status word (see brr_sync_status).
enum : uint32_t { kDevZeroBound = 1u, kDevOverflow = 2u };

// Key of one word stream: the seed halves (Philox key) and the instance
// halves (upper counter words).
struct StreamKey {
    uint32_t seed_lo, seed_hi, inst_lo, inst_hi;
};

__host__ __device__ inline StreamKey make_key(uint64_t seed, uint64_t inst)
{
    return StreamKey{(uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)inst, (uint32_t)(inst >> 32)};
}

// Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds, each two 32x32->64 multiplies (one v_mad_u64_u32 each) whose high
// halves are xored with the other counter words and the round key; the key
// advances by the Weyl increments between rounds. The key is wave-uniform
// in every caller, so its schedule stays in scalar registers.
__host__ __device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t m1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Words 2*blk (even half) and 2*blk+1 (odd half) of a stream.
__device__ __forceinline__ void word_pair(uint64_t blk, const StreamKey &key, uint64_t &w_even,
                                          uint64_t &w_odd)
{
    const uint4 x = philox4x32_10((uint32_t)blk, (uint32_t)(blk >> 32), key.inst_lo, key.inst_hi,
                                  key.seed_lo, key.seed_hi);
    w_even = (uint64_t)x.x | ((uint64_t)x.y << 32);
    w_odd = (uint64_t)x.z | ((uint64_t)x.w << 32);
}

// Word c of a stream.
__device__ __forceinline__ uint64_t word_at(uint64_t c, const StreamKey &key)
{
    uint64_t e, o;
    word_pair(c >> 1, key, e, o);
    return (c & 1) ? o : e;
}

// One link of the Theorem 1 chain for a bound b < 2^32:
// (a, r) <- b (x) r, a = high 64 bits (< b), r = low 64 bits of b*r.
// b*r = b*r_hi*2^32 + b*r_lo; two 32x32->64 multiply-adds.
__host__ __device__ __forceinline__ uint32_t mul_roll(uint32_t b, uint64_t &r)
{
    const uint64_t lo = (uint64_t)b * (uint32_t)r;
    const uint64_t hi = (uint64_t)b * (uint32_t)(r >> 32) + (lo >> 32);
    r = (hi << 32) | (uint32_t)lo;
    return (uint32_t)(hi >> 32);
}

// 2^64 mod B for 1 <= B < 2^64 (Lemire's threshold of a bound product).
// For 2^32 < B <= 2^62 the quotient q = floor(2^64 / B) < 2^32 comes from
// one f64 division: (double)B and the quotient are each rounded to nearest,
// so qd is within q * 2^-52 < 2^-20 of 2^64 / B and floor(qd) - 1 is one of
// q - 2, q - 1, q. Then 2^64 - q0 * B = t + (q - q0) * B < 3B (no wrap) and
// at most two subtractions of B give t exactly. Above 2^62, q < 4 and the
// remainder follows from 2^64 - B by at most two subtractions. Small B (only
// reached with probability below 2^-32 per roll) uses the integer remainder.
__host__ __device__ __forceinline__ uint64_t pow2_64_mod(uint64_t B)
{
    if (B > (1ull << 62)) {
        uint64_t t = 0 - B;
        if (t >= B) t -= B;
        if (t >= B) t -= B;
        return t;
    }
    if (B <= (1ull << 32)) return (0 - B) % B;
    const double qd = 18446744073709551616.0 / (double)B;
    const uint32_t q0 = (uint32_t)qd - 1u;
    uint64_t t = 0 - (uint64_t)q0 * B;
    if (t >= B) t -= B;
    if (t >= B) t -= B;
    return t;
}

// The division form of batched dice (Sec. 2.1): the next die of the value V
// below the remaining bound product is V mod b, and V continues as V div b.
// One 64-by-32-bit division (the compiler's expansion; the form exists as the
// division-based comparison, so it keeps the plain operation).
__host__ __device__ __forceinline__ uint32_t div_digit(uint32_t b, uint64_t &V)
{
    const uint64_t q = V / b;
    const uint32_t d = (uint32_t)(V - q * b);
    V = q;
    return d;
}

// Exact product of u32 bounds as long as it is at most 2^64.
// p holds the product modulo 2^64; e64 marks a product of exactly 2^64
// (then p == 0); over marks a product above 2^64; zero marks a zero bound.
struct BoundProduct {
    uint64_t p;
    bool e64, over, zero;

    __host__ __device__ __forceinline__ void init(uint32_t b)
    {
        p = b;
        e64 = false;
        over = false;
        zero = (b == 0);
    }

    // Branch-free (lanes of a wavefront all take the same steps).
    __host__ __device__ __forceinline__ void mul(uint32_t b)
    {
        zero |= (b == 0);
        over |= e64 && b > 1; // 2^64 * b exceeds 2^64 for b > 1 (p is 0 and stays 0)
        const uint64_t lo = (uint64_t)(uint32_t)p * b;
        const uint64_t hi = (uint64_t)(uint32_t)(p >> 32) * b + (lo >> 32); // < 2^64
        const uint32_t top = (uint32_t)(hi >> 32); // bits 64.. of the product
        p = (hi << 32) | (uint32_t)lo;
        const bool exact = top == 1 && p == 0;
        e64 |= exact;
        over |= top != 0 && !exact;
    }
};

// The product of a group's K bounds. The usual case (no zero bound, product
// below 2^64) takes plain multiplies, the first two bounds in one step (two
// u32 factors never exceed 2^64), and only notes whether any step carried
// past 64 bits; a zero bound or a carry sends the group through the exact
// steps of BoundProduct, which tell a product of exactly 2^64 from a larger
// one.
template <int K>
__host__ __device__ __forceinline__ BoundProduct bound_product(const uint32_t *b)
{
    BoundProduct P;
    if constexpr (K == 1) {
        P.init(b[0]);
    } else {
        uint64_t p = (uint64_t)b[0] * b[1];
        uint32_t carry = 0, low = b[0] < b[1] ? b[0] : b[1];
#pragma unroll
        for (int i = 2; i < K; ++i) {
            const uint64_t lo = (uint64_t)(uint32_t)p * b[i];
            const uint64_t hi = (uint64_t)(uint32_t)(p >> 32) * b[i] + (lo >> 32);
            carry |= (uint32_t)(hi >> 32);
            p = (hi << 32) | (uint32_t)lo;
            low = low < b[i] ? low : b[i];
        }
        if (carry == 0 && low != 0) {
            P.p = p;
            P.e64 = P.over = P.zero = false;
        } else {
            P.init(b[0]);
#pragma unroll
            for (int i = 1; i < K; ++i) P.mul(b[i]);
        }
    }
    return P;
}

// Acceptance of a rolled group with exact product P (Lemire's criterion on
// the leftover, Theorem 1): returns the threshold t to compare r against.
// Only called when r < P, so t is computed on the rare slow path.
__host__ __device__ __forceinline__ uint64_t group_threshold(const BoundProduct &P)
{
    return P.e64 ? 0 : pow2_64_mod(P.p);
}

// Wave64 inclusive prefix sum of v across the lanes of the wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

} // namespace brr
