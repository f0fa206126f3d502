// ChaCha20 (Bernstein 2008) in counter mode as a word source: word c of
// instance `inst` under `seed` is output words 2m, 2m+1 (low half first,
// m = c mod 8) of block c/8, whose input state holds the four constant
// words, key words (lo32 seed, hi32 seed, 0, 0, 0, 0, 0, 0), the 64-bit block
// counter in words 12-13 and the 64-bit nonce inst in words 14-15.
#pragma once

#include "device.hpp"

namespace brr {
namespace {

constexpr int kWordsPerBlock = 8;

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int n)
{
    return __builtin_amdgcn_alignbit(x, x, 32 - n); // rotate right by 32 - n
}

__device__ __forceinline__ void quarter(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d)
{
    a += b;
    d = rotl32(d ^ a, 16);
    c += d;
    b = rotl32(b ^ c, 12);
    a += b;
    d = rotl32(d ^ a, 8);
    c += d;
    b = rotl32(b ^ c, 7);
}

// The 16 output words of block `blk` (20 rounds: ten column/diagonal pairs,
// then the input state added back).
__device__ __forceinline__ void chacha20_block(const StreamKey &key, uint64_t blk,
                                               uint32_t (&x)[16])
{
    const uint32_t in[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                             key.seed_lo, key.seed_hi, 0u, 0u, 0u, 0u, 0u, 0u,
                             (uint32_t)blk, (uint32_t)(blk >> 32), key.inst_lo, key.inst_hi};
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = in[i];
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        quarter(x[0], x[4], x[8], x[12]);
        quarter(x[1], x[5], x[9], x[13]);
        quarter(x[2], x[6], x[10], x[14]);
        quarter(x[3], x[7], x[11], x[15]);
        quarter(x[0], x[5], x[10], x[15]);
        quarter(x[1], x[6], x[11], x[12]);
        quarter(x[2], x[7], x[8], x[13]);
        quarter(x[3], x[4], x[9], x[14]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] += in[i];
}

// Word c alone (kept out of line so that a kernel holds one copy of the
// rounds for it).
__device__ __noinline__ uint64_t chacha_word_at(uint64_t c, StreamKey key)
{
    uint32_t x[16];
    chacha20_block(key, c / kWordsPerBlock, x);
    const uint32_t m = (uint32_t)(c % kWordsPerBlock);
    uint64_t w = 0;
#pragma unroll
    for (uint32_t j = 0; j < kWordsPerBlock; ++j)
        if (j == m) w = (uint64_t)x[2 * j] | ((uint64_t)x[2 * j + 1] << 32);
    return w;
}

// Words 2m and 2m + 1 (one block).
struct WordPair {
    uint64_t w0, w1;
};
[[maybe_unused]] __device__ __noinline__ WordPair chacha_pair_at(uint64_t m, StreamKey key)
{
    uint32_t x[16];
    chacha20_block(key, m / (kWordsPerBlock / 2), x);
    const uint32_t j = (uint32_t)(m % (kWordsPerBlock / 2)); // pair j of the block
    WordPair p{0, 0};
#pragma unroll
    for (uint32_t q = 0; q < kWordsPerBlock / 2; ++q)
        if (q == j) {
            p.w0 = (uint64_t)x[4 * q] | ((uint64_t)x[4 * q + 1] << 32);
            p.w1 = (uint64_t)x[4 * q + 2] | ((uint64_t)x[4 * q + 3] << 32);
        }
    return p;
}

} // namespace
} // namespace brr
