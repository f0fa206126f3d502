// Host build of the kernels' integer helpers (device.hpp), checked against
// unsigned __int128 arithmetic: the Theorem 1 link, the bound product with
// its 2^64 / overflow flags, the threshold 2^64 mod B, and Philox known
// answers. Prints "ok" or the first mismatch.
#include <cstdio>
#include <random>

#include "device.hpp"

typedef unsigned __int128 u128;
static const u128 TWO64 = (u128)1 << 64;

static int fail(const char *what, unsigned long long a, unsigned long long b)
{
    std::printf("mismatch in %s: %llu %llu\n", what, a, b);
    return 1;
}

int main()
{
    std::mt19937_64 rng(2408);
    // 2^64 mod B: edges around powers of two and the f64 branch limits
    std::vector<unsigned long long> Bs = {1, 2, 3, 5, 6, 7, 720, 0xFFFFFFFFull};
    for (int e = 31; e <= 63; ++e)
        for (long long d = -3; d <= 3; ++d) Bs.push_back((1ull << e) + (unsigned long long)d);
    // near-divisors of 2^64: 2^64 mod B tiny, where the rounded f64 quotient
    // can fall just below the true quotient
    for (int i = 0; i < 200000; ++i) {
        const unsigned long long q = 4 + (rng() >> (31 + rng() % 30));
        const unsigned long long B0 = 0xFFFFFFFFFFFFFFFFull / q;
        for (long long d = -2; d <= 2; ++d) Bs.push_back(B0 + (unsigned long long)d);
    }
    Bs.push_back(0xFFFFFFFFFFFFFFFFull);
    Bs.push_back(0xFFFFFFFFFFFFFFFEull);
    for (int i = 0; i < 2000000; ++i) {
        const int sh = (int)(rng() % 64);
        unsigned long long B = rng() >> sh;
        if (B == 0) B = 1;
        Bs.push_back(B);
    }
    for (unsigned long long B : Bs) {
        const unsigned long long want = (unsigned long long)(TWO64 % B);
        const unsigned long long got = brr::pow2_64_mod(B);
        if (got != want) return fail("pow2_64_mod", B, got);
    }
    // (a, r) <- b (x) r
    for (int i = 0; i < 2000000; ++i) {
        const uint32_t b = (uint32_t)(rng() >> (rng() % 33));
        uint64_t r = rng();
        const u128 p = (u128)b * r;
        const uint32_t a = brr::mul_roll(b, r);
        if (a != (uint64_t)(p >> 64) || r != (uint64_t)p) return fail("mul_roll", b, a);
    }
    // exact bound products with flags
    for (int i = 0; i < 1000000; ++i) {
        const int k = 1 + (int)(rng() % 8);
        uint32_t b[8];
        for (int j = 0; j < k; ++j) b[j] = (uint32_t)(rng() >> (32 + rng() % 33));
        if (i % 97 == 0) { // products at exactly 2^64
            b[0] = 1u << 31;
            b[1] = 1u << 31;
            b[2] = 4;
            for (int j = 3; j < k; ++j) b[j] = 1;
        }
        brr::BoundProduct P;
        P.init(b[0]);
        for (int j = 1; j < k; ++j) P.mul(b[j]);
        u128 ref = 1;
        bool zero = false, over = false;
        for (int j = 0; j < k; ++j) {
            zero |= b[j] == 0;
            if (!over) {
                ref *= b[j];
                if (ref > TWO64) over = true;
            }
        }
        if (zero) {
            if (!P.zero) return fail("product zero flag", b[0], k);
            continue;
        }
        if (P.zero) return fail("product spurious zero", b[0], k);
        if (over != P.over) return fail("product overflow flag", b[0], k);
        if (!over) {
            if ((ref == TWO64) != P.e64) return fail("product 2^64 flag", b[0], k);
            if (ref < TWO64 && P.p != (uint64_t)ref) return fail("product value", b[0], k);
        }
    }
    // Philox4x32-10 known answers
    const uint4 x = brr::philox4x32_10(0x243f6a88u, 0x85a308d3u, 0x13198a2eu, 0x03707344u,
                                       0xa4093822u, 0x299f31d0u);
    if (x.x != 0xd16cfe09u || x.y != 0x94fdccebu || x.z != 0x5001e420u || x.w != 0x24126ea1u)
        return fail("philox", x.x, x.y);
    const uint4 y = brr::philox4x32_10(0, 0, 0, 0, 0, 0);
    if (y.x != 0x6627e8d5u || y.w != 0x9b00dbd8u) return fail("philox zero", y.x, y.w);
    std::printf("ok\n");
    return 0;
}
