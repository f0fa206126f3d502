/*
 * Plain CPU oracle for batched ranged random integer generation
 * (Brackett-Rozinsky and Lemire, "Batched Ranged Random Integer Generation").
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only callers. The product library shares no
 * source, header or helper with this file and never loads it.
 *
 * Everything here is the slow, direct form of a definition in the paper,
 * written with unsigned __int128 so that every full-width product is exact:
 *   - full-width multiply b (x) r = (x, y), 2^L x + y = b r      (Sec. 1.1)
 *   - Theorem 1 chain + Lemire's criterion on the leftover       (Sec. 4)
 *   - Algorithm 2 (known threshold) and Algorithm 3 (unknown)    (Sec. 5),
 *     at word width 64 and, for dice streams, 32
 *   - Algorithm 4 (batched partial shuffle with carried bound u) (Sec. 6)
 *   - a second word source: ChaCha20 in counter mode (Bernstein 2008), the
 *     slow generator of the paper's experiments; shuffles also take the
 *     32-bit halves of the Philox words (L = 32)
 *   - the division form of batched dice: one roll of the product of the
 *     bounds, digits as successive remainders of quotients  (Sec. 2.1,
 *     and the naive batched shuffle of Appendix A)
 *   - the full-shuffle procedure with batch sizes growing as the
 *     array shrinks, and one last batch at the end              (Sec. 6, 6.1)
 *
 * Where the paper is silent these readings apply (also listed in the design
 * notes of the repository):
 *   - Word source: the paper draws L-bit words from a sequential generator.
 *     Here word c of instance `inst` under `seed` is one 64-bit half of
 *     Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *     key = (lo32 seed, hi32 seed) and counter = (lo32 c/2, hi32 c/2,
 *     lo32 inst, hi32 inst); even c takes x0 | x1<<32, odd c x2 | x3<<32.
 *   - Word addressing: attempt a (0 = first) of batch/group s of an
 *     instance that has S batches/groups uses word c = a*S + s. Without
 *     rejections this is the paper's sequential consumption of words 0..S-1.
 *   - Digit order: b_1 is applied first and a_1 is the most significant
 *     digit; in a shuffle batch at size n the bounds are n, n-1, ..., n-k+1
 *     and the swaps run z[n-1] first.
 *
 * Error codes: 0 ok, 1 invalid argument (e.g. a zero bound),
 * 2 overflow (a bound product above 2^L).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_EOVERFLOW 2

/* ------------------------------------------------------------------ */
/* Word source: Philox4x32-10, from its published description.         */
/* ------------------------------------------------------------------ */

/* One Philox4x32 round: two 32x32->64 products with the round multipliers,
 * the high halves mixed with the other two counter words and the key. */
static void philox_round(uint32_t x[4], const uint32_t key[2])
{
    const uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    const uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    uint32_t y[4];
    y[0] = (uint32_t)(prod_b >> 32) ^ x[1] ^ key[0];
    y[1] = (uint32_t)prod_b;
    y[2] = (uint32_t)(prod_a >> 32) ^ x[3] ^ key[1];
    y[3] = (uint32_t)prod_a;
    memcpy(x, y, sizeof y);
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t key[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* Weyl key schedule between rounds */
            key[0] += 0x9E3779B9u;
            key[1] += 0xBB67AE85u;
        }
        philox_round(x, key);
    }
    memcpy(out, x, sizeof x);
}

uint64_t orc_word(uint64_t seed, uint64_t inst, uint64_t c)
{
    const uint64_t block = c / 2;
    const uint32_t ctr[4] = {(uint32_t)block, (uint32_t)(block >> 32), (uint32_t)inst,
                             (uint32_t)(inst >> 32)};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    if (c % 2 == 0) return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    return (uint64_t)x[2] | ((uint64_t)x[3] << 32);
}

/* ------------------------------------------------------------------ */
/* Second word source: ChaCha in counter mode (Bernstein 2008), the     */
/* paper's slow cryptographic generator                                */
/* ------------------------------------------------------------------ */

static uint32_t rotl32(uint32_t x, unsigned n) { return (x << n) | (x >> (32 - n)); }

/* One quarter round on four state words: add, xor, rotate by 16, 12, 8, 7. */
void orc_chacha_quarter(uint32_t *a, uint32_t *b, uint32_t *c, uint32_t *d)
{
    *a += *b; *d ^= *a; *d = rotl32(*d, 16);
    *c += *d; *b ^= *c; *b = rotl32(*b, 12);
    *a += *b; *d ^= *a; *d = rotl32(*d, 8);
    *c += *d; *b ^= *c; *b = rotl32(*b, 7);
}

/* The block function on a full 16-word input state: `rounds` rounds (an
 * even number; column rounds and diagonal rounds alternate), then the input
 * added word by word. */
void orc_chacha_block(const uint32_t in[16], unsigned rounds, uint32_t out[16])
{
    uint32_t x[16];
    memcpy(x, in, sizeof x);
    for (unsigned r = 0; r < rounds; r += 2) {
        orc_chacha_quarter(&x[0], &x[4], &x[8], &x[12]);
        orc_chacha_quarter(&x[1], &x[5], &x[9], &x[13]);
        orc_chacha_quarter(&x[2], &x[6], &x[10], &x[14]);
        orc_chacha_quarter(&x[3], &x[7], &x[11], &x[15]);
        orc_chacha_quarter(&x[0], &x[5], &x[10], &x[15]);
        orc_chacha_quarter(&x[1], &x[6], &x[11], &x[12]);
        orc_chacha_quarter(&x[2], &x[7], &x[8], &x[13]);
        orc_chacha_quarter(&x[3], &x[4], &x[9], &x[14]);
    }
    for (int i = 0; i < 16; ++i) out[i] = x[i] + in[i];
}

/* Word c of instance `inst` under `seed` from ChaCha20: input state = the
 * four constant words of a 256-bit key ("expand 32-byte k"), key words
 * (lo32 seed, hi32 seed, 0, 0, 0, 0, 0, 0), a 64-bit block counter c/8 in
 * words 12-13 and a 64-bit nonce inst in words 14-15 (the original layout);
 * the word is output words 2m and 2m+1 (low half first), m = c mod 8. */
uint64_t orc_word_chacha(uint64_t seed, uint64_t inst, uint64_t c)
{
    const uint64_t blk = c / 8;
    const unsigned m = (unsigned)(c % 8);
    const uint32_t in[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                             (uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0,
                             (uint32_t)blk, (uint32_t)(blk >> 32), (uint32_t)inst,
                             (uint32_t)(inst >> 32)};
    uint32_t out[16];
    orc_chacha_block(in, 20, out);
    return (uint64_t)out[2 * m] | ((uint64_t)out[2 * m + 1] << 32);
}

/* ------------------------------------------------------------------ */
/* Theorem 1 at word width L (1..64)                                   */
/* ------------------------------------------------------------------ */

/* (a_i, r_i) <- b_i (x) r_{i-1}, i = 1..k: a_i takes the high L bits and
 * r_i the low L bits of the 2L-bit product. Returns r_k. */
uint64_t orc_chain(unsigned L, const uint64_t *b, unsigned k, uint64_t r0, uint64_t *a)
{
    const u128 two_L = (u128)1 << L;
    u128 r = r0;
    for (unsigned i = 0; i < k; ++i) {
        const u128 product = (u128)b[i] * r; /* b < 2^64, r < 2^64: exact */
        a[i] = (uint64_t)(product / two_L);
        r = product % two_L;
    }
    return (uint64_t)r;
}

/* The bound product prod b_i as an exact integer, or an error if a bound is
 * zero or the product exceeds 2^L (Theorem 1 requires prod b_i <= 2^L). */
static int bound_product(unsigned L, const uint64_t *b, unsigned k, u128 *prod)
{
    const u128 two_L = (u128)1 << L;
    u128 p = 1;
    for (unsigned i = 0; i < k; ++i) {
        if (b[i] == 0) return ORC_EINVAL;
        if ((u128)b[i] > two_L) return ORC_EOVERFLOW;
        p *= b[i]; /* both factors <= 2^64 here, so no 128-bit wrap */
        if (p > two_L) return ORC_EOVERFLOW;
    }
    *prod = p;
    return ORC_OK;
}

/* t = 2^L mod prod b_i (Lemire's criterion threshold of the whole batch). */
int orc_threshold(unsigned L, const uint64_t *b, unsigned k, uint64_t *t)
{
    u128 prod;
    const int err = bound_product(L, b, k, &prod);
    if (err) return err;
    *t = (uint64_t)((((u128)1) << L) % prod);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Dice streams: Algorithm 3 per group, groups of k consecutive bounds */
/* ------------------------------------------------------------------ */

static uint64_t ceil_div(uint64_t x, uint64_t y) { return x / y + (x % y != 0); }

/* One group of dice by Algorithm 3: roll, form the exact product, and only
 * when the leftover is below it compute the threshold and reroll. */
static int roll_group_alg3(const uint64_t *b, unsigned k, uint64_t seed, uint64_t inst,
                           uint64_t S, uint64_t s, uint64_t *a)
{
    u128 prod;
    const int err = bound_product(64, b, k, &prod);
    if (err) return err;
    uint64_t attempt = 0;
    uint64_t r = orc_chain(64, b, k, orc_word(seed, inst, attempt * S + s), a);
    if ((u128)r < prod) {
        const uint64_t t = (uint64_t)((((u128)1) << 64) % prod);
        while (r < t) {
            ++attempt;
            r = orc_chain(64, b, k, orc_word(seed, inst, attempt * S + s), a);
        }
    }
    return ORC_OK;
}

/* Algorithm 3 for one group with the ChaCha20 words (orc_word_chacha). */
static int roll_group_chacha(const uint64_t *b, unsigned k, uint64_t seed, uint64_t inst,
                             uint64_t S, uint64_t s, uint64_t *a)
{
    u128 prod;
    const int err = bound_product(64, b, k, &prod);
    if (err) return err;
    uint64_t attempt = 0;
    uint64_t r = orc_chain(64, b, k, orc_word_chacha(seed, inst, s), a);
    if ((u128)r < prod) {
        const uint64_t t = (uint64_t)((((u128)1) << 64) % prod);
        while (r < t) {
            ++attempt;
            r = orc_chain(64, b, k, orc_word_chacha(seed, inst, attempt * S + s), a);
        }
    }
    return ORC_OK;
}

/* The dice stream of orc_dice with ChaCha20 words in place of Philox (same
 * groups, same attempt addressing). */
int orc_dice_chacha(const uint32_t *bounds, uint32_t *out, uint64_t count, unsigned k,
                    uint64_t seed, uint64_t inst)
{
    if (k == 0 || k > 64) return ORC_EINVAL;
    const uint64_t S = ceil_div(count, k);
    int status = ORC_OK;
    for (uint64_t s = 0; s < S; ++s) {
        const uint64_t first = s * k;
        const unsigned kk = (unsigned)((count - first < k) ? count - first : k);
        uint64_t b[64], a[64];
        for (unsigned i = 0; i < kk; ++i) b[i] = bounds[first + i];
        const int err = roll_group_chacha(b, kk, seed, inst, S, s, a);
        if (err) {
            if (!status) status = err;
            continue;
        }
        for (unsigned i = 0; i < kk; ++i) out[first + i] = (uint32_t)a[i];
    }
    return status;
}

/* Group s alone of a ChaCha20-word stream with S groups. */
int orc_dice_chacha_group(const uint32_t *group_bounds, unsigned kk, uint64_t S, uint64_t s,
                          uint64_t seed, uint64_t inst, uint32_t *out)
{
    if (kk == 0 || kk > 64) return ORC_EINVAL;
    uint64_t b[64], a[64];
    for (unsigned i = 0; i < kk; ++i) b[i] = group_bounds[i];
    const int err = roll_group_chacha(b, kk, seed, inst, S, s, a);
    if (err) return err;
    for (unsigned i = 0; i < kk; ++i) out[i] = (uint32_t)a[i];
    return ORC_OK;
}

/* Group g holds bounds[g*k .. g*k+k-1]; the last group keeps count mod k
 * bounds when that is non-zero. out[j] is the die rolled against bounds[j]. */
int orc_dice(const uint32_t *bounds, uint32_t *out, uint64_t count, unsigned k, uint64_t seed,
             uint64_t inst)
{
    if (k == 0 || k > 64) return ORC_EINVAL;
    const uint64_t S = ceil_div(count, k);
    int status = ORC_OK;
    for (uint64_t s = 0; s < S; ++s) {
        const uint64_t first = s * k;
        const unsigned kk = (unsigned)((count - first < k) ? count - first : k);
        uint64_t b[64], a[64];
        for (unsigned i = 0; i < kk; ++i) b[i] = bounds[first + i];
        const int err = roll_group_alg3(b, kk, seed, inst, S, s, a);
        if (err) {
            if (!status) status = err;
            continue;
        }
        for (unsigned i = 0; i < kk; ++i) out[first + i] = (uint32_t)a[i];
    }
    return status;
}

/* Group s alone of a stream with S groups (its kk bounds given): the dice
 * that orc_dice writes for it. Lets a test check single groups of a stream
 * too long to roll on the CPU in full. */
int orc_dice_group(const uint32_t *group_bounds, unsigned kk, uint64_t S, uint64_t s,
                   uint64_t seed, uint64_t inst, uint32_t *out)
{
    if (kk == 0 || kk > 64) return ORC_EINVAL;
    uint64_t b[64], a[64];
    for (unsigned i = 0; i < kk; ++i) b[i] = group_bounds[i];
    const int err = roll_group_alg3(b, kk, seed, inst, S, s, a);
    if (err) return err;
    for (unsigned i = 0; i < kk; ++i) out[i] = (uint32_t)a[i];
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* The division form of batched dice (Sec. 2.1)                        */
/* ------------------------------------------------------------------ */

/* Digits of V in [0, b_1 ... b_k) as successive remainders of quotients:
 * a_1 = V mod b_1, then V <- V div b_1, a_2 = V mod b_2, and so on (the
 * first die is the remainder on dividing by b_1). */
static void division_digits(u128 V, const uint64_t *b, unsigned k, uint64_t *a)
{
    for (unsigned i = 0; i < k; ++i) {
        a[i] = (uint64_t)(V % b[i]);
        V /= b[i];
    }
}

/* Lemire's method (Sec. 2) for one value in [0, prod), prod <= 2^64, on
 * the words of attempts 0, 1, ... of batch s: (V, y) = prod (x) r, accept
 * when y >= 2^64 mod prod, which is only computed once y < prod. */
static u128 lemire_value(u128 prod, uint64_t seed, uint64_t inst, uint64_t S, uint64_t s)
{
    uint64_t attempt = 0;
    u128 x = prod * orc_word(seed, inst, s);
    if ((u128)(uint64_t)x < prod) {
        const u128 t = (((u128)1) << 64) % prod;
        while ((u128)(uint64_t)x < t) {
            ++attempt;
            x = prod * orc_word(seed, inst, attempt * S + s);
        }
    }
    return x >> 64;
}

/* The dice stream of orc_dice (same groups, same word addressing) with the
 * division form in place of Theorem 1: each group rolls one value below the
 * product of its bounds and splits it into digits. */
int orc_dice_div(const uint32_t *bounds, uint32_t *out, uint64_t count, unsigned k, uint64_t seed,
                 uint64_t inst)
{
    if (k == 0 || k > 64) return ORC_EINVAL;
    const uint64_t S = ceil_div(count, k);
    int status = ORC_OK;
    for (uint64_t s = 0; s < S; ++s) {
        const uint64_t first = s * k;
        const unsigned kk = (unsigned)((count - first < k) ? count - first : k);
        uint64_t b[64], a[64];
        for (unsigned i = 0; i < kk; ++i) b[i] = bounds[first + i];
        u128 prod;
        const int err = bound_product(64, b, kk, &prod);
        if (err) {
            if (!status) status = err;
            continue;
        }
        division_digits(lemire_value(prod, seed, inst, S, s), b, kk, a);
        for (unsigned i = 0; i < kk; ++i) out[first + i] = (uint32_t)a[i];
    }
    return status;
}

/* Group s alone of a division-form stream with S groups. */
int orc_dice_div_group(const uint32_t *group_bounds, unsigned kk, uint64_t S, uint64_t s,
                       uint64_t seed, uint64_t inst, uint32_t *out)
{
    if (kk == 0 || kk > 64) return ORC_EINVAL;
    uint64_t b[64], a[64];
    for (unsigned i = 0; i < kk; ++i) b[i] = group_bounds[i];
    u128 prod;
    const int err = bound_product(64, b, kk, &prod);
    if (err) return err;
    division_digits(lemire_value(prod, seed, inst, S, s), b, kk, a);
    for (unsigned i = 0; i < kk; ++i) out[i] = (uint32_t)a[i];
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Dice streams at word width L = 32                                   */
/* ------------------------------------------------------------------ */

/* Word c of the 32-bit stream: the 32-bit half c mod 2 (low half first) of
 * 64-bit word c/2, i.e. x[c mod 4] of Philox block c/4. */
uint32_t orc_word32(uint64_t seed, uint64_t inst, uint64_t c)
{
    const uint64_t w = orc_word(seed, inst, c / 2);
    return (c % 2 == 0) ? (uint32_t)w : (uint32_t)(w >> 32);
}

/* Algorithm 3 for one group at L = 32: the chain on 32-bit words, the
 * product of the bounds at most 2^32, the threshold 2^32 mod product. Same
 * attempt addressing as at L = 64 (attempt a of group s reads word a*S + s
 * of the 32-bit stream). */
static int roll_group32(const uint64_t *b, unsigned k, uint64_t seed, uint64_t inst, uint64_t S,
                        uint64_t s, uint64_t *a)
{
    u128 prod;
    const int err = bound_product(32, b, k, &prod);
    if (err) return err;
    uint64_t attempt = 0;
    uint64_t r = orc_chain(32, b, k, orc_word32(seed, inst, s), a);
    if ((u128)r < prod) {
        const uint64_t t = (uint64_t)((((u128)1) << 32) % prod);
        while (r < t) {
            ++attempt;
            r = orc_chain(32, b, k, orc_word32(seed, inst, attempt * S + s), a);
        }
    }
    return ORC_OK;
}

/* Group s alone of an L = 32 stream with S groups (its kk bounds given). */
int orc_dice32_group(const uint32_t *group_bounds, unsigned kk, uint64_t S, uint64_t s,
                     uint64_t seed, uint64_t inst, uint32_t *out)
{
    if (kk == 0 || kk > 32) return ORC_EINVAL;
    uint64_t b[32], a[32];
    for (unsigned i = 0; i < kk; ++i) b[i] = group_bounds[i];
    const int err = roll_group32(b, kk, seed, inst, S, s, a);
    if (err) return err;
    for (unsigned i = 0; i < kk; ++i) out[i] = (uint32_t)a[i];
    return ORC_OK;
}

/* The dice stream of orc_dice at L = 32 (groups of k bounds, the last group
 * keeping count mod k). */
int orc_dice32(const uint32_t *bounds, uint32_t *out, uint64_t count, unsigned k, uint64_t seed,
               uint64_t inst)
{
    if (k == 0 || k > 32) return ORC_EINVAL;
    const uint64_t S = ceil_div(count, k);
    int status = ORC_OK;
    for (uint64_t s = 0; s < S; ++s) {
        const uint64_t first = s * k;
        const unsigned kk = (unsigned)((count - first < k) ? count - first : k);
        uint64_t b[32], a[32];
        for (unsigned i = 0; i < kk; ++i) b[i] = bounds[first + i];
        const int err = roll_group32(b, kk, seed, inst, S, s, a);
        if (err) {
            if (!status) status = err;
            continue;
        }
        for (unsigned i = 0; i < kk; ++i) out[first + i] = (uint32_t)a[i];
    }
    return status;
}

/* Sampling with replacement from [0, bound): Algorithm 2, with the threshold
 * of a full group and of the last short group computed once up front. */
int orc_dice_const(uint32_t bound, uint32_t *out, uint64_t count, unsigned k, uint64_t seed,
                   uint64_t inst)
{
    if (k == 0 || k > 64) return ORC_EINVAL;
    if (bound == 0) return count ? ORC_EINVAL : ORC_OK;
    const uint64_t S = ceil_div(count, k);
    uint64_t b[64], a[64];
    for (unsigned i = 0; i < k; ++i) b[i] = bound;
    uint64_t t_full = 0, t_last = 0;
    int err = orc_threshold(64, b, k, &t_full);
    if (err && count >= k) return err;
    const unsigned k_last = (unsigned)(count - (S ? (S - 1) * k : 0));
    if (S) {
        err = orc_threshold(64, b, k_last, &t_last);
        if (err) return err;
    }
    for (uint64_t s = 0; s < S; ++s) {
        const unsigned kk = (s + 1 == S) ? k_last : k;
        const uint64_t t = (s + 1 == S) ? t_last : t_full;
        uint64_t attempt = 0, r;
        do {
            r = orc_chain(64, b, kk, orc_word(seed, inst, attempt * S + s), a);
            ++attempt;
        } while (r < t);
        for (unsigned i = 0; i < kk; ++i) out[s * k + i] = (uint32_t)a[i];
    }
    return ORC_OK;
}

/* Algorithm 2 for a fixed tuple of k bounds known ahead of time: the
 * threshold t = 2^64 mod (b_1 ... b_k) is computed once (and once more for
 * a short last group holding the first count mod k bounds of the tuple);
 * each group repeats the chain on its next word until the leftover is at
 * least t. out[j] is the die rolled against tuple[j mod k]. */
int orc_dice_tuple(const uint32_t *tuple, unsigned k, uint32_t *out, uint64_t count,
                   uint64_t seed, uint64_t inst)
{
    if (k == 0 || k > 64) return ORC_EINVAL;
    uint64_t b[64], a[64];
    for (unsigned i = 0; i < k; ++i) b[i] = tuple[i];
    uint64_t t_full = 0, t_last = 0;
    int err = orc_threshold(64, b, k, &t_full);
    if (err) return err;
    const uint64_t S = ceil_div(count, k);
    const unsigned k_last = (unsigned)(count - (S ? (S - 1) * k : 0));
    if (S) {
        err = orc_threshold(64, b, k_last, &t_last);
        if (err) return err;
    }
    for (uint64_t s = 0; s < S; ++s) {
        const unsigned kk = (s + 1 == S) ? k_last : k;
        const uint64_t t = (s + 1 == S) ? t_last : t_full;
        uint64_t attempt = 0, r;
        do {
            r = orc_chain(64, b, kk, orc_word(seed, inst, attempt * S + s), a);
            ++attempt;
        } while (r < t);
        for (unsigned i = 0; i < kk; ++i) out[s * k + i] = (uint32_t)a[i];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Shuffles: Algorithm 4 batches under a batch-size schedule           */
/* ------------------------------------------------------------------ */

/* A schedule lists segments in order: while the number i of elements still
 * to shuffle exceeds thr[s], roll batches of k[s] dice with the upper bound
 * starting at u[s] (u[s] = 0: the exact falling factorial is the bound).
 * form[s] = 0 takes the dice of a batch from Theorem 1's chain (Alg. 4),
 * form[s] = 1 from the division form of Sec. 2.1 (one value below the
 * falling product by Lemire's method, digits as successive remainders of
 * quotients: the naive batched shuffle of Appendix A; u is not used).
 * If `tail` is set and i > 1 afterwards, one last batch of i-1 dice with
 * bound u_tail finishes the shuffle (Theorem 1 form).
 * words selects the word stream of every batch: 0 = Philox 64-bit words
 * (orc_word), 1 = their 32-bit halves with the chain and the threshold at
 * L = 32 (orc_word32; every product at most 2^32; multiply form only),
 * 2 = ChaCha20 64-bit words (orc_word_chacha). */
typedef struct {
    uint32_t nseg;
    uint32_t tail;
    uint64_t thr[16];
    uint32_t k[16];
    uint64_t u[16];
    uint64_t u_tail;
    uint32_t form[16];
    uint32_t words;
} orc_schedule;

enum { WORDS_PHILOX64 = 0, WORDS_PHILOX32 = 1, WORDS_CHACHA20 = 2 };

/* The paper's schedules: max_k = 6 is shuffle_6 (one die above 2^30
 * elements, then 2/3/4/5/6 dice at or below 2^30/2^19/2^14/2^11/2^9, with
 * bounds 2^60/2^57/2^56/2^55/2^54 and a last batch bounded by 720);
 * max_k = 2 is "at most two dice" with the same tail rule; max_k = 1 is the
 * unbatched shuffle. */
int orc_schedule_paper(int max_k, orc_schedule *out)
{
    memset(out, 0, sizeof *out);
    if (max_k == 1) {
        out->nseg = 1;
        out->thr[0] = 1;
        out->k[0] = 1;
        out->u[0] = 0;
        return ORC_OK;
    }
    if (max_k == 2) {
        out->nseg = 2;
        out->thr[0] = (uint64_t)1 << 30; out->k[0] = 1; out->u[0] = 0;
        out->thr[1] = 2;                 out->k[1] = 2; out->u[1] = (uint64_t)1 << 60;
        out->tail = 1;
        out->u_tail = 720;
        return ORC_OK;
    }
    if (max_k == 6) {
        const uint64_t thr[6] = {(uint64_t)1 << 30, (uint64_t)1 << 19, (uint64_t)1 << 14,
                                 (uint64_t)1 << 11, (uint64_t)1 << 9, 6};
        const uint64_t u[6] = {0, (uint64_t)1 << 60, (uint64_t)1 << 57, (uint64_t)1 << 56,
                               (uint64_t)1 << 55, (uint64_t)1 << 54};
        out->nseg = 6;
        for (int s = 0; s < 6; ++s) {
            out->thr[s] = thr[s];
            out->k[s] = (uint32_t)(s + 1);
            out->u[s] = u[s];
        }
        out->tail = 1;
        out->u_tail = 720;
        return ORC_OK;
    }
    return ORC_EINVAL;
}

/* n^(falling k) = n (n-1) ... (n-k+1), exact; any value above 2^64 is
 * reported as 2^64 + 1 so that the product never wraps. */
static u128 falling(uint64_t n, unsigned k)
{
    const u128 cap = ((u128)1 << 64) + 1;
    u128 p = 1;
    for (unsigned i = 0; i < k; ++i) {
        p *= (u128)(n - i);
        if (p > cap) return cap;
    }
    return p;
}

/* The greedy largest-batch schedule (KMAX): while i elements remain, roll
 * the largest k <= kcap whose batch product i (i-1) ... (i-k+1) fits in one
 * 64-bit word (Theorem 1 needs the product at most 2^64). With N_k the
 * largest n whose k-th falling power is at most 2^64, that is k dice while
 * N_{k+1} < i <= N_k; each segment is guarded by the product at its top,
 * N_k^(falling k). Batches of kcap dice run while more than kcap - 1
 * elements remain and a last batch of i - 1 dice ends the shuffle. Each N_k
 * comes from a bisection on the exact falling power. */
int orc_schedule_kmax(unsigned kcap, orc_schedule *out)
{
    if (kcap < 1 || kcap > 16) return ORC_EINVAL;
    memset(out, 0, sizeof *out);
    const u128 two64 = (u128)1 << 64;
    uint64_t N[18] = {0};
    for (unsigned k = 2; k <= kcap + 1 && k <= 17; ++k) {
        uint64_t lo = k, hi = (uint64_t)1 << 33; /* falling(lo) <= 2^64 < falling(hi) */
        while (hi - lo > 1) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (falling(mid, k) <= two64) lo = mid; else hi = mid;
        }
        N[k] = lo;
    }
    unsigned g = 0;
    for (unsigned k = 1; k <= kcap; ++k) {
        out->k[g] = k;
        out->thr[g] = (k < kcap) ? N[k + 1] : kcap - 1;
        out->u[g] = (k == 1) ? 0 : (uint64_t)falling(N[k], k);
        ++g;
    }
    out->nseg = g;
    out->tail = 1;
    out->u_tail = 0;
    return ORC_OK;
}

typedef struct {
    /* word source: the schedule's stream (words == NULL) or an explicit
     * attempt-major list */
    uint64_t seed, inst;
    const uint64_t *words;
    uint64_t nwords;
    uint64_t S; /* batches in this instance */
    int exhausted;
    unsigned source; /* WORDS_* */
} word_src;

static unsigned word_bits(const word_src *w) { return w->source == WORDS_PHILOX32 ? 32 : 64; }

static uint64_t next_word(word_src *w, uint64_t attempt, uint64_t s)
{
    const uint64_t c = attempt * w->S + s;
    if (w->words) {
        if (c >= w->nwords) {
            w->exhausted = 1;
            return ~(uint64_t)0;
        }
        return w->words[c];
    }
    if (w->source == WORDS_PHILOX32) return orc_word32(w->seed, w->inst, c);
    if (w->source == WORDS_CHACHA20) return orc_word_chacha(w->seed, w->inst, c);
    return orc_word(w->seed, w->inst, c);
}

static void swap_elems(uint8_t *z, uint64_t p, uint64_t q, unsigned eb)
{
    uint8_t tmp[8];
    memcpy(tmp, z + p * eb, eb);
    memcpy(z + p * eb, z + q * eb, eb);
    memcpy(z + q * eb, tmp, eb);
}

/* Algorithm 4 on the first n elements of z with k dice and upper bound u
 * (u = 0: no bound known, use the exact product), as batch s of the
 * instance. Returns the bound for the next batch. */
static u128 partial_shuffle(uint8_t *z, uint64_t n, unsigned k, u128 u, unsigned eb, word_src *w,
                            uint64_t s)
{
    const unsigned L = word_bits(w);
    uint64_t bounds[64], a[64];
    for (unsigned i = 1; i <= k; ++i) bounds[i - 1] = n + 1 - i;
    uint64_t attempt = 0;
    uint64_t r = orc_chain(L, bounds, k, next_word(w, attempt, s), a);
    if (u == 0 || (u128)r < u) {
        u = falling(n, k);
        const uint64_t t = (uint64_t)((((u128)1) << L) % u);
        while (r < t && !w->exhausted) {
            ++attempt;
            r = orc_chain(L, bounds, k, next_word(w, attempt, s), a);
        }
    }
    for (unsigned i = 1; i <= k; ++i) swap_elems(z, a[i - 1], n - i, eb);
    return u;
}

/* Batch s at size n with k dice in the division form: V below the falling
 * product n (n-1) ... (n-k+1) by Lemire's method on the batch's words, the
 * die for bound n - i + 1 the i-th remainder of the successive quotients,
 * and the swaps in the order of Algorithm 4 (z[n-1] first). */
static void partial_shuffle_div(uint8_t *z, uint64_t n, unsigned k, unsigned eb, word_src *w,
                                uint64_t s)
{
    uint64_t bounds[64], a[64];
    for (unsigned i = 1; i <= k; ++i) bounds[i - 1] = n + 1 - i;
    const u128 prod = falling(n, k);
    uint64_t attempt = 0;
    u128 x = prod * next_word(w, attempt, s);
    if ((u128)(uint64_t)x < prod) {
        const u128 t = (((u128)1) << 64) % prod;
        while ((u128)(uint64_t)x < t && !w->exhausted) {
            ++attempt;
            x = prod * next_word(w, attempt, s);
        }
    }
    division_digits(x >> 64, bounds, k, a);
    for (unsigned i = 1; i <= k; ++i) swap_elems(z, a[i - 1], n - i, eb);
}

enum { RUN_COUNT = 0, RUN_CHECK = 1, RUN_EXEC = 2 };

/* Walks the batches of an n-element shuffle that performs `steps`
 * Fisher-Yates steps (steps = n-1 for a full shuffle): counts them,
 * checks each against the requirements of Algorithm 4 (bound product at
 * most 2^64, a non-zero upper bound at least the product it guards), or
 * executes them on z. A batch cut short by `steps` rolls only the dice it
 * needs. Returns the number of batches, or ~0 when a check fails (the
 * reason in *err). */
static uint64_t run_schedule(int mode, uint8_t *z, uint64_t n, uint64_t steps, unsigned eb,
                             const orc_schedule *sch, word_src *w, int *err)
{
    const u128 two64 = (u128)1 << (sch->words == WORDS_PHILOX32 ? 32 : 64); /* 2^L */
    uint64_t i = n, s = 0, done = 0;
    for (uint32_t g = 0; g < sch->nseg && done < steps; ++g) {
        const u128 u0 = sch->u[g];
        u128 u = u0;
        while (i > sch->thr[g] && done < steps) {
            unsigned k = sch->k[g];
            if (steps - done < k) k = (unsigned)(steps - done);
            if (mode == RUN_CHECK) {
                const u128 p = falling(i, k);
                if (p > two64) { *err = ORC_EOVERFLOW; return ~(uint64_t)0; }
                if (u0 && u < p) { *err = ORC_EINVAL; return ~(uint64_t)0; }
            }
            if (mode == RUN_EXEC && sch->form[g] == 1) {
                partial_shuffle_div(z, i, k, eb, w, s);
            } else if (mode == RUN_EXEC) {
                const u128 next_u = partial_shuffle(z, i, k, u, eb, w, s);
                if (u0) u = next_u; /* carry the bound only when one was given */
            }
            ++s;
            i -= k;
            done += k;
        }
    }
    if (sch->tail && i > 1 && done < steps) {
        unsigned k = (unsigned)(i - 1);
        if (steps - done < k) k = (unsigned)(steps - done);
        if (mode == RUN_CHECK) {
            const u128 p = falling(i, k);
            if (p > two64) { *err = ORC_EOVERFLOW; return ~(uint64_t)0; }
            if (sch->u_tail && (u128)sch->u_tail < p) { *err = ORC_EINVAL; return ~(uint64_t)0; }
        }
        if (mode == RUN_EXEC) partial_shuffle(z, i, k, sch->u_tail, eb, w, s);
        ++s;
        done += k;
    }
    if (mode == RUN_CHECK && done < steps) { *err = ORC_EINVAL; return ~(uint64_t)0; }
    return s;
}

/* Structural requirements on a schedule: 1..16 segments, non-increasing
 * thresholds, 1 <= k <= 64, and thr >= k - 1 so that no bound reaches 0. */
static int check_segments(const orc_schedule *sch)
{
    if (sch->nseg == 0 || sch->nseg > 16) return ORC_EINVAL;
    if (sch->words > WORDS_CHACHA20) return ORC_EINVAL;
    for (uint32_t g = 0; g < sch->nseg; ++g) {
        if (sch->k[g] == 0 || sch->k[g] > 64) return ORC_EINVAL;
        if (sch->form[g] > 1) return ORC_EINVAL;
        if (sch->form[g] == 1 && sch->words == WORDS_PHILOX32) return ORC_EINVAL;
        if (sch->thr[g] + 1 < sch->k[g]) return ORC_EINVAL;
        if (g > 0 && sch->thr[g] > sch->thr[g - 1]) return ORC_EINVAL;
    }
    return ORC_OK;
}

uint64_t orc_count_batches(uint64_t n, uint64_t steps, const orc_schedule *sch)
{
    word_src w = {0};
    int err = 0;
    return run_schedule(RUN_COUNT, NULL, n, steps, 8, sch, &w, &err);
}

static int shuffle_impl(void *data, uint64_t n, uint64_t steps, unsigned eb,
                        const orc_schedule *sch, word_src *w)
{
    if (eb != 4 && eb != 8) return ORC_EINVAL;
    if (n <= 1) return ORC_OK;
    if (n > 0xFFFFFFFFull) return ORC_EINVAL;
    int err = check_segments(sch);
    if (err) return err;
    w->source = sch->words;
    if (run_schedule(RUN_CHECK, NULL, n, steps, eb, sch, w, &err) == ~(uint64_t)0) return err;
    w->S = run_schedule(RUN_COUNT, NULL, n, steps, eb, sch, w, &err);
    run_schedule(RUN_EXEC, (uint8_t *)data, n, steps, eb, sch, w, &err);
    return w->exhausted ? ORC_EINVAL : ORC_OK;
}

int orc_shuffle(void *data, uint64_t n, unsigned eb, const orc_schedule *sch, uint64_t seed,
                uint64_t inst)
{
    word_src w = {seed, inst, NULL, 0, 0, 0, 0};
    return shuffle_impl(data, n, n ? n - 1 : 0, eb, sch, &w);
}

/* The same shuffle fed from an explicit attempt-major word list
 * (word c = words[c]); used to pin the method to hand-worked cases. */
int orc_shuffle_words(void *data, uint64_t n, unsigned eb, const orc_schedule *sch,
                      const uint64_t *words, uint64_t nwords)
{
    word_src w = {0, 0, words, nwords, 0, 0, 0};
    return shuffle_impl(data, n, n ? n - 1 : 0, eb, sch, &w);
}

/* Shuffle q of a CSR batch covers elements offsets[q] .. offsets[q+1]-1
 * and uses instance inst_base + q. */
int orc_shuffle_batched(void *data, const uint64_t *offsets, uint64_t count, unsigned eb,
                        const orc_schedule *sch, uint64_t seed, uint64_t inst_base)
{
    int status = ORC_OK;
    for (uint64_t q = 0; q < count; ++q) {
        if (offsets[q + 1] < offsets[q]) return ORC_EINVAL;
        const int err = orc_shuffle((uint8_t *)data + offsets[q] * eb, offsets[q + 1] - offsets[q],
                                    eb, sch, seed, inst_base + q);
        if (err && !status) status = err;
    }
    return status;
}

/* The first m steps of the scheduled shuffle, in place. */
int orc_partial_shuffle(void *data, uint64_t n, uint64_t m, unsigned eb, const orc_schedule *sch,
                        uint64_t seed, uint64_t inst)
{
    if (m > n) return ORC_EINVAL;
    word_src w = {seed, inst, NULL, 0, 0, 0, 0};
    const uint64_t steps = (m < n) ? m : n - 1;
    return shuffle_impl(data, n, steps, eb, sch, &w);
}

/* Sample m of n without replacement: out[t] = z[n-1-t] after the first m
 * steps of the scheduled shuffle of a copy of the input. */
int orc_sample(const void *data, uint64_t n, uint64_t m, unsigned eb, void *out,
               const orc_schedule *sch, uint64_t seed, uint64_t inst)
{
    if (eb != 4 && eb != 8) return ORC_EINVAL;
    if (m > n) return ORC_EINVAL;
    if (m == 0) return ORC_OK;
    uint8_t *z = (uint8_t *)malloc(n * eb);
    if (!z) return ORC_EINVAL;
    memcpy(z, data, n * eb);
    const int err = orc_partial_shuffle(z, n, m, eb, sch, seed, inst);
    if (!err)
        for (uint64_t t = 0; t < m; ++t) memcpy((uint8_t *)out + t * eb, z + (n - 1 - t) * eb, eb);
    free(z);
    return err;
}

/* Number of words (Philox halves) that the first attempts of a dice stream
 * or a shuffle consume: S. Exposed so tests can check word accounting. */
uint64_t orc_dice_groups(uint64_t count, unsigned k) { return k ? ceil_div(count, k) : 0; }

/* ------------------------------------------------------------------ */
/* Group ranges of a dice stream                                       */
/* ------------------------------------------------------------------ */

/* Groups g0 .. g1-1 of the dice stream that the whole-stream function of
 * `kind` rolls over `count` bounds in groups of k (S = ceil(count / k)
 * groups; the last keeps count mod k bounds when that is non-zero); out and
 * bounds are the whole stream's arrays, and only out[g0*k .. min(g1*k,
 * count)-1] is written. kind: 0 Theorem 1 on Philox words (orc_dice),
 * 1 the division form (orc_dice_div), 2 ChaCha20 words (orc_dice_chacha),
 * 3 word width 32 (orc_dice32). Every group is rolled by the same routine
 * the whole-stream function calls, so disjoint ranges can run on separate
 * threads and together write what that function writes. */
int orc_dice_range(unsigned kind, const uint32_t *bounds, uint32_t *out, uint64_t count,
                   unsigned k, uint64_t g0, uint64_t g1, uint64_t seed, uint64_t inst)
{
    if (k == 0 || k > 64 || kind > 3 || (kind == 3 && k > 32)) return ORC_EINVAL;
    const uint64_t S = ceil_div(count, k);
    if (g1 > S) g1 = S;
    int status = ORC_OK;
    for (uint64_t s = g0; s < g1; ++s) {
        const uint64_t first = s * k;
        const unsigned kk = (unsigned)((count - first < k) ? count - first : k);
        uint64_t b[64], a[64];
        for (unsigned i = 0; i < kk; ++i) b[i] = bounds[first + i];
        int err;
        if (kind == 0) {
            err = roll_group_alg3(b, kk, seed, inst, S, s, a);
        } else if (kind == 1) {
            u128 prod;
            err = bound_product(64, b, kk, &prod);
            if (!err) division_digits(lemire_value(prod, seed, inst, S, s), b, kk, a);
        } else if (kind == 2) {
            err = roll_group_chacha(b, kk, seed, inst, S, s, a);
        } else {
            err = roll_group32(b, kk, seed, inst, S, s, a);
        }
        if (err) {
            if (!status) status = err;
            continue;
        }
        for (unsigned i = 0; i < kk; ++i) out[first + i] = (uint32_t)a[i];
    }
    return status;
}
