// Dice streams with ChaCha20 words (Bernstein 2008, counter mode): the slow
// cryptographic generator of the paper's experiments (Sec. 7), where one
// word costs far more than the dice drawn from it, so batching k dice per
// word approaches a k-fold saving. The dice themselves follow Theorem 1 and
// Algorithm 3 exactly as in brr_dice; only the word source differs.
//
// Word c of instance `inst` under `seed`: block c/8 of ChaCha20 with key
// words (lo32 seed, hi32 seed, 0, 0, 0, 0, 0, 0), the 64-bit block counter
// in state words 12-13 and the 64-bit nonce inst in words 14-15; the word is
// output words 2m, 2m+1 (low half first), m = c mod 8. Attempt a of group s
// reads word a*S + s.
//
// Work mapping, as for the Philox stream: a wavefront owns a tile of 64 x 8
// groups and lane L takes groups g0 + 64j + L (j < 8), so that every load
// and store instruction covers one contiguous span. The eight lanes of an
// octet hold eight consecutive groups per j, which share one ChaCha block:
// lane q of the octet computes the block of slot j = q, and an 8 x 8
// transpose in registers (three exchange stages, partners q ^ 1, q ^ 2,
// q ^ 4) hands every lane its word of all eight blocks.
//
// Rerolls. A reroll costs one block for one word, and the lanes of a
// wavefront compute in lockstep, so a wave that rerolls its own few
// rejected groups pays a full block per pass for each of them while most of
// its lanes idle (and as many passes as its unluckiest group needs). So the
// first pass records each tile's rejected groups (up to kTileSlots of them)
// in device memory, and a second kernel of persistent waves works through
// them with every lane busy: each wave owns a run of tiles, a lane takes
// the next recorded group as soon as its current one is accepted, and keeps
// rerolling a group until it is; when the run is drained, idle lanes try
// the remaining groups' next attempts side by side. A tile with more
// rejected groups rerolls them in place, one block per lane and pass for
// the lane's lowest rejected group (as does every tile when the memory
// cannot be had). Pooling the rerolls of a block's four tiles in LDS inside
// the first kernel instead was slower: a pool of about 64 groups per block
// still pays its tail passes, 16 times as many tails as the persistent
// waves have.
#include <algorithm>

#include "chacha.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace brr {

namespace {

constexpr uint64_t kMaxAttemptsChaCha = 1024;

// Value of lane L ^ D (D = 1, 2: quad DPP; D = 4: through the LDS crossbar).
template <int D> __device__ __forceinline__ uint32_t from_lane_xor(uint32_t v)
{
    if (D == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    if (D == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    return (uint32_t)__shfl_xor((int)v, D, 64);
}

// One exchange stage of the octet transpose: for each index pair (i, i + D)
// (bit D of i clear), a lane keeps the element whose index bit D equals its
// lane bit D and swaps the other with lane L ^ D.
template <int D> __device__ __forceinline__ void exchange(uint32_t (&lo)[8], uint32_t (&hi)[8],
                                                          bool bit)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (i & D) continue;
        const uint32_t rlo = from_lane_xor<D>(bit ? lo[i] : lo[i + D]);
        const uint32_t rhi = from_lane_xor<D>(bit ? hi[i] : hi[i + D]);
        if (bit) {
            lo[i] = rlo;
            hi[i] = rhi;
        } else {
            lo[i + D] = rlo;
            hi[i + D] = rhi;
        }
    }
}

// First-attempt words of this lane's groups g0 + 64j + lane, j = 0..7.
__device__ __forceinline__ void tile_words_chacha(uint64_t g0, uint32_t lane, const StreamKey &key,
                                                  uint64_t (&r)[8])
{
    const uint32_t q = lane & 7, o = lane >> 3;
    // block of slot j = q for groups g0 + 64q + 8o + m, m = 0..7
    uint32_t x[16];
    chacha20_block(key, g0 / kWordsPerBlock + 8 * q + o, x);
    uint32_t lo[8], hi[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        lo[m] = x[2 * m];
        hi[m] = x[2 * m + 1];
    }
    exchange<1>(lo, hi, lane & 1);
    exchange<2>(lo, hi, lane & 2);
    exchange<4>(lo, hi, lane & 4);
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = (uint64_t)lo[j] | ((uint64_t)hi[j] << 32);
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

// The chain on word r for one group: dice into a, returns the leftover.
// A short group's bounds are padded with 1 past its dice: a bound of 1
// rolls a 0 and leaves the leftover and the product as they are, so the
// chain and the product run over all K without a branch per die.
template <int K>
__device__ __forceinline__ uint64_t chain(const uint32_t *b, uint32_t *a, uint64_t r)
{
#pragma unroll
    for (int i = 0; i < K; ++i) a[i] = mul_roll(b[i], r);
    return r;
}

// Lemire's threshold of the group's product, or 0 when the leftover rr
// already accepts (r >= P > t, or P = 2^64); flags bad groups in err.
template <int K>
__device__ __forceinline__ uint64_t group_threshold(const uint32_t *b, uint64_t rr,
                                                    uint32_t &err)
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
    if (P.e64 || rr >= P.p) return 0;
    return pow2_64_mod(P.p);
}

// The group's product when its threshold decides (the leftover rr is below
// it), else 0: accepted at once (r >= P > t, or P = 2^64), or a bad group,
// flagged in err (its dice are stored as they are).
template <int K>
__device__ __forceinline__ uint64_t undecided_product(const uint32_t *b, uint64_t rr,
                                                      uint32_t &err)
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
    return (P.e64 || rr >= P.p) ? 0 : P.p; // P >= 1 here
}

// Dice count of group g (K, the short last group's count, or 0 past it).
template <int K>
__device__ __forceinline__ int group_dice(uint64_t g, uint64_t full, uint64_t S, uint64_t count)
{
    return (g < full) ? K : (g < S ? (int)(count - (uint64_t)K * g) : 0);
}

template <int K, bool VEC>
__device__ __forceinline__ void load_bounds(const uint32_t *__restrict__ bounds, uint64_t g, int kk,
                                            bool whole, uint32_t *b)
{
    if (whole) {
        load_group<K, VEC>(bounds + (uint64_t)K * g, b);
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) b[i] = (i < kk) ? bounds[(uint64_t)K * g + i] : 1u;
    }
}

template <int K, bool VEC>
__device__ __forceinline__ void store_dice(uint32_t *__restrict__ out, uint64_t g, int kk,
                                           bool whole, const uint32_t *a)
{
    if (whole) {
        store_group<K, VEC>(out + (uint64_t)K * g, a);
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < kk) out[(uint64_t)K * g + i] = a[i];
    }
}

// Registers: the eight words (16) stay live from the transpose to the last
// group; each group's bounds are loaded after the rounds, when it is rolled
// (holding all 8K bounds through the rounds cost more in resident
// wavefronts than it saved in latency: k = 2 took 0.76 ms that way, 0.57 ms
// this way). A rejected group is left for the reroll passes, which reload
// its bounds.
// Rejected groups of the first pass, per tile of 512 groups: count[t] and
// their offsets in the tile, slot[t * kTileSlots + i] (t counts tiles from
// the start of the stream). tiles = 0: no record, every tile rerolls in
// place.
constexpr uint32_t kTileSlots = 32;
constexpr uint32_t kUndecided = 64;
constexpr uint64_t kNoGroup = ~0ull;
// The offsets follow the counts, from the next multiple of 16 bytes.
__host__ __device__ constexpr uint64_t slot_offset(uint64_t tiles)
{
    return (4 * tiles + 15) & ~15ull;
}
struct RerollRecord {
    uint32_t *count;
    uint16_t *slot;
    uint64_t tiles;
};

// Attempt `attempt` of group g (word attempt * S + g): its dice into a;
// true if accepted, or at the attempt cap, which only bounds the loop
// against corrupted inputs (each attempt is rejected with probability
// t / 2^64 < 1/2).
template <int K>
__device__ __forceinline__ bool try_attempt(const uint32_t *b, uint64_t g,
                                            uint64_t attempt, uint64_t S, const StreamKey &key,
                                            uint32_t *a)
{
    const uint64_t rr = chain<K>(b, a, chacha_word_at(attempt * S + g, key));
    uint32_t e = 0; // bad groups were flagged by their first attempt
    return rr >= group_threshold<K>(b, rr, e) || attempt >= kMaxAttemptsChaCha;
}

template <int K>
__device__ __forceinline__ void load_group_bounds(const uint32_t *__restrict__ bounds, uint64_t g,
                                                  int kk, uint32_t *b)
{
#pragma unroll
    for (int i = 0; i < K; ++i) b[i] = (i < kk) ? bounds[(uint64_t)K * g + i] : 1u;
}

template <int K>
__device__ __forceinline__ void store_group_dice(uint32_t *__restrict__ out, uint64_t g, int kk,
                                                 const uint32_t *a)
{
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i < kk) out[(uint64_t)K * g + i] = a[i];
}

template <int K, bool VEC>
__global__ __launch_bounds__(256) void dice_chacha_kernel(const uint32_t *__restrict__ bounds,
                                                          uint32_t *__restrict__ out,
                                                          uint64_t count, uint64_t S,
                                                          uint64_t full, StreamKey key,
                                                          uint32_t *status, RerollRecord rec)
{
    constexpr int G = 8; // groups per lane
    // Groups whose threshold decides (rr < P: one in 16 at k = 4 with
    // 16-bit bounds) are not decided in the loop, where nearly every j
    // would have a lane on that path and the whole wave would run it:
    // their product and leftover are set aside (up to kUndecided per wave)
    // and decided after the loop, one group per lane, in one pass.
    __shared__ uint64_t und_p[4][kUndecided], und_r[4][kUndecided];
    __shared__ uint16_t und_at[4][kUndecided]; // 64 j + lane
    __shared__ uint32_t rejected[4][64];      // bit j: group 64 j + lane rejected
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt_mask = (1ull << lane) - 1;
    const uint64_t g0 = (((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * (64 * G);
    if (g0 >= S) return; // the whole wavefront leaves together
    const bool whole = g0 + 64 * G <= full; // every group of the tile has K dice
    rejected[w][lane] = 0;
    uint64_t r[G];
    tile_words_chacha(g0, lane, key, r);
    uint32_t err = 0, pending = 0, nu = 0; // nu: set aside (uniform)
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const uint64_t g = g0 + 64 * j + lane;
        const int kk = whole ? K : group_dice<K>(g, full, S, count);
        uint64_t ps = 0, rr = 0;
        uint32_t a[K];
        if (kk > 0) {
            uint32_t b[K];
            load_bounds<K, VEC>(bounds, g, kk, whole, b);
            rr = chain<K>(b, a, r[j]);
            ps = undecided_product<K>(b, rr, err);
        }
        const uint64_t um = __ballot(ps != 0);
        const uint32_t at = nu + (uint32_t)__builtin_popcountll(um & lt_mask);
        nu += (uint32_t)__builtin_popcountll(um);
        bool keep = kk > 0;
        if (ps != 0) {
            if (at < kUndecided) { // its dice are stored, and rewritten if it rerolls
                und_p[w][at] = ps;
                und_r[w][at] = rr;
                und_at[w][at] = (uint16_t)(64 * j + lane);
            } else if (rr < pow2_64_mod(ps)) {
                pending |= 1u << j;
                keep = false;
            }
        }
        if (keep) store_dice<K, VEC>(out, g, kk, whole, a);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < std::min(nu, kUndecided) && und_r[w][lane] < pow2_64_mod(und_p[w][lane])) {
        const uint32_t at = und_at[w][lane];
        atomicOr(&rejected[w][at & 63], 1u << (at >> 6));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    pending |= rejected[w][lane];
    // record the rejected groups for the reroll kernel, if they fit
    if (rec.tiles) {
        const uint64_t t = g0 / (64 * 8);
        const uint32_t mine = __builtin_popcount(pending);
        const uint32_t incl = wave_inclusive_scan(mine);
        const uint32_t total = __shfl(incl, 63, 64);
        if (total <= kTileSlots) {
            uint32_t slot = incl - mine;
            for (uint32_t p = pending; p; p &= p - 1, ++slot)
                rec.slot[t * kTileSlots + slot] = (uint16_t)(64 * __builtin_ctz(p) + lane);
            pending = 0;
        }
        if (lane == 0) rec.count[t] = total <= kTileSlots ? total : 0;
    }
    // rerolls in place (more than kTileSlots rejected), compacted: a lane
    // works on its lowest pending group
    uint64_t attempt = 1;
    while (__any(pending != 0)) {
        if (pending) {
            const int m = __builtin_ctz(pending);
            const uint64_t g = g0 + 64 * (uint64_t)m + lane;
            const int kk = group_dice<K>(g, full, S, count);
            uint32_t b[K], a[K];
            load_group_bounds<K>(bounds, g, kk, b);
            if (try_attempt<K>(b, g, attempt, S, key, a)) {
                store_group_dice<K>(out, g, kk, a);
                pending &= pending - 1;
                attempt = 1;
            } else {
                ++attempt;
            }
        }
    }
    if (err) atomicOr(status, err);
}

// Works through the recorded rejected groups: wave w owns the tiles
// [w * per, (w + 1) * per), taken in chunks of up to 64 tiles (one count
// per lane). A chunk's records are first gathered into a list in the
// wave's LDS (the tile's counts scanned across the wave give each tile its
// place in the list), so taking a group is one LDS read and the only
// global reads left in the loop are the groups' bounds. A lane holding a
// group tries its next attempt; idle lanes take the next listed groups. A
// group is rerolled until accepted (or at the attempt cap), and its first
// accepted word is the one that counts. Once the wave's list is drained and
// at most half its lanes hold a group, the idle lanes try those groups'
// next attempts side by side (spread passes), so that a group rejected
// again and again does not keep the wave running one pass per attempt with
// its other lanes idle.
constexpr uint32_t kRerollChunk = 64;
template <int K>
__global__ __launch_bounds__(256) void dice_chacha_rerolls(const uint32_t *__restrict__ bounds,
                                                           uint32_t *__restrict__ out,
                                                           uint64_t count, uint64_t S,
                                                           uint64_t full, StreamKey key,
                                                           RerollRecord rec, uint64_t per)
{
    // entry (tile in chunk << 9) | group offset in the tile
    __shared__ uint16_t lists[4][kRerollChunk * kTileSlots];
    __shared__ uint8_t holders[4][64]; // lanes of the active groups, in order (spread passes)
    uint16_t *list = lists[threadIdx.x >> 6];
    uint8_t *holder = holders[threadIdx.x >> 6];
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t lt_mask = (1ull << lane) - 1;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t t_begin = std::min<uint64_t>(wave * per, rec.tiles);
    const uint64_t t_end = std::min<uint64_t>(t_begin + per, rec.tiles);
    uint64_t t0 = t_begin, chunk = t_begin; // next chunk, chunk in the list
    uint32_t n = 0, next = 0;               // listed, taken (uniform)
    uint64_t g = kNoGroup;
    uint32_t attempt = 1, b[K];
    while (true) {
        if (next == n && t0 < t_end) {
            const uint32_t nt = (uint32_t)std::min<uint64_t>(kRerollChunk, t_end - t0);
            const uint32_t c = lane < nt ? rec.count[t0 + lane] : 0;
            const uint32_t incl = wave_inclusive_scan(c);
            // 16 bytes (eight offsets) per lane and pass, four per tile
            for (uint32_t e0 = 0; e0 < 4 * nt; e0 += 64) {
                const uint32_t e = e0 + lane, tile = e >> 2, base = (e & 3) * 8;
                const uint32_t tc = (uint32_t)__shfl((int)c, (int)(tile & 63), 64);
                const uint32_t tx = (uint32_t)__shfl((int)incl, (int)(tile & 63), 64) - tc;
                if (tile < nt && base < tc) {
                    const u32x4 v = *reinterpret_cast<const u32x4 *>(
                        rec.slot + (t0 + tile) * kTileSlots + base);
                    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (base + j < tc)
                            list[tx + base + j] =
                                (uint16_t)((tile << 9) | ((w[j >> 1] >> (16 * (j & 1))) & 0xFFFF));
                }
            }
            n = (uint32_t)__shfl((int)incl, 63, 64);
            next = 0;
            chunk = t0;
            t0 += nt;
            // the list's writes land before any lane of the wave reads it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // idle lanes take the next listed groups
        const uint64_t idle = __ballot(g == kNoGroup);
        const uint32_t take = std::min<uint32_t>((uint32_t)__builtin_popcountll(idle), n - next);
        const uint32_t rank = (uint32_t)__builtin_popcountll(idle & lt_mask);
        if (g == kNoGroup && rank < take) {
            const uint32_t e = list[next + rank];
            g = (chunk + (e >> 9)) * (64 * 8) + (e & 511);
            attempt = 1;
            load_group_bounds<K>(bounds, g, group_dice<K>(g, full, S, count), b);
        }
        next += take;
        const bool drained = t0 >= t_end && next == n;
        const uint64_t act = __ballot(g != kNoGroup);
        if (!act) {
            if (drained) break;
            continue;
        }
        const uint32_t c = (uint32_t)__builtin_popcountll(act);
        if (!drained || 2 * c > 64) {
            if (g != kNoGroup) {
                const int kk = group_dice<K>(g, full, S, count);
                uint32_t a[K];
                if (try_attempt<K>(b, g, attempt, S, key, a)) {
                    store_group_dice<K>(out, g, kk, a);
                    g = kNoGroup;
                } else {
                    ++attempt;
                }
            }
            continue;
        }
        // Spread pass (the list drained, at most half the lanes busy): the
        // q-th active group, in lane order, gets the m = 64 / c lanes
        // [q m, q m + m) for its attempts attempt .. attempt + m - 1; the
        // lowest accepted of them is the one a lane trying them in order
        // would have taken.
        const uint32_t m = 64 / c;
        if (g != kNoGroup) holder[__builtin_popcountll(act & lt_mask)] = (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t q = lane / m;
        const bool mine = q < c;
        const int src = holder[mine ? q : 0];
        const uint64_t gs = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(g >> 32), src, 64) << 32) |
                            (uint32_t)__shfl((int)(uint32_t)g, src, 64);
        const uint32_t as = (uint32_t)__shfl((int)attempt, src, 64) + lane % m;
        uint32_t bs[K];
#pragma unroll
        for (int i = 0; i < K; ++i) bs[i] = (uint32_t)__shfl((int)b[i], src, 64);
        bool acc = false;
        int kk = 0;
        uint32_t a[K];
        if (mine) {
            kk = group_dice<K>(gs, full, S, count);
            acc = try_attempt<K>(bs, gs, as, S, key, a);
        }
        const uint64_t seg = mine ? (~0ull >> (64 - m)) << (q * m) : 0ull;
        const uint64_t hits = __ballot(acc) & seg;
        g = kNoGroup;
        if (hits) {
            if (lane == (uint32_t)__builtin_ctzll(hits)) store_group_dice<K>(out, gs, kk, a);
        } else if (mine && lane == q * m) { // none accepted: on from attempt as + m
            g = gs;
            attempt = as + m;
#pragma unroll
            for (int i = 0; i < K; ++i) b[i] = bs[i];
        }
    }
}

template <int K>
hipError_t launch_dice_chacha_k(const uint32_t *bounds, uint32_t *out, uint64_t count,
                                StreamKey key, uint32_t *status, void *mem, hipStream_t stream)
{
    const uint64_t S = (count + K - 1) / K;
    const uint64_t full = count / K;
    const uint64_t waves = (S + 64 * 8 - 1) / (64 * 8); // 8 groups per lane
    const uint64_t blocks = (waves + 3) / 4;           // 4 wavefronts per block
    if (blocks > 0xFFFFFFFFull) return hipErrorInvalidValue;
    // the record: a count and kTileSlots offsets per tile (68 bytes per 512
    // groups, the offsets 16-byte aligned); without memory for it, every
    // tile rerolls in place
    RerollRecord rec{nullptr, nullptr, mem ? waves : 0};
    if (mem) {
        rec.count = static_cast<uint32_t *>(mem);
        rec.slot = reinterpret_cast<uint16_t *>(static_cast<char *>(mem) + slot_offset(waves));
    }
    const bool vec = ((((uintptr_t)bounds) | ((uintptr_t)out)) & 15) == 0;
    if (vec)
        dice_chacha_kernel<K, true><<<(uint32_t)blocks, 256, 0, stream>>>(bounds, out, count, S,
                                                                          full, key, status, rec);
    else
        dice_chacha_kernel<K, false><<<(uint32_t)blocks, 256, 0, stream>>>(bounds, out, count, S,
                                                                           full, key, status, rec);
    if (mem) {
        // persistent waves, four per block (16 per CU), each owning a run of
        // tiles
        const uint64_t rwaves = std::min<uint64_t>(waves, 4096);
        const uint64_t per = (waves + rwaves - 1) / rwaves;
        dice_chacha_rerolls<K><<<(uint32_t)((rwaves + 3) / 4), 256, 0, stream>>>(
            bounds, out, count, S, full, key, rec, per);
    }
    return hipGetLastError();
}

} // namespace

uint64_t chacha_record_bytes(uint64_t count, uint32_t k)
{
    const uint64_t S = (count + k - 1) / k;
    const uint64_t tiles = (S + 64 * 8 - 1) / (64 * 8);
    return slot_offset(tiles) + tiles * 2 * kTileSlots;
}

hipError_t launch_dice_chacha(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                              StreamKey key, uint32_t *status, void *rec, hipStream_t stream)
{
    switch (k) {
    case 1: return launch_dice_chacha_k<1>(bounds, out, count, key, status, rec, stream);
    case 2: return launch_dice_chacha_k<2>(bounds, out, count, key, status, rec, stream);
    case 3: return launch_dice_chacha_k<3>(bounds, out, count, key, status, rec, stream);
    case 4: return launch_dice_chacha_k<4>(bounds, out, count, key, status, rec, stream);
    case 5: return launch_dice_chacha_k<5>(bounds, out, count, key, status, rec, stream);
    case 6: return launch_dice_chacha_k<6>(bounds, out, count, key, status, rec, stream);
    case 7: return launch_dice_chacha_k<7>(bounds, out, count, key, status, rec, stream);
    case 8: return launch_dice_chacha_k<8>(bounds, out, count, key, status, rec, stream);
    default: return hipErrorInvalidValue;
    }
}

} // namespace brr
