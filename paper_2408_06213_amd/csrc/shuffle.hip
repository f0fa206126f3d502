// Shuffles and samples: Algorithm 4 batches (Sec. 6) applied in the order of
// Algorithm 1, evaluated in parallel with the exact sequential result.
//
// Dice. Batch s of a shuffle (k dice at size i) reads word s on its first
// attempt and a*S + s on attempt a, rolls the bounds i, i-1, ..., i-k+1
// through the Theorem 1 chain and is accepted when the leftover r satisfies
// r >= 2^64 mod i^(falling k); the schedule's guard u only decides when that
// threshold is formed (r >= u >= product implies acceptance). Die l of the
// batch is j_p for position p = i-1-l: step p swaps z[p] with z[j_p], j_p <= p.
// Every batch is independent, so all dice are rolled at once. A schedule
// may instead read the 32-bit halves of the words (chain and threshold at
// L = 32) or ChaCha20 words, and a step may take its dice in the division
// form of Sec. 2.1 (V below i^(falling k) by Lemire's method, then
// successive remainders); batch_state and next_die cover every case, and
// kernels that carry the other word streams are separate instantiations.
//
// Swaps. Sequential Fisher-Yates runs p = n-1 down to 1. Position p is final
// after its own step, so the value it ends with is what z[j_p] held just
// before step p. Let T(x) = {steps p > x with j_p = x} and V(x) the value at
// x just before step x (for x = 0: at the end). Position x changes only at
// the steps of T(x), each depositing V(p), the last (smallest p) one winning:
//   V(x) = A0[x] if T(x) is empty, else V(min T(x));
//   final z[p] = V(p)                    if p = 0 or j_p = p,
//              = V(next larger element of T(j_p) after p)   if there is one,
//              = A0[j_p]                 otherwise.
// V(x) follows head pointers x -> min T(x) upwards to a position whose T is
// empty. T(x) is built by a counting sort of steps by target (atomic counts,
// exclusive scan, scatter). The result is a source index for every
// position; one gather of the original array finishes the shuffle.
// A sample of m of n runs only the steps p >= n - m and gathers those
// positions into the output (the input is untouched).
#include <cstring>

#include "chacha.hpp"
#include "device.hpp"
#include "internal.hpp"

namespace brr {

namespace {

constexpr uint16_t kNone16 = 0xFFFF;
constexpr uint32_t kNone32 = 0xFFFFFFFFu;
constexpr int kWaveP = 8;        // positions per lane in the wavefront tier
constexpr int kWgThreads = 1024; // workgroup tier and single-workgroup global tier
constexpr int kWgP = 16;         // positions per thread in the workgroup tier
constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanTile = kScanThreads * 16; // entries per block of the device-wide scan
constexpr uint64_t kMaxAttempts = 1024;
constexpr int kTileShift = 8; // 256 indices per tile of the item tables

__device__ __forceinline__ void batch_at(uint32_t s, const Seg *seg, uint32_t nseg, uint32_t &i,
                                         uint32_t &k, uint64_t &u, uint32_t &form)
{
    uint32_t g = 0;
    while (g + 1 < nseg && s >= seg[g + 1].s0) ++g;
    i = seg[g].i0 - (s - seg[g].s0) * seg[g].k;
    k = seg[g].k;
    u = seg[g].u;
    form = seg[g].form;
}

// Word c of a schedule's stream (BRR_WORDS_*); the 32-bit stream's word is
// returned zero-extended.
__device__ uint64_t stream_word(uint32_t src, uint64_t c, const StreamKey &key)
{
    if (src == BRR_WORDS_CHACHA20) return chacha_word_at(c, key);
    if (src == BRR_WORDS_PHILOX32) {
        const uint64_t w = word_at(c >> 1, key);
        return (c & 1) ? (w >> 32) : (uint64_t)(uint32_t)w;
    }
    return word_at(c, key);
}

// Words 2m and 2m + 1 of a schedule's stream (the first attempts of batches
// 2m and 2m + 1): one Philox block, one 64-bit Philox word (its halves), or
// one ChaCha20 block.
__device__ __forceinline__ void first_pair(uint32_t src, uint64_t m, const StreamKey &key,
                                           uint64_t &w0, uint64_t &w1)
{
    if (src == BRR_WORDS_PHILOX64) {
        word_pair(m, key, w0, w1);
    } else if (src == BRR_WORDS_PHILOX32) {
        const uint64_t w = word_at(m, key);
        w0 = (uint32_t)w;
        w1 = w >> 32;
    } else {
        const WordPair p = chacha_pair_at(m, key);
        w0 = p.w0;
        w1 = p.w1;
    }
}

// (a, r) <- b (x) r at L = 32 (r holds a 32-bit word).
__device__ __forceinline__ uint32_t mul_roll32(uint32_t b, uint64_t &r)
{
    const uint64_t x = (uint64_t)b * (uint32_t)r;
    r = (uint32_t)x;
    return (uint32_t)(x >> 32);
}

// The accepted word of batch s (k dice at size i, guard u) whose first
// attempt reads r, at L = 32: the chain on 32-bit words and Lemire's
// threshold 2^32 mod B of the product B <= 2^32 (checked on the host).
__device__ uint64_t accept_word32(uint32_t i, uint32_t k, uint64_t u, uint64_t r, uint32_t S,
                                  uint32_t s, const StreamKey &key)
{
    uint64_t rr = r;
    for (uint32_t l = 0; l < k; ++l) (void)mul_roll32(i - l, rr);
    if (u == 0 || rr < u) {
        uint64_t B = i;
        for (uint32_t l = 1; l < k; ++l) B *= (uint64_t)(i - l);
        const uint64_t t = (1ull << 32) % B;
        // each attempt is rejected with probability t / 2^32 < 1/2; the cap
        // only bounds the loop against corrupted inputs
        for (uint64_t attempt = 1; rr < t && attempt <= kMaxAttempts; ++attempt) {
            r = stream_word(BRR_WORDS_PHILOX32, attempt * S + s, key);
            rr = r;
            for (uint32_t l = 0; l < k; ++l) (void)mul_roll32(i - l, rr);
        }
    }
    return r;
}

// The accepted word of batch s (k dice at size i, guard u) whose first
// attempt reads r, on a 64-bit stream (rerolls read stream src).
__device__ __forceinline__ uint64_t accept_word(uint32_t i, uint32_t k, uint64_t u, uint64_t r,
                                                uint32_t S, uint32_t s, const StreamKey &key,
                                                uint32_t src = BRR_WORDS_PHILOX64)
{
    uint64_t rr = r;
    for (uint32_t l = 0; l < k; ++l) (void)mul_roll(i - l, rr);
    if (u == 0 || rr < u) {
        uint64_t B = i;
        for (uint32_t l = 1; l < k; ++l) B *= (uint64_t)(i - l);
        const uint64_t t = pow2_64_mod(B);
        // each attempt is rejected with probability t / 2^64 < 1/2; the cap
        // only bounds the loop against corrupted inputs
        for (uint64_t attempt = 1; rr < t && attempt <= kMaxAttempts; ++attempt) {
            r = (src == BRR_WORDS_PHILOX64) ? word_at(attempt * S + s, key)
                                            : stream_word(src, attempt * S + s, key);
            rr = r;
            for (uint32_t l = 0; l < k; ++l) (void)mul_roll(i - l, rr);
        }
    }
    return r;
}

// The division form (Sec. 2.1) of batch s: the value V below the exact
// falling product B = i (i-1) ... (i-k+1) (below 2^64: checked on the host)
// by Lemire's method on the batch's words; div_digit then takes its dice.
// Same words as the multiply form: both accept when the low half of B*r is
// at least 2^64 mod B.
__device__ uint64_t accept_div(uint32_t i, uint32_t k, uint64_t w, uint32_t S, uint32_t s,
                               const StreamKey &key, uint32_t src)
{
    uint64_t B = i;
    for (uint32_t l = 1; l < k; ++l) B *= (uint64_t)(i - l);
    uint64_t V = __umul64hi(B, w), y = B * w;
    if (y < B) {
        const uint64_t t = pow2_64_mod(B);
        for (uint64_t attempt = 1; y < t && attempt <= kMaxAttempts; ++attempt) {
            const uint64_t r = stream_word(src, attempt * S + s, key);
            V = __umul64hi(B, r);
            y = B * r;
        }
    }
    return V;
}

// The state a batch's dice are drawn from, given its first word w of stream
// src: the accepted word (multiply form, at L = 32 for the 32-bit stream) or
// the value V (division form).
__device__ __forceinline__ uint64_t batch_state(uint32_t src, uint32_t form, uint32_t i, uint32_t k,
                                                uint64_t u, uint64_t w, uint32_t S, uint32_t s,
                                                const StreamKey &key)
{
    if (src == BRR_WORDS_PHILOX32) return accept_word32(i, k, u, w, S, s, key);
    return form == BRR_FORM_DIVISION ? accept_div(i, k, w, S, s, key, src)
                                     : accept_word(i, k, u, w, S, s, key, src);
}

// The next die of a batch, for bound b = i - l (l = 0, 1, ... in order).
__device__ __forceinline__ uint32_t next_die(uint32_t src, uint32_t form, uint32_t b, uint64_t &r)
{
    if (src == BRR_WORDS_PHILOX32) return mul_roll32(b, r);
    return form == BRR_FORM_DIVISION ? div_digit(b, r) : mul_roll(b, r);
}

// Exclusive prefix sums of a[0..len) in place, offset by base, by the whole
// block; returns the total (without base). Each wavefront owns a contiguous
// run of 64-entry rows and walks it row by row (lane l touches entry 64r + l,
// so LDS accesses are conflict-free and global ones coalesced): a first pass
// sums the run, the runs' sums are scanned across wavefronts, and a second
// pass writes the prefix sums with a running carry. Ends with a barrier.
template <int BLOCK>
__device__ uint32_t block_scan_array(uint32_t *a, uint32_t len, uint32_t base, uint32_t *wsum)
{
    constexpr uint32_t NW = BLOCK / 64;
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t nrows = (len + 63) / 64, R = (nrows + NW - 1) / NW;
    const uint32_t r0 = min(nrows, wid * R), r1 = min(nrows, r0 + R);
    uint32_t sum = 0;
    for (uint32_t r = r0; r < r1; ++r) {
        const uint32_t x = r * 64 + lane;
        sum += (x < len) ? a[x] : 0u;
    }
    sum = __shfl(wave_inclusive_scan(sum), 63, 64);
    if (lane == 0) wsum[wid] = sum;
    __syncthreads();
    uint32_t carry = base, total = 0;
    for (uint32_t w = 0; w < NW; ++w) {
        const uint32_t v = wsum[w];
        carry += (w < wid) ? v : 0u;
        total += v;
    }
    for (uint32_t r = r0; r < r1; ++r) {
        const uint32_t x = r * 64 + lane;
        const uint32_t v = (x < len) ? a[x] : 0u;
        const uint32_t incl = wave_inclusive_scan(v);
        if (x < len) a[x] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    __syncthreads();
    return total;
}


__global__ void k_set_args(RunArgs *dev, RunArgs val)
{
    if (threadIdx.x == 0) *dev = val;
}

// ---------------------------------------------------------------------------
// LDS tier: one block per shuffle, index arrays in LDS, per-position state in
// registers (position p = tid + r*BLOCK, r < P).
// LDS: jb u16[n] (dice, then buckets) | cnt u32[n+1] | head u16[n].
// ---------------------------------------------------------------------------

__host__ __device__ inline uint32_t lds_bytes(uint32_t n)
{
    return ((2u * n + 3u) & ~3u) + 4u * (n + 1u) + ((2u * n + 3u) & ~3u);
}

// W: the schedule may read a stream other than the 64-bit Philox words (a
// separate instantiation, so that the Philox-only kernels carry none of that
// code); the same holds for every kernel below that takes W.
template <typename Elem, int BLOCK, int P, bool W>
__device__ void lds_tier_run(global_t<Elem> *z, uint32_t n, uint32_t steps, uint32_t out_lo,
                             global_t<Elem> *out,
                             const Seg *seg, uint32_t nseg, uint32_t S, uint32_t words,
                             const StreamKey &key, char *smem, uint32_t *wsum)
{
    const uint32_t src = W ? words : BRR_WORDS_PHILOX64;
    const uint32_t tid = threadIdx.x;
    const uint32_t lo = n - steps; // positions lo..n-1 take a step
    uint16_t *jb = reinterpret_cast<uint16_t *>(smem);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(smem + ((2u * n + 3u) & ~3u));
    uint16_t *head = reinterpret_cast<uint16_t *>(cnt + n + 1);

    for (uint32_t x = tid; x <= n; x += BLOCK) cnt[x] = 0;

    // dice: thread takes batch pairs (2m, 2m+1), which share Philox block m
    for (uint32_t m = tid; 2 * m < S; m += BLOCK) {
        uint64_t w[2];
        first_pair(src, m, key, w[0], w[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t s = 2 * m + h;
            if (s < S) {
                uint32_t i, k, f;
                uint64_t u;
                batch_at(s, seg, nseg, i, k, u, f);
                uint64_t r = batch_state(src, f, i, k, u, w[h], S, s, key);
                for (uint32_t l = 0; l < k; ++l)
                    jb[i - 1 - l] = (uint16_t)next_die(src, f, i - l, r);
            }
        }
    }
    __syncthreads();

    uint32_t q[P], slot[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t p = tid + r * BLOCK;
        q[r] = p;
        slot[r] = 0;
        if (p < n && p >= lo) {
            q[r] = jb[p];
            if (q[r] < p) slot[r] = atomicAdd(&cnt[q[r]], 1u);
        }
    }
    __syncthreads();
    block_scan_array<BLOCK>(cnt, n + 1, 0, wsum);

#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t p = tid + r * BLOCK;
        if (p < n && q[r] < p) jb[cnt[q[r]] + slot[r]] = (uint16_t)p;
    }
    __syncthreads();

    uint32_t succ[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t p = tid + r * BLOCK;
        succ[r] = kNone32;
        if (p < n) {
            uint32_t h = kNone16;
            for (uint32_t e = cnt[p], e1 = cnt[p + 1]; e < e1; ++e) h = min(h, (uint32_t)jb[e]);
            head[p] = (uint16_t)h;
            if (q[r] < p) {
                for (uint32_t e = cnt[q[r]], e1 = cnt[q[r] + 1]; e < e1; ++e) {
                    const uint32_t v = jb[e];
                    if (v > p && v < succ[r]) succ[r] = v;
                }
            }
        }
    }
    __syncthreads();

    Elem val[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const uint32_t p = tid + r * BLOCK;
        if (p < n && p >= out_lo) {
            uint32_t src;
            if (p < lo || q[r] == p || succ[r] != kNone32) {
                uint32_t x = (p < lo || q[r] == p) ? p : succ[r];
                for (uint32_t it = 0; it < n && head[x] != kNone16; ++it) x = head[x];
                src = x;
            } else {
                src = q[r];
            }
            val[r] = z[src];
        }
    }
    if (out == nullptr) {
        __syncthreads(); // every gather is done before any position is overwritten
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const uint32_t p = tid + r * BLOCK;
            if (p < n) z[p] = val[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const uint32_t p = tid + r * BLOCK;
            if (p < n && p >= out_lo) out[n - 1 - p] = val[r];
        }
    }
}

// Takes one instance from a device counter on the stream (see DevClaim);
// returns the claimed value to the calling thread.
__device__ __forceinline__ uint64_t take_claim(const DevClaim &c)
{
    const uint64_t v = *c.counter;
    *c.counter = v + 1;
    const uint64_t inst = c.base + v;
    *c.slot = inst;
    return inst;
}

template <typename Elem, int BLOCK, int P, bool W>
__global__ __launch_bounds__(BLOCK) void k_lds_single(Elem *z, uint32_t n, uint32_t steps,
                                                      uint32_t out_lo, Elem *out, SegTable st,
                                                      uint64_t seed, uint64_t inst,
                                                      DevClaim claim)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ Seg seg[kMaxSegs];
    __shared__ uint32_t wsum[BLOCK / 64];
    __shared__ uint64_t claimed;
    if (threadIdx.x < st.nseg) seg[threadIdx.x] = st.seg[threadIdx.x];
    if (threadIdx.x == 0) claimed = claim.counter ? take_claim(claim) : (claim.slot ? *claim.slot : 0);
    __syncthreads();
    const StreamKey key = make_key(seed, inst + claimed);
    lds_tier_run<Elem, BLOCK, P, W>(as_global(z), n, steps, out_lo, as_global(out), seg, st.nseg, st.S,
                                    st.words, key,
                                    smem, wsum);
}

template <typename Elem, int BLOCK, int P, bool W>
__global__ __launch_bounds__(BLOCK) void k_lds_batched(const RunArgs *__restrict__ args, const uint32_t *items,
                                                       DevSched sc)
{
    const RunArgs A = *args;
    global_t<Elem> *data = as_global(static_cast<Elem *>(A.data));
    const global_t<const uint64_t> *offsets = as_global(A.offsets);
    const uint64_t seed = A.seed, inst_base = A.inst;
    extern __shared__ __align__(16) char smem[];
    __shared__ SegTable st;
    __shared__ uint32_t wsum[BLOCK / 64];
    const uint32_t q = items ? items[blockIdx.x] : blockIdx.x;
    const uint64_t off = offsets[q];
    const uint32_t n = (uint32_t)(offsets[q + 1] - off);
    if (n <= 1) return; // the whole block leaves together
    if (threadIdx.x == 0) build_segments(n, n - 1, sc, st);
    __syncthreads();
    lds_tier_run<Elem, BLOCK, P, W>(data + off, n, n - 1, 0, nullptr, st.seg, st.nseg, st.S,
                                    st.words, make_key(seed, inst_base + q), smem, wsum);
}

// Independent requests (shuffles or samples of separate arrays) in one
// launch, one block each, every one with its instance in slots[] (written
// by an earlier kernel on the stream).
template <typename Elem, int BLOCK, int P, bool W>
__global__ __launch_bounds__(BLOCK) void k_lds_requests(ReqBatch b, DevSched sc, uint64_t seed,
                                                        const uint64_t *slots)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ SegTable st;
    __shared__ uint32_t wsum[BLOCK / 64];
    const ReqDesc r = b.r[blockIdx.x];
    if (threadIdx.x == 0) build_segments(r.n, r.steps, sc, st);
    __syncthreads();
    lds_tier_run<Elem, BLOCK, P, W>(as_global(static_cast<Elem *>(r.data)), r.n, r.steps, r.out_lo,
                                    as_global(static_cast<Elem *>(r.out)), st.seg, st.nseg, st.S, st.words,
                                    make_key(seed, slots[r.slot]), smem, wsum);
}

// ---------------------------------------------------------------------------
// Lane tier: small shuffles, one lane each, the sequential batched
// Fisher-Yates of Algorithm 4. A block of kLaneItems lanes owns up to 64
// shuffles (the plan sorts them by size so lanes stay in step). Each lane
// shuffles a byte permutation of its indices in LDS (n <= 256), so the
// payload is not resident while the dice are rolled; the block then moves
// the payload in chunks of whole arrays: the original elements of a chunk
// into an LDS stage, then out[x] = stage[perm[x]] back to HBM.
// ---------------------------------------------------------------------------

constexpr int kLaneItems = 64;           // threads (one wavefront) per block
// Shuffles per block (lanes 0 .. A-1 roll dice, all 64 move data): 64, or
// 32 for the largest arrays, whose dice phase is long enough that two
// blocks per SIMD overlap one's dice with the other's data movement.
constexpr uint32_t kLaneHalfAbove = 192;
__host__ __device__ inline uint32_t lane_arrays(uint32_t max_n)
{
    return max_n > kLaneHalfAbove ? 32u : 64u;
}
constexpr uint32_t kLaneMaxN = 256;      // byte permutations
constexpr uint32_t kLaneStageBytes = 8192;
constexpr int kLaneU = 8;                // loads in flight per lane

__device__ __forceinline__ uint32_t lane_div(uint32_t e, uint32_t n, float rcp)
{
    uint32_t t = (uint32_t)((float)e * rcp); // off by at most one for e < 2^16
    if (t * n > e)
        --t;
    else if (e - t * n >= n)
        ++t;
    return t;
}

// LDS of a lane-tier block whose largest array has max_n elements:
// offs u64[64] | pre u32[65] (+pad) | permutation rows u32[64 * row_words] |
// stage Elem[stage_cap + 16 / eb] (16-byte aligned).
struct LaneLds {
    uint32_t row_words, stage_cap, perm_off, stage_off, bytes;
};

__host__ __device__ inline LaneLds lane_lds(uint32_t max_n, uint32_t eb)
{
    const uint32_t arrays = lane_arrays(max_n);
    LaneLds L;
    L.row_words = ((max_n + 3) / 4) | 1u; // odd: lanes' rows start in distinct banks
    const uint32_t all = arrays * max(max_n, 1u);
    L.stage_cap = min(kLaneStageBytes / eb, all);
    L.perm_off = 8 * kLaneItems + 4 * (kLaneItems + 4);
    L.stage_off = (L.perm_off + 4 * arrays * L.row_words + 15) & ~15u;
    L.bytes = L.stage_off + (L.stage_cap + 16 / eb) * eb;
    return L;
}

// One batch of K dice at i elements left on a lane's byte permutation a:
// the dice come from one pass of the chain, all 2K bytes the batch touches
// are read at once, the K sequential swaps are resolved in registers and
// written back in order (a later write to a position wins, as in the
// sequential algorithm). Position p_l = i-1-l is final after swap l, and a
// later die never reaches it, so the value each swap moves is the original
// byte unless an earlier die of the batch wrote that position.
template <int K>
__device__ __forceinline__ void lane_batch(uint8_t *a, uint32_t i, uint64_t u, uint64_t w,
                                           uint32_t S, uint32_t s, const StreamKey &key)
{
    uint32_t j[K];
    uint64_t r = w;
#pragma unroll
    for (int l = 0; l < K; ++l) j[l] = mul_roll(i - l, r);
    if (u == 0 || r < u) { // not cleared by the guard: exact test, rerolls
        r = accept_word(i, K, u, w, S, s, key);
#pragma unroll
        for (int l = 0; l < K; ++l) j[l] = mul_roll(i - l, r);
    }
    uint8_t vp[K], vj[K];
#pragma unroll
    for (int l = 0; l < K; ++l) {
        vp[l] = a[i - 1 - l];
        vj[l] = a[j[l]];
    }
    uint8_t to_j[K], to_p[K]; // what swap l writes at j_l and at p_l
#pragma unroll
    for (int l = 0; l < K; ++l) {
        uint8_t bp = vp[l], bj = vj[l];
#pragma unroll
        for (int m = 0; m < l; ++m) {
            if (j[m] == i - 1 - (uint32_t)l) bp = to_j[m];
            if (j[m] == j[l]) bj = to_j[m];
        }
        to_j[l] = bp;
        to_p[l] = bj;
    }
#pragma unroll
    for (int l = 0; l < K; ++l) {
        a[i - 1 - l] = to_p[l];
        a[j[l]] = to_j[l];
    }
}

template <int K>
__device__ __forceinline__ void lane_segment(uint8_t *a, const Seg &g, uint32_t S,
                                             const StreamKey &key, uint64_t &w_odd)
{
    for (uint32_t b = 0; b < g.cnt; ++b) {
        const uint32_t s = g.s0 + b, i = g.i0 - b * g.k;
        uint64_t w;
        if ((s & 1) == 0)
            word_pair(s >> 1, key, w, w_odd);
        else
            w = w_odd; // batches run in order: s - 1 made the pair
        lane_batch<K>(a, i, g.u, w, S, s, key);
    }
}

template <typename Elem, bool W>
__global__ __launch_bounds__(kLaneItems) void k_lane_batched(const RunArgs *__restrict__ args,
                                                            const uint32_t *items, uint32_t nitems,
                                                            uint32_t max_n, DevSched sc)
{
    const RunArgs A = *args;
    global_t<Elem> *data = as_global(static_cast<Elem *>(A.data));
    const global_t<const uint64_t> *offsets = as_global(A.offsets);
    const uint64_t seed = A.seed, inst_base = A.inst;
    constexpr uint32_t V = 16 / sizeof(Elem); // elements per 16-byte vector
    const uint32_t src = W ? sc.words : BRR_WORDS_PHILOX64;
    extern __shared__ __align__(16) char smem[];
    const LaneLds L = lane_lds(max_n, sizeof(Elem));
    const uint32_t C = L.stage_cap, RW = L.row_words;
    uint64_t *offs = reinterpret_cast<uint64_t *>(smem);
    uint32_t *pre = reinterpret_cast<uint32_t *>(smem + 8 * kLaneItems);
    uint32_t *permw = reinterpret_cast<uint32_t *>(smem + L.perm_off);
    Elem *stage = reinterpret_cast<Elem *>(smem + L.stage_off);
    const uint8_t *perm_bytes = reinterpret_cast<const uint8_t *>(permw);
    const uint32_t lane = threadIdx.x;
    const uint32_t arrays = lane_arrays(max_n);
    const uint32_t first = blockIdx.x * arrays;
    const uint32_t mine = min<uint32_t>(arrays, nitems - first);
    uint32_t my_n = 0, my_q = 0;
    uint64_t my_off = 0;
    if (lane < mine) {
        my_q = items[first + lane];
        my_off = offsets[my_q];
        my_n = (uint32_t)(offsets[my_q + 1] - my_off);
    }
    pre[lane + 1] = wave_inclusive_scan(my_n);
    if (lane == 0) pre[0] = 0;
    offs[lane] = my_off;
    // equal sizes stored back to back (the usual case after sorting): the
    // block's arrays are one contiguous range
    const uint32_t n0 = __shfl(my_n, 0);
    const uint64_t off0 = __shfl(my_off, 0);
    const bool uniform =
        __all(lane >= mine || (my_n == n0 && my_off == off0 + (uint64_t)lane * n0));

    // Uniform blocks move whole arrays in chunks of at most C elements:
    // 16-byte vectors where they fit, single elements at the two ends, with
    // stage[sh + e] holding chunk element e (sh aligns the vectors in LDS
    // too). A chunk is loaded into registers while the previous one is being
    // written out, the first one while the dice are rolled.
    struct Chunk {
        uint32_t t0, t1, E, head, sh, nv, tail0;
    };
    auto plan_chunk = [&](uint32_t t0) {
        Chunk c;
        c.t0 = t0;
        c.t1 = min(mine, t0 + max(1u, C / max(n0, 1u)));
        c.E = (c.t1 - t0) * n0;
        const uintptr_t a = reinterpret_cast<uintptr_t>(data + off0 + (uint64_t)t0 * n0);
        c.head = min<uint32_t>(c.E, (uint32_t)((16 - (a & 15)) & 15) / sizeof(Elem));
        c.sh = (V - c.head % V) % V;
        c.nv = (c.E - c.head) / V;
        c.tail0 = c.head + c.nv * V;
        return c;
    };
    u32x4 v[kLaneU];
    Elem hv = 0, tv = 0;
    auto issue = [&](const Chunk &c) {
        const global_t<Elem> *src = data + off0 + (uint64_t)c.t0 * n0;
        if (lane < c.head) hv = src[lane];
        if (c.tail0 + lane < c.E) tv = src[c.tail0 + lane];
        const global_t<u32x4> *vs = reinterpret_cast<const global_t<u32x4> *>(src + c.head);
#pragma unroll
        for (int u = 0; u < kLaneU; ++u) {
            const uint32_t i = u * kLaneItems + lane;
            if (i < c.nv) v[u] = __builtin_nontemporal_load(vs + i);
        }
    };
    auto park = [&](const Chunk &c) {
        if (lane < c.head) stage[c.sh + lane] = hv;
        if (c.tail0 + lane < c.E) stage[c.sh + c.tail0 + lane] = tv;
        u32x4 *vstage = reinterpret_cast<u32x4 *>(stage + c.sh + c.head);
#pragma unroll
        for (int u = 0; u < kLaneU; ++u) {
            const uint32_t i = u * kLaneItems + lane;
            if (i < c.nv) vstage[i] = v[u];
        }
    };
    Chunk cur{};
    if (uniform) {
        cur = plan_chunk(0);
        issue(cur);
    }

    if (lane < mine && my_n > 1) {
        uint32_t *row = permw + lane * RW;
        for (uint32_t w = 0; w < (my_n + 3) / 4; ++w) // identity, four bytes a word
            row[w] = (4 * w) * 0x01010101u + 0x03020100u;
        uint8_t *a = reinterpret_cast<uint8_t *>(row);
        const uint32_t n = my_n;
        const StreamKey key = make_key(seed, inst_base + my_q);
        const uint32_t S = walk_segments(n, n - 1, sc, [](const Seg &) {});
        uint64_t w_odd = 0;
        walk_segments(n, n - 1, sc, [&](const Seg &g) {
            // the division form and the other word streams take the general path
            switch ((g.form == BRR_FORM_DIVISION || src != BRR_WORDS_PHILOX64) ? 0u : g.k) {
            case 1: lane_segment<1>(a, g, S, key, w_odd); break;
            case 2: lane_segment<2>(a, g, S, key, w_odd); break;
            case 3: lane_segment<3>(a, g, S, key, w_odd); break;
            case 4: lane_segment<4>(a, g, S, key, w_odd); break;
            case 5: lane_segment<5>(a, g, S, key, w_odd); break;
            case 6: lane_segment<6>(a, g, S, key, w_odd); break;
            case 7: lane_segment<7>(a, g, S, key, w_odd); break;
            case 8: lane_segment<8>(a, g, S, key, w_odd); break;
            default: // larger batches one swap at a time
                for (uint32_t b = 0; b < g.cnt; ++b) {
                    const uint32_t s = g.s0 + b, i = g.i0 - b * g.k;
                    uint64_t w;
                    if ((s & 1) == 0)
                        first_pair(src, s >> 1, key, w, w_odd);
                    else
                        w = w_odd;
                    uint64_t r = batch_state(src, g.form, i, g.k, g.u, w, S, s, key);
                    for (uint32_t l = 0; l < g.k; ++l) {
                        const uint32_t j = next_die(src, g.form, i - l, r), p = i - 1 - l;
                        const uint8_t x = a[p];
                        a[p] = a[j];
                        a[j] = x;
                    }
                }
            }
        });
    }
    __syncthreads();

    if (uniform) {
        const float rcp = 1.0f / (float)max(n0, 1u);
        for (;;) {
            park(cur);
            __syncthreads();
            const bool more = cur.t1 < mine;
            Chunk nxt{};
            if (more) {
                nxt = plan_chunk(cur.t1);
                issue(nxt);
            }
            // chunk element e is x = e mod n0 of local array e / n0
            global_t<Elem> *dst = data + off0 + (uint64_t)cur.t0 * n0;
            auto out = [&](uint32_t e) {
                const uint32_t lt = lane_div(e, n0, rcp), x = e - lt * n0;
                const uint32_t px = perm_bytes[(cur.t0 + lt) * RW * 4 + x];
                return stage[cur.sh + lt * n0 + px];
            };
            if (lane < cur.head) dst[lane] = out(lane);
            if (cur.tail0 + lane < cur.E) dst[cur.tail0 + lane] = out(cur.tail0 + lane);
            global_t<u32x4> *vd = reinterpret_cast<global_t<u32x4> *>(dst + cur.head);
            for (uint32_t i = lane; i < cur.nv; i += kLaneItems) {
                Elem tmp[V];
                // the V elements of one vector usually sit in one array and in
                // one word of its byte permutation: one division, one
                // permutation read for all of them
                const uint32_t e0 = cur.head + i * V;
                const uint32_t lt = lane_div(e0, n0, rcp), x0 = e0 - lt * n0;
                if ((x0 & 3u) + V <= 4 && x0 + V <= n0) {
                    const uint32_t pw = *reinterpret_cast<const uint32_t *>(
                        perm_bytes + (cur.t0 + lt) * RW * 4 + (x0 & ~3u));
                    const Elem *row = stage + cur.sh + lt * n0;
#pragma unroll
                    for (uint32_t j = 0; j < V; ++j) tmp[j] = row[(pw >> (8 * ((x0 & 3u) + j))) & 255u];
                } else {
#pragma unroll
                    for (uint32_t j = 0; j < V; ++j) tmp[j] = out(e0 + j);
                }
                u32x4 w;
                __builtin_memcpy(&w, tmp, 16);
                __builtin_nontemporal_store(w, vd + i);
            }
            __syncthreads();
            if (!more) break;
            cur = nxt;
        }
        return;
    }

    // arrays apart: element by element in chunks of whole arrays, each lane
    // walking the array table forward as its positions grow
    for (uint32_t t0 = 0; t0 < mine;) {
        uint32_t t1 = t0 + 1;
        while (t1 < mine && pre[t1 + 1] - pre[t0] <= C) ++t1;
        const uint32_t E = pre[t1] - pre[t0];
        const uint32_t base = pre[t0];
        uint32_t t = t0;
        for (uint32_t e0 = 0; e0 < E; e0 += kLaneU * kLaneItems) {
            Elem x[kLaneU];
#pragma unroll
            for (int u = 0; u < kLaneU; ++u) {
                const uint32_t e = e0 + u * kLaneItems + lane;
                if (e < E) {
                    while (pre[t + 1] - base <= e) ++t;
                    x[u] = data[offs[t] + (e - (pre[t] - base))];
                }
            }
#pragma unroll
            for (int u = 0; u < kLaneU; ++u) {
                const uint32_t e = e0 + u * kLaneItems + lane;
                if (e < E) stage[e] = x[u];
            }
        }
        __syncthreads();
        t = t0;
        for (uint32_t e = lane; e < E; e += kLaneItems) {
            while (pre[t + 1] - base <= e) ++t;
            const uint32_t lo = pre[t] - base, xi = e - lo;
            const uint32_t px = perm_bytes[t * RW * 4 + xi];
            data[offs[t] + xi] = stage[lo + px];
        }
        __syncthreads();
        t0 = t1;
    }
}

constexpr uint32_t kPeel = 6144;       // positions per peel while the array is in HBM/L2
constexpr uint32_t kPeelHashBits = 13; // 8192 hash chains, load factor <= 0.75
constexpr uint32_t kPeelRes = 4096;    // positions per peel once the array is in LDS
constexpr uint32_t kPeelResHashBits = 13;
constexpr uint32_t kPeelTierMax = 1u << 20;
constexpr int kPeelThreads = 1024;
// One dynamic LDS buffer per workgroup (one workgroup per CU): the peel
// state, or the resident rest of the array followed by the state of the
// smaller peels.
constexpr uint32_t kPeelLdsBytes = 160u * 1024u - 1024u;

__host__ __device__ constexpr uint32_t peel_state_bytes(uint32_t peel, uint32_t hash_bits)
{
    return peel * (4u + 2u + 4u) + (4u << hash_bits); // qof, nxt, root, heads
}
// Positions that stay in LDS together with the state of their peels.
__host__ __device__ constexpr uint32_t peel_resident_max(uint32_t eb)
{
    return (kPeelLdsBytes - peel_state_bytes(kPeelRes, kPeelResHashBits)) / eb / 4u * 4u;
}
static_assert(peel_state_bytes(kPeel, kPeelHashBits) <= kPeelLdsBytes, "peel state exceeds LDS");

template <uint32_t HB>
__device__ __forceinline__ uint32_t peel_hash(uint32_t q)
{
    return (q * 2654435761u) >> (32 - HB);
}

// Peel state. Chain heads and head-chain parents carry the round that wrote
// them in their upper 16 bits, so a round never clears what an earlier one
// left: an entry of another round reads as empty.
//  table[b]: round << 16 | the last local position pushed on chain b
//  root[x]:  round << 16 | (0xFFFF - e), e the smallest step above x that
//            targets x (kept by atomic maximum)
template <uint32_t PEEL, uint32_t HB>
struct PeelLds {
    uint32_t *qof;   // target of the step at local position e (= p - i_end)
    uint32_t *root;
    uint32_t *table;
    uint16_t *nxt;   // next entry of the same hash chain
    __device__ explicit PeelLds(char *base)
    {
        qof = reinterpret_cast<uint32_t *>(base);
        root = qof + PEEL;
        table = root + PEEL;
        nxt = reinterpret_cast<uint16_t *>(table + (1u << HB));
    }
    // every entry empty (rounds count from 1)
    __device__ void clear(int block) const
    {
        for (uint32_t x = threadIdx.x; x < PEEL; x += block) root[x] = 0;
        for (uint32_t x = threadIdx.x; x < (1u << HB); x += block) table[x] = 0;
    }
};

// Bounds of the peel that starts at batch s (i elements left): whole
// batches, at most PEEL positions, a segment at a time.
template <uint32_t PEEL>
__device__ inline void peel_bounds(const SegTable &st, uint32_t s, uint32_t i, uint32_t &s_end,
                                   uint32_t &i_end)
{
    const uint32_t i0 = i;
    uint32_t g = 0;
    while (g + 1 < st.nseg && s >= st.seg[g + 1].s0) ++g;
    for (; g < st.nseg && s < st.S; ++g) {
        const Seg &sg = st.seg[g];
        const uint32_t left = sg.s0 + sg.cnt - s;
        uint32_t nb = (PEEL - (i0 - i)) / sg.k;
        if (nb > left) nb = left;
        s += nb;
        i -= nb * sg.k;
        if (nb < left) break;
    }
    s_end = s;
    i_end = i;
}

// A peel run over z (the array in HBM or in LDS), from batch s_begin at
// i_begin elements left, while batches remain and (until_le) more than
// until_le elements are left; returns with s_begin/i_begin advanced, every
// write done and every thread past a barrier.
//
// Each peel [i_end, i_begin) takes two phases:
//  A: roll its dice; push every moving step on the hash chain of its target
//     and offer it as head-chain parent of its target (if in the peel);
//     meanwhile write the previous peel's results;
//  B: for each step p with target q, the value that ends at p: the value at
//     the end of p's head chain if q = p (x -> smallest step above x that
//     targets x -> ...; the chain's end holds its value unmoved), else the
//     value at the chain end of the next step above p that targets q, else
//     z[q]; a target q below the peel receives, from the smallest step that
//     targets it, the value at that step's chain end.
// A barrier follows each phase; the next peel's phase A writes this one's
// results, which phase B holds in registers.
template <typename Elem, bool W, int BLOCK, uint32_t PEEL, uint32_t HB, typename ZP>
__device__ __forceinline__ void peel_run(ZP z, const PeelLds<PEEL, HB> &L, const SegTable &st,
                                         const StreamKey &key, uint32_t &s_begin, uint32_t &i_begin,
                                         uint32_t until_le, uint32_t (&next)[2][2])
{
    constexpr int P = (PEEL + BLOCK - 1) / BLOCK;
    const uint32_t tid = threadIdx.x;
    const uint32_t src_words = W ? st.words : BRR_WORDS_PHILOX64;
    if (tid == 0) peel_bounds<PEEL>(st, s_begin, i_begin, next[0][0], next[0][1]);
    __syncthreads();
    uint32_t s_end = next[0][0], i_end = next[0][1];
    // results of the previous peel, written in the next phase A
    uint32_t w_lo = 0, w_cnt = 0, ext_mask = 0;
    uint32_t ext_q[P];
    Elem val[P], ext_val[P];
    auto write_back = [&]() {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const uint32_t e = tid + r * BLOCK;
            if (e >= w_cnt) continue;
            z[w_lo + e] = val[r];
            if (ext_mask & (1u << r)) z[ext_q[r]] = ext_val[r];
        }
    };
    for (uint32_t round = 1; s_begin < s_end && i_begin > until_le; ++round) {
        const uint32_t tag = round << 16, H = i_begin - i_end;
        // phase A
        if (tid == 0)
            peel_bounds<PEEL>(st, s_end, i_end, next[round & 1][0], next[round & 1][1]);
        write_back();
        auto roll = [&](uint32_t s, uint64_t w) {
            uint32_t i, k, f;
            uint64_t u;
            batch_at(s, st.seg, st.nseg, i, k, u, f);
            uint64_t r = batch_state(src_words, f, i, k, u, w, st.S, s, key);
            for (uint32_t l = 0; l < k; ++l) {
                const uint32_t q = next_die(src_words, f, i - l, r);
                const uint32_t e = i - 1 - l - i_end;
                L.qof[e] = q;
                if (q == i - 1 - l) continue; // stays
                // push e on the chain of q: compare-and-swap on its head
                uint32_t *head = L.table + peel_hash<HB>(q);
                uint32_t cur = *head, seen;
                do {
                    seen = cur;
                    cur = atomicCAS(head, seen, tag | e);
                } while (cur != seen);
                L.nxt[e] = (seen & 0xFFFF0000u) == tag ? (uint16_t)seen : kNone16;
                if (q >= i_end) atomicMax(&L.root[q - i_end], tag | (0xFFFFu - e));
            }
        };
        if (W && src_words == BRR_WORDS_CHACHA20) {
            // a ChaCha20 block costs as much for one word as for two: a
            // thread takes both batches of a word pair
            for (uint32_t m = s_begin / 2 + tid; 2 * m < s_end; m += BLOCK) {
                uint64_t w[2];
                first_pair(src_words, m, key, w[0], w[1]);
                if (2 * m >= s_begin) roll(2 * m, w[0]);
                if (2 * m + 1 < s_end) roll(2 * m + 1, w[1]);
            }
        } else {
            // one batch per thread (the two batches of a word pair compute
            // its cheap Philox block twice: more threads roll and push at
            // once)
            for (uint32_t s = s_begin + tid; s < s_end; s += BLOCK) {
                uint64_t w[2];
                first_pair(src_words, s / 2, key, w[0], w[1]);
                roll(s, (s & 1u) ? w[1] : w[0]);
            }
        }
        __syncthreads();
        // phase B
        auto chain_end = [&](uint32_t x) {
            for (uint32_t guard = 0; guard < H; ++guard) {
                const uint32_t v = L.root[x];
                if ((v & 0xFFFF0000u) != tag) break;
                x = 0xFFFFu - (v & 0xFFFFu);
            }
            return x;
        };
        ext_mask = 0;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const uint32_t e = tid + r * BLOCK;
            if (e >= H) continue;
            const uint32_t p = i_end + e, q = L.qof[e];
            const uint32_t own = i_end + chain_end(e);
            uint32_t src = own;
            if (q != p) {
                // the chain of q: the smallest step above p that targets q,
                // and whether a step below p targets q
                uint32_t succ = kNone32;
                bool below = false;
                const uint32_t hv = L.table[peel_hash<HB>(q)];
                uint32_t c = (hv & 0xFFFF0000u) == tag ? (hv & 0xFFFFu) : kNone16;
                for (uint32_t guard = 0; c != kNone16 && guard < H; ++guard) {
                    if (L.qof[c] == q) {
                        if (c > e && c < succ) succ = c;
                        below |= c < e;
                    }
                    c = L.nxt[c];
                }
                src = succ == kNone32 ? q : i_end + chain_end(succ);
                if (q < i_end && !below) {
                    ext_mask |= 1u << r;
                    ext_q[r] = q;
                    ext_val[r] = z[own];
                }
            }
            val[r] = z[src];
        }
        w_lo = i_end;
        w_cnt = H;
        __syncthreads();
        s_begin = s_end;
        i_begin = i_end;
        s_end = next[round & 1][0];
        i_end = next[round & 1][1];
    }
    write_back();
    __syncthreads();
}

// Peel tier: one workgroup of kPeelThreads per shuffle (one per CU, it
// takes the whole LDS), positions taken top-down in peels of whole batches.
// While more than peel_resident_max(eb) positions are left, the peels read
// and write the array in HBM/L2, one random gather per position; the rest
// of the array then moves into LDS (one coalesced read), the remaining
// peels run there, and it goes back in one coalesced write. Arrays up to
// that size never leave LDS between load and store.
template <typename Elem, bool W, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_peel_batched(const RunArgs *__restrict__ args,
                                                        const uint32_t *items, DevSched sc)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ SegTable st;
    __shared__ uint32_t next[2][2];
    const RunArgs A = *args;
    global_t<Elem> *data = as_global(static_cast<Elem *>(A.data));
    const global_t<const uint64_t> *offsets = as_global(A.offsets);
    const uint32_t tid = threadIdx.x;
    const uint32_t q_item = items[blockIdx.x];
    const uint64_t off = offsets[q_item];
    const uint32_t n = (uint32_t)(offsets[q_item + 1] - off);
    if (n <= 1) return;
    global_t<Elem> *z = data + off;
    const StreamKey key = make_key(A.seed, A.inst + q_item);
    constexpr uint32_t R = peel_resident_max(sizeof(Elem));
    if (tid == 0) build_segments(n, n - 1, sc, st);
    if (n > R) {
        const PeelLds<kPeel, kPeelHashBits> L(smem);
        L.clear(BLOCK);
    }
    __syncthreads();
    uint32_t s_begin = 0, i_begin = n;
    if (n > R) {
        const PeelLds<kPeel, kPeelHashBits> L(smem);
        peel_run<Elem, W, BLOCK>(z, L, st, key, s_begin, i_begin, R, next);
    }
    if (s_begin >= st.S) return;
    // the rest of the array, positions below i_begin, into LDS (the peels
    // above ended with their writes and a barrier)
    const uint32_t nres = i_begin;
    Elem *zl = reinterpret_cast<Elem *>(smem);
    const PeelLds<kPeelRes, kPeelResHashBits> L(smem + R * sizeof(Elem));
    constexpr int U = 8;
    for (uint32_t x0 = 0; x0 < nres; x0 += U * BLOCK) {
        Elem v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t x = x0 + u * BLOCK + tid;
            if (x < nres) v[u] = z[x];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t x = x0 + u * BLOCK + tid;
            if (x < nres) zl[x] = v[u];
        }
    }
    L.clear(BLOCK);
    __syncthreads();
    peel_run<Elem, W, BLOCK>(zl, L, st, key, s_begin, i_begin, 0, next);
    for (uint32_t x = tid; x < nres; x += BLOCK) z[x] = zl[x];
}

// ---------------------------------------------------------------------------
// Device-wide tier: any number of shuffles/samples ("items") too large for
// LDS, processed together by grid-wide kernels. Item i owns positions
// pos_base[i] .. pos_base[i+1]-1 of the concatenated index arrays and batch
// pairs pair_base[i] .. pair_base[i+1]-1; a step's target as a global index
// is pos_base[i] + j_p.
// Steps are grouped by target in one of two ways:
//  counting (up to kCountMaxPositions, where the counters stay in L2):
//   dice:    jj[x] = j_p; slot[x] = rank of step x among the steps into its
//            target (returning atomic add on cnt[target])
//   scan:    cnt = exclusive prefix of the per-target counts
//   scatter: bucket[cnt[target] + slot[x]] = x
//  sorting (larger problems, where returning atomics on scattered counters
//  cost more than sorting):
//   init:    no target has a step yet; positions that take no step get the
//            sort key "none"
//   dice:    sort key of step x = its global target (steps with j_p = p
//            keep "none"); the value of the key at index x is x, which the
//            first sort pass generates
//   sort:    stable LSD radix sort of (target, step) pairs, 8..10-bit digits;
//            steps into one target end up adjacent and in increasing order
// Then the permutation is resolved forwards, element by element (the
// element first at y, A0[y]):
//   - if steps take y as their target, the first of them in time, the
//     largest p in T(y), swaps A0[y] into p, which is final: dest(y) =
//     max T(y);
//   - else A0[y] is at y when step y runs. If j_y = y (or y takes no step)
//     it stays: dest = y. Else it moves to x = j_y, where the next step
//     into x in time, the largest step of T(x) below y (y's predecessor in
//     T(x)), moves it on to that step's position, which is final; if y is
//     the smallest step into x, nothing moves it until step x, and from x it
//     goes on in the same way.
// So every position z, as a step, gets a move: "stay" (no step or j_z = z),
// "prev q" (q is z's predecessor among the steps into j_z) or "down x"
// (z is the smallest step into x = j_z). The group pass writes these moves
// and every target's largest step; an element goes to its position's
// largest step if it has one, else to the end of the moves followed from
// its position (the walk pass). The "down" moves link positions into disjoint
// paths (a position is the smallest step into at most one target, and at
// most one step is the smallest into it), so every position is passed by
// one walk at most: about half a random read per position. The passes keep
// random reads and random writes apart, and each writes one array at random
// (moves; placed values), since random writes are cheap only while their
// array fits the last-level cache.
//   group:   moves, and each target's largest step (in target order)
//   walk:    the destination of every element that no step targets
//   place:   every element written at its destination
//   copy:    in-place shuffles copy the placed values back
// ---------------------------------------------------------------------------

constexpr uint32_t kSortThreads = 512;
constexpr uint32_t kSortItems = 8;
constexpr uint32_t kSortTile = kSortThreads * kSortItems; // pairs per sort block
static_assert(kSortThreads % 64 == 0 && kSortTile < 65536, "16-bit digit counters");
// A pass sorts on a digit of 8..kSortDigitMax bits: as few passes as the
// key width allows, each digit as narrow as that many passes allow (wider
// digits split a tile into shorter runs, whose writes coalesce worse).
constexpr uint32_t kSortDigitMax = 10;
constexpr uint32_t kSortNone = 0xFFFFFFFFu;               // sorts after every target

constexpr uint64_t kCountMaxPositions = 1ull << 21;

struct GArrays {
    uint32_t *jj;              // counting: j_p of every position (item-local)
    uint32_t *key[2], *val[2]; // sort ping-pong: global target, global step
                               // (counting: slot = key[0], bucket = key[1])
    uint32_t *cnt;             // counting: per-target counts, then offsets
    void *move;                // per position as a step: its move (Move words)
    uint32_t *last;            // per position as a target: largest step into it, or kNone32
    uint32_t *hist;            // per-block digit counts, digit-major, then scanned
    uint32_t *tiles;           // scan partial sums
    void *tmp;                 // placed values of in-place shuffles
};

// Move of an element that arrives at position z (z as a step): the kind in
// the top two bits of a Move word, a global position below them. Problems
// below 2^30 positions use 32-bit words (the array that the group pass
// writes at random then stays within the last-level cache longer), larger
// ones 64-bit words.
template <typename Move> struct MoveBits {
    static constexpr uint32_t kShift = 8 * sizeof(Move) - 2;
    static constexpr Move kDown = 0;                   // on to target j_z (z is its smallest step)
    static constexpr Move kPrev = (Move)1 << kShift;   // to the previous step into j_z: final
    static constexpr Move kStay = (Move)2 << kShift;   // stays at z: final
    static constexpr Move kPos = ((Move)1 << kShift) - 1;
};
constexpr uint64_t kMove32MaxPositions = 1ull << 30;

__host__ __device__ inline uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

__host__ __device__ inline uint64_t scan_tiles(uint64_t len) { return (len + kScanTile - 1) / kScanTile; }

__host__ __device__ inline uint64_t sort_blocks(uint64_t npos)
{
    return (npos + kSortTile - 1) / kSortTile;
}

__host__ __device__ inline uint64_t garrays_bytes(uint64_t npos, uint32_t eb)
{
    const uint64_t w = align256(4 * npos), nh = ((uint64_t)1 << kSortDigitMax) * sort_blocks(npos);
    const uint64_t nt = scan_tiles(nh > npos + 1 ? nh : npos + 1);
    const uint64_t mb = npos < kMove32MaxPositions ? 4 : 8;
    return 6 * w + align256(mb * npos) + align256(4 * (npos + 1)) + align256(4 * nh) +
           align256(4 * nt) + align256(eb * npos);
}

__host__ __device__ inline GArrays garrays(void *base, uint64_t npos)
{
    char *p = static_cast<char *>(base);
    const uint64_t w = align256(4 * npos), nh = ((uint64_t)1 << kSortDigitMax) * sort_blocks(npos);
    GArrays g;
    uint32_t **arr[6] = {&g.jj, &g.key[0], &g.val[0], &g.key[1], &g.val[1], &g.last};
    for (int a = 0; a < 6; ++a) {
        *arr[a] = reinterpret_cast<uint32_t *>(p);
        p += w;
    }
    g.move = p;
    p += align256((npos < kMove32MaxPositions ? 4 : 8) * npos);
    g.cnt = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * (npos + 1));
    g.hist = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * nh);
    g.tiles = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * scan_tiles(nh > npos + 1 ? nh : npos + 1));
    g.tmp = p;
    return g;
}

// Everything the device-wide kernels read about the items. With one item
// the descriptor travels by value (items/segs/bases may then be null).
struct GProblem {
    const GItem *items;
    const SegTable *segs;
    const uint64_t *pos_base;  // nitems + 1
    const uint64_t *pair_base; // nitems + 1
    const uint32_t *pos_tile;  // item of position 256*t, for every tile t
    const uint32_t *pair_tile; // item of batch pair 256*t
    uint32_t nitems;
    uint64_t npos, npairs;
    uint64_t inst_base;       // added to every item's instance
    DevClaim claim;           // if set, the claimed instance is added as well
    const RunArgs *dyn;       // if set, the data, seed and inst_base to use
    GItem one;
    SegTable one_seg;
};

// Seed, instance base and data of a problem: by value, or from the plan's
// device block.
__device__ __forceinline__ uint64_t problem_seed(const GProblem &P, uint64_t seed)
{
    return P.dyn ? P.dyn->seed : seed;
}
__device__ __forceinline__ uint64_t problem_inst_base(const GProblem &P)
{
    return (P.dyn ? P.dyn->inst : P.inst_base) + (P.claim.slot ? *P.claim.slot : 0);
}
template <typename Elem>
__device__ __forceinline__ global_t<Elem> *problem_data(const GProblem &P, Elem *data)
{
    return as_global(P.dyn ? static_cast<Elem *>(P.dyn->data) : data);
}

// Item that owns index x: the tile table names the owner of the tile's
// first index; items that start inside the tile are stepped over (every
// item of this tier is longer than a tile, so at most one step is taken).
__device__ __forceinline__ uint32_t find_item(const uint32_t *tile, const uint64_t *base,
                                              uint32_t nitems, uint64_t x)
{
    uint32_t i = tile[x >> kTileShift];
    while (i + 1 < nitems && base[i + 1] <= x) ++i;
    return i;
}

__device__ __forceinline__ const GItem &item_at(const GProblem &P, uint32_t i)
{
    return P.items ? P.items[i] : P.one;
}

__device__ __forceinline__ const SegTable &segs_at(const GProblem &P, uint32_t i)
{
    return P.segs ? P.segs[i] : P.one_seg;
}

__device__ __forceinline__ uint32_t item_of_pos(const GProblem &P, uint64_t x)
{
    return P.items ? find_item(P.pos_tile, P.pos_base, P.nitems, x) : 0u;
}

// No target has a step into it yet; positions that take no step (below
// n - steps) get their sort pair here, every other one from the dice.
__global__ __launch_bounds__(256) void k_gp_init(GProblem P, GArrays g, uint64_t npos)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && P.claim.counter) (void)take_claim(P.claim);
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (!P.items) { // one item at position 0: 16-byte vectors (last[] is 256-byte aligned)
        const u32x4 none = {kNone32, kNone32, kNone32, kNone32};
        u32x4 *last4 = reinterpret_cast<u32x4 *>(g.last);
        for (uint64_t x = t; x < npos / 4; x += stride) __builtin_nontemporal_store(none, last4 + x);
        for (uint64_t x = npos / 4 * 4 + t; x < npos; x += stride) g.last[x] = kNone32;
        for (uint64_t x = t; x < P.one.n - P.one.steps; x += stride) g.key[0][x] = kSortNone;
        return;
    }
    for (uint64_t x = t; x < npos; x += stride) {
        g.last[x] = kNone32;
        const GItem &it = item_at(P, item_of_pos(P, x));
        if (x - it.pos_base < it.n - it.steps) g.key[0][x] = kSortNone;
    }
}

template <bool W>
__global__ __launch_bounds__(256) void k_gp_dice(GProblem P, GArrays g, uint64_t seed)
{
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < P.npairs;
         w += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = P.items ? find_item(P.pair_tile, P.pair_base, P.nitems, w) : 0u;
        const GItem &it = item_at(P, i);
        const SegTable &st = segs_at(P, i);
        const uint32_t src = W ? st.words : BRR_WORDS_PHILOX64;
        const uint32_t m = (uint32_t)(w - (P.items ? P.pair_base[i] : 0));
        const StreamKey key = make_key(problem_seed(P, seed), problem_inst_base(P) + it.inst);
        uint64_t wd[2];
        first_pair(src, m, key, wd[0], wd[1]);
        uint32_t *sk = g.key[0] + it.pos_base;
        const uint32_t tb = (uint32_t)it.pos_base;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t s = 2 * m + h;
            if (s >= st.S) continue;
            uint32_t i0, k, f;
            uint64_t u;
            batch_at(s, st.seg, st.nseg, i0, k, u, f);
            uint64_t r = batch_state(src, f, i0, k, u, wd[h], st.S, s, key);
            for (uint32_t l = 0; l < k; ++l) {
                const uint32_t p = i0 - 1 - l;
                const uint32_t a = next_die(src, f, i0 - l, r);
                sk[p] = (a < p) ? tb + a : kSortNone;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_gc_init(GProblem P, uint32_t *cnt, uint64_t len)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && P.claim.counter) (void)take_claim(P.claim);
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < len;
         x += (uint64_t)gridDim.x * blockDim.x)
        cnt[x] = 0;
}

constexpr uint32_t kFastK = 6; // batches up to this size keep their dice in registers

template <bool W>
__global__ __launch_bounds__(256) void k_gc_dice(GProblem P, GArrays g, uint64_t seed)
{
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < P.npairs;
         w += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = P.items ? find_item(P.pair_tile, P.pair_base, P.nitems, w) : 0u;
        const GItem &it = item_at(P, i);
        const SegTable &st = segs_at(P, i);
        const uint32_t src = W ? st.words : BRR_WORDS_PHILOX64;
        const uint32_t m = (uint32_t)(w - (P.items ? P.pair_base[i] : 0));
        const StreamKey key = make_key(problem_seed(P, seed), problem_inst_base(P) + it.inst);
        uint64_t wd[2];
        first_pair(src, m, key, wd[0], wd[1]);
        uint32_t i0[2] = {0, 0}, kk[2] = {0, 0}, f[2] = {0, 0};
        uint64_t r[2] = {0, 0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t s = 2 * m + h;
            if (s >= st.S) continue;
            uint64_t u;
            batch_at(s, st.seg, st.nseg, i0[h], kk[h], u, f[h]);
            r[h] = batch_state(src, f[h], i0[h], kk[h], u, wd[h], st.S, s, key);
        }
        uint32_t *jj = g.jj + it.pos_base, *slot = g.key[0] + it.pos_base;
        uint32_t *cnt = g.cnt + it.pos_base;
        if (kk[0] <= kFastK && kk[1] <= kFastK) {
            // every die of the pair first, then all counting atomics in
            // flight together, then their slots
            uint32_t a[2 * kFastK], sl[2 * kFastK];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (uint32_t l = 0; l < kFastK; ++l)
                    if (l < kk[h]) {
                        a[h * kFastK + l] = next_die(src, f[h], i0[h] - l, r[h]);
                        jj[i0[h] - 1 - l] = a[h * kFastK + l];
                    }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (uint32_t l = 0; l < kFastK; ++l)
                    if (l < kk[h] && a[h * kFastK + l] < i0[h] - 1 - l)
                        sl[h * kFastK + l] = atomicAdd(&cnt[a[h * kFastK + l]], 1u);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (uint32_t l = 0; l < kFastK; ++l)
                    if (l < kk[h] && a[h * kFastK + l] < i0[h] - 1 - l)
                        slot[i0[h] - 1 - l] = sl[h * kFastK + l];
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                for (uint32_t l = 0; l < kk[h]; ++l) {
                    const uint32_t p = i0[h] - 1 - l;
                    const uint32_t a = next_die(src, f[h], i0[h] - l, r[h]);
                    jj[p] = a;
                    if (a < p) slot[p] = atomicAdd(&cnt[a], 1u);
                }
        }
    }
}

__global__ __launch_bounds__(256) void k_gc_scatter(GProblem P, GArrays g)
{
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P.npos;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const GItem &it = item_at(P, item_of_pos(P, x));
        const uint32_t p = (uint32_t)(x - it.pos_base);
        if (p < it.n - it.steps) continue;
        const uint32_t q = g.jj[x];
        if (q < p) g.key[1][g.cnt[it.pos_base + q] + g.key[0][x]] = (uint32_t)x;
    }
}

// Writes an element's final value: into the placement buffer of an in-place
// shuffle, or, for a sample, into its output if the destination is one of
// the positions sampled.
template <typename Elem>
__device__ __forceinline__ void place(const GItem &it, Elem *tmp, uint64_t dest, Elem v)
{
    if (it.out) {
        const uint32_t p = (uint32_t)(dest - it.pos_base);
        if (p >= it.out_lo) static_cast<Elem *>(it.out)[it.n - 1 - p] = v;
    } else {
        tmp[dest] = v;
    }
}

// Counting form of the group pass. Position x as a step that stays (no step,
// or j_p = p) gets "stay"; as a target with steps into it (its bucket,
// unordered): the smallest step moves down to x, every other one to its
// predecessor in the bucket, and the largest is recorded as x's last step.
template <typename Move>
__global__ __launch_bounds__(256) void k_gc_group(GProblem P, GArrays g)
{
    using MB = MoveBits<Move>;
    const uint32_t *bucket = g.key[1];
    Move *move = static_cast<Move *>(g.move);
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P.npos;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const GItem &it = item_at(P, item_of_pos(P, x));
        const uint32_t p = (uint32_t)(x - it.pos_base);
        if (p < it.n - it.steps || g.jj[x] == p) move[x] = MB::kStay;
        const uint32_t b0 = g.cnt[x], b1 = g.cnt[x + 1];
        uint32_t lo = kNone32, hi = kNone32;
        if (b1 > b0) {
            hi = 0;
            for (uint32_t e = b0; e < b1; ++e) {
                const uint32_t t = bucket[e];
                lo = min(lo, t);
                hi = max(hi, t);
            }
        }
        g.last[x] = hi;
        for (uint32_t e = b0; e < b1; ++e) {
            const uint32_t t = bucket[e];
            if (t == lo) {
                move[t] = MB::kDown | (Move)x;
                continue;
            }
            uint32_t pred = lo;
            for (uint32_t f = b0; f < b1; ++f) {
                const uint32_t u = bucket[f];
                if (u < t && u > pred) pred = u;
            }
            move[t] = MB::kPrev | (Move)pred;
        }
    }
}

// Exclusive scan of one u64 per thread over a block of kSortThreads, in
// thread order; *total receives the block's sum. Ends with a barrier.
__device__ __forceinline__ uint64_t sort_block_scan(uint64_t v, uint64_t *wsum, uint64_t &total)
{
    constexpr uint32_t NW = kSortThreads / 64;
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += o;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (uint32_t w = 0; w < NW; ++w) {
        before += (w < wid) ? wsum[w] : 0;
        all += wsum[w];
    }
    total = all;
    __syncthreads();
    return before + incl - v;
}

__device__ __forceinline__ uint32_t sort_pad(uint32_t i) { return i + (i >> 3); }

// The hardware deals the workgroups of a launch to the chip's 8 XCDs in turn
// (workgroup w to XCD w mod 8), and each XCD has an L2 of its own. This maps
// workgroup w of n to a tile so that every XCD takes one contiguous range of
// tiles: workgroups resident together on an XCD then hold neighbouring tiles,
// and their short writes into one output line meet in the same L2. The map
// is a bijection of [0, n) for any n, so a part with another XCD count (or
// another dispatch order) only loses the locality, never correctness.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t w, uint32_t n)
{
    constexpr uint32_t kXcds = 8;
    const uint32_t q = n / kXcds, r = n % kXcds, x = w % kXcds;
    return x * q + (x < r ? x : r) + w / kXcds;
}

// Digit of a sort key: RB bits from bit sh on (the host keeps sh + RB <= 32).
template <uint32_t RB>
__device__ __forceinline__ uint32_t sort_digit(uint32_t key, uint32_t sh)
{
    return (key >> sh) & ((1u << RB) - 1u);
}

// Radix sort, pass on the RB-bit digit at bit sh: digit counts of every
// tile. A block counts kHistTiles consecutive tiles, one after the other,
// in one LDS histogram (atomic adds), with the keys of every tile loaded up
// front so that they are in flight together; blocks take their tile groups
// XCD by XCD, as the scatter blocks take their tiles.
constexpr uint32_t kHistTiles = 4;
__host__ __device__ inline uint32_t hist_blocks(uint32_t nblk)
{
    return (nblk + kHistTiles - 1) / kHistTiles;
}

template <uint32_t RB>
__global__ __launch_bounds__(kSortThreads) void k_rs_hist(const uint32_t *keys, uint64_t n,
                                                          uint32_t sh, uint32_t *hist,
                                                          uint32_t nblk)
{
    constexpr uint32_t NB = 1u << RB;
    __shared__ uint32_t cnt[NB];
    const uint32_t tid = threadIdx.x;
    const uint32_t t0 = xcd_tile(blockIdx.x, hist_blocks(nblk)) * kHistTiles;
    for (uint32_t d = tid; d < NB; d += kSortThreads) cnt[d] = 0;
    uint32_t k[kHistTiles][kSortItems];
#pragma unroll
    for (uint32_t t = 0; t < kHistTiles; ++t) {
        const uint64_t base = (uint64_t)(t0 + t) * kSortTile;
#pragma unroll
        for (uint32_t u = 0; u < kSortItems; ++u) {
            const uint64_t i = base + u * kSortThreads + tid;
            k[t][u] = (t0 + t < nblk && i < n) ? keys[i] : 0u;
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t t = 0; t < kHistTiles; ++t) {
        if (t0 + t >= nblk) break; // the same for the whole block
        const uint64_t base = (uint64_t)(t0 + t) * kSortTile;
#pragma unroll
        for (uint32_t u = 0; u < kSortItems; ++u)
            if (base + u * kSortThreads + tid < n) atomicAdd(&cnt[sort_digit<RB>(k[t][u], sh)], 1u);
        __syncthreads();
        for (uint32_t d = tid; d < NB; d += kSortThreads) {
            hist[(uint64_t)d * nblk + t0 + t] = cnt[d];
            cnt[d] = 0;
        }
        __syncthreads();
    }
}

// Radix sort, pass on the RB-bit digit at bit sh: the block ranks its tile
// by the digit in LDS, stably, then writes each digit's run to its place:
// the scanned count of that digit over all earlier digits and blocks, plus
// the rank inside the tile's run.
// Ranking: wavefront w holds the tile's items w*512 + u*64 + lane (u < 8),
// a contiguous eighth, so tile order is (w, u, lane). For each u in turn the
// lanes holding the same digit are found with one ballot per digit bit; an
// item's rank among its wavefront's items of that digit is the wavefront's
// running count of the digit (a 16-bit LDS counter per wavefront and digit)
// plus the same-digit lanes below it, and the lowest of them advances the
// counter. The counters then become per-digit prefixes over the wavefronts,
// and a block scan gives every digit's start in the tile.
// IOTA: the pass's input values are their own indices (the first pass, whose
// value for the key at index x is x), generated rather than read.
template <uint32_t RB, bool IOTA>
__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(const uint32_t *kin,
                                                             const uint32_t *vin, uint32_t *kout,
                                                             uint32_t *vout, uint64_t n,
                                                             uint32_t sh, const uint32_t *hist,
                                                             uint32_t nblk)
{
    constexpr uint32_t NB = 1u << RB, NW = kSortThreads / 64;
    constexpr uint32_t DPT = (NB + kSortThreads - 1) / kSortThreads; // digits per thread
    constexpr uint32_t WI = 64 * kSortItems;                         // items per wavefront
    static_assert(kSortTile <= 0xFFFFu, "16-bit digit counters");
    // tile index i lives at i + i/8 (sort_pad)
    __shared__ uint32_t sk[kSortTile + kSortTile / 8], sv[kSortTile + kSortTile / 8];
    __shared__ uint16_t wcnt[NW][NB];
    __shared__ uint32_t dstart[NB], dst[NB];
    __shared__ uint64_t wsum[NW];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t tile = xcd_tile(blockIdx.x, nblk);
    const uint64_t base = (uint64_t)tile * kSortTile;
    const uint32_t valid = (uint32_t)min<uint64_t>(kSortTile, n - base);
    for (uint32_t d = lane; d < NB; d += 64) wcnt[w][d] = 0; // own row, used only by this wave
    for (uint32_t d = tid; d < NB; d += kSortThreads) dst[d] = hist[(uint64_t)d * nblk + tile];
    uint32_t k[kSortItems], v[kSortItems], r[kSortItems];
#pragma unroll
    for (uint32_t u = 0; u < kSortItems; ++u) { // coalesced; padding sorts last
        const uint32_t i = w * WI + u * 64 + lane;
        k[u] = (i < valid) ? kin[base + i] : kSortNone;
        v[u] = IOTA ? (uint32_t)(base + i) : ((i < valid) ? vin[base + i] : 0u);
    }
    const uint64_t below_mask = (1ull << lane) - 1ull;
#pragma unroll
    for (uint32_t u = 0; u < kSortItems; ++u) {
        const uint32_t d = sort_digit<RB>(k[u], sh);
        uint64_t same = ~0ull;
#pragma unroll
        for (uint32_t bit = 0; bit < RB; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bal = __ballot(on);
            same &= on ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__builtin_popcountll(same & below_mask);
        const uint32_t run = wcnt[w][d];
        r[u] = run + below;
        if (below == 0) wcnt[w][d] = (uint16_t)(run + (uint32_t)__builtin_popcountll(same));
    }
    __syncthreads();
    // per digit: the wavefronts' counts become exclusive prefixes over the
    // wavefronts; the digit's count in the tile
    uint32_t tot[DPT];
    uint64_t mine = 0;
#pragma unroll
    for (uint32_t j = 0; j < DPT; ++j) {
        const uint32_t d = tid * DPT + j;
        uint32_t acc = 0;
        if (d < NB) {
#pragma unroll
            for (uint32_t x = 0; x < NW; ++x) {
                const uint32_t c = wcnt[x][d];
                wcnt[x][d] = (uint16_t)acc;
                acc += c;
            }
        }
        tot[j] = acc;
        mine += acc;
    }
    uint64_t all;
    uint32_t start = (uint32_t)sort_block_scan(mine, wsum, all); // ends with a barrier
#pragma unroll
    for (uint32_t j = 0; j < DPT; ++j) {
        const uint32_t d = tid * DPT + j;
        if (d < NB) dstart[d] = start;
        start += tot[j];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < kSortItems; ++u) {
        const uint32_t d = sort_digit<RB>(k[u], sh);
        const uint32_t pos = dstart[d] + wcnt[w][d] + r[u];
        sk[sort_pad(pos)] = k[u];
        sv[sort_pad(pos)] = v[u];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < kSortItems; ++u) {
        const uint32_t i = u * kSortThreads + tid;
        if (i < valid) {
            const uint32_t key = sk[sort_pad(i)], d = sort_digit<RB>(key, sh);
            const uint32_t o = dst[d] + (i - dstart[d]);
            kout[o] = key;
            vout[o] = sv[sort_pad(i)];
        }
    }
}

// Sorting form of the group pass, over the sorted pairs (runs of steps into
// one target, steps increasing): each step's move (down for the first of
// its run, else to the step before it), and each target's last step.
template <typename Move>
__global__ __launch_bounds__(256) void k_gp_group(GProblem P, GArrays g, const uint32_t *keys,
                                                  const uint32_t *vals)
{
    using MB = MoveBits<Move>;
    Move *move = static_cast<Move *>(g.move);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.npos;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = keys[i], z = vals[i];
        if (x == kSortNone) { // no step, or j_p = p
            move[z] = MB::kStay;
            continue;
        }
        const bool first = i == 0 || keys[i - 1] != x;
        const bool last = i + 1 == P.npos || keys[i + 1] != x;
        move[z] = first ? (MB::kDown | (Move)x) : (MB::kPrev | (Move)vals[i - 1]);
        if (last) g.last[x] = z;
    }
}

// Walk pass: the destination of the element first at x. If some step
// targets x it is x's last step, already in last[x]; else the walk follows
// the moves from x and stores where it ends in last[x]. Only reads are
// random here; the values move in the place pass.
template <typename Move>
__global__ __launch_bounds__(256) void k_g_walk(GProblem P, GArrays g)
{
    using MB = MoveBits<Move>;
    const Move *move = static_cast<const Move *>(g.move);
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P.npos;
         x += (uint64_t)gridDim.x * blockDim.x) {
        if (g.last[x] != kNone32) continue;
        const GItem &it = item_at(P, item_of_pos(P, x));
        Move m = move[x];
        uint64_t z = x;
        // every move down ends at a smaller position, so a walk is shorter
        // than its array; the cap only bounds it against corrupted scratch
        for (uint32_t guard = 0; guard < it.n && (m >> MB::kShift) == 0; ++guard) {
            z = m & MB::kPos;
            m = move[z];
        }
        g.last[x] = (m >> MB::kShift) == 1 ? (uint32_t)(m & MB::kPos) : (uint32_t)z;
    }
}

// Place pass: every element written at its destination (the only random
// writes of the pass).
template <typename Elem>
__global__ __launch_bounds__(256) void k_g_place(GProblem P, GArrays g, const Elem *data_arg)
{
    const global_t<const Elem> *data = problem_data(P, data_arg);
    Elem *tmp = static_cast<Elem *>(g.tmp);
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P.npos;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const GItem &it = item_at(P, item_of_pos(P, x));
        place(it, tmp, g.last[x], data[it.data_off + (x - it.pos_base)]);
    }
}

template <typename Elem>
__global__ __launch_bounds__(256) void k_gp_copy(GProblem P, GArrays g, Elem *data_arg)
{
    global_t<Elem> *data = problem_data(P, data_arg);
    const Elem *tmp = static_cast<const Elem *>(g.tmp);
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < P.npos;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const GItem &it = item_at(P, item_of_pos(P, x));
        if (it.out) continue;
        data[it.data_off + (x - it.pos_base)] = tmp[x];
    }
}

// The copy pass of one in-place shuffle whose array starts 16-byte aligned
// (as the placement buffer does): 16-byte vectors, then the tail.
template <typename Elem>
__global__ __launch_bounds__(256) void k_gp_copy_vec(Elem *data, const Elem *tmp, uint64_t n)
{
    constexpr uint32_t V = 16 / sizeof(Elem);
    const uint64_t nv = n / V, stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const u32x4 *src = reinterpret_cast<const u32x4 *>(tmp);
    global_t<u32x4> *dst = reinterpret_cast<global_t<u32x4> *>(as_global(data));
    for (uint64_t x = t; x < nv; x += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + x), dst + x);
    for (uint64_t x = nv * V + t; x < n; x += stride) as_global(data)[x] = tmp[x];
}

__global__ __launch_bounds__(kScanThreads) void k_gp_scan_tiles(const uint32_t *a,
                                                                 uint32_t *tiles, uint64_t len)
{
    constexpr int NW = kScanThreads / 64;
    __shared__ uint32_t wsum[NW];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile;
    const uint32_t n = (uint32_t)min((uint64_t)kScanTile, len - b0);
    uint32_t local = 0;
    for (uint32_t x = threadIdx.x; x < n; x += kScanThreads) local += a[b0 + x];
    local = wave_inclusive_scan(local);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < NW; ++w) t += wsum[w];
        tiles[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_gp_scan_sums(uint32_t *tiles, uint32_t ntiles)
{
    __shared__ uint32_t wsum[16];
    block_scan_array<1024>(tiles, ntiles, 0, wsum);
}

// Exclusive scan of one tile of kScanTile counts starting at the tile's
// base: coalesced loads into LDS, an LDS scan, coalesced stores.
__global__ __launch_bounds__(kScanThreads) void k_gp_scan_apply(uint32_t *a,
                                                                 const uint32_t *tiles,
                                                                 uint64_t len)
{
    __shared__ uint32_t buf[kScanTile];
    __shared__ uint32_t wsum[kScanThreads / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile;
    const uint32_t n = (uint32_t)min((uint64_t)kScanTile, len - b0);
    for (uint32_t x = threadIdx.x; x < n; x += kScanThreads) buf[x] = a[b0 + x];
    __syncthreads();
    block_scan_array<kScanThreads>(buf, n, tiles[blockIdx.x], wsum);
    for (uint32_t x = threadIdx.x; x < n; x += kScanThreads) a[b0 + x] = buf[x];
}

uint32_t grid_for(uint64_t work, uint32_t block)
{
    uint64_t b = (work + block - 1) / block;
    if (b < 1) b = 1;
    if (b > (1u << 20)) b = 1u << 20;
    return (uint32_t)b;
}

void scan_exclusive(uint32_t *a, uint32_t *tiles, uint64_t len, hipStream_t stream)
{
    const uint64_t ntiles = scan_tiles(len);
    k_gp_scan_tiles<<<(uint32_t)ntiles, kScanThreads, 0, stream>>>(a, tiles, len);
    k_gp_scan_sums<<<1, 1024, 0, stream>>>(tiles, (uint32_t)ntiles);
    k_gp_scan_apply<<<(uint32_t)ntiles, kScanThreads, 0, stream>>>(a, tiles, len);
}

// One radix sort pass on the RB-bit digit at bit sh, from buffer cur into
// cur ^ 1.
template <uint32_t RB>
void sort_pass(const GArrays &g, int cur, uint64_t npos, uint32_t sh, uint32_t nblk,
               hipStream_t stream)
{
    k_rs_hist<RB><<<hist_blocks(nblk), kSortThreads, 0, stream>>>(g.key[cur], npos, sh, g.hist, nblk);
    scan_exclusive(g.hist, g.tiles, ((uint64_t)1 << RB) * nblk, stream);
    if (sh == 0)
        k_rs_scatter<RB, true><<<nblk, kSortThreads, 0, stream>>>(
            g.key[cur], nullptr, g.key[cur ^ 1], g.val[cur ^ 1], npos, sh, g.hist, nblk);
    else
        k_rs_scatter<RB, false><<<nblk, kSortThreads, 0, stream>>>(
            g.key[cur], g.val[cur], g.key[cur ^ 1], g.val[cur ^ 1], npos, sh, g.hist, nblk);
}

// The copy pass: by 16-byte vectors for one in-place shuffle whose array is
// aligned like the placement buffer, else element by element.
template <typename Elem>
void launch_copy(const GProblem &P, const GArrays &g, void *data, hipStream_t stream)
{
    Elem *z = static_cast<Elem *>(data) + P.one.data_off;
    if (!P.items && !P.dyn && !P.one.out && (reinterpret_cast<uintptr_t>(z) & 15) == 0 &&
        (reinterpret_cast<uintptr_t>(g.tmp) & 15) == 0) {
        const uint64_t nv = P.npos / (16 / sizeof(Elem)) + 1;
        k_gp_copy_vec<Elem><<<grid_for(nv, 256), 256, 0, stream>>>(z, static_cast<const Elem *>(g.tmp),
                                                                   P.npos);
        return;
    }
    k_gp_copy<Elem><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g, static_cast<Elem *>(data));
}

template <typename Elem, bool W>
hipError_t gproblem_t(const GProblem &P, void *data, uint64_t seed, void *scratch,
                      hipStream_t stream)
{
    const GArrays g = garrays(scratch, P.npos);
    if (P.npos <= kCountMaxPositions) {
        k_gc_init<<<grid_for(P.npos + 1, 256), 256, 0, stream>>>(P, g.cnt, P.npos + 1);
        k_gc_dice<W><<<grid_for(P.npairs, 256), 256, 0, stream>>>(P, g, seed);
        scan_exclusive(g.cnt, g.tiles, P.npos + 1, stream);
        k_gc_scatter<<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g);
        k_gc_group<uint32_t><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g);
        k_g_walk<uint32_t><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g);
        k_g_place<Elem><<<grid_for(P.npos, 256), 256, 0, stream>>>(
            P, g, static_cast<const Elem *>(data));
        launch_copy<Elem>(P, g, data, stream);
        return hipGetLastError();
    }
    // one item: a thread per 16-byte vector of last[]
    k_gp_init<<<grid_for(P.items ? P.npos : P.npos / 4 + 1, 256), 256, 0, stream>>>(P, g, P.npos);
    k_gp_dice<W><<<grid_for(P.npairs, 256), 256, 0, stream>>>(P, g, seed);
    // targets are < npos, so bit_length(npos) bits order them all, and the
    // "none" key (all ones) after them
    uint32_t bits = 0;
    while (bits < 32 && (P.npos >> bits) != 0) ++bits;
    const uint32_t nblk = (uint32_t)sort_blocks(P.npos);
    const uint32_t passes = (bits + kSortDigitMax - 1) / kSortDigitMax;
    const uint32_t rb0 = (bits + passes - 1) / passes, rb = rb0 < 8 ? 8 : rb0;
    int cur = 0;
    for (uint32_t sh = 0; sh < bits; sh += rb, cur ^= 1) {
        if (rb == 8) sort_pass<8>(g, cur, P.npos, sh, nblk, stream);
        else if (rb == 9) sort_pass<9>(g, cur, P.npos, sh, nblk, stream);
        else sort_pass<10>(g, cur, P.npos, sh, nblk, stream);
    }
    if (P.npos < kMove32MaxPositions) {
        k_gp_group<uint32_t><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g, g.key[cur],
                                                                        g.val[cur]);
        k_g_walk<uint32_t><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g);
    } else {
        k_gp_group<uint64_t><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g, g.key[cur],
                                                                        g.val[cur]);
        k_g_walk<uint64_t><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g);
    }
    k_g_place<Elem><<<grid_for(P.npos, 256), 256, 0, stream>>>(P, g,
                                                               static_cast<const Elem *>(data));
    launch_copy<Elem>(P, g, data, stream);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sparse samples: m of n without replacement for n above the LDS tier. Only
// positions base .. n-1 (base = n - m) are output and only the steps p >= lo
// (lo = n - steps) run. A step's head chain climbs through larger steps, so
// every chain that decides an output stays among positions base .. n-1:
// index arrays of m entries (entry e = position base + e) suffice, and the
// work is O(m) sort passes and gathers whatever n is.
//   init:    heads "none"; entries below lo (position 0, when m = n) take no
//            step: j = own position, sort key "none"
//   dice:    j_p of every step and its sort key (target, or "none" if j_p = p)
//   sort:    the (target, entry) pairs by target (targets below 2^bits, bits
//            the bit length of n), as in the device-wide tier
//   links:   over the sorted runs: head[x - base] = smallest step into x for
//            every target x >= base; succ[e] = next larger step into the
//            target of entry e
//   resolve: the source of every output position, as in the LDS tier: a
//            position that takes no step or targets itself follows the head
//            chain from itself; another follows it from its successor, or
//            takes its target's original element if it has none
// ---------------------------------------------------------------------------

struct SArrays {
    uint32_t *jj;              // j_p of each entry's position
    uint32_t *key[2], *val[2]; // sort ping-pong: target, entry
    uint32_t *head;            // per entry as a target: smallest step into it
    uint32_t *succ;            // per entry as a step: next larger step into its target
    uint32_t *hist, *tiles;    // sort histograms, scan partial sums
};

__host__ __device__ inline uint64_t sarrays_bytes(uint64_t m)
{
    const uint64_t w = align256(4 * m), nh = ((uint64_t)1 << kSortDigitMax) * sort_blocks(m);
    return 7 * w + align256(4 * nh) + align256(4 * scan_tiles(nh > m + 1 ? nh : m + 1));
}

inline SArrays sarrays(void *base, uint64_t m)
{
    char *p = static_cast<char *>(base);
    const uint64_t w = align256(4 * m), nh = ((uint64_t)1 << kSortDigitMax) * sort_blocks(m);
    SArrays a;
    uint32_t **arr[7] = {&a.jj, &a.key[0], &a.val[0], &a.key[1], &a.val[1], &a.head, &a.succ};
    for (int i = 0; i < 7; ++i) {
        *arr[i] = reinterpret_cast<uint32_t *>(p);
        p += w;
    }
    a.hist = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * nh);
    a.tiles = reinterpret_cast<uint32_t *>(p);
    return a;
}

// What the sparse-sample kernels share: the sample, its batches and the
// instance (with the server's claim added, if any).
struct SProblem {
    uint32_t n, steps, m, base; // base = n - m; steps run at positions >= n - steps
    SegTable seg;
    uint64_t inst;
    DevClaim claim;
};

__global__ __launch_bounds__(256) void k_sp_init(SProblem Q, SArrays a)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && Q.claim.counter) (void)take_claim(Q.claim);
    const uint32_t lo = Q.n - Q.steps;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < Q.m; e += gridDim.x * blockDim.x) {
        a.head[e] = kNone32;
        const uint32_t p = Q.base + e;
        if (p < lo) {
            a.jj[e] = p;
            a.key[0][e] = kSortNone;
        }
    }
}

template <bool W>
__global__ __launch_bounds__(256) void k_sp_dice(SProblem Q, SArrays a, uint64_t seed)
{
    const uint32_t npairs = (Q.seg.S + 1) / 2;
    const uint32_t src = W ? Q.seg.words : BRR_WORDS_PHILOX64;
    const StreamKey key = make_key(seed, Q.inst + (Q.claim.slot ? *Q.claim.slot : 0));
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < npairs;
         w += gridDim.x * blockDim.x) {
        uint64_t wd[2];
        first_pair(src, w, key, wd[0], wd[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t s = 2 * w + h;
            if (s >= Q.seg.S) continue;
            uint32_t i0, k, f;
            uint64_t u;
            batch_at(s, Q.seg.seg, Q.seg.nseg, i0, k, u, f);
            uint64_t r = batch_state(src, f, i0, k, u, wd[h], Q.seg.S, s, key);
            for (uint32_t l = 0; l < k; ++l) {
                const uint32_t p = i0 - 1 - l;
                const uint32_t t = next_die(src, f, i0 - l, r);
                a.jj[p - Q.base] = t;
                a.key[0][p - Q.base] = (t < p) ? t : kSortNone;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_sp_links(SProblem Q, SArrays a, const uint32_t *keys,
                                                  const uint32_t *vals)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < Q.m; i += gridDim.x * blockDim.x) {
        const uint32_t x = keys[i], e = vals[i];
        if (x == kSortNone) continue;
        if ((i == 0 || keys[i - 1] != x) && x >= Q.base) a.head[x - Q.base] = Q.base + e;
        a.succ[e] = (i + 1 < Q.m && keys[i + 1] == x) ? Q.base + vals[i + 1] : kNone32;
    }
}

template <typename Elem>
__global__ __launch_bounds__(256) void k_sp_resolve(SProblem Q, SArrays a, const Elem *data,
                                                    Elem *out)
{
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < Q.m; e += gridDim.x * blockDim.x) {
        const uint32_t p = Q.base + e, q = a.jj[e];
        uint32_t y = p, src;
        bool walk = true;
        if (q != p) {
            const uint32_t sc = a.succ[e];
            if (sc == kNone32) {
                walk = false;
                src = q;
            } else {
                y = sc;
            }
        }
        if (walk) {
            uint32_t h;
            for (uint32_t guard = 0; guard < Q.m && (h = a.head[y - Q.base]) != kNone32; ++guard)
                y = h;
            src = y;
        }
        out[Q.n - 1 - p] = data[src];
    }
}

template <typename Elem, bool W>
hipError_t sample_sparse_t(const SProblem &Q, const void *data, void *out, uint64_t seed,
                           void *scratch, hipStream_t stream)
{
    const SArrays a = sarrays(scratch, Q.m);
    k_sp_init<<<grid_for(Q.m, 256), 256, 0, stream>>>(Q, a);
    k_sp_dice<W><<<grid_for((Q.seg.S + 1) / 2, 256), 256, 0, stream>>>(Q, a, seed);
    uint32_t bits = 0;
    while (bits < 32 && (Q.n >> bits) != 0) ++bits;
    GArrays g;
    std::memset(&g, 0, sizeof g);
    for (int c = 0; c < 2; ++c) {
        g.key[c] = a.key[c];
        g.val[c] = a.val[c];
    }
    g.hist = a.hist;
    g.tiles = a.tiles;
    const uint32_t nblk = (uint32_t)sort_blocks(Q.m);
    const uint32_t passes = (bits + kSortDigitMax - 1) / kSortDigitMax;
    const uint32_t rb0 = (bits + passes - 1) / passes, rb = rb0 < 8 ? 8 : rb0;
    int cur = 0;
    for (uint32_t sh = 0; sh < bits; sh += rb, cur ^= 1) {
        if (rb == 8) sort_pass<8>(g, cur, Q.m, sh, nblk, stream);
        else if (rb == 9) sort_pass<9>(g, cur, Q.m, sh, nblk, stream);
        else sort_pass<10>(g, cur, Q.m, sh, nblk, stream);
    }
    k_sp_links<<<grid_for(Q.m, 256), 256, 0, stream>>>(Q, a, a.key[cur], a.val[cur]);
    k_sp_resolve<Elem><<<grid_for(Q.m, 256), 256, 0, stream>>>(
        Q, a, static_cast<const Elem *>(data), static_cast<Elem *>(out));
    return hipGetLastError();
}

template <typename Elem, bool W>
hipError_t lds_single_t(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, void *out,
                        const DevSched &sc, uint64_t seed, uint64_t inst, const DevClaim &claim,
                        hipStream_t stream)
{
    SegTable st;
    build_segments(n, steps, sc, st);
    const uint32_t bytes = lds_bytes(n);
    Elem *z = static_cast<Elem *>(data), *o = static_cast<Elem *>(out);
    // the smallest block of the size classes that holds the array
    if (n <= lds_class_max_n(0))
        k_lds_single<Elem, 64, kWaveP, W><<<1, 64, bytes, stream>>>(z, n, steps, out_lo, o, st, seed,
                                                                 inst, claim);
    else if (n <= lds_class_max_n(1))
        k_lds_single<Elem, 256, 8, W><<<1, 256, bytes, stream>>>(z, n, steps, out_lo, o, st, seed,
                                                              inst, claim);
    else if (n <= lds_class_max_n(2))
        k_lds_single<Elem, 256, 16, W><<<1, 256, bytes, stream>>>(z, n, steps, out_lo, o, st, seed,
                                                               inst, claim);
    else if (n <= lds_class_max_n(3))
        k_lds_single<Elem, 512, 16, W><<<1, 512, bytes, stream>>>(z, n, steps, out_lo, o, st, seed,
                                                               inst, claim);
    else
        k_lds_single<Elem, kWgThreads, kWgP, W><<<1, kWgThreads, bytes, stream>>>(
            z, n, steps, out_lo, o, st, seed, inst, claim);
    return hipGetLastError();
}

template <typename Elem, int BLOCK, int P, bool W>
hipError_t batched_lds_t(const RunArgs *b, const uint32_t *items, uint32_t nitems, uint32_t max_n,
                         const DevSched &sc, hipStream_t stream)
{
    if (nitems == 0) return hipSuccess;
    const uint32_t bytes = lds_bytes(max_n);
    k_lds_batched<Elem, BLOCK, P, W><<<nitems, BLOCK, bytes, stream>>>(b, items, sc);
    return hipGetLastError();
}

template <typename Elem, bool W>
hipError_t batched_peel_t(const RunArgs *b, const uint32_t *items, uint32_t nitems,
                          const DevSched &sc, hipStream_t stream)
{
    if (nitems == 0) return hipSuccess;
    k_peel_batched<Elem, W, kPeelThreads><<<nitems, kPeelThreads, kPeelLdsBytes, stream>>>(b, items, sc);
    return hipGetLastError();
}

template <typename Elem, bool W>
hipError_t batched_lane_t(const RunArgs *b, const uint32_t *items, uint32_t nitems, uint32_t max_n,
                          const DevSched &sc, hipStream_t stream)
{
    if (nitems == 0) return hipSuccess;
    const uint32_t arrays = lane_arrays(max_n);
    const uint32_t blocks = (nitems + arrays - 1) / arrays;
    const LaneLds L = lane_lds(max_n, sizeof(Elem));
    k_lane_batched<Elem, W><<<blocks, kLaneItems, L.bytes, stream>>>(b, items, nitems, max_n, sc);
    return hipGetLastError();
}

} // namespace

uint32_t lds_tier_max_n() { return kWgThreads * kWgP; }
uint32_t lane_tier_max_n() { return kLaneMaxN; }

hipError_t launch_batched_lane(const RunArgs *b, const uint32_t *items, uint32_t nitems,
                               uint32_t max_n, uint32_t eb, const DevSched &sc, hipStream_t stream)
{
    if (max_n > lane_tier_max_n()) return hipErrorInvalidValue;
    if (sc.words != BRR_WORDS_PHILOX64)
        return eb == 4 ? batched_lane_t<uint32_t, true>(b, items, nitems, max_n, sc, stream)
                       : batched_lane_t<uint64_t, true>(b, items, nitems, max_n, sc, stream);
    return eb == 4 ? batched_lane_t<uint32_t, false>(b, items, nitems, max_n, sc, stream)
                   : batched_lane_t<uint64_t, false>(b, items, nitems, max_n, sc, stream);
}

hipError_t launch_set_args(RunArgs *dev, const RunArgs &val, hipStream_t stream)
{
    k_set_args<<<1, 64, 0, stream>>>(dev, val);
    return hipGetLastError();
}
uint32_t peel_tier_max_n() { return kPeelTierMax; }

hipError_t launch_batched_peel(const RunArgs *b, const uint32_t *items, uint32_t nitems,
                               uint32_t eb, const DevSched &sc, hipStream_t stream)
{
    if (sc.words != BRR_WORDS_PHILOX64)
        return eb == 4 ? batched_peel_t<uint32_t, true>(b, items, nitems, sc, stream)
                       : batched_peel_t<uint64_t, true>(b, items, nitems, sc, stream);
    return eb == 4 ? batched_peel_t<uint32_t, false>(b, items, nitems, sc, stream)
                   : batched_peel_t<uint64_t, false>(b, items, nitems, sc, stream);
}

hipError_t prepare_shuffle_kernels()
{
    const int wg = (int)lds_bytes(kWgThreads * kWgP);
    const int c0 = (int)lds_bytes(lds_class_max_n(0)), c1 = (int)lds_bytes(lds_class_max_n(1));
    const int c2 = (int)lds_bytes(lds_class_max_n(2)), c3 = (int)lds_bytes(lds_class_max_n(3));
    struct Attr {
        const void *fn;
        int bytes;
    };
#define BRR_LDS_ATTRS(W)                                                                   \
    {(const void *)k_lds_single<uint32_t, kWgThreads, kWgP, W>, wg},                       \
        {(const void *)k_lds_single<uint64_t, kWgThreads, kWgP, W>, wg},                   \
        {(const void *)k_lds_single<uint32_t, 512, 16, W>, c3},                            \
        {(const void *)k_lds_single<uint64_t, 512, 16, W>, c3},                            \
        {(const void *)k_lds_batched<uint32_t, 64, kWaveP, W>, c0},                        \
        {(const void *)k_lds_batched<uint64_t, 64, kWaveP, W>, c0},                        \
        {(const void *)k_lds_batched<uint32_t, 256, 8, W>, c1},                            \
        {(const void *)k_lds_batched<uint64_t, 256, 8, W>, c1},                            \
        {(const void *)k_lds_batched<uint32_t, 256, 16, W>, c2},                           \
        {(const void *)k_lds_batched<uint64_t, 256, 16, W>, c2},                           \
        {(const void *)k_lds_batched<uint32_t, 512, 16, W>, c3},                           \
        {(const void *)k_lds_batched<uint64_t, 512, 16, W>, c3},                           \
        {(const void *)k_lds_batched<uint32_t, kWgThreads, kWgP, W>, wg},                  \
        {(const void *)k_lds_batched<uint64_t, kWgThreads, kWgP, W>, wg},                  \
        {(const void *)k_lds_requests<uint32_t, 64, kWaveP, W>, c0},                       \
        {(const void *)k_lds_requests<uint64_t, 64, kWaveP, W>, c0},                       \
        {(const void *)k_lds_requests<uint32_t, 256, 8, W>, c1},                           \
        {(const void *)k_lds_requests<uint64_t, 256, 8, W>, c1},                           \
        {(const void *)k_lds_requests<uint32_t, 256, 16, W>, c2},                          \
        {(const void *)k_lds_requests<uint64_t, 256, 16, W>, c2},                          \
        {(const void *)k_lds_requests<uint32_t, 512, 16, W>, c3},                          \
        {(const void *)k_lds_requests<uint64_t, 512, 16, W>, c3},                          \
        {(const void *)k_lds_requests<uint32_t, kWgThreads, kWgP, W>, wg},                 \
        {(const void *)k_lds_requests<uint64_t, kWgThreads, kWgP, W>, wg}
    const int pl = (int)kPeelLdsBytes;
    const Attr attrs[] = {BRR_LDS_ATTRS(false), BRR_LDS_ATTRS(true),
                          {(const void *)k_peel_batched<uint32_t, false, kPeelThreads>, pl},
                          {(const void *)k_peel_batched<uint64_t, false, kPeelThreads>, pl},
                          {(const void *)k_peel_batched<uint32_t, true, kPeelThreads>, pl},
                          {(const void *)k_peel_batched<uint64_t, true, kPeelThreads>, pl}};
#undef BRR_LDS_ATTRS
    for (const Attr &a : attrs) {
        const hipError_t e =
            hipFuncSetAttribute(a.fn, hipFuncAttributeMaxDynamicSharedMemorySize, a.bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

uint32_t wave_tier_max_n() { return 64 * kWaveP; }
uint64_t gtier_scratch_bytes(uint64_t npos, uint32_t eb) { return garrays_bytes(npos, eb); }
uint32_t gtier_tile_shift() { return kTileShift; }

hipError_t launch_lds_single(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, uint32_t eb,
                             void *out, const DevSched &sc, uint64_t seed, uint64_t inst,
                             const DevClaim &claim, hipStream_t stream)
{
    if (n > lds_tier_max_n() || steps == 0 || steps >= n || out_lo > n - steps)
        return hipErrorInvalidValue;
    if (sc.words != BRR_WORDS_PHILOX64)
        return eb == 4 ? lds_single_t<uint32_t, true>(data, n, steps, out_lo, out, sc, seed, inst,
                                                      claim, stream)
                       : lds_single_t<uint64_t, true>(data, n, steps, out_lo, out, sc, seed, inst,
                                                      claim, stream);
    return eb == 4 ? lds_single_t<uint32_t, false>(data, n, steps, out_lo, out, sc, seed, inst,
                                                   claim, stream)
                   : lds_single_t<uint64_t, false>(data, n, steps, out_lo, out, sc, seed, inst,
                                                   claim, stream);
}

uint64_t one_scratch_bytes(uint64_t n, uint32_t eb, uint64_t m)
{
    if (n <= lds_tier_max_n()) return 0;
    return m ? sarrays_bytes(m) : gtier_scratch_bytes(n, eb);
}

hipError_t launch_one(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, uint32_t eb,
                      void *out, const DevSched &ds, uint64_t seed, uint64_t inst,
                      const DevClaim &claim, hipStream_t s, void *scratch_given)
{
    if (n <= lds_tier_max_n())
        return launch_lds_single(data, n, steps, out_lo, eb, out, ds, seed, inst, claim, s);
    SegTable st;
    build_segments(n, steps, ds, st);
    if (out) {
        SProblem Q;
        std::memset(&Q, 0, sizeof Q);
        Q.n = n;
        Q.steps = steps;
        Q.m = n - out_lo;
        Q.base = out_lo;
        Q.seg = st;
        Q.inst = inst;
        Q.claim = claim;
        void *scratch = scratch_given;
        hipError_t e = hipSuccess;
        if (!scratch && (e = hipMallocAsync(&scratch, sarrays_bytes(Q.m), s)) != hipSuccess) return e;
        const bool w = ds.words != BRR_WORDS_PHILOX64;
        e = eb == 4 ? (w ? sample_sparse_t<uint32_t, true>(Q, data, out, seed, scratch, s)
                         : sample_sparse_t<uint32_t, false>(Q, data, out, seed, scratch, s))
                    : (w ? sample_sparse_t<uint64_t, true>(Q, data, out, seed, scratch, s)
                         : sample_sparse_t<uint64_t, false>(Q, data, out, seed, scratch, s));
        if (scratch_given) return e;
        const hipError_t f = hipFreeAsync(scratch, s);
        return e != hipSuccess ? e : f;
    }
    const GItem it{0, 0, inst, n, steps, out_lo, 0, out};
    GTierArgs a;
    std::memset(&a, 0, sizeof a);
    a.data = data;
    a.eb = eb;
    a.seed = seed;
    a.claim = claim;
    a.words = ds.words;
    a.nitems = 1;
    a.npos = n;
    a.npairs = (st.S + 1) / 2;
    a.one_item = &it;
    a.one_seg = &st;
    if (scratch_given) {
        a.scratch = scratch_given;
        return launch_gtier(a, s);
    }
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, gtier_scratch_bytes(n, eb), s);
    if (e != hipSuccess) return e;
    a.scratch = scratch;
    e = launch_gtier(a, s);
    const hipError_t f = hipFreeAsync(scratch, s);
    return e != hipSuccess ? e : f;
}

hipError_t launch_gtier(const GTierArgs &a, hipStream_t stream)
{
    if (a.nitems == 0) return hipSuccess;
    if (a.npos > kMaxGtierPositions) return hipErrorInvalidValue;
    GProblem P;
    std::memset(&P, 0, sizeof P);
    P.nitems = a.nitems;
    P.npos = a.npos;
    P.npairs = a.npairs;
    P.inst_base = a.inst_base;
    P.claim = a.claim;
    P.dyn = a.dyn;
    if (a.nitems == 1 && a.one_item) {
        P.one = *a.one_item;
        P.one_seg = *a.one_seg;
    } else {
        P.items = a.items;
        P.segs = a.segs;
        P.pos_base = a.pos_base;
        P.pair_base = a.pair_base;
        P.pos_tile = a.pos_tile;
        P.pair_tile = a.pair_tile;
    }
    if (a.words != BRR_WORDS_PHILOX64)
        return a.eb == 4 ? gproblem_t<uint32_t, true>(P, a.data, a.seed, a.scratch, stream)
                         : gproblem_t<uint64_t, true>(P, a.data, a.seed, a.scratch, stream);
    return a.eb == 4 ? gproblem_t<uint32_t, false>(P, a.data, a.seed, a.scratch, stream)
                     : gproblem_t<uint64_t, false>(P, a.data, a.seed, a.scratch, stream);
}

uint32_t lds_class_max_n(int c)
{
    static const uint32_t cap[kLdsClasses] = {64 * kWaveP, 256 * 8, 256 * 16, 512 * 16,
                                              kWgThreads * kWgP};
    return (c >= 0 && c < kLdsClasses) ? cap[c] : 0;
}

int lds_request_class(uint32_t n)
{
    for (int c = 0; c < kLdsClasses; ++c)
        if (n <= lds_class_max_n(c)) return c;
    return -1;
}

hipError_t launch_lds_requests(int c, uint32_t eb, const ReqBatch &b, uint32_t max_n,
                               const DevSched &sc, uint64_t seed, const uint64_t *slots,
                               hipStream_t stream)
{
    if (b.count == 0) return hipSuccess;
    if (b.count > kMaxFusedRequests || max_n > lds_class_max_n(c)) return hipErrorInvalidValue;
    const bool w = sc.words != BRR_WORDS_PHILOX64;
    const uint32_t bytes = lds_bytes(max_n);
#define BRR_REQ_CLASS(B, P)                                                                       \
    if (eb == 4) {                                                                                \
        if (w) k_lds_requests<uint32_t, B, P, true><<<b.count, B, bytes, stream>>>(b, sc, seed, slots); \
        else k_lds_requests<uint32_t, B, P, false><<<b.count, B, bytes, stream>>>(b, sc, seed, slots); \
    } else {                                                                                      \
        if (w) k_lds_requests<uint64_t, B, P, true><<<b.count, B, bytes, stream>>>(b, sc, seed, slots); \
        else k_lds_requests<uint64_t, B, P, false><<<b.count, B, bytes, stream>>>(b, sc, seed, slots); \
    }
    switch (c) {
    case 0: BRR_REQ_CLASS(64, kWaveP) break;
    case 1: BRR_REQ_CLASS(256, 8) break;
    case 2: BRR_REQ_CLASS(256, 16) break;
    case 3: BRR_REQ_CLASS(512, 16) break;
    default: BRR_REQ_CLASS(kWgThreads, kWgP) break;
    }
#undef BRR_REQ_CLASS
    return hipGetLastError();
}

hipError_t launch_batched_lds(int c, const RunArgs *b, const uint32_t *items, uint32_t nitems,
                              uint32_t max_n, uint32_t eb, const DevSched &sc, hipStream_t stream)
{
    if (max_n > lds_class_max_n(c)) return hipErrorInvalidValue;
    const bool w = sc.words != BRR_WORDS_PHILOX64;
#define BRR_LDS_CLASS(B, P)                                                                      \
    return w ? (eb == 4 ? batched_lds_t<uint32_t, B, P, true>(b, items, nitems, max_n, sc, stream) \
                        : batched_lds_t<uint64_t, B, P, true>(b, items, nitems, max_n, sc, stream)) \
             : (eb == 4 ? batched_lds_t<uint32_t, B, P, false>(b, items, nitems, max_n, sc, stream) \
                        : batched_lds_t<uint64_t, B, P, false>(b, items, nitems, max_n, sc, stream))
    switch (c) {
    case 0: BRR_LDS_CLASS(64, kWaveP);
    case 1: BRR_LDS_CLASS(256, 8);
    case 2: BRR_LDS_CLASS(256, 16);
    case 3: BRR_LDS_CLASS(512, 16);
    default: BRR_LDS_CLASS(kWgThreads, kWgP);
    }
#undef BRR_LDS_CLASS
}

} // namespace brr
