// Shuffles and samples: Algorithm 4 batches (Sec. 6) applied in the order of
// Algorithm 1, evaluated in parallel with the exact sequential result.
//
// Dice. Batch s of a shuffle (k dice at size i) reads word s on its first
// attempt and a*S + s on attempt a, rolls the bounds i, i-1, ..., i-k+1
// through the Theorem 1 chain and is accepted when the leftover r satisfies
// r >= 2^64 mod i^(falling k); the schedule's guard u only decides when that
// threshold is formed (r >= u >= product implies acceptance). Die l of the
// batch is j_p for position p = i-1-l: step p swaps z[p] with z[j_p], j_p <= p.
// Every batch is independent, so all dice are rolled at once.
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
#include "device.hpp"
#include "internal.hpp"

namespace brr {

namespace {

constexpr uint16_t kNone16 = 0xFFFF;
constexpr uint32_t kNone32 = 0xFFFFFFFFu;
constexpr int kWaveP = 8;        // positions per lane in the wavefront tier
constexpr int kWgThreads = 1024; // workgroup tier and single-workgroup global tier
constexpr int kWgP = 16;         // positions per thread in the workgroup tier
constexpr uint32_t kScanTile = 1024 * 16;
constexpr uint64_t kMaxAttempts = 1024;

__device__ __forceinline__ void batch_at(uint32_t s, const Seg *seg, uint32_t nseg, uint32_t &i,
                                         uint32_t &k, uint64_t &u)
{
    uint32_t g = 0;
    while (g + 1 < nseg && s >= seg[g + 1].s0) ++g;
    i = seg[g].i0 - (s - seg[g].s0) * seg[g].k;
    k = seg[g].k;
    u = seg[g].u;
}

// The accepted word of batch s (k dice at size i, guard u) whose first
// attempt reads r.
__device__ __forceinline__ uint64_t accept_word(uint32_t i, uint32_t k, uint64_t u, uint64_t r,
                                                uint32_t S, uint32_t s, const StreamKey &key)
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
            r = word_at(attempt * S + s, key);
            rr = r;
            for (uint32_t l = 0; l < k; ++l) (void)mul_roll(i - l, rr);
        }
    }
    return r;
}

// Exclusive prefix sums of a[0..len) in place, by the whole block (contiguous
// chunks per thread); returns the total. Ends with a barrier.
template <int BLOCK>
__device__ uint32_t block_scan_array(uint32_t *a, uint32_t len, uint32_t base, uint32_t *wsum)
{
    constexpr int NW = BLOCK / 64;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const uint32_t chunk = (len + BLOCK - 1) / BLOCK;
    const uint32_t b0 = min(len, tid * chunk), b1 = min(len, b0 + chunk);
    uint32_t local = 0;
    for (uint32_t x = b0; x < b1; ++x) local += a[x];
    uint32_t incl = wave_inclusive_scan(local);
    uint32_t total;
    if (NW > 1) {
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        if (wid == 0) {
            uint32_t w = (lane < (uint32_t)NW) ? wsum[lane] : 0u;
            w = wave_inclusive_scan(w);
            if (lane < (uint32_t)NW) wsum[lane] = w;
        }
        __syncthreads();
        if (wid > 0) incl += wsum[wid - 1];
        total = wsum[NW - 1];
    } else {
        total = __shfl(incl, 63, 64);
    }
    uint32_t run = base + incl - local;
    for (uint32_t x = b0; x < b1; ++x) {
        const uint32_t v = a[x];
        a[x] = run;
        run += v;
    }
    __syncthreads();
    return total;
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

template <typename Elem, int BLOCK, int P>
__device__ void lds_tier_run(Elem *z, uint32_t n, uint32_t steps, uint32_t out_lo, Elem *out,
                             const Seg *seg, uint32_t nseg, uint32_t S, const StreamKey &key,
                             char *smem, uint32_t *wsum)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t lo = n - steps; // positions lo..n-1 take a step
    uint16_t *jb = reinterpret_cast<uint16_t *>(smem);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(smem + ((2u * n + 3u) & ~3u));
    uint16_t *head = reinterpret_cast<uint16_t *>(cnt + n + 1);

    for (uint32_t x = tid; x <= n; x += BLOCK) cnt[x] = 0;

    // dice: thread takes batch pairs (2m, 2m+1), which share Philox block m
    for (uint32_t m = tid; 2 * m < S; m += BLOCK) {
        uint64_t w[2];
        word_pair(m, key, w[0], w[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t s = 2 * m + h;
            if (s < S) {
                uint32_t i, k;
                uint64_t u;
                batch_at(s, seg, nseg, i, k, u);
                uint64_t r = accept_word(i, k, u, w[h], S, s, key);
                for (uint32_t l = 0; l < k; ++l) jb[i - 1 - l] = (uint16_t)mul_roll(i - l, r);
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

template <typename Elem, int BLOCK, int P>
__global__ __launch_bounds__(BLOCK) void k_lds_single(Elem *z, uint32_t n, uint32_t steps,
                                                      uint32_t out_lo, Elem *out, SegTable st,
                                                      StreamKey key)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ Seg seg[kMaxSegs];
    __shared__ uint32_t wsum[BLOCK / 64];
    if (threadIdx.x < st.nseg) seg[threadIdx.x] = st.seg[threadIdx.x];
    __syncthreads();
    lds_tier_run<Elem, BLOCK, P>(z, n, steps, out_lo, out, seg, st.nseg, st.S, key, smem, wsum);
}

template <typename Elem, int BLOCK, int P>
__global__ __launch_bounds__(BLOCK) void k_lds_batched(Elem *data, const uint64_t *offsets,
                                                       const uint32_t *items, DevSched sc,
                                                       uint64_t seed, uint64_t inst_base)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ SegTable st;
    __shared__ uint32_t wsum[BLOCK / 64];
    const uint32_t q = items ? items[blockIdx.x] : blockIdx.x;
    const uint64_t off = offsets[q];
    const uint32_t n = (uint32_t)(offsets[q + 1] - off);
    if (n <= 1) return; // the whole block leaves together
    if (threadIdx.x == 0) build_segments(n, n - 1, sc, st);
    __syncthreads();
    lds_tier_run<Elem, BLOCK, P>(data + off, n, n - 1, 0, nullptr, st.seg, st.nseg, st.S,
                                 make_key(seed, inst_base + q), smem, wsum);
}

// ---------------------------------------------------------------------------
// Global tier: the same steps with every array in device scratch.
// Layout for n: jj u32[n] | slot u32[n] | cnt u32[n+1] | head u32[n] |
//               bucket u32[n] | tiles u32[ntiles] | tmp Elem[n].
// ---------------------------------------------------------------------------

struct GArrays {
    uint32_t *jj, *slot, *cnt, *head, *bucket, *tiles;
    void *tmp;
};

__host__ __device__ inline uint64_t align16(uint64_t x) { return (x + 15) & ~(uint64_t)15; }

__host__ __device__ inline uint32_t scan_tiles(uint32_t n) { return (n + 1 + kScanTile - 1) / kScanTile; }

__host__ __device__ inline uint64_t garrays_bytes(uint64_t n, uint32_t eb)
{
    const uint64_t w = align16(4 * n);
    return 4 * w + align16(4 * (n + 1)) + align16(4 * (uint64_t)scan_tiles((uint32_t)n)) +
           align16(eb * n);
}

__host__ __device__ inline GArrays garrays(void *base, uint32_t n)
{
    char *p = static_cast<char *>(base);
    const uint64_t w = align16(4 * (uint64_t)n);
    GArrays g;
    g.jj = reinterpret_cast<uint32_t *>(p);
    p += w;
    g.slot = reinterpret_cast<uint32_t *>(p);
    p += w;
    g.cnt = reinterpret_cast<uint32_t *>(p);
    p += align16(4 * ((uint64_t)n + 1));
    g.head = reinterpret_cast<uint32_t *>(p);
    p += w;
    g.bucket = reinterpret_cast<uint32_t *>(p);
    p += w;
    g.tiles = reinterpret_cast<uint32_t *>(p);
    p += align16(4 * (uint64_t)scan_tiles(n));
    g.tmp = p;
    return g;
}

// Phase helpers, each over items idx = start, start+stride, ... < end.
__device__ __forceinline__ void g_init_range(const GArrays &g, uint32_t n, uint32_t start,
                                             uint32_t stride)
{
    for (uint32_t x = start; x <= n; x += stride) {
        g.cnt[x] = 0;
        if (x < n) g.head[x] = kNone32;
    }
}

__device__ __forceinline__ void g_dice_range(const GArrays &g, const Seg *seg, uint32_t nseg,
                                             uint32_t S, const StreamKey &key, uint32_t start,
                                             uint32_t stride)
{
    for (uint32_t m = start; 2 * m < S; m += stride) {
        uint64_t w[2];
        word_pair(m, key, w[0], w[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t s = 2 * m + h;
            if (s < S) {
                uint32_t i, k;
                uint64_t u;
                batch_at(s, seg, nseg, i, k, u);
                uint64_t r = accept_word(i, k, u, w[h], S, s, key);
                for (uint32_t l = 0; l < k; ++l) {
                    const uint32_t p = i - 1 - l;
                    const uint32_t a = mul_roll(i - l, r);
                    g.jj[p] = a;
                    if (a < p) {
                        g.slot[p] = atomicAdd(&g.cnt[a], 1u);
                        atomicMin(&g.head[a], p);
                    }
                }
            }
        }
    }
}

__device__ __forceinline__ void g_scatter_range(const GArrays &g, uint32_t n, uint32_t lo,
                                                uint32_t start, uint32_t stride)
{
    for (uint32_t p = lo + start; p < n; p += stride) {
        const uint32_t q = g.jj[p];
        if (q < p) g.bucket[g.cnt[q] + g.slot[p]] = p;
    }
}

template <typename Elem>
__device__ __forceinline__ void g_resolve_range(const GArrays &g, const Elem *z, Elem *dst,
                                                bool reversed, uint32_t n, uint32_t lo,
                                                uint32_t out_lo, uint32_t start, uint32_t stride)
{
    for (uint32_t p = out_lo + start; p < n; p += stride) {
        const uint32_t q = (p >= lo) ? g.jj[p] : p;
        uint32_t src;
        uint32_t x = p;
        bool walk = true;
        if (p >= lo && q != p) {
            uint32_t sc = kNone32;
            for (uint32_t e = g.cnt[q], e1 = g.cnt[q + 1]; e < e1; ++e) {
                const uint32_t v = g.bucket[e];
                if (v > p && v < sc) sc = v;
            }
            if (sc == kNone32) {
                walk = false;
                src = q;
            } else {
                x = sc;
            }
        }
        if (walk) {
            uint32_t h;
            for (uint32_t it = 0; it < n && (h = g.head[x]) != kNone32; ++it) x = h;
            src = x;
        }
        dst[reversed ? n - 1 - p : p] = z[src];
    }
}

// Device-wide kernels (grid-stride loops).
__global__ __launch_bounds__(256) void k_g_init(GArrays g, uint32_t n)
{
    g_init_range(g, n, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ __launch_bounds__(256) void k_g_dice(GArrays g, SegTable st, StreamKey key)
{
    __shared__ Seg seg[kMaxSegs];
    if (threadIdx.x < st.nseg) seg[threadIdx.x] = st.seg[threadIdx.x];
    __syncthreads();
    g_dice_range(g, seg, st.nseg, st.S, key, blockIdx.x * blockDim.x + threadIdx.x,
                 gridDim.x * blockDim.x);
}

__global__ __launch_bounds__(1024) void k_g_scan_tiles(GArrays g, uint32_t len)
{
    __shared__ uint32_t wsum[16];
    const uint32_t b0 = blockIdx.x * kScanTile;
    const uint32_t cnt = min(kScanTile, len - b0);
    uint32_t local = 0;
    for (uint32_t x = threadIdx.x; x < cnt; x += 1024) local += g.cnt[b0 + x];
    local = wave_inclusive_scan(local);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        g.tiles[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_g_scan_sums(GArrays g, uint32_t ntiles)
{
    __shared__ uint32_t wsum[16];
    block_scan_array<1024>(g.tiles, ntiles, 0, wsum);
}

__global__ __launch_bounds__(1024) void k_g_scan_apply(GArrays g, uint32_t len)
{
    __shared__ uint32_t wsum[16];
    const uint32_t b0 = blockIdx.x * kScanTile;
    const uint32_t cnt = min(kScanTile, len - b0);
    block_scan_array<1024>(g.cnt + b0, cnt, g.tiles[blockIdx.x], wsum);
}

__global__ __launch_bounds__(256) void k_g_scatter(GArrays g, uint32_t n, uint32_t lo)
{
    g_scatter_range(g, n, lo, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <typename Elem>
__global__ __launch_bounds__(256) void k_g_resolve(GArrays g, const Elem *z, Elem *dst,
                                                   int reversed, uint32_t n, uint32_t lo,
                                                   uint32_t out_lo)
{
    g_resolve_range<Elem>(g, z, dst, reversed != 0, n, lo, out_lo,
                          blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <typename Elem>
__global__ __launch_bounds__(256) void k_g_copy(Elem *z, const Elem *tmp, uint32_t n)
{
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
        z[p] = tmp[p];
}

// Barrier between phases that communicate through device memory, including
// atomics performed in L2: an agent-scope fence on each side makes the
// writes visible and drops stale lines from the CU's vector cache.
__device__ __forceinline__ void phase_barrier()
{
    __threadfence();
    __syncthreads();
    __threadfence();
}

// One workgroup per shuffle with arrays in scratch (batched, large n).
template <typename Elem>
__global__ __launch_bounds__(kWgThreads) void k_big_batched(Elem *data, const uint64_t *offsets,
                                                            const uint32_t *items, DevSched sc,
                                                            uint64_t seed, uint64_t inst_base,
                                                            char *scratch,
                                                            const uint64_t *scratch_off)
{
    __shared__ SegTable st;
    __shared__ uint32_t wsum[kWgThreads / 64];
    const uint32_t q = items[blockIdx.x];
    const uint64_t off = offsets[q];
    const uint32_t n = (uint32_t)(offsets[q + 1] - off);
    if (n <= 1) return;
    Elem *z = data + off;
    const GArrays g = garrays(scratch + scratch_off[blockIdx.x], n);
    Elem *tmp = static_cast<Elem *>(g.tmp);
    const StreamKey key = make_key(seed, inst_base + q);
    const uint32_t tid = threadIdx.x;
    if (tid == 0) build_segments(n, n - 1, sc, st);
    g_init_range(g, n, tid, kWgThreads);
    phase_barrier();
    g_dice_range(g, st.seg, st.nseg, st.S, key, tid, kWgThreads);
    phase_barrier();
    block_scan_array<kWgThreads>(g.cnt, n + 1, 0, wsum);
    phase_barrier();
    g_scatter_range(g, n, 1, tid, kWgThreads);
    phase_barrier();
    g_resolve_range<Elem>(g, z, tmp, false, n, 1, 0, tid, kWgThreads);
    phase_barrier();
    for (uint32_t p = tid; p < n; p += kWgThreads) z[p] = tmp[p];
}

uint32_t grid_for(uint64_t work, uint32_t block)
{
    uint64_t b = (work + block - 1) / block;
    if (b < 1) b = 1;
    if (b > (1u << 20)) b = 1u << 20;
    return (uint32_t)b;
}

template <typename Elem>
hipError_t lds_single_t(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, void *out,
                        const DevSched &sc, StreamKey key, hipStream_t stream)
{
    SegTable st;
    build_segments(n, steps, sc, st);
    const uint32_t bytes = lds_bytes(n);
    k_lds_single<Elem, kWgThreads, kWgP><<<1, kWgThreads, bytes, stream>>>(static_cast<Elem *>(data), n, steps, out_lo,
                                           static_cast<Elem *>(out), st, key);
    return hipGetLastError();
}

template <typename Elem>
hipError_t global_single_t(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, void *out,
                           const DevSched &sc, StreamKey key, void *scratch, hipStream_t stream)
{
    SegTable st;
    build_segments(n, steps, sc, st);
    const GArrays g = garrays(scratch, n);
    const uint32_t lo = n - steps;
    if (!out) out_lo = 0;
    Elem *z = static_cast<Elem *>(data);
    k_g_init<<<grid_for((uint64_t)n + 1, 256), 256, 0, stream>>>(g, n);
    k_g_dice<<<grid_for((st.S + 1) / 2, 256), 256, 0, stream>>>(g, st, key);
    const uint32_t ntiles = scan_tiles(n);
    k_g_scan_tiles<<<ntiles, 1024, 0, stream>>>(g, n + 1);
    k_g_scan_sums<<<1, 1024, 0, stream>>>(g, ntiles);
    k_g_scan_apply<<<ntiles, 1024, 0, stream>>>(g, n + 1);
    k_g_scatter<<<grid_for(steps, 256), 256, 0, stream>>>(g, n, lo);
    if (out) {
        k_g_resolve<Elem><<<grid_for(n - out_lo, 256), 256, 0, stream>>>(
            g, z, static_cast<Elem *>(out), 1, n, lo, out_lo);
    } else {
        Elem *tmp = static_cast<Elem *>(g.tmp);
        k_g_resolve<Elem><<<grid_for(n, 256), 256, 0, stream>>>(g, z, tmp, 0, n, lo, 0);
        k_g_copy<Elem><<<grid_for(n, 256), 256, 0, stream>>>(z, tmp, n);
    }
    return hipGetLastError();
}

template <typename Elem, int BLOCK, int P>
hipError_t batched_lds_t(void *data, const uint64_t *offsets, const uint32_t *items,
                         uint32_t nitems, uint32_t max_n, const DevSched &sc, uint64_t seed,
                         uint64_t inst_base, hipStream_t stream)
{
    if (nitems == 0) return hipSuccess;
    const uint32_t bytes = lds_bytes(max_n);
    k_lds_batched<Elem, BLOCK, P><<<nitems, BLOCK, bytes, stream>>>(static_cast<Elem *>(data), offsets, items, sc, seed,
                                           inst_base);
    return hipGetLastError();
}

} // namespace

uint32_t lds_tier_max_n() { return kWgThreads * kWgP; }

hipError_t prepare_shuffle_kernels()
{
    const int wg = (int)lds_bytes(kWgThreads * kWgP), wave = (int)lds_bytes(64 * kWaveP);
    const void *fns[] = {(const void *)k_lds_single<uint32_t, kWgThreads, kWgP>,
                         (const void *)k_lds_single<uint64_t, kWgThreads, kWgP>,
                         (const void *)k_lds_batched<uint32_t, kWgThreads, kWgP>,
                         (const void *)k_lds_batched<uint64_t, kWgThreads, kWgP>,
                         (const void *)k_lds_batched<uint32_t, 64, kWaveP>,
                         (const void *)k_lds_batched<uint64_t, 64, kWaveP>};
    const int bytes[] = {wg, wg, wg, wg, wave, wave};
    for (int f = 0; f < 6; ++f) {
        const hipError_t e =
            hipFuncSetAttribute(fns[f], hipFuncAttributeMaxDynamicSharedMemorySize, bytes[f]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
uint32_t wave_tier_max_n() { return 64 * kWaveP; }
uint64_t global_scratch_bytes(uint64_t n, uint32_t eb) { return garrays_bytes(n, eb); }

hipError_t launch_lds_single(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, uint32_t eb,
                             void *out, const DevSched &sc, StreamKey key, hipStream_t stream)
{
    if (n > lds_tier_max_n() || steps == 0 || steps >= n || out_lo > n - steps)
        return hipErrorInvalidValue;
    return eb == 4 ? lds_single_t<uint32_t>(data, n, steps, out_lo, out, sc, key, stream)
                   : lds_single_t<uint64_t>(data, n, steps, out_lo, out, sc, key, stream);
}

hipError_t launch_global_single(void *data, uint32_t n, uint32_t steps, uint32_t out_lo,
                                uint32_t eb, void *out, const DevSched &sc, StreamKey key,
                                void *scratch, hipStream_t stream)
{
    if (steps == 0 || steps >= n || out_lo > n - steps) return hipErrorInvalidValue;
    return eb == 4 ? global_single_t<uint32_t>(data, n, steps, out_lo, out, sc, key, scratch, stream)
                   : global_single_t<uint64_t>(data, n, steps, out_lo, out, sc, key, scratch,
                                               stream);
}

hipError_t launch_batched_wave(void *data, const uint64_t *offsets, const uint32_t *items,
                               uint32_t nitems, uint32_t max_n, uint32_t eb, const DevSched &sc,
                               uint64_t seed, uint64_t inst_base, hipStream_t stream)
{
    if (max_n > wave_tier_max_n()) return hipErrorInvalidValue;
    return eb == 4 ? batched_lds_t<uint32_t, 64, kWaveP>(data, offsets, items, nitems, max_n, sc,
                                                         seed, inst_base, stream)
                   : batched_lds_t<uint64_t, 64, kWaveP>(data, offsets, items, nitems, max_n, sc,
                                                         seed, inst_base, stream);
}

hipError_t launch_batched_wg(void *data, const uint64_t *offsets, const uint32_t *items,
                             uint32_t nitems, uint32_t max_n, uint32_t eb, const DevSched &sc,
                             uint64_t seed, uint64_t inst_base, hipStream_t stream)
{
    if (max_n > lds_tier_max_n()) return hipErrorInvalidValue;
    return eb == 4 ? batched_lds_t<uint32_t, kWgThreads, kWgP>(data, offsets, items, nitems, max_n,
                                                               sc, seed, inst_base, stream)
                   : batched_lds_t<uint64_t, kWgThreads, kWgP>(data, offsets, items, nitems, max_n,
                                                               sc, seed, inst_base, stream);
}

hipError_t launch_batched_big(void *data, const uint64_t *offsets, const uint32_t *items,
                              uint32_t nitems, uint32_t eb, const DevSched &sc, uint64_t seed,
                              uint64_t inst_base, void *scratch, const uint64_t *scratch_off,
                              hipStream_t stream)
{
    if (nitems == 0) return hipSuccess;
    if (eb == 4)
        k_big_batched<uint32_t><<<nitems, kWgThreads, 0, stream>>>(
            static_cast<uint32_t *>(data), offsets, items, sc, seed, inst_base,
            static_cast<char *>(scratch), scratch_off);
    else
        k_big_batched<uint64_t><<<nitems, kWgThreads, 0, stream>>>(
            static_cast<uint64_t *>(data), offsets, items, sc, seed, inst_base,
            static_cast<char *>(scratch), scratch_off);
    return hipGetLastError();
}

} // namespace brr
