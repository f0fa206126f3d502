// Internal interfaces between the host API (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "brr.h"
#include "device.hpp"

namespace brr {

// Checks once per device that the current device is a gfx950 and sets up
// the library's per-device state.
brr_status ensure_device();

// Device scratch of single calls, one buffer per (device, stream): at least
// `bytes`, valid while `hold` (the buffer's lock, taken here) is held, which
// the caller keeps until its kernels are enqueued. Grown (after the
// stream's earlier work ends) when a call needs more; kept for later calls
// on the stream, whose stream order keeps them from overlapping.
brr_status stream_scratch(hipStream_t s, uint64_t bytes, std::unique_lock<std::mutex> &hold,
                          void **out);
// Frees the current device's scratch buffer of stream s, whose work must
// have ended (a stream's owner calls it before destroying the stream).
brr_status drop_stream_scratch(hipStream_t s);

// A validated schedule in the form the kernels read (thresholds clamped to
// 32 bits: every shuffle here has n < 2^32).
struct DevSched {
    uint32_t nsteps, tail;
    uint32_t thr[16];
    uint32_t k[16];
    uint64_t u[16];
    uint64_t u_tail;
    uint32_t form[16]; // BRR_FORM_* of each step (the tail batch multiplies)
    uint32_t words;    // BRR_WORDS_*
};

// The kernels' form of a schedule that brr_schedule_check accepted.
inline DevSched dev_schedule(const brr_schedule &sc)
{
    DevSched d{};
    d.nsteps = sc.nsteps;
    d.tail = sc.tail;
    for (uint32_t g = 0; g < sc.nsteps; ++g) {
        d.thr[g] = sc.step[g].n_above < 0xFFFFFFFFull ? (uint32_t)sc.step[g].n_above : 0xFFFFFFFFu;
        d.k[g] = sc.step[g].k;
        d.u[g] = sc.step[g].u0;
        d.form[g] = sc.step[g].form;
    }
    d.u_tail = sc.u_tail;
    d.words = sc.words;
    return d;
}

// A run of cnt consecutive batches (batch indices s0 .. s0+cnt-1) of k dice
// each; the first starts with i0 elements left, each next one k fewer. u is
// the guard of Algorithm 4 (0 = compare against the exact product); form is
// how the batches take their dice (BRR_FORM_*).
struct Seg {
    uint32_t s0, i0, k, cnt;
    uint64_t u;
    uint32_t form, pad;
};

constexpr int kMaxSegs = 18; // 16 steps + one truncated batch + the last batch

struct SegTable {
    Seg seg[kMaxSegs];
    uint32_t nseg;
    uint32_t S;     // batches in total
    uint32_t words; // BRR_WORDS_* of the schedule
};

// Batches of the first `steps` Fisher-Yates steps of an n-element shuffle
// under schedule sc (steps = n - 1 for a full shuffle): while more than
// thr[g] elements remain, batches of k[g] dice; a batch that would pass
// `steps` keeps only the dice it needs; then, with a tail, one batch of
// i - 1 dice. Calls f(Seg) for each run in order and returns the number of
// batches. Requires thr[g] + 1 >= k[g] (checked on the host).
template <typename F>
__host__ __device__ inline uint32_t walk_segments(uint32_t n, uint32_t steps, const DevSched &sc,
                                                  F &&f)
{
    uint32_t i = n, s = 0, done = 0;
    for (uint32_t g = 0; g < sc.nsteps && done < steps; ++g) {
        const uint32_t thr = sc.thr[g], k = sc.k[g];
        if (i <= thr) continue;
        const uint32_t cnt = (uint32_t)(((uint64_t)(i - thr) + k - 1) / k);
        const uint32_t left = steps - done;
        uint32_t nb = cnt;
        if ((uint64_t)nb * k > left) nb = left / k;
        if (nb) {
            f(Seg{s, i, k, nb, sc.u[g], sc.form[g], 0});
            s += nb;
            i -= nb * k;
            done += nb * k;
        }
        if (nb < cnt && done < steps) {
            const uint32_t kk = steps - done;
            f(Seg{s, i, kk, 1, sc.u[g], sc.form[g], 0});
            s += 1;
            i -= kk;
            done += kk;
        }
    }
    if (sc.tail && i > 1 && done < steps) {
        uint32_t kk = i - 1;
        if (kk > steps - done) kk = steps - done;
        f(Seg{s, i, kk, 1, sc.u_tail, BRR_FORM_MULTIPLY, 0});
        s += 1;
        done += kk;
    }
    return s;
}

// The runs of walk_segments as a table.
__host__ __device__ inline void build_segments(uint32_t n, uint32_t steps, const DevSched &sc,
                                               SegTable &t)
{
    uint32_t ns = 0;
    t.S = walk_segments(n, steps, sc, [&](const Seg &g) { t.seg[ns++] = g; });
    t.nseg = ns;
    t.words = sc.words;
}

// Whether a device pointer is not aligned to its element size.
inline bool misaligned(const void *p, uint32_t bytes)
{
    return (reinterpret_cast<uintptr_t>(p) & (uintptr_t)(bytes - 1)) != 0;
}

// Kernel launchers (dice.hip, shuffle.hip).
hipError_t launch_dice(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                       StreamKey key, uint32_t *status, hipStream_t stream);
// Known bounds of a dice stream (Algorithm 2): group g rolls b[0..k).
struct BoundTuple {
    uint32_t b[8];
};
hipError_t launch_dice_const(const BoundTuple &tb, uint32_t *out, uint64_t count, uint32_t k,
                             StreamKey key, uint64_t t_full, uint64_t t_last, hipStream_t stream);
// The dice stream in the division form (dice.hip).
hipError_t launch_dice_div(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                           StreamKey key, uint32_t *status, hipStream_t stream);
// The dice stream with ChaCha20 words (dice_chacha.hip).
// rec: device memory of chacha_record_bytes(count, k) bytes for the
// records of rejected groups, or nullptr (every group rerolls in place).
uint64_t chacha_record_bytes(uint64_t count, uint32_t k);
hipError_t launch_dice_chacha(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                              StreamKey key, uint32_t *status, void *rec, hipStream_t stream);
// The dice stream at word width 32 (dice32.hip).
hipError_t launch_dice32(const uint32_t *bounds, uint32_t *out, uint64_t count, uint32_t k,
                         StreamKey key, uint32_t *status, hipStream_t stream);

// Largest n that one workgroup shuffles with its index arrays in LDS.
uint32_t lds_tier_max_n();
// Largest n of the one-wavefront-per-shuffle tier.
uint32_t wave_tier_max_n();
// Raises the dynamic-LDS limit of the LDS-tier kernels (once per device).
hipError_t prepare_shuffle_kernels();

// A device-side instance claim. With counter set, the first kernel of a
// launch takes c = *counter, stores c + 1 back and base + c into *slot (one
// thread), and the launch's instance is inst + base + c. Claims on one
// stream therefore follow stream order. counter == nullptr and slot set:
// the instance was claimed by an earlier kernel on the stream, and is
// inst + *slot. Neither set: no claim.
struct DevClaim {
    uint64_t *counter;
    uint64_t *slot;
    uint64_t base;
};

// One shuffle (steps = n - 1, out = nullptr, in place) or one sample
// (out != nullptr: out[n-1-p] = final z[p] for out_lo <= p < n, the input
// untouched) by one workgroup with its index arrays in LDS;
// n <= lds_tier_max_n(), 1 <= steps < n, out_lo <= n - steps.
hipError_t launch_lds_single(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, uint32_t eb,
                             void *out, const DevSched &sc, uint64_t seed, uint64_t inst,
                             const DevClaim &claim, hipStream_t stream);

// The arguments a plan's run binds: the payload, its CSR offsets, the seed
// and the instance of shuffle 0. The batched kernels read them from the
// plan's device block, which a kernel enqueued before each run writes, so
// that a captured graph replays with other arguments.
struct RunArgs {
    void *data;
    const uint64_t *offsets;
    uint64_t seed, inst;
};
// Pointers that reach a kernel through memory (an argument block) rather
// than as kernel arguments are generic to the compiler, which then accesses
// them with flat instructions; those count against the LDS wait counter as
// well, so every wait for an LDS read also waits for the global loads in
// flight. Data buffers are always device memory: kernels hold them as
// global_t pointers, which compile to global loads and stores.
template <typename T>
using global_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ global_t<T> *as_global(T *p)
{
    return (global_t<T> *)p;
}

// Writes a run's arguments into a plan's device block, on the stream.
hipError_t launch_set_args(RunArgs *dev, const RunArgs &val, hipStream_t stream);

// One item of the device-wide tier: the array at element offset data_off of
// the shared data pointer, n elements, the first `steps` Fisher-Yates steps
// (n - 1 for a shuffle), its positions at pos_base in the index arrays, its
// word-stream instance. out == nullptr: shuffle in place; else a sample:
// out[n-1-p] = final z[p] for out_lo <= p < n.
struct GItem {
    uint64_t data_off, pos_base, inst;
    uint32_t n, steps, out_lo, pad;
    void *out;
};

// A device-wide problem: items, their segment tables and the prefix sums of
// their positions and batch pairs (device arrays of nitems + 1), or, for a
// single item, host copies of its descriptor (one_item/one_seg).
struct GTierArgs {
    void *data;
    uint32_t eb;
    uint64_t seed;
    uint64_t inst_base; // item q uses instance inst_base + items[q].inst
    DevClaim claim;     // if set, the claimed instance is added to inst_base
    uint32_t nitems;
    uint64_t npos, npairs;
    const GItem *items;      // device
    const SegTable *segs;    // device
    const uint64_t *pos_base, *pair_base; // device
    const uint32_t *pos_tile, *pair_tile; // device: item of index 2^shift * t
    const GItem *one_item;   // host, nitems == 1
    const SegTable *one_seg; // host, nitems == 1
    void *scratch;           // gtier_scratch_bytes(npos, eb)
    uint32_t words;          // BRR_WORDS_* of the items' schedule
    const RunArgs *dyn;      // if set, data, seed and inst_base are read from it (plans)
};
uint64_t gtier_scratch_bytes(uint64_t npos, uint32_t eb);
// Positions (summed over items) one device-wide launch takes: indices are u32.
constexpr uint64_t kMaxGtierPositions = 0xFFFFFFFFull;

// One shuffle (out == nullptr) or sample of m = n - out_lo elements through
// the LDS tier or, for n > lds_tier_max_n(), the device-wide tier (a
// shuffle) or the sparse sample path (O(m) work and scratch), with
// one_scratch_bytes(n, eb, m) bytes of scratch (m = 0 for a shuffle): the
// caller's (scratch != nullptr; nothing is allocated) or taken from the
// stream-ordered allocator and freed on the stream (whose allocation or
// release waits for the device here: the library's own callers pass the
// stream's scratch buffer, see stream_scratch).
uint64_t one_scratch_bytes(uint64_t n, uint32_t eb, uint64_t m = 0);
hipError_t launch_one(void *data, uint32_t n, uint32_t steps, uint32_t out_lo, uint32_t eb,
                      void *out, const DevSched &ds, uint64_t seed, uint64_t inst,
                      const DevClaim &claim, hipStream_t s, void *scratch = nullptr);
uint32_t gtier_tile_shift(); // log2 of the indices per tile-table entry
hipError_t launch_gtier(const GTierArgs &a, hipStream_t stream);

// Independent requests in one launch (the server's small requests): each
// a shuffle (out == nullptr, steps = n - 1, out_lo = 0) or a sample of
// separate arrays, n <= lds_class_max_n(c) for the launch's class c, its
// instance in slots[slot].
struct ReqDesc {
    void *data, *out;
    uint32_t n, steps, out_lo, slot;
};
constexpr uint32_t kMaxFusedRequests = 32;
struct ReqBatch {
    ReqDesc r[kMaxFusedRequests];
    uint32_t count;
};
// The LDS class of an array of n elements (-1 above lds_tier_max_n()).
int lds_request_class(uint32_t n);
hipError_t launch_lds_requests(int c, uint32_t eb, const ReqBatch &b, uint32_t max_n,
                               const DevSched &sc, uint64_t seed, const uint64_t *slots,
                               hipStream_t stream);

// Batched shuffles of one LDS size class: one block per shuffle with its
// index arrays in LDS, class c holding n <= lds_class_max_n(c) (0: one
// wavefront, n <= wave_tier_max_n(); kLdsClasses - 1: 1024 threads,
// n <= lds_tier_max_n()). items: device u32[nitems] of shuffle indices into
// the CSR offsets; max_n: the largest n among them (sizes the LDS).
constexpr int kLdsClasses = 5;
uint32_t lds_class_max_n(int c);
hipError_t launch_batched_lds(int c, const RunArgs *b, const uint32_t *items, uint32_t nitems,
                              uint32_t max_n, uint32_t eb, const DevSched &sc, hipStream_t stream);
// Lane tier: one lane per in-place shuffle of 2 <= n <= lane_tier_max_n()
// (items sorted by size for the plan), max_n = largest n among the items.
uint32_t lane_tier_max_n();
hipError_t launch_batched_lane(const RunArgs *b, const uint32_t *items, uint32_t nitems,
                               uint32_t max_n, uint32_t eb, const DevSched &sc, hipStream_t stream);
// Peel tier: one workgroup per in-place shuffle of 2 <= n <=
// peel_tier_max_n(), processed top-down in LDS-sized peels (the plan sends
// it the arrays too large for its LDS classes).
uint32_t peel_tier_max_n();
hipError_t launch_batched_peel(const RunArgs *b, const uint32_t *items, uint32_t nitems,
                               uint32_t eb, const DevSched &sc, hipStream_t stream);

} // namespace brr
