// Host side of libbrr: argument checks, schedules, the per-device status
// word, plans for batched shuffles (size classes, scratch, hip graphs) and
// the extern "C" entry points declared in brr.h.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "brr.h"
#include "internal.hpp"

using namespace brr;

// Scratch of brr_shuffle_noalloc (file scope; see noalloc_scratch).
static __device__ __align__(256) char scratch[BRR_NOALLOC_SCRATCH_BYTES];

namespace {

typedef unsigned __int128 u128;

constexpr int kMaxDevices = 64;

struct DeviceState {
    bool checked = false;
    bool ok = false;
    uint32_t *status = nullptr;
};

std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

// Scratch of brr_shuffle_noalloc: one array per device, held while the
// process lives. Host code never passes its name (a host-side stand-in) to a
// kernel or a copy; it uses the device address that hipGetSymbolAddress
// returns for the current device (noalloc_scratch below).
constexpr uint64_t kNoAllocScratchBytes = BRR_NOALLOC_SCRATCH_BYTES;

struct NoAllocState {
    bool done = false;
    void *ptr = nullptr;
};
NoAllocState g_noalloc[kMaxDevices];

// The device address of the current device's scratch array, looked up once
// per device (with that device current) and kept.
brr_status noalloc_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BRR_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    NoAllocState &d = g_noalloc[dev];
    if (!d.done) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BRR_EHIP;
        d.ptr = ptr;
        d.done = true;
    }
    *out = d.ptr;
    return BRR_OK;
}

// Checks once per device that it is a gfx950 and allocates its status word.
brr_status device_ready(uint32_t **status_out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BRR_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState &d = g_dev[dev];
    if (!d.checked) {
        d.checked = true;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return BRR_EDEVICE;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BRR_EDEVICE;
        if (hipMalloc(reinterpret_cast<void **>(&d.status), sizeof(uint32_t)) != hipSuccess)
            return BRR_ENOMEM;
        if (hipMemset(d.status, 0, sizeof(uint32_t)) != hipSuccess) return BRR_EHIP;
        if (hipDeviceSynchronize() != hipSuccess) return BRR_EHIP;
        if (prepare_shuffle_kernels() != hipSuccess) return BRR_EHIP;
        d.ok = true;
    }
    if (!d.ok) return BRR_EDEVICE;
    if (status_out) *status_out = d.status;
    return BRR_OK;
}

brr_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return BRR_OK;
    return e == hipErrorOutOfMemory ? BRR_ENOMEM : BRR_EHIP;
}

// n^(falling k), or 2^64 + 1 for anything above 2^64.
u128 falling(uint64_t n, uint64_t k)
{
    const u128 cap = ((u128)1 << 64) + 1;
    u128 p = 1;
    for (uint64_t l = 0; l < k; ++l) {
        p *= (u128)(n - l);
        if (p > cap) return cap;
    }
    return p;
}

const brr_schedule &paper6()
{
    static brr_schedule s = [] {
        brr_schedule t;
        brr_schedule_paper(6, &t);
        return t;
    }();
    return s;
}

// Walks the batches of the first `steps` steps of an n-element shuffle one
// segment at a time. With check set, verifies that the first (largest)
// batch of every segment has a product of at most 2^64 and that a given
// upper bound covers it. Returns the number of batches, or sets *err.
uint64_t walk_schedule(const brr_schedule &sc, uint64_t n, uint64_t steps, bool check,
                       brr_status *err)
{
    const u128 two64 = (u128)1 << (sc.words == BRR_WORDS_PHILOX32 ? 32 : 64); // 2^L
    uint64_t i = n, s = 0, done = 0;
    for (uint32_t g = 0; g < sc.nsteps && done < steps; ++g) {
        const uint64_t thr = sc.step[g].n_above, k = sc.step[g].k;
        if (i <= thr) continue;
        const uint64_t cnt = (i - thr + k - 1) / k;
        const uint64_t left = steps - done;
        const uint64_t first_k = std::min<uint64_t>(k, left);
        if (check) {
            const u128 p = falling(i, first_k);
            if (p > two64) { *err = BRR_EOVERFLOW; return 0; }
            if (sc.step[g].u0 && (u128)sc.step[g].u0 < p) { *err = BRR_EINVAL; return 0; }
        }
        uint64_t nb = cnt;
        if (nb * k > left) nb = left / k;
        s += nb;
        i -= nb * k;
        done += nb * k;
        if (nb < cnt && done < steps) {
            const uint64_t kk = steps - done;
            s += 1;
            i -= kk;
            done += kk;
        }
    }
    if (sc.tail && i > 1 && done < steps) {
        const uint64_t kk = std::min<uint64_t>(i - 1, steps - done);
        if (check) {
            const u128 p = falling(i, kk);
            if (p > two64) { *err = BRR_EOVERFLOW; return 0; }
            if (sc.u_tail && (u128)sc.u_tail < p) { *err = BRR_EINVAL; return 0; }
        }
        s += 1;
        done += kk;
    }
    if (check && done < steps) { *err = BRR_EINVAL; return 0; }
    return s;
}

brr_status check_structure(const brr_schedule &sc)
{
    if (sc.nsteps == 0 || sc.nsteps > BRR_MAX_STEPS) return BRR_EINVAL;
    if (sc.words > BRR_WORDS_CHACHA20 || sc.reserved != 0) return BRR_EINVAL;
    for (uint32_t g = 0; g < sc.nsteps; ++g) {
        const brr_step &st = sc.step[g];
        if (st.k == 0 || st.k > BRR_MAX_K) return BRR_EINVAL;
        if (st.form != BRR_FORM_MULTIPLY && st.form != BRR_FORM_DIVISION) return BRR_EINVAL;
        if (st.form == BRR_FORM_DIVISION && sc.words == BRR_WORDS_PHILOX32) return BRR_EINVAL;
        if (st.n_above + 1 < st.k) return BRR_EINVAL;
        if (g > 0 && st.n_above > sc.step[g - 1].n_above) return BRR_EINVAL;
    }
    return BRR_OK;
}

brr_status check_for(const brr_schedule &sc, uint64_t n, uint64_t steps)
{
    brr_status e = check_structure(sc);
    if (e != BRR_OK) return e;
    if (n <= 1) return BRR_OK;
    e = BRR_OK;
    walk_schedule(sc, n, steps, true, &e);
    return e;
}

// Every shuffle of at most max_n elements (and every sample from one), as a
// plan or a server meets them. check_for(max_n) alone does not cover them:
// where a segment's first batch falls depends on n, so a guard that covers
// the first batch of the largest shuffle can be below the product of a
// smaller one's. The largest batch a segment can roll is its first at the
// largest size it can start from, min(max_n, n_above of the segment before)
// (k dice, fewer where fewer steps remain); the tail's is at min(max_n, the
// last n_above). Falling products grow with the size, so these bound every
// batch of every such shuffle; check_for(max_n) adds the completeness check
// (no element left without a step), and without a tail the last step must
// run down to one element (n_above <= 1), else the smallest shuffles stop
// short.
brr_status check_upto(const brr_schedule &sc, uint64_t max_n)
{
    brr_status e = check_for(sc, max_n, max_n ? max_n - 1 : 0);
    if (e != BRR_OK || max_n <= 1) return e;
    const u128 two_l = (u128)1 << (sc.words == BRR_WORDS_PHILOX32 ? 32 : 64);
    uint64_t top = max_n;
    for (uint32_t g = 0; g < sc.nsteps; ++g) {
        const brr_step &st = sc.step[g];
        if (top > st.n_above && top > 1) {
            const u128 p = falling(top, std::min<uint64_t>(st.k, top - 1));
            if (p > two_l) return BRR_EOVERFLOW;
            if (st.u0 && (u128)st.u0 < p) return BRR_EINVAL;
        }
        top = std::min<uint64_t>(top, st.n_above);
    }
    if (sc.tail && top > 1) {
        const u128 p = falling(top, top - 1);
        if (p > two_l) return BRR_EOVERFLOW;
        if (sc.u_tail && (u128)sc.u_tail < p) return BRR_EINVAL;
    }
    // without a tail a shuffle of top elements (2 <= top <= the last
    // n_above) would roll no batch at all
    if (!sc.tail && top > 1) return BRR_EINVAL;
    return BRR_OK;
}

DevSched to_dev(const brr_schedule &sc) { return dev_schedule(sc); }

// Scratch of single calls (brr_shuffle, brr_sample, brr_dice_chacha, the
// server's large requests): one buffer per (device, stream), grown to the
// largest need seen on that stream and kept for the calls after it. Stream
// order keeps the calls on one stream from overlapping; the buffer's lock
// keeps two host threads from enqueueing on it while it is replaced. The
// stream-ordered allocator would do the same job per call, but on this
// stack its allocation or release waits for the device, which made every
// such call block the host until its kernels had run.
struct StreamScratch {
    int dev = -1;
    hipStream_t stream = nullptr;
    void *ptr = nullptr;
    uint64_t bytes = 0;
    std::mutex mu;
};
std::mutex g_scratch_mu;
std::vector<StreamScratch *> g_scratch; // entries live as long as the process

} // namespace

brr_status brr::ensure_device() { return device_ready(nullptr); }

brr_status brr::stream_scratch(hipStream_t s, uint64_t bytes, std::unique_lock<std::mutex> &hold,
                               void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return BRR_EDEVICE;
    StreamScratch *e = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        for (StreamScratch *x : g_scratch)
            if (x->dev == dev && x->stream == s) e = x;
        if (!e) {
            e = new (std::nothrow) StreamScratch;
            if (!e) return BRR_ENOMEM;
            e->dev = dev;
            e->stream = s;
            g_scratch.push_back(e);
        }
    }
    hold = std::unique_lock<std::mutex>(e->mu);
    if (e->bytes < bytes) {
        if (e->ptr) { // earlier calls on the stream may still read the old buffer
            if (hipStreamSynchronize(s) != hipSuccess) return BRR_EHIP;
            (void)hipFree(e->ptr);
            e->ptr = nullptr;
            e->bytes = 0;
        }
        if (hipMalloc(&e->ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            e->ptr = nullptr;
            return BRR_ENOMEM;
        }
        e->bytes = bytes;
    }
    *out = e->ptr;
    return BRR_OK;
}

brr_status brr::drop_stream_scratch(hipStream_t s)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return BRR_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    brr_status st = BRR_OK;
    for (StreamScratch *e : g_scratch) {
        if (e->dev != dev || e->stream != s) continue;
        std::lock_guard<std::mutex> hold(e->mu);
        if (e->ptr && hipFree(e->ptr) != hipSuccess) st = BRR_EHIP;
        e->ptr = nullptr;
        e->bytes = 0;
    }
    return st;
}

brr_status brr_release_scratch(void)
{
    // Streams may have been destroyed since their buffers were made, so the
    // wait is for each device as a whole, never for a stream handle.
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    int cur = -1;
    (void)hipGetDevice(&cur);
    brr_status st = BRR_OK;
    std::vector<int> synced;
    for (StreamScratch *e : g_scratch) {
        std::lock_guard<std::mutex> hold(e->mu);
        if (!e->ptr) continue;
        if (std::find(synced.begin(), synced.end(), e->dev) == synced.end()) {
            if (hipSetDevice(e->dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
                st = BRR_EHIP;
                continue;
            }
            synced.push_back(e->dev);
        } else if (hipSetDevice(e->dev) != hipSuccess) {
            st = BRR_EHIP;
            continue;
        }
        if (hipFree(e->ptr) != hipSuccess) st = BRR_EHIP;
        e->ptr = nullptr;
        e->bytes = 0;
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    return st;
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------

namespace {
// lane, the LDS size classes, peel, device-wide
constexpr int kTiers = 3 + kLdsClasses;
}

struct brr_plan {
    int device = -1;
    uint32_t eb = 4;
    uint64_t count = 0;
    brr_schedule sched;
    DevSched ds;
    brr_mapping map;
    std::vector<uint64_t> h_off;
    // classification (made on first run, after the mapping is final)
    bool classified = false;
    uint32_t n_lane = 0, n_peel = 0, n_big = 0, lane_max_n = 0;
    uint32_t n_cls[kLdsClasses] = {}, max_cls[kLdsClasses] = {};
    uint32_t *d_items = nullptr; // [lane items | LDS class 0, 1, ... items | peel items]
    // device-wide tier for the shuffles too large for LDS
    GItem *d_gitems = nullptr;
    SegTable *d_gsegs = nullptr;
    uint64_t *d_gbase = nullptr; // pos_base[n_big + 1] | pair_base[n_big + 1]
    uint32_t *d_gtile = nullptr; // item of each position tile | of each pair tile
    uint64_t g_pos_tiles = 0;
    uint64_t g_npos = 0, g_npairs = 0;
    void *d_scratch = nullptr;
    // size classes run side by side: each non-empty class but the last on a
    // branch stream forked from and joined back to the caller's stream
    bool fork_classes = true; // off for one-shot plans: streams cost more than they save
    hipStream_t branch[kTiers - 1] = {};
    hipEvent_t fork = nullptr, join[kTiers - 1] = {};
    // graph of the launch sequence, captured on the first run; its kernels
    // read the run's buffers, seed and instance from d_args, which a kernel
    // enqueued before every replay writes
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    RunArgs *d_args = nullptr;
    RunArgs last_args{};     // what d_args holds (or will, once the stream gets there)
    bool args_written = false;
    uint32_t captures = 0;
    // recorded on the caller's stream after every run: the executable graph
    // (and everything else the plan owns) is released or replaced only
    // after the last run that may use it has finished
    hipEvent_t done = nullptr;
    bool ran = false; // done has been recorded at least once
    // serialises host calls on the plan (runs, mapping, tuning)
    std::mutex mu;
};

namespace {

void release(brr_plan *p)
{
    if (p->done) {
        (void)hipEventSynchronize(p->done);
        (void)hipEventDestroy(p->done);
        p->done = nullptr;
    }
    for (int t = 0; t < kTiers - 1; ++t) {
        if (p->branch[t]) (void)hipStreamDestroy(p->branch[t]);
        if (p->join[t]) (void)hipEventDestroy(p->join[t]);
        p->branch[t] = nullptr;
        p->join[t] = nullptr;
    }
    if (p->fork) (void)hipEventDestroy(p->fork);
    p->fork = nullptr;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_gitems) (void)hipFree(p->d_gitems);
    if (p->d_gsegs) (void)hipFree(p->d_gsegs);
    if (p->d_gbase) (void)hipFree(p->d_gbase);
    if (p->d_gtile) (void)hipFree(p->d_gtile);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    if (p->d_args) (void)hipFree(p->d_args);
    p->d_args = nullptr;
    p->args_written = false;
    p->exec = nullptr;
    p->graph = nullptr;
    p->capture_stream = nullptr;
    p->d_items = nullptr;
    p->d_gitems = nullptr;
    p->d_gsegs = nullptr;
    p->d_gbase = nullptr;
    p->d_gtile = nullptr;
    p->d_scratch = nullptr;
}

template <typename T> brr_status upload(T **dst, const std::vector<T> &src)
{
    if (src.empty()) return BRR_OK;
    if (hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T)) != hipSuccess)
        return BRR_ENOMEM;
    if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return BRR_EHIP;
    return BRR_OK;
}

brr_status classify(brr_plan *p)
{
    std::vector<uint32_t> lane, cls[kLdsClasses], peel;
    std::vector<GItem> gitems;
    std::vector<SegTable> gsegs;
    std::vector<uint64_t> pos_base(1, 0), pair_base(1, 0);
    const uint32_t wave_cap = std::min<uint32_t>(p->map.wave_max, wave_tier_max_n());
    const uint32_t lane_cap = std::min<uint32_t>(p->map.lane_max, lane_tier_max_n());
    // LDS classes up to workgroups of wg_threads; larger arrays take peels
    const uint32_t lds_cap = lds_class_max_n(p->map.wg_threads == 256   ? 2
                                             : p->map.wg_threads == 512 ? 3
                                                                        : kLdsClasses - 1);
    for (uint64_t q = 0; q < p->count; ++q) {
        const uint64_t n = p->h_off[q + 1] - p->h_off[q];
        if (n <= 1) continue;
        if (n <= lane_cap) {
            lane.push_back((uint32_t)q);
            p->lane_max_n = std::max<uint32_t>(p->lane_max_n, (uint32_t)n);
        } else if (n <= lds_cap) {
            // the one-wavefront class up to wave_max, then the smallest
            // workgroup that holds the array
            int c = 0;
            if (n > wave_cap)
                for (c = 1; n > lds_class_max_n(c); ++c) {
                }
            cls[c].push_back((uint32_t)q);
            p->max_cls[c] = std::max<uint32_t>(p->max_cls[c], (uint32_t)n);
        } else if (n <= peel_tier_max_n()) {
            peel.push_back((uint32_t)q);
        } else {
            SegTable st;
            build_segments((uint32_t)n, (uint32_t)(n - 1), p->ds, st);
            gitems.push_back(GItem{p->h_off[q], pos_base.back(), q, (uint32_t)n,
                                   (uint32_t)(n - 1), 0, 0, nullptr});
            gsegs.push_back(st);
            pos_base.push_back(pos_base.back() + n);
            pair_base.push_back(pair_base.back() + (st.S + 1) / 2);
        }
    }
    // largest first: lanes of one block run in step when their sizes are
    // close, and for the block tiers the long blocks start first, so the
    // short ones fill the tail of the launch
    auto larger = [&](uint32_t a, uint32_t b) {
        return p->h_off[a + 1] - p->h_off[a] > p->h_off[b + 1] - p->h_off[b];
    };
    std::stable_sort(lane.begin(), lane.end(), larger);
    for (int c = 0; c < kLdsClasses; ++c) std::stable_sort(cls[c].begin(), cls[c].end(), larger);
    std::stable_sort(peel.begin(), peel.end(), larger);
    p->n_lane = (uint32_t)lane.size();
    p->n_peel = (uint32_t)peel.size();
    p->n_big = (uint32_t)gitems.size();
    std::vector<uint32_t> items(lane);
    for (int c = 0; c < kLdsClasses; ++c) {
        p->n_cls[c] = (uint32_t)cls[c].size();
        items.insert(items.end(), cls[c].begin(), cls[c].end());
    }
    items.insert(items.end(), peel.begin(), peel.end());
    brr_status st = upload(&p->d_items, items);
    if (st != BRR_OK) return st;
    if (p->n_big) {
        std::vector<uint64_t> bases(pos_base);
        bases.insert(bases.end(), pair_base.begin(), pair_base.end());
        if ((st = upload(&p->d_gitems, gitems)) != BRR_OK) return st;
        if ((st = upload(&p->d_gsegs, gsegs)) != BRR_OK) return st;
        if ((st = upload(&p->d_gbase, bases)) != BRR_OK) return st;
        if (pos_base.back() > kMaxGtierPositions) return BRR_EINVAL;
        p->g_npos = pos_base.back();
        p->g_npairs = pair_base.back();
        // owner of the first index of every tile, positions then pairs
        const uint32_t sh = gtier_tile_shift();
        std::vector<uint32_t> tiles;
        for (int which = 0; which < 2; ++which) {
            const std::vector<uint64_t> &base = which ? pair_base : pos_base;
            const uint64_t ntiles = (base.back() + (1ull << sh) - 1) >> sh;
            if (!which) p->g_pos_tiles = ntiles;
            uint32_t i = 0;
            for (uint64_t t = 0; t < ntiles; ++t) {
                while (i + 1 < p->n_big && base[i + 1] <= (t << sh)) ++i;
                tiles.push_back(i);
            }
        }
        if ((st = upload(&p->d_gtile, tiles)) != BRR_OK) return st;
        if (hipMalloc(&p->d_scratch, gtier_scratch_bytes(p->g_npos, p->eb)) != hipSuccess)
            return BRR_ENOMEM;
    }
    if (hipMalloc(reinterpret_cast<void **>(&p->d_args), sizeof(RunArgs)) != hipSuccess)
        return BRR_ENOMEM;
    if (p->fork_classes) {
        if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess)
            return BRR_EHIP;
        for (int t = 0; t < kTiers - 1; ++t) {
            if (hipStreamCreateWithFlags(&p->branch[t], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&p->join[t], hipEventDisableTiming) != hipSuccess)
                return BRR_EHIP;
        }
    }
    p->classified = true;
    return BRR_OK;
}

// The kernels read the run's arguments from the plan's device block, which
// run_plan writes before each run.
hipError_t launch_tier(brr_plan *p, int tier, void *data, hipStream_t s)
{
    const RunArgs *b = p->d_args;
    const uint32_t *items = p->d_items;
    if (tier == 0)
        return launch_batched_lane(b, items, p->n_lane, p->lane_max_n, p->eb, p->ds, s);
    items += p->n_lane;
    for (int c = 0; c < kLdsClasses; ++c) {
        if (tier == 1 + c)
            return launch_batched_lds(c, b, items, p->n_cls[c], p->max_cls[c], p->eb, p->ds, s);
        items += p->n_cls[c];
    }
    if (tier == 1 + kLdsClasses)
        return launch_batched_peel(b, items, p->n_peel, p->eb, p->ds, s);
    if (p->n_big == 0) return hipSuccess;
    GTierArgs a;
    std::memset(&a, 0, sizeof a);
    a.dyn = b; // data, seed and instance base from the plan's device block
    a.data = data;
    a.words = p->ds.words;
    a.eb = p->eb;
    a.nitems = p->n_big;
    a.npos = p->g_npos;
    a.npairs = p->g_npairs;
    a.items = p->d_gitems;
    a.segs = p->d_gsegs;
    a.pos_base = p->d_gbase;
    a.pair_base = p->d_gbase + p->n_big + 1;
    a.pos_tile = p->d_gtile;
    a.pair_tile = p->d_gtile + p->g_pos_tiles;
    a.scratch = p->d_scratch;
    return launch_gtier(a, s);
}

bool tier_used(const brr_plan *p, int tier)
{
    if (tier == 0) return p->n_lane != 0;
    if (tier <= kLdsClasses) return p->n_cls[tier - 1] != 0;
    return (tier == 1 + kLdsClasses ? p->n_peel : p->n_big) != 0;
}

// The size classes are independent (disjoint arrays): all but the last
// non-empty one run on branch streams that fork from s and join back into it.
hipError_t enqueue(brr_plan *p, void *data, hipStream_t s)
{
    int used[kTiers], nu = 0;
    for (int t = 0; t < kTiers; ++t)
        if (tier_used(p, t)) used[nu++] = t;
    if (nu == 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (!p->fork_classes) {
        for (int b = 0; b < nu; ++b)
            if ((e = launch_tier(p, used[b], data, s)) != hipSuccess) return e;
        return hipSuccess;
    }
    if (nu > 1) {
        if ((e = hipEventRecord(p->fork, s)) != hipSuccess) return e;
        for (int b = 0; b + 1 < nu; ++b) {
            if ((e = hipStreamWaitEvent(p->branch[b], p->fork, 0)) != hipSuccess) return e;
            if ((e = launch_tier(p, used[b], data, p->branch[b])) != hipSuccess) return e;
            if ((e = hipEventRecord(p->join[b], p->branch[b])) != hipSuccess) return e;
        }
    }
    if ((e = launch_tier(p, used[nu - 1], data, s)) != hipSuccess) return e;
    for (int b = 0; b + 1 < nu; ++b)
        if ((e = hipStreamWaitEvent(s, p->join[b], 0)) != hipSuccess) return e;
    return hipSuccess;
}

// A plan whose arrays all fall in one class other than the device-wide one
// is one kernel: launched directly, it costs less than a graph launch
// (65,536 x 256: 53 against 59 us a run).
bool single_kernel(const brr_plan *p)
{
    int nu = 0;
    for (int t = 0; t < kTiers; ++t) nu += tier_used(p, t) ? 1 : 0;
    return nu == 1 && !tier_used(p, kTiers - 1);
}

brr_status run_plan(brr_plan *p, void *data, const uint64_t *offsets, uint64_t seed, uint64_t inst,
                    hipStream_t s)
{
    if (!p->classified) {
        const brr_status st = classify(p);
        if (st != BRR_OK) return st;
    }
    if (!p->done && hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
        p->done = nullptr;
        return BRR_EHIP;
    }
    // runs on any stream follow the plan's previous run: they share its
    // scratch and its branch streams
    if (p->ran && hipStreamWaitEvent(s, p->done, 0) != hipSuccess) return BRR_EHIP;
    // this run's arguments, on the caller's stream behind the previous run
    // (waited on above), so no run reads arguments that a later one wrote;
    // a run with the previous run's arguments finds them there already
    const RunArgs args{data, offsets, seed, inst};
    if (!p->args_written || std::memcmp(&args, &p->last_args, sizeof args) != 0) {
        if (launch_set_args(p->d_args, args, s) != hipSuccess) return BRR_EHIP;
        p->last_args = args;
        p->args_written = true;
    }
    if (!p->map.use_graph || single_kernel(p)) {
        const hipError_t e = enqueue(p, data, s);
        const brr_status st = hip_status(e == hipSuccess ? hipEventRecord(p->done, s) : e);
        if (st == BRR_OK) p->ran = true;
        return st;
    }
    if (!p->exec) {
        // captured once: the kernels read their arguments from d_args
        if (!p->capture_stream &&
            hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return BRR_EHIP;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return BRR_EHIP;
        const hipError_t le = enqueue(p, data, p->capture_stream);
        const hipError_t ce = hipStreamEndCapture(p->capture_stream, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return BRR_EHIP;
        }
        p->graph = g;
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            p->exec = nullptr;
            return BRR_EHIP;
        }
        ++p->captures;
    }
    const hipError_t e = hipGraphLaunch(p->exec, s);
    const brr_status st = hip_status(e == hipSuccess ? hipEventRecord(p->done, s) : e);
    if (st == BRR_OK) p->ran = true;
    return st;
}

} // namespace

// ---------------------------------------------------------------------------
// extern "C" entry points
// ---------------------------------------------------------------------------

extern "C" {

brr_status brr_schedule_paper(int max_k, brr_schedule *out)
{
    if (!out) return BRR_EINVAL;
    brr_schedule s;
    std::memset(&s, 0, sizeof s);
    if (max_k == 1) {
        s.nsteps = 1;
        s.step[0] = brr_step{1, 1, 0, 0};
    } else if (max_k == 2) {
        s.nsteps = 2;
        s.step[0] = brr_step{1ull << 30, 1, 0, 0};
        s.step[1] = brr_step{2, 2, 0, 1ull << 60};
        s.tail = 1;
        s.u_tail = 720;
    } else if (max_k == 6) {
        // one die above 2^30 elements, then k = 2..6 dice while more than
        // 2^19, 2^14, 2^11, 2^9, 6 elements remain (k = 2 from 2^30 down),
        // each k with the paper's upper bound on its bound product
        const uint64_t above[6] = {1ull << 30, 1ull << 19, 1ull << 14, 1ull << 11, 1ull << 9, 6};
        const uint64_t bound[6] = {0, 1ull << 60, 1ull << 57, 1ull << 56, 1ull << 55, 1ull << 54};
        s.nsteps = 6;
        for (uint32_t g = 0; g < 6; ++g) s.step[g] = brr_step{above[g], g + 1, 0, bound[g]};
        s.tail = 1;
        s.u_tail = 720;
    } else {
        return BRR_EINVAL;
    }
    *out = s;
    return BRR_OK;
}

brr_status brr_schedule_kmax(uint32_t kcap, brr_schedule *out)
{
    if (!out || kcap < 1 || kcap > BRR_MAX_STEPS) return BRR_EINVAL;
    const u128 two64 = (u128)1 << 64;
    // N[k]: the largest n with n (n-1) ... (n-k+1) <= 2^64, by bisection
    uint64_t N[BRR_MAX_STEPS + 2] = {};
    for (uint32_t k = 2; k <= kcap + 1; ++k) {
        uint64_t lo = k, hi = 1ull << 33; // falling(lo, k) <= 2^64 < falling(hi, k)
        while (hi - lo > 1) {
            const uint64_t mid = lo + (hi - lo) / 2;
            (falling(mid, k) <= two64 ? lo : hi) = mid;
        }
        N[k] = lo;
    }
    brr_schedule s;
    std::memset(&s, 0, sizeof s);
    s.nsteps = kcap;
    for (uint32_t k = 1; k <= kcap; ++k) {
        const uint64_t above = (k < kcap) ? N[k + 1] : kcap - 1;
        const uint64_t guard = (k == 1) ? 0 : (uint64_t)falling(N[k], k);
        s.step[k - 1] = brr_step{above, k, BRR_FORM_MULTIPLY, guard};
    }
    s.tail = 1;
    s.u_tail = 0;
    *out = s;
    return BRR_OK;
}

brr_status brr_schedule_naive2(brr_schedule *out)
{
    if (!out) return BRR_EINVAL;
    brr_schedule s;
    std::memset(&s, 0, sizeof s);
    s.nsteps = 2;
    s.step[0] = brr_step{1ull << 32, 1, BRR_FORM_DIVISION, 0};
    s.step[1] = brr_step{1, 2, BRR_FORM_DIVISION, 0};
    s.tail = 0;
    *out = s;
    return BRR_OK;
}

uint64_t brr_schedule_batches(const brr_schedule *sched, uint64_t n, uint64_t steps)
{
    if (!sched || check_structure(*sched) != BRR_OK) return 0;
    brr_status e = BRR_OK;
    return walk_schedule(*sched, n, steps, false, &e);
}

brr_status brr_schedule_check(const brr_schedule *sched, uint64_t n)
{
    if (!sched) return BRR_EINVAL;
    return check_for(*sched, n, n ? n - 1 : 0);
}

brr_status brr_schedule_check_upto(const brr_schedule *sched, uint64_t max_n)
{
    if (!sched) return BRR_EINVAL;
    return check_upto(*sched, max_n);
}

brr_status brr_dice(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                    uint64_t seed, uint64_t inst, void *stream)
{
    if (k < 1 || k > 8) return BRR_EINVAL;
    if (count == 0) return BRR_OK;
    if (!d_bounds || !d_out || misaligned(d_bounds, 4) || misaligned(d_out, 4)) return BRR_EINVAL;
    uint32_t *status = nullptr;
    const brr_status st = device_ready(&status);
    if (st != BRR_OK) return st;
    return hip_status(launch_dice(d_bounds, d_out, count, k, make_key(seed, inst), status,
                                  static_cast<hipStream_t>(stream)));
}

brr_status brr_dice_div(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                        uint64_t seed, uint64_t inst, void *stream)
{
    if (k < 1 || k > 8) return BRR_EINVAL;
    if (count == 0) return BRR_OK;
    if (!d_bounds || !d_out || misaligned(d_bounds, 4) || misaligned(d_out, 4)) return BRR_EINVAL;
    uint32_t *status = nullptr;
    const brr_status st = device_ready(&status);
    if (st != BRR_OK) return st;
    return hip_status(launch_dice_div(d_bounds, d_out, count, k, make_key(seed, inst), status,
                                      static_cast<hipStream_t>(stream)));
}

brr_status brr_dice_chacha(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                           uint64_t seed, uint64_t inst, void *stream)
{
    if (k < 1 || k > 8) return BRR_EINVAL;
    if (count == 0) return BRR_OK;
    if (!d_bounds || !d_out || misaligned(d_bounds, 4) || misaligned(d_out, 4)) return BRR_EINVAL;
    uint32_t *status = nullptr;
    brr_status st = device_ready(&status);
    if (st != BRR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::unique_lock<std::mutex> hold;
    void *rec = nullptr;
    if (stream_scratch(s, chacha_record_bytes(count, k), hold, &rec) != BRR_OK)
        rec = nullptr; // no record: every group rerolls in place
    return hip_status(launch_dice_chacha(d_bounds, d_out, count, k, make_key(seed, inst), status,
                                         rec, s));
}

brr_status brr_dice32(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                      uint64_t seed, uint64_t inst, void *stream)
{
    if (k < 1 || k > 8) return BRR_EINVAL;
    if (count == 0) return BRR_OK;
    if (!d_bounds || !d_out || misaligned(d_bounds, 4) || misaligned(d_out, 4)) return BRR_EINVAL;
    uint32_t *status = nullptr;
    const brr_status st = device_ready(&status);
    if (st != BRR_OK) return st;
    return hip_status(launch_dice32(d_bounds, d_out, count, k, make_key(seed, inst), status,
                                    static_cast<hipStream_t>(stream)));
}

namespace {
// Algorithm 2 with the thresholds of a full group and of the short last
// group computed here, once.
brr_status dice_known(const BoundTuple &tb, uint32_t *d_out, uint64_t count, uint32_t k,
                      uint64_t seed, uint64_t inst, void *stream)
{
    const u128 two64 = (u128)1 << 64;
    const uint64_t S = (count + k - 1) / k;
    const uint64_t k_last = count - (S - 1) * k;
    // products capped just above 2^64 so that eight 32-bit factors never wrap
    u128 p_full = 1, p_last = 1;
    for (uint32_t i = 0; i < k; ++i) {
        p_full *= tb.b[i];
        if (i < k_last) p_last *= tb.b[i];
        if (p_full > two64) p_full = two64 + 1; // stays above 2^64 (bounds >= 1)
        if (p_last > two64) p_last = two64 + 1;
    }
    if (p_full > two64 && count >= k) return BRR_EOVERFLOW;
    if (p_last > two64) return BRR_EOVERFLOW;
    const uint64_t t_full = p_full > two64 ? 0 : (uint64_t)(two64 % p_full);
    const uint64_t t_last = (uint64_t)(two64 % p_last);
    const brr_status st = device_ready(nullptr);
    if (st != BRR_OK) return st;
    return hip_status(launch_dice_const(tb, d_out, count, k, make_key(seed, inst), t_full, t_last,
                                        static_cast<hipStream_t>(stream)));
}
} // namespace

brr_status brr_dice_const(uint32_t bound, uint32_t *d_out, uint64_t count, uint32_t k,
                          uint64_t seed, uint64_t inst, void *stream)
{
    if (k < 1 || k > 8) return BRR_EINVAL;
    if (count == 0) return BRR_OK;
    if (!d_out || bound == 0 || misaligned(d_out, 4)) return BRR_EINVAL;
    BoundTuple tb{};
    for (uint32_t i = 0; i < 8; ++i) tb.b[i] = bound;
    return dice_known(tb, d_out, count, k, seed, inst, stream);
}

brr_status brr_dice_tuple(const uint32_t *h_bounds, uint32_t k, uint32_t *d_out, uint64_t count,
                          uint64_t seed, uint64_t inst, void *stream)
{
    if (k < 1 || k > 8 || !h_bounds) return BRR_EINVAL;
    BoundTuple tb{};
    for (uint32_t i = 0; i < k; ++i) {
        if (h_bounds[i] == 0) return BRR_EINVAL;
        tb.b[i] = h_bounds[i];
    }
    if (count == 0) return BRR_OK;
    if (!d_out || misaligned(d_out, 4)) return BRR_EINVAL;
    return dice_known(tb, d_out, count, k, seed, inst, stream);
}

brr_status brr_shuffle(void *d_data, uint64_t n, uint32_t elem_bytes, const brr_schedule *sched,
                       uint64_t seed, uint64_t inst, void *stream)
{
    if (elem_bytes != 4 && elem_bytes != 8) return BRR_EINVAL;
    if (n <= 1) return BRR_OK;
    if (!d_data || n > 0xFFFFFFFFull || misaligned(d_data, elem_bytes)) return BRR_EINVAL;
    const brr_schedule &sc = sched ? *sched : paper6();
    brr_status st = check_for(sc, n, n - 1);
    if (st != BRR_OK) return st;
    st = device_ready(nullptr);
    if (st != BRR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::unique_lock<std::mutex> hold;
    void *scr = nullptr;
    const uint64_t bytes = one_scratch_bytes(n, elem_bytes);
    if (bytes && (st = stream_scratch(s, bytes, hold, &scr)) != BRR_OK) return st;
    return hip_status(launch_one(d_data, (uint32_t)n, (uint32_t)(n - 1), 0, elem_bytes, nullptr,
                                 to_dev(sc), seed, inst, DevClaim{}, s, scr));
}

brr_status brr_shuffle_noalloc(void *d_data, uint64_t n, uint32_t elem_bytes,
                               const brr_schedule *sched, uint64_t seed, uint64_t inst,
                               void *stream)
{
    if (elem_bytes != 4 && elem_bytes != 8) return BRR_EINVAL;
    if (n <= 1) return BRR_OK;
    if (!d_data || misaligned(d_data, elem_bytes)) return BRR_EINVAL;
    if (n > BRR_NOALLOC_MAX_N || one_scratch_bytes(n, elem_bytes) > kNoAllocScratchBytes)
        return BRR_EINVAL;
    const brr_schedule &sc = sched ? *sched : paper6();
    brr_status st = check_for(sc, n, n - 1);
    if (st != BRR_OK) return st;
    st = device_ready(nullptr);
    if (st != BRR_OK) return st;
    void *scr = nullptr;
    st = noalloc_scratch(&scr);
    if (st != BRR_OK) return st;
    // the kernels initialise every part of the scratch they read
    return hip_status(launch_one(d_data, (uint32_t)n, (uint32_t)(n - 1), 0, elem_bytes, nullptr,
                                 to_dev(sc), seed, inst, DevClaim{},
                                 static_cast<hipStream_t>(stream), scr));
}

uint64_t brr_scratch_bytes(uint64_t n, uint64_t m, uint32_t elem_bytes)
{
    if ((elem_bytes != 4 && elem_bytes != 8) || m > n || n > 0xFFFFFFFFull) return 0;
    return one_scratch_bytes(n, elem_bytes, m);
}

brr_status brr_sample(const void *d_data, uint64_t n, uint64_t m, uint32_t elem_bytes, void *d_out,
                      const brr_schedule *sched, uint64_t seed, uint64_t inst, void *stream)
{
    if (elem_bytes != 4 && elem_bytes != 8) return BRR_EINVAL;
    if (m > n) return BRR_EINVAL;
    if (m == 0) return BRR_OK;
    if (!d_data || !d_out || n > 0xFFFFFFFFull) return BRR_EINVAL;
    if (misaligned(d_data, elem_bytes) || misaligned(d_out, elem_bytes)) return BRR_EINVAL;
    const brr_schedule &sc = sched ? *sched : paper6();
    const uint64_t steps = std::min<uint64_t>(m, n - 1);
    brr_status st = check_for(sc, n, steps);
    if (st != BRR_OK) return st;
    st = device_ready(nullptr);
    if (st != BRR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 1) // one element, no step: the sample is the element itself
        return hip_status(hipMemcpyAsync(d_out, d_data, elem_bytes, hipMemcpyDeviceToDevice, s));
    void *data = const_cast<void *>(d_data); // only read when an output buffer is given
    std::unique_lock<std::mutex> hold;
    void *scr = nullptr;
    const uint64_t bytes = one_scratch_bytes(n, elem_bytes, m);
    if (bytes && (st = stream_scratch(s, bytes, hold, &scr)) != BRR_OK) return st;
    return hip_status(launch_one(data, (uint32_t)n, (uint32_t)steps, (uint32_t)(n - m), elem_bytes,
                                 d_out, to_dev(sc), seed, inst, DevClaim{}, s, scr));
}

brr_status brr_plan_create(brr_plan **out, const uint64_t *h_offsets, uint64_t count,
                           uint32_t elem_bytes, const brr_schedule *sched)
{
    if (!out) return BRR_EINVAL;
    *out = nullptr;
    if (elem_bytes != 4 && elem_bytes != 8) return BRR_EINVAL;
    if (count > 0xFFFFFFFFull || (count && !h_offsets)) return BRR_EINVAL;
    const brr_schedule &sc = sched ? *sched : paper6();
    uint64_t max_n = 0;
    for (uint64_t q = 0; q < count; ++q) {
        if (h_offsets[q + 1] < h_offsets[q]) return BRR_EINVAL;
        max_n = std::max<uint64_t>(max_n, h_offsets[q + 1] - h_offsets[q]);
    }
    if (max_n > 0xFFFFFFFFull) return BRR_EINVAL;
    // every size up to the largest shuffle's may occur
    brr_status st = check_upto(sc, max_n);
    if (st != BRR_OK) return st;
    st = device_ready(nullptr);
    if (st != BRR_OK) return st;
    brr_plan *p = new (std::nothrow) brr_plan();
    if (!p) return BRR_ENOMEM;
    try {
        (void)hipGetDevice(&p->device);
        p->eb = elem_bytes;
        p->count = count;
        p->sched = sc;
        p->ds = to_dev(sc);
        p->map = brr_mapping{lane_tier_max_n(), wave_tier_max_n(), 1024, 1};
        p->h_off.assign(h_offsets, h_offsets + (count ? count + 1 : 0));
    } catch (...) {
        delete p;
        return BRR_ENOMEM;
    }
    *out = p;
    return BRR_OK;
}

void brr_plan_destroy(brr_plan *plan)
{
    if (!plan) return;
    release(plan);
    delete plan;
}

uint32_t brr_plan_captures(const brr_plan *plan)
{
    if (!plan) return 0;
    std::lock_guard<std::mutex> lock(const_cast<brr_plan *>(plan)->mu);
    return plan->captures;
}

brr_status brr_plan_get_mapping(const brr_plan *plan, brr_mapping *out)
{
    if (!plan || !out) return BRR_EINVAL;
    std::lock_guard<std::mutex> lock(const_cast<brr_plan *>(plan)->mu);
    *out = plan->map;
    return BRR_OK;
}

brr_status brr_plan_set_mapping(brr_plan *plan, const brr_mapping *m)
{
    if (!plan || !m) return BRR_EINVAL;
    std::lock_guard<std::mutex> lock(plan->mu);
    if (plan->classified) return BRR_EINVAL; // the mapping is fixed by the first run
    if (m->lane_max > lane_tier_max_n()) return BRR_EINVAL;
    if (m->wave_max > wave_tier_max_n()) return BRR_EINVAL;
    if (m->wg_threads != 256 && m->wg_threads != 512 && m->wg_threads != 1024) return BRR_EINVAL;
    plan->map = *m;
    return BRR_OK;
}

brr_status brr_shuffle_batched(void *d_data, const uint64_t *d_offsets, uint64_t count,
                               uint32_t elem_bytes, brr_plan *plan, uint64_t seed,
                               uint64_t inst_base, void *stream)
{
    if (elem_bytes != 4 && elem_bytes != 8) return BRR_EINVAL;
    if (count == 0) return BRR_OK;
    if (!d_data || !d_offsets || misaligned(d_data, elem_bytes) || misaligned(d_offsets, 8))
        return BRR_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (plan) {
        if (plan->eb != elem_bytes || plan->count != count) return BRR_EINVAL;
        int dev = -1;
        (void)hipGetDevice(&dev);
        if (dev != plan->device) return BRR_EINVAL;
        try {
            std::lock_guard<std::mutex> lock(plan->mu);
            return run_plan(plan, d_data, d_offsets, seed, inst_base, s);
        } catch (...) {
            return BRR_ENOMEM;
        }
    }
    // no plan: classify from a host copy of the offsets, run, wait, release
    std::vector<uint64_t> h;
    try {
        h.resize(count + 1);
    } catch (...) {
        return BRR_ENOMEM;
    }
    if (hipMemcpyAsync(h.data(), d_offsets, (count + 1) * 8, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return BRR_EHIP;
    brr_plan *tmp = nullptr;
    brr_status st = brr_plan_create(&tmp, h.data(), count, elem_bytes, nullptr);
    if (st != BRR_OK) return st;
    tmp->map.use_graph = 0;
    tmp->fork_classes = false;
    try {
        st = run_plan(tmp, d_data, d_offsets, seed, inst_base, s);
    } catch (...) {
        st = BRR_ENOMEM;
    }
    if (hipStreamSynchronize(s) != hipSuccess && st == BRR_OK) st = BRR_EHIP;
    brr_plan_destroy(tmp);
    return st;
}

brr_status brr_sync_status(void *stream)
{
    uint32_t *status = nullptr;
    brr_status st = device_ready(&status);
    if (st != BRR_OK) return st;
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return BRR_EHIP;
    uint32_t v = 0;
    if (hipMemcpy(&v, status, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return BRR_EHIP;
    if (v == 0) return BRR_OK;
    if (hipMemset(status, 0, sizeof v) != hipSuccess) return BRR_EHIP;
    if (hipDeviceSynchronize() != hipSuccess) return BRR_EHIP;
    return (v & kDevZeroBound) ? BRR_EINVAL : BRR_EOVERFLOW;
}

const char *brr_strerror(brr_status status)
{
    switch (status) {
    case BRR_OK: return "ok";
    case BRR_EINVAL: return "invalid argument (null pointer, k, zero bound, m > n or schedule)";
    case BRR_EOVERFLOW: return "bound product above 2^64";
    case BRR_ENOMEM: return "device memory allocation failed";
    case BRR_EHIP: return "HIP runtime error";
    case BRR_EDEVICE: return "no usable gfx950 device";
    default: return "unknown status";
    }
}

} // extern "C"

namespace {

__global__ void k_add_one(uint32_t *a, uint64_t n)
{
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (uint64_t)gridDim.x * blockDim.x)
        a[x] += 1;
}

// Average time of `reps` launches of fn on stream s, after one warm-up.
// Median of `reps` single timed runs after one untimed run: tuning compares
// candidates a few percent apart, which a single timing cannot resolve.
template <class F> float time_median_ms(F &&fn, hipStream_t s, int reps, brr_status *st)
{
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    for (hipEvent_t &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            *st = BRR_EHIP;
            for (hipEvent_t &f : ev)
                if (f) (void)hipEventDestroy(f);
            return 0;
        }
    *st = fn();
    for (int r = 0; r < reps && *st == BRR_OK; ++r) {
        (void)hipEventRecord(ev[2 * r], s);
        *st = fn();
        (void)hipEventRecord(ev[2 * r + 1], s);
    }
    std::vector<float> t;
    if (*st == BRR_OK) {
        if (hipEventSynchronize(ev.back()) != hipSuccess) *st = BRR_EHIP;
        for (int r = 0; r < reps && *st == BRR_OK; ++r) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]);
            t.push_back(ms);
        }
    }
    for (hipEvent_t &e : ev) (void)hipEventDestroy(e);
    if (t.empty()) return 0;
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    return t[t.size() / 2];
}

template <class F> float time_ms(F &&fn, hipStream_t s, int reps, brr_status *st)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        *st = BRR_EHIP;
        return 0;
    }
    *st = fn();
    float ms = 0;
    if (*st == BRR_OK) {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && *st == BRR_OK; ++r) *st = fn();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) *st = BRR_EHIP;
        (void)hipEventElapsedTime(&ms, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / reps;
}

std::mutex g_tune_mu;
std::map<std::pair<int, int>, uint32_t> g_dice_k; // (bit length, log2 count) -> k

bool same_steps(const brr_schedule &a, const brr_schedule &b)
{
    if (a.nsteps != b.nsteps || a.tail != b.tail || a.words != b.words) return false;
    for (uint32_t g = 0; g < a.nsteps; ++g)
        if (a.step[g].n_above != b.step[g].n_above || a.step[g].k != b.step[g].k ||
            a.step[g].form != b.step[g].form)
            return false;
    return true;
}

// Plan features for the cost model: sizes, payload, how the schedule
// batches the steps, and how the mapping splits the sizes into tiers.
void plan_features(const uint64_t *off, uint64_t count, uint32_t eb, const brr_schedule &sc,
                   uint32_t wave_max, float *f)
{
    const DevSched ds = to_dev(sc);
    double total = 0, sum_lg = 0, sum_lg2 = 0, words = 0, steps = 0, d_hi = 0, d_lo = 0;
    double band[5] = {0, 0, 0, 0, 0}, in_wave = 0;
    uint32_t kmax = 1;
    for (uint32_t g = 0; g < sc.nsteps; ++g) kmax = std::max(kmax, sc.step[g].k);
    for (uint64_t q = 0; q < count; ++q) {
        const uint64_t n = off[q + 1] - off[q];
        if (n <= 1) continue;
        const double w = (double)n, lg = std::log2(w);
        total += w;
        sum_lg += w * lg;
        sum_lg2 += w * lg * lg;
        band[n <= 64 ? 0 : n <= 512 ? 1 : n <= 16384 ? 2 : n <= (1u << 20) ? 3 : 4] += w;
        if (n <= wave_max) in_wave += w;
        if (n > 0xFFFFFFFFull) continue;
        SegTable st;
        build_segments((uint32_t)n, (uint32_t)(n - 1), ds, st);
        words += st.S;
        steps += (double)(n - 1);
        for (uint32_t g = 0; g < st.nseg; ++g) {
            const double dice = (double)st.seg[g].cnt * st.seg[g].k;
            if (st.seg[g].k >= 4) d_hi += dice;
            if (st.seg[g].k <= 2) d_lo += dice;
        }
    }
    const double mean = total > 0 ? sum_lg / total : 0;
    const double var = total > 0 ? std::max(0.0, sum_lg2 / total - mean * mean) : 0;
    f[0] = (float)(std::log2(total + 1) / 32);
    f[1] = (float)(std::log2((double)count + 1) / 16);
    f[2] = (float)eb / 8;
    for (int b = 0; b < 5; ++b) f[3 + b] = total > 0 ? (float)(band[b] / total) : 0.0f;
    f[8] = (float)(mean / 32);
    f[9] = (float)(std::sqrt(var) / 8);
    f[10] = steps > 0 ? (float)(words / steps) : 0.0f;
    f[11] = steps > 0 ? (float)(d_hi / steps) : 0.0f;
    f[12] = steps > 0 ? (float)(d_lo / steps) : 0.0f;
    f[13] = (float)kmax / 8;
    f[14] = (float)(std::log2((double)std::max<uint32_t>(wave_max, 1)) / 10);
    f[15] = total > 0 ? (float)(in_wave / total) : 0.0f;
}

struct Candidate {
    brr_schedule sched;
    uint32_t wave_max;
};

// The plan's own configuration first, then the paper's schedules and
// cost-model schedules (kmax 3..8, several generator/division cost ratios)
// under wavefront-tier limits 64..512.
std::vector<Candidate> candidates(const brr_plan *plan, uint64_t max_n)
{
    std::vector<brr_schedule> scheds{plan->sched};
    // every candidate reads the plan's word stream: the stream is the
    // caller's choice, only batch sizes and the mapping are tuned
    const uint32_t words = plan->sched.words;
    const int lflag = (words == BRR_WORDS_PHILOX32) ? BRR_COSTS_L32 : 0;
    auto add = [&](brr_schedule c) {
        c.words = words;
        if (check_upto(c, max_n) != BRR_OK) return;
        for (const brr_schedule &o : scheds)
            if (same_steps(o, c)) return;
        scheds.push_back(c);
    };
    for (int mk : {6, 2, 1}) {
        brr_schedule c;
        if (brr_schedule_paper(mk, &c) == BRR_OK) add(c);
    }
    const double ratios[][2] = {{2, 16}, {1, 16}, {4, 16}, {8, 16}, {2, 64}};
    for (uint32_t kmax = 3; kmax <= 8; ++kmax)
        for (const auto &r : ratios) {
            brr_schedule c;
            if (brr_schedule_from_costs(kmax, r[0], r[1],
                                        BRR_COSTS_POW2 | BRR_COSTS_SMOOTH | lflag, &c) == BRR_OK)
                add(c);
        }
    std::vector<Candidate> out;
    out.push_back(Candidate{plan->sched, plan->map.wave_max});
    for (const brr_schedule &sc : scheds)
        for (uint32_t wm : {64u, 128u, 256u, 512u}) {
            if (wm > wave_tier_max_n()) continue;
            if (same_steps(sc, plan->sched) && wm == plan->map.wave_max) continue;
            out.push_back(Candidate{sc, wm});
        }
    return out;
}

// Picks the plan's configuration. Without a model: time the wavefront limits
// under the plan's schedule, then every schedule under the best limit. With
// a model: rank every candidate by predicted time and time the plan's own
// configuration and the `top` best predicted ones.
brr_status tune_plan(brr_plan *plan, brr_mlp *model, uint32_t top, const void *d_data,
                     const uint64_t *d_offsets, uint64_t seed, uint64_t inst_base, void *stream,
                     brr_tune_report *report)
{
    if (!plan || !d_data || !d_offsets) return BRR_EINVAL;
    std::lock_guard<std::mutex> plan_lock(plan->mu);
    if (plan->classified) return BRR_EINVAL; // must precede the first run
    brr_status st = device_ready(nullptr);
    if (st != BRR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t total = plan->count ? plan->h_off[plan->count] : 0;
    uint64_t max_n = 0;
    for (uint64_t q = 0; q < plan->count; ++q)
        max_n = std::max<uint64_t>(max_n, plan->h_off[q + 1] - plan->h_off[q]);
    const std::vector<Candidate> cands = candidates(plan, max_n);
    void *work = nullptr;
    if (total && hipMallocAsync(&work, total * plan->eb, s) != hipSuccess) return BRR_ENOMEM;
    if (total && hipMemcpyAsync(work, d_data, total * plan->eb, hipMemcpyDeviceToDevice, s) !=
                     hipSuccess)
        st = BRR_EHIP;
    auto time_config = [&](const Candidate &c, float *ms) -> brr_status {
        brr_plan *t = nullptr;
        brr_status e = brr_plan_create(&t, plan->h_off.data(), plan->count, plan->eb, &c.sched);
        if (e != BRR_OK) return e;
        t->map = plan->map;
        t->map.wave_max = c.wave_max;
        t->map.use_graph = 0;
        *ms = time_median_ms(
            [&] { return brr_shuffle_batched(work, d_offsets, plan->count, plan->eb, t, seed,
                                             inst_base, stream); },
            s, 5, &e);
        if (hipStreamSynchronize(s) != hipSuccess && e == BRR_OK) e = BRR_EHIP;
        brr_plan_destroy(t);
        return e;
    };
    std::vector<size_t> order; // candidates to time, in order
    if (model && st == BRR_OK) {
        const uint32_t F = BRR_PLAN_FEATURES;
        std::vector<float> feats(cands.size() * F), pred(cands.size());
        for (size_t c = 0; c < cands.size(); ++c)
            plan_features(plan->h_off.data(), plan->count, plan->eb, cands[c].sched,
                          cands[c].wave_max, feats.data() + c * F);
        float *d_f = nullptr, *d_p = nullptr;
        if (hipMallocAsync(reinterpret_cast<void **>(&d_f), feats.size() * 4, s) != hipSuccess ||
            hipMallocAsync(reinterpret_cast<void **>(&d_p), pred.size() * 4, s) != hipSuccess)
            st = BRR_ENOMEM;
        if (st == BRR_OK &&
            hipMemcpyAsync(d_f, feats.data(), feats.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            st = BRR_EHIP;
        if (st == BRR_OK) st = brr_mlp_forward(model, d_f, (uint32_t)cands.size(), d_p, stream);
        if (st == BRR_OK &&
            hipMemcpyAsync(pred.data(), d_p, pred.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = BRR_EHIP;
        if (d_f) (void)hipFreeAsync(d_f, s);
        if (d_p) (void)hipFreeAsync(d_p, s);
        if (hipStreamSynchronize(s) != hipSuccess && st == BRR_OK) st = BRR_EHIP;
        std::vector<size_t> rank(cands.size());
        for (size_t c = 0; c < rank.size(); ++c) rank[c] = c;
        std::stable_sort(rank.begin(), rank.end(), [&](size_t a, size_t b) { return pred[a] < pred[b]; });
        order.push_back(0);
        for (size_t r = 0; r < rank.size() && order.size() < (size_t)top + 1; ++r)
            if (rank[r] != 0) order.push_back(rank[r]);
    }
    uint32_t n_tried = 0;
    float ms_default = 0, best = 0;
    size_t best_c = 0;
    if (model) {
        for (size_t i = 0; i < order.size() && st == BRR_OK; ++i) {
            float ms = 0;
            st = time_config(cands[order[i]], &ms);
            ++n_tried;
            if (i == 0) ms_default = best = ms;
            if (st == BRR_OK && ms < best) {
                best = ms;
                best_c = order[i];
            }
        }
    } else {
        if (st == BRR_OK) st = time_config(cands[0], &ms_default);
        ++n_tried;
        best = ms_default;
        uint32_t best_wave = plan->map.wave_max;
        for (size_t c = 1; c < cands.size() && st == BRR_OK; ++c) { // limits, plan's schedule
            if (!same_steps(cands[c].sched, plan->sched)) continue;
            float ms = 0;
            st = time_config(cands[c], &ms);
            ++n_tried;
            if (st == BRR_OK && ms < best) {
                best = ms;
                best_c = c;
                best_wave = cands[c].wave_max;
            }
        }
        for (size_t c = 1; c < cands.size() && st == BRR_OK; ++c) { // schedules, best limit
            if (same_steps(cands[c].sched, plan->sched) || cands[c].wave_max != best_wave) continue;
            float ms = 0;
            st = time_config(cands[c], &ms);
            ++n_tried;
            if (st == BRR_OK && ms < best) {
                best = ms;
                best_c = c;
            }
        }
    }
    if (work) (void)hipFreeAsync(work, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == BRR_OK) st = BRR_EHIP;
    if (st != BRR_OK) return st;
    plan->sched = cands[best_c].sched;
    plan->ds = to_dev(plan->sched);
    plan->map.wave_max = cands[best_c].wave_max;
    if (report) {
        report->candidates = n_tried;
        report->ms_best = best;
        report->ms_default = ms_default;
        report->schedule = plan->sched;
        report->mapping = plan->map;
    }
    return BRR_OK;
}

} // namespace

extern "C" {

brr_status brr_dice_autotune(uint32_t max_bound, uint64_t count, void *stream, uint32_t *best_k,
                             float *ms_per_k)
{
    if (!best_k || max_bound == 0 || count == 0) return BRR_EINVAL;
    brr_status st = device_ready(nullptr);
    if (st != BRR_OK) return st;
    const uint64_t n = std::min<uint64_t>(count, 1ull << 26);
    int bits = 0;
    while (bits < 32 && (max_bound >> bits)) ++bits;
    int lg = 0;
    while ((1ull << (lg + 1)) <= n) ++lg;
    if (!ms_per_k) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_dice_k.find({bits, lg});
        if (it != g_dice_k.end()) {
            *best_k = it->second;
            return BRR_OK;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t *bounds = nullptr, *out = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&bounds), n * 4, s) != hipSuccess) return BRR_ENOMEM;
    if (hipMallocAsync(reinterpret_cast<void **>(&out), n * 4, s) != hipSuccess) {
        (void)hipFreeAsync(bounds, s);
        return BRR_ENOMEM;
    }
    // bounds uniform in [1, max_bound]: rolled by this library, then shifted
    st = brr_dice_const(max_bound, bounds, n, 1, 0x5eedull, ~0ull, stream);
    if (st == BRR_OK) {
        k_add_one<<<1024, 256, 0, s>>>(bounds, n);
        if (hipGetLastError() != hipSuccess) st = BRR_EHIP;
    }
    const u128 two64 = (u128)1 << 64;
    float best = 0;
    uint32_t bk = 1;
    if (ms_per_k)
        for (int k = 0; k <= 8; ++k) ms_per_k[k] = 0;
    for (uint32_t k = 1; k <= 8 && st == BRR_OK; ++k) {
        u128 p = 1;
        for (uint32_t i = 0; i < k; ++i) p *= max_bound;
        if (p > two64) break;
        const float ms = time_ms([&] { return brr_dice(bounds, out, n, k, 1, 0, stream); }, s, 3, &st);
        if (st != BRR_OK) break;
        if (ms_per_k) ms_per_k[k] = ms;
        if (k == 1 || ms < best) {
            best = ms;
            bk = k;
        }
    }
    (void)hipFreeAsync(bounds, s);
    (void)hipFreeAsync(out, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == BRR_OK) st = BRR_EHIP;
    if (st != BRR_OK) return st;
    *best_k = bk;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_dice_k[{bits, lg}] = bk;
    return BRR_OK;
}

brr_status brr_plan_get_schedule(const brr_plan *plan, brr_schedule *out)
{
    if (!plan || !out) return BRR_EINVAL;
    std::lock_guard<std::mutex> lock(const_cast<brr_plan *>(plan)->mu);
    *out = plan->sched;
    return BRR_OK;
}

brr_status brr_plan_autotune(brr_plan *plan, const void *d_data, const uint64_t *d_offsets,
                             uint64_t seed, uint64_t inst_base, void *stream,
                             brr_tune_report *report)
{
    return tune_plan(plan, nullptr, 0, d_data, d_offsets, seed, inst_base, stream, report);
}

brr_status brr_plan_features(const uint64_t *h_offsets, uint64_t count, uint32_t elem_bytes,
                             const brr_schedule *sched, uint32_t wave_max, float *out)
{
    if (!out || (count && !h_offsets) || (elem_bytes != 4 && elem_bytes != 8)) return BRR_EINVAL;
    const brr_schedule &sc = sched ? *sched : paper6();
    if (check_structure(sc) != BRR_OK) return BRR_EINVAL;
    plan_features(h_offsets, count, elem_bytes, sc, wave_max, out);
    return BRR_OK;
}

brr_status brr_plan_autotune_learned(brr_plan *plan, brr_mlp *model, uint32_t top,
                                     const void *d_data, const uint64_t *d_offsets, uint64_t seed,
                                     uint64_t inst_base, void *stream, brr_tune_report *report)
{
    if (!model || top == 0) return BRR_EINVAL;
    return tune_plan(plan, model, top, d_data, d_offsets, seed, inst_base, stream, report);
}

} // extern "C"
