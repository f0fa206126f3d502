// Serving loop with continuous batching: shuffle and sample requests are
// admitted as in-flight slots and device scratch free up, and retired as
// their completion events fire. Each pass of the worker admits what it can
// (a tick) and launches the tick's requests together:
//   - one claim kernel on the control stream hands every admitted request,
//     in submission order, the next instance of its session from the
//     session's counter in device memory (session * 2^40 + counter); a
//     request's result is therefore fixed by (session, its place in the
//     session), whatever else runs beside it;
//   - the requests small enough for one workgroup's LDS run as one launch
//     per LDS size class and element width (one block per request) on the
//     control stream, behind the claim;
//   - larger ones (the device-wide shuffle tier, sparse samples) each run
//     their own kernels on a pool of streams, after the claim;
// so a tick of many small requests costs a few launches, not one or more
// per request, and the large requests overlap with them and each other.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "brr.h"
#include "internal.hpp"

using namespace brr;

namespace {

using clock_t_ = std::chrono::steady_clock;

constexpr uint32_t kMaxSessions = 4096;
constexpr uint64_t kSessionShift = 40;

constexpr uint32_t kMaxTick = 64; // requests admitted per tick

// The instances of one tick's requests, in submission order: request e takes
// the next value of its session's counter.
struct ClaimBatch {
    uint32_t count;
    uint32_t sidx[kMaxTick];    // session counter
    uint32_t slot[kMaxTick];    // where the instance goes
    uint64_t session[kMaxTick];
};

__global__ void k_claim_tick(uint64_t *counters, uint64_t *slots, ClaimBatch b)
{
    if (threadIdx.x != 0) return;
    for (uint32_t e = 0; e < b.count; ++e) {
        const uint64_t c = counters[b.sidx[e]];
        counters[b.sidx[e]] = c + 1;
        slots[b.slot[e]] = (b.session[e] << kSessionShift) + c;
    }
}

struct Req {
    brr_request r;
    uint64_t footprint = 0;
    clock_t_::time_point t_submit, t_done;
    int slot = -1;
    uint32_t stream = 0;
    hipEvent_t ev = nullptr;
    brr_status status = BRR_OK;
    bool admitted = false, done = false;
};

double us_between(clock_t_::time_point a, clock_t_::time_point b)
{
    return std::chrono::duration<double, std::micro>(b - a).count();
}

} // namespace

struct brr_server {
    brr_server_config cfg;
    int device = 0;
    DevSched ds;
    hipStream_t control = nullptr;  // claims, fused small requests
    hipEvent_t claimed = nullptr;   // the last tick's claims are done
    std::vector<hipStream_t> streams;
    uint64_t *d_counters = nullptr; // [kMaxSessions]
    uint64_t *d_slots = nullptr;    // [max_inflight] instance of each in-flight request
    std::vector<hipEvent_t> slot_events; // [max_inflight] completion of each slot's request
    std::map<uint64_t, uint32_t> session_index;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<uint64_t> inflight;
    std::vector<int> free_slots;
    uint64_t next_id = 1, footprint = 0, peak_footprint = 0;
    uint32_t peak_inflight = 0;
    std::vector<double> latencies;
    uint64_t elems_done = 0, completed = 0;
    bool any_submit = false;
    clock_t_::time_point t_first, t_last;
    std::thread worker;
    bool stop = false;
};

namespace {

uint32_t session_of(brr_server *sv, uint64_t session, bool *ok)
{
    auto it = sv->session_index.find(session);
    if (it != sv->session_index.end()) return it->second;
    if (sv->session_index.size() >= kMaxSessions) {
        *ok = false;
        return 0;
    }
    const uint32_t sidx = (uint32_t)sv->session_index.size();
    sv->session_index.emplace(session, sidx);
    return sidx;
}

// One admitted request as the tick's launches see it: copied out of the
// request table, so that the launches run without the server's lock.
struct TickReq {
    uint64_t id;
    brr_request r;
    uint64_t footprint;
    int slot;
    uint32_t stream;
    hipEvent_t ev = nullptr;
    brr_status status = BRR_OK;
};

// Launches one tick of admitted requests; sets each request's status and
// completion event. Called with the server's lock held; the lock is
// released while the tick's kernels are launched (clients submit and wait
// meanwhile) and held again on return. Requests that fail are finished by
// the caller.
void launch_tick(brr_server *sv, const std::vector<uint64_t> &ids,
                 std::unique_lock<std::mutex> &lock)
{
    ClaimBatch cb;
    std::memset(&cb, 0, sizeof cb);
    std::vector<TickReq> t;
    t.reserve(ids.size());
    std::vector<size_t> fused, big, trivial;
    for (uint64_t id : ids) {
        Req &q = sv->reqs[id];
        bool ok = true;
        const uint32_t sidx = session_of(sv, q.r.session, &ok);
        if (!ok) {
            q.status = BRR_EINVAL;
            continue;
        }
        // every request takes its instance, even one that runs no kernel, so
        // each session's counter advances once per request in order
        cb.sidx[cb.count] = sidx;
        cb.slot[cb.count] = (uint32_t)q.slot;
        cb.session[cb.count] = q.r.session;
        ++cb.count;
        q.stream = sidx % (uint32_t)sv->streams.size();
        t.push_back(TickReq{id, q.r, q.footprint, q.slot, q.stream});
        const uint64_t n = q.r.n;
        const bool work = q.r.kind == BRR_REQ_SHUFFLE ? n > 1 : (n > 1 && q.r.m > 0);
        if (!work)
            trivial.push_back(t.size() - 1);
        else if (n <= lds_tier_max_n())
            fused.push_back(t.size() - 1);
        else
            big.push_back(t.size() - 1);
    }
    lock.unlock();
    hipStream_t ctl = sv->control;
    hipError_t e = hipSuccess;
    if (cb.count) {
        k_claim_tick<<<1, 64, 0, ctl>>>(sv->d_counters, sv->d_slots, cb);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(sv->claimed, ctl);
    }
    auto fail = [&](TickReq &q, hipError_t err) {
        q.status = err == hipErrorOutOfMemory ? BRR_ENOMEM : BRR_EHIP;
    };
    // small requests: one launch per (class, element width), up to
    // kMaxFusedRequests requests each
    if (e == hipSuccess) {
        for (int c = 0; c < kLdsClasses; ++c)
            for (uint32_t eb : {4u, 8u}) {
                ReqBatch rb;
                rb.count = 0;
                uint32_t max_n = 0;
                auto flush = [&] {
                    if (!rb.count || e != hipSuccess) return;
                    e = launch_lds_requests(c, eb, rb, max_n, sv->ds, sv->cfg.seed, sv->d_slots,
                                            ctl);
                    rb.count = 0;
                    max_n = 0;
                };
                for (size_t i : fused) {
                    const TickReq &q = t[i];
                    if (q.r.elem_bytes != eb || lds_request_class((uint32_t)q.r.n) != c) continue;
                    const uint32_t n = (uint32_t)q.r.n;
                    const bool sample = q.r.kind == BRR_REQ_SAMPLE;
                    const uint32_t steps = sample ? (uint32_t)std::min<uint64_t>(q.r.m, n - 1) : n - 1;
                    rb.r[rb.count++] = ReqDesc{q.r.d_data, sample ? q.r.d_out : nullptr, n, steps,
                                               sample ? (uint32_t)(n - q.r.m) : 0u,
                                               (uint32_t)q.slot};
                    max_n = std::max(max_n, n);
                    if (rb.count == kMaxFusedRequests) flush();
                }
                flush();
            }
    }
    for (size_t i : trivial) {
        const TickReq &q = t[i];
        if (e == hipSuccess && q.r.kind == BRR_REQ_SAMPLE && q.r.n == 1 && q.r.m == 1)
            e = hipMemcpyAsync(q.r.d_out, q.r.d_data, q.r.elem_bytes, hipMemcpyDeviceToDevice, ctl);
    }
    // the tick's small and trivial requests complete with the control stream
    for (const std::vector<size_t> *group : {&fused, &trivial})
        for (size_t i : *group) {
            TickReq &q = t[i];
            if (e != hipSuccess) {
                fail(q, e);
                continue;
            }
            q.ev = sv->slot_events[q.slot];
            if (hipEventRecord(q.ev, ctl) != hipSuccess) q.status = BRR_EHIP;
        }
    // large requests: each on its session's stream, behind the claims
    for (size_t i : big) {
        TickReq &q = t[i];
        if (e != hipSuccess) {
            fail(q, e);
            continue;
        }
        hipStream_t st = sv->streams[q.stream];
        const DevClaim claim{nullptr, sv->d_slots + q.slot, 0};
        const uint64_t n = q.r.n;
        // the stream's scratch buffer (requests on one stream run in turn)
        std::unique_lock<std::mutex> hold;
        void *scr = nullptr;
        const brr_status ss = stream_scratch(st, q.footprint, hold, &scr);
        if (ss != BRR_OK) {
            q.status = ss;
            continue;
        }
        hipError_t f = hipStreamWaitEvent(st, sv->claimed, 0);
        if (f == hipSuccess && q.r.kind == BRR_REQ_SHUFFLE)
            f = launch_one(q.r.d_data, (uint32_t)n, (uint32_t)(n - 1), 0, q.r.elem_bytes, nullptr,
                           sv->ds, sv->cfg.seed, 0, claim, st, scr);
        else if (f == hipSuccess)
            f = launch_one(q.r.d_data, (uint32_t)n, (uint32_t)std::min<uint64_t>(q.r.m, n - 1),
                           (uint32_t)(n - q.r.m), q.r.elem_bytes, q.r.d_out, sv->ds,
                           sv->cfg.seed, 0, claim, st, scr);
        if (f != hipSuccess) {
            fail(q, f);
            continue;
        }
        q.ev = sv->slot_events[q.slot];
        if (hipEventRecord(q.ev, st) != hipSuccess) q.status = BRR_EHIP;
    }
    lock.lock();
    for (const TickReq &q : t) {
        Req &r = sv->reqs[q.id];
        r.status = q.status;
        r.ev = q.ev;
    }
}

void finish(brr_server *sv, Req &q, uint64_t id)
{
    q.done = true;
    q.t_done = clock_t_::now();
    q.ev = nullptr;
    if (q.slot >= 0) sv->free_slots.push_back(q.slot);
    q.slot = -1;
    if (q.admitted) sv->footprint -= q.footprint;
    if (q.status == BRR_OK) {
        sv->latencies.push_back(us_between(q.t_submit, q.t_done));
        sv->elems_done += (q.r.kind == BRR_REQ_SHUFFLE) ? q.r.n : q.r.m;
        ++sv->completed;
        sv->t_last = q.t_done;
    }
    sv->inflight.erase(std::remove(sv->inflight.begin(), sv->inflight.end(), id),
                       sv->inflight.end());
}

void worker_loop(brr_server *sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lock(sv->mu);
    for (;;) {
        bool progress = false;
        // retire finished requests
        for (size_t i = 0; i < sv->inflight.size();) {
            const uint64_t id = sv->inflight[i];
            Req &q = sv->reqs[id];
            const hipError_t e = hipEventQuery(q.ev);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            if (e != hipSuccess) q.status = BRR_EHIP;
            finish(sv, q, id);
            progress = true;
        }
        // admit in arrival order while a slot and the scratch budget allow (an
        // idle device always takes the next request, whatever its
        // footprint), up to a tick's worth, then launch the tick together
        std::vector<uint64_t> tick;
        while (!sv->pending.empty() && tick.size() < kMaxTick) {
            const uint64_t id = sv->pending.front();
            Req &q = sv->reqs[id];
            const bool fits = sv->footprint + q.footprint <= sv->cfg.hbm_budget;
            if (sv->free_slots.empty() || (!fits && !sv->inflight.empty())) break;
            sv->pending.pop_front();
            q.slot = sv->free_slots.back();
            sv->free_slots.pop_back();
            q.admitted = true;
            sv->footprint += q.footprint;
            sv->peak_footprint = std::max(sv->peak_footprint, sv->footprint);
            sv->inflight.push_back(id);
            sv->peak_inflight = std::max<uint32_t>(sv->peak_inflight, (uint32_t)sv->inflight.size());
            tick.push_back(id);
        }
        if (!tick.empty()) {
            launch_tick(sv, tick, lock);
            for (uint64_t id : tick) {
                Req &q = sv->reqs[id];
                if (q.status != BRR_OK) finish(sv, q, id);
            }
            progress = true;
        }
        if (progress) sv->cv.notify_all();
        if (sv->stop && sv->pending.empty() && sv->inflight.empty()) break;
        if (!progress) {
            // nothing to do: wait for a submission, or keep polling the device
            // (a timed sleep would add its own wake-up latency to every
            // request)
            if (sv->inflight.empty()) {
                sv->cv.wait_for(lock, std::chrono::milliseconds(5));
            } else {
                lock.unlock();
                std::this_thread::yield();
                lock.lock();
            }
        }
    }
}

double percentile(std::vector<double> v, double p)
{
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    const size_t i = (size_t)std::min<double>(v.size() - 1, std::ceil(p * v.size()) - 1);
    return v[i];
}

} // namespace

extern "C" {

brr_status brr_server_create(brr_server **out, const brr_server_config *cfg)
{
    if (!out || !cfg || cfg->max_inflight == 0 || cfg->nstreams == 0 || cfg->nstreams > 64)
        return BRR_EINVAL;
    *out = nullptr;
    brr_schedule s6;
    brr_schedule_paper(6, &s6);
    const brr_schedule &sc = cfg->schedule ? *cfg->schedule : s6;
    if (brr_schedule_check_upto(&sc, 0xFFFFFFFFull) != BRR_OK) return BRR_EINVAL;
    const brr_status st = ensure_device();
    if (st != BRR_OK) return st;
    brr_server *sv = new (std::nothrow) brr_server();
    if (!sv) return BRR_ENOMEM;
    sv->cfg = *cfg;
    sv->cfg.schedule = nullptr;
    (void)hipGetDevice(&sv->device);
    // DevSched from the checked schedule
    sv->ds = dev_schedule(sc);
    bool ok = hipStreamCreateWithFlags(&sv->control, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&sv->claimed, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&sv->d_counters), kMaxSessions * 8) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&sv->d_slots), cfg->max_inflight * 8ull) == hipSuccess &&
              hipMemset(sv->d_counters, 0, kMaxSessions * 8) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
    for (uint32_t i = 0; ok && i < cfg->nstreams; ++i) {
        hipStream_t s;
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
        if (ok) sv->streams.push_back(s);
    }
    for (uint32_t i = 0; ok && i < cfg->max_inflight; ++i) {
        hipEvent_t ev;
        ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) sv->slot_events.push_back(ev);
    }
    if (!ok) {
        brr_server_destroy(sv);
        return BRR_EHIP;
    }
    for (int i = (int)cfg->max_inflight - 1; i >= 0; --i) sv->free_slots.push_back(i);
    sv->worker = std::thread(worker_loop, sv);
    *out = sv;
    return BRR_OK;
}

brr_status brr_server_submit(brr_server *sv, const brr_request *req, uint64_t *id)
{
    if (!sv || !req || !id) return BRR_EINVAL;
    const brr_request &r = *req;
    if (r.kind != BRR_REQ_SHUFFLE && r.kind != BRR_REQ_SAMPLE) return BRR_EINVAL;
    if ((r.elem_bytes != 4 && r.elem_bytes != 8) || r.n > 0xFFFFFFFFull) return BRR_EINVAL;
    if (r.n > 0 && !r.d_data) return BRR_EINVAL;
    if (misaligned(r.d_data, r.elem_bytes) || misaligned(r.d_out, r.elem_bytes)) return BRR_EINVAL;
    if (r.session >= (1ull << 24)) return BRR_EINVAL;
    if (r.kind == BRR_REQ_SAMPLE && (r.m > r.n || (r.m && !r.d_out))) return BRR_EINVAL;
    Req q;
    q.r = r;
    q.footprint = one_scratch_bytes(r.n, r.elem_bytes, r.kind == BRR_REQ_SAMPLE ? r.m : 0);
    q.t_submit = clock_t_::now();
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->stop) return BRR_EINVAL;
    const uint64_t nid = sv->next_id++;
    if (!sv->any_submit) {
        sv->any_submit = true;
        sv->t_first = q.t_submit;
    }
    sv->reqs.emplace(nid, q);
    sv->pending.push_back(nid);
    *id = nid;
    sv->cv.notify_all();
    return BRR_OK;
}

brr_status brr_server_wait(brr_server *sv, uint64_t id, double timeout_s, double *latency_us)
{
    if (!sv) return BRR_EINVAL;
    std::unique_lock<std::mutex> lock(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return BRR_EINVAL;
    const auto deadline = clock_t_::now() + std::chrono::duration<double>(timeout_s);
    while (!sv->reqs[id].done) {
        if (sv->cv.wait_until(lock, deadline) == std::cv_status::timeout && !sv->reqs[id].done)
            return BRR_EDEVICE;
    }
    const Req &q = sv->reqs[id];
    if (latency_us) *latency_us = us_between(q.t_submit, q.t_done);
    const brr_status st = q.status;
    sv->reqs.erase(id);
    return st;
}

brr_status brr_server_drain(brr_server *sv, double timeout_s)
{
    if (!sv) return BRR_EINVAL;
    std::unique_lock<std::mutex> lock(sv->mu);
    const auto deadline = clock_t_::now() + std::chrono::duration<double>(timeout_s);
    while (!sv->pending.empty() || !sv->inflight.empty()) {
        if (sv->cv.wait_until(lock, deadline) == std::cv_status::timeout &&
            (!sv->pending.empty() || !sv->inflight.empty()))
            return BRR_EDEVICE;
    }
    for (auto it = sv->reqs.begin(); it != sv->reqs.end();)
        it = it->second.done ? sv->reqs.erase(it) : std::next(it);
    return BRR_OK;
}

brr_status brr_server_get_stats(brr_server *sv, brr_server_stats *out)
{
    if (!sv || !out) return BRR_EINVAL;
    std::lock_guard<std::mutex> lock(sv->mu);
    std::memset(out, 0, sizeof *out);
    out->completed = sv->completed;
    out->elements = sv->elems_done;
    out->p50_us = percentile(sv->latencies, 0.50);
    out->p99_us = percentile(sv->latencies, 0.99);
    double sum = 0;
    for (double v : sv->latencies) sum += v;
    out->mean_us = sv->latencies.empty() ? 0 : sum / sv->latencies.size();
    out->max_us = sv->latencies.empty() ? 0 : *std::max_element(sv->latencies.begin(), sv->latencies.end());
    const double wall = sv->completed ? us_between(sv->t_first, sv->t_last) * 1e-6 : 0;
    out->wall_s = wall;
    out->requests_per_s = wall > 0 ? sv->completed / wall : 0;
    out->elements_per_s = wall > 0 ? sv->elems_done / wall : 0;
    out->peak_inflight = sv->peak_inflight;
    out->peak_footprint = sv->peak_footprint;
    return BRR_OK;
}

brr_status brr_server_reset_stats(brr_server *sv)
{
    if (!sv) return BRR_EINVAL;
    std::lock_guard<std::mutex> lock(sv->mu);
    sv->latencies.clear();
    sv->completed = sv->elems_done = 0;
    sv->peak_inflight = 0;
    sv->peak_footprint = sv->footprint;
    sv->any_submit = false;
    return BRR_OK;
}

brr_status brr_server_session_counter(brr_server *sv, uint64_t session, uint64_t *value)
{
    if (!sv || !value) return BRR_EINVAL;
    uint32_t sidx;
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        auto it = sv->session_index.find(session);
        if (it == sv->session_index.end()) {
            *value = 0;
            return BRR_OK;
        }
        sidx = it->second;
        if (hipStreamSynchronize(sv->control) != hipSuccess) return BRR_EHIP;
    }
    if (hipMemcpy(value, sv->d_counters + sidx, 8, hipMemcpyDeviceToHost) != hipSuccess)
        return BRR_EHIP;
    return BRR_OK;
}

void brr_server_destroy(brr_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(sv->device);
    for (hipStream_t s : sv->streams) {
        (void)hipStreamSynchronize(s);
        (void)drop_stream_scratch(s); // the stream's scratch buffer goes with it
        (void)hipStreamDestroy(s);
    }
    if (sv->control) {
        (void)hipStreamSynchronize(sv->control);
        (void)hipStreamDestroy(sv->control);
    }
    if (sv->claimed) (void)hipEventDestroy(sv->claimed);
    for (hipEvent_t ev : sv->slot_events) (void)hipEventDestroy(ev);
    if (sv->d_counters) (void)hipFree(sv->d_counters);
    if (sv->d_slots) (void)hipFree(sv->d_slots);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete sv;
}

} // extern "C"
