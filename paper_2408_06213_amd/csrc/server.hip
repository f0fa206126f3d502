// Serving loop with continuous batching: shuffle and sample requests are
// admitted as in-flight slots and device scratch free up, run concurrently on
// a pool of HIP streams, and retired as their completion events fire.
//
// Generator counters live on the device: every session owns a counter, and a
// one-thread claim kernel on the session's stream hands each request the
// next instance (session * 2^40 + counter) in submission order. A request's
// result is therefore fixed by (session, its place in the session), whatever
// else runs beside it.
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

__global__ void k_claim(uint64_t *counter, uint64_t *slot, uint64_t session)
{
    const uint64_t c = *counter;
    *counter = c + 1;
    *slot = (session << kSessionShift) + c;
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

// Launches an admitted request on its session's stream (lock held).
brr_status launch(brr_server *sv, Req &q)
{
    const brr_request &r = q.r;
    uint32_t sidx;
    auto it = sv->session_index.find(r.session);
    if (it == sv->session_index.end()) {
        if (sv->session_index.size() >= kMaxSessions) return BRR_EINVAL;
        sidx = (uint32_t)sv->session_index.size();
        sv->session_index.emplace(r.session, sidx);
    } else {
        sidx = it->second;
    }
    q.stream = sidx % (uint32_t)sv->streams.size();
    hipStream_t s = sv->streams[q.stream];
    uint64_t *slot = sv->d_slots + q.slot;
    // the request's first kernel claims its instance; a request that runs no
    // kernel still takes one, so every session's counter advances once per
    // request in submission order
    const DevClaim claim{sv->d_counters + sidx, slot, r.session << kSessionShift};
    const uint64_t n = r.n;
    hipError_t e = hipSuccess;
    bool claimed = false;
    if (r.kind == BRR_REQ_SHUFFLE) {
        if (n > 1) {
            e = launch_one(r.d_data, (uint32_t)n, (uint32_t)(n - 1), 0, r.elem_bytes, nullptr,
                           sv->ds, sv->cfg.seed, 0, claim, s);
            claimed = true;
        }
    } else {
        if (n == 1) {
            e = hipMemcpyAsync(r.d_out, r.d_data, r.elem_bytes, hipMemcpyDeviceToDevice, s);
        } else if (r.m > 0) {
            e = launch_one(r.d_data, (uint32_t)n, (uint32_t)std::min<uint64_t>(r.m, n - 1),
                           (uint32_t)(n - r.m), r.elem_bytes, r.d_out, sv->ds, sv->cfg.seed, 0,
                           claim, s);
            claimed = true;
        }
    }
    // a device-wide request whose scratch could not be allocated failed before
    // its first kernel: its instance is still taken
    if (!claimed || e == hipErrorOutOfMemory) {
        k_claim<<<1, 1, 0, s>>>(sv->d_counters + sidx, slot, r.session);
        const hipError_t f = hipGetLastError();
        if (e == hipSuccess) e = f;
    }
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? BRR_ENOMEM : BRR_EHIP;
    q.ev = sv->slot_events[q.slot];
    if (hipEventRecord(q.ev, s) != hipSuccess) return BRR_EHIP;
    return BRR_OK;
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
        // admit in arrival order while a slot and the scratch budget allow; an
        // idle device always takes the next request, whatever its footprint
        while (!sv->pending.empty()) {
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
            q.status = launch(sv, q);
            if (q.status != BRR_OK) finish(sv, q, id);
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
    bool ok = hipMalloc(reinterpret_cast<void **>(&sv->d_counters), kMaxSessions * 8) == hipSuccess &&
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
        hipStream_t s = sv->streams[sidx % sv->streams.size()];
        if (hipStreamSynchronize(s) != hipSuccess) return BRR_EHIP;
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
    for (hipStream_t s : sv->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t ev : sv->slot_events) (void)hipEventDestroy(ev);
    if (sv->d_counters) (void)hipFree(sv->d_counters);
    if (sv->d_slots) (void)hipFree(sv->d_slots);
    delete sv;
}

} // extern "C"
