// Continuous-batching request loop on top of the batched search (serving entry points of mrq.h).
//
// A host worker thread owns two batch slots, each with its own HIP stream, its own auxiliary stream and
// events for the search's seed-pass fork, pinned staging buffers and a device buffer.  Requests wait in a
// FIFO until a slot is free; the worker then admits requests in arrival order while the slot has room
// (max_slots queries) and the device memory of the batch (workspace + staging, sized for the admitted mix
// of k and nprobe) fits the slot's buffer.  With a memory budget each slot's buffer is half of it,
// allocated when the server is created, so the server's device memory never exceeds the budget and
// nothing is allocated or freed while batches run (a free would synchronise the device and stall the
// other slot).  The batch is copied to the device, searched with per-query k / nprobe, and copied back on
// the slot's stream; the worker polls the slot's event and hands finished rows to mrq_server_poll.  With
// two slots one batch is packed and launched while the other is still running.  Search results do not
// depend on the batch a query is in, so a request returns the same ids and distances alone and in any mix.
// The server shares only the index's read-only arrays: the index may be searched directly meanwhile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mrq_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id;
    int32_t k, nprobe;
    std::vector<float> q;
    Clock::time_point t0;
};

struct Done {
    uint64_t id;
    int32_t k;
    std::vector<int64_t> ids;
    std::vector<float> dists;
    double latency_ms;
};

template <class T>
struct Pinned {
    T* p = nullptr;
    size_t n = 0;
    bool reserve(size_t want) {
        if (want <= n) return true;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        if (hipHostMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(want, 1) * sizeof(T), 0) != hipSuccess) return false;
        n = want;
        return true;
    }
    ~Pinned() { if (p) (void)hipHostFree(p); }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    hipStream_t aux = nullptr;                     // the seed pass of this slot's searches
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool busy = false;
    std::vector<Request> reqs;
    std::vector<int64_t> out_off;
    size_t reserved = 0;           // device bytes this batch accounts for
    void* dev = nullptr;           // device buffer: metadata, queries, outputs, workspace
    size_t dev_bytes = 0;
    Pinned<char> h_meta;
    Pinned<float> h_q;
    Pinned<int64_t> h_ids;
    Pinned<float> h_d;
};

}  // namespace

struct mrq_server {
    const mrq_index* ix = nullptr;
    const mrq::Index* core = nullptr;
    size_t budget = 0;
    int max_slots = 1;
    mrq_search_opts opts;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    std::deque<Done> done;
    std::atomic<int64_t> submitted{0}, completed{0};
    std::atomic<bool> stop{false};
    std::string error;
    Slot slots[2];
    std::thread worker;
    std::vector<void*> retired;          // outgrown slot buffers (no budget), freed with the server
    std::atomic<int64_t> dev_bytes{0};   // device bytes the server holds
    std::atomic<int64_t> dev_peak{0};
    std::atomic<int64_t> batches{0};
    std::atomic<int32_t> max_in_flight{0};
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device bytes of a batch: metadata, queries, outputs and the search workspace.
size_t batch_bytes(const mrq::Index& ix, int64_t nq, int64_t slots, int64_t pairs, int np_max,
                   const mrq_search_opts& o) {
    size_t b = align256(nq * 4) * 2 + align256((nq + 1) * 8) * 2 + align256(nq * 8);
    b += align256(nq * (size_t)ix.D * 4) + align256(slots * 8) + align256(slots * 4);
    b += mrq::search_workspace_bytes(ix, nq, slots, pairs, o.bq, np_max, o.method, o.rerank);
    return b;
}

bool launch_batch(mrq_server* sv, Slot& sl) {
    const mrq::Index& ix = *sv->core;
    const int64_t nq = (int64_t)sl.reqs.size();
    int64_t tslots = 0, tpairs = 0;
    int np_max = 0, k_max = 0;
    for (auto& r : sl.reqs) {
        tslots += r.k;
        tpairs += r.nprobe;
        np_max = std::max(np_max, r.nprobe);
        k_max = std::max(k_max, r.k);
    }
    const size_t need = batch_bytes(ix, nq, tslots, tpairs, np_max, sv->opts);
    if (sl.dev_bytes < need) {
        // only without a budget (a budgeted slot's buffer is allocated at creation and admission keeps the
        // batch within it); the old buffer is kept until the server ends, as freeing it would synchronise
        if (sv->budget) return false;
        void* nb = nullptr;
        if (hipMalloc(&nb, need + need / 4) != hipSuccess) return false;
        if (sl.dev) sv->retired.push_back(sl.dev);
        sl.dev = nb;
        sl.dev_bytes = need + need / 4;
        const int64_t tot = sv->dev_bytes += (int64_t)sl.dev_bytes;
        int64_t pk = sv->dev_peak.load();
        while (tot > pk && !sv->dev_peak.compare_exchange_weak(pk, tot)) {}
    }
    sl.reserved = need;
    // carve the device buffer
    char* p = reinterpret_cast<char*>(sl.dev);
    auto take = [&](size_t b) { char* r = p; p += align256(b); return r; };
    int32_t* d_kq = reinterpret_cast<int32_t*>(take(nq * 4));
    int32_t* d_np = reinterpret_cast<int32_t*>(take(nq * 4));
    int64_t* d_so = reinterpret_cast<int64_t*>(take((nq + 1) * 8));
    int64_t* d_po = reinterpret_cast<int64_t*>(take((nq + 1) * 8));
    int64_t* d_oo = reinterpret_cast<int64_t*>(take(nq * 8));
    float* d_q = reinterpret_cast<float*>(take(nq * (size_t)ix.D * 4));
    int64_t* d_ids = reinterpret_cast<int64_t*>(take(tslots * 8));
    float* d_d = reinterpret_cast<float*>(take(tslots * 4));
    void* ws = p;
    const size_t ws_bytes = sl.dev_bytes - (size_t)(p - reinterpret_cast<char*>(sl.dev));
    // host staging: metadata packed in the same order as on the device
    const size_t meta_bytes = nq * 4 * 2 + (nq + 1) * 8 * 2 + nq * 8;
    if (!sl.h_meta.reserve(meta_bytes) || !sl.h_q.reserve(nq * (size_t)ix.D) || !sl.h_ids.reserve(tslots) ||
        !sl.h_d.reserve(tslots))
        return false;  // sized for max_slots at creation: only grows when that failed
    int32_t* h_kq = reinterpret_cast<int32_t*>(sl.h_meta.p);
    int32_t* h_np = h_kq + nq;
    int64_t* h_so = reinterpret_cast<int64_t*>(h_np + nq);
    int64_t* h_po = h_so + nq + 1;
    int64_t* h_oo = h_po + nq + 1;
    sl.out_off.assign(nq, 0);
    h_so[0] = 0;
    h_po[0] = 0;
    for (int64_t i = 0; i < nq; i++) {
        const Request& r = sl.reqs[i];
        h_kq[i] = r.k;
        h_np[i] = r.nprobe;
        h_so[i + 1] = h_so[i] + r.k;
        h_po[i + 1] = h_po[i] + r.nprobe;
        h_oo[i] = h_so[i];
        sl.out_off[i] = h_so[i];
        std::memcpy(sl.h_q.p + i * ix.D, r.q.data(), sizeof(float) * ix.D);
    }
    hipStream_t s = sl.stream;
    if (hipMemcpyAsync(d_kq, h_kq, nq * 4, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    if (hipMemcpyAsync(d_np, h_np, nq * 4, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    if (hipMemcpyAsync(d_so, h_so, (nq + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    if (hipMemcpyAsync(d_po, h_po, (nq + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    if (hipMemcpyAsync(d_oo, h_oo, nq * 8, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    if (hipMemcpyAsync(d_q, sl.h_q.p, nq * (size_t)ix.D * 4, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    mrq::SearchArgs a;
    a.ix = &ix;
    a.Q = d_q;
    a.nq = nq;
    a.kq = d_kq;
    a.npq = d_np;
    a.slot_off = d_so;
    a.pair_off = d_po;
    a.out_off = d_oo;
    a.total_slots = tslots;
    a.total_pairs = tpairs;
    a.np_max = np_max;
    a.k_max = k_max;
    a.bq = sv->opts.bq;
    a.eps0 = sv->opts.eps0;
    a.m = sv->opts.m;
    a.stage2 = sv->opts.stage2;
    a.use_ext = sv->opts.use_ext;
    a.group = sv->opts.group > 0 ? sv->opts.group : ix.group_default;
    a.method = sv->opts.method;
    a.rerank = sv->opts.rerank;
    a.phase_shift = mrq::phase_shift_of(sv->opts.phase_growth, ix.phase_shift_default);
    a.ids = d_ids;
    a.dists = d_d;
    a.counters = nullptr;
    a.timed = false;
    a.aux = sl.aux;
    a.ev_fork = sl.ev_fork;
    a.ev_join = sl.ev_join;
    if (mrq::launch_search(a, ws, ws_bytes, s) != hipSuccess) return false;
    if (hipMemcpyAsync(sl.h_ids.p, d_ids, tslots * 8, hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipMemcpyAsync(sl.h_d.p, d_d, tslots * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipEventRecord(sl.done_ev, s) != hipSuccess) return false;
    sl.busy = true;
    sv->batches++;
    const int32_t now = (int32_t)sv->slots[0].busy + (int32_t)sv->slots[1].busy;
    int32_t m = sv->max_in_flight.load();
    while (now > m && !sv->max_in_flight.compare_exchange_weak(m, now)) {}
    return true;
}

void harvest(mrq_server* sv, Slot& sl) {
    const auto now = Clock::now();
    std::vector<Done> out;
    out.reserve(sl.reqs.size());
    for (size_t i = 0; i < sl.reqs.size(); i++) {
        const Request& r = sl.reqs[i];
        Done d;
        d.id = r.id;
        d.k = r.k;
        d.ids.assign(sl.h_ids.p + sl.out_off[i], sl.h_ids.p + sl.out_off[i] + r.k);
        d.dists.assign(sl.h_d.p + sl.out_off[i], sl.h_d.p + sl.out_off[i] + r.k);
        d.latency_ms = std::chrono::duration<double, std::milli>(now - r.t0).count();
        out.push_back(std::move(d));
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto& d : out) sv->done.push_back(std::move(d));
    }
    sv->completed += (int64_t)sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    sl.reserved = 0;
    sv->cv.notify_all();
}

void worker_loop(mrq_server* sv) {
    (void)hipSetDevice(sv->core->device);
    while (!sv->stop.load()) {
        bool progressed = false;
        for (Slot& sl : sv->slots) {
            if (sl.busy && hipEventQuery(sl.done_ev) == hipSuccess) {
                harvest(sv, sl);
                progressed = true;
            }
        }
        for (int si = 0; si < 2; si++) {
            Slot& sl = sv->slots[si];
            if (sl.busy) continue;
            const size_t cap = sv->budget ? sl.dev_bytes : 0;  // a budgeted slot's fixed buffer
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                int64_t tslots = 0, tpairs = 0;
                int np_max = 0;
                while (!sv->queue.empty() && (int)sl.reqs.size() < sv->max_slots) {
                    const Request& r = sv->queue.front();
                    const int np2 = std::max(np_max, r.nprobe);
                    const size_t need = batch_bytes(*sv->core, (int64_t)sl.reqs.size() + 1, tslots + r.k,
                                                    tpairs + r.nprobe, np2, sv->opts);
                    if (cap && need > cap) break;  // admit later, in the next batch of a slot
                    tslots += r.k;
                    tpairs += r.nprobe;
                    np_max = np2;
                    sl.reqs.push_back(std::move(sv->queue.front()));
                    sv->queue.pop_front();
                }
            }
            if (!sl.reqs.empty()) {
                if (!launch_batch(sv, sl)) {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    sv->error = "batch launch failed";
                    // fail the batch: report every request with an empty result
                    for (auto& r : sl.reqs) {
                        Done d;
                        d.id = r.id;
                        d.k = r.k;
                        d.ids.assign(r.k, -1);
                        d.dists.assign(r.k, INFINITY);
                        d.latency_ms = -1.0;
                        sv->done.push_back(std::move(d));
                    }
                    sv->completed += (int64_t)sl.reqs.size();
                    sl.reqs.clear();
                    sl.busy = false;
                }
                progressed = true;
            }
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(sv->mu);
            const bool any_busy = sv->slots[0].busy || sv->slots[1].busy;
            if (sv->queue.empty() && !any_busy)
                sv->cv.wait_for(lk, std::chrono::milliseconds(5));
            else
                sv->cv.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

}  // namespace

extern "C" {

mrq_status mrq_server_create(const mrq_index* index, size_t mem_budget, int32_t max_slots,
                             const mrq_search_opts* opts, mrq_server** out) {
    if (!index || !out) return MRQ_EINVAL;
    if (max_slots < 1 || max_slots > 65536) return MRQ_EINVAL;
    mrq_server* sv = new (std::nothrow) mrq_server();
    if (!sv) return MRQ_ENOMEM;
    sv->ix = index;
    sv->core = index;
    sv->budget = mem_budget;
    sv->max_slots = max_slots;
    mrq_search_opts_default(&sv->opts);
    if (opts) {
        sv->opts = *opts;
        if (sv->opts.bq == 0) sv->opts.bq = 4;
        if (!(sv->opts.eps0 > 0.f)) sv->opts.eps0 = 1.9f;
        if (!(sv->opts.m > 0.f)) sv->opts.m = 3.f;
    }
    sv->opts.counters = nullptr;
    sv->opts.mode = MRQ_BATCHED;
    if (sv->opts.bq < 1 || sv->opts.bq > 8) { delete sv; return MRQ_EINVAL; }
    if (sv->opts.rerank == 0) sv->opts.rerank = 500;
    if ((sv->opts.method != MRQ_METHOD_MRQ && sv->opts.method != MRQ_METHOD_MRSQ) || sv->opts.rerank < 1 ||
        sv->opts.rerank > 16384) { delete sv; return MRQ_EINVAL; }
    if (sv->opts.method == MRQ_METHOD_MRSQ && sv->core->dq == 0) { delete sv; return MRQ_ESTATE; }
    if (mrq::phase_shift_of(sv->opts.phase_growth, 1) < 0) { delete sv; return MRQ_EINVAL; }
    (void)hipSetDevice(sv->core->device);
    const mrq::Index& ix = *sv->core;
    for (Slot& sl : sv->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) != hipSuccess ||
            hipStreamCreateWithFlags(&sl.aux, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev_join, hipEventDisableTiming) != hipSuccess) {
            mrq_server_destroy(sv);
            return MRQ_EDEVICE;
        }
        // pinned staging for a full batch of the largest requests
        const size_t ms = (size_t)max_slots;
        if (!sl.h_meta.reserve(ms * 4 * 2 + (ms + 1) * 8 * 2 + ms * 8) || !sl.h_q.reserve(ms * (size_t)ix.D) ||
            !sl.h_ids.reserve(ms * mrq::kMaxK) || !sl.h_d.reserve(ms * mrq::kMaxK)) {
            mrq_server_destroy(sv);
            return MRQ_ENOMEM;
        }
        if (sv->budget) {  // each slot holds half of the budget for the server's lifetime
            sl.dev_bytes = (sv->budget / 2) & ~(size_t)255;
            if (hipMalloc(&sl.dev, std::max<size_t>(sl.dev_bytes, 256)) != hipSuccess) {
                sl.dev = nullptr;
                sl.dev_bytes = 0;
                mrq_server_destroy(sv);
                return MRQ_ENOMEM;
            }
            sv->dev_bytes += (int64_t)sl.dev_bytes;
        }
    }
    sv->dev_peak = sv->dev_bytes.load();
    sv->worker = std::thread(worker_loop, sv);
    *out = sv;
    return MRQ_OK;
}

mrq_status mrq_server_submit(mrq_server* sv, uint64_t req_id, const float* q_host, int32_t k, int32_t nprobe) {
    if (!sv || !q_host) return MRQ_EINVAL;
    const mrq::Index& ix = *sv->core;
    if (k < 1 || k > mrq::kMaxK || nprobe < 1 || nprobe > std::min(ix.nlist, mrq::kMaxProbe)) return MRQ_EINVAL;
    if (sv->opts.method == MRQ_METHOD_MRSQ && k > sv->opts.rerank) return MRQ_EINVAL;
    if (sv->budget && batch_bytes(ix, 1, k, nprobe, nprobe, sv->opts) > sv->slots[0].dev_bytes) return MRQ_ENOMEM;
    Request r;
    r.id = req_id;
    r.k = k;
    r.nprobe = nprobe;
    r.q.assign(q_host, q_host + ix.D);
    r.t0 = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->queue.push_back(std::move(r));
    }
    sv->submitted++;
    sv->cv.notify_all();
    return MRQ_OK;
}

int mrq_server_poll(mrq_server* sv, uint64_t* req_ids, int32_t* ks, int64_t* ids, float* dists, int32_t row,
                    int32_t max_done, double* latency_ms) {
    if (!sv || max_done < 0 || (max_done > 0 && (!req_ids || !ids || !dists || row < 1))) return -1;
    std::lock_guard<std::mutex> lk(sv->mu);
    int n = 0;
    while (n < max_done && !sv->done.empty()) {
        Done& d = sv->done.front();
        if (d.k > row) return n > 0 ? n : -1;
        req_ids[n] = d.id;
        if (ks) ks[n] = d.k;
        std::copy(d.ids.begin(), d.ids.end(), ids + (int64_t)n * row);
        std::copy(d.dists.begin(), d.dists.end(), dists + (int64_t)n * row);
        if (latency_ms) latency_ms[n] = d.latency_ms;
        sv->done.pop_front();
        n++;
    }
    return n;
}

mrq_status mrq_server_drain(mrq_server* sv, int64_t timeout_ms) {
    if (!sv) return MRQ_EINVAL;
    const auto until = Clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (sv->completed.load() < sv->submitted.load()) {
        if (sv->cv.wait_until(lk, until) == std::cv_status::timeout && sv->completed.load() < sv->submitted.load())
            return MRQ_ESTATE;
    }
    return MRQ_OK;
}

void mrq_server_destroy(mrq_server* sv) {
    if (!sv) return;
    sv->stop = true;
    sv->cv.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    for (Slot& sl : sv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.aux) (void)hipStreamSynchronize(sl.aux);
    }
    for (Slot& sl : sv->slots) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
        if (sl.ev_fork) (void)hipEventDestroy(sl.ev_fork);
        if (sl.ev_join) (void)hipEventDestroy(sl.ev_join);
        if (sl.aux) (void)hipStreamDestroy(sl.aux);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (void* p : sv->retired) (void)hipFree(p);
    delete sv;
}

mrq_status mrq_server_stats(const mrq_server* sv, int64_t* device_bytes, int64_t* peak_device_bytes,
                            int64_t* batches, int32_t* max_in_flight) {
    if (!sv) return MRQ_EINVAL;
    if (device_bytes) *device_bytes = sv->dev_bytes.load();
    if (peak_device_bytes) *peak_device_bytes = sv->dev_peak.load();
    if (batches) *batches = sv->batches.load();
    if (max_in_flight) *max_in_flight = sv->max_in_flight.load();
    return MRQ_OK;
}

}  // extern "C"
