// Serving loop: resident label indexes answer streams of query requests with
// continuous batching, and labeling jobs are admitted by free device memory.
//
// A scheduler thread owns a pool of slots (one stream, pinned staging and
// device buffers each).  Whenever a slot is free it packs the queued query
// requests of one index, oldest first, into one device batch (a request
// larger than the batch is carried by several batches), launches the
// merge-join query kernel and copies results back on the slot's stream.
// Completed batches are scattered to their requests.  Slots run
// concurrently, so batches overlap on the device with each other and with
// label builds, which a second thread runs on their own stream: it admits
// queued labeling jobs while hipMemGetInfo reports room for them and labels
// all admitted jobs in one launch.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "pll_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t id = 0;
    pll_request r{};
    double t_arrival = 0, t_admit = -1, t_done = 0;
    int status = PLL_OK;
    uint64_t next = 0;       // first pair not yet given to a batch
    uint64_t remaining = 0;  // pairs not yet answered
    uint32_t batch_requests = 0;
    uint32_t new_index = 0;
    // device interval (seconds after the server's reference event) of the
    // query kernels that carried its pairs, or of the build launch of a job
    double dev_start = -1, dev_end = -1;
};

struct Member {
    Req* req;
    uint64_t src;    // first pair of the request carried by this batch
    uint64_t dst;    // position in the batch
    uint64_t count;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t k0 = nullptr, k1 = nullptr;  // around the batch's query kernel (timing events)
    uint32_t *h_u = nullptr, *h_v = nullptr, *h_out = nullptr;
    uint32_t *d_u = nullptr, *d_v = nullptr, *d_out = nullptr;
    uint64_t cap = 0;
    bool busy = false;
    std::vector<Member> members;
};

// The server holds one reference on every resident index: the caller's
// handed-over reference (take_ownership, and the indexes the server built),
// or one it takes itself; pll_server_destroy drops them all.
struct IndexEntry {
    pll_index* idx = nullptr;
};

uint64_t build_bytes_estimate(uint32_t n, uint64_t nnz, uint32_t b) {
    const uint64_t W = (b + 63) / 64;
    const uint64_t work = n * (64 * W)                 // distance table
                          + n * 8 * W * 4              // C, msgs, two active deltas
                          + n * 4ull * PLL_SHARDS * 3  // sharded queues
                          + n * 64ull                  // per-vertex arrays
                          + 16 * nnz;                  // CSR copies
    const uint64_t labels = 3 * (16ull * n + 4 * nnz * 8) * 4;  // label arena, generous
    return work + labels;
}

}  // namespace

struct pll_server {
    int device = 0;
    pll_server_opts opts{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Req*> queries;
    std::deque<Req*> builds;
    std::vector<Req*> completed;  // not yet polled
    std::map<uint64_t, Req*> all;
    std::map<uint32_t, IndexEntry> indexes;
    uint32_t next_index = 1;
    uint64_t next_id = 1;
    uint64_t outstanding = 0;
    bool stop = false;
    std::vector<Slot> slots;
    hipStream_t build_stream = nullptr;
    hipEvent_t ev_ref = nullptr;  // device time origin of the results' dev_start / dev_end
    std::thread sched, builder;

    // seconds from ev_ref to a completed timing event (-1 if unavailable)
    double dev_time(hipEvent_t e) const {
        float ms = 0;
        return hipEventElapsedTime(&ms, ev_ref, e) == hipSuccess ? ms / 1e3 : -1.0;
    }

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    void finish(Req* q, int status) {  // caller holds mu
        q->status = status;
        q->t_done = now();
        completed.push_back(q);
        --outstanding;
        done_cv.notify_all();
    }

    // scheduler: retire finished batches, then fill free slots
    void run_sched() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool any_busy = false;
            for (Slot& s : slots) {
                if (!s.busy) continue;
                const hipError_t q = hipEventQuery(s.done);
                if (q == hipErrorNotReady) {
                    any_busy = true;
                    continue;
                }
                // finished, or failed: a device error ends the batch's requests
                // with PLL_EDEVICE instead of keeping the slot busy for ever
                const bool ok = q == hipSuccess;
                const double d0 = ok ? dev_time(s.k0) : -1, d1 = ok ? dev_time(s.k1) : -1;
                for (const Member& m : s.members) {
                    Req* r = m.req;
                    if (ok) std::memcpy(r->r.h_out + m.src, s.h_out + m.dst, sizeof(uint32_t) * m.count);
                    else r->status = PLL_EDEVICE;
                    if (r->dev_start < 0 || (d0 >= 0 && d0 < r->dev_start)) r->dev_start = d0;
                    r->dev_end = std::max(r->dev_end, d1);
                    r->remaining -= m.count;
                    if (r->remaining == 0) finish(r, r->status);
                }
                s.members.clear();
                s.busy = false;
            }
            for (Slot& s : slots) {
                if (s.busy || queries.empty()) continue;
                fill_slot(s);
                any_busy = any_busy || s.busy;
            }
            if (stop && queries.empty() && !any_busy) break;
            if (any_busy)
                cv.wait_for(lk, std::chrono::microseconds(20));
            else
                cv.wait_for(lk, std::chrono::milliseconds(2));
        }
    }

    // pack queued requests of the head's index into slot s (mu held)
    void fill_slot(Slot& s) {
        Req* head = queries.front();
        auto it = indexes.find(head->r.index_id);
        if (it == indexes.end()) {
            queries.pop_front();
            finish(head, PLL_EINVAL);
            return;
        }
        const uint32_t index_id = head->r.index_id;
        const pll_index* idx = it->second.idx;
        uint64_t used = 0;
        uint32_t nreq = 0;
        for (auto q = queries.begin(); q != queries.end() && used < s.cap;) {
            Req* r = *q;
            if (r->r.index_id != index_id) {
                ++q;
                continue;
            }
            const uint64_t take = std::min<uint64_t>(r->r.count - r->next, s.cap - used);
            std::memcpy(s.h_u + used, r->r.h_u + r->next, sizeof(uint32_t) * take);
            std::memcpy(s.h_v + used, r->r.h_v + r->next, sizeof(uint32_t) * take);
            s.members.push_back(Member{r, r->next, used, take});
            if (r->t_admit < 0) r->t_admit = now();
            r->next += take;
            used += take;
            ++nreq;
            if (r->next == r->r.count)
                q = queries.erase(q);
            else
                break;  // the batch is full
        }
        for (const Member& m : s.members)
            if (m.src == 0) m.req->batch_requests = nreq;
        bool ok = hipMemcpyAsync(s.d_u, s.h_u, sizeof(uint32_t) * used, hipMemcpyHostToDevice, s.stream) == hipSuccess &&
                  hipMemcpyAsync(s.d_v, s.h_v, sizeof(uint32_t) * used, hipMemcpyHostToDevice, s.stream) == hipSuccess &&
                  hipEventRecord(s.k0, s.stream) == hipSuccess &&
                  pll_query_launch(idx, used, s.d_u, s.d_v, s.d_out, s.stream) == PLL_OK &&
                  hipEventRecord(s.k1, s.stream) == hipSuccess &&
                  hipMemcpyAsync(s.h_out, s.d_out, sizeof(uint32_t) * used, hipMemcpyDeviceToHost, s.stream) == hipSuccess &&
                  hipEventRecord(s.done, s.stream) == hipSuccess;
        if (!ok) {
            for (const Member& m : s.members) {
                m.req->remaining -= m.count;
                if (m.req->remaining == 0) finish(m.req, PLL_EDEVICE);
            }
            s.members.clear();
            return;
        }
        s.busy = true;
    }

    // build worker: admit queued labeling jobs, oldest first, while their
    // estimated footprint fits in free device memory (less the reserve), and
    // label everything admitted together: one many-graph persistent launch
    // for small graphs, the grid-wide single-graph build for a lone or large
    // one.  A job that could never fit on the device fails with ENOMEM.
    void run_builder() {
        (void)hipSetDevice(device);
        const uint32_t b = opts.build_batch_size ? opts.build_batch_size : PLL_BMAX;
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            if (builds.empty()) {
                if (stop) break;
                cv.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            if (stop) {  // shutting down: jobs not started yet are dropped
                Req* q = builds.front();
                builds.pop_front();
                finish(q, PLL_ENOMEM);
                continue;
            }
            size_t free_b = 0, total_b = 0;
            lk.unlock();
            const bool info_ok = hipMemGetInfo(&free_b, &total_b) == hipSuccess;
            free_b += pll_ws_cached(device);  // cached build workspace is free for builds
            lk.lock();
            std::vector<Req*> take;
            uint64_t need_sum = opts.mem_reserve;
            while (info_ok && !builds.empty() && take.size() < kMaxJobsPerLaunch) {
                Req* q = builds.front();
                const uint64_t need = build_bytes_estimate(q->r.n, q->r.nnz, b);
                if (need + opts.mem_reserve > total_b) {  // can never fit
                    builds.pop_front();
                    finish(q, PLL_ENOMEM);
                    continue;
                }
                if (need_sum + need > free_b) break;
                need_sum += need;
                builds.pop_front();
                q->t_admit = now();
                take.push_back(q);
            }
            if (take.empty()) {
                cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
            lk.unlock();
            std::vector<pll_index*> idx(take.size(), nullptr);
            std::vector<int> rc(take.size(), PLL_OK);
            const bool timed = hipEventRecord(b0, build_stream) == hipSuccess;
            build_jobs(take, b, idx.data(), rc.data());
            const bool timed_end = timed && hipEventRecord(b1, build_stream) == hipSuccess;
            (void)hipStreamSynchronize(build_stream);
            const double d0 = timed_end ? dev_time(b0) : -1, d1 = timed_end ? dev_time(b1) : -1;
            lk.lock();
            for (Req* q : take) {
                q->dev_start = d0;
                q->dev_end = d1;
            }
            for (size_t i = 0; i < take.size(); ++i) {
                if (rc[i] == PLL_OK) {
                    const uint32_t id = next_index++;
                    indexes[id] = IndexEntry{idx[i]};
                    take[i]->new_index = id;
                }
                finish(take[i], rc[i]);
            }
        }
    }

    static constexpr size_t kMaxJobsPerLaunch = 256;
    static constexpr uint32_t kBuildWorkgroups = 128;  // of 1,024 threads: a quarter of the device's wave slots
    static constexpr uint32_t kLargeGraph = 1u << 16;  // built alone, grid-wide

    hipEvent_t b0 = nullptr, b1 = nullptr;  // around each build launch (timing events)

    // device staging for the host CSRs of admitted jobs (grows, kept)
    void* stage = nullptr;
    uint64_t stage_cap = 0;

    static uint64_t up256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

    // upload the CSRs of `jobs` and label them; rc[i] is job i's status
    void build_jobs(const std::vector<Req*>& jobs, uint32_t b, pll_index** idx, int* rc) {
        const size_t k = jobs.size();
        uint64_t bytes = 0;
        for (Req* q : jobs) {
            const pll_request& r = q->r;
            if (r.n && (!r.h_row_ptr || !r.h_order || (r.nnz && !r.h_col))) continue;
            bytes += up256(8 * (uint64_t(r.n) + 1)) + up256(4 * r.nnz) + up256(4 * uint64_t(r.n));
        }
        if (bytes > stage_cap) {
            if (stage) (void)hipFree(stage);
            stage = nullptr;
            stage_cap = 0;
            if (hipMalloc(&stage, bytes) != hipSuccess) {
                stage = nullptr;
                for (size_t i = 0; i < k; ++i) rc[i] = PLL_ENOMEM;
                return;
            }
            stage_cap = bytes;
        }
        std::vector<pll_graph_desc> desc(k);
        std::vector<size_t> small;  // jobs for the many-graph launch
        char* p = static_cast<char*>(stage);
        for (size_t i = 0; i < k; ++i) {
            const pll_request& r = jobs[i]->r;
            if (r.n && (!r.h_row_ptr || !r.h_order || (r.nnz && !r.h_col))) {
                rc[i] = PLL_EINVAL;
                continue;
            }
            pll_graph_desc& d = desc[i];
            d.n = r.n;
            d.nnz = r.nnz;
            d.d_row_ptr = reinterpret_cast<const uint64_t*>(p);
            p += up256(8 * (uint64_t(r.n) + 1));
            d.d_col = reinterpret_cast<const uint32_t*>(p);
            p += up256(4 * r.nnz);
            d.d_order = reinterpret_cast<const uint32_t*>(p);
            p += up256(4 * uint64_t(r.n));
            const bool ok =
                (!r.n || (hipMemcpyAsync(const_cast<uint64_t*>(d.d_row_ptr), r.h_row_ptr, 8 * (uint64_t(r.n) + 1),
                                         hipMemcpyHostToDevice, build_stream) == hipSuccess &&
                          hipMemcpyAsync(const_cast<uint32_t*>(d.d_order), r.h_order, 4 * uint64_t(r.n),
                                         hipMemcpyHostToDevice, build_stream) == hipSuccess)) &&
                (!r.nnz || hipMemcpyAsync(const_cast<uint32_t*>(d.d_col), r.h_col, 4 * r.nnz, hipMemcpyHostToDevice,
                                          build_stream) == hipSuccess);
            if (!ok) {
                rc[i] = PLL_EDEVICE;
                continue;
            }
            if (r.n < kLargeGraph) small.push_back(i);
        }
        pll_build_opts o{};
        o.batch_size = b;
        o.flags = PLL_FLAG_VALIDATE;
        o.max_workgroups = opts.build_workgroups ? opts.build_workgroups : kBuildWorkgroups;
        bool batched = false;
        if (small.size() > 1) {
            std::vector<pll_graph_desc> sd(small.size());
            std::vector<pll_index*> so(small.size(), nullptr);
            for (size_t j = 0; j < small.size(); ++j) sd[j] = desc[small[j]];
            if (pll_build_multi(uint32_t(small.size()), sd.data(), &o, build_stream, so.data()) == PLL_OK) {
                for (size_t j = 0; j < small.size(); ++j) idx[small[j]] = so[j];
                batched = true;
            }
            // on failure every job is built alone below, so that only the
            // offending job reports the error
        }
        for (size_t i = 0; i < k; ++i) {
            if (rc[i] != PLL_OK || idx[i]) continue;
            if (batched && jobs[i]->r.n < kLargeGraph) continue;
            const pll_request& r = jobs[i]->r;
            rc[i] = pll_build_one(r.n, r.nnz, desc[i].d_row_ptr, desc[i].d_col, desc[i].d_order, &o, build_stream,
                                  &idx[i]);
        }
    }
};

namespace {

void destroy_server(pll_server* s) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->sched.joinable()) s->sched.join();
    if (s->builder.joinable()) s->builder.join();
    (void)hipSetDevice(s->device);
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.k0) (void)hipEventDestroy(sl.k0);
        if (sl.k1) (void)hipEventDestroy(sl.k1);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.h_u) (void)hipHostFree(sl.h_u);
        if (sl.h_v) (void)hipHostFree(sl.h_v);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.d_u) (void)hipFree(sl.d_u);
        if (sl.d_v) (void)hipFree(sl.d_v);
        if (sl.d_out) (void)hipFree(sl.d_out);
    }
    if (s->build_stream) (void)hipStreamSynchronize(s->build_stream);
    if (s->stage) (void)hipFree(s->stage);
    if (s->build_stream) (void)hipStreamDestroy(s->build_stream);
    if (s->b0) (void)hipEventDestroy(s->b0);
    if (s->b1) (void)hipEventDestroy(s->b1);
    if (s->ev_ref) (void)hipEventDestroy(s->ev_ref);
    for (auto& kv : s->indexes) pll_index_free(kv.second.idx);  // the server's reference
    for (auto& kv : s->all) delete kv.second;
    delete s;
}

int submit_locked(pll_server* s, const pll_request* req, double arrival, uint64_t* id) {
    if (req->kind == PLL_REQ_QUERY) {
        if (req->count && (!req->h_u || !req->h_v || !req->h_out)) return PLL_EINVAL;
    } else if (req->kind != PLL_REQ_BUILD) {
        return PLL_EINVAL;
    }
    Req* q = new (std::nothrow) Req{};
    if (!q) return PLL_ENOMEM;
    q->id = s->next_id++;
    q->r = *req;
    q->t_arrival = arrival;
    q->remaining = req->count;
    s->all[q->id] = q;
    ++s->outstanding;
    if (req->kind == PLL_REQ_QUERY) {
        if (req->count == 0) {
            q->t_admit = s->now();
            s->finish(q, PLL_OK);
        } else {
            s->queries.push_back(q);
        }
    } else {
        s->builds.push_back(q);
    }
    if (id) *id = q->id;
    return PLL_OK;
}

void fill_result(const Req* q, pll_result* r) {
    r->id = q->id;
    r->status = q->status;
    r->kind = q->r.kind;
    r->index_id = q->r.kind == PLL_REQ_BUILD ? q->new_index : q->r.index_id;
    r->batch_requests = q->batch_requests;
    r->t_arrival = q->t_arrival;
    r->t_admit = q->t_admit;
    r->t_done = q->t_done;
    r->t_dev_start = q->dev_start;
    r->t_dev_end = q->dev_end;
}

}  // namespace

extern "C" {

int pll_server_create(const pll_server_opts* opts, pll_server** out) {
    if (!out) return PLL_EINVAL;
    *out = nullptr;
    pll_server_opts o{};
    if (opts) o = *opts;
    for (uint32_t r : o.reserved)
        if (r) return PLL_EINVAL;
    const uint32_t nslots = o.slots ? o.slots : 4;
    if (nslots > 16) return PLL_EINVAL;
    const uint64_t cap = o.max_batch_pairs ? o.max_batch_pairs : (1ull << 20);
    if (o.mem_reserve == 0) o.mem_reserve = 1ull << 30;
    pll_server* s = new (std::nothrow) pll_server{};
    if (!s) return PLL_ENOMEM;
    s->opts = o;
    s->t0 = Clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return PLL_EDEVICE;
    }
    s->slots.resize(nslots);
    bool ok = hipStreamCreateWithFlags(&s->build_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreate(&s->b0) == hipSuccess && hipEventCreate(&s->b1) == hipSuccess &&
              hipEventCreate(&s->ev_ref) == hipSuccess && hipEventRecord(s->ev_ref, s->build_stream) == hipSuccess &&
              hipEventSynchronize(s->ev_ref) == hipSuccess;
    for (Slot& sl : s->slots) {
        sl.cap = cap;
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
             hipEventCreate(&sl.k0) == hipSuccess && hipEventCreate(&sl.k1) == hipSuccess &&
             hipHostMalloc((void**)&sl.h_u, 4 * cap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&sl.h_v, 4 * cap, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&sl.h_out, 4 * cap, hipHostMallocDefault) == hipSuccess &&
             hipMalloc((void**)&sl.d_u, 4 * cap) == hipSuccess && hipMalloc((void**)&sl.d_v, 4 * cap) == hipSuccess &&
             hipMalloc((void**)&sl.d_out, 4 * cap) == hipSuccess;
    }
    if (!ok) {
        destroy_server(s);
        return PLL_ENOMEM;
    }
    try {
        s->sched = std::thread([s] { s->run_sched(); });
        s->builder = std::thread([s] { s->run_builder(); });
    } catch (...) {
        destroy_server(s);
        return PLL_ENOMEM;
    }
    *out = s;
    return PLL_OK;
}

int pll_server_add_index(pll_server* s, pll_index* idx, int take_ownership, uint32_t* index_id) {
    if (!s || !idx || !index_id) return PLL_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const uint32_t id = s->next_index++;
    if (!take_ownership) pll_index_retain(idx);  // the caller keeps its own reference
    s->indexes[id] = IndexEntry{idx};
    *index_id = id;
    return PLL_OK;
}

int pll_server_index(pll_server* s, uint32_t index_id, pll_index** idx) {
    if (!s || !idx) return PLL_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->indexes.find(index_id);
    if (it == s->indexes.end()) return PLL_EINVAL;
    *idx = it->second.idx;
    return PLL_OK;
}

int pll_server_submit(pll_server* s, const pll_request* req, uint64_t* id) {
    if (!s || !req) return PLL_EINVAL;
    int rc;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        rc = submit_locked(s, req, s->now(), id);
    }
    s->cv.notify_all();
    return rc;
}

int pll_server_poll(pll_server* s, pll_result* out, uint32_t max, uint32_t* got, int wait) {
    if (!s || !got || (max && !out)) return PLL_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (wait)
        s->done_cv.wait(lk, [s] { return !s->completed.empty() || s->outstanding == 0; });
    const uint32_t k = (uint32_t)std::min<size_t>(max, s->completed.size());
    for (uint32_t i = 0; i < k; ++i) {
        Req* q = s->completed[i];
        fill_result(q, &out[i]);
        s->all.erase(q->id);
        delete q;
    }
    s->completed.erase(s->completed.begin(), s->completed.begin() + k);
    *got = k;
    return PLL_OK;
}

int pll_server_replay(pll_server* s, uint64_t count, const pll_request* reqs, pll_result* results) {
    if (!s || (count && (!reqs || !results))) return PLL_EINVAL;
    std::vector<uint64_t> ids(count, 0);
    const double start = s->now();
    for (uint64_t i = 0; i < count;) {
        const double due = start + reqs[i].at;
        for (;;) {  // open loop: wait for the arrival time, never for earlier requests
            const double t = s->now();
            if (t >= due) break;
            if (due - t > 2e-4)
                std::this_thread::sleep_for(std::chrono::duration<double>(due - t - 1e-4));
        }
        // every request already due goes in under one lock and one wake-up,
        // so a burst reaches the scheduler whole instead of one by one
        int rc = PLL_OK;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const double t = s->now();
            do {
                rc = submit_locked(s, &reqs[i], start + reqs[i].at, &ids[i]);
                ++i;
            } while (rc == PLL_OK && i < count && start + reqs[i].at <= t);
        }
        s->cv.notify_all();
        if (rc != PLL_OK) return rc;
    }
    // collect every replayed request
    std::map<uint64_t, uint64_t> pos;
    for (uint64_t i = 0; i < count; ++i) pos[ids[i]] = i;
    uint64_t left = count;
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<Req*> others;  // finished requests that are not this replay's
    while (left) {
        s->done_cv.wait(lk, [s] { return !s->completed.empty(); });
        std::vector<Req*> done;
        done.swap(s->completed);
        for (Req* q : done) {
            auto p = pos.find(q->id);
            if (p == pos.end()) {
                others.push_back(q);
                continue;
            }
            fill_result(q, &results[p->second]);
            s->all.erase(q->id);
            delete q;
            --left;
        }
    }
    s->completed.insert(s->completed.begin(), others.begin(), others.end());
    return PLL_OK;
}

void pll_server_destroy(pll_server* s) {
    if (s) destroy_server(s);
}

}  // extern "C"
