// Serving loop: continuous batching of (c,k)-ANN requests on a resident
// index. Requests wait in arrival order; one host worker thread forms each
// launch from the waiting requests in arrival order, whatever their k, c,
// confidence, beta and r_min (Algorithm 2 is run per query with its own
// parameters, so a launch changes no answer), gathers their queries and
// per-query parameters into the buffers of a launch slot, runs the batched
// ANN path on them and scatters the answers. A launch is admitted while a
// slot is free and the workspace of the launches in flight stays within the
// HBM budget. Each slot owns its device buffers (queries, answers,
// parameters, workspace), a pinned host buffer for the parameters and a
// completion event, all created with the server and grown only when a
// launch needs more, so serving does not allocate.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

#include "internal.hpp"

namespace pmlsh {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const float* q = nullptr;
    int64_t nq = 0;
    int32_t k = 0;
    double c = 0, confidence = 0, beta = 0, r_min = 0;
    AnnQueryParams params{};      // the plan of every query of the request
    int64_t* out_ids = nullptr;
    float* out_dist = nullptr;
    hipEvent_t ready = nullptr;   // work of the submitting stream, or null
    bool ready_waited = false;
    int64_t issued = 0;           // queries handed to launches
    int64_t finished = 0;         // queries whose launch completed
    int status = PMLSH_OK;
    bool done = false;
    Clock::time_point t_submit;
};

struct Segment {
    std::shared_ptr<Request> req;
    int64_t req_off, count;
};

// Buffers of one launch slot, grown (never shrunk) to the largest launch
// it has served.
struct Slot {
    float* q = nullptr;                 // queries, max_batch x d
    int64_t* ids = nullptr;             // answers, rows of kcap
    float* dist = nullptr;
    AnnQueryParams* params = nullptr;   // device, per query
    AnnQueryParams* hparams = nullptr;  // pinned host staging of the same
    void* ws = nullptr;                 // ANN workspace
    int64_t rows = 0, kcap = 0, ws_bytes = 0;
    hipEvent_t done = nullptr;
};

struct Launch {
    std::vector<Segment> segs;
    int slot = -1;
    int64_t bytes = 0;
    int status = PMLSH_OK;
};

}  // namespace
}  // namespace pmlsh

struct pmlsh_server {
    const pmlsh_index* idx = nullptr;
    int64_t max_batch = 1024;
    int max_inflight = 2;
    int64_t hbm_budget = int64_t(8) << 30;
    hipStream_t stream = nullptr;

    std::mutex mu;
    std::condition_variable cv_work;   // worker: new requests or stop
    std::condition_variable cv_done;   // waiters: a request completed
    std::deque<std::shared_ptr<pmlsh::Request>> waiting;   // queries left to issue
    std::unordered_map<uint64_t, std::shared_ptr<pmlsh::Request>> by_ticket;
    uint64_t next_ticket = 1;
    bool stop = false;

    // worker-only state
    std::deque<pmlsh::Launch> inflight;
    int64_t bytes_inflight = 0;
    std::vector<pmlsh::Slot> slots;
    std::vector<int> free_slots;

    // counters (under mu)
    int64_t n_requests = 0, n_queries = 0, n_launches = 0;
    std::vector<double> latency_ms;

    std::thread worker;
};

namespace pmlsh {
namespace {

// Finishes the oldest launch if its slot's event has completed (or fails
// it); with block, waits for it. Returns true if a launch was retired.
bool retire_one(pmlsh_server* s, bool block) {
    if (s->inflight.empty()) return false;
    Launch& L = s->inflight.front();
    Slot& sl = s->slots[(size_t)L.slot];
    hipError_t e = block ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess && L.status == PMLSH_OK) L.status = PMLSH_EDEVICE;
    const auto now = Clock::now();
    {
        std::lock_guard<std::mutex> g(s->mu);
        for (auto& sg : L.segs) {
            Request& r = *sg.req;
            if (L.status != PMLSH_OK && r.status == PMLSH_OK) r.status = L.status;
            r.finished += sg.count;
            if (r.finished == r.nq && !r.done) {
                r.done = true;
                if (r.ready) (void)hipEventDestroy(r.ready);
                r.ready = nullptr;
                ++s->n_requests;
                s->n_queries += r.nq;
                s->latency_ms.push_back(
                    std::chrono::duration<double, std::milli>(now - r.t_submit).count());
            }
        }
        ++s->n_launches;
    }
    s->bytes_inflight -= L.bytes;
    s->free_slots.push_back(L.slot);
    s->inflight.pop_front();
    s->cv_done.notify_all();
    return true;
}

// Takes the next launch's segments from the waiting requests (under mu): in
// arrival order, up to max_batch queries; a larger request is split.
std::vector<Segment> take_batch(pmlsh_server* s) {
    std::vector<Segment> segs;
    int64_t room = s->max_batch;
    for (auto it = s->waiting.begin(); it != s->waiting.end() && room > 0;) {
        Request& r = **it;
        const int64_t take = std::min(room, r.nq - r.issued);
        segs.push_back({*it, r.issued, take});
        r.issued += take;
        room -= take;
        if (r.issued == r.nq) it = s->waiting.erase(it);
        else ++it;
    }
    return segs;
}

// Puts segments back at the front of the queue (a launch that could not be
// admitted yet).
void untake(pmlsh_server* s, std::vector<Segment>& segs) {
    for (auto it = segs.rbegin(); it != segs.rend(); ++it) {
        Request& r = *it->req;
        const bool was_out = r.issued == r.nq;
        r.issued -= it->count;
        if (was_out) s->waiting.push_front(it->req);
    }
    // restore arrival order of the requests put back
    std::stable_sort(s->waiting.begin(), s->waiting.end(),
                     [](const std::shared_ptr<Request>& a, const std::shared_ptr<Request>& b) {
                         return a->ticket < b->ticket;
                     });
}

// Shape of a launch: queries, largest k and budget.
struct Shape {
    int64_t nb = 0;
    int kmax = 1;
    int64_t bmax = 1;
};

Shape shape_of(const std::vector<Segment>& segs) {
    Shape sh;
    for (auto& sg : segs) {
        sh.nb += sg.count;
        sh.kmax = std::max(sh.kmax, sg.req->params.k);
        sh.bmax = std::max<int64_t>(sh.bmax, sg.req->params.budget);
    }
    return sh;
}

int64_t launch_bytes(const pmlsh_server* s, const Shape& sh) {
    return ann_workspace_bytes_mixed(s->idx, sh.nb, sh.kmax, sh.bmax);
}

void slot_release(Slot& sl) {
    (void)hipFree(sl.q);
    (void)hipFree(sl.ids);
    (void)hipFree(sl.dist);
    (void)hipFree(sl.params);
    (void)hipHostFree(sl.hparams);
    (void)hipFree(sl.ws);
    sl.q = nullptr;
    sl.ids = nullptr;
    sl.dist = nullptr;
    sl.params = nullptr;
    sl.hparams = nullptr;
    sl.ws = nullptr;
    sl.rows = sl.kcap = sl.ws_bytes = 0;
}

// Sizes a slot for `rows` queries with answers of up to kcap entries and a
// workspace of ws_bytes (called with the slot idle).
void slot_reserve(const pmlsh_server* s, Slot& sl, int64_t rows, int64_t kcap, int64_t ws_bytes) {
    if (rows > sl.rows || kcap > sl.kcap) {
        rows = std::max(rows, sl.rows);
        kcap = std::max(kcap, sl.kcap);
        (void)hipFree(sl.q);
        (void)hipFree(sl.ids);
        (void)hipFree(sl.dist);
        (void)hipFree(sl.params);
        (void)hipHostFree(sl.hparams);
        sl.q = nullptr;
        sl.ids = nullptr;
        sl.dist = nullptr;
        sl.params = nullptr;
        sl.hparams = nullptr;
        sl.rows = sl.kcap = 0;
        PMLSH_HIP(hipMalloc(&sl.q, (size_t)rows * s->idx->d * sizeof(float)));
        PMLSH_HIP(hipMalloc(&sl.ids, (size_t)rows * kcap * sizeof(int64_t)));
        PMLSH_HIP(hipMalloc(&sl.dist, (size_t)rows * kcap * sizeof(float)));
        PMLSH_HIP(hipMalloc(&sl.params, (size_t)rows * sizeof(AnnQueryParams)));
        PMLSH_HIP(hipHostMalloc(&sl.hparams, (size_t)rows * sizeof(AnnQueryParams),
                                hipHostMallocDefault));
        sl.rows = rows;
        sl.kcap = kcap;
    }
    if (ws_bytes > sl.ws_bytes) {
        (void)hipFree(sl.ws);
        sl.ws = nullptr;
        sl.ws_bytes = 0;
        PMLSH_HIP(hipMalloc(&sl.ws, (size_t)ws_bytes));
        sl.ws_bytes = ws_bytes;
    }
}

// Issues one launch on the server's stream in its slot. Errors fail the
// launch's requests; the slot's event still marks the point after which its
// buffers are free.
void issue(pmlsh_server* s, Launch& L, const Shape& shp) {
    const int d = s->idx->d;
    hipStream_t st = s->stream;
    Slot& sl = s->slots[(size_t)L.slot];
    L.status = guarded([&] {
        slot_reserve(s, sl, shp.nb, shp.kmax, L.bytes);
        if (L.segs.size() == 1) {
            // one request: its own queries and outputs, its plan as scalars
            const Segment& sg = L.segs.front();
            Request& r = *sg.req;
            if (r.ready && !r.ready_waited) {
                PMLSH_HIP(hipStreamWaitEvent(st, r.ready, 0));
                r.ready_waited = true;
            }
            const AnnQueryParams& p = r.params;
            run_ann_planned(s->idx, r.q + sg.req_off * d, sg.count, p, r.out_ids + sg.req_off * r.k,
                            r.out_dist + sg.req_off * r.k, st, sl.ws, sl.ws_bytes);
            return;
        }
        int64_t off = 0;
        for (auto& sg : L.segs) {
            Request& r = *sg.req;
            if (r.ready && !r.ready_waited) {
                PMLSH_HIP(hipStreamWaitEvent(st, r.ready, 0));
                r.ready_waited = true;
            }
            PMLSH_HIP(hipMemcpyAsync(sl.q + off * d, r.q + sg.req_off * d,
                                     (size_t)sg.count * d * 4, hipMemcpyDeviceToDevice, st));
            for (int64_t i = 0; i < sg.count; ++i) sl.hparams[off + i] = r.params;
            off += sg.count;
        }
        PMLSH_HIP(hipMemcpyAsync(sl.params, sl.hparams, (size_t)shp.nb * sizeof(AnnQueryParams),
                                 hipMemcpyHostToDevice, st));
        run_ann_mixed(s->idx, sl.q, shp.nb, sl.params, shp.kmax, shp.bmax, shp.kmax, sl.ids,
                      sl.dist, nullptr, st, sl.ws, sl.ws_bytes);
        off = 0;
        for (auto& sg : L.segs) {
            Request& r = *sg.req;
            const size_t k = (size_t)r.k;
            PMLSH_HIP(hipMemcpy2DAsync(r.out_ids + sg.req_off * r.k, k * 8, sl.ids + off * shp.kmax,
                                       (size_t)shp.kmax * 8, k * 8, (size_t)sg.count,
                                       hipMemcpyDeviceToDevice, st));
            PMLSH_HIP(hipMemcpy2DAsync(r.out_dist + sg.req_off * r.k, k * 4,
                                       sl.dist + off * shp.kmax, (size_t)shp.kmax * 4, k * 4,
                                       (size_t)sg.count, hipMemcpyDeviceToDevice, st));
            off += sg.count;
        }
    });
    if (hipEventRecord(sl.done, st) != hipSuccess) {
        (void)hipStreamSynchronize(st);
        if (L.status == PMLSH_OK) L.status = PMLSH_EDEVICE;
        // the event's last record stands for an earlier launch: its query
        // would report this one as complete, which after the synchronisation
        // above it is
    }
}

void worker_loop(pmlsh_server* s) {
    (void)hipSetDevice(s->idx->device);
    for (;;) {
        // retire what has completed
        while (retire_one(s, false)) {
        }
        // admit launches while a slot and the budget allow
        while (!s->free_slots.empty()) {
            std::vector<Segment> segs;
            Shape shp;
            int64_t bytes = 0;
            {
                std::lock_guard<std::mutex> g(s->mu);
                segs = take_batch(s);
                if (segs.empty()) break;
                shp = shape_of(segs);
                bytes = launch_bytes(s, shp);
                if (!s->inflight.empty() && s->bytes_inflight + bytes > s->hbm_budget) {
                    untake(s, segs);
                    break;
                }
            }
            s->inflight.emplace_back();
            Launch& L = s->inflight.back();
            L.segs = std::move(segs);
            L.bytes = bytes;
            L.slot = s->free_slots.back();
            s->free_slots.pop_back();
            s->bytes_inflight += bytes;
            issue(s, L, shp);
        }
        if (!s->inflight.empty()) {
            bool can_admit = false;
            {
                std::lock_guard<std::mutex> g(s->mu);
                can_admit = !s->waiting.empty() && !s->free_slots.empty();
            }
            if (!can_admit) {
                // nothing to admit until a launch completes: wait for the
                // oldest, unless requests arrive that a free slot could take
                std::unique_lock<std::mutex> lk(s->mu);
                if (s->free_slots.empty() || s->waiting.empty()) {
                    if (s->free_slots.empty()) {
                        lk.unlock();
                        retire_one(s, true);
                    } else {
                        s->cv_work.wait_for(lk, std::chrono::microseconds(10),
                                            [&] { return s->stop || !s->waiting.empty(); });
                    }
                }
            }
            continue;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->waiting.empty()) {
            if (s->stop) break;
            s->cv_work.wait(lk, [&] { return s->stop || !s->waiting.empty(); });
            if (s->stop && s->waiting.empty()) break;
        }
    }
}

}  // namespace
}  // namespace pmlsh

using namespace pmlsh;

extern "C" {

int pmlsh_server_create(const pmlsh_index* index, const pmlsh_server_args* args,
                        pmlsh_server** out) {
    return guarded([&] {
        if (!index || !out) fail(PMLSH_EINVAL, "NULL argument");
        auto s = std::make_unique<pmlsh_server>();
        s->idx = index;
        if (args) {
            if (args->max_batch < 0 || args->max_batch > 65535)
                fail(PMLSH_EINVAL, "max_batch must be in 0..65535");
            if (args->max_inflight < 0 || args->max_inflight > 64)
                fail(PMLSH_EINVAL, "max_inflight must be in 0..64");
            if (args->hbm_budget < 0) fail(PMLSH_EINVAL, "hbm_budget must be >= 0");
            if (args->max_batch > 0) s->max_batch = args->max_batch;
            if (args->max_inflight > 0) s->max_inflight = args->max_inflight;
            if (args->hbm_budget > 0) s->hbm_budget = args->hbm_budget;
        }
        PMLSH_HIP(hipSetDevice(index->device));
        PMLSH_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        auto cleanup = [&] {
            for (auto& sl : s->slots) {
                slot_release(sl);
                if (sl.done) (void)hipEventDestroy(sl.done);
            }
            (void)hipStreamDestroy(s->stream);
        };
        try {
            // slots sized for full launches of k up to 100 within the
            // batched path's budget limit; larger launches grow them
            s->slots.resize((size_t)s->max_inflight);
            const int64_t ws0 =
                ann_workspace_bytes_mixed(index, s->max_batch, std::min<int64_t>(100, index->n),
                                          std::min<int64_t>(2048, index->n));
            for (int i = 0; i < s->max_inflight; ++i) {
                Slot& sl = s->slots[(size_t)i];
                PMLSH_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
                slot_reserve(s.get(), sl, s->max_batch, std::min<int64_t>(100, index->n), ws0);
                s->free_slots.push_back(s->max_inflight - 1 - i);
            }
        } catch (...) {
            cleanup();
            throw;
        }
        try {
            s->worker = std::thread(worker_loop, s.get());
        } catch (const std::exception&) {
            cleanup();
            fail(PMLSH_EDEVICE, "cannot start the server thread");
        }
        *out = s.release();
    });
}

int pmlsh_server_submit(pmlsh_server* server, const float* queries, int64_t nq, int32_t k,
                        double c, double confidence, double beta, double r_min,
                        int64_t* out_ids, float* out_dist, void* stream, uint64_t* ticket) {
    return guarded([&] {
        if (!server || !ticket) fail(PMLSH_EINVAL, "NULL argument");
        validate_ann(server->idx, queries, nq, k, out_ids, out_dist, r_min);
        // the request's plan (parameter checks included), before anything is queued
        const pmlsh_query_args qa{k, 0, c, confidence, beta, r_min};
        std::vector<AnnQueryParams> plan;
        int kmax = 1;
        int64_t bmax = 1;
        plan_queries(server->idx, &qa, 1, &plan, &kmax, &bmax);
        auto r = std::make_shared<Request>();
        r->params = plan[0];
        r->q = queries;
        r->nq = nq;
        r->k = k;
        r->c = c;
        r->confidence = confidence;
        r->beta = beta;
        r->r_min = r_min > 0.0 ? r_min : 0.0;
        r->out_ids = out_ids;
        r->out_dist = out_dist;
        r->t_submit = Clock::now();
        if (stream && nq > 0) {
            PMLSH_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
            if (hipEventRecord(r->ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
                (void)hipEventDestroy(r->ready);
                fail(PMLSH_EDEVICE, "hipEventRecord on the submitting stream failed");
            }
        }
        std::lock_guard<std::mutex> g(server->mu);
        if (server->stop) fail(PMLSH_EINVAL, "server is shutting down");
        r->ticket = server->next_ticket++;
        server->by_ticket[r->ticket] = r;
        if (nq == 0) {
            r->done = true;
        } else {
            server->waiting.push_back(r);
            server->cv_work.notify_one();
        }
        *ticket = r->ticket;
    });
}

int pmlsh_server_test(pmlsh_server* server, uint64_t ticket, int* done) {
    return guarded([&] {
        if (!server || !done) fail(PMLSH_EINVAL, "NULL argument");
        std::lock_guard<std::mutex> g(server->mu);
        auto it = server->by_ticket.find(ticket);
        if (it == server->by_ticket.end()) fail(PMLSH_EINVAL, "unknown ticket");
        *done = it->second->done ? 1 : 0;
    });
}

int pmlsh_server_wait(pmlsh_server* server, uint64_t ticket) {
    int status = PMLSH_OK;
    const int rc = guarded([&] {
        if (!server) fail(PMLSH_EINVAL, "server is NULL");
        std::unique_lock<std::mutex> lk(server->mu);
        auto it = server->by_ticket.find(ticket);
        if (it == server->by_ticket.end()) fail(PMLSH_EINVAL, "unknown ticket");
        std::shared_ptr<Request> r = it->second;
        server->cv_done.wait(lk, [&] { return r->done; });
        server->by_ticket.erase(ticket);
        status = r->status;
    });
    if (rc != PMLSH_OK) return rc;
    if (status != PMLSH_OK) set_error("the request's launch failed");
    return status;
}

int pmlsh_server_get_stats(pmlsh_server* server, pmlsh_server_stats* out) {
    return guarded([&] {
        if (!server || !out) fail(PMLSH_EINVAL, "NULL argument");
        std::vector<double> lat;
        pmlsh_server_stats st{};
        {
            std::lock_guard<std::mutex> g(server->mu);
            st.requests = server->n_requests;
            st.queries = server->n_queries;
            st.launches = server->n_launches;
            lat = server->latency_ms;
        }
        if (!lat.empty()) {
            std::sort(lat.begin(), lat.end());
            auto pct = [&](double p) {
                const size_t i = (size_t)std::ceil(p * (double)lat.size()) - 1;
                return lat[std::min(i, lat.size() - 1)];
            };
            st.latency_p50_ms = pct(0.50);
            st.latency_p99_ms = pct(0.99);
            st.latency_max_ms = lat.back();
        }
        *out = st;
    });
}

void pmlsh_server_destroy(pmlsh_server* server) {
    if (!server) return;
    {
        std::lock_guard<std::mutex> g(server->mu);
        server->stop = true;
    }
    server->cv_work.notify_all();
    if (server->worker.joinable()) server->worker.join();
    if (server->stream) {
        (void)hipStreamSynchronize(server->stream);
        for (auto& sl : server->slots) {
            slot_release(sl);
            if (sl.done) (void)hipEventDestroy(sl.done);
        }
        (void)hipStreamDestroy(server->stream);
    }
    delete server;
}

}  // extern "C"
