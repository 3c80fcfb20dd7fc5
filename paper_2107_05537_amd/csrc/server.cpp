// Serving loop: continuous batching of (c,k)-ANN requests on a resident
// index. Requests wait in arrival order; one host worker thread forms each
// launch from the oldest waiting request and the later requests with the same
// parameters (Algorithm 2 is run per query, so queries of different requests
// with equal parameters can share a launch without changing any answer),
// gathers their queries into a staging buffer on the server's stream, runs
// the batched ANN path and scatters the answers. Launches are admitted while
// a launch slot is free and the staging plus workspace bytes in flight stay
// within the HBM budget; completions are found by polling one HIP event per
// launch.
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
    int64_t* out_ids = nullptr;
    float* out_dist = nullptr;
    hipEvent_t ready = nullptr;   // work of the submitting stream, or null
    bool ready_waited = false;
    int64_t issued = 0;           // queries handed to launches
    int64_t finished = 0;         // queries whose launch completed
    int status = PMLSH_OK;
    bool done = false;
    Clock::time_point t_submit;

    bool same_class(const Request& o) const {
        return k == o.k && c == o.c && confidence == o.confidence && beta == o.beta &&
               r_min == o.r_min;
    }
};

struct Segment {
    std::shared_ptr<Request> req;
    int64_t req_off, count;
};

struct Launch {
    std::vector<Segment> segs;
    hipEvent_t done = nullptr;
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

    // counters (under mu)
    int64_t n_requests = 0, n_queries = 0, n_launches = 0;
    std::vector<double> latency_ms;

    std::thread worker;
};

namespace pmlsh {
namespace {

// Finishes the oldest launch if its event has completed (or fails it).
// Returns true if a launch was retired.
bool retire_one(pmlsh_server* s, bool block) {
    if (s->inflight.empty()) return false;
    Launch& L = s->inflight.front();
    // a launch without an event had its stream synchronised when issued
    hipError_t e = hipSuccess;
    if (L.done) e = block ? hipEventSynchronize(L.done) : hipEventQuery(L.done);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess && L.status == PMLSH_OK) L.status = PMLSH_EDEVICE;
    if (L.done) (void)hipEventDestroy(L.done);
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
    s->inflight.pop_front();
    s->cv_done.notify_all();
    return true;
}

// Takes the next launch's segments from the waiting requests (under mu):
// the oldest request's parameters, then every later request with the same
// ones, in arrival order, up to max_batch queries.
std::vector<Segment> take_batch(pmlsh_server* s) {
    std::vector<Segment> segs;
    if (s->waiting.empty()) return segs;
    const Request head = *s->waiting.front();
    int64_t room = s->max_batch;
    for (auto it = s->waiting.begin(); it != s->waiting.end() && room > 0;) {
        Request& r = **it;
        if (!r.same_class(head)) {
            ++it;
            continue;
        }
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

int64_t launch_bytes(const pmlsh_server* s, const Request& r, int64_t nb) {
    const int64_t staging = nb * ((int64_t)s->idx->d * 4 + (int64_t)r.k * 12);
    return staging + ann_workspace_bytes(s->idx, nb, r.k, r.c, r.confidence, r.beta);
}

// Issues one launch on the server's stream. Errors fail the launch's
// requests; the event still marks the point after which its buffers are free.
void issue(pmlsh_server* s, Launch& L) {
    const Request& p = *L.segs.front().req;
    const int d = s->idx->d;
    const int k = p.k;
    int64_t nb = 0;
    for (auto& sg : L.segs) nb += sg.count;
    hipStream_t st = s->stream;
    L.status = guarded([&] {
        // staging buffers, released in stream order after the scatter copies
        struct Staging {
            void* p = nullptr;
            hipStream_t st;
            explicit Staging(hipStream_t s_) : st(s_) {}
            ~Staging() { ws_free(p, st); }
        } bq(st), bid(st), bdist(st);
        bq.p = ws_alloc((size_t)nb * d * 4, st);
        bid.p = ws_alloc((size_t)nb * k * 8, st);
        bdist.p = ws_alloc((size_t)nb * k * 4, st);
        float* sq = static_cast<float*>(bq.p);
        int64_t* sid = static_cast<int64_t*>(bid.p);
        float* sdist = static_cast<float*>(bdist.p);
        int64_t off = 0;
        for (auto& sg : L.segs) {
            Request& r = *sg.req;
            if (r.ready && !r.ready_waited) {
                PMLSH_HIP(hipStreamWaitEvent(st, r.ready, 0));
                r.ready_waited = true;
            }
            PMLSH_HIP(hipMemcpyAsync(sq + off * d, r.q + sg.req_off * d, (size_t)sg.count * d * 4,
                                     hipMemcpyDeviceToDevice, st));
            off += sg.count;
        }
        run_ann(s->idx, sq, nb, k, p.c, p.confidence, p.beta, p.r_min, sid, sdist, nullptr, st);
        off = 0;
        for (auto& sg : L.segs) {
            Request& r = *sg.req;
            PMLSH_HIP(hipMemcpyAsync(r.out_ids + sg.req_off * k, sid + off * k,
                                     (size_t)sg.count * k * 8, hipMemcpyDeviceToDevice, st));
            PMLSH_HIP(hipMemcpyAsync(r.out_dist + sg.req_off * k, sdist + off * k,
                                     (size_t)sg.count * k * 4, hipMemcpyDeviceToDevice, st));
            off += sg.count;
        }
    });
    if (hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
        L.done = nullptr;
        (void)hipStreamSynchronize(st);
        if (L.status == PMLSH_OK) L.status = PMLSH_EDEVICE;
        return;
    }
    if (hipEventRecord(L.done, st) != hipSuccess) {
        (void)hipEventDestroy(L.done);
        L.done = nullptr;
        (void)hipStreamSynchronize(st);
        if (L.status == PMLSH_OK) L.status = PMLSH_EDEVICE;
    }
}

void worker_loop(pmlsh_server* s) {
    (void)hipSetDevice(s->idx->device);
    for (;;) {
        // retire what has completed
        while (retire_one(s, false)) {
        }
        // admit launches while a slot and the budget allow
        bool issued = false;
        while ((int)s->inflight.size() < s->max_inflight) {
            std::vector<Segment> segs;
            {
                std::lock_guard<std::mutex> g(s->mu);
                segs = take_batch(s);
                if (segs.empty()) break;
                int64_t nb = 0;
                for (auto& sg : segs) nb += sg.count;
                const int64_t bytes = launch_bytes(s, *segs.front().req, nb);
                if (!s->inflight.empty() && s->bytes_inflight + bytes > s->hbm_budget) {
                    untake(s, segs);
                    break;
                }
                s->inflight.emplace_back();
                s->inflight.back().segs = std::move(segs);
                s->inflight.back().bytes = bytes;
                s->bytes_inflight += bytes;
            }
            issue(s, s->inflight.back());
            issued = true;
        }
        if (!s->inflight.empty()) {
            if (!issued) std::this_thread::sleep_for(std::chrono::microseconds(20));
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
        try {
            s->worker = std::thread(worker_loop, s.get());
        } catch (const std::exception&) {
            (void)hipStreamDestroy(s->stream);
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
        // parameter checks of the planner, before anything is queued
        pmlsh_plan plan;
        plan_params(server->idx->n, server->idx->m, k, c, confidence, beta, &plan);
        auto r = std::make_shared<Request>();
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
        (void)hipStreamDestroy(server->stream);
    }
    delete server;
}

}  // extern "C"
