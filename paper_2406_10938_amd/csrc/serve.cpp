// Serving loop: many query requests (each an Alg. 7 query batch) on one index,
// with continuous batching over a workspace allocated once.
//
// Worker threads ("slots") each own a default-priority HIP stream and an equal
// share of the workspace.  A free slot takes the oldest request that still has
// queries to start and fills its batch with the waiting queries of later
// requests that share (k, c, beta, options), up to what its workspace holds.
// Queries of a merged batch are staged into the slot's workspace, answered by
// one pass of the query kernels and copied back to their owners.  Each query's
// arithmetic is independent of the others in its batch, so a request's results
// do not depend on what it was batched with.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.h"
#include "detlsh.h"

namespace {

double now_s() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

detlsh_status errf(detlsh_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
detlsh_status errf(detlsh_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return dl_error(s, buf);
}

// Query parameters; requests merge into one batch only when these are equal.
// Under the MAGIC start radius the query stops in its first round and c never
// enters the computation, so c is compared only for the FIXED ladder.
struct Params {
    int32_t k = 0;
    double c = 0, beta = 0;
    detlsh_query_opts o{};
    bool same(const Params& p) const {
        const bool c_ok = o.rmin_policy == DETLSH_RMIN_MAGIC || c == p.c;
        return k == p.k && c_ok && beta == p.beta && o.precision == p.o.precision &&
               o.rerank_mult == p.o.rerank_mult && o.rmin_policy == p.o.rmin_policy &&
               o.max_rounds == p.o.max_rounds && o.r_min == p.o.r_min && o.verify == p.o.verify &&
               o.granularity == p.o.granularity && o.filter == p.o.filter;
    }
};

struct Request {
    uint64_t ticket = 0;
    const float* Q = nullptr;
    int64_t nq = 0;
    int64_t* out_ids = nullptr;
    float* out_d = nullptr;
    Params P;
    int64_t cap_solo = 0;     // queries per pass on a slot, unstaged
    int64_t cap_merged = 0;   // queries per pass on a slot, staged with others
    int64_t next = 0;         // first query not yet handed to a batch
    int64_t done = 0;         // queries whose batch has ended
    int running = 0;          // batches in flight holding its queries
    bool cancelled = false;
    bool finished = false;
    detlsh_status status = DETLSH_OK;
    std::string msg;
    detlsh_request_info info{};
};

struct Seg {
    Request* r;
    int64_t off, cnt;
};

}  // namespace

struct detlsh_server_s {
    detlsh_index ix = nullptr;
    int device = 0;
    int32_t d = 0;
    size_t slot_bytes = 0;
    int64_t max_batch = 1024;
    void* ws = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> threads;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;   // requests with queries not yet handed out, oldest first
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    bool stopping = false;

    size_t staging_bytes(int64_t nq, int32_t k) const {
        return align256((size_t)nq * d * 4) + align256((size_t)nq * k * 8) + align256((size_t)nq * k * 4);
    }

    // Largest number of queries in [1, max_batch] whose pass fits one slot
    // (0 if not even one does).
    int64_t capacity(const Params& P, bool staged) const {
        auto fits = [&](int64_t nq) {
            size_t need = 0;
            if (dl_query_check(ix, nq, P.k, P.c, P.beta, &P.o, &need) != DETLSH_OK) return false;
            if (staged) need += staging_bytes(nq, P.k);
            return need <= slot_bytes;
        };
        if (!fits(1)) return 0;
        int64_t lo = 1, hi = max_batch;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo + 1) / 2;
            if (fits(mid)) lo = mid; else hi = mid - 1;
        }
        return lo;
    }

    // Called with mu held.
    void maybe_finish(Request* r) {
        if (r->finished || r->running > 0) return;
        if (r->done < r->nq && !r->cancelled) return;
        r->finished = true;
        r->info.t_end = now_s();
        if (r->cancelled && r->status == DETLSH_OK) {
            r->status = DETLSH_ECANCELED;
            r->msg = "request cancelled";
        }
    }

    // Runs one batch on a slot (mu not held).  On failure *msg says why.
    detlsh_status run_batch(const std::vector<Seg>& segs, char* base, hipStream_t st, std::string* msg) {
        const Params& P = segs[0].r->P;
        const int32_t k = P.k;
        detlsh_status s = DETLSH_OK;
        if (segs.size() == 1) {
            const Seg& g = segs[0];
            s = dl_query_in_arena(ix, g.r->Q + g.off * d, g.cnt, k, P.c, P.beta, &P.o, g.r->out_ids + g.off * k,
                                  g.r->out_d + g.off * k, base, slot_bytes, st);
            if (s) *msg = detlsh_last_error();
            return s;
        }
        int64_t total = 0;
        for (const Seg& g : segs) total += g.cnt;
        char* p = base;
        float* Qs = reinterpret_cast<float*>(p);
        p += align256((size_t)total * d * 4);
        int64_t* ids = reinterpret_cast<int64_t*>(p);
        p += align256((size_t)total * k * 8);
        float* ds = reinterpret_cast<float*>(p);
        p += align256((size_t)total * k * 4);
        const size_t used = (size_t)(p - base);
        auto hip_fail = [&](hipError_t e, const char* what) {
            *msg = std::string(what) + ": " + hipGetErrorString(e);
            return DETLSH_EDEVICE;
        };
        int64_t row = 0;
        for (const Seg& g : segs) {
            hipError_t e = hipMemcpyAsync(Qs + row * d, g.r->Q + g.off * d, (size_t)g.cnt * d * 4,
                                          hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "staging queries");
            row += g.cnt;
        }
        s = dl_query_in_arena(ix, Qs, total, k, P.c, P.beta, &P.o, ids, ds, p, slot_bytes - used, st);
        if (s) {
            *msg = detlsh_last_error();
            return s;
        }
        row = 0;
        for (const Seg& g : segs) {
            hipError_t e = hipMemcpyAsync(g.r->out_ids + g.off * k, ids + row * k, (size_t)g.cnt * k * 8,
                                          hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(g.r->out_d + g.off * k, ds + row * k, (size_t)g.cnt * k * 4,
                                   hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "returning results");
            row += g.cnt;
        }
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        return DETLSH_OK;
    }

    // Called with mu held and the queue not empty: hands out the next batch.
    std::vector<Seg> form_batch() {
        std::vector<Seg> segs;
        Request* h = queue.front();
        const int64_t rem = h->nq - h->next;
        if (rem >= h->cap_merged) {
            const int64_t cnt = std::min(rem, h->cap_solo);
            segs.push_back({h, h->next, cnt});
            h->next += cnt;
        } else {
            int64_t room = h->cap_merged;
            for (Request* r : queue) {
                if (room == 0) break;
                if (!r->P.same(h->P)) continue;
                const int64_t cnt = std::min(r->nq - r->next, room);
                segs.push_back({r, r->next, cnt});
                r->next += cnt;
                room -= cnt;
            }
        }
        queue.erase(std::remove_if(queue.begin(), queue.end(), [](Request* r) { return r->next >= r->nq; }),
                    queue.end());
        return segs;
    }

    void worker(int slot) {
        const hipError_t dev_err = hipSetDevice(device);
        char* base = static_cast<char*>(ws) + (size_t)slot * slot_bytes;
        hipStream_t st = streams[slot];
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
            if (stopping) break;
            std::vector<Seg> segs = form_batch();
            int64_t total = 0;
            for (const Seg& g : segs) total += g.cnt;
            const double t0 = now_s();
            for (const Seg& g : segs) {
                Request* r = g.r;
                r->running += 1;
                if (r->info.batches == 0) r->info.t_start = t0;
                r->info.batches += 1;
                r->info.max_batch_requests = std::max<int32_t>(r->info.max_batch_requests, (int32_t)segs.size());
                r->info.max_batch_queries = std::max(r->info.max_batch_queries, total);
            }
            lk.unlock();
            std::string msg;
            detlsh_status s = DETLSH_OK;
            if (dev_err != hipSuccess) {
                s = DETLSH_EDEVICE;
                msg = std::string("hipSetDevice: ") + hipGetErrorString(dev_err);
            } else {
                s = run_batch(segs, base, st, &msg);
            }
            lk.lock();
            for (const Seg& g : segs) {
                Request* r = g.r;
                r->running -= 1;
                r->done += g.cnt;
                if (s != DETLSH_OK && r->status == DETLSH_OK) {
                    r->status = s;
                    r->msg = msg;
                }
                maybe_finish(r);
            }
            cv_done.notify_all();
        }
    }
};

extern "C" {

detlsh_status detlsh_server_create(detlsh_index idx, size_t workspace_bytes, int32_t slots, int32_t max_batch,
                                   detlsh_server* out) {
    if (!out) return errf(DETLSH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!idx) return errf(DETLSH_EINVAL, "NULL index");
    if (slots == 0) slots = 2;
    if (max_batch == 0) max_batch = 1024;
    if (slots < 1 || slots > 16) return errf(DETLSH_EINVAL, "slots must be in [1, 16], got %d", slots);
    if (max_batch < 1 || max_batch > 65535)
        return errf(DETLSH_EINVAL, "max_batch must be in [1, 65535], got %d", max_batch);
    if (workspace_bytes < ((size_t)1 << 20))
        return errf(DETLSH_EINVAL, "workspace_bytes must be >= 1 MiB, got %zu", workspace_bytes);
    std::unique_ptr<detlsh_server_s> srv;
    try {
        srv.reset(new detlsh_server_s);
    } catch (const std::bad_alloc&) {
        return errf(DETLSH_ENOMEM, "server state");
    }
    srv->ix = idx;
    srv->device = dl_index_device(idx);
    srv->d = dl_index_dim(idx);
    srv->max_batch = max_batch;
    srv->slot_bytes = (workspace_bytes / (size_t)slots) & ~(size_t)255;
    hipError_t e = hipSetDevice(srv->device);
    if (e != hipSuccess) return errf(DETLSH_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    e = hipMalloc(&srv->ws, srv->slot_bytes * (size_t)slots);
    if (e != hipSuccess) {
        srv->ws = nullptr;
        return errf(DETLSH_ENOMEM, "server workspace of %zu bytes: %s", srv->slot_bytes * (size_t)slots,
                    hipGetErrorString(e));
    }
    auto cleanup = [&]() {
        for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
        (void)hipFree(srv->ws);
    };
    for (int i = 0; i < slots; ++i) {
        hipStream_t s = nullptr;
        e = hipStreamCreate(&s);   // default priority
        if (e != hipSuccess) {
            cleanup();
            return errf(DETLSH_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        srv->streams.push_back(s);
    }
    try {
        for (int i = 0; i < slots; ++i) srv->threads.emplace_back([p = srv.get(), i] { p->worker(i); });
    } catch (...) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stopping = true;
        }
        srv->cv_work.notify_all();
        for (auto& t : srv->threads) t.join();
        cleanup();
        return errf(DETLSH_EINTERNAL, "could not start the worker threads");
    }
    *out = srv.release();
    return DETLSH_OK;
}

detlsh_status detlsh_server_submit(detlsh_server srv, const float* Q, int64_t nq, int32_t k, double c, double beta,
                                   const detlsh_query_opts* opts, int64_t* out_ids, float* out_dists,
                                   uint64_t* ticket) {
    if (!srv) return errf(DETLSH_EINVAL, "NULL server");
    if (!ticket) return errf(DETLSH_EINVAL, "ticket is NULL");
    *ticket = 0;
    Params P;
    P.k = k;
    P.c = c;
    P.beta = beta;
    if (opts) P.o = *opts;
    P.o.workspace_bytes = 0;
    if (detlsh_status s = dl_query_check(srv->ix, nq, k, c, beta, &P.o, nullptr)) return s;
    if (nq > 0) {
        if (!dl_is_device_ptr(Q)) return errf(DETLSH_EINVAL, "Q must be a device pointer");
        if (!dl_is_device_ptr(out_ids) || !dl_is_device_ptr(out_dists))
            return errf(DETLSH_EINVAL, "outputs must be device pointers");
    }
    std::unique_ptr<Request> r;
    try {
        r.reset(new Request);
    } catch (const std::bad_alloc&) {
        return errf(DETLSH_ENOMEM, "request state");
    }
    r->Q = Q;
    r->nq = nq;
    r->out_ids = out_ids;
    r->out_d = out_dists;
    r->P = P;
    if (nq > 0) {
        r->cap_solo = srv->capacity(P, false);
        if (r->cap_solo == 0) {
            size_t need = 0;
            (void)dl_query_check(srv->ix, 1, k, c, beta, &P.o, &need);
            return errf(DETLSH_ENOMEM, "one query needs %zu bytes of workspace; a slot has %zu", need,
                        srv->slot_bytes);
        }
        r->cap_merged = std::max<int64_t>(srv->capacity(P, true), 1);
    }
    r->info.t_submit = now_s();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return errf(DETLSH_EINVAL, "server is stopping");
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    Request* raw = r.get();
    try {
        srv->reqs.emplace(raw->ticket, std::move(r));
        if (nq == 0) {
            raw->info.t_start = raw->info.t_submit;
            srv->maybe_finish(raw);
        } else {
            srv->queue.push_back(raw);
        }
    } catch (const std::bad_alloc&) {
        srv->reqs.erase(raw->ticket);
        *ticket = 0;
        return errf(DETLSH_ENOMEM, "request queue");
    }
    srv->cv_work.notify_one();
    return DETLSH_OK;
}

detlsh_status detlsh_server_wait(detlsh_server srv, uint64_t ticket, int64_t timeout_us, detlsh_request_info* info) {
    if (!srv) return errf(DETLSH_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto done = [&] {
        auto it = srv->reqs.find(ticket);
        return it == srv->reqs.end() || it->second->finished;
    };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, done);
    } else if (timeout_us > 0) {
        srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
    }
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return errf(DETLSH_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->finished) return errf(DETLSH_EBUSY, "request %llu is still running", (unsigned long long)ticket);
    std::unique_ptr<Request> r = std::move(it->second);
    srv->reqs.erase(it);
    lk.unlock();
    if (info) *info = r->info;
    if (r->status != DETLSH_OK) return dl_error(r->status, r->msg.c_str());
    return dl_error(DETLSH_OK, "");
}

detlsh_status detlsh_server_cancel(detlsh_server srv, uint64_t ticket) {
    if (!srv) return errf(DETLSH_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return errf(DETLSH_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request* r = it->second.get();
    if (r->finished) return errf(DETLSH_EBUSY, "request %llu has already finished", (unsigned long long)ticket);
    r->cancelled = true;
    r->next = r->nq;
    srv->queue.erase(std::remove(srv->queue.begin(), srv->queue.end(), r), srv->queue.end());
    srv->maybe_finish(r);
    srv->cv_done.notify_all();
    return dl_error(DETLSH_OK, "");
}

void detlsh_server_destroy(detlsh_server srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        for (Request* r : srv->queue) {
            r->cancelled = true;
            r->next = r->nq;
            srv->maybe_finish(r);
        }
        srv->queue.clear();
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    for (auto& t : srv->threads) t.join();
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    if (srv->ws) (void)hipFree(srv->ws);
    delete srv;
}

}  // extern "C"
