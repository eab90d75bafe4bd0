// Request server: continuous batching of steady-state solves.
//
// A worker thread per server runs the loop: admit submitted requests (in
// submission order, later ones passing one that does not fit for a bounded
// number of intervals) while their buffers fit the device pool, advance the
// batch by one interval, hand the results of requests that left to the host,
// return their memory, repeat; it sleeps while nothing is submitted.
// Requests are submitted and results polled from any thread (prc_server_*);
// prc_serve replays a trace of arrivals through such a server.
// The pool is one hipMalloc'd region managed by a first-fit allocator with
// coalescing free lists, so requests come and go without hipMalloc/hipFree
// (hipFree synchronises the device).  The ABI is declared in include/prc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "prc.h"
#include "prc_batch.hpp"
#include "prc_host.hpp"

namespace prc {

// First-fit allocator over [0, size) in 256-byte units.
class Pool {
  public:
    static constexpr size_t kAlign = 256;

    explicit Pool(size_t size) { free_[0] = size / kAlign * kAlign; }

    // offset of a block of `bytes`, or SIZE_MAX if none is free
    size_t alloc(size_t bytes)
    {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return off;
        }
        return SIZE_MAX;
    }

    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {  // merge with the next block
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {  // merge with the previous block
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

  private:
    std::map<size_t, size_t> free_;  // offset -> size of each free block
};

// Requests passed over by later ones that fit are admitted before anything
// else once they have waited this many intervals.
constexpr int kMaxBypassIntervals = 8;

}  // namespace prc

// The online server: a device pool, a batch and a worker thread.
struct prc_server {
    prc_serve_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    char *base = nullptr;  // the pool: cfg.hbm_budget device bytes
    std::chrono::steady_clock::time_point t0;

    struct Pending {
        int64_t ticket;
        prc_params p;
        double *ux, *uy;
        double submit_s;
    };
    std::mutex mu;
    std::condition_variable work;  // the worker waits here for requests or stop
    std::condition_variable done;  // pollers wait here for results
    std::deque<Pending> queue;     // submitted, not yet seen by the worker
    std::deque<prc_server_result> results;  // finished, not yet polled
    int64_t next_ticket = 0;
    int32_t n_waiting = 0, n_active = 0;  // as the worker last saw them
    bool stop = false;
    prc_status fatal = PRC_OK;     // a failure of the worker ends the server
    std::string fatal_msg;
    std::thread worker;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace prc {

namespace {

struct Slot {
    prc_server::Pending req;
    double admit_s = 0.0;
    size_t off_a = 0, off_b = 0, off_u = 0, state = 0, snap = 0;
};

void publish(prc_server &srv, const prc_server_result &r)
{
    std::lock_guard<std::mutex> lock(srv.mu);
    srv.results.push_back(r);
    srv.done.notify_all();
}

// The serving loop of one server, on its own thread: admit, advance one
// interval, hand finished requests to the host, repeat; sleep while idle.
prc_status serve_loop(prc_server &srv)
{
    HIP_TRY(hipSetDevice(srv.device));
    const prc_serve_config &cfg = srv.cfg;
    const hipStream_t s = srv.stream;
    char *const base = srv.base;
    Pool pool(cfg.hbm_budget);
    const size_t capacity = cfg.hbm_budget / Pool::kAlign * Pool::kAlign;
    prc_batch *b = nullptr;
    prc_status st = prc_batch_create(cfg.storage, cfg.bc, &b);
    if (st != PRC_OK) return st;
    struct BatchGuard {
        prc_batch *b;
        ~BatchGuard() { prc_batch_destroy(b); }
    } guard{b};
    if (cfg.tile >= 0 && (st = prc_batch_set_tile(b, cfg.tile)) != PRC_OK) return st;
    std::vector<Slot> slots;  // by batch member id
    std::deque<prc_server::Pending> waiting;
    std::vector<BatchLeft> left;
    int32_t active = 0;
    int64_t head = -1;   // ticket at the head of the waiting list
    int head_waits = 0;  // intervals it has waited while others were admitted

    for (;;) {
        {
            std::unique_lock<std::mutex> lock(srv.mu);
            if (active == 0 && waiting.empty() && srv.queue.empty() && !srv.stop) {
                srv.n_waiting = 0;
                srv.n_active = 0;
                srv.work.wait(lock, [&] { return srv.stop || !srv.queue.empty(); });
            }
            if (srv.stop) return PRC_OK;
            while (!srv.queue.empty()) {
                waiting.push_back(srv.queue.front());
                srv.queue.pop_front();
            }
        }
        // admission in submission order; a request that does not fit yet is
        // passed by later ones that do, for at most kMaxBypassIntervals
        if (!waiting.empty() && waiting.front().ticket != head) {
            head = waiting.front().ticket;
            head_waits = 0;
        }
        bool head_blocked = false;
        for (auto it = waiting.begin(); it != waiting.end();) {
            if (cfg.max_active > 0 && active >= cfg.max_active) break;
            const prc_params &p = it->p;
            Slot sl;
            sl.req = *it;
            const bool valid = validate(&p) == PRC_OK && p.storage == cfg.storage && p.bc == cfg.bc;
            if (valid) {
                sl.state = prc_state_bytes(&p);
                sl.snap = 2 * sizeof(double) * (size_t)p.nx * (size_t)p.ny;
            }
            const size_t need = 2 * ((sl.state + 255) / 256 * 256) + (sl.snap + 255) / 256 * 256;
            if (!valid || need > capacity) {  // can never run
                const double t = srv.now();
                publish(srv, prc_server_result{it->ticket, PRC_EINVAL, 0, 0, NAN, it->submit_s, t, t});
                it = waiting.erase(it);
                continue;
            }
            sl.off_a = pool.alloc(sl.state);
            sl.off_b = sl.off_a == SIZE_MAX ? SIZE_MAX : pool.alloc(sl.state);
            sl.off_u = sl.off_b == SIZE_MAX ? SIZE_MAX : pool.alloc(sl.snap);
            if (sl.off_u == SIZE_MAX) {  // no room yet
                if (sl.off_b != SIZE_MAX) pool.release(sl.off_b, sl.state);
                if (sl.off_a != SIZE_MAX) pool.release(sl.off_a, sl.state);
                if (it == waiting.begin()) {
                    head_blocked = true;
                    if (head_waits >= kMaxBypassIntervals) break;  // nothing passes it now
                }
                ++it;
                continue;
            }
            if ((st = prc_init(&p, base + sl.off_a, s)) != PRC_OK) return st;
            int32_t id = -1;
            if ((st = prc_batch_add(b, &p, base + sl.off_a, base + sl.off_b,
                                    (double *)(base + sl.off_u), &id)) != PRC_OK)
                return st;
            if ((size_t)id >= slots.size()) slots.resize(id + 1);
            sl.admit_s = srv.now();
            slots[id] = sl;
            it = waiting.erase(it);
            ++active;
        }
        if (head_blocked) ++head_waits;
        {
            std::lock_guard<std::mutex> lock(srv.mu);
            srv.n_waiting = (int32_t)waiting.size();
            srv.n_active = active;
        }
        if (active == 0) {
            if (!waiting.empty()) {  // nothing running and nothing fits: cannot happen
                return fail(PRC_EHIP, "server: a request that fits the empty pool was not admitted");
            }
            continue;
        }
        left.clear();
        if ((st = batch_interval(b, cfg.tol, cfg.check_every, cfg.max_steps, nullptr, &left, s)) !=
            PRC_OK)
            return st;
        if (left.empty()) continue;
        // results to the host: the snapshot of the last check is the velocity
        // of the final state (u_x plane, then u_y plane)
        hipError_t e = hipSuccess;
        for (const BatchLeft &l : left) {
            const Slot &sl = slots[l.id];
            const size_t plane = sl.snap / 2;
            if (sl.req.ux && e == hipSuccess)
                e = hipMemcpyAsync(sl.req.ux, base + sl.off_u, plane, hipMemcpyDeviceToHost, s);
            if (sl.req.uy && e == hipSuccess)
                e = hipMemcpyAsync(sl.req.uy, base + sl.off_u + plane, plane, hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail(PRC_EHIP, "server result copy: %s", hipGetErrorString(e));
        const double td = srv.now();
        std::vector<prc_server_result> fin;
        for (const BatchLeft &l : left) {
            const Slot &sl = slots[l.id];
            fin.push_back(prc_server_result{sl.req.ticket, l.status, 0, l.steps, l.R,
                                            sl.req.submit_s, sl.admit_s, td});
            pool.release(sl.off_a, sl.state);
            pool.release(sl.off_b, sl.state);
            pool.release(sl.off_u, sl.snap);
            --active;
        }
        {
            std::lock_guard<std::mutex> lock(srv.mu);
            srv.n_active = active;
            srv.results.insert(srv.results.end(), fin.begin(), fin.end());
            srv.done.notify_all();
        }
    }
}

void worker_main(prc_server *srv)
{
    const prc_status st = serve_loop(*srv);
    std::lock_guard<std::mutex> lock(srv->mu);
    if (st != PRC_OK) {
        srv->fatal = st;
        srv->fatal_msg = prc_last_error();
    }
    srv->stop = true;
    srv->done.notify_all();
}

prc_status check_config(const prc_serve_config *cfg)
{
    if (!cfg) return fail(PRC_EINVAL, "NULL config");
    if (cfg->storage < PRC_F64 || cfg->storage > PRC_BF16 || cfg->bc < PRC_BC_CAVITY ||
        cfg->bc > PRC_BC_CHANNEL)
        return fail(PRC_EINVAL, "unknown storage or bc");
    if (cfg->check_every <= 0 || (cfg->check_every & 1))
        return fail(PRC_EINVAL, "check_every must be even and > 0");
    if (cfg->max_steps < 0 || cfg->max_steps % cfg->check_every)
        return fail(PRC_EINVAL, "max_steps must be a non-negative multiple of check_every");
    if (!(cfg->tol >= 0.0)) return fail(PRC_EINVAL, "tol must be >= 0");
    if (cfg->tile < -1 || cfg->tile >= kNumBatchTiles) return fail(PRC_EINVAL, "tile out of range");
    if (cfg->hbm_budget < 4096) return fail(PRC_EINVAL, "hbm_budget too small");
    if (cfg->max_active < 0) return fail(PRC_EINVAL, "max_active < 0");
    return PRC_OK;
}

}  // namespace

}  // namespace prc

using namespace prc;

extern "C" {

prc_status prc_server_create(const prc_serve_config *cfg, hipStream_t stream, prc_server **out)
{
    prc_status st = check_config(cfg);
    if (st != PRC_OK) return st;
    if (!out) return fail(PRC_EINVAL, "NULL out");
    *out = nullptr;
    auto *srv = new prc_server;
    srv->cfg = *cfg;
    srv->stream = stream;
    hipError_t e = hipGetDevice(&srv->device);
    if (e == hipSuccess) e = hipMalloc((void **)&srv->base, cfg->hbm_budget);
    if (e != hipSuccess) {
        delete srv;
        return fail(PRC_EHIP, "server pool of %zu bytes: %s", cfg->hbm_budget, hipGetErrorString(e));
    }
    srv->t0 = std::chrono::steady_clock::now();
    try {
        srv->worker = std::thread(worker_main, srv);
    } catch (...) {
        (void)hipFree(srv->base);
        delete srv;
        return fail(PRC_EHIP, "server: cannot start its worker thread");
    }
    *out = srv;
    return PRC_OK;
}

prc_status prc_server_submit(prc_server *srv, const prc_params *p, double *ux, double *uy,
                             int64_t *ticket)
{
    if (!srv || !p) return fail(PRC_EINVAL, "NULL server or params");
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->fatal != PRC_OK) return fail(srv->fatal, "server failed: %s", srv->fatal_msg.c_str());
    if (srv->stop) return fail(PRC_EINVAL, "server is stopping");
    const int64_t t = srv->next_ticket++;
    srv->queue.push_back(prc_server::Pending{t, *p, ux, uy, srv->now()});
    srv->work.notify_one();
    if (ticket) *ticket = t;
    return PRC_OK;
}

prc_status prc_server_poll(prc_server *srv, double wait_s, prc_server_result *out, int32_t cap,
                           int32_t *n)
{
    if (!srv || !n || cap < 0 || (!out && cap > 0)) return fail(PRC_EINVAL, "bad poll arguments");
    *n = 0;
    std::unique_lock<std::mutex> lock(srv->mu);
    if (srv->results.empty() && wait_s > 0.0 && srv->fatal == PRC_OK && !srv->stop)
        srv->done.wait_for(lock, std::chrono::duration<double>(wait_s),
                           [&] { return !srv->results.empty() || srv->stop; });
    while (*n < cap && !srv->results.empty()) {
        out[(*n)++] = srv->results.front();
        srv->results.pop_front();
    }
    if (*n == 0 && srv->fatal != PRC_OK)
        return fail(srv->fatal, "server failed: %s", srv->fatal_msg.c_str());
    return PRC_OK;
}

prc_status prc_server_status(prc_server *srv, int32_t *waiting, int32_t *active, int32_t *unpolled)
{
    if (!srv) return fail(PRC_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(srv->mu);
    if (waiting) *waiting = srv->n_waiting + (int32_t)srv->queue.size();
    if (active) *active = srv->n_active;
    if (unpolled) *unpolled = (int32_t)srv->results.size();
    if (srv->fatal != PRC_OK) return fail(srv->fatal, "server failed: %s", srv->fatal_msg.c_str());
    return PRC_OK;
}

prc_status prc_server_destroy(prc_server *srv)
{
    if (!srv) return PRC_OK;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
        srv->work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    const hipError_t e = hipStreamSynchronize(srv->stream);
    (void)hipFree(srv->base);
    delete srv;
    if (e != hipSuccess) return fail(PRC_EHIP, "server stream: %s", hipGetErrorString(e));
    return PRC_OK;
}

prc_status prc_serve(const prc_serve_config *cfg, const prc_request *reqs, int32_t n,
                     prc_result *res, hipStream_t stream)
{
    prc_status st = check_config(cfg);
    if (st != PRC_OK) return st;
    if ((!reqs && n > 0) || (!res && n > 0) || n < 0)
        return fail(PRC_EINVAL, "need reqs, res and n >= 0");
    for (int32_t i = 1; i < n; ++i)
        if (!(reqs[i].arrival_s >= reqs[i - 1].arrival_s))
            return fail(PRC_EINVAL, "arrivals must be non-decreasing (request %d)", i);
    if (n == 0) return PRC_OK;
    prc_server *srv = nullptr;
    if ((st = prc_server_create(cfg, stream, &srv)) != PRC_OK) return st;
    // submit each request at its arrival time (from the server's start), and
    // collect results meanwhile
    std::vector<int32_t> index_of(n);
    std::vector<prc_server_result> got(n);
    int32_t submitted = 0, finished = 0;
    while (finished < n && st == PRC_OK) {
        const double t = srv->now();
        while (submitted < n && reqs[submitted].arrival_s <= t) {
            int64_t ticket = -1;
            const prc_request &r = reqs[submitted];
            if ((st = prc_server_submit(srv, &r.p, r.ux, r.uy, &ticket)) != PRC_OK) break;
            index_of[ticket] = submitted++;
        }
        if (st != PRC_OK) break;
        const double wait = submitted < n ? std::max(0.0, reqs[submitted].arrival_s - srv->now()) : 1.0;
        int32_t m = 0;
        if ((st = prc_server_poll(srv, wait, got.data(), n, &m)) != PRC_OK) break;
        for (int32_t k = 0; k < m; ++k) {
            const prc_server_result &g = got[k];
            res[index_of[g.ticket]] = prc_result{g.status, 0, g.steps, g.residual, g.admit_s, g.done_s};
            ++finished;
        }
    }
    const prc_status sd = prc_server_destroy(srv);
    return st != PRC_OK ? st : sd;
}

}  // extern "C"
