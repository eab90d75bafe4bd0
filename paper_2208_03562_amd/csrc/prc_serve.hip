// Request server: continuous batching of steady-state solves.
//
// One host thread runs the loop: admit arrived requests (FIFO) while their
// buffers fit the device pool, advance the batch by one interval, hand the
// results of requests that left to the host, return their memory, repeat.
// The pool is one hipMalloc'd region managed by a first-fit allocator with
// coalescing free lists, so requests come and go without hipMalloc/hipFree
// (hipFree synchronises the device).  The ABI is declared in include/prc.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <deque>
#include <iterator>
#include <map>
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

struct Slot {
    int32_t req = -1;
    size_t off_a = 0, off_b = 0, off_u = 0, state = 0, snap = 0;
};

static prc_status serve_loop(const prc_serve_config &cfg, const prc_request *reqs, int32_t n,
                             prc_result *res, hipStream_t s, char *base)
{
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    auto now = [&] { return std::chrono::duration<double>(clock::now() - t0).count(); };

    Pool pool(cfg.hbm_budget);
    const size_t capacity = cfg.hbm_budget / Pool::kAlign * Pool::kAlign;
    prc_batch *b = nullptr;
    prc_status st = prc_batch_create(cfg.storage, cfg.bc, &b);
    if (st != PRC_OK) return st;
    if (cfg.tile >= 0 && (st = prc_batch_set_tile(b, cfg.tile)) != PRC_OK) {
        prc_batch_destroy(b);
        return st;
    }
    std::vector<Slot> slots;  // by batch member id
    std::deque<int32_t> waiting;
    std::vector<BatchLeft> left;
    int32_t next = 0, done = 0, active = 0;

    while (done < n && st == PRC_OK) {
        const double t = now();
        while (next < n && reqs[next].arrival_s <= t) waiting.push_back(next++);
        // admission, in arrival order
        while (!waiting.empty() && (cfg.max_active <= 0 || active < cfg.max_active)) {
            const int32_t i = waiting.front();
            const prc_params &p = reqs[i].p;
            Slot sl;
            sl.req = i;
            const bool valid = validate(&p) == PRC_OK && p.storage == cfg.storage && p.bc == cfg.bc;
            if (valid) {
                sl.state = prc_state_bytes(&p);
                sl.snap = 2 * sizeof(double) * (size_t)p.nx * (size_t)p.ny;
            }
            const size_t need = 2 * ((sl.state + 255) / 256 * 256) + (sl.snap + 255) / 256 * 256;
            if (!valid || need > capacity) {  // can never run
                res[i] = prc_result{PRC_EINVAL, 0, 0, NAN, t, t};
                waiting.pop_front();
                ++done;
                continue;
            }
            sl.off_a = pool.alloc(sl.state);
            sl.off_b = sl.off_a == SIZE_MAX ? SIZE_MAX : pool.alloc(sl.state);
            sl.off_u = sl.off_b == SIZE_MAX ? SIZE_MAX : pool.alloc(sl.snap);
            if (sl.off_u == SIZE_MAX) {  // wait for memory (head of line)
                if (sl.off_b != SIZE_MAX) pool.release(sl.off_b, sl.state);
                if (sl.off_a != SIZE_MAX) pool.release(sl.off_a, sl.state);
                break;
            }
            if ((st = prc_init(&p, base + sl.off_a, s)) != PRC_OK) break;
            int32_t id = -1;
            if ((st = prc_batch_add(b, &p, base + sl.off_a, base + sl.off_b,
                                    (double *)(base + sl.off_u), &id)) != PRC_OK)
                break;
            if ((size_t)id >= slots.size()) slots.resize(id + 1);
            slots[id] = sl;
            res[i] = prc_result{PRC_MEMBER_ACTIVE, 0, 0, NAN, now(), NAN};
            waiting.pop_front();
            ++active;
        }
        if (st != PRC_OK) break;
        if (active == 0) {
            // idle: sleep until the next arrival
            if (next < n) {
                const double wait = reqs[next].arrival_s - now();
                if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
            }
            continue;
        }
        left.clear();
        if ((st = batch_interval(b, cfg.tol, cfg.check_every, cfg.max_steps, nullptr, &left, s)) !=
            PRC_OK)
            break;
        if (left.empty()) continue;
        // results to the host: the snapshot of the last check is the velocity
        // of the final state (u_x plane, then u_y plane)
        hipError_t e = hipSuccess;
        for (const BatchLeft &l : left) {
            const Slot &sl = slots[l.id];
            const prc_request &r = reqs[sl.req];
            const size_t plane = sl.snap / 2;
            if (r.ux && e == hipSuccess)
                e = hipMemcpyAsync(r.ux, base + sl.off_u, plane, hipMemcpyDeviceToHost, s);
            if (r.uy && e == hipSuccess)
                e = hipMemcpyAsync(r.uy, base + sl.off_u + plane, plane, hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = fail(PRC_EHIP, "prc_serve result copy: %s", hipGetErrorString(e));
            break;
        }
        const double td = now();
        for (const BatchLeft &l : left) {
            const Slot &sl = slots[l.id];
            prc_result &o = res[sl.req];
            o.status = l.status;
            o.steps = l.steps;
            o.residual = l.R;
            o.done_s = td;
            pool.release(sl.off_a, sl.state);
            pool.release(sl.off_b, sl.state);
            pool.release(sl.off_u, sl.snap);
            --active;
            ++done;
        }
    }
    prc_batch_destroy(b);
    return st;
}

}  // namespace prc

using namespace prc;

extern "C" prc_status prc_serve(const prc_serve_config *cfg, const prc_request *reqs, int32_t n,
                                prc_result *res, hipStream_t stream)
{
    if (!cfg || (!reqs && n > 0) || (!res && n > 0) || n < 0)
        return fail(PRC_EINVAL, "need cfg, reqs, res and n >= 0");
    if (cfg->storage < PRC_F64 || cfg->storage > PRC_BF16 || cfg->bc < PRC_BC_CAVITY ||
        cfg->bc > PRC_BC_CHANNEL)
        return fail(PRC_EINVAL, "unknown storage or bc");
    if (cfg->check_every <= 0 || (cfg->check_every & 1))
        return fail(PRC_EINVAL, "check_every must be even and > 0");
    if (cfg->max_steps < 0 || cfg->max_steps % cfg->check_every)
        return fail(PRC_EINVAL, "max_steps must be a non-negative multiple of check_every");
    if (!(cfg->tol >= 0.0)) return fail(PRC_EINVAL, "tol must be >= 0");
    if (cfg->tile < -1 || cfg->tile >= kNumBatchTiles ||
        (cfg->tile >= 0 && kTiles[cfg->tile].steps == 2 && cfg->storage == PRC_F64))
        return fail(PRC_EINVAL, "tile out of range");
    if (cfg->hbm_budget < 4096) return fail(PRC_EINVAL, "hbm_budget too small");
    for (int32_t i = 1; i < n; ++i)
        if (!(reqs[i].arrival_s >= reqs[i - 1].arrival_s))
            return fail(PRC_EINVAL, "arrivals must be non-decreasing (request %d)", i);
    if (n == 0) return PRC_OK;
    void *base = nullptr;
    HIP_TRY(hipMalloc(&base, cfg->hbm_budget));
    const prc_status st = serve_loop(*cfg, reqs, n, res, stream, (char *)base);
    const hipError_t e = hipStreamSynchronize(stream);
    (void)hipFree(base);
    if (st != PRC_OK) return st;
    if (e != hipSuccess) return fail(PRC_EHIP, "prc_serve: %s", hipGetErrorString(e));
    return PRC_OK;
}
