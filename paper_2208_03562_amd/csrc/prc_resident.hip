// Host side of the resident sweep (k_resident, prc_resident.hpp): which
// problems it can run, the per-device synchronisation block, the launches
// (serialised across streams), the report of an aborted wait, and the
// release of the per-device resources.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <atomic>
#include <mutex>
#include <utility>

#include "prc.h"
#include "prc_host.hpp"
#include "prc_launch.hpp"
#include "prc_resident.hpp"

namespace prc {

namespace {

constexpr int kMaxDevices = 64;
// steps per launch at most (a launch that long takes well under a second)
constexpr int64_t kResidentMaxSteps = 1 << 16;

struct ResidentDevice {
    ResidentSync *sync = nullptr;
    void *xch = nullptr;  // exchange blocks: two parities of every subdomain, tagged
    // pinned host word a timed-out wait sets (read without synchronising)
    volatile uint64_t *mailbox = nullptr;
    // completion of the latest resident launch on this device, and its stream:
    // a launch on another stream waits for it, so that two launches never
    // share the exchange buffer and the compute units at once
    hipEvent_t last = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
    int cus = 0;  // compute units
    int lds = 0;  // LDS a workgroup may use, bytes
};
std::mutex g_res_mu;
ResidentDevice g_res[kMaxDevices];
// whether any device has its resident buffers (reports need no device query
// in a process that never ran the resident sweep)
std::atomic<int> g_res_devices{0};
// how long a workgroup waits for a neighbour's value before it gives up, in
// ticks of the 100 MHz real-time clock (prc_set_resident_wait)
std::atomic<uint64_t> g_wait_ticks{kResidentWaitTicks};

prc_status current_device(ResidentDevice **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PRC_EHIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_res_mu);
    ResidentDevice &d = g_res[dev];
    if (d.cus == 0) {
        HIP_TRY(hipDeviceGetAttribute(&d.lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        HIP_TRY(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
    }
    *out = &d;
    return PRC_OK;
}

size_t resident_lds_bytes(int storage)
{
    const size_t ct = storage == PRC_F64 ? 8 : 4;
    const size_t row = storage == PRC_F32 ? kResidentRowP<float> : kResidentRowP<uint16_t>;
    return elem_bytes(storage) * (9 * (kResidentSY + 4) * row + 64) +
           ct * (kResidentSY + 2) * kResidentRowD + 16;
}

int resident_tiles(const prc_params &p)
{
    return ((p.nx + kResidentSX - 1) / kResidentSX) * ((p.ny + kResidentSY - 1) / kResidentSY);
}

template <typename ST, int BC>
prc_status launch_res(const prc_params &p, const void *src, void *dst, int nsteps,
                      const ResidentDevice &d, hipStream_t s, hipEvent_t start, hipEvent_t stop)
{
    if constexpr (sizeof(ST) > 4) {  // an FP64 subdomain does not fit the LDS
        return fail(PRC_EINVAL, "the resident sweep has no FP64 instance");
    } else {
    auto c = coef_of<ST>(p);
    c.tiles_x = (p.nx + kResidentSX - 1) / kResidentSX;
    c.tiles_y = (p.ny + kResidentSY - 1) / kResidentSY;
    c.tiles_per_xcd = (c.tiles_x * c.tiles_y + kXcds - 1) / kXcds;
    const dim3 grid(c.tiles_per_xcd * kXcds), block(kResidentThreads);
    const uint64_t wait = g_wait_ticks.load(std::memory_order_relaxed);
    auto kern = is_plain_method(p) ? k_resident<ST, BC, false, true> : k_resident<ST, BC, true, false>;
    if (start || stop)  // events taken by the dispatch itself: the kernel's own start and end
        hipExtLaunchKernelGGL(kern, grid, block, 0, s, start, stop, 0, (ST *)src, (ST *)dst, d.xch,
                              c, d.sync, (uint64_t *)d.mailbox, wait, nsteps);
    else
        hipLaunchKernelGGL(kern, grid, block, 0, s, (ST *)src, (ST *)dst, d.xch, c, d.sync,
                           (uint64_t *)d.mailbox, wait, nsteps);
    HIP_TRY(hipGetLastError());
    return PRC_OK;
    }
}

}  // namespace

bool resident_allowed(const prc_params &p)
{
    ResidentDevice *d = nullptr;
    if (current_device(&d) != PRC_OK) return false;
    if (p.storage == PRC_F64 || (size_t)d->lds < resident_lds_bytes(p.storage)) return false;
    const int tiles = resident_tiles(p);
    if (tiles > d->cus || tiles > kResidentMaxGroups) return false;
    // a periodic side must fall on a subdomain boundary
    if (p.bc != PRC_BC_CAVITY && p.nx % kResidentSX != 0) return false;
    if (p.bc == PRC_BC_PERIODIC && p.ny % kResidentSY != 0) return false;
    return true;
}

prc_status resident_prepare(hipStream_t s)
{
    ResidentDevice *d = nullptr;
    prc_status st = current_device(&d);
    if (st != PRC_OK) return st;
    std::lock_guard<std::mutex> lock(g_res_mu);
    if (d->sync) return PRC_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fail(PRC_EHIP, "resident sweep: its flags are set up by the first call on a "
                              "device, which must not be under graph capture");
    void *m = nullptr, *x = nullptr, *h = nullptr;
    hipEvent_t ev = nullptr;
    const size_t xbytes = (size_t)2 * kResidentMaxGroups * kXchElems * kXchPair;
    hipError_t e = hipMalloc(&m, sizeof(ResidentSync));
    if (e == hipSuccess) e = hipMalloc(&x, xbytes);
    if (e == hipSuccess) e = hipHostMalloc(&h, sizeof(uint64_t), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemset(m, 0, sizeof(ResidentSync));
    if (e == hipSuccess) e = hipMemset(x, 0, xbytes);  // every tag 0: no step yet
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (m) (void)hipFree(m);
        if (x) (void)hipFree(x);
        if (h) (void)hipHostFree(h);
        if (ev) (void)hipEventDestroy(ev);
        return fail(PRC_EHIP, "resident sweep: setting up its flags: %s", hipGetErrorString(e));
    }
    *(volatile uint64_t *)h = 0;
    d->sync = (ResidentSync *)m;
    d->xch = x;
    d->mailbox = (volatile uint64_t *)h;
    d->last = ev;
    d->has_last = false;
    g_res_devices.fetch_add(1);
    return PRC_OK;
}

prc_status launch_resident(const prc_params &p, const void *src, void *dst, int64_t nsteps,
                           hipStream_t s, int capturing, hipEvent_t start, hipEvent_t stop,
                           hipEvent_t after)
{
    ResidentDevice *d = nullptr;
    prc_status st = current_device(&d);
    if (st != PRC_OK) return st;
    if (p.storage == PRC_F64 || (size_t)d->lds < resident_lds_bytes(p.storage) ||
        resident_tiles(p) > d->cus || resident_tiles(p) > kResidentMaxGroups ||
        (p.bc != PRC_BC_CAVITY && p.nx % kResidentSX != 0) ||
        (p.bc == PRC_BC_PERIODIC && p.ny % kResidentSY != 0))
        return fail(PRC_EINVAL, "the resident sweep cannot run a %d x %d grid of storage %d",
                    p.nx, p.ny, p.storage);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (capturing < 0) HIP_TRY(hipStreamIsCapturing(s, &cap));
    else cap = capturing ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
    std::lock_guard<std::mutex> lock(g_res_mu);
    if (!d->sync) return fail(PRC_EHIP, "resident sweep: flags not set up on this device");
    // a launch on another stream than the latest one waits for that one
    // (launches captured into a graph are ordered by whoever replays it)
    const bool track = cap == hipStreamCaptureStatusNone;
    if (track && d->has_last && d->last_stream != s) HIP_TRY(hipStreamWaitEvent(s, d->last, 0));
    // The caller's event after the call is recorded by the last dispatch
    // itself, at the kernel's end, and the ordering event by a marker after
    // it: a marker right after a kernel adds no latency, but a second marker
    // behind the caller's added about 4 us to the call.  Under graph capture
    // every event is a marker (an event-record node) around plain launches.
    hipEvent_t first_ev = start, end = stop ? stop : after;
    if (!track) {
        if (start) HIP_TRY(hipEventRecord(start, s));
        first_ev = end = nullptr;
    }
    void *a = const_cast<void *>(src), *b = dst;
    bool first = true;
    while (nsteps > 0 && st == PRC_OK) {
        const int64_t n = nsteps < kResidentMaxSteps ? nsteps : kResidentMaxSteps;
        const bool last = n == nsteps;
        st = PRC_DISPATCH(p, launch_res, p, a, b, (int)n, *d, s, first ? first_ev : nullptr,
                          last ? end : nullptr);
        first = false;
        if (n & 1) std::swap(a, b);  // an odd count leaves the state in the second buffer
        nsteps -= n;
    }
    if (!track && st == PRC_OK) {
        if (stop) HIP_TRY(hipEventRecord(stop, s));
        if (after) HIP_TRY(hipEventRecord(after, s));
    } else if (stop && after && st == PRC_OK) {
        HIP_TRY(hipEventRecord(after, s));
    }
    if (track && st == PRC_OK) {
        HIP_TRY(hipEventRecord(d->last, s));
        d->has_last = true;
        d->last_stream = s;
    }
    return st;
}

prc_status resident_report()
{
    if (g_res_devices.load() == 0) return PRC_OK;
    ResidentDevice *d = nullptr;
    prc_status st = current_device(&d);
    if (st != PRC_OK || !d->mailbox) return st;
    if (*d->mailbox == 0) return PRC_OK;
    *d->mailbox = 0;
    return fail(PRC_EHIP, "resident sweep: a workgroup of an earlier launch on this device waited "
                          "in vain for a neighbour (not every subdomain had a compute unit at "
                          "once); the state it produced is invalid");
}

prc_status resident_release()
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PRC_EHIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_res_mu);
    ResidentDevice &d = g_res[dev];
    if (!d.sync) return PRC_OK;
    HIP_TRY(hipDeviceSynchronize());  // no launch may still use them
    hipError_t e = hipFree(d.sync);
    if (hipFree(d.xch) != hipSuccess && e == hipSuccess) e = hipErrorInvalidValue;
    if (hipHostFree((void *)d.mailbox) != hipSuccess && e == hipSuccess) e = hipErrorInvalidValue;
    if (hipEventDestroy(d.last) != hipSuccess && e == hipSuccess) e = hipErrorInvalidValue;
    d.sync = nullptr;
    d.xch = nullptr;
    d.mailbox = nullptr;
    d.last = nullptr;
    d.has_last = false;
    d.last_stream = nullptr;
    g_res_devices.fetch_sub(1);
    if (e != hipSuccess)
        return fail(PRC_EHIP, "resident sweep: releasing its buffers: %s", hipGetErrorString(e));
    return PRC_OK;
}

}  // namespace prc

namespace prc {
prc_status resident_set_wait(int64_t ticks)
{
    if (ticks < -1) return fail(PRC_EINVAL, "wait %lld ticks: need >= 0, or -1 for the default",
                                (long long)ticks);
    g_wait_ticks.store(ticks < 0 ? kResidentWaitTicks : (uint64_t)ticks, std::memory_order_relaxed);
    return PRC_OK;
}
}  // namespace prc
