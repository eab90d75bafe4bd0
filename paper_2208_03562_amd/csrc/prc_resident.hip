// Host side of the resident sweep (k_resident, prc_resident.hpp): which
// problems it can run, the per-device synchronisation block, the launches and
// the report of an aborted wait.
#include <hip/hip_runtime.h>

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
    int cus = 0;  // compute units
    int lds = 0;  // LDS a workgroup may use, bytes
};
std::mutex g_res_mu;
ResidentDevice g_res[kMaxDevices];

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
    return elem_bytes(storage) * 9 * (kResidentSY + 4) * (kResidentSX + 4) +
           ct * (kResidentSY + 2) * (kResidentSX + 2) + 8;
}

int resident_tiles(const prc_params &p)
{
    return ((p.nx + kResidentSX - 1) / kResidentSX) * ((p.ny + kResidentSY - 1) / kResidentSY);
}

template <typename ST, int BC>
prc_status launch_res(const prc_params &p, const void *src, void *dst, int nsteps,
                      const ResidentDevice &d, hipStream_t s)
{
    if constexpr (sizeof(ST) > 4) {  // an FP64 subdomain does not fit the LDS
        return fail(PRC_EINVAL, "the resident sweep has no FP64 instance");
    } else {
    auto c = coef_of<ST>(p);
    c.tiles_x = (p.nx + kResidentSX - 1) / kResidentSX;
    c.tiles_y = (p.ny + kResidentSY - 1) / kResidentSY;
    c.tiles_per_xcd = (c.tiles_x * c.tiles_y + kXcds - 1) / kXcds;
    const dim3 grid(c.tiles_per_xcd * kXcds), block(kResidentThreads);
    if (is_plain_method(p))
        hipLaunchKernelGGL((k_resident<ST, BC, false, true>), grid, block, 0, s, (ST *)src,
                           (ST *)dst, d.xch, c, d.sync, nsteps);
    else
        hipLaunchKernelGGL((k_resident<ST, BC, true, false>), grid, block, 0, s, (ST *)src,
                           (ST *)dst, d.xch, c, d.sync, nsteps);
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
    void *m = nullptr, *x = nullptr;
    const size_t xbytes = (size_t)2 * kResidentMaxGroups * kXchElems * kXchPair;
    hipError_t e = hipMalloc(&m, sizeof(ResidentSync));
    if (e == hipSuccess) e = hipMalloc(&x, xbytes);
    if (e == hipSuccess) e = hipMemset(m, 0, sizeof(ResidentSync));
    if (e == hipSuccess) e = hipMemset(x, 0, xbytes);  // every tag 0: no step yet
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (m) (void)hipFree(m);
        if (x) (void)hipFree(x);
        return fail(PRC_EHIP, "resident sweep: setting up its flags: %s", hipGetErrorString(e));
    }
    d->sync = (ResidentSync *)m;
    d->xch = x;
    return PRC_OK;
}

prc_status launch_resident(const prc_params &p, const void *src, void *dst, int64_t nsteps,
                           hipStream_t s)
{
    if (!resident_allowed(p))
        return fail(PRC_EINVAL, "the resident sweep cannot run a %d x %d grid of storage %d",
                    p.nx, p.ny, p.storage);
    ResidentDevice *d = nullptr;
    prc_status st = current_device(&d);
    if (st != PRC_OK) return st;
    if (!d->sync) return fail(PRC_EHIP, "resident sweep: flags not set up on this device");
    void *a = const_cast<void *>(src), *b = dst;
    while (nsteps > 0 && st == PRC_OK) {
        const int64_t n = nsteps < kResidentMaxSteps ? nsteps : kResidentMaxSteps;
        st = PRC_DISPATCH(p, launch_res, p, a, b, (int)n, *d, s);
        if (n & 1) std::swap(a, b);  // an odd count leaves the state in the second buffer
        nsteps -= n;
    }
    return st;
}

prc_status resident_check(hipStream_t s)
{
    ResidentDevice *d = nullptr;
    prc_status st = current_device(&d);
    if (st != PRC_OK || !d->sync) return st;
    uint64_t abort = 0;
    HIP_TRY(hipMemcpyAsync(&abort, &d->sync->abort, sizeof abort, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (abort == 0) return PRC_OK;
    HIP_TRY(hipMemsetAsync(&d->sync->abort, 0, sizeof abort, s));
    HIP_TRY(hipStreamSynchronize(s));
    return fail(PRC_EHIP, "resident sweep: a workgroup waited in vain for a neighbour (not every "
                          "subdomain had a compute unit); the state is invalid");
}

}  // namespace prc
