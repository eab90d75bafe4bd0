// Launch of one sweep (one or two time steps) on a tile shape, shared by the
// library's source files.
#pragma once

#include <hip/hip_runtime.h>

#include "prc.h"
#include "prc_coef.hpp"
#include "prc_host.hpp"
#include "prc_sweep.hpp"
#include "prc_sweep2.hpp"

namespace prc {

template <typename ST, int BC, int TX, int TY, bool FORCE, bool ALL, int STEPS>
inline prc_status launch_sweep_shape(const prc_params &p, const void *src, void *dst, hipStream_t s)
{
    auto c = coef_of<ST>(p);
    c.tiles_x = (p.nx + TX - 1) / TX;
    c.tiles_y = (p.ny + TY - 1) / TY;
    const int tiles = c.tiles_x * c.tiles_y;
    c.tiles_per_xcd = (tiles + kXcds - 1) / kXcds;
    if constexpr (STEPS == 2) {
        // the load order differs for 1024-thread tiles of a state streamed
        // from HBM (non-temporal stores mark it)
        if constexpr (TX * TY > 512) {
            if (c.nt)
                hipLaunchKernelGGL((k_sweep2<ST, BC, TX, TY, FORCE, ALL, true>),
                                   dim3(c.tiles_per_xcd * kXcds), dim3(TX * TY), 0, s,
                                   (const ST *)src, (ST *)dst, c);
            else
                hipLaunchKernelGGL((k_sweep2<ST, BC, TX, TY, FORCE, ALL, false>),
                                   dim3(c.tiles_per_xcd * kXcds), dim3(TX * TY), 0, s,
                                   (const ST *)src, (ST *)dst, c);
        } else {
            hipLaunchKernelGGL((k_sweep2<ST, BC, TX, TY, FORCE, ALL, false>),
                               dim3(c.tiles_per_xcd * kXcds), dim3(TX * TY), 0, s,
                               (const ST *)src, (ST *)dst, c);
        }
    } else {
        hipLaunchKernelGGL((k_sweep<ST, BC, TX, TY, FORCE, ALL>), dim3(c.tiles_per_xcd * kXcds),
                           dim3(TX * TY), 0, s, (const ST *)src, (ST *)dst, c);
    }
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

// The method as the paper runs it (every correction, no body force, central
// frame, unit non-hydrodynamic rates) runs a specialised kernel; anything
// else runs the general one.
template <typename ST, int BC, int TX, int TY, int STEPS = 1>
inline prc_status launch_sweep_variant(const prc_params &p, const void *src, void *dst,
                                       hipStream_t s)
{
    if (is_plain_method(p))
        return launch_sweep_shape<ST, BC, TX, TY, false, true, STEPS>(p, src, dst, s);
    return launch_sweep_shape<ST, BC, TX, TY, true, false, STEPS>(p, src, dst, s);
}

// One two-step launch on the 1024-thread tile shapes 7 (64 x 16) and 8
// (32 x 32), defined in prc_wide.hip.
prc_status launch_sweep_wide(const prc_params &p, int tile, const void *src, void *dst,
                             hipStream_t s);

// The resident sweep (prc_resident.hip): setting up its flags on the current
// device (once, not under graph capture); nsteps time steps from src (the
// state after an odd count in dst, after an even count back in src), after
// the latest resident launch on the device if that was on another stream;
// the report, without synchronising, of a launch that lost a workgroup's wait
// (PRC_EHIP once per such report; launches still running may report later);
// and the release of the device's resident buffers (after a device
// synchronise).
prc_status resident_prepare(hipStream_t s);
// (capturing: whether s is under graph capture, -1 to ask the runtime;
// start/stop, if given, are recorded by the dispatch of the first and the
// last kernel: the start of the first, the end of the last; after, if given,
// marks the end of the call's work: the last kernel's dispatch records it
// when stop is not given, a marker behind it otherwise; under capture all
// three are markers around the launches)
prc_status launch_resident(const prc_params &p, const void *src, void *dst, int64_t nsteps,
                           hipStream_t s, int capturing = -1, hipEvent_t start = nullptr,
                           hipEvent_t stop = nullptr, hipEvent_t after = nullptr);
prc_status resident_report();
prc_status resident_release();
// wait limit of later resident launches, in 100 MHz ticks (-1: the default)
prc_status resident_set_wait(int64_t ticks);

}  // namespace prc
