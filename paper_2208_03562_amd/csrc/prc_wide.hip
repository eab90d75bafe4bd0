// The two-step sweep on the 1024-thread tile shapes (64 x 16, 32 x 32),
// compiled on its own: build.py gives this file the instruction scheduler
// that favours instruction-level parallelism, which measured 6-9 % faster
// for these workgroups (1024 x 512 FP32 two-step on 64 x 16 tiles: 6.62 ->
// 6.16 us per step; 4096 x 2048 FP16: 68.1 -> 62.0 us) and slower for the
// 512-thread two-step shapes, which stay in prc_lib.hip.  Scheduling does not
// change the arithmetic: the results are the same bits.
#include <hip/hip_runtime.h>

#include "prc.h"
#include "prc_launch.hpp"

namespace prc {

template <typename ST, int BC>
static prc_status launch_wide(const prc_params &p, int tile, const void *src, void *dst,
                              hipStream_t s)
{
    if (tile == 7) return launch_sweep_variant<ST, BC, 64, 16, 2>(p, src, dst, s);
    return launch_sweep_variant<ST, BC, 32, 32, 2>(p, src, dst, s);
}

prc_status launch_sweep_wide(const prc_params &p, int tile, const void *src, void *dst,
                             hipStream_t s)
{
    if (tile != 7 && tile != 8) return fail(PRC_EINVAL, "tile %d is not a 1024-thread shape", tile);
    return PRC_DISPATCH(p, launch_wide, p, tile, src, dst, s);
}

}  // namespace prc
