// Host-side helpers shared by the library's source files: error reporting,
// state layout, parameter validation, per-launch constants, tile shapes and
// the dispatch over storage and boundary types.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "prc.h"
#include "prc_coef.hpp"
#include "prc_device.hpp"

namespace prc {

// ---------------------------------------------------------------- errors --
// Message of the last failed call, per thread (shared by every source file
// of the library).
inline std::string &err_slot()
{
    static thread_local std::string s;
    return s;
}

inline prc_status fail(prc_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
inline prc_status fail(prc_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err_slot() = buf;
    return s;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(PRC_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),         \
                        __FILE__, __LINE__);                                             \
    } while (0)

// ---------------------------------------------------------------- layout --
constexpr int kPitchAlignBytes = 256;
constexpr int kRedBlock = 256;
constexpr int kRedMaxBlocks = 1024;

inline size_t elem_bytes(int storage)
{
    switch (storage) {
    case PRC_F64: return 8;
    case PRC_F32: return 4;
    default: return 2;
    }
}

// State layouts (element (a, j, i) at a * plane + j * row + i):
//   0  plane-major: nine whole planes one after the other
//   1  plane-major with each plane padded by kPlanePadBytes, so that the nine
//      loads of a node do not all fall on addresses a power of two apart
//   2  row-interleaved: row j of all nine planes stored together
//      ([j][a][i]), so a tile's loads and stores stay within a few DRAM pages
constexpr int kLayoutDefault = 2;
constexpr int64_t kPlanePadBytes = 4096 + 256;

inline int layout_mode()
{
    static const int v = [] {
        const char *e = std::getenv("PRC_LAYOUT");
        const int m = e ? std::atoi(e) : kLayoutDefault;
        return (m >= 0 && m <= 2) ? m : kLayoutDefault;
    }();
    return v;
}

// row and plane strides and total size, in elements
inline void layout(const prc_params &p, int64_t &row, int64_t &plane, int64_t &total)
{
    const int64_t E = (int64_t)elem_bytes(p.storage);
    const int64_t per = kPitchAlignBytes / E;
    const int64_t pitch = ((int64_t)p.nx + per - 1) / per * per;
    switch (layout_mode()) {
    case 1:
        row = pitch;
        plane = pitch * p.ny + kPlanePadBytes / E;
        total = 9 * plane;
        break;
    case 2:
        row = 9 * pitch;
        plane = pitch;
        total = row * p.ny;
        break;
    default:
        row = pitch;
        plane = pitch * p.ny;
        total = 9 * plane;
    }
}

inline prc_status validate(const prc_params *p)
{
    if (!p) return fail(PRC_EINVAL, "params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(PRC_EINVAL, "nx, ny must be >= 3 (got %d, %d)", p->nx, p->ny);
    if ((int64_t)p->nx * p->ny > ((int64_t)1 << 30))
        return fail(PRC_EINVAL, "grid too large (%d x %d)", p->nx, p->ny);
    if (!(p->r > 0.0) || !std::isfinite(p->r)) return fail(PRC_EINVAL, "r must be > 0");
    if (!(p->gamma > 0.0 && p->gamma <= 1.0)) return fail(PRC_EINVAL, "gamma must be in (0, 1]");
    const double om[5] = {p->omega_nu, p->omega_xi, p->omega_1, p->omega_3, p->omega_4};
    for (double w : om)
        if (!(w > 0.0 && w < 2.0)) return fail(PRC_EINVAL, "relaxation rates must be in (0, 2)");
    const double q = p->r < 1.0 ? p->r : 1.0;
    if (!(std::fabs(p->u_lid) < q / std::sqrt(3.0)))
        return fail(PRC_EINVAL, "|u_lid| must be below the sound speed q/sqrt(3)");
    if (!std::isfinite(p->fx) || !std::isfinite(p->fy)) return fail(PRC_EINVAL, "force not finite");
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(PRC_EINVAL, "rho0 must be > 0");
    if (p->bc < PRC_BC_CAVITY || p->bc > PRC_BC_CHANNEL) return fail(PRC_EINVAL, "unknown bc %d", p->bc);
    if (p->storage < PRC_F64 || p->storage > PRC_BF16)
        return fail(PRC_EINVAL, "unknown storage %d", p->storage);
    if (p->corrections < 0 || p->corrections > PRC_CORR_ALL)
        return fail(PRC_EINVAL, "corrections bitmask out of range");
    if (p->frame != PRC_FRAME_CENTRAL && p->frame != PRC_FRAME_RAW)
        return fail(PRC_EINVAL, "unknown frame %d", p->frame);
    int64_t row, plane, total;
    layout(*p, row, plane, total);
    // byte offsets into one state buffer are 32-bit (buffer addressing)
    if (total * (int64_t)elem_bytes(p->storage) > (int64_t)0xFFFFFFFF)
        return fail(PRC_EINVAL, "state of %d x %d exceeds 4 GiB", p->nx, p->ny);
    return PRC_OK;
}

inline prc_status check_buf(const void *b, const char *name)
{
    if (!b) return fail(PRC_EINVAL, "%s is NULL", name);
    if ((uintptr_t)b % 256 != 0) return fail(PRC_EINVAL, "%s is not 256-byte aligned", name);
    return PRC_OK;
}

template <typename ST>
inline Coef<typename Mem<ST>::CT> coef_of(const prc_params &p)
{
    int64_t row, plane, total;
    layout(p, row, plane, total);
    return make_coef<typename Mem<ST>::CT>(p, row, plane, total, (int64_t)sizeof(ST));
}

// The method as the paper runs it, for which the sweep has a specialised
// instance: every correction, no body force, central frame, and the unit
// rates omega_xi = omega_1 = omega_3 = omega_4 = 1 of Appendix A.
inline bool is_plain_method(const prc_params &p)
{
    return p.corrections == PRC_CORR_ALL && p.fx == 0.0 && p.fy == 0.0 &&
           p.frame == PRC_FRAME_CENTRAL && p.omega_xi == 1.0 && p.omega_1 == 1.0 &&
           p.omega_3 == 1.0 && p.omega_4 == 1.0;
}

// blocks of the residual reduction for a grid (each block strides over the
// nodes with gridDim * kRedBlock; the partition fixes the summation order)
inline int red_blocks(const prc_params &p)
{
    const int64_t N = (int64_t)p.nx * p.ny;
    int64_t b = (N + kRedBlock - 1) / kRedBlock;
    return (int)(b < kRedMaxBlocks ? b : kRedMaxBlocks);
}

// Sweep tile shapes (threads along x, along y).  A taller tile needs fewer
// ring densities per node; a wider one gives longer contiguous row segments.
struct TileShape {
    int tx, ty;
    int steps;  // time steps per launch: 1 (k_sweep), 2 (k_sweep2), 0 any (k_resident)
};
// Narrow shapes waste fewer threads on grids whose width is not a multiple
// of 64 (batches of small problems); a wavefront then spans two or four rows.
// The two-step shapes (5 and 6 also for batches) trade the collisions of two
// extra rings per tile for half the state traffic and half the launches;
// squarer tiles have relatively smaller rings.  The last entry is the
// resident sweep: 64 x 32-node subdomains, two nodes per thread, any number
// of steps per launch, for grids whose state fits the chip's LDS.
constexpr TileShape kTiles[] = {{64, 4, 1},  {64, 8, 1},  {128, 4, 1}, {32, 8, 1},
                                {32, 16, 1}, {64, 8, 2},  {32, 16, 2}, {64, 16, 2},
                                {32, 32, 2}, {64, 32, 0}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kNumSingleStepTiles = 5;  // indices below this advance one step
// Batches use the shapes below this index: the single-step ones and the
// two-step shapes, each of which has a single-step twin of the same tile
// (64 x 8 -> 1, 32 x 16 -> 4; 64 x 16 has a 1024-thread single-step instance
// of its own for batches), so that one tile list serves both.
constexpr int kNumBatchTiles = 8;
constexpr int kResidentTile = 9;

// Whether the resident sweep can run problem p on the current device
// (prc_resident.hip).
bool resident_allowed(const prc_params &p);

// Whether tile shape `tile` may run problem p (every sweep shape runs every
// storage; the resident sweep needs a state that fits the LDS).
inline bool tile_allowed(const prc_params &p, int tile)
{
    if (tile == kResidentTile) return resident_allowed(p);
    return tile >= 0 && tile < kNumTiles;
}

// run F<ST, BC>(args...) for the storage and boundary type of p
#define PRC_DISPATCH(p, FN, ...)                                                          \
    [&]() -> prc_status {                                                                \
        switch ((p).storage * 3 + (p).bc) {                                              \
        case PRC_F64 * 3 + 0: return FN<double, 0>(__VA_ARGS__);                         \
        case PRC_F64 * 3 + 1: return FN<double, 1>(__VA_ARGS__);                         \
        case PRC_F64 * 3 + 2: return FN<double, 2>(__VA_ARGS__);                         \
        case PRC_F32 * 3 + 0: return FN<float, 0>(__VA_ARGS__);                          \
        case PRC_F32 * 3 + 1: return FN<float, 1>(__VA_ARGS__);                          \
        case PRC_F32 * 3 + 2: return FN<float, 2>(__VA_ARGS__);                          \
        case PRC_F16 * 3 + 0: return FN<__half, 0>(__VA_ARGS__);                         \
        case PRC_F16 * 3 + 1: return FN<__half, 1>(__VA_ARGS__);                         \
        case PRC_F16 * 3 + 2: return FN<__half, 2>(__VA_ARGS__);                         \
        case PRC_BF16 * 3 + 0: return FN<__hip_bfloat16, 0>(__VA_ARGS__);                \
        case PRC_BF16 * 3 + 1: return FN<__hip_bfloat16, 1>(__VA_ARGS__);                \
        case PRC_BF16 * 3 + 2: return FN<__hip_bfloat16, 2>(__VA_ARGS__);                \
        }                                                                                \
        return fail(PRC_EINVAL, "bad storage/bc");                                       \
    }()

// Steps per captured launch graph (a multiple of four, so that the newest
// state is back in the first buffer after every replay for one- and
// two-step launches alike).
constexpr int kGraphStepsDefault = 64;

// sweeps per graph; PRC_GRAPH_STEPS overrides (0 disables graphs)
inline int graph_steps()
{
    static const int v = [] {
        const char *e = std::getenv("PRC_GRAPH_STEPS");
        if (!e) return kGraphStepsDefault;
        const int n = std::atoi(e);
        return n <= 0 ? 0 : (n + 3) / 4 * 4;
    }();
    return v;
}

}  // namespace prc
