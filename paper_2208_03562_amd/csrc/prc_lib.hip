// C ABI of the PRC-LBM library for MI355X (gfx950): single problems.
//
// Kernels launched here:
//   k_sweep     one fused time step: pull with boundaries, fields, density
//               gradient from an LDS tile of densities, collision, store
//               (prc_sweep.hpp, prc_collide.hpp)
//   k_sweep2    two time steps per launch (prc_sweep2.hpp); the 1024-thread
//               tile shapes are launched from prc_wide.hip
//   k_macros    fields of a state (for output)
//   k_residual  per-block FP64 partial sums of the convergence check
//   k_finish    fixed-order reduction of the partial sums (prc_reduce.hpp)
//   k_zero      rest state
// Batches are in prc_batch.hip, the request server in prc_serve.hip.  The
// ABI is declared and documented in include/prc.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "prc.h"
#include "prc_coef.hpp"
#include "prc_device.hpp"
#include "prc_host.hpp"
#include "prc_launch.hpp"
#include "prc_reduce.hpp"
#include "prc_sweep.hpp"
#include "prc_sweep2.hpp"

namespace prc {

// ------------------------------------------------------------- kernels --

template <typename ST, int BC>
__global__ void k_macros(const ST *__restrict__ f, const Coef<typename Mem<ST>::CT> c, double *rho,
                         double *ux, double *uy)
{
    using CT = typename Mem<ST>::CT;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)c.nx * c.ny) return;
    const int x = (int)(n % c.nx), y = (int)(n / c.nx);
    CT d[9];
    pull_checked<ST, BC>(c, make_rsrc(f, c.state_bytes), x, y, d);
    CT drho, u, v;
    fields(c, d, drho, u, v);
    if (rho) rho[n] = (double)c.rho0 + (double)drho;
    if (ux) ux[n] = (double)u;
    if (uy) uy[n] = (double)v;
}


// The state of an nx x ny grid from one storage type and layout into
// another (grid-stride over population planes, rows, nodes); each value goes
// through the wider of the two compute types, so widening is exact.
template <typename SRC, typename DST>
__global__ void k_convert(const SRC *__restrict__ src, DST *__restrict__ dst, int nx, int ny,
                          uint32_t s_row, uint32_t s_plane, uint32_t s_bytes, uint32_t d_row,
                          uint32_t d_plane, uint32_t d_bytes)
{
    const rsrc_t rs = make_rsrc(src, s_bytes), rd = make_rsrc(dst, d_bytes);
    const int64_t n = (int64_t)9 * nx * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k % nx);
        const int64_t q = k / nx;
        const int j = (int)(q % ny), a = (int)(q / ny);
        const auto v = Mem<SRC>::ld(rs, (uint32_t)a * s_plane + (uint32_t)j * s_row +
                                            (uint32_t)i * (uint32_t)sizeof(SRC), 0);
        Mem<DST>::st(rd, (uint32_t)a * d_plane + (uint32_t)j * d_row + (uint32_t)i * (uint32_t)sizeof(DST),
                     0, (typename Mem<DST>::CT)v);
    }
}

// Nine per-population constants passed by value.
template <typename CT>
struct Nine {
    CT v[9];
};

// Adds delta.v[a] to population a of every node of the state (grid-stride).
template <typename ST>
__global__ void k_add_rest(ST *__restrict__ f, int nx, int ny, uint32_t row, uint32_t plane,
                           uint32_t bytes, const Nine<typename Mem<ST>::CT> delta)
{
    const rsrc_t r = make_rsrc(f, bytes);
    const int64_t n = (int64_t)9 * nx * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k % nx);
        const int64_t q = k / nx;
        const int j = (int)(q % ny), a = (int)(q / ny);
        const uint32_t o = (uint32_t)a * plane + (uint32_t)j * row + (uint32_t)i * (uint32_t)sizeof(ST);
        Mem<ST>::st(r, o, 0, Mem<ST>::ld(r, o, 0) + delta.v[a]);
    }
}

// zero fill of n 16-byte words (grid-stride)
__global__ void k_zero(uint4 *__restrict__ p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Tile shape per problem: what prc_tune measured for this grid, else a
// default (wide tiles for wide grids); PRC_TILE=<index> forces one shape.
// storage, boundary type, grid and layout mode of a problem
struct TuneKey {
    int32_t nx, ny, mode;
    bool operator==(const TuneKey &o) const { return nx == o.nx && ny == o.ny && mode == o.mode; }
};
struct TuneKeyHash {
    size_t operator()(const TuneKey &k) const
    {
        return std::hash<uint64_t>()(((uint64_t)(uint32_t)k.nx << 32) ^ (uint64_t)(uint32_t)k.ny ^
                                     ((uint64_t)(uint32_t)k.mode << 48));
    }
};
static std::mutex g_tune_mu;
static std::unordered_map<TuneKey, int, TuneKeyHash> g_tuned;

static TuneKey tune_key(const prc_params &p)
{
    return TuneKey{p.nx, p.ny, (p.storage * 3 + p.bc) * 3 + layout_mode()};
}

static int tile_choice(const prc_params &p)
{
    static const int forced = [] {
        const char *e = std::getenv("PRC_TILE");
        const int i = e ? std::atoi(e) : -1;
        return (i >= 0 && i < kNumTiles) ? i : -1;
    }();
    if (forced >= 0 && tile_allowed(p, forced)) return forced;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(tune_key(p));
        if (it != g_tuned.end()) return it->second;
    }
    // measured on MI355X: a grid whose state fits the LDS of the chip with
    // one subdomain per CU runs the resident sweep (1024 x 512 FP32: 3.5
    // against 6.2 us per step for two steps per launch); on other grids that
    // fill the chip two steps per launch pay for every storage type.  FP32
    // and 16-bit: 64 x 16 tiles (4096 x 2048 FP32: 71.5 against 73.1 us per
    // step on 32 x 32); FP64 (twice the LDS per tile, so 512-thread tiles):
    // 64 x 8 in the last-level cache, 32 x 16 from HBM
    if (p.nx >= 256 && p.ny >= 64) {
        if (resident_allowed(p)) return kResidentTile;
        if (p.storage == PRC_F64) {
            int64_t row, plane, total;
            layout(p, row, plane, total);
            const bool cached = 2 * total * (int64_t)elem_bytes(p.storage) <= kNtPairBytes;
            return cached ? 5 : 6;
        }
        return 7;
    }
    return p.nx >= 256 ? 2 : 0;
}

// Steps of one resident launch when shapes are timed against each other:
// one convergence-check interval, as the solver runs it.
constexpr int kResidentTuneSteps = 1000;

// One launch of tile shape `tile`: kTiles[tile].steps time steps, src -> dst
// (the resident sweep: kResidentTuneSteps steps, the state back in src).
template <typename ST, int BC>
static prc_status launch_sweep_tile(const prc_params &p, int tile, const void *src, void *dst,
                                    hipStream_t s)
{
    switch (tile) {
    case 1: return launch_sweep_variant<ST, BC, 64, 8>(p, src, dst, s);
    case 2: return launch_sweep_variant<ST, BC, 128, 4>(p, src, dst, s);
    case 3: return launch_sweep_variant<ST, BC, 32, 8>(p, src, dst, s);
    case 4: return launch_sweep_variant<ST, BC, 32, 16>(p, src, dst, s);
    case 5: return launch_sweep_variant<ST, BC, 64, 8, 2>(p, src, dst, s);
    case 6: return launch_sweep_variant<ST, BC, 32, 16, 2>(p, src, dst, s);
    case 7:
    case 8: return launch_sweep_wide(p, tile, src, dst, s);  // prc_wide.hip
    case kResidentTile: return launch_resident(p, src, dst, kResidentTuneSteps, s);
    default: return launch_sweep_variant<ST, BC, 64, 4>(p, src, dst, s);
    }
}

// The single-step shape used next to a two-step one for the odd steps.
static int single_step_tile(int tile)
{
    return kTiles[tile].steps == 1 ? tile : (kTiles[tile].tx >= 64 ? 1 : 4);
}

// Launch sequence for steps [k0, k0 + n) from buffers (f_a, f_b): step k reads
// f_a when k is even.  A two-step launch moves the state across one buffer
// flip for two steps, so pairs of them (f_a -> f_b -> f_a) cover the steps in
// fours from an even step and leave every state a caller can see on the
// buffer the single-step sequence puts it in; single steps do the rest.
static prc_status run_steps(const prc_params &p, int tile, void *f_a, void *f_b, int64_t k0,
                            int64_t n, hipStream_t s, int capturing = -1,
                            hipEvent_t start = nullptr, hipEvent_t stop = nullptr,
                            hipEvent_t after = nullptr)
{
    if (tile == kResidentTile)  // any number of steps per launch
        return launch_resident(p, (k0 & 1) ? f_b : f_a, (k0 & 1) ? f_a : f_b, n, s, capturing,
                               start, stop, after);
    prc_status st = PRC_OK;
    int64_t k = k0;
    const int64_t end = k0 + n;
    const int one = single_step_tile(tile);
    auto single = [&]() {
        const void *src = (k & 1) ? f_b : f_a;
        void *dst = (k & 1) ? f_a : f_b;
        ++k;
        return PRC_DISPATCH(p, launch_sweep_tile, p, one, src, dst, s);
    };
    if (kTiles[tile].steps == 2) {
        if (k < end && (k & 1)) st = single();
        for (; k + 4 <= end && st == PRC_OK; k += 4) {
            // steps k, k+1: f_a -> f_b; steps k+2, k+3: f_b -> f_a
            st = PRC_DISPATCH(p, launch_sweep_tile, p, tile, f_a, f_b, s);
            if (st == PRC_OK) st = PRC_DISPATCH(p, launch_sweep_tile, p, tile, f_b, f_a, s);
        }
    }
    while (k < end && st == PRC_OK) st = single();
    return st;
}

template <typename ST, int BC>
static prc_status launch_macros(const prc_params &p, const void *f, double *rho, double *ux,
                                double *uy, hipStream_t s)
{
    const auto c = coef_of<ST>(p);
    const int64_t N = (int64_t)p.nx * p.ny;
    hipLaunchKernelGGL((k_macros<ST, BC>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       (const ST *)f, c, rho, ux, uy);
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

template <typename ST, int BC>
static prc_status launch_residual(const prc_params &p, const void *f, double *u_prev,
                                  double *scratch, hipStream_t s)
{
    const auto c = coef_of<ST>(p);
    const int nb = red_blocks(p);
    hipLaunchKernelGGL((k_residual<ST, BC>), dim3(nb), dim3(kRedBlock), 0, s, (const ST *)f, c,
                       u_prev, scratch);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_finish<>, dim3(1), dim3(kRedBlock), 0, s, (const double *)scratch, nb,
                       scratch + 4 * kRedMaxBlocks);
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

template <typename SRC, typename DST>
static prc_status launch_convert_to(const prc_params &pf, const void *f, const prc_params &pt,
                                    void *g, hipStream_t s)
{
    int64_t sr, sp, st_, dr, dp, dt;
    layout(pf, sr, sp, st_);
    layout(pt, dr, dp, dt);
    const int64_t n = (int64_t)9 * pf.nx * pf.ny;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_convert<SRC, DST>), dim3(blocks), dim3(256), 0, s, (const SRC *)f,
                       (DST *)g, pf.nx, pf.ny, (uint32_t)(sr * sizeof(SRC)),
                       (uint32_t)(sp * sizeof(SRC)), (uint32_t)(st_ * sizeof(SRC)),
                       (uint32_t)(dr * sizeof(DST)), (uint32_t)(dp * sizeof(DST)),
                       (uint32_t)(dt * sizeof(DST)));
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

template <typename SRC>
static prc_status launch_convert(const prc_params &pf, const void *f, const prc_params &pt, void *g,
                                 hipStream_t s)
{
    switch (pt.storage) {
    case PRC_F64: return launch_convert_to<SRC, double>(pf, f, pt, g, s);
    case PRC_F32: return launch_convert_to<SRC, float>(pf, f, pt, g, s);
    case PRC_F16: return launch_convert_to<SRC, __half>(pf, f, pt, g, s);
    case PRC_BF16: return launch_convert_to<SRC, __hip_bfloat16>(pf, f, pt, g, s);
    }
    return fail(PRC_EINVAL, "bad storage %d", pt.storage);
}

template <typename ST, int BC>
static prc_status launch_add_rest(const prc_params &p, void *f, double drho, hipStream_t s)
{
    using CT = typename Mem<ST>::CT;
    // rest weights: products of the one-dimensional weights of variance c2
    // along x and c2 / r^2 along y (velocity order of Sec. 2)
    static const int EXh[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static const int EYh[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const double c2 = lattice_c2(p.r), vy = c2 / (p.r * p.r);
    Nine<CT> d;
    for (int a = 0; a < 9; ++a) {
        const double wx = EXh[a] == 0 ? 1.0 - c2 : 0.5 * c2;
        const double wy = EYh[a] == 0 ? 1.0 - vy : 0.5 * vy;
        d.v[a] = (CT)(drho * wx * wy);
    }
    int64_t row, plane, total;
    layout(p, row, plane, total);
    const int64_t n = (int64_t)9 * p.nx * p.ny;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL((k_add_rest<ST>), dim3(blocks), dim3(256), 0, s, (ST *)f, p.nx, p.ny,
                       (uint32_t)(row * sizeof(ST)), (uint32_t)(plane * sizeof(ST)),
                       (uint32_t)(total * sizeof(ST)), d);
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

// --------------------------------------------------------- launch graphs --
// prc_step replays captured graphs of sweeps for long runs: one graph per
// (device, problem, buffer pair), cached until prc_release_graphs(); when the
// cache is full the least recently used graph leaves it.  A caller holds its
// entry while replaying it, and an entry is destroyed only after its device
// has finished every replay.
constexpr size_t kGraphCacheMax = 32;

static_assert(sizeof(prc_params) == 8 + 11 * 8 + 4 * 4, "prc_params has no padding");

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int dev = 0;
    uint64_t used = 0;  // cache clock of the latest lookup
    GraphEntry() = default;
    GraphEntry(const GraphEntry &) = delete;
    GraphEntry &operator=(const GraphEntry &) = delete;
    ~GraphEntry()
    {
        // replays still in flight must finish before the exec goes away
        int cur = -1;
        const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != dev;
        if (switch_dev) (void)hipSetDevice(dev);
        (void)hipDeviceSynchronize();
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (switch_dev) (void)hipSetDevice(cur);
    }
};
static std::mutex g_graph_mu;
static std::unordered_map<std::string, std::shared_ptr<GraphEntry>> g_graphs;
static uint64_t g_graph_clock = 0;

static prc_status get_graph(const prc_params &p, int tile, void *f_a, void *f_b, int nsteps,
                            std::shared_ptr<GraphEntry> *out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const int streamed = g_streamed_mode.load(std::memory_order_relaxed);
    std::string key(reinterpret_cast<const char *>(&p), sizeof p);
    key.append(reinterpret_cast<const char *>(&tile), sizeof tile);
    key.append(reinterpret_cast<const char *>(&f_a), sizeof f_a);
    key.append(reinterpret_cast<const char *>(&f_b), sizeof f_b);
    key.append(reinterpret_cast<const char *>(&dev), sizeof dev);
    key.append(reinterpret_cast<const char *>(&nsteps), sizeof nsteps);
    key.append(reinterpret_cast<const char *>(&streamed), sizeof streamed);
    std::shared_ptr<GraphEntry> evicted;  // destroyed after the lock is released
    std::lock_guard<std::mutex> lock(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
        it->second->used = ++g_graph_clock;
        *out = it->second;
        return PRC_OK;
    }
    if (g_graphs.size() >= kGraphCacheMax) {
        auto lru = g_graphs.begin();
        for (auto j = g_graphs.begin(); j != g_graphs.end(); ++j)
            if (j->second->used < lru->second->used) lru = j;
        evicted = std::move(lru->second);
        g_graphs.erase(lru);
    }
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    prc_status st = PRC_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = run_steps(p, tile, f_a, f_b, 0, nsteps, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess && st == PRC_OK) {
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            if (e == hipSuccess) {
                auto entry = std::make_shared<GraphEntry>();
                entry->graph = g;
                entry->exec = x;
                entry->dev = dev;
                entry->used = ++g_graph_clock;
                g_graphs.emplace(key, entry);
                *out = std::move(entry);
            } else {
                (void)hipGraphDestroy(g);
            }
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (st != PRC_OK) return st;
    if (e != hipSuccess)
        return fail(PRC_EHIP, "graph capture of %d sweeps: %s", nsteps, hipGetErrorString(e));
    return PRC_OK;
}

// The convergence check with its block partials and result in sc (device,
// 4 * kRedMaxBlocks + 4 doubles): launches, copies the result to the host,
// synchronises the stream, reports a failed resident launch, and adds the
// rest part of the mass.
static prc_status residual_into(const prc_params &p, const void *f, double *u_prev, double *sc,
                                double out[4], hipStream_t stream)
{
    prc_status st = PRC_DISPATCH(p, launch_residual, p, f, u_prev, sc, stream);
    if (st != PRC_OK) return st;
    HIP_TRY(hipMemcpyAsync(out, sc + 4 * kRedMaxBlocks, 4 * sizeof(double),
                           hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if ((st = resident_report()) != PRC_OK) return st;
    out[2] += p.rho0 * (double)p.nx * (double)p.ny;  // rest part of the mass
    return PRC_OK;
}

// ------------------------------------------ scratch that needs no allocation --
// prc_residual_noalloc keeps the block partials and the result of the check
// here instead of in a caller's buffer: 4 * kRedMaxBlocks + 4 doubles (32 KiB
// + 32 bytes; the largest partition of any problem), one copy on every device
// the library runs on, held until the process ends.  Every call on a device
// shares that device's copy.  Host code must not use this name as an address
// (it is a host-side stand-in): the device address comes from
// hipGetSymbolAddress, once per device, in static_scratch().
static __device__ __align__(256) double scratch[4 * kRedMaxBlocks + 4];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on each device, with that device current).
static prc_status static_scratch(double **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(PRC_EHIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PRC_EHIP, "address of the static scratch array on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return PRC_OK;
}

}  // namespace prc

using namespace prc;

// ----------------------------------------------------------------- ABI --
extern "C" {

prc_status prc_params_default(prc_params *p)
{
    if (!p) return fail(PRC_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->r = 1.0;
    p->gamma = 1.0;
    p->omega_nu = p->omega_xi = p->omega_1 = p->omega_3 = p->omega_4 = 1.0;
    p->rho0 = 1.0;
    p->bc = PRC_BC_CAVITY;
    p->storage = PRC_F32;
    p->corrections = PRC_CORR_ALL;
    p->frame = PRC_FRAME_CENTRAL;
    return PRC_OK;
}

prc_status prc_params_from_re(prc_params *p, double re)
{
    if (!p) return fail(PRC_EINVAL, "params is NULL");
    if (!(re > 0.0) || p->u_lid == 0.0 || !(p->r > 0.0) || !(p->gamma > 0.0) || p->ny <= 0)
        return fail(PRC_EINVAL, "need re > 0, u_lid != 0, r > 0, gamma > 0, ny > 0");
    const double H = (double)p->ny * p->r;
    const double nu = std::fabs(p->u_lid) * H / re;
    const double w = 1.0 / (nu / (p->gamma * lattice_c2(p->r)) + 0.5);
    if (!(w > 0.0 && w < 2.0)) return fail(PRC_EINVAL, "omega_nu %g out of (0, 2)", w);
    p->omega_nu = w;
    return PRC_OK;
}

prc_status prc_validate(const prc_params *p) { return validate(p); }

prc_status prc_layout(const prc_params *p, int64_t *row_stride, int64_t *plane_stride)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if (!row_stride || !plane_stride) return fail(PRC_EINVAL, "NULL output");
    int64_t total;
    layout(*p, *row_stride, *plane_stride, total);
    return PRC_OK;
}

size_t prc_state_bytes(const prc_params *p)
{
    if (validate(p) != PRC_OK) return 0;
    int64_t row, plane, total;
    layout(*p, row, plane, total);
    return (size_t)total * elem_bytes(p->storage);
}

size_t prc_scratch_bytes(const prc_params *p)
{
    if (validate(p) != PRC_OK) return 0;
    return (size_t)(4 * kRedMaxBlocks + 4) * sizeof(double);
}

prc_status prc_init(const prc_params *p, void *f, hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if ((st = check_buf(f, "f")) != PRC_OK) return st;
    // all-zero bits are +0 in every storage type; a kernel rather than a
    // memset node, so that the call can be captured into a graph
    const size_t words = prc_state_bytes(p) / sizeof(uint4);  // a multiple of 256 B
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, stream, (uint4 *)f, words);
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

static prc_status step_impl(const prc_params *p, void *f_a, void *f_b, int64_t nsteps,
                            hipEvent_t start, hipEvent_t stop, bool kernel_only,
                            hipStream_t stream);

prc_status prc_step(const prc_params *p, void *f_a, void *f_b, int64_t nsteps, hipStream_t stream)
{
    return step_impl(p, f_a, f_b, nsteps, nullptr, nullptr, false, stream);
}

prc_status prc_step_timed(const prc_params *p, void *f_a, void *f_b, int64_t nsteps,
                          hipEvent_t start, hipEvent_t stop, int32_t kernel_only,
                          hipStream_t stream)
{
    if (!start || !stop) return fail(PRC_EINVAL, "NULL start or stop event");
    return step_impl(p, f_a, f_b, nsteps, start, stop, kernel_only != 0, stream);
}

static prc_status step_impl(const prc_params *p, void *f_a, void *f_b, int64_t nsteps,
                            hipEvent_t start, hipEvent_t stop, bool kernel_only,
                            hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if ((st = check_buf(f_a, "f_a")) != PRC_OK || (st = check_buf(f_b, "f_b")) != PRC_OK) return st;
    if (f_a == f_b) return fail(PRC_EINVAL, "f_a and f_b must be distinct buffers");
    if (nsteps < 0) return fail(PRC_EINVAL, "nsteps < 0");
    // an earlier resident launch on this device that lost a wait is reported
    // here, before anything builds on its state
    if ((st = resident_report()) != PRC_OK) return st;
    int64_t k = 0;
    const int tile = tile_choice(*p);
    if (tile == kResidentTile && (st = resident_prepare(stream)) != PRC_OK) return st;
    // Long runs replay a captured graph of graph_steps() steps (a multiple of
    // four, so the newest state is back in f_a after every replay whether the
    // shape takes one or two steps per launch).  Not while the caller's stream
    // is itself being captured.
    const int gsteps = graph_steps();
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cap));
    const int capturing = cap == hipStreamCaptureStatusNone ? 0 : 1;
    // timed calls: the events bracket the call's work on the stream; for the
    // resident sweep with kernel_only its dispatch records them (the
    // kernel's own start and end), otherwise start is a marker ahead of the
    // launch and the last dispatch records stop (ahead of the launch's own
    // ordering event)
    if (tile == kResidentTile && nsteps > 0) {
        if (kernel_only) return run_steps(*p, tile, f_a, f_b, 0, nsteps, stream, capturing, start, stop);
        if (start) HIP_TRY(hipEventRecord(start, stream));
        return run_steps(*p, tile, f_a, f_b, 0, nsteps, stream, capturing, nullptr, nullptr, stop);
    }
    if (start) HIP_TRY(hipEventRecord(start, stream));
    // (the resident sweep takes any number of steps in one launch: no graph)
    if (tile != kResidentTile && gsteps > 0 && !capturing && nsteps >= 2 * gsteps) {
        std::shared_ptr<GraphEntry> g;  // held while replaying
        if ((st = get_graph(*p, tile, f_a, f_b, gsteps, &g)) != PRC_OK) return st;
        for (; k + gsteps <= nsteps; k += gsteps) HIP_TRY(hipGraphLaunch(g->exec, stream));
    }
    st = run_steps(*p, tile, f_a, f_b, k, nsteps - k, stream, capturing);
    if (st == PRC_OK && stop) HIP_TRY(hipEventRecord(stop, stream));
    return st;
}

prc_status prc_residual(const prc_params *p, const void *f, double *u_prev, void *scratch,
                        double out[4], hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if ((st = check_buf(f, "f")) != PRC_OK) return st;
    if (!u_prev || !scratch || !out) return fail(PRC_EINVAL, "NULL u_prev, scratch or out");
    return residual_into(*p, f, u_prev, (double *)scratch, out, stream);
}

prc_status prc_residual_noalloc(const prc_params *p, const void *f, double *u_prev,
                                double out[4], hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if ((st = check_buf(f, "f")) != PRC_OK) return st;
    if (!u_prev || !out) return fail(PRC_EINVAL, "NULL u_prev or out");
    if (prc_scratch_bytes(p) > sizeof(scratch))
        return fail(PRC_EINVAL, "the check needs %zu bytes of scratch, more than the %zu of the "
                                "static array", prc_scratch_bytes(p), sizeof(scratch));
    double *sc = nullptr;
    if ((st = static_scratch(&sc)) != PRC_OK) return st;
    return residual_into(*p, f, u_prev, sc, out, stream);
}

prc_status prc_convert(const prc_params *p, const void *f, int32_t storage_to, void *f_to,
                       hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    prc_params q = *p;
    q.storage = storage_to;
    if ((st = validate(&q)) != PRC_OK) return st;
    if ((st = check_buf(f, "f")) != PRC_OK || (st = check_buf(f_to, "f_to")) != PRC_OK) return st;
    if (f == f_to) return fail(PRC_EINVAL, "f and f_to must be distinct buffers");
    switch (p->storage) {
    case PRC_F64: return launch_convert<double>(*p, f, q, f_to, stream);
    case PRC_F32: return launch_convert<float>(*p, f, q, f_to, stream);
    case PRC_F16: return launch_convert<__half>(*p, f, q, f_to, stream);
    case PRC_BF16: return launch_convert<__hip_bfloat16>(*p, f, q, f_to, stream);
    }
    return fail(PRC_EINVAL, "bad storage %d", p->storage);
}

prc_status prc_add_density(const prc_params *p, void *f, double drho, hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if ((st = check_buf(f, "f")) != PRC_OK) return st;
    if (!std::isfinite(drho)) return fail(PRC_EINVAL, "drho must be finite");
    return PRC_DISPATCH(*p, launch_add_rest, *p, f, drho, stream);
}

prc_status prc_macros(const prc_params *p, const void *f, double *rho, double *ux, double *uy,
                      hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if ((st = check_buf(f, "f")) != PRC_OK) return st;
    if ((st = resident_report()) != PRC_OK) return st;
    return PRC_DISPATCH(*p, launch_macros, *p, f, rho, ux, uy, stream);
}

prc_status prc_solve(const prc_params *p, void *f_a, void *f_b, double *u_prev, void *scratch,
                     double tol, int64_t check_every, int64_t max_steps, int64_t *steps_out,
                     double *hist, int64_t hist_cap, int64_t *hist_len, hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if (check_every <= 0 || max_steps < 0 || !steps_out)
        return fail(PRC_EINVAL, "need check_every > 0, max_steps >= 0, steps_out");
    if (!(tol >= 0.0)) return fail(PRC_EINVAL, "tol must be >= 0");
    double out[4];
    // snapshot of the initial velocity
    if ((st = prc_residual(p, f_a, u_prev, scratch, out, stream)) != PRC_OK) return st;
    int64_t n = 0, nh = 0;
    prc_status result = PRC_NOT_CONVERGED;
    while (n + check_every <= max_steps) {
        void *cur = (n & 1) ? f_b : f_a, *oth = (n & 1) ? f_a : f_b;
        if ((st = prc_step(p, cur, oth, check_every, stream)) != PRC_OK) return st;
        n += check_every;
        void *now = (n & 1) ? f_b : f_a;
        if ((st = prc_residual(p, now, u_prev, scratch, out, stream)) != PRC_OK) return st;
        // a NaN in either sum makes R non-finite (diverged), never 0
        const double R = out[1] > 0.0 ? std::sqrt(out[0] / out[1])
                                      : (out[1] == 0.0 && out[0] == 0.0 ? 0.0 : INFINITY);
        if (hist && nh < hist_cap) hist[nh] = R;
        ++nh;
        if (!std::isfinite(R) || !std::isfinite(out[2]) || !(out[3] < 1.0)) {
            result = (prc_status)fail(PRC_EDIVERGED, "diverged at step %lld (R=%g, max|u|^2=%g)",
                                      (long long)n, R, out[3]);
            break;
        }
        if (R < tol) {
            result = PRC_OK;
            break;
        }
    }
    if (result == PRC_NOT_CONVERGED && n < max_steps) {
        void *cur = (n & 1) ? f_b : f_a, *oth = (n & 1) ? f_a : f_b;
        if ((st = prc_step(p, cur, oth, max_steps - n, stream)) != PRC_OK) return st;
        n = max_steps;
        HIP_TRY(hipStreamSynchronize(stream));
        if ((st = resident_report()) != PRC_OK) return st;
    }
    *steps_out = n;
    if (hist_len) *hist_len = nh;
    return result;
}

prc_status prc_tune(const prc_params *p, int32_t *tile_out, hipStream_t stream)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    constexpr int kWarm = 4, kTimed = 20;
    const size_t bytes = prc_state_bytes(p);
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = -1;
    float best_ms = 0.0f;
    hipError_t he = hipMalloc(&a, bytes);
    if (he == hipSuccess) he = hipMalloc(&b, bytes);
    if (he == hipSuccess) he = hipMemsetAsync(a, 0, bytes, stream);
    if (he == hipSuccess) he = hipMemsetAsync(b, 0, bytes, stream);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    for (int t = 0; t < kNumTiles && he == hipSuccess && st == PRC_OK; ++t) {
        if (!tile_allowed(*p, t)) continue;
        if (t == kResidentTile && resident_prepare(stream) != PRC_OK) continue;
        for (int k = 0; k < kWarm + kTimed && st == PRC_OK; ++k) {
            if (k == kWarm) he = hipEventRecord(e0, stream);
            st = PRC_DISPATCH(*p, launch_sweep_tile, *p, t, (k & 1) ? b : a, (k & 1) ? a : b,
                              stream);
        }
        if (st != PRC_OK || he != hipSuccess) break;
        he = hipEventRecord(e1, stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        // a resident launch that lost a wait does not count
        if (he == hipSuccess && t == kResidentTile && resident_report() != PRC_OK) continue;
        ms /= (float)(t == kResidentTile ? kResidentTuneSteps : kTiles[t].steps);  // per step
        if (he == hipSuccess && (best < 0 || ms < best_ms)) {
            best = t;
            best_ms = ms;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (st != PRC_OK) return st;
    if (he != hipSuccess) return fail(PRC_EHIP, "prc_tune: %s", hipGetErrorString(he));
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[tune_key(*p)] = best;
    }
    if (tile_out) *tile_out = best;
    return PRC_OK;
}

prc_status prc_tile_info(int32_t tile, int32_t *tx, int32_t *ty, int32_t *steps)
{
    if (tile < 0 || tile >= kNumTiles) return fail(PRC_EINVAL, "tile %d out of range", tile);
    if (tx) *tx = kTiles[tile].tx;
    if (ty) *ty = kTiles[tile].ty;
    if (steps) *steps = kTiles[tile].steps;
    return PRC_OK;
}

prc_status prc_set_tile(const prc_params *p, int32_t tile)
{
    prc_status st = validate(p);
    if (st != PRC_OK) return st;
    if (tile < -1 || (tile >= 0 && !tile_allowed(*p, tile)))
        return fail(PRC_EINVAL, "tile %d out of range", tile);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (tile < 0)
        g_tuned.erase(tune_key(*p));
    else
        g_tuned[tune_key(*p)] = tile;
    return PRC_OK;
}

prc_status prc_release_graphs(void)
{
    decltype(g_graphs) old;  // destroyed (after their devices finish) outside the lock
    {
        std::lock_guard<std::mutex> lock(g_graph_mu);
        old.swap(g_graphs);
    }
    old.clear();
    return PRC_OK;
}

prc_status prc_release_resident(void) { return resident_release(); }

prc_status prc_resident_status(void) { return resident_report(); }

prc_status prc_set_resident_wait(int64_t ticks) { return resident_set_wait(ticks); }

prc_status prc_set_streamed(int32_t mode)
{
    if (mode < -1 || mode > 1) return fail(PRC_EINVAL, "streamed mode %d not in {-1, 0, 1}", mode);
    g_streamed_mode.store(mode, std::memory_order_relaxed);
    return PRC_OK;
}

const char *prc_last_error(void) { return err_slot().c_str(); }

}  // extern "C"
