// Two time steps per launch (temporal blocking).
//
// A single step per launch moves the whole state through memory every step
// (HBM, or the last-level cache for a small state), and a launch over a
// cache-resident grid is one wave of workgroups whose loads, collisions and
// stores hardly overlap.  Here a
// workgroup produces its tile two steps ahead from the state three rings
// further out, keeping the intermediate step in LDS:
//
//   region R3 = tile + 3 rings: streamed step-1 populations, step-1 densities
//   region R2 = tile + 2 rings: step-1 collisions, post-collision state in LDS
//   region R1 = tile + 1 ring : step-2 streaming out of LDS, step-2 densities
//   tile                      : step-2 collision, stored to the output state
//
// (the density gradient needs the neighbours' densities at the same step, so
// each step needs one ring more than streaming alone).  Every node passes
// through exactly the functions of the single-step sweep, in the same order
// and with the intermediate state rounded to the storage type as a stored
// state would be, so two steps here give the bits of two single steps.
//
// Slots of the rings that fall outside the grid stand in for the node they
// map to: across a wall the clamped node (the density-gradient reading at
// walls), across a periodic side the wrapped node.
#pragma once

#include "prc_collide.hpp"
#include "prc_device.hpp"
#include "prc_sweep.hpp"

namespace prc {

// Population a of LDS-resident state: element type of the storage, so that
// the intermediate step is rounded exactly as a stored state.
template <typename ST> struct LdsVal;
template <> struct LdsVal<double> {
    static __device__ __forceinline__ double put(double x) { return x; }
    static __device__ __forceinline__ double get(double x) { return x; }
};
template <> struct LdsVal<float> {
    static __device__ __forceinline__ float put(float x) { return x; }
    static __device__ __forceinline__ float get(float x) { return x; }
};
template <> struct LdsVal<__half> {
    static __device__ __forceinline__ __half put(float x) { return __float2half_rn(as_computed(x)); }
    static __device__ __forceinline__ float get(__half x) { return __half2float(x); }
};
template <> struct LdsVal<__hip_bfloat16> {
    static __device__ __forceinline__ __hip_bfloat16 put(float x)
    {
        return __float2bfloat16(as_computed(x));
    }
    static __device__ __forceinline__ float get(__hip_bfloat16 x) { return __bfloat162float(x); }
};

template <int TX, int TY>
struct Regions2 {
    static constexpr int T = TX * TY;
    static constexpr int W3 = TX + 6, H3 = TY + 6, N3 = W3 * H3;
    static constexpr int W2 = TX + 4, H2 = TY + 4, N2 = W2 * H2;
    static constexpr int NB = N3 - N2;             // ring 3 alone
    static constexpr int S2 = (N2 + T - 1) / T;    // R2 slots per thread
    static constexpr int SB = (NB + T - 1) / T;    // ring-3 slots per thread
};

// Tile-relative position of ring-3 slot k (top row, bottom row, left column,
// right column).
template <int TX, int TY>
__device__ __forceinline__ void ring3_pos(int k, int &i, int &j)
{
    constexpr int W3 = TX + 6, H2 = TY + 4;
    if (k < W3) { i = k - 3; j = -3; }
    else if (k < 2 * W3) { i = k - W3 - 3; j = TY + 2; }
    else if (k < 2 * W3 + H2) { i = -3; j = k - 2 * W3 - 2; }
    else { i = TX + 2; j = k - 2 * W3 - H2 - 2; }
}

// Streaming out of the LDS-resident state P (planes [9][H2][W2], tile-relative
// origin at index (2, 2)) for node (x, y) of the grid whose slot is (hi, hj):
// the same boundary rules as pull_checked.
template <typename ST, int BC, int TX, int TY>
__device__ __forceinline__ void pull_lds(const Coef<typename Mem<ST>::CT> &c,
                                         const ST (*P)[TY + 4][TX + 4], int x, int y, int hi,
                                         int hj, typename Mem<ST>::CT d[9])
{
    using CT = typename Mem<ST>::CT;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const int sx = x - EX[a], sy = y - EY[a];
        bool out = false;
        if (!Bc<BC>::wrap_x) out |= (sx < 0) | (sx >= c.nx);
        if (!Bc<BC>::wrap_y) out |= (sy < 0) | (sy >= c.ny);
        if (!out) {
            d[a] = LdsVal<ST>::get(P[a][hj - EY[a] + 2][hi - EX[a] + 2]);
        } else {
            CT v = LdsVal<ST>::get(P[OPP[a]][hj + 2][hi + 2]);
            if (Bc<BC>::lid && LIDC[a] != 0 && sy >= c.ny) v += CT(LIDC[a]) * c.lid;
            d[a] = v;
        }
    }
}

// The same for a slot whose sources all lie inside the grid (PW: the row
// length of the LDS array, TX + 4 or more).
template <typename ST, int TX, int TY, int PW = TX + 4>
__device__ __forceinline__ void pull_lds_inner(const ST (*P)[TY + 4][PW], int hi, int hj,
                                               typename Mem<ST>::CT d[9])
{
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = LdsVal<ST>::get(P[a][hj - EY[a] + 2][hi - EX[a] + 2]);
}

// Node of the grid that slot (i, j) of the tile at (x0, y0) stands for, and
// the slot whose LDS data that node's streaming reads: across a wall the
// clamped node and its own slot, across a periodic side the wrapped node and
// the slot itself (which holds the wrapped node's data).
template <int BC>
__device__ __forceinline__ void slot_node(const int nx, const int ny, int x0, int y0, int i,
                                          int j, int &x, int &y, int &hi, int &hj)
{
    x = x0 + i;
    y = y0 + j;
    fix_coord<BC>(x, y, nx, ny);
    hi = Bc<BC>::wrap_x ? i : x - x0;
    hj = Bc<BC>::wrap_y ? j : y - y0;
}

// Two steps for the tile at (x0, y0) of one problem: src (state at step n) ->
// dst (state at step n + 2).  Called by the whole workgroup.  STREAMED: the
// state is streamed from HBM (it does not stay in the last-level cache from
// one launch to the next), which changes only the order of the first loads.
template <typename ST, int BC, int TX, int TY, bool FORCE, bool ALL, bool STREAMED>
__device__ __forceinline__ void sweep2_tile(const Coef<typename Mem<ST>::CT> &c,
                                            const void *src, void *dst, int x0, int y0)
{
    using CT = typename Mem<ST>::CT;
    using R = Regions2<TX, TY>;
    __shared__ CT D1[R::H3][R::W3];        // step-1 densities, origin (3, 3)
    __shared__ ST P1[9][R::H2][R::W2];     // step-1 post-collision state, origin (2, 2)
    __shared__ CT D2[TY + 2][TX + 2];      // step-2 densities, origin (1, 1)

    const int t = threadIdx.x;
    constexpr uint32_t E = sizeof(ST);
    const rsrc_t rs = make_rsrc(src, c.state_bytes);
    // every source of every slot of R3 lies inside the grid
    const bool inner = x0 >= 4 && y0 >= 4 && x0 + TX + 4 <= c.nx && y0 + TY + 4 <= c.ny;
    auto load1 = [&](int i, int j, CT d[9]) {
        if (inner) {
            pull_inner<ST>(c, rs, (uint32_t)(y0 + j) * c.row_bytes + (uint32_t)(x0 + i - 1) * E, d);
        } else {
            int x = x0 + i, y = y0 + j;
            fix_coord<BC>(x, y, c.nx, c.ny);
            pull_checked_ld<ST, BC>(c, rs, x, y, d);
        }
    };
    auto finish1 = [&](int i, int j, CT d[9]) {  // lid term, density
        if (!inner) {
            int x = x0 + i, y = y0 + j;
            fix_coord<BC>(x, y, c.nx, c.ny);
            add_lid<BC>(c, y, d);
        }
        D1[j + 3][i + 3] = sum9(d);
    };

    // step 1: streaming and densities over R3; the R2 populations are kept
    // for the collision.  Workgroups of up to 512 threads, and every
    // workgroup of a state streamed from HBM, issue every load of the region
    // before the first use; 1024-thread workgroups over a state in the
    // last-level cache load the ring only after the densities of R2, which
    // measured faster for them there (and slower in the other cases).  The
    // streamed instance keeps both orders behind the run-time flag c.nt
    // (set for such states): compiled that way it measured 5 % faster than
    // with the eager order alone (4096 x 2048 FP32 on 32 x 32 tiles: 72.9
    // against 79.2 us per step), a difference in instruction scheduling only.
    CT keep[R::S2][9];
    bool eager;
    if constexpr (R::T <= 512) eager = true;
    else if constexpr (STREAMED) eager = c.nt;
    else eager = false;
    if (eager) {
        CT ring[R::SB][9];
#pragma unroll
        for (int s = 0; s < R::SB; ++s) {
            const int k = t + s * R::T;
            if (k < R::NB) {
                int i, j;
                ring3_pos<TX, TY>(k, i, j);
                load1(i, j, ring[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < R::S2; ++s) {
            const int k = t + s * R::T;
            if (k < R::N2) load1(k % R::W2 - 2, k / R::W2 - 2, keep[s]);
        }
#pragma unroll
        for (int s = 0; s < R::SB; ++s) {
            const int k = t + s * R::T;
            if (k < R::NB) {
                int i, j;
                ring3_pos<TX, TY>(k, i, j);
                finish1(i, j, ring[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < R::S2; ++s) {
            const int k = t + s * R::T;
            if (k < R::N2) finish1(k % R::W2 - 2, k / R::W2 - 2, keep[s]);
        }
    } else {
#pragma unroll
        for (int s = 0; s < R::S2; ++s) {
            const int k = t + s * R::T;
            if (k < R::N2) load1(k % R::W2 - 2, k / R::W2 - 2, keep[s]);
        }
#pragma unroll
        for (int s = 0; s < R::S2; ++s) {
            const int k = t + s * R::T;
            if (k < R::N2) finish1(k % R::W2 - 2, k / R::W2 - 2, keep[s]);
        }
#pragma unroll
        for (int s = 0; s < R::SB; ++s) {
            const int k = t + s * R::T;
            if (k < R::NB) {
                int i, j;
                ring3_pos<TX, TY>(k, i, j);
                CT d[9];
                load1(i, j, d);
                finish1(i, j, d);
            }
        }
    }
    __syncthreads();

    // step 1: collisions over R2 into LDS
#pragma unroll
    for (int s = 0; s < R::S2; ++s) {
        const int k = t + s * R::T;
        if (k < R::N2) {
            const int i = k % R::W2 - 2, j = k / R::W2 - 2;
            CT gx, gy;
            density_gradient(c, D1, i + 3, j + 3, gx, gy);
            collide_node<CT, FORCE, ALL>(c, keep[s], gx, gy);
#pragma unroll
            for (int a = 0; a < 9; ++a) P1[a][j + 2][i + 2] = LdsVal<ST>::put(keep[s][a]);
        }
    }
    __syncthreads();

    // step 2: streaming out of LDS over R1 (this thread's tile node, and its
    // ring node if any), densities
    const TileGeom<TX, TY> g(t);
    CT d[9];
    // every source of every slot of R1 lies inside the grid
    const bool inner2 = x0 >= 2 && y0 >= 2 && x0 + TX + 2 <= c.nx && y0 + TY + 2 <= c.ny;
    if (inner2) {
        CT e[9];
        pull_lds_inner<ST, TX, TY>(P1, g.tx, g.ty, d);
        if (g.ring) pull_lds_inner<ST, TX, TY>(P1, g.hx, g.hy, e);
        D2[g.ty + 1][g.tx + 1] = sum9(d);
        if (g.ring) D2[g.hy + 1][g.hx + 1] = sum9(e);
    } else {
        {
            int x, y, hi, hj;
            slot_node<BC>(c.nx, c.ny, x0, y0, g.tx, g.ty, x, y, hi, hj);
            pull_lds<ST, BC, TX, TY>(c, P1, x, y, hi, hj, d);
            D2[g.ty + 1][g.tx + 1] = sum9(d);
        }
        if (g.ring) {
            int x, y, hi, hj;
            slot_node<BC>(c.nx, c.ny, x0, y0, g.hx, g.hy, x, y, hi, hj);
            CT e[9];
            pull_lds<ST, BC, TX, TY>(c, P1, x, y, hi, hj, e);
            D2[g.hy + 1][g.hx + 1] = sum9(e);
        }
    }
    __syncthreads();

    // step 2: collision of the tile, stored
    tile_finish<ST, TX, TY, FORCE, ALL>(c, make_rsrc(dst, c.state_bytes), D2, g, x0, y0, d);
}

// Waves per SIMD that the LDS of sweep2_tile leaves room for (160 KB per CU,
// four SIMDs, at most eight waves each considered): the kernels ask the
// compiler to fit their registers to it, so that the general variant, whose
// collision needs a few more registers, keeps the occupancy the LDS allows.
template <typename ST, int TX, int TY>
constexpr int two_step_waves_per_simd()
{
    using CT = typename Mem<ST>::CT;
    using R = Regions2<TX, TY>;
    constexpr int lds = int(sizeof(CT)) * R::H3 * R::W3 + int(sizeof(ST)) * 9 * R::H2 * R::W2 +
                        int(sizeof(CT)) * (TY + 2) * (TX + 2);
    constexpr int w = (163840 / lds) * (R::T / 64) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// One problem, one tile per workgroup, XCD-aware order as k_sweep.
template <typename ST, int BC, int TX, int TY, bool FORCE, bool ALL, bool STREAMED>
__global__ void __launch_bounds__(TX *TY)
    __attribute__((amdgpu_waves_per_eu(two_step_waves_per_simd<ST, TX, TY>())))
    k_sweep2(const ST *__restrict__ src, ST *__restrict__ dst, const Coef<typename Mem<ST>::CT> c)
{
    const int tile = (blockIdx.x % kXcds) * c.tiles_per_xcd + blockIdx.x / kXcds;
    if (tile >= c.tiles_x * c.tiles_y) return;
    const int x0 = (tile % c.tiles_x) * TX, y0 = (tile / c.tiles_x) * TY;
    sweep2_tile<ST, BC, TX, TY, FORCE, ALL, STREAMED>(c, src, dst, x0, y0);
}

// A tile list over many problems (batches), as k_sweep_batch: two steps from
// buf[parity] into buf[parity ^ 1].  STREAMED as for k_sweep2 (the instance
// keeps both load orders behind the members' run-time flag, so either
// instance gives the same bits).
template <typename ST, int BC, int TX, int TY, bool FORCE, bool ALL, bool STREAMED>
__global__ void __launch_bounds__(TX *TY)
    __attribute__((amdgpu_waves_per_eu(two_step_waves_per_simd<ST, TX, TY>())))
    k_sweep_batch2(const BatchTile *__restrict__ tiles, int ntiles, int tiles_per_xcd,
                   const BatchMember<typename Mem<ST>::CT> *__restrict__ members, int parity)
{
    const int t = (blockIdx.x % kXcds) * tiles_per_xcd + blockIdx.x / kXcds;
    if (t >= ntiles) return;
    const BatchTile tl = tiles[t];
    const BatchMember<typename Mem<ST>::CT> &m = members[tl.member];
    sweep2_tile<ST, BC, TX, TY, FORCE, ALL, STREAMED>(m.c, m.buf[parity],
                                                      const_cast<void *>(m.buf[parity ^ 1]), tl.x0,
                                                      tl.y0);
}

}  // namespace prc
