// Sweep kernels: one fused PRC-LBM time step over a grid of tiles.
//
// A tile is TX x TY nodes, one node per thread.  Each thread streams its node
// (pull with boundaries); the first RING threads also stream one node of the
// one-node ring around the tile, because the density gradient at a node needs
// the streamed densities of its eight neighbours at the same time level.  The
// densities go to an LDS tile, one barrier, then each thread computes the
// gradient, collides and stores its node.
//
// k_sweep        one tile per workgroup (the grid covers all tiles once)
// k_sweep_batch  the same over a list of tiles of many independent problems
#pragma once

#include "prc_collide.hpp"
#include "prc_device.hpp"

namespace prc {

template <int TX, int TY>
struct TileGeom {
    static constexpr int RING = 2 * (TX + 2) + 2 * TY;
    static_assert(TX * TY >= RING, "one ring node per thread at most");
    int tx, ty;   // this thread's node in the tile
    int hx, hy;   // this thread's ring node (tile-relative), if ring
    bool ring;

    __device__ __forceinline__ explicit TileGeom(int tid)
    {
        tx = tid % TX;
        ty = tid / TX;
        ring = tid < RING;
        if (tid < TX + 2) { hx = tid - 1; hy = -1; }
        else if (tid < 2 * (TX + 2)) { hx = tid - (TX + 2) - 1; hy = TY; }
        else if (tid < 2 * (TX + 2) + TY) { hx = -1; hy = tid - 2 * (TX + 2); }
        else { hx = TX; hy = tid - 2 * (TX + 2) - TY; }
    }
};

// Issue the loads of this thread's node and ring node of the tile at (x0, y0).
template <typename ST, int BC, int TX, int TY>
__device__ __forceinline__ void tile_load(const Coef<typename Mem<ST>::CT> &c, rsrc_t rs,
                                          const TileGeom<TX, TY> &g, int x0, int y0,
                                          typename Mem<ST>::CT d[9],
                                          typename Mem<ST>::CT e[9])
{
    constexpr uint32_t E = sizeof(ST);
    // every source of every node of the tile and of its ring lies inside the
    // grid: no boundary logic needed
    const bool inner = x0 >= 2 && y0 >= 2 && x0 + TX + 2 <= c.nx && y0 + TY + 2 <= c.ny;
    int x = x0 + g.tx, y = y0 + g.ty, rx = x0 + g.hx, ry = y0 + g.hy;
    if (inner) {
        pull_inner<ST>(c, rs, (uint32_t)y * c.row_bytes + (uint32_t)(x - 1) * E, d);
        if (g.ring) pull_inner<ST>(c, rs, (uint32_t)ry * c.row_bytes + (uint32_t)(rx - 1) * E, e);
    } else {
        fix_coord<BC>(x, y, c.nx, c.ny);  // slots beyond the grid stand in for their image
        fix_coord<BC>(rx, ry, c.nx, c.ny);
        pull_checked_ld<ST, BC>(c, rs, x, y, d);
        if (g.ring) pull_checked_ld<ST, BC>(c, rs, rx, ry, e);
        add_lid<BC>(c, y, d);
        if (g.ring) add_lid<BC>(c, ry, e);
    }
}

template <typename CT, int TX, int TY>
__device__ __forceinline__ void tile_densities(CT (*srho)[TX + 2], const TileGeom<TX, TY> &g,
                                               const CT d[9], const CT e[9])
{
    srho[g.ty + 1][g.tx + 1] = sum9(d);
    if (g.ring) srho[g.hy + 1][g.hx + 1] = sum9(e);
}

// Density gradient at LDS position (lx, ly) of a density tile: rest-weighted
// central differences over the eight neighbours (exact for linear rho; the
// [4,1,1]/12 stencil at r = 1).
template <typename CT, int W>
__device__ __forceinline__ void density_gradient(const Coef<CT> &c, const CT (*D)[W], int lx,
                                                 int ly, CT &gx, CT &gy)
{
    const CT rE = D[ly][lx + 1], rW = D[ly][lx - 1];
    const CT rN = D[ly + 1][lx], rS = D[ly - 1][lx];
    const CT rNE = D[ly + 1][lx + 1], rNW = D[ly + 1][lx - 1];
    const CT rSE = D[ly - 1][lx + 1], rSW = D[ly - 1][lx - 1];
    gx = c.gxa * (rE - rW) + c.gxb * ((rNE - rNW) + (rSE - rSW));
    gy = c.gya * (rN - rS) + c.gyb * ((rNE + rNW) - (rSE + rSW));
}

// The collision of one node: the specialised update of the method as the
// paper runs it, or in the general instance the frame read at run time.
template <typename CT, bool FORCE, bool ALL>
__device__ __forceinline__ void collide_node(const Coef<CT> &c, CT d[9], CT gx, CT gy)
{
    if constexpr (ALL) {
        static_assert(!FORCE, "the method as published has no body force");
        collide_plain<CT>(c, d, gx, gy);
    } else {
        if (c.frame == PRC_FRAME_RAW)
            collide_raw<CT, FORCE>(c, d, gx, gy);
        else
            collide<CT, FORCE>(c, d, gx, gy);
    }
}

// Density gradient, collision and store of this thread's node (after the
// barrier that publishes the LDS densities).
template <typename ST, int TX, int TY, bool FORCE, bool ALL>
__device__ __forceinline__ void tile_finish(const Coef<typename Mem<ST>::CT> &c, rsrc_t rd,
                                            const typename Mem<ST>::CT (*srho)[TX + 2],
                                            const TileGeom<TX, TY> &g, int x0, int y0,
                                            typename Mem<ST>::CT d[9])
{
    using CT = typename Mem<ST>::CT;
    constexpr uint32_t E = sizeof(ST);
    const int x = x0 + g.tx, y = y0 + g.ty;
    if (x >= c.nx || y >= c.ny) return;
    CT gx, gy;
    density_gradient(c, srho, g.tx + 1, g.ty + 1, gx, gy);
    collide_node<CT, FORCE, ALL>(c, d, gx, gy);

    const uint32_t o = (uint32_t)y * c.row_bytes + (uint32_t)x * E;
    if (c.nt) {
#pragma unroll
        for (int a = 0; a < 9; ++a) Mem<ST>::template st<kNt>(rd, o, a * c.plane_bytes, d[a]);
    } else {
#pragma unroll
        for (int a = 0; a < 9; ++a) Mem<ST>::st(rd, o, a * c.plane_bytes, d[a]);
    }
}

// XCD-aware tile order: the hardware hands workgroup i to XCD i mod 8.  Each
// XCD owns one contiguous band of tiles (tiles_per_xcd of them, row-major),
// so the density halo a tile shares with the tiles above and below is read
// through the same L2.
template <typename ST, int BC, int TX, int TY, bool FORCE, bool ALL>
__global__ void __launch_bounds__(TX *TY)
    k_sweep(const ST *__restrict__ src, ST *__restrict__ dst, const Coef<typename Mem<ST>::CT> c)
{
    using CT = typename Mem<ST>::CT;
    __shared__ CT srho[TY + 2][TX + 2];
    const int tile = (blockIdx.x % kXcds) * c.tiles_per_xcd + blockIdx.x / kXcds;
    if (tile >= c.tiles_x * c.tiles_y) return;
    const int x0 = (tile % c.tiles_x) * TX, y0 = (tile / c.tiles_x) * TY;
    const TileGeom<TX, TY> g(threadIdx.x);
    CT d[9], e[9];
    tile_load<ST, BC>(c, make_rsrc(src, c.state_bytes), g, x0, y0, d, e);
    tile_densities<CT>(srho, g, d, e);
    __syncthreads();
    tile_finish<ST, TX, TY, FORCE, ALL>(c, make_rsrc(dst, c.state_bytes), srho, g, x0, y0, d);
}

// ---- batches ---------------------------------------------------------------
// One member of a batch: its per-launch constants and its two state buffers.
template <typename CT>
struct BatchMember {
    Coef<CT> c;
    const void *buf[2];  // buf[parity] is read, buf[parity ^ 1] written
    double *u_prev;      // velocity snapshot of the convergence check
};

// One tile of a member: its top-left node.
struct BatchTile {
    int32_t member, x0, y0, pad;
};

// One sweep over the tiles of many members.  The tile list is ordered member
// by member; workgroup i runs on XCD i mod 8 and the list is split into eight
// contiguous bands, so each member's tiles (and the halos they share) stay
// within one or two XCDs' L2.  Member constants are read through the scalar
// cache (the member index is uniform over the workgroup).
template <typename ST, int BC, int TX, int TY, bool FORCE, bool ALL>
__global__ void __launch_bounds__(TX *TY)
    k_sweep_batch(const BatchTile *__restrict__ tiles, int ntiles, int tiles_per_xcd,
                  const BatchMember<typename Mem<ST>::CT> *__restrict__ members, int parity)
{
    using CT = typename Mem<ST>::CT;
    __shared__ CT srho[TY + 2][TX + 2];
    const int t = (blockIdx.x % kXcds) * tiles_per_xcd + blockIdx.x / kXcds;
    if (t >= ntiles) return;
    const BatchTile tl = tiles[t];
    const BatchMember<CT> &m = members[tl.member];
    const Coef<CT> &c = m.c;
    const TileGeom<TX, TY> g(threadIdx.x);
    CT d[9], e[9];
    tile_load<ST, BC>(c, make_rsrc(m.buf[parity], c.state_bytes), g, tl.x0, tl.y0, d, e);
    tile_densities<CT>(srho, g, d, e);
    __syncthreads();
    tile_finish<ST, TX, TY, FORCE, ALL>(c, make_rsrc(m.buf[parity ^ 1], c.state_bytes), srho, g,
                                        tl.x0, tl.y0, d);
}

}  // namespace prc
