// Device building blocks of the PRC-LBM sweep for gfx950: state access,
// streaming with boundaries, hydrodynamic fields.  The collision itself is in
// prc_collide.hpp.
//
// Populations are held as deviations d = f - rho0 w from the rest state
// (w: product of the one-dimensional rest weights of variance c_s^2 along x
// and c_s^2/r^2 along y, in lattice units of each axis).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "prc_coef.hpp"

namespace prc {

// Velocity set of Sec. 2 (e_y in units of r) and its opposite directions.
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// Lid term of an incoming population bounced at the top wall, in units of
// Coef::lid: f_7 = f~_5 - lid, f_8 = f~_6 + lid, f_4 = f~_2.
constexpr int LIDC[9] = {0, 0, 0, 0, 0, 0, 0, -1, 1};
// Position of population a in the 3 x 3 velocity grid [e_y + 1][e_x + 1].
constexpr int QI[9] = {1, 2, 1, 0, 1, 2, 0, 0, 2};
constexpr int QJ[9] = {1, 1, 2, 1, 0, 2, 2, 0, 0};

// ---- buffer access --------------------------------------------------------
// All state accesses go through raw buffer instructions: one resource for the
// whole state, the plane offset as a scalar (uniform) offset and the node's
// byte offset in a vector register, so that the nine loads of a node share
// three address registers (one per source row) plus immediate offsets.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data (gfx9 family)
// Cache policy bits of buffer accesses: kNt marks a non-temporal (streaming)
// access.  The sweeps store non-temporally when the two state buffers do not
// fit the last-level cache (the new state is read by the next sweep only,
// after every other line of this one has been written); a state that fits is
// stored normally so that the next sweep finds it in the cache.
constexpr int kNt = 2;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

// x as computed, for a conversion to a 16-bit type: the empty register
// constraint keeps the compiler from fusing the conversion into the
// multiply-add that produced x (one rounding of the exact result to 16 bits,
// v_fma_mixlo_f16), which it does or not depending on the shape of the code
// around it; so every kernel rounds twice, to float and then to 16 bits, as
// the source says, and kernels of different shape give the same bits.
__device__ __forceinline__ float as_computed(float x)
{
    asm("" : "+v"(x));
    return x;
}

template <typename ST> struct Mem;
template <> struct Mem<double> {
    using CT = double;
    template <int POL = 0>
    static __device__ __forceinline__ double ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, POL));
    }
    template <int POL = 0>
    static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, double x)
    {
        using v2u = __attribute__((ext_vector_type(2))) unsigned int;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, x), r, v, s, POL);
    }
};
template <> struct Mem<float> {
    using CT = float;
    template <int POL = 0>
    static __device__ __forceinline__ float ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, POL));
    }
    template <int POL = 0>
    static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, float x)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, v, s, POL);
    }
};
template <> struct Mem<__half> {
    using CT = float;
    template <int POL = 0>
    static __device__ __forceinline__ float ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return __half2float(
            __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, POL)));
    }
    template <int POL = 0>
    static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, float x)
    {
        __builtin_amdgcn_raw_buffer_store_b16(
            __builtin_bit_cast(unsigned short, __float2half_rn(as_computed(x))), r, v, s, POL);
    }
};
template <> struct Mem<__hip_bfloat16> {
    using CT = float;
    template <int POL = 0>
    static __device__ __forceinline__ float ld(rsrc_t r, uint32_t v, uint32_t s)
    {
        return __bfloat162float(__builtin_bit_cast(
            __hip_bfloat16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, POL)));
    }
    template <int POL = 0>
    static __device__ __forceinline__ void st(rsrc_t r, uint32_t v, uint32_t s, float x)
    {
        __builtin_amdgcn_raw_buffer_store_b16(
            __builtin_bit_cast(unsigned short, __float2bfloat16(as_computed(x))), r, v, s, POL);
    }
};

// reciprocal: the hardware estimate (1 ulp) in single precision, a correctly
// rounded division in double precision
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// ---- boundary traits -----------------------------------------------------
template <int BC> struct Bc {
    static constexpr bool wrap_x = BC != PRC_BC_CAVITY;
    static constexpr bool wrap_y = BC == PRC_BC_PERIODIC;
    static constexpr bool lid = BC != PRC_BC_PERIODIC;
};

// one period of wrap-around: v in [-n, 2n)
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// any v
__device__ __forceinline__ int wrap_any(int v, int n) { const int m = v % n; return m < 0 ? m + n : m; }
__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Coordinates of the node whose density stands in for (x, y) in the density
// gradient stencil: periodic directions wrap, walls clamp to the nearest node
// inside the domain.  Also maps tile slots beyond the grid (ragged edges, and
// grids narrower than a tile) onto real nodes.
template <int BC>
__device__ __forceinline__ void fix_coord(int &x, int &y, int nx, int ny)
{
    x = Bc<BC>::wrap_x ? wrap_any(x, nx) : clampi(x, nx);
    y = Bc<BC>::wrap_y ? wrap_any(y, ny) : clampi(y, ny);
}

// Streaming (Appendix A, "stream"): d_a(x) = d~_a(x - e_a), for a node whose
// nine sources all lie inside the grid.  rw = byte offset of (x - 1, y).
template <typename ST>
__device__ __forceinline__ void pull_inner(const Coef<typename Mem<ST>::CT> &c, rsrc_t rs,
                                           uint32_t rw, typename Mem<ST>::CT d[9])
{
    constexpr uint32_t E = sizeof(ST);
    const uint32_t rS = rw - c.row_bytes, rN = rw + c.row_bytes;  // rows y - 1, y + 1
    const uint32_t pb = c.plane_bytes;
    d[0] = Mem<ST>::ld(rs, rw + E, 0);
    d[1] = Mem<ST>::ld(rs, rw, pb);                 // from (x-1, y)
    d[2] = Mem<ST>::ld(rs, rS + E, 2 * pb);         // from (x, y-1)
    d[3] = Mem<ST>::ld(rs, rw + 2 * E, 3 * pb);     // from (x+1, y)
    d[4] = Mem<ST>::ld(rs, rN + E, 4 * pb);         // from (x, y+1)
    d[5] = Mem<ST>::ld(rs, rS, 5 * pb);             // from (x-1, y-1)
    d[6] = Mem<ST>::ld(rs, rS + 2 * E, 6 * pb);     // from (x+1, y-1)
    d[7] = Mem<ST>::ld(rs, rN + 2 * E, 7 * pb);     // from (x+1, y+1)
    d[8] = Mem<ST>::ld(rs, rN, 8 * pb);             // from (x-1, y+1)
}

// Streaming with boundaries for any node (x, y) of the grid, loads only.  A
// source outside a wall means half-way bounce-back: the population that left
// this node along opp(a) returns along a.  A source above the top row also
// crosses the lid, whose momentum term add_lid() adds once the loads are in
// flight (a use of a loaded value right after its load would make the next
// node's loads wait for it).
template <typename ST, int BC>
__device__ __forceinline__ void pull_checked_ld(const Coef<typename Mem<ST>::CT> &c, rsrc_t rs,
                                                int x, int y, typename Mem<ST>::CT d[9])
{
    constexpr uint32_t E = sizeof(ST);
    const uint32_t own = (uint32_t)y * c.row_bytes + (uint32_t)x * E;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        int sx = x - EX[a], sy = y - EY[a];
        bool out = false;
        if (Bc<BC>::wrap_x) sx = wrap(sx, c.nx);
        else out |= (sx < 0) | (sx >= c.nx);
        if (Bc<BC>::wrap_y) sy = wrap(sy, c.ny);
        else out |= (sy < 0) | (sy >= c.ny);
        // the whole offset in the vector register (a per-lane choice of the
        // scalar plane offset would make the compiler loop over its values)
        const uint32_t off = out ? own + OPP[a] * c.plane_bytes
                                 : (uint32_t)sy * c.row_bytes + (uint32_t)sx * E + a * c.plane_bytes;
        d[a] = Mem<ST>::ld(rs, off, 0);
    }
}

// Lid term of the populations a node of row y streamed across the top wall:
// the two diagonal ones of the top row (f_7 = f~_5 - lid, f_8 = f~_6 + lid;
// f_4 = f~_2 takes none), the top corners included.
template <int BC, typename CT>
__device__ __forceinline__ void add_lid(const Coef<CT> &c, int y, CT d[9])
{
    if (Bc<BC>::lid) {
        const bool top = y >= c.ny - 1;
        d[7] = top ? d[7] + CT(LIDC[7]) * c.lid : d[7];
        d[8] = top ? d[8] + CT(LIDC[8]) * c.lid : d[8];
    }
}

template <typename ST, int BC>
__device__ __forceinline__ void pull_checked(const Coef<typename Mem<ST>::CT> &c, rsrc_t rs,
                                             int x, int y, typename Mem<ST>::CT d[9])
{
    pull_checked_ld<ST, BC>(c, rs, x, y, d);
    add_lid<BC>(c, y, d);
}

// Sum of the nine populations, row by row of the velocity set (e_y = -1, 0,
// +1) and within a row the two moving ones first: the same operations as the
// density inside the collision, so that a thread that needs both computes it
// once.
template <typename CT>
__device__ __forceinline__ CT sum9(const CT d[9])
{
    return (((d[8] + d[7]) + d[4]) + ((d[1] + d[3]) + d[0])) + ((d[5] + d[6]) + d[2]);
}

// Hydrodynamic fields of streamed deviations (eq. hydrodynamicfields):
// rho = rho0 + sum d, rho u = sum d e + F / (2 gamma) (the rest state carries
// no momentum).
template <typename CT>
__device__ __forceinline__ void fields(const Coef<CT> &c, const CT d[9], CT &drho, CT &ux,
                                       CT &uy)
{
    drho = sum9(d);
    const CT jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    const CT jy = ((d[2] - d[4]) + (d[5] - d[8]) + (d[6] - d[7])) * c.r;
    const CT irho = CT(1) / (c.rho0 + drho);
    ux = (jx + c.fxh) * irho;
    uy = (jy + c.fyh) * irho;
}


}  // namespace prc
