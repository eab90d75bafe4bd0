// FP64 reductions of the convergence check (shared by the single-grid and
// the batched entry points, so that both sum in the same order).
#pragma once

#include "prc_device.hpp"
#include "prc_host.hpp"

namespace prc {

// block-wide fixed-order sum of four doubles (and a max in slot 3)
__device__ __forceinline__ void block_reduce4(double v[4], double *sh /* [4][kRedBlock] */)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k * kRedBlock + t] = v[k];
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sh[k * kRedBlock + t] += sh[k * kRedBlock + t + s];
            const double a = sh[3 * kRedBlock + t], b = sh[3 * kRedBlock + t + s];
            sh[3 * kRedBlock + t] = (a >= b || a != a) ? a : b;  // NaN sticks
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = sh[k * kRedBlock];
}

// Partial sums of the convergence check over the nodes n = b * kRedBlock + t,
// b * kRedBlock + t + nb * kRedBlock, ... of state f (block b of nb), written
// to part[0..3]; u_prev is updated at the same nodes.
template <typename ST, int BC>
__device__ __forceinline__ void residual_block(const ST *__restrict__ f,
                                               const Coef<typename Mem<ST>::CT> &c,
                                               double *__restrict__ u_prev, int b, int nb,
                                               double *__restrict__ part, double *sh)
{
    using CT = typename Mem<ST>::CT;
    const int64_t N = (int64_t)c.nx * c.ny;
    const rsrc_t rs = make_rsrc(f, c.state_bytes);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t n = (int64_t)b * kRedBlock + threadIdx.x; n < N; n += (int64_t)nb * kRedBlock) {
        const int x = (int)(n % c.nx), y = (int)(n / c.nx);
        CT d[9];
        pull_checked<ST, BC>(c, rs, x, y, d);
        CT drho, u, v;
        fields(c, d, drho, u, v);
        const double du = (double)u - u_prev[n], dv = (double)v - u_prev[N + n];
        const double u2 = (double)u * (double)u + (double)v * (double)v;
        acc[0] += du * du + dv * dv;
        acc[1] += u2;
        acc[2] += (double)drho;
        if (!(u2 <= acc[3])) acc[3] = u2;
        u_prev[n] = (double)u;
        u_prev[N + n] = (double)v;
    }
    block_reduce4(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) part[k] = acc[k];
    }
}

// Fixed-order total of nblocks partial sums (4 doubles each) into out[0..3].
__device__ __forceinline__ void finish_block(const double *__restrict__ partial, int nblocks,
                                             double *__restrict__ out, double *sh)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kRedBlock) {
        for (int k = 0; k < 3; ++k) acc[k] += partial[4 * b + k];
        const double m = partial[4 * b + 3];
        if (!(m <= acc[3])) acc[3] = m;
    }
    block_reduce4(acc, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) out[k] = acc[k];
}

template <typename ST, int BC>
__global__ void __launch_bounds__(kRedBlock)
    k_residual(const ST *__restrict__ f, const Coef<typename Mem<ST>::CT> c,
               double *__restrict__ u_prev, double *__restrict__ partial)
{
    __shared__ double sh[4 * kRedBlock];
    residual_block<ST, BC>(f, c, u_prev, blockIdx.x, gridDim.x, partial + 4 * blockIdx.x, sh);
}

// (a template only so that each source file may hold its own instance)
template <int Unused = 0>
__global__ void __launch_bounds__(kRedBlock)
    k_finish(const double *__restrict__ partial, int nblocks, double *__restrict__ out)
{
    __shared__ double sh[4 * kRedBlock];
    finish_block(partial, nblocks, out, sh);
}

}  // namespace prc
