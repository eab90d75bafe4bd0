// Resident sweep: many time steps per launch, the state held in LDS.
//
// A grid whose state fits the chip's LDS (256 CUs x 160 KB) is cut into
// subdomains of 64 x 32 nodes, one per workgroup and one workgroup per CU.
// Each workgroup keeps the post-collision state of its subdomain and of the
// two rings around it in LDS and advances it step after step; per step only
// the two outer rows and columns of each subdomain cross memory, to the
// neighbouring workgroups.  Streaming, densities, the density gradient and
// the collision are the functions of the single-step sweep, in the same
// order, with the state rounded to the storage type between steps, so the
// result is bitwise that of single steps.
//
// Exchange through memory: after step s a subdomain stores its two outer
// rows and columns into an exchange buffer of its own (parity s mod 2), laid
// out as row blocks [9][2][SX] and column blocks [9][SY][2] so that each
// neighbour reads its part as a few contiguous lines; the last step of a
// launch stores the whole subdomain into the output state instead.  Every
// exchanged value travels with the step that produced it, in one 8-byte
// store (value bits, step tag), stored and loaded at agent scope (through to
// the memory side of the XCDs' L2 caches, which are not coherent with each
// other).  A neighbour loads the values it needs and loads again those whose
// tag is not yet the step it waits for: no flag, no wait for the stores to
// complete, no whole-cache write-back or invalidation.  Two parities
// suffice: a subdomain overwrites its edges of step s - 2 only after it has
// read its neighbours' edges of step s - 1, which they stored after reading
// those of step s - 2.
//
// Every workgroup of the launch must be resident at once: one per CU (the
// LDS of a subdomain leaves no room for a second), at most as many
// subdomains as CUs.  Waits are bounded: a value that does not arrive within
// about half a second (a workgroup that never got a CU) sets an abort word
// that ends every other wait of the launch, and a word in host memory that
// the host reads without synchronising; the launch's last workgroup clears
// the abort word, so the next launch starts clean.
#pragma once

#include "prc_sweep2.hpp"

namespace prc {

constexpr int kResidentSX = 64, kResidentSY = 32;  // subdomain, nodes
constexpr int kResidentThreads = 1024;              // two nodes per thread
constexpr int kResidentMaxGroups = 512;
constexpr uint64_t kResidentWaitTicks = 1ull << 26;  // default wait: ~0.67 s of the 100 MHz clock
// Step tags are 32-bit: the step counter restarts from zero (and the exchange
// buffer is cleared) before it reaches this.
constexpr uint64_t kResidentStepLimit = 1ull << 31;
// Exchange buffer of one subdomain and parity, in (value, tag) pairs: row
// blocks (bottom rows 0-1, top rows SY-2, SY-1) of [9][2][SX], then column
// blocks (left columns 0-1, right columns SX-2, SX-1) of [9][SY][2].
constexpr int kXchRowPlane = 2 * kResidentSX, kXchColPlane = 2 * kResidentSY;
constexpr int kXchBot = 0, kXchTop = 9 * kXchRowPlane, kXchLeft = 18 * kXchRowPlane,
              kXchRight = kXchLeft + 9 * kXchColPlane;
constexpr int kXchElems = kXchRight + 9 * kXchColPlane;
constexpr uint32_t kXchPair = 8;  // bytes per exchanged value
// Row lengths of the LDS state (elements) and density (words) arrays: 32
// banks of 4 bytes, the inner nodes in rows of SX - 4 = 60; a row length of
// 60 + 32 k words (FP32 state, densities) or 60 + 64 k elements (16-bit
// state) puts consecutive inner nodes on consecutive banks
template <typename ST> constexpr int kResidentRowP = sizeof(ST) == 4 ? 92 : 124;
constexpr int kResidentRowD = 92;
// cache policy of the exchanged values: agent scope (sc1)
constexpr int kAgent = 16;

// Counters of the resident sweep, one block per device, zeroed once.
struct ResidentSync {
    uint64_t step;   // steps run by earlier resident launches: the tags' base
    uint64_t done;   // workgroups finished in the current launch
    uint64_t abort;  // a wait of the current launch timed out (cleared by its last workgroup)
};

__device__ __forceinline__ uint64_t ld_agent(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// bits of a stored value and back
template <typename ST>
__device__ __forceinline__ uint32_t value_bits(ST v)
{
    if constexpr (sizeof(ST) == 4) return __builtin_bit_cast(uint32_t, v);
    else return (uint32_t)__builtin_bit_cast(uint16_t, v);
}
template <typename ST>
__device__ __forceinline__ ST bits_value(uint32_t b)
{
    if constexpr (sizeof(ST) == 4) return __builtin_bit_cast(ST, b);
    else return __builtin_bit_cast(ST, (uint16_t)b);
}

using pair_t = __attribute__((ext_vector_type(2))) unsigned int;

// Subdomain-relative position of slot k of the two rings around an SX x SY
// subdomain: two top rows, two bottom rows, two left columns, two right
// columns (4 (SX + 4) + 4 SY slots).
template <int SX, int SY>
__device__ __forceinline__ void halo_pos(int k, int &i, int &j)
{
    constexpr int W2 = SX + 4;
    if (k < 2 * W2) { i = k % W2 - 2; j = k / W2 - 2; }
    else if (k < 4 * W2) { k -= 2 * W2; i = k % W2 - 2; j = SY + k / W2; }
    else if (k < 4 * W2 + 2 * SY) { k -= 4 * W2; i = k / SY - 2; j = k % SY; }
    else { k -= 4 * W2 + 2 * SY; i = SX + k / SY; j = k % SY; }
}

// Subdomain-relative position of edge node k (the nodes within one of the
// subdomain's boundary: two bottom rows, two top rows, then the two left and
// two right columns between them, four nodes of one row after another, so
// that the lanes of a wave fall on different LDS banks; 4 SX + 4 (SY - 4)
// nodes).
template <int SX, int SY>
__device__ __forceinline__ void edge_pos(int k, int &i, int &j)
{
    if (k < 2 * SX) { i = k % SX; j = k / SX; }
    else if (k < 4 * SX) { k -= 2 * SX; i = k % SX; j = SY - 2 + k / SX; }
    else { k -= 4 * SX; const int q = k % 4; i = q < 2 ? q : SX - 4 + q; j = 2 + k / 4; }
}

// Half-way bounce-back through ghost slots: for the in-grid slot (i, j)
// whose post-collision populations are v, every population a whose source
// (i, j) - e_a lies beyond a wall gets, in that source slot, the value
// streaming along a must deliver there: the population that left (i, j)
// along opp(a).  Each ghost value has exactly one such slot, and the pull out
// of LDS then needs no boundary test (the lid term is added afterwards, as in
// pull_checked).
template <typename ST, int BC, int SX, int SY, int PW, typename CT>
__device__ __forceinline__ void reflect(const Coef<CT> &c, ST (*P)[SY + 4][PW], int x0, int y0,
                                        int i, int j, const ST *v)
{
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const int sx = x0 + i - EX[a], sy = y0 + j - EY[a];
        bool out = false;
        if (!Bc<BC>::wrap_x) out |= (sx < 0) | (sx >= c.nx);
        if (!Bc<BC>::wrap_y) out |= (sy < 0) | (sy >= c.ny);
        if (out) P[a][j - EY[a] + 2][i - EX[a] + 2] = v[OPP[a]];
    }
}

// The populations that stream to grid node (x, y) from beyond a wall (x or
// y next to a side that does not wrap): bit a set when (x, y) - e_a lies
// beyond one.  Only nodes with some bit set have ghost slots to fill.
template <int BC>
__device__ __forceinline__ uint32_t wall_dirs(int nx, int ny, int x, int y)
{
    uint32_t m = 0;
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const int sx = x - EX[a], sy = y - EY[a];
        bool out = false;
        if (!Bc<BC>::wrap_x) out |= (sx < 0) | (sx >= nx);
        if (!Bc<BC>::wrap_y) out |= (sy < 0) | (sy >= ny);
        m |= out ? 1u << a : 0u;
    }
    return m;
}

// The ghost slots of slot (i, j) whose directions beyond a wall are `dirs`
// (wall_dirs), as reflect above, without branches: a direction not in dirs
// writes its value into `dump` instead, a slot of the lane's own that nothing
// reads.  dirs is tested here, in the time loop, not kept as lane masks
// across it.
template <typename ST, int SX, int SY, int PW>
__device__ __forceinline__ void reflect_dirs(ST (*P)[SY + 4][PW], ST *dump, int i, int j,
                                             uint32_t dirs, const ST *v)
{
    asm volatile("" : "+v"(dirs));
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        ST *dst = ((dirs >> a) & 1u) ? &P[a][j - EY[a] + 2][i - EX[a] + 2] : dump;
        *dst = v[OPP[a]];
    }
}

// One subdomain per workgroup, two nodes per thread.  Each thread owns one
// node at least two nodes from the subdomain's boundary (an inner node) and
// a second node that collides early for threads below L0 (another inner
// node) and late for the others (the edge nodes, and inner nodes for the
// rest of them).  The late half is waves 8-15, two on each SIMD, so every
// SIMD collides six waves' nodes early and two late.  Per step:
//   X  streaming and densities of the nodes whose sources are the
//      subdomain's own (every node but the outermost ring)
//   Y  the neighbours' edges of the previous step are loaded (in flight)
//      while the inner nodes collide; then the edges go into the two rings
//      of LDS
//   Z  streaming and densities of the outermost ring and of the ring around
//      the subdomain
//   W  the late nodes collide; the new state goes into LDS, the edges into
//      the exchange blocks.
template <typename ST, int BC, bool FORCE, bool ALL>
__global__ void __launch_bounds__(kResidentThreads)
    k_resident(ST *__restrict__ buf0, ST *__restrict__ buf1, void *__restrict__ xch,
               const Coef<typename Mem<ST>::CT> c, ResidentSync *__restrict__ sy,
               uint64_t *__restrict__ mailbox, uint64_t wait_ticks, int nsteps)
{
    using CT = typename Mem<ST>::CT;
    constexpr int SX = kResidentSX, SY = kResidentSY, T = kResidentThreads;
    constexpr int W2 = SX + 4, H2 = SY + 4, N2 = W2 * H2;
    // row lengths of the LDS arrays: consecutive inner nodes (rows of IW)
    // stay on consecutive LDS banks across a row's end, where their slots
    // lie PW - IW + 1 elements (DW - IW + 1 words) apart, one element more
    // than a whole number of 128-byte bank rounds
    constexpr int PW = kResidentRowP<ST>, DW = kResidentRowD;
    constexpr int HALO = 4 * W2 + 4 * SY;
    constexpr int FILL = (N2 + T - 1) / T;
    constexpr int IW = SX - 4, NI = (SX - 4) * (SY - 4);  // nodes two or more from the boundary
    constexpr int L0 = T / 2;                              // first thread whose second node is late
    constexpr int NE = 4 * SX + 4 * (SY - 4);              // edge nodes
    constexpr int LI = T - L0 - NE;                        // late inner nodes
    constexpr uint32_t E = sizeof(ST);
    static_assert(NI + NE == 2 * T && LI >= 0 && HALO <= T, "subdomain shape");
    __shared__ ST P[9][H2][PW];        // post-collision state, origin (2, 2)
    __shared__ CT D[SY + 2][DW];       // densities, origin (1, 1)
    __shared__ ST dump[64];           // writes of reflect_dirs that go nowhere
    __shared__ uint64_t s_base;
    __shared__ uint32_t s_abort, s_last;

    const int ntiles = c.tiles_x * c.tiles_y;
    const int sub = (blockIdx.x % kXcds) * c.tiles_per_xcd + blockIdx.x / kXcds;
    if (sub >= ntiles) return;
    const int sxi = sub % c.tiles_x, syi = sub / c.tiles_x;
    const int x0 = sxi * SX, y0 = syi * SY;
    const int t = threadIdx.x;
    // every source of every slot of the subdomain and its ring lies inside
    // the grid (no wall, no lid, no ghost slot)
    const bool inner = x0 >= 2 && y0 >= 2 && x0 + SX + 2 <= c.nx && y0 + SY + 2 <= c.ny;
    auto in_grid = [&](int i, int j) {
        const int x = x0 + i, y = y0 + j;
        return (Bc<BC>::wrap_x || (x >= 0 && x < c.nx)) && (Bc<BC>::wrap_y || (y >= 0 && y < c.ny));
    };

    // the input state into P (every slot that stands for a node of the grid)
    if (t == 0) {
        s_base = ld_agent(&sy->step);
        s_abort = 0;
    }
    // (the loads first; this thread's set-up below overlaps their latency)
    CT v[FILL][9];
    bool ok[FILL];
    {
        const rsrc_t rs = make_rsrc(buf0, c.state_bytes);
        uint32_t o[FILL];
#pragma unroll
        for (int m = 0; m < FILL; ++m) {
            const int k = t + m * T, i = k % W2 - 2, j = k / W2 - 2;
            ok[m] = k < N2 && in_grid(i, j);
            if (ok[m]) {
                int x = x0 + i, y = y0 + j;
                if (Bc<BC>::wrap_x) x = wrap_any(x, c.nx);
                if (Bc<BC>::wrap_y) y = wrap_any(y, c.ny);
                o[m] = (uint32_t)y * c.row_bytes + (uint32_t)x * E;
#pragma unroll
                for (int a = 0; a < 9; ++a) v[m][a] = Mem<ST>::ld(rs, o[m], a * c.plane_bytes);
            }
        }
    }

    // this thread's two nodes (si, sj), whether each is in the grid, the
    // slot its streaming reads around (the clamped node for a node beyond a
    // wall), that node's row (lid), and whether its sources are all the
    // subdomain's own
    int si[2], sj[2], hx[2], hy[2], ly[2];
    bool act[2], own[2];
    uint32_t wdir[2];  // wall_dirs of each node (0 beside no wall, or not in the grid)
    si[0] = 2 + t % IW;
    sj[0] = 2 + t / IW;
    if (t < L0 + LI) {  // inner nodes T .. NI - 1
        si[1] = 2 + (t + T) % IW;
        sj[1] = 2 + (t + T) / IW;
    } else {
        edge_pos<SX, SY>(t - L0 - LI, si[1], sj[1]);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        int x, y;
        slot_node<BC>(c.nx, c.ny, x0, y0, si[m], sj[m], x, y, hx[m], hy[m]);
        ly[m] = y;
        act[m] = x0 + si[m] < c.nx && y0 + sj[m] < c.ny;
        own[m] = hx[m] >= 1 && hx[m] <= SX - 2 && hy[m] >= 1 && hy[m] <= SY - 2;
        wdir[m] = act[m] ? wall_dirs<BC>(c.nx, c.ny, x0 + si[m], y0 + sj[m]) : 0u;
    }
    // the ring slot of this thread (threads below 2 (SX + 2) + 2 SY)
    const TileGeom<SX, SY> g(t);
    int rhx = 0, rhy = 0, rly = 0;
    if (g.ring) {
        int x;
        slot_node<BC>(c.nx, c.ny, x0, y0, g.hx, g.hy, x, rly, rhx, rhy);
    }
    // this thread's slot of the two rings, and where its neighbour keeps it
    int qi = 0, qj = 0, qsub = 0;
    bool qv = false;
    uint32_t qo = 0, qstride = 0;
    if (t < HALO) {
        halo_pos<SX, SY>(t, qi, qj);
        qv = in_grid(qi, qj);
        const int dx = qi < 0 ? -1 : (qi >= SX ? 1 : 0);
        const int dy = qj < 0 ? -1 : (qj >= SY ? 1 : 0);
        qsub = wrap(syi + dy, c.tiles_y) * c.tiles_x + wrap(sxi + dx, c.tiles_x);
        if (dy != 0) {  // the neighbour's top rows (below us) or bottom rows (above)
            const int col = qi - dx * SX;
            qo = dy < 0 ? kXchTop + (qj + 2) * SX + col : kXchBot + (qj - SY) * SX + col;
            qstride = kXchRowPlane * kXchPair;
        } else {        // its right columns (left of us) or left columns (right)
            qo = dx < 0 ? kXchRight + 2 * qj + (qi + 2) : kXchLeft + 2 * qj + (qi - SX);
            qstride = kXchColPlane * kXchPair;
        }
    }
    const bool qring1 = qv && qi >= -1 && qi <= SX && qj >= -1 && qj <= SY;
    const uint32_t qdir = qring1 ? wall_dirs<BC>(c.nx, c.ny, x0 + qi, y0 + qj) : 0u;

    // the loaded state into LDS
    {
#pragma unroll
        for (int m = 0; m < FILL; ++m) {
            const int k = t + m * T;
            if (ok[m]) {
#pragma unroll
                for (int a = 0; a < 9; ++a) P[a][k / W2][k % W2] = LdsVal<ST>::put(v[m][a]);
            }
        }
    }
    __syncthreads();
    const uint64_t base = s_base;

    // ghost slots of the input state: every in-grid slot that streaming reads
    // from (own nodes, ring slots) reflects into the walls
    if (!inner) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (wdir[m] != 0) {
                ST v[9];
#pragma unroll
                for (int a = 0; a < 9; ++a) v[a] = P[a][sj[m] + 2][si[m] + 2];
                reflect<ST, BC, SX, SY, PW>(c, P, x0, y0, si[m], sj[m], v);
            }
        }
        if (g.ring && in_grid(g.hx, g.hy) && wall_dirs<BC>(c.nx, c.ny, x0 + g.hx, y0 + g.hy) != 0) {
            ST v[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = P[a][g.hy + 2][g.hx + 2];
            reflect<ST, BC, SX, SY, PW>(c, P, x0, y0, g.hx, g.hy, v);
        }
        __syncthreads();
    }

    const rsrc_t rx = make_rsrc(xch, (uint32_t)(2 * ntiles * kXchElems) * kXchPair);
    auto pull = [&](int hi, int hj, int y, CT d[9]) {
        pull_lds_inner<ST, SX, SY, PW>(P, hi, hj, d);
        if (!inner) add_lid<BC>(c, y, d);
    };
    auto collide_at = [&](int i, int j, CT d[9]) {
        CT gx, gy;
        density_gradient(c, D, i + 1, j + 1, gx, gy);
        collide_node<CT, FORCE, ALL>(c, d, gx, gy);
    };
    CT d[2][9];
    for (int s = 1; s <= nsteps; ++s) {
        const bool last = s == nsteps;

        // X: streaming and densities of the nodes with own sources
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (own[m]) {
                pull(hx[m], hy[m], ly[m], d[m]);
                D[sj[m] + 1][si[m] + 1] = sum9(d[m]);
            }
        }
        __syncthreads();

        // Y: the neighbours' edges of step s - 1 in flight while the inner
        // nodes collide; values whose tag is not that step yet are loaded
        // again (bounded wait)
        const bool load = s > 1 && qv;
        const uint32_t want = (uint32_t)(base + (uint64_t)(s - 1));
        const uint32_t qaddr = (uint32_t)((((s - 1) & 1) * ntiles + qsub) * kXchElems + qo) * kXchPair;
        pair_t h[9];
        if (load) {
#pragma unroll
            for (int a = 0; a < 9; ++a)
                h[a] = __builtin_amdgcn_raw_buffer_load_b64(rx, qaddr + a * qstride, 0, kAgent);
        }
        if (act[0]) collide_at(si[0], sj[0], d[0]);
        if (t < L0 && act[1]) collide_at(si[1], sj[1], d[1]);
        if (load) {
            uint32_t miss = 0;
#pragma unroll
            for (int a = 0; a < 9; ++a) miss |= (h[a].y != want) ? 1u << a : 0u;
            if (miss) {
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                while (miss) {
                    if (ld_agent(&sy->abort) != 0) {
                        s_abort = 1;
                        break;
                    }
                    if (__builtin_amdgcn_s_memrealtime() - t0 > wait_ticks) {
                        st_agent(&sy->abort, 1);
                        // host-visible report (pinned host memory, system scope)
                        __hip_atomic_store(mailbox, (uint64_t)1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        s_abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
#pragma unroll
                    for (int a = 0; a < 9; ++a)
                        if (miss & (1u << a))
                            h[a] = __builtin_amdgcn_raw_buffer_load_b64(rx, qaddr + a * qstride, 0,
                                                                        kAgent);
#pragma unroll
                    for (int a = 0; a < 9; ++a)
                        if (h[a].y == want) miss &= ~(1u << a);
                }
            }
            ST v[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = bits_value<ST>(h[a].x);
#pragma unroll
            for (int a = 0; a < 9; ++a) P[a][qj + 2][qi + 2] = v[a];
            if (!inner && qdir != 0) reflect_dirs<ST, SX, SY, PW>(P, &dump[t % 64], qi, qj, qdir, v);
        }
        __syncthreads();
        if (s_abort != 0) break;

        // Z: streaming and densities of the outermost ring and the ring around
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (!own[m]) {
                pull(hx[m], hy[m], ly[m], d[m]);
                D[sj[m] + 1][si[m] + 1] = sum9(d[m]);
            }
        }
        if (g.ring) {
            CT e[9];
            pull(rhx, rhy, rly, e);
            D[g.hy + 1][g.hx + 1] = sum9(e);
        }
        __syncthreads();

        // W: the late nodes collide; the new state into LDS (and its ghost
        // slots), the edges into the exchange blocks tagged with this step;
        // at the last step every node into the output state instead.  A late
        // thread stores its edge node's values for the neighbours, who wait
        // for them, before anything else goes into LDS.
        const uint32_t xb = (uint32_t)(((s & 1) * ntiles + sub) * kXchElems) * kXchPair;
        const uint32_t tag = (uint32_t)(base + (uint64_t)s);
        auto put = [&](int m, const ST *v) {
            const int i = si[m], j = sj[m];
            if (last) {
                const rsrc_t ro = make_rsrc((s & 1) ? buf1 : buf0, c.state_bytes);
                const uint32_t o = (uint32_t)(y0 + j) * c.row_bytes + (uint32_t)(x0 + i) * E;
#pragma unroll
                for (int a = 0; a < 9; ++a) Mem<ST>::st(ro, o, a * c.plane_bytes, d[m][a]);
                return;
            }
#pragma unroll
            for (int a = 0; a < 9; ++a) P[a][j + 2][i + 2] = v[a];
            if (!inner && wdir[m] != 0) reflect_dirs<ST, SX, SY, PW>(P, &dump[t % 64], i, j, wdir[m], v);
        };
        auto put_node = [&](int m) {
            ST v[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = LdsVal<ST>::put(d[m][a]);
            put(m, v);
        };
        if (t < L0) {  // both nodes collided in Y
            if (act[0]) put_node(0);
            if (act[1]) put_node(1);
        } else {
            // the late waves are the phase's critical path: their
            // instructions go first wherever the early waves' LDS writes
            // compete with them (measured 1 % faster per step)
            __builtin_amdgcn_s_setprio(3);
            if (act[1]) {
                collide_at(si[1], sj[1], d[1]);
                const int i = si[1], j = sj[1];
                ST v[9];
#pragma unroll
                for (int a = 0; a < 9; ++a) v[a] = LdsVal<ST>::put(d[1][a]);
                if (!last && t >= L0 + LI) {
                    if (j < 2 || j >= SY - 2) {  // a row block
                        const uint32_t o =
                            xb + (uint32_t)((j < 2 ? kXchBot + j * SX : kXchTop + (j - SY + 2) * SX) + i) *
                                     kXchPair;
#pragma unroll
                        for (int a = 0; a < 9; ++a)
                            __builtin_amdgcn_raw_buffer_store_b64(pair_t{value_bits<ST>(v[a]), tag}, rx, o,
                                                                  a * kXchRowPlane * kXchPair, kAgent);
                    }
                    if (i < 2 || i >= SX - 2) {  // a column block
                        const uint32_t o = xb + (uint32_t)((i < 2 ? kXchLeft + i : kXchRight + i - SX + 2) +
                                                           2 * j) * kXchPair;
#pragma unroll
                        for (int a = 0; a < 9; ++a)
                            __builtin_amdgcn_raw_buffer_store_b64(pair_t{value_bits<ST>(v[a]), tag}, rx, o,
                                                                  a * kXchColPlane * kXchPair, kAgent);
                    }
                }
                put(1, v);
            }
            if (act[0]) put_node(0);
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
    }

    // The last workgroup to finish advances the tags' base for the next
    // launch and clears the abort word (no wait of this launch is left);
    // near the end of the 32-bit tags it clears the exchange buffer (no other
    // workgroup of this launch touches it any more) and restarts the count,
    // so no old tag can match a new step.
    if (t == 0) {
        const uint64_t old =
            __hip_atomic_fetch_add(&sy->done, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = old == (uint64_t)ntiles - 1;
    }
    __syncthreads();
    if (s_last) {
        const uint64_t next = base + (uint64_t)nsteps;
        if (next >= kResidentStepLimit) {
            const uint32_t bytes = (uint32_t)(2 * kResidentMaxGroups * kXchElems) * kXchPair;
            const rsrc_t rz = make_rsrc(xch, bytes);
            for (uint32_t o = (uint32_t)t * 16u; o < bytes; o += T * 16u)
                __builtin_amdgcn_raw_buffer_store_b128(
                    (__attribute__((ext_vector_type(4))) unsigned int){0u, 0u, 0u, 0u}, rz, o, 0, 0);
        }
        if (t == 0) {
            st_agent(&sy->done, 0);
            st_agent(&sy->abort, 0);
            st_agent(&sy->step, next >= kResidentStepLimit ? 0 : next);
        }
    }
}

}  // namespace prc
