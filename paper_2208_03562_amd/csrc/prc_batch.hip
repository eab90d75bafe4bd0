// Batches of independent PRC-LBM problems advanced by shared launches.
//
// Kernels:
//   k_sweep_batch     one time step over the tile list of every member
//                     (prc_sweep.hpp; the per-tile code is that of k_sweep)
//   k_residual_batch  per-block FP64 partial sums of the convergence check of
//                     many members, with each member split into exactly the
//                     blocks prc_residual would use for it
//   k_finish_batch    per-member fixed-order total of those partial sums
// Because every member runs the single-problem code paths with the same
// constants and the same reduction order, its results are bit for bit those
// of the problem run alone.  The ABI is declared in include/prc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "prc.h"
#include "prc_batch.hpp"
#include "prc_coef.hpp"
#include "prc_device.hpp"
#include "prc_host.hpp"
#include "prc_reduce.hpp"
#include "prc_sweep.hpp"
#include "prc_sweep2.hpp"

namespace prc {

// block b (of nb) of the check of member `member`; partial sums at slot part + b
struct ResItem {
    int32_t member, b, nb, part;
};
// total of nb partial sums from slot part into out slot `out`
struct FinItem {
    int32_t part, nb, out, pad;
};

template <typename ST, int BC>
__global__ void __launch_bounds__(kRedBlock)
    k_residual_batch(const ResItem *__restrict__ items,
                     const BatchMember<typename Mem<ST>::CT> *__restrict__ members,
                     double *__restrict__ partial)
{
    __shared__ double sh[4 * kRedBlock];
    const ResItem it = items[blockIdx.x];
    const BatchMember<typename Mem<ST>::CT> &m = members[it.member];
    residual_block<ST, BC>((const ST *)m.buf[0], m.c, m.u_prev, it.b, it.nb,
                           partial + 4 * (it.part + it.b), sh);
}

template <int Unused = 0>
__global__ void __launch_bounds__(kRedBlock)
    k_finish_batch(const FinItem *__restrict__ items, const double *__restrict__ partial,
                   double *__restrict__ out)
{
    __shared__ double sh[4 * kRedBlock];
    const FinItem it = items[blockIdx.x];
    finish_block(partial + 4 * it.part, it.nb, out + 4 * it.out, sh);
}

// Device buffer that grows on demand (the batch's own tables).
struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
    prc_status ensure(size_t bytes)
    {
        if (bytes <= cap) return PRC_OK;
        size_t n = std::max<size_t>(bytes + bytes / 2, 4096);
        if (ptr) HIP_TRY(hipFree(ptr));
        ptr = nullptr;
        cap = 0;
        HIP_TRY(hipMalloc(&ptr, n));
        cap = n;
        return PRC_OK;
    }
    void release()
    {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
};

// Sweep variants, as for the single-problem sweep: the method as the paper
// runs it, and everything else.
inline int variant_of(const prc_params &p) { return is_plain_method(p) ? 0 : 1; }

struct Member {
    prc_params p;
    void *fa, *fb;
    double *up;
    int32_t status;  // prc_member_status
    bool fresh;      // no velocity snapshot taken yet
    int64_t steps;   // since the member joined
    double R;        // relative residual of its last check
};

}  // namespace prc

using namespace prc;

struct prc_batch {
    int32_t storage, bc;
    int tile = -1;       // -1: default shape
    int auto_tile = 6;   // the default shape for the current tables
    std::vector<Member> mem;
    std::vector<int32_t> active;  // ids of active members, ascending; slot = index
    bool dirty = true;            // tables do not match `active` / `tile`
    // device tables of the active members
    DevBuf d_members, d_tiles[2], d_res, d_fin, d_partial, d_out;
    int ntiles[2] = {0, 0};
    // host copies (kept alive until the uploads that read them have completed)
    std::vector<char> h_members;
    std::vector<BatchTile> h_tiles[2];
    std::vector<ResItem> h_res;
    std::vector<FinItem> h_fin;
    std::vector<double> h_out;
    // launch graph of graph_steps() sweeps of the current tables
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
    int calls_since_rebuild = 0;  // step calls served by the current tables
};

namespace prc {

static int batch_tile(const prc_batch &b)
{
    return b.tile >= 0 ? b.tile : b.auto_tile;
}

// The default shape, measured on MI355X for batches of 64..512-wide
// cavities: two steps per launch halve the state traffic; 32 x 16 tiles
// waste few threads at ragged edges, and once the members' states together
// are streamed from HBM the 64 x 16 shape's instance for such states is
// faster still (256 such cavities, 0.9 GB: 104,700 against 101,000 MLUPS in
// the sweep).  FP64 keeps 32 x 16 (twice the LDS per tile).
static int default_batch_tile(int storage, int64_t pair_bytes)
{
    return storage != PRC_F64 && pair_bytes > kNtPairBytes ? 7 : 6;
}

static void drop_graph(prc_batch &b)
{
    if (b.gexec) (void)hipGraphExecDestroy(b.gexec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.gexec = nullptr;
    b.graph = nullptr;
    b.gsteps = 0;
}

// Rebuild and upload the member table, the tile lists of both variants and
// the residual lists for the active members.
template <typename ST, int BC>
static prc_status build_tables(prc_batch &b, hipStream_t s)
{
    using CT = typename Mem<ST>::CT;
    HIP_TRY(hipStreamSynchronize(s));  // earlier work may still read the tables
    drop_graph(b);
    const size_t n = b.active.size();
    b.h_members.assign(n * sizeof(BatchMember<CT>), 0);
    auto *bm = reinterpret_cast<BatchMember<CT> *>(b.h_members.data());
    b.h_tiles[0].clear();
    b.h_tiles[1].clear();
    b.h_res.clear();
    b.h_fin.clear();
    int32_t part = 0;
    // the members' buffers share the last-level cache: non-temporal stores
    // when all of them together do not fit it
    int64_t pair_bytes = 0;
    for (size_t k = 0; k < n; ++k) pair_bytes += 2 * (int64_t)coef_of<ST>(b.mem[b.active[k]].p).state_bytes;
    b.auto_tile = default_batch_tile(b.storage, pair_bytes);
    const TileShape ts = kTiles[batch_tile(b)];
    for (size_t k = 0; k < n; ++k) {
        const Member &m = b.mem[b.active[k]];
        bm[k].c = coef_of<ST>(m.p);
        bm[k].c.nt = pair_bytes > kNtPairBytes;
        bm[k].buf[0] = m.fa;
        bm[k].buf[1] = m.fb;
        bm[k].u_prev = m.up;
        auto &tl = b.h_tiles[variant_of(m.p)];
        for (int y0 = 0; y0 < m.p.ny; y0 += ts.ty)
            for (int x0 = 0; x0 < m.p.nx; x0 += ts.tx) tl.push_back({(int32_t)k, x0, y0, 0});
        const int nb = red_blocks(m.p);
        for (int i = 0; i < nb; ++i) b.h_res.push_back({(int32_t)k, i, nb, part});
        b.h_fin.push_back({part, nb, (int32_t)k, 0});
        part += nb;
    }
    prc_status st;
    if ((st = b.d_members.ensure(std::max<size_t>(b.h_members.size(), 1))) != PRC_OK) return st;
    for (int v = 0; v < 2; ++v) {
        b.ntiles[v] = (int)b.h_tiles[v].size();
        const size_t bytes = b.h_tiles[v].size() * sizeof(BatchTile);
        if ((st = b.d_tiles[v].ensure(std::max<size_t>(bytes, 1))) != PRC_OK) return st;
        if (bytes)
            HIP_TRY(hipMemcpyAsync(b.d_tiles[v].ptr, b.h_tiles[v].data(), bytes,
                                   hipMemcpyHostToDevice, s));
    }
    if ((st = b.d_res.ensure(std::max<size_t>(b.h_res.size() * sizeof(ResItem), 1))) != PRC_OK)
        return st;
    if ((st = b.d_fin.ensure(std::max<size_t>(b.h_fin.size() * sizeof(FinItem), 1))) != PRC_OK)
        return st;
    if ((st = b.d_partial.ensure(std::max<size_t>((size_t)part * 4 * sizeof(double), 1))) != PRC_OK)
        return st;
    if ((st = b.d_out.ensure(std::max<size_t>(n * 4 * sizeof(double), 1))) != PRC_OK) return st;
    if (n) {
        HIP_TRY(hipMemcpyAsync(b.d_members.ptr, b.h_members.data(), b.h_members.size(),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b.d_res.ptr, b.h_res.data(), b.h_res.size() * sizeof(ResItem),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b.d_fin.ptr, b.h_fin.data(), b.h_fin.size() * sizeof(FinItem),
                               hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    b.dirty = false;
    b.calls_since_rebuild = 0;
    return PRC_OK;
}

static prc_status ensure_tables(prc_batch &b, hipStream_t s)
{
    if (!b.dirty) return PRC_OK;
    prc_params q{};
    q.storage = b.storage;
    q.bc = b.bc;
    return PRC_DISPATCH(q, build_tables, b, s);
}

template <typename ST, int BC, int TX, int TY, bool FORCE, bool ALL, int STEPS>
static prc_status launch_batch_shape(const prc_batch &b, int v, int parity, hipStream_t s)
{
    using CT = typename Mem<ST>::CT;
    const int nt = b.ntiles[v];
    const int per_xcd = (nt + kXcds - 1) / kXcds;
    if constexpr (STEPS == 2) {
        // 1024-thread tiles: the instance for states streamed from HBM, as
        // for single problems of that size
        hipLaunchKernelGGL((k_sweep_batch2<ST, BC, TX, TY, FORCE, ALL, TX * TY == 1024>),
                           dim3(per_xcd * kXcds),
                           dim3(TX * TY), 0, s, (const BatchTile *)b.d_tiles[v].ptr, nt, per_xcd,
                           (const BatchMember<CT> *)b.d_members.ptr, parity);
    } else {
        hipLaunchKernelGGL((k_sweep_batch<ST, BC, TX, TY, FORCE, ALL>), dim3(per_xcd * kXcds),
                           dim3(TX * TY), 0, s, (const BatchTile *)b.d_tiles[v].ptr, nt, per_xcd,
                           (const BatchMember<CT> *)b.d_members.ptr, parity);
    }
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

template <typename ST, int BC, int TX, int TY, int STEPS>
static prc_status launch_batch_variants(const prc_batch &b, int parity, hipStream_t s)
{
    prc_status st = PRC_OK;
    if (b.ntiles[0] > 0)
        st = launch_batch_shape<ST, BC, TX, TY, false, true, STEPS>(b, 0, parity, s);
    if (st == PRC_OK && b.ntiles[1] > 0)
        st = launch_batch_shape<ST, BC, TX, TY, true, false, STEPS>(b, 1, parity, s);
    return st;
}

// One launch over every active member, reading buf[parity] and writing the
// other: two steps if `two` (the batch's shape must be a two-step one), else
// one step with the batch's shape or its single-step twin.
template <typename ST, int BC>
static prc_status launch_batch_sweep(const prc_batch &b, int parity, bool two, hipStream_t s)
{
    switch (batch_tile(b)) {
    case 1: return launch_batch_variants<ST, BC, 64, 8, 1>(b, parity, s);
    case 2: return launch_batch_variants<ST, BC, 128, 4, 1>(b, parity, s);
    case 3: return launch_batch_variants<ST, BC, 32, 8, 1>(b, parity, s);
    case 4: return launch_batch_variants<ST, BC, 32, 16, 1>(b, parity, s);
    case 5:
        return two ? launch_batch_variants<ST, BC, 64, 8, 2>(b, parity, s)
                   : launch_batch_variants<ST, BC, 64, 8, 1>(b, parity, s);
    case 6:
        return two ? launch_batch_variants<ST, BC, 32, 16, 2>(b, parity, s)
                   : launch_batch_variants<ST, BC, 32, 16, 1>(b, parity, s);
    case 7:
        return two ? launch_batch_variants<ST, BC, 64, 16, 2>(b, parity, s)
                   : launch_batch_variants<ST, BC, 64, 16, 1>(b, parity, s);
    default: return launch_batch_variants<ST, BC, 64, 4, 1>(b, parity, s);
    }
}

static prc_status batch_sweep(const prc_batch &b, int parity, hipStream_t s, bool two = false)
{
    prc_params q{};
    q.storage = b.storage;
    q.bc = b.bc;
    return PRC_DISPATCH(q, launch_batch_sweep, b, parity, two, s);
}

// Steps [k0, k0 + n) of every active member (step k reads buf[k & 1]); with a
// two-step shape, pairs of two-step launches cover the steps in fours from an
// even step (as for single problems), single steps the rest.
static prc_status batch_run(const prc_batch &b, int64_t k0, int64_t n, hipStream_t s)
{
    prc_status st = PRC_OK;
    int64_t k = k0;
    const int64_t end = k0 + n;
    if (kTiles[batch_tile(b)].steps == 2) {
        if (k < end && (k & 1)) st = batch_sweep(b, (int)(k++ & 1), s);
        for (; k + 4 <= end && st == PRC_OK; k += 4) {
            st = batch_sweep(b, 0, s, true);
            if (st == PRC_OK) st = batch_sweep(b, 1, s, true);
        }
    }
    for (; k < end && st == PRC_OK; ++k) st = batch_sweep(b, (int)(k & 1), s);
    return st;
}

static prc_status capture_graph(prc_batch &b, int nsteps)
{
    drop_graph(b);
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    prc_status st = PRC_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = batch_run(b, 0, nsteps, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess && st == PRC_OK) {
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            if (e == hipSuccess) {
                b.graph = g;
                b.gexec = x;
                b.gsteps = nsteps;
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
        return fail(PRC_EHIP, "batch graph capture of %d sweeps: %s", nsteps, hipGetErrorString(e));
    return PRC_OK;
}

static prc_status batch_steps(prc_batch &b, int64_t nsteps, hipStream_t s)
{
    prc_status st = ensure_tables(b, s);
    if (st != PRC_OK || b.active.empty()) return st;
    int64_t k = 0;
    const int gsteps = graph_steps();
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    // graphs only for tables that have already served a call: a batch whose
    // membership changes at every interval would otherwise capture each time
    const bool stable = b.calls_since_rebuild++ > 0;
    if (gsteps > 0 && stable && cap == hipStreamCaptureStatusNone && nsteps >= 2 * gsteps) {
        if (!b.gexec || b.gsteps != gsteps)
            if ((st = capture_graph(b, gsteps)) != PRC_OK) return st;
        for (; k + gsteps <= nsteps; k += gsteps) HIP_TRY(hipGraphLaunch(b.gexec, s));
    }
    return batch_run(b, k, nsteps - k, s);
}

template <typename ST, int BC>
static prc_status launch_batch_residual(const prc_batch &b, const ResItem *items, int nitems,
                                        const FinItem *fin, int nfin, hipStream_t s)
{
    using CT = typename Mem<ST>::CT;
    hipLaunchKernelGGL((k_residual_batch<ST, BC>), dim3(nitems), dim3(kRedBlock), 0, s, items,
                       (const BatchMember<CT> *)b.d_members.ptr, (double *)b.d_partial.ptr);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_finish_batch<>, dim3(nfin), dim3(kRedBlock), 0, s, fin,
                       (const double *)b.d_partial.ptr, (double *)b.d_out.ptr);
    HIP_TRY(hipGetLastError());
    return PRC_OK;
}

// Check of the active members in `slots` (all of them if empty == false and
// slots == nullptr).  Results land in b.h_out[4 * slot + k].
static prc_status batch_check(prc_batch &b, const std::vector<int32_t> *slots, hipStream_t s)
{
    prc_status st = ensure_tables(b, s);
    if (st != PRC_OK) return st;
    const size_t n = b.active.size();
    if (n == 0) return PRC_OK;
    const ResItem *items = (const ResItem *)b.d_res.ptr;
    const FinItem *fin = (const FinItem *)b.d_fin.ptr;
    int nitems = (int)b.h_res.size(), nfin = (int)b.h_fin.size();
    // a subset: its items and totals go behind the full lists' storage
    DevBuf sub_res, sub_fin;
    std::vector<ResItem> r;
    std::vector<FinItem> f;
    if (slots) {
        if (slots->empty()) return PRC_OK;
        for (int32_t k : *slots) {
            const FinItem &fi = b.h_fin[k];
            for (int i = 0; i < fi.nb; ++i) r.push_back({k, i, fi.nb, fi.part});
            f.push_back(fi);
        }
        if ((st = sub_res.ensure(r.size() * sizeof(ResItem))) != PRC_OK) return st;
        if ((st = sub_fin.ensure(f.size() * sizeof(FinItem))) != PRC_OK) {
            sub_res.release();
            return st;
        }
        hipError_t e = hipMemcpyAsync(sub_res.ptr, r.data(), r.size() * sizeof(ResItem),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sub_fin.ptr, f.data(), f.size() * sizeof(FinItem),
                               hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            sub_res.release();
            sub_fin.release();
            return fail(PRC_EHIP, "batch check upload: %s", hipGetErrorString(e));
        }
        items = (const ResItem *)sub_res.ptr;
        fin = (const FinItem *)sub_fin.ptr;
        nitems = (int)r.size();
        nfin = (int)f.size();
    }
    prc_params q{};
    q.storage = b.storage;
    q.bc = b.bc;
    st = PRC_DISPATCH(q, launch_batch_residual, b, items, nitems, fin, nfin, s);
    b.h_out.assign(n * 4, 0.0);
    hipError_t e = hipSuccess;
    if (st == PRC_OK)
        e = hipMemcpyAsync(b.h_out.data(), b.d_out.ptr, n * 4 * sizeof(double),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    sub_res.release();
    sub_fin.release();
    if (st != PRC_OK) return st;
    if (e != hipSuccess) return fail(PRC_EHIP, "batch check: %s", hipGetErrorString(e));
    for (size_t k = 0; k < n; ++k) {  // rest part of the mass, as prc_residual
        const prc_params &p = b.mem[b.active[k]].p;
        b.h_out[4 * k + 2] += p.rho0 * (double)p.nx * (double)p.ny;
    }
    return PRC_OK;
}

static void retire(prc_batch &b, int32_t id, int32_t status)
{
    b.mem[id].status = status;
    b.active.erase(std::find(b.active.begin(), b.active.end(), id));
    b.dirty = true;
}

static prc_status batch_ok(const prc_batch *b)
{
    if (!b) return fail(PRC_EINVAL, "batch is NULL");
    return PRC_OK;
}

static void leave(prc_batch &b, int32_t id, int32_t status, std::vector<BatchLeft> *left)
{
    retire(b, id, status);
    if (left) left->push_back({id, status, b.mem[id].steps, b.mem[id].R});
}

prc_status batch_interval(prc_batch *b, double tol, int64_t check_every, int64_t max_steps,
                          std::vector<BatchChecked> *checked, std::vector<BatchLeft> *left,
                          hipStream_t s)
{
    prc_status st = ensure_tables(*b, s);
    if (st != PRC_OK) return st;
    // velocity snapshots of members that have none yet (as prc_solve's first
    // prc_residual)
    std::vector<int32_t> slots;
    for (size_t k = 0; k < b->active.size(); ++k)
        if (b->mem[b->active[k]].fresh) slots.push_back((int32_t)k);
    if (!slots.empty()) {
        if ((st = batch_check(*b, &slots, s)) != PRC_OK) return st;
        for (int32_t k : slots) b->mem[b->active[k]].fresh = false;
    }
    for (int32_t id : std::vector<int32_t>(b->active))
        if (b->mem[id].steps >= max_steps) leave(*b, id, PRC_MEMBER_MAX_STEPS, left);
    if (b->active.empty()) return PRC_OK;
    if ((st = batch_steps(*b, check_every, s)) != PRC_OK) return st;
    if ((st = batch_check(*b, nullptr, s)) != PRC_OK) return st;
    const std::vector<int32_t> ids = b->active;
    for (size_t k = 0; k < ids.size(); ++k) {
        Member &m = b->mem[ids[k]];
        m.steps += check_every;
        const double *o = &b->h_out[4 * k];
        // as prc_solve: a NaN in either sum makes R non-finite
        m.R = o[1] > 0.0 ? std::sqrt(o[0] / o[1]) : (o[1] == 0.0 && o[0] == 0.0 ? 0.0 : INFINITY);
        if (checked) checked->push_back({ids[k], m.R});
        if (!std::isfinite(m.R) || !std::isfinite(o[2]) || !(o[3] < 1.0))
            leave(*b, ids[k], PRC_MEMBER_DIVERGED, left);
        else if (m.R < tol)
            leave(*b, ids[k], PRC_MEMBER_CONVERGED, left);
        else if (m.steps >= max_steps)
            leave(*b, ids[k], PRC_MEMBER_MAX_STEPS, left);
    }
    return PRC_OK;
}

}  // namespace prc

// ----------------------------------------------------------------- ABI --
extern "C" {

prc_status prc_batch_create(int32_t storage, int32_t bc, prc_batch **out)
{
    if (!out) return fail(PRC_EINVAL, "out is NULL");
    *out = nullptr;
    if (storage < PRC_F64 || storage > PRC_BF16) return fail(PRC_EINVAL, "unknown storage %d", storage);
    if (bc < PRC_BC_CAVITY || bc > PRC_BC_CHANNEL) return fail(PRC_EINVAL, "unknown bc %d", bc);
    prc_batch *b = new (std::nothrow) prc_batch;
    if (!b) return fail(PRC_ENOMEM, "batch allocation failed");
    b->storage = storage;
    b->bc = bc;
    *out = b;
    return PRC_OK;
}

prc_status prc_batch_destroy(prc_batch *b)
{
    if (!b) return PRC_OK;
    drop_graph(*b);
    b->d_members.release();
    b->d_tiles[0].release();
    b->d_tiles[1].release();
    b->d_res.release();
    b->d_fin.release();
    b->d_partial.release();
    b->d_out.release();
    delete b;
    return PRC_OK;
}

prc_status prc_batch_add(prc_batch *b, const prc_params *p, void *f_a, void *f_b, double *u_prev,
                         int32_t *id_out)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    if ((st = validate(p)) != PRC_OK) return st;
    if (p->storage != b->storage || p->bc != b->bc)
        return fail(PRC_EINVAL, "member storage/bc (%d/%d) differ from the batch's (%d/%d)",
                    p->storage, p->bc, b->storage, b->bc);
    if ((st = check_buf(f_a, "f_a")) != PRC_OK || (st = check_buf(f_b, "f_b")) != PRC_OK) return st;
    if (f_a == f_b) return fail(PRC_EINVAL, "f_a and f_b must be distinct buffers");
    if (!u_prev) return fail(PRC_EINVAL, "u_prev is NULL");
    if (b->mem.size() >= (size_t)INT32_MAX) return fail(PRC_EINVAL, "too many members");
    b->mem.push_back(Member{*p, f_a, f_b, u_prev, PRC_MEMBER_ACTIVE, true, 0, NAN});
    const int32_t id = (int32_t)(b->mem.size() - 1);
    b->active.push_back(id);
    b->dirty = true;
    if (id_out) *id_out = id;
    return PRC_OK;
}

prc_status prc_batch_remove(prc_batch *b, int32_t id)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    if (id < 0 || (size_t)id >= b->mem.size()) return fail(PRC_EINVAL, "no member %d", id);
    if (b->mem[id].status != PRC_MEMBER_ACTIVE) return fail(PRC_EINVAL, "member %d is not active", id);
    retire(*b, id, PRC_MEMBER_REMOVED);
    return PRC_OK;
}

prc_status prc_batch_count(const prc_batch *b, int32_t *n_added, int32_t *n_active)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    if (n_added) *n_added = (int32_t)b->mem.size();
    if (n_active) *n_active = (int32_t)b->active.size();
    return PRC_OK;
}

prc_status prc_batch_step(prc_batch *b, int64_t nsteps, hipStream_t stream)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    if (nsteps < 0 || (nsteps & 1)) return fail(PRC_EINVAL, "nsteps must be even and >= 0");
    if ((st = batch_steps(*b, nsteps, stream)) != PRC_OK) return st;
    for (int32_t id : b->active) b->mem[id].steps += nsteps;
    return PRC_OK;
}

prc_status prc_batch_residual(prc_batch *b, double *out, hipStream_t stream)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    if (!out) return fail(PRC_EINVAL, "out is NULL");
    if ((st = batch_check(*b, nullptr, stream)) != PRC_OK) return st;
    for (size_t k = 0; k < b->active.size(); ++k) {
        const int32_t id = b->active[k];
        b->mem[id].fresh = false;
        for (int j = 0; j < 4; ++j) out[4 * (size_t)id + j] = b->h_out[4 * k + j];
    }
    return PRC_OK;
}

prc_status prc_batch_solve(prc_batch *b, double tol, int64_t check_every, int64_t max_steps,
                           int32_t *status, int64_t *steps, double *hist, int64_t hist_cap,
                           int64_t *hist_len, hipStream_t stream)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    if (check_every <= 0 || (check_every & 1)) return fail(PRC_EINVAL, "check_every must be even and > 0");
    if (max_steps < 0 || max_steps % check_every)
        return fail(PRC_EINVAL, "max_steps must be a non-negative multiple of check_every");
    if (!(tol >= 0.0)) return fail(PRC_EINVAL, "tol must be >= 0");
    if (hist && hist_cap < 0) return fail(PRC_EINVAL, "hist_cap < 0");
    const size_t n_added = b->mem.size();
    std::vector<int64_t> nh(n_added, 0);
    std::vector<BatchChecked> checked;
    do {
        checked.clear();
        if ((st = batch_interval(b, tol, check_every, max_steps, &checked, nullptr, stream)) != PRC_OK)
            return st;
        for (const BatchChecked &c : checked) {
            if (hist && nh[c.id] < hist_cap) hist[(size_t)c.id * hist_cap + nh[c.id]] = c.R;
            ++nh[c.id];
        }
    } while (!b->active.empty());
    for (size_t id = 0; id < n_added; ++id) {
        if (status) status[id] = b->mem[id].status;
        if (steps) steps[id] = b->mem[id].steps;
        if (hist_len) hist_len[id] = nh[id];
    }
    return PRC_OK;
}

prc_status prc_batch_tune(prc_batch *b, int32_t *tile_out, hipStream_t stream)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    constexpr int kWarm = 4, kTimed = 20;
    const int keep = b->tile;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = -1;
    float best_ms = 0.0f;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    for (int t = 0; t < kNumBatchTiles && he == hipSuccess && st == PRC_OK; ++t) {
        b->tile = t;
        b->dirty = true;
        if ((st = ensure_tables(*b, stream)) != PRC_OK) break;
        if (b->active.empty()) break;
        // always f_a -> f_b: the state in f_a is only read
        for (int k = 0; k < kWarm + kTimed && st == PRC_OK && he == hipSuccess; ++k) {
            if (k == kWarm) he = hipEventRecord(e0, stream);
            st = batch_sweep(*b, 0, stream, kTiles[t].steps == 2);
        }
        if (st != PRC_OK || he != hipSuccess) break;
        he = hipEventRecord(e1, stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)kTiles[t].steps;  // per time step
        if (he == hipSuccess && (best < 0 || ms < best_ms)) {
            best = t;
            best_ms = ms;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    b->tile = best >= 0 ? best : keep;
    b->dirty = true;
    if (st != PRC_OK) return st;
    if (he != hipSuccess) return fail(PRC_EHIP, "prc_batch_tune: %s", hipGetErrorString(he));
    if (tile_out) *tile_out = batch_tile(*b);
    return PRC_OK;
}

prc_status prc_batch_set_tile(prc_batch *b, int32_t tile)
{
    prc_status st = batch_ok(b);
    if (st != PRC_OK) return st;
    if (tile < 0 || tile >= kNumBatchTiles)
        return fail(PRC_EINVAL, "tile %d out of range for a batch (0 .. %d)", tile,
                    kNumBatchTiles - 1);
    if (tile != b->tile) {
        b->tile = tile;
        b->dirty = true;
    }
    return PRC_OK;
}

}  // extern "C"
