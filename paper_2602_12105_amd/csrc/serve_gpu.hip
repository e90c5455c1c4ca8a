// Serving loop on the GPU: the executor behind the scheduler core, its
// batched kernels, and the dgo_server_* C entry points.
//
// Batched execution. Every active request is described by a SrvDesc (its
// topology, its device arrays and this tick's plan) in one device array that
// is rewritten before each tick. The kernels are persistent: a fixed grid
// splits the concatenated row tiles of all active requests into contiguous
// ranges, one per workgroup; a workgroup finds the request of its first tile
// by binary search over the requests' tile offsets and steps to the next
// request as its range crosses into it, and runs each tile with the same
// per-tile code as the per-mesh kernels. One tick is: assembly and solver
// start for requests that joined, then `cg_chunk` PCG iterations (the
// one-reduction form of the per-mesh solver: vector update with r.z and r.r,
// w = A D^-1 r with w.z, per-request finalize) for every request that still
// has iterations left. The launch sequence of a tick never changes, so it is
// captured once as a graph and replayed every tick.
//
// A request's tiles, partial sums and reduction order depend only on the
// request, so its result is bitwise the same alone or in any batch.
#include <cstring>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "../../include/dgo_serve.h"
#include "internal.hpp"
#include "kernels.hpp"
#include "serve_core.hpp"

namespace dgo {
namespace {

using namespace kern;
using R = float;

constexpr int kSrvBlocks = 2048;      // persistent grid of the batched streaming kernels
constexpr int kSrvAsmBlocks = 2048;   // persistent grid of the batched assembly
constexpr int kSrvMaxSlots = 256;
constexpr int kSrvMaxK = 16;
// Row tiles per work unit of the batched streaming kernels: a workgroup runs
// a unit's tiles back to back, adding each thread's terms in registers, and
// reduces once per unit (the unit is fixed per request, so the sums do not
// depend on the batch).
constexpr int kSrvTilesPerUnit = 8;
// LDS of one assembly row block: eight resident workgroups per CU (a row
// block of 64 rows of a mesh of degree up to about 8 needs less in FP32).
constexpr int64_t kSrvLdsBytes = 20 * 1024;

struct SrvDesc {
    AsmView view;
    const int32_t *diag;
    const int32_t *ell_col, *ell_src;  // padded rows in natural order (ell_w = 0: none)
    int64_t nnz;
    int32_t ell_w, pad0;
    const R *X, *f;
    R *K, *M, *u, *r, *p, *s, *w, *invD, *v;
    double *part, *part2;
    CgCol *st;
    int32_t k, KP, init, iters;
    int32_t tiles_s, tiles_v, units_s, units_v, off_a, off_s, off_v, nblocks;
};

struct SrvHdr {
    int32_t n, tot_a, tot_s, tot_v;
};

enum Space { SP_A = 0, SP_S = 1, SP_V = 2 };

__device__ __forceinline__ int32_t off_of(const SrvDesc &d, int sp) {
    return sp == SP_A ? d.off_a : (sp == SP_S ? d.off_s : d.off_v);
}

// The request owning global tile v: the last r with off(r) <= v (requests
// with no tiles share their offset with the next one and are skipped).
__device__ __forceinline__ int find_req(const SrvDesc *d, int n, int32_t v, int sp) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off_of(d[mid], sp) <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Calls f(request, unit of the request) for each unit of this workgroup's
// contiguous range of the tick's units in space sp (SP_A: one assembly row
// block per unit). Uniform over the workgroup (f may synchronise).
template <class F>
__device__ __forceinline__ void for_tiles(const SrvDesc *d, int n, int32_t tot, int sp, F &&f) {
    int64_t t0, t1;
    tile_range(tot, t0, t1);
    if (t0 >= t1) return;
    int r = find_req(d, n, (int32_t)t0, sp);
    for (int32_t v = (int32_t)t0; v < (int32_t)t1; ++v) {
        while (r + 1 < n && off_of(d[r + 1], sp) <= v) ++r;
        f(d[r], v - off_of(d[r], sp));
    }
}

__global__ void __launch_bounds__(kAssembleThreads)
ks_assemble(const SrvHdr *hdr, const SrvDesc *d, int32_t *ndeg) {
    extern __shared__ __align__(16) unsigned char smem[];
    for_tiles(d, hdr->n, hdr->tot_a, SP_A, [&](const SrvDesc &q, int32_t tile) {
        assemble_block<R, 2>(q.view, (uint32_t)tile, q.X, q.K, q.M, 0, R(0), ndeg, smem);
    });
}

// Start of the solve (x0 = 0): D^-1, b = M f, r = b, p = s = 0; partial sums
// of r.z, r.r, b.b per unit.
__global__ void __launch_bounds__(T)
ks_init(const SrvHdr *hdr, const SrvDesc *d, R alpha, R beta) {
    __shared__ double s_part[3 * kSrvMaxK];
    __shared__ double s_red[red_scratch(T, 3)];
    for_tiles(d, hdr->n, hdr->tot_v, SP_V, [&](const SrvDesc &q, int32_t unit) {
        if (!q.init) return;
        const VLane L = vlane(q.k, q.KP);
        double dd[3] = {0.0, 0.0, 0.0};
        const int32_t tb = unit * kSrvTilesPerUnit, te = min(tb + kSrvTilesPerUnit, q.tiles_v);
        for (int32_t tile = tb; tile < te; ++tile) {
            const int64_t i = (int64_t)tile * L.gpb + L.grp;
            if (!L.act || i >= q.view.nV) continue;
            const R inv = R(1) / (alpha * q.M[i] + beta * q.K[q.diag[i]]);
            if (L.c == 0) q.invD[i] = inv;
            const int64_t e = i * q.k + L.c;
            const R b = q.M[i] * q.f[e];
            const R z = inv * b;
            q.u[e] = R(0);
            q.r[e] = b;
            q.p[e] = R(0);
            q.s[e] = R(0);
            dd[0] += (double)b * (double)z;
            dd[1] += (double)b * (double)b;
        }
        dd[2] = dd[1];
        column_partials(dd, 3, q.k, q.KP, L.act, s_red, s_part);
        const int W = 3 * q.k;
        if ((int)threadIdx.x < W) q.part[(size_t)threadIdx.x * q.units_v + unit] = s_part[threadIdx.x];
        __syncthreads();
    });
}

// Operator values scaled by the preconditioner, v_ij = A_ij d_j (after
// ks_init has stored D^-1), in padded-row layout when the request has one
// (padding 0), else aligned with the CSR entries.
__global__ void __launch_bounds__(T)
ks_values(const SrvHdr *hdr, const SrvDesc *d, R alpha, R beta) {
    for_tiles(d, hdr->n, hdr->tot_a, SP_A, [&](const SrvDesc &q, int32_t tile) {
        const int32_t r0 = tile * q.view.rpb, r1 = min(r0 + q.view.rpb, q.view.nV);
        if (q.ell_w) {
            const int32_t W = q.ell_w;
            for (int32_t e = r0 * W + (int32_t)threadIdx.x; e < r1 * W; e += blockDim.x) {
                const int32_t t = q.ell_src[e];
                R val = R(0);
                if (t >= 0) {
                    const int32_t j = q.view.col[t];
                    R a = beta * q.K[t];
                    if (q.diag[j] == t) a += alpha * q.M[j];  // the diagonal entry
                    val = a * q.invD[j];
                }
                q.v[e] = val;
            }
            return;
        }
        const int32_t s0 = q.view.rowptr[r0], s1 = q.view.rowptr[r1];
        for (int32_t t = s0 + (int32_t)threadIdx.x; t < s1; t += blockDim.x) {
            const int32_t j = q.view.col[t];
            R a = beta * q.K[t];
            if (q.diag[j] == t) a += alpha * q.M[j];  // the diagonal entry of row j = i
            q.v[t] = a * q.invD[j];
        }
    });
}

template <int KP>
__device__ __forceinline__ void sdot_unit(const SrvDesc &q, int32_t unit, double *s_red,
                                          double *s_part) {
    constexpr int G = KP < 8 ? 8 : KP;
    constexpr int GPB = T / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int gbase = (threadIdx.x & 63) - lane;
    const bool out_lane = lane < q.k && lane < KP;
    double ds = 0.0;
    const int32_t tb = unit * kSrvTilesPerUnit, te = min(tb + kSrvTilesPerUnit, q.tiles_s);
    if (q.ell_w && q.ell_w <= G) {
        // padded rows, the next tile's entries loaded while this tile's
        // gathers are in flight
        const int32_t nV = q.view.nV, W = q.ell_w;
        int32_t row = tb * GPB + grp, cj;
        R aj;
        ell_entry(q.ell_col, q.v, W, row < nV ? row : 0, lane, cj, aj);
        for (int32_t tile = tb; tile < te; ++tile, row += GPB) {
            const int32_t cj0 = cj;
            const R aj0 = aj;
            if (tile + 1 < te && row + GPB < nV) ell_entry(q.ell_col, q.v, W, row + GPB, lane, cj, aj);
            if (row >= nV) continue;  // uniform over the lane group
            R ri = 0;
            const R acc = ell_row<R, G, KP>(cj0, aj0, q.r, row, q.k, W, lane, gbase, &ri);
            if (out_lane) {
                const int64_t e = (int64_t)row * q.k + lane;
                q.w[e] = acc;
                if (G != KP) ri = q.r[e];  // ell_row returns r[i, c] only when G == KP
                ds += (double)acc * (double)(q.invD[row] * ri);
            }
        }
        column_partials(&ds, 1, q.k, G, out_lane, s_red, s_part);
        if ((int)threadIdx.x < q.k) q.part2[(size_t)threadIdx.x * q.units_s + unit] = s_part[threadIdx.x];
        __syncthreads();
        return;
    }
    for (int32_t tile = tb; tile < te; ++tile) {
        const int32_t row = tile * GPB + grp;
        if (row >= q.view.nV) continue;  // uniform over the lane group
        int32_t rb, len;
        const int32_t *col;
        if (q.ell_w) {  // padded rows: no row pointer load
            rb = row * q.ell_w;
            len = q.ell_w;
            col = q.ell_col;
        } else {
            rb = q.view.rowptr[row];
            len = q.view.rowptr[row + 1] - rb;
            col = q.view.col;
        }
        R ri = 0;
        const R acc = row_apply<R, G, KP, false>(col, q.v, R(1), R(0), nullptr, q.r, row, rb, len,
                                                 q.k, lane, gbase, &ri);
        if (out_lane) {
            const int64_t e = (int64_t)row * q.k + lane;
            q.w[e] = acc;
            if (G != KP) ri = q.r[e];  // row_apply returns r[i, c] only when G == KP
            ds += (double)acc * (double)(q.invD[row] * ri);
        }
    }
    column_partials(&ds, 1, q.k, G, out_lane, s_red, s_part);
    if ((int)threadIdx.x < q.k) q.part2[(size_t)threadIdx.x * q.units_s + unit] = s_part[threadIdx.x];
    __syncthreads();
}

// w = A D^-1 r with the partial sums of w.z; j < 0: the start of the solve.
__global__ void __launch_bounds__(T, 6)
ks_sdot(const SrvHdr *hdr, const SrvDesc *d, int j) {
    __shared__ double s_part[kSrvMaxK];
    __shared__ double s_red[red_scratch(T, 1)];
    for_tiles(d, hdr->n, hdr->tot_s, SP_S, [&](const SrvDesc &q, int32_t unit) {
        if (j < 0 ? !q.init : j >= q.iters) return;
        switch (q.KP) {
            case 1: sdot_unit<1>(q, unit, s_red, s_part); break;
            case 2: sdot_unit<2>(q, unit, s_red, s_part); break;
            case 4: sdot_unit<4>(q, unit, s_red, s_part); break;
            case 8: sdot_unit<8>(q, unit, s_red, s_part); break;
            default: sdot_unit<16>(q, unit, s_red, s_part); break;
        }
    });
}

// One workgroup per request: reduce its partial sums and advance its state
// (FIN_SR_INIT at the start of the solve, FIN_SR_ITER after iteration j).
template <int MODE>
__global__ void __launch_bounds__(kFinThreads)
ks_fin(const SrvHdr *hdr, const SrvDesc *d, int j, CgParams prm) {
    __shared__ double s_tot[4 * kSrvMaxK];
    for (int r = blockIdx.x; r < hdr->n; r += gridDim.x) {
        const SrvDesc &q = d[r];
        if (MODE == FIN_SR_INIT ? !q.init : j >= q.iters) continue;
        const int W = fin_width(MODE, q.k);
        fin_sum2(q.part, q.units_v, W, q.part2, q.units_s, q.k, s_tot);
        if ((int)threadIdx.x < q.k) {
            CgCol c = MODE == FIN_SR_INIT ? CgCol{} : q.st[threadIdx.x];
            cg_sr_update(MODE, c, s_tot, s_tot + W, threadIdx.x, q.k, prm);
            q.st[threadIdx.x] = c;
        }
        __syncthreads();
    }
}

// p = z + beta p, s = w + beta s, x += alpha p, r -= alpha s on the active
// columns (z = D^-1 r); partial sums of r.z and r.r of the new residual.
__global__ void __launch_bounds__(T)
ks_vupdate(const SrvHdr *hdr, const SrvDesc *d, int j) {
    __shared__ double s_part[2 * kSrvMaxK];
    __shared__ double s_red[red_scratch(T, 2)];
    for_tiles(d, hdr->n, hdr->tot_v, SP_V, [&](const SrvDesc &q, int32_t unit) {
        if (j >= q.iters) return;
        const VLane L = vlane(q.k, q.KP);
        const bool on = L.act && q.st[L.c].active;
        double dd[2] = {0.0, 0.0};
        if (on) {
            const R a = (R)q.st[L.c].alpha, bt = (R)q.st[L.c].beta;
            const int32_t tb = unit * kSrvTilesPerUnit, te = min(tb + kSrvTilesPerUnit, q.tiles_v);
            for (int32_t tile = tb; tile < te; ++tile) {
                const int64_t i = (int64_t)tile * L.gpb + L.grp;
                if (i >= q.view.nV) continue;
                const int64_t e = i * q.k + L.c;
                const R rv = q.r[e], dv = q.invD[i];
                const R pn = dv * rv + bt * q.p[e];
                const R sn = q.w[e] + bt * q.s[e];
                const R rn = rv - a * sn;
                q.p[e] = pn;
                q.s[e] = sn;
                q.u[e] += a * pn;
                q.r[e] = rn;
                const R zn = dv * rn;
                dd[0] += (double)rn * (double)zn;
                dd[1] += (double)rn * (double)rn;
            }
        }
        column_partials(dd, 2, q.k, q.KP, on, s_red, s_part);
        const int W = 2 * q.k;
        if ((int)threadIdx.x < W) q.part[(size_t)threadIdx.x * q.units_v + unit] = s_part[threadIdx.x];
        __syncthreads();
    });
}

// ------------------------------------------------------------- footprint

int64_t rnd(int64_t b) { return (b + 255) & ~int64_t(255); }

int64_t tiles_for(int32_t nV, int rows) { return ((int64_t)nV + rows - 1) / rows; }

// Upper bound of the bytes one request takes from the arena: its inputs, the
// topology (persistent arrays and the temporaries of its construction, with
// the edge count bounded by 3 nF) and its solver arrays.
int64_t footprint_of(int32_t nV, int64_t nF, int32_t k, bool per_mesh_path) {
    const int64_t nE = 3 * nF, nnz = (int64_t)nV + 2 * nE, V1 = (int64_t)nV + 1;
    const int KP = pow2ceil(k), G = KP < 8 ? 8 : KP;
    const int64_t tv = (tiles_for(nV, T / KP) + kSrvTilesPerUnit - 1) / kSrvTilesPerUnit;
    const int64_t ts = (tiles_for(nV, T / G) + kSrvTilesPerUnit - 1) / kSrvTilesPerUnit;
    int64_t b = 0;
    b += rnd(12 * nF) + rnd(12 * (int64_t)nV) + rnd(4 * (int64_t)nV * k);  // F, X, f
    // topology construction
    b += rnd(12 * nF) + rnd(32) + 5 * rnd(4 * V1) + rnd(4 * (V1 / 1000 + 64)) + rnd(8 * 3 * nF);
    b += rnd(8 * nE) + rnd(12 * nF) + rnd(3 * nF) + rnd(4 * V1) + rnd(4 * nnz) + rnd(4 * (int64_t)nV) +
         rnd(4 * V1) + rnd(12 * nF) + rnd(nV) + rnd(12 * nF) + rnd(4 * nE);
    // solver arrays: K, M, u r p s w, D^-1, v, the two partial-sum arrays, state
    b += rnd(4 * nnz) + rnd(4 * (int64_t)nV) + 5 * rnd(4 * (int64_t)nV * k) + rnd(4 * (int64_t)nV);
    b += rnd(4 * std::max<int64_t>(nnz, (int64_t)kEllMaxWidth * nV)) + rnd(8 * 3 * k * tv) +
         rnd(8 * k * ts) + rnd((int64_t)sizeof(CgCol) * k);
    // row descriptors and the padded-row pattern (natural order)
    b += rnd(8 * (int64_t)nV) + rnd(nV) + 2 * rnd(4 * (int64_t)kEllMaxWidth * nV);
    if (per_mesh_path) {
        // the per-mesh PCG workspace (grown once, with headroom) and the
        // assembly counter
        const int64_t nvals = std::max<int64_t>(nnz, (int64_t)kEllMaxWidth * nV);
        const int64_t ws = (int64_t)pcg_layout(nV, nvals, k, sizeof(float)).total;
        b += rnd(ws + ws / 4) + rnd(320);
    }
    return b + 8192;
}

// --------------------------------------------------------------- executor

struct Bump {
    char *base = nullptr;
    int64_t cap = 0, used = 0;
};

void *bump_alloc(size_t bytes, dgo_stream, void *ctx) {
    Bump *b = (Bump *)ctx;
    const int64_t need = rnd((int64_t)bytes);
    if (b->used + need > b->cap) return nullptr;
    void *p = b->base + b->used;
    b->used += need;
    return p;
}

void bump_free(void *, dgo_stream, void *) {}  // the request's range is released whole

struct ReqDev {
    Bump bump;
    dgo_mesh *mesh = nullptr;
    SrvDesc desc{};
};

class GpuExec {
  public:
    explicit GpuExec(const dgo_server_opts &o) : o_(o) {}

    dgo_status init() {
        DGO_HIP(hipGetDevice(&dev_));
        DGO_HIP(hipMalloc(&arena_, (size_t)o_.hbm_budget_bytes));
        DGO_HIP(hipStreamCreateWithFlags(&cs_, hipStreamNonBlocking));
        DGO_HIP(hipStreamCreateWithFlags(&xs_, hipStreamNonBlocking));
        const size_t db = sizeof(SrvHdr) + sizeof(SrvDesc) * kSrvMaxSlots;
        DGO_HIP(hipHostMalloc(&h_desc_, db, hipHostMallocDefault));
        DGO_HIP(hipMalloc(&d_desc_, db));
        DGO_HIP(hipMalloc(&d_ndeg_, 256));
        DGO_HIP(hipMemset(d_ndeg_, 0, 256));
        return DGO_OK;
    }

    ~GpuExec() {
        if (graph_) (void)hipGraphExecDestroy(graph_);
        for (auto &kv : prep_)
            if (kv.second->stream) (void)hipStreamDestroy(kv.second->stream);
        if (cs_) (void)hipStreamDestroy(cs_);
        if (xs_) (void)hipStreamDestroy(xs_);
        if (h_desc_) (void)hipHostFree(h_desc_);
        if (d_desc_) (void)hipFree(d_desc_);
        if (d_ndeg_) (void)hipFree(d_ndeg_);
        if (arena_) (void)hipFree(arena_);
    }

    int64_t footprint(const dgo_request &r) const {
        return footprint_of(r.nV, r.nF, r.k, o_.batched == 0);
    }

    dgo_status prepare(srv::Req &q) {
        (void)hipSetDevice(dev_);
        PrepCtx *pc = prep_ctx();
        if (!pc || !pc->stream) return DGO_ERR_DEVICE;
        hipStream_t ps = pc->stream;
        // every return drains the stream first: on a failure the scheduler
        // releases the request's arena range and its caller may free its
        // host buffers, so no copy or kernel of it may still be in flight
        struct Drain {
            hipStream_t s;
            ~Drain() { (void)hipStreamSynchronize(s); }
        } drain{ps};
        ReqDev *rd = new (std::nothrow) ReqDev();
        if (!rd) return DGO_ERR_NOMEM;
        q.exec = rd;
        rd->bump.base = (char *)arena_ + q.arena_off;
        rd->bump.cap = q.footprint;
        const dgo_request &in = q.in;
        const int64_t nV = in.nV, k = in.k;
        auto take = [&](int64_t bytes) { return bump_alloc((size_t)bytes, nullptr, &rd->bump); };
        int32_t *dF = (int32_t *)take(12 * in.nF);
        R *dX = (R *)take(12 * nV);
        R *df = (R *)take(4 * nV * k);
        if (!dF || !dX || !df) return DGO_ERR_NOMEM;
        // the inputs go through this thread's pinned staging buffer (the
        // caller's arrays are pageable)
        const size_t bF = 12 * (size_t)in.nF, bX = 12 * (size_t)nV, bf = 4 * (size_t)(nV * k);
        char *stage = (char *)pc->staging(bF + bX + bf);
        if (!stage) return DGO_ERR_NOMEM;
        memcpy(stage, in.h_F, bF);
        memcpy(stage + bF, in.h_X, bX);
        memcpy(stage + bF + bX, in.h_f, bf);
        DGO_HIP(hipMemcpyAsync(dF, stage, bF, hipMemcpyHostToDevice, ps));
        DGO_HIP(hipMemcpyAsync(dX, stage + bF, bX, hipMemcpyHostToDevice, ps));
        DGO_HIP(hipMemcpyAsync(df, stage + bF + bX, bf, hipMemcpyHostToDevice, ps));
        dgo_allocator al{bump_alloc, bump_free, &rd->bump};
        // the batched kernels read the CSR directly; the one-at-a-time
        // baseline goes through the SpMV entry points, which need row
        // descriptors (natural order: no host-side reordering per request)
        dgo_status st = mesh_create(2, in.nV, in.nF, dF, &al, ps, ROWS_NATURAL,
                                    o_.batched ? kSrvLdsBytes : 0, &rd->mesh);
        if (st != DGO_OK) return st;
        dgo_mesh *m = rd->mesh;
        SrvDesc &D = rd->desc;
        D.view = view_of(m);
        D.diag = m->diag;
        D.ell_col = m->ell_col;
        D.ell_src = m->ell_src;
        D.ell_w = m->ell_w;
        D.nnz = m->nnz;
        D.X = dX;
        D.f = df;
        D.k = in.k;
        D.KP = pow2ceil(in.k);
        const int G = D.KP < 8 ? 8 : D.KP;
        D.tiles_v = (int32_t)tiles_for(in.nV, T / D.KP);
        D.tiles_s = (int32_t)tiles_for(in.nV, T / G);
        D.units_v = (D.tiles_v + kSrvTilesPerUnit - 1) / kSrvTilesPerUnit;
        D.units_s = (D.tiles_s + kSrvTilesPerUnit - 1) / kSrvTilesPerUnit;
        D.nblocks = m->nblocks;
        D.K = (R *)take(4 * m->nnz);
        D.M = (R *)take(4 * nV);
        D.u = (R *)take(4 * nV * k);
        D.r = (R *)take(4 * nV * k);
        D.p = (R *)take(4 * nV * k);
        D.s = (R *)take(4 * nV * k);
        D.w = (R *)take(4 * nV * k);
        D.invD = (R *)take(4 * nV);
        D.v = (R *)take(4 * (m->ell_w ? (int64_t)m->ell_w * nV : m->nnz));
        D.part = (double *)take(8 * 3 * k * (int64_t)D.units_v);
        D.part2 = (double *)take(8 * k * (int64_t)D.units_s);
        D.st = (CgCol *)take((int64_t)sizeof(CgCol) * k);
        if (!D.K || !D.M || !D.u || !D.r || !D.p || !D.s || !D.w || !D.invD || !D.v || !D.part ||
            !D.part2 || !D.st)
            return DGO_ERR_NOMEM;
        DGO_HIP(hipStreamSynchronize(ps));
        return DGO_OK;
    }

    dgo_status tick(std::vector<srv::Req *> &active, int32_t chunk) {
        (void)hipSetDevice(dev_);
        if (o_.batched == 0) return tick_single(active);
        const int n = (int)active.size();
        SrvHdr *h = (SrvHdr *)h_desc_;
        SrvDesc *hd = (SrvDesc *)((char *)h_desc_ + sizeof(SrvHdr));
        int32_t oa = 0, os = 0, ov = 0;
        for (int i = 0; i < n; ++i) {
            srv::Req *q = active[i];
            ReqDev *rd = (ReqDev *)q->exec;
            SrvDesc D = rd->desc;
            D.init = q->initialised ? 0 : 1;
            D.iters = std::min(chunk, q->target - q->done_iters);
            D.off_a = oa;
            D.off_s = os;
            D.off_v = ov;
            oa += D.init ? D.nblocks : 0;
            os += D.units_s;
            ov += D.units_v;
            hd[i] = D;
        }
        *h = SrvHdr{n, oa, os, ov};
        const size_t bytes = sizeof(SrvHdr) + sizeof(SrvDesc) * n;
        DGO_HIP(hipMemcpyAsync(d_desc_, h_desc_, bytes, hipMemcpyHostToDevice, cs_));
        const bool use_graph = !trace_active() && !(getenv("DGO_SERVE_GRAPH") && atoi(getenv("DGO_SERVE_GRAPH")) == 0);
        if (use_graph) {
            if (!graph_ || graph_chunk_ != chunk) {
                if (graph_) (void)hipGraphExecDestroy(graph_);
                graph_ = nullptr;
                hipGraph_t g = nullptr;
                DGO_HIP(hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal));
                launch_tick(chunk);
                DGO_HIP(hipStreamEndCapture(cs_, &g));
                hipError_t e = hipGraphInstantiate(&graph_, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    graph_ = nullptr;
                    return hip_fail(e, "hipGraphInstantiate", __FILE__, __LINE__);
                }
                graph_chunk_ = chunk;
            }
            DGO_HIP(hipGraphLaunch(graph_, cs_));
        } else {
            launch_tick(chunk);
        }
        DGO_HIP(hipGetLastError());
        DGO_HIP(hipStreamSynchronize(cs_));
        for (int i = 0; i < n; ++i) active[i]->done_iters += hd[i].iters;
        return DGO_OK;
    }

    // On the completion thread, after the tick that finished the request has
    // completed; its own stream lets the copy overlap the next tick.
    dgo_status finish(srv::Req &q) {
        ReqDev *rd = (ReqDev *)q.exec;
        (void)hipSetDevice(dev_);
        const size_t bytes = 4 * (size_t)q.in.nV * q.in.k;
        void *stage = res_stage_.staging(bytes);  // pinned; the caller's h_u is pageable
        if (!stage) return DGO_ERR_NOMEM;
        DGO_HIP(hipMemcpyAsync(stage, rd->desc.u, bytes, hipMemcpyDeviceToHost, xs_));
        DGO_HIP(hipStreamSynchronize(xs_));
        memcpy(q.in.h_u, stage, bytes);
        return DGO_OK;
    }

    void release(srv::Req &q) {
        ReqDev *rd = (ReqDev *)q.exec;
        if (!rd) return;
        (void)hipSetDevice(dev_);
        if (rd->mesh) dgo_mesh_destroy(rd->mesh);
        delete rd;
        q.exec = nullptr;
    }

  private:
    // Pinned host staging, grown on demand (one per preparation thread and
    // one for the completion thread; each is used by one thread only).
    struct Staging {
        void *p = nullptr;
        size_t cap = 0;
        void *staging(size_t bytes) {
            if (bytes <= cap) return p;
            if (p) (void)hipHostFree(p);
            p = nullptr;
            cap = 0;
            const size_t want = bytes + bytes / 4;
            if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                return nullptr;
            }
            cap = want;
            return p;
        }
        ~Staging() {
            if (p) (void)hipHostFree(p);
        }
    };
    struct PrepCtx : Staging {
        hipStream_t stream = nullptr;
    };

    // The calling preparation thread's stream and staging buffer (created on
    // its first request; NULL if the stream cannot be created).
    PrepCtx *prep_ctx() {
        std::lock_guard<std::mutex> lk(mu_);
        auto id = std::this_thread::get_id();
        auto it = prep_.find(id);
        if (it != prep_.end()) return it->second.get();
        auto pc = std::make_unique<PrepCtx>();
        if (hipStreamCreateWithFlags(&pc->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        PrepCtx *r = pc.get();
        prep_[id] = std::move(pc);
        return r;
    }

    void launch_tick(int32_t chunk) {
        const SrvHdr *hd = (const SrvHdr *)d_desc_;
        const SrvDesc *dd = (const SrvDesc *)((char *)d_desc_ + sizeof(SrvHdr));
        const R a = (R)o_.alpha, b = (R)o_.beta;
        CgParams prm;
        prm.rtol = 0.0;
        prm.rtol0 = 0.0;
        prm.atol = 0.0;
        prm.max_iter = o_.cg_iters;
        prm.fixed = 1;
        prm.stall = 0;
        prm.k = 0;
        const unsigned nfin = (unsigned)std::min(o_.max_slots, kSrvMaxSlots);
        DGO_LAUNCH("srv_assemble", cs_,
                   ks_assemble<<<kSrvAsmBlocks, kAssembleThreads, kSrvLdsBytes, cs_>>>(hd, dd, d_ndeg_));
        DGO_LAUNCH("srv_init", cs_, ks_init<<<kSrvBlocks, T, 0, cs_>>>(hd, dd, a, b));
        DGO_LAUNCH("srv_values", cs_, ks_values<<<kSrvAsmBlocks, T, 0, cs_>>>(hd, dd, a, b));
        DGO_LAUNCH("srv_sdot", cs_, ks_sdot<<<kSrvBlocks, T, 0, cs_>>>(hd, dd, -1));
        DGO_LAUNCH("srv_fin", cs_, ks_fin<FIN_SR_INIT><<<nfin, kFinThreads, 0, cs_>>>(hd, dd, 0, prm));
        for (int j = 0; j < chunk; ++j) {
            DGO_LAUNCH("srv_vupdate", cs_, ks_vupdate<<<kSrvBlocks, T, 0, cs_>>>(hd, dd, j));
            DGO_LAUNCH("srv_sdot", cs_, ks_sdot<<<kSrvBlocks, T, 0, cs_>>>(hd, dd, j));
            DGO_LAUNCH("srv_fin", cs_, ks_fin<FIN_SR_ITER><<<nfin, kFinThreads, 0, cs_>>>(hd, dd, j, prm));
        }
    }

    // One request with the per-mesh entry points (the baseline path).
    dgo_status tick_single(std::vector<srv::Req *> &active) {
        for (srv::Req *q : active) {
            ReqDev *rd = (ReqDev *)q->exec;
            const SrvDesc &D = rd->desc;
            dgo_stream s = (dgo_stream)cs_;
            DGO_TRY(dgo_assemble(rd->mesh, DGO_F32, 1, D.X, nullptr, D.K, D.M, nullptr, s));
            DGO_TRY(dgo_spmv(rd->mesh, DGO_F32, 1, 1.0, D.M, 0.0, D.K, D.k, D.f, D.r, s));
            DGO_HIP(hipMemsetAsync(D.u, 0, 4 * (size_t)D.view.nV * D.k, cs_));
            dgo_cg_opts co{};
            co.rtol = 0.0;
            co.max_iter = q->target;
            co.fixed_iters = 1;
            co.check_every = q->target;
            DGO_TRY(dgo_pcg(rd->mesh, DGO_F32, o_.alpha, D.M, o_.beta, D.K, nullptr, nullptr, D.k,
                            D.r, D.u, &co, nullptr, s));
            q->done_iters = q->target;
        }
        return DGO_OK;
    }

    dgo_server_opts o_;
    int dev_ = 0;
    void *arena_ = nullptr, *h_desc_ = nullptr, *d_desc_ = nullptr;
    int32_t *d_ndeg_ = nullptr;
    hipStream_t cs_ = nullptr, xs_ = nullptr;  // ticks; result copies
    hipGraphExec_t graph_ = nullptr;
    int32_t graph_chunk_ = -1;
    std::mutex mu_;
    std::unordered_map<std::thread::id, std::unique_ptr<PrepCtx>> prep_;
    Staging res_stage_;  // result copies (completion thread)
};

}  // namespace
}  // namespace dgo

using namespace dgo;

struct dgo_server {
    GpuExec *ex = nullptr;
    srv::Scheduler<GpuExec> *sch = nullptr;
};

extern "C" int64_t dgo_server_footprint(int32_t nV, int64_t nF, int32_t k) {
    if (nV < 1 || nF < 1 || k < 1) return -1;
    return footprint_of(nV, nF, k, false);
}

extern "C" dgo_status dgo_server_create(const dgo_server_opts *opts, dgo_server **out) {
    clear_error();
    if (!opts || !out) return fail(DGO_ERR_INVALID_ARG, "dgo_server_create: NULL argument");
    *out = nullptr;
    dgo_server_opts o = *opts;
    if (o.max_slots < 1 || o.max_slots > kSrvMaxSlots || o.cg_iters < 1 || o.cg_chunk < 0 ||
        o.hbm_budget_bytes <= 0 || o.prep_threads < 0)
        return fail(DGO_ERR_INVALID_ARG, "dgo_server_create: bad options");
    if (o.cg_chunk == 0 || o.cg_chunk > o.cg_iters) o.cg_chunk = o.cg_iters;
    if (o.prep_threads == 0) o.prep_threads = 2;
    if (!o.batched) {
        o.max_slots = 1;
        o.cg_chunk = o.cg_iters;
    }
    dgo_server *s = new (std::nothrow) dgo_server();
    if (!s) return fail(DGO_ERR_NOMEM, "dgo_server_create: host allocation failed");
    s->ex = new (std::nothrow) GpuExec(o);
    if (!s->ex) {
        delete s;
        return fail(DGO_ERR_NOMEM, "dgo_server_create: host allocation failed");
    }
    const dgo_status st = s->ex->init();
    if (st != DGO_OK) {
        delete s->ex;
        delete s;
        return st;
    }
    s->sch = new srv::Scheduler<GpuExec>(*s->ex, o);
    *out = s;
    return DGO_OK;
}

extern "C" dgo_status dgo_server_submit(dgo_server *s, const dgo_request *r, uint64_t *ticket) {
    clear_error();
    if (!s || !r || !ticket) return fail(DGO_ERR_INVALID_ARG, "dgo_server_submit: NULL argument");
    if (r->nV < 3 || r->nF < 1 || r->k < 1 || r->k > kSrvMaxK || !r->h_F || !r->h_X || !r->h_f ||
        !r->h_u)
        return fail(DGO_ERR_INVALID_ARG, "dgo_server_submit: bad request (nV >= 3, nF >= 1, 1 <= k <= 16, buffers)");
    const dgo_status st = s->sch->submit(*r, ticket);
    if (st == DGO_ERR_BUDGET) return fail(st, "dgo_server_submit: request larger than the HBM budget");
    if (st == DGO_ERR_SHUTDOWN) return fail(st, "dgo_server_submit: server is shutting down");
    return st;
}

extern "C" dgo_status dgo_server_wait(dgo_server *s, uint64_t ticket, double timeout_s,
                                      dgo_req_stats *st) {
    clear_error();
    if (!s) return fail(DGO_ERR_INVALID_ARG, "dgo_server_wait: NULL server");
    const dgo_status r = s->sch->wait(ticket, timeout_s, st);
    if (r == DGO_ERR_TIMEOUT) return fail(r, "dgo_server_wait: timed out");
    if (r == DGO_ERR_INVALID_ARG) return fail(r, "dgo_server_wait: unknown ticket");
    if (r != DGO_OK) return fail(r, "dgo_server_wait: the request failed");
    return r;
}

extern "C" dgo_status dgo_server_stats(dgo_server *s, dgo_server_counters *out) {
    clear_error();
    if (!s || !out) return fail(DGO_ERR_INVALID_ARG, "dgo_server_stats: NULL argument");
    s->sch->stats(out);
    return DGO_OK;
}

extern "C" void dgo_server_destroy(dgo_server *s) {
    if (!s) return;
    delete s->sch;  // drains
    delete s->ex;
    delete s;
}
