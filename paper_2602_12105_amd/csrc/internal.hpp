// Internal declarations of libdgo (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/dgo.h"

namespace dgo {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
void clear_error();

// A failed HIP call becomes DGO_ERR_DEVICE (or NOMEM) with the message kept.
dgo_status hip_fail(hipError_t e, const char *what, const char *file, int line);

#define DGO_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) return ::dgo::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define DGO_TRY(call)                          \
    do {                                       \
        dgo_status s_ = (call);                \
        if (s_ != DGO_OK) return s_;           \
    } while (0)

inline dgo_status fail(dgo_status s, const std::string &msg) {
    set_error(msg);
    return s;
}

// --------------------------------------------------------------- tracing

// Brackets one kernel launch with hipEvents when tracing is on and the name
// matches the filter (see dgo_trace_enable).
struct TraceScope {
    const char *name;
    hipStream_t stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TraceScope(const char *n, hipStream_t s);
    ~TraceScope();
};

#define DGO_LAUNCH(name, stream, ...)               \
    do {                                            \
        ::dgo::TraceScope trace_scope_(name, stream); \
        __VA_ARGS__;                                \
    } while (0)

// Timing carried by the dispatch itself: the start and stop events of
// hipExtLaunchKernel mark the kernel's own start and end (what a profiler's
// kernel trace measures), without event packets between back-to-back
// kernels. Used for the kernels whose rates are reported.
struct TracePair {
    const char *name;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    explicit TracePair(const char *n);
    ~TracePair();
};

#define DGO_LAUNCH_EXT(name, stream, kernel, grid, block, shmem, ...)                          \
    do {                                                                                       \
        ::dgo::TracePair trace_pair_(name);                                                    \
        if (trace_pair_.e0)                                                                    \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, trace_pair_.e0,          \
                                  trace_pair_.e1, 0, __VA_ARGS__);                             \
        else                                                                                   \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);               \
    } while (0)

// ------------------------------------------------------------ allocation

struct Alloc {
    dgo_allocator user{};
    bool has_user = false;
    void *get(size_t bytes, hipStream_t s) const;
    void put(void *p, hipStream_t s) const;
};

// --------------------------------------------------------------- mesh

// Rows per workgroup of the row-centric kernels and the LDS they need are
// fixed at mesh creation from the longest block of rows.
struct dgo_mesh_impl;

}  // namespace dgo

struct dgo_mesh {
    int32_t dim = 0;       // 2 or 3
    int32_t nv_elem = 0;   // 3 or 4 vertices per element
    int32_t nl = 0;        // 3 or 6 edges per element
    int32_t nV = 0;
    int64_t n_elem = 0;
    int64_t nE = 0;
    int64_t nnz = 0;
    int64_t n_inc = 0;     // vertex-element incidences = n_elem * nv_elem
    int64_t n_bfaces = 0;
    int64_t n_boundary = 0;
    int32_t max_row = 0;
    int device = 0;
    dgo::Alloc alloc;
    hipStream_t home = nullptr;  // stream of creation (used for frees)

    // device topology
    int32_t *elem = nullptr;       // n_elem x nv_elem
    int32_t *EV = nullptr;         // nE x 2
    int32_t *elem_edge = nullptr;  // n_elem x nl
    int8_t *elem_sign = nullptr;   // n_elem x nl
    int32_t *rowptr = nullptr;     // nV + 1
    int32_t *col = nullptr;        // nnz
    int32_t *diag = nullptr;       // nV, CSR slot of (i, i)
    int32_t *vtptr = nullptr;      // nV + 1, incidence offsets
    uint32_t *inc = nullptr;       // n_inc packed incidence records
    uint8_t *bmask = nullptr;      // nV boundary mask
    // row order of the SpMV kernels: position r visits row rdesc[r].x, whose
    // CSR entries start at rdesc[r].y, rlen[r] of them
    int2 *rdesc = nullptr;         // nV
    uint8_t *rlen = nullptr;       // nV
    int32_t *order = nullptr;      // nV, row at each position (NULL: natural order)
    // padded-row copy of the pattern in that order, for meshes whose rows
    // have at most kEllMaxWidth entries (ell_w = 0: none): position p's
    // entries are slots [p * ell_w, (p + 1) * ell_w), holding column
    // positions (padding: p itself) and the CSR slot of each entry (-1)
    int32_t ell_w = 0;
    int32_t *ell_col = nullptr;    // nV x ell_w
    int32_t *ell_src = nullptr;    // nV x ell_w
    // topology of the row-block VJP (built on its first call): per CSR slot
    // (i, j) the slot of (j, i) and the diagonal slot of column j; per
    // incidence (i, triangle (i, a, b)) the slots of (a, b) and (b, a)
    int32_t *vjp_mirror = nullptr;   // nnz
    int32_t *vjp_coldiag = nullptr;  // nnz
    int32_t *vjp_opp = nullptr;      // 2 x n_inc
    // element of each incidence record (built on first use by the kernels
    // that need the element itself: intrinsic assembly, divergence)
    int32_t *inc_elem = nullptr;     // n_inc
    // per corner p of triangle f, at 3 f + p: the incidence record of that
    // corner's vertex (built on first use by the divergence)
    int32_t *face_islot = nullptr;   // 3 x n_elem
    // conformal Laplacian topology (built on first use): per CSR slot (i, j)
    // +1 if i -> j is a boundary edge in its triangle's orientation, -1 if
    // j -> i is, else 0; offsets of each row's boundary entries
    int8_t *conf_bslot = nullptr;    // nnz
    int32_t *conf_bptr = nullptr;    // nV + 1

    // row blocks for the row-centric kernels
    int32_t rpb = 0;            // rows per workgroup
    int32_t nblocks = 0;        // ceil(nV / rpb)
    int32_t max_block_nnz = 0;  // largest CSR span of one block of rows
    int32_t max_block_inc = 0;  // most incidence records of one block of rows
    // the row blocks of FP32 assembly (tetrahedral meshes: twice the rows of
    // the FP64 blocks, whose LDS the FP32 terms halve; triangle meshes: the
    // same blocks as FP64)
    int32_t rpb_f32 = 0, nblocks_f32 = 0, max_block_nnz_f32 = 0, max_block_inc_f32 = 0;
    int64_t lds_budget = 0;     // LDS bytes a row block may take (0: kRowBlockLdsBytes)

    // scratch workspace reused by numeric calls (grows on demand)
    void *ws = nullptr;
    size_t ws_bytes = 0;

    // PCG progress polling: pinned host copies of the per-column state after
    // each chunk of iterations and the events that mark them (two slots)
    void *poll_host = nullptr;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
};

namespace dgo {

// True while kernel tracing is enabled (the serving loop then launches
// directly instead of replaying graphs).
bool trace_active();

// Build a mesh (dgo_mesh_create). `rows` selects the row descriptors of the
// SpMV kernels: none (a mesh swept only by the serving loop's batched
// kernels, which never reach the SpMV entry points), natural order, or
// automatic (breadth-first order for meshes of at least kRowOrderMinRows
// vertices, natural below).
enum RowsMode { ROWS_NONE = 0, ROWS_NATURAL = 1, ROWS_AUTO = 2 };
constexpr int32_t kRowOrderMinRows = 16384;
// Most elements at one vertex that a mesh may have: every manifold mesh whose
// vertices have at most 254 neighbours stays below it (a vertex of degree d
// lies in at most d triangles, or 2 d - 4 tetrahedra).
constexpr int32_t kMaxVertexElems = 1024;
constexpr int32_t kEllMaxWidth = 16;
// lds_budget: the LDS bytes one row block of the assembly may take (0: the
// default, kRowBlockLdsBytes); rows per block are halved until it fits.
dgo_status mesh_create(int32_t dim, int32_t nV, int64_t n_elem, const int32_t *d_elem,
                       const dgo_allocator *alloc, hipStream_t s, RowsMode rows,
                       int64_t lds_budget, dgo_mesh **out);

// Workspace of one PCG solve (byte offsets): vectors r, p, s, w, the
// effective right-hand side and x in row order, D^-1 in natural and in row
// order, the scaled operator values, workgroup partial sums (two alternating
// arrays of the vector update, one of the SpMV), the per-column state (two
// alternating copies) and the true residuals.
struct PcgLayout {
    size_t off_r, off_p, off_s, off_w, off_b, off_x, off_d, off_dp, off_v, off_pt, off_pt2, off_st,
        off_tr, total;
};
// nvals: operator values stored per solve (nnz, or nV x ell_w)
PcgLayout pcg_layout(int64_t nV, int64_t nvals, int k, size_t elem);


// Grow the mesh workspace to at least `bytes`; contents are not preserved.
dgo_status mesh_workspace(dgo_mesh *m, size_t bytes, hipStream_t s, void **out);

// Build m->inc_elem if it is not there yet (stream-ordered on s).
dgo_status mesh_inc_elem(dgo_mesh *m, hipStream_t s);

// Exclusive prefix sum of n int32 values into out[0..n]; out[n] = total.
// `tmp` must hold scan_tmp_elems(n) int32. in and out may alias.
size_t scan_tmp_elems(int64_t n);
dgo_status exclusive_scan(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp,
                          hipStream_t s);

// Row blocks of the assembly kernels: rows per workgroup (a power of two of
// at most 64, halved to fit the LDS budget) and the LDS a block needs: the
// block's CSR span (values and column ids), one record and CW contributions
// per incidence, and the block's row and incidence offsets.
constexpr int32_t kRowsPerBlockTri = 64;
// tets: 16 rows per block in FP64 (32 rows: 4 instead of 8 resident blocks per
// CU, 1.40 -> 1.60 ms at the Kuhn cube 160^3), 32 in FP32 (still 8 per CU, and
// phase B on 32 lanes: 1.30 -> 0.84 ms; 64 rows: 1.11 ms)
constexpr int32_t kRowsPerBlockTet = 16;
constexpr int32_t kRowsPerBlockTetF32 = 32;
constexpr int64_t kRowBlockLdsBytes = 64 * 1024;
constexpr int kAssembleThreads = 256;

inline int64_t assembly_lds_bytes(int dim, int s, int64_t rpb, int64_t span, int64_t ninc) {
    const int cw = dim == 2 ? 3 : 4;
    // + the per-row shift of the contribution records (cw / 2 values a row)
    return span * (s + 4) + ninc * (cw * s + 4) + rpb * (cw / 2) * s + 2 * (rpb + 1) * 4 + 64;
}

inline unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : g);
}

// Map a workgroup id to a logical tile so that each of the 8 XCDs (which get
// workgroups round-robin) works on one contiguous range of tiles: neighbouring
// tiles then share an L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nb) {
    constexpr uint32_t NX = 8;
    uint32_t per = nb / NX, rem = nb % NX;
    uint32_t x = bid % NX, q = bid / NX;
    // XCD x receives tiles [start_x, start_x + count_x)
    uint32_t start = x * per + (x < rem ? x : rem);
    uint32_t count = per + (x < rem ? 1u : 0u);
    return q < count ? start + q : bid;  // bid >= NX*per + rem cannot happen
}

}  // namespace dgo
