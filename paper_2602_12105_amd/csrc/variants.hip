// Operator variants on the mesh's CSR pattern: the COO form of the pattern,
// the per-element slot map, and the conformal Laplacian of the spectral conformal parameterization
// (Sec. 7.2).
//
// Conformal Laplacian: for a map u = (x, y) of the mesh into the plane, the
// conformal energy E_D - A is 1/2 u^T L_C u with L_C = [[K, -S], [S, K]]
// (unknowns ordered all x, then all y): E_D = 1/2 (x^T K x + y^T K y) the
// Dirichlet energy and A = x^T S y the signed area of the image by the
// shoelace formula over the boundary edges, S_ij = 1/2 and S_ji = -1/2 for a
// boundary edge running i -> j in its one triangle's orientation.
//
// L_C is stored as CSR over 2 nV rows: row x_i holds K's row i (columns j)
// followed by -S_ij at columns nV + j for the boundary edges at i; row y_i
// holds S_ij at columns j followed by K's row i at columns nV + j. Columns are
// sorted. The boundary orientation per CSR slot (+1: i -> j is a boundary
// edge, -1: j -> i is, 0: neither) and its per-row counts are topological:
// built once per mesh and cached. Every output entry is a copy of a K value or
// +-1/2, so the result is exact.
#include "internal.hpp"
#include "kernels.hpp"

namespace dgo {
namespace {

constexpr int T = 256;

__global__ void k_coo_rows(const int32_t *__restrict__ rowptr, int32_t nV, int32_t *__restrict__ rows) {
    const int32_t i = blockIdx.x * T + threadIdx.x;
    if (i >= nV) return;
    for (int32_t s = rowptr[i]; s < rowptr[i + 1]; ++s) rows[s] = i;
}

__global__ void k_edge_count(const int32_t *__restrict__ elem_edge, int64_t n, int32_t *__restrict__ cnt) {
    const int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n) return;
    atomicAdd(&cnt[elem_edge[o]], 1);
}

__device__ __forceinline__ int32_t slot_of(const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ col, int32_t i, int32_t j) {
    int32_t b = rowptr[i], e = rowptr[i + 1];
    while (b < e) {
        const int32_t m = (b + e) >> 1;
        if (col[m] < j) b = m + 1; else e = m;
    }
    return b;
}

// One thread per (element, local pair j): the CSR slots of (a, b) in row a and
// of (b, a) in row b. Local pairs: triangles, pair j is the edge opposite
// vertex j, (j + 1, j + 2); tetrahedra 01 02 03 12 13 23.
__global__ void k_slot_map(const int32_t *__restrict__ elem, int64_t n_elem, int dim,
                           const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           int32_t *__restrict__ slots) {
    const int nv = dim + 1, nl = dim == 2 ? 3 : 6;
    const int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_elem * nl) return;
    const int64_t e = o / nl;
    const int j = (int)(o - e * nl);
    int a, b;
    if (dim == 2) {
        a = j == 2 ? 0 : j + 1;
        b = j == 0 ? 2 : j - 1;
    } else {
        a = j < 3 ? 0 : (j < 5 ? 1 : 2);
        b = j < 3 ? j + 1 : (j < 5 ? j - 1 : 3);
    }
    const int32_t va = elem[e * nv + a], vb = elem[e * nv + b];
    slots[2 * o] = slot_of(rowptr, col, va, vb);
    slots[2 * o + 1] = slot_of(rowptr, col, vb, va);
}

// One thread per (triangle, local edge): a boundary edge (one triangle) runs
// from local vertex j + 1 to j + 2 (the edge opposite j, in the triangle's
// cyclic order). Each boundary edge has one occurrence, so every slot is
// written by at most one thread.
__global__ void k_boundary_slots(const int32_t *__restrict__ elem, const int32_t *__restrict__ elem_edge,
                                 const int32_t *__restrict__ fcount, int64_t nF,
                                 const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                 int8_t *__restrict__ bslot, int32_t *__restrict__ nb) {
    const int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= 3 * nF) return;
    if (fcount[elem_edge[o]] != 1) return;
    const int64_t f = o / 3;
    const int j = (int)(o - 3 * f);
    const int32_t a = elem[3 * f + (j == 2 ? 0 : j + 1)], b = elem[3 * f + (j == 0 ? 2 : j - 1)];
    bslot[slot_of(rowptr, col, a, b)] = 1;
    bslot[slot_of(rowptr, col, b, a)] = -1;
    atomicAdd(&nb[a], 1);
    atomicAdd(&nb[b], 1);
}

template <typename R>
__global__ void k_conformal(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            const int8_t *__restrict__ bslot, const int32_t *__restrict__ bptr,
                            int32_t nV, const R *__restrict__ K, int32_t *__restrict__ rowptr2,
                            int32_t *__restrict__ col2, R *__restrict__ val2) {
    const int32_t i = blockIdx.x * T + threadIdx.x;
    if (i >= nV) return;
    const int32_t nnz = rowptr[nV], nb = bptr[nV];
    const int32_t b = rowptr[i], e = rowptr[i + 1];
    const int32_t rx = b + bptr[i], ry = nnz + nb + b + bptr[i];
    if (rowptr2) {
        rowptr2[i] = rx;
        rowptr2[nV + i] = ry;
        if (i == nV - 1) rowptr2[2 * nV] = 2 * (nnz + nb);
    }
    int32_t px = rx, py = ry;
    for (int32_t s = b; s < e; ++s) {  // x row: K, then -S; y row: S first
        if (col2) col2[px] = col[s];
        val2[px++] = K[s];
        if (bslot[s]) {
            if (col2) col2[py] = col[s];
            val2[py++] = R(0.5) * R(bslot[s]);
        }
    }
    for (int32_t s = b; s < e; ++s) {
        if (bslot[s]) {
            if (col2) col2[px] = nV + col[s];
            val2[px++] = R(-0.5) * R(bslot[s]);
        }
        if (col2) col2[py] = nV + col[s];
        val2[py++] = K[s];
    }
}

// Cache the boundary orientation per slot and its per-row offsets.
dgo_status conformal_topology(dgo_mesh *m, hipStream_t s) {
    if (m->conf_bslot) return DGO_OK;
    const int32_t nV = m->nV;
    const int64_t nnz = m->nnz, nF = m->n_elem;
    int8_t *bslot = (int8_t *)m->alloc.get((size_t)(nnz ? nnz : 1), s);
    int32_t *bptr = (int32_t *)m->alloc.get(sizeof(int32_t) * ((size_t)nV + 1), s);
    int32_t *fc = (int32_t *)m->alloc.get(sizeof(int32_t) * (size_t)(m->nE ? m->nE : 1), s);
    const size_t st = scan_tmp_elems((int64_t)nV + 1);
    int32_t *tmp = (int32_t *)m->alloc.get(sizeof(int32_t) * (st + 1), s);
    if (!bslot || !bptr || !fc || !tmp) {
        for (void *p : {(void *)bslot, (void *)bptr, (void *)fc, (void *)tmp}) m->alloc.put(p, s);
        return fail(DGO_ERR_NOMEM, "conformal Laplacian: topology allocation failed");
    }
    DGO_HIP(hipMemsetAsync(bslot, 0, (size_t)(nnz ? nnz : 1), s));
    DGO_HIP(hipMemsetAsync(bptr, 0, sizeof(int32_t) * ((size_t)nV + 1), s));
    DGO_HIP(hipMemsetAsync(fc, 0, sizeof(int32_t) * (size_t)(m->nE ? m->nE : 1), s));
    if (nF) {
        k_edge_count<<<grid_for(3 * nF, T), T, 0, s>>>(m->elem_edge, 3 * nF, fc);
        k_boundary_slots<<<grid_for(3 * nF, T), T, 0, s>>>(m->elem, m->elem_edge, fc, nF, m->rowptr,
                                                           m->col, bslot, bptr);
    }
    DGO_HIP(hipGetLastError());
    DGO_TRY(exclusive_scan(bptr, bptr, nV, tmp, s));
    m->alloc.put(fc, s);
    m->alloc.put(tmp, s);
    m->conf_bslot = bslot;
    m->conf_bptr = bptr;
    return DGO_OK;
}

}  // namespace
}  // namespace dgo

using namespace dgo;

extern "C" dgo_status dgo_mesh_coo(const dgo_mesh *m, int32_t *d_row, int32_t *d_col,
                                   dgo_stream stream) {
    clear_error();
    if (!m || (!d_row && !d_col)) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_coo: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (d_row) k_coo_rows<<<grid_for(m->nV, T), T, 0, s>>>(m->rowptr, m->nV, d_row);
    if (d_col)
        DGO_HIP(hipMemcpyAsync(d_col, m->col, sizeof(int32_t) * (size_t)m->nnz, hipMemcpyDeviceToDevice, s));
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

extern "C" dgo_status dgo_mesh_slots(const dgo_mesh *m, int32_t *d_slots, dgo_stream stream) {
    clear_error();
    if (!m || !d_slots) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_slots: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = m->n_elem * m->nl;
    if (n) k_slot_map<<<grid_for(n, T), T, 0, s>>>(m->elem, m->n_elem, m->dim, m->rowptr, m->col, d_slots);
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

extern "C" dgo_status dgo_conformal_laplacian(const dgo_mesh *m, dgo_dtype dtype, const void *d_Kvals,
                                              int32_t *d_rowptr2, int32_t *d_col2, void *d_vals2,
                                              dgo_stream stream) {
    clear_error();
    if (!m || !d_Kvals || !d_vals2)
        return fail(DGO_ERR_INVALID_ARG, "dgo_conformal_laplacian: NULL argument");
    if (dtype != DGO_F32 && dtype != DGO_F64)
        return fail(DGO_ERR_INVALID_ARG, "dgo_conformal_laplacian: bad dtype");
    if (m->dim != 2) return fail(DGO_ERR_UNSUPPORTED, "dgo_conformal_laplacian: triangle meshes only");
    if (2 * (m->nnz + 2 * m->n_bfaces) > INT32_MAX)
        return fail(DGO_ERR_UNSUPPORTED, "dgo_conformal_laplacian: more than 2^31 entries");
    hipStream_t s = (hipStream_t)stream;
    dgo_mesh *mm = const_cast<dgo_mesh *>(m);
    DGO_TRY(conformal_topology(mm, s));
    if (dtype == DGO_F64)
        DGO_LAUNCH("conformal_laplacian", s,
                   k_conformal<double><<<grid_for(m->nV, T), T, 0, s>>>(
                       m->rowptr, m->col, m->conf_bslot, m->conf_bptr, m->nV,
                       (const double *)d_Kvals, d_rowptr2, d_col2, (double *)d_vals2));
    else
        DGO_LAUNCH("conformal_laplacian", s,
                   k_conformal<float><<<grid_for(m->nV, T), T, 0, s>>>(
                       m->rowptr, m->col, m->conf_bslot, m->conf_bptr, m->nV,
                       (const float *)d_Kvals, d_rowptr2, d_col2, (float *)d_vals2));
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}
