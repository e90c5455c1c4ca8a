// Assembly of the cotangent stiffness K and the lumped mass M, and its
// vector-Jacobian product with respect to the vertex positions.
//
// Design: a "pull" (row-centric) formulation. One thread owns one CSR row i
// and walks the elements incident to vertex i in ascending element order,
// accumulating each element's contribution to the row's off-diagonal slots in
// LDS. A workgroup owns a contiguous block of rows, so its slots form one
// contiguous span of Kvals: the span's column ids are staged in LDS on the way
// in and the finished values leave with coalesced stores. No float atomics are
// used: every sum has a fixed order and the output is bitwise deterministic.
//
// Bitwise symmetry: the weight of edge ij is summed in row i and in row j over
// the same elements in the same order, and each element term is evaluated from
// the same operands in the same order in both rows (triangle cotangents take
// the edge's endpoints sorted by vertex id; tetrahedron gradients are computed
// in the element's own vertex order), so K_ij == K_ji exactly.
#include "internal.hpp"
#include "kernels.hpp"

namespace dgo {
namespace {

using namespace kern;

template <typename R, int DIM>
__global__ void __launch_bounds__(kAssembleThreads)
k_assemble(AsmView v, int32_t nblocks, int64_t nnz, const R *__restrict__ X,
           R *__restrict__ Kvals, R *__restrict__ Mdiag, int use_clamp, R cmin,
           int32_t *__restrict__ n_degenerate) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
    const int64_t bt = blockIdx.y;
    assemble_block<R, DIM>(v, tile, X + bt * 3 * (int64_t)v.nV, Kvals + bt * nnz,
                           Mdiag + bt * (int64_t)v.nV, use_clamp, cmin, n_degenerate, smem);
}

// ------------------------------------------------------------------- VJP

template <typename R>
struct CotD {  // d cot / d e1 and d cot / d e2
    V3<R> d1, d2;
};

// cot of the angle between e1 and e2 differentiated: with d = e1.e2,
// s = |e1 x e2|: d cot/d e1 = e2/s - d (|e2|^2 e1 - d e2)/s^3, and
// symmetrically for e2.
template <typename R>
__device__ __forceinline__ CotD<R> cot_diff(V3<R> e1, V3<R> e2) {
    const V3<R> n = cross(e1, e2);
    const R s = sqrt(dot(n, n));
    const R d = dot(e1, e2), l1 = dot(e1, e1), l2 = dot(e2, e2);
    const R is = R(1) / s, ds3 = d * is * is * is;
    CotD<R> r;
    r.d1 = {e2.x * is - ds3 * (l2 * e1.x - d * e2.x), e2.y * is - ds3 * (l2 * e1.y - d * e2.y),
            e2.z * is - ds3 * (l2 * e1.z - d * e2.z)};
    r.d2 = {e1.x * is - ds3 * (l1 * e2.x - d * e1.x), e1.y * is - ds3 * (l1 * e2.y - d * e1.y),
            e1.z * is - ds3 * (l1 * e2.z - d * e1.z)};
    return r;
}

__device__ __forceinline__ int32_t find_slot(const int32_t *__restrict__ rowptr,
                                             const int32_t *__restrict__ col, int32_t i, int32_t j) {
    int32_t b = rowptr[i], e = rowptr[i + 1];
    while (b < e) {
        int32_t m = (b + e) >> 1;
        if (col[m] < j) b = m + 1; else e = m;
    }
    return b;
}

template <typename R>
__global__ void __launch_bounds__(T)
k_assemble_vjp_tri(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                   const int32_t *__restrict__ diag, const int32_t *__restrict__ vtptr,
                   const uint32_t *__restrict__ inc, int32_t nV, int32_t nblocks, int64_t nnz,
                   const R *__restrict__ X, const R *__restrict__ gK, const R *__restrict__ gM,
                   R *__restrict__ gX) {
    const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
    const int32_t i = (int32_t)tile * T + (int32_t)threadIdx.x;
    if (i >= nV) return;
    const int64_t bt = blockIdx.y;
    X += bt * 3 * (int64_t)nV;
    gX += bt * 3 * (int64_t)nV;
    if (gK) gK += bt * nnz;
    if (gM) gM += bt * (int64_t)nV;
    const V3<R> xi = ld3(X, i);
    const int32_t rb = rowptr[i];
    const R gKii = gK ? gK[diag[i]] : R(0);
    const R gMi = gM ? gM[i] : R(0);
    V3<R> g = {R(0), R(0), R(0)};
    for (int32_t q = vtptr[i]; q < vtptr[i + 1]; ++q) {
        const uint32_t rec = inc[q];
        const int32_t sia = rb + (int32_t)(rec & 255u), sib = rb + (int32_t)((rec >> 8) & 255u);
        const int32_t a = col[sia], b = col[sib];
        const V3<R> xa = ld3(X, a), xb = ld3(X, b);
        // weight gradients: w_pq enters K_pq, K_qp with -1 and K_pp, K_qq with +1
        R gia = 0, gib = 0, gab = 0;
        if (gK) {
            const R gKaa = gK[diag[a]], gKbb = gK[diag[b]];
            gia = -gK[sia] - gK[find_slot(rowptr, col, a, i)] + gKii + gKaa;
            gib = -gK[sib] - gK[find_slot(rowptr, col, b, i)] + gKii + gKbb;
            gab = -gK[find_slot(rowptr, col, a, b)] - gK[find_slot(rowptr, col, b, a)] + gKaa + gKbb;
        }
        // 1/2 cot(at b) on edge ia: e1 = xi - xb, e2 = xa - xb; d/dxi = d/de1
        const CotD<R> cb = cot_diff(sub(xi, xb), sub(xa, xb));
        g = axpy(R(0.5) * gia, cb.d1, g);
        // 1/2 cot(at a) on edge ib: e1 = xi - xa, e2 = xb - xa
        const CotD<R> ca = cot_diff(sub(xi, xa), sub(xb, xa));
        g = axpy(R(0.5) * gib, ca.d1, g);
        // 1/2 cot(at i) on edge ab: e1 = xa - xi, e2 = xb - xi; d/dxi = -(d1 + d2)
        const CotD<R> ci = cot_diff(sub(xa, xi), sub(xb, xi));
        const R hi = R(-0.5) * gab;
        g = axpy(hi, ci.d1, g);
        g = axpy(hi, ci.d2, g);
        if (gM) {
            // area = |e1 x e2|/2 with e1 = xa - xi, e2 = xb - xi:
            // d area/dxi = -[(|e2|^2 e1 - d e2) + (|e1|^2 e2 - d e1)] / (2 s)
            const V3<R> e1 = sub(xa, xi), e2 = sub(xb, xi);
            const V3<R> n = cross(e1, e2);
            const R s = sqrt(dot(n, n));
            const R d = dot(e1, e2), l1 = dot(e1, e1), l2 = dot(e2, e2);
            const R ga = -(gMi + gM[a] + gM[b]) / R(3) / (R(2) * s);
            g = axpy(ga, V3<R>{l2 * e1.x - d * e2.x + l1 * e2.x - d * e1.x,
                               l2 * e1.y - d * e2.y + l1 * e2.y - d * e1.y,
                               l2 * e1.z - d * e2.z + l1 * e2.z - d * e1.z},
                     g);
        }
    }
    gX[3 * (int64_t)i + 0] = g.x;
    gX[3 * (int64_t)i + 1] = g.y;
    gX[3 * (int64_t)i + 2] = g.z;
}

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

template <typename R>
dgo_status launch_assemble(const dgo_mesh *m, int32_t batch, const void *X,
                           const dgo_assemble_opts *o, void *K, void *M, int32_t *ndeg,
                           hipStream_t s) {
    const size_t lds = (size_t)assembly_lds_bytes(m->dim, (int)sizeof(R), m->rpb, m->max_block_nnz,
                                                  m->max_block_inc);
    dim3 grid((unsigned)m->nblocks, (unsigned)batch);
    const int uc = o && o->use_clamp ? 1 : 0;
    const R cm = o ? (R)o->clamp_min : R(0);
    if (m->dim == 2)
        DGO_LAUNCH("assemble_tri", s,
                   k_assemble<R, 2><<<grid, kAssembleThreads, lds, s>>>(
                       view_of(m), m->nblocks, m->nnz, (const R *)X, (R *)K, (R *)M, uc, cm, ndeg));
    else
        DGO_LAUNCH("assemble_tet", s,
                   k_assemble<R, 3><<<grid, kAssembleThreads, lds, s>>>(
                       view_of(m), m->nblocks, m->nnz, (const R *)X, (R *)K, (R *)M, uc, cm, ndeg));
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

}  // namespace
}  // namespace dgo

using namespace dgo;

extern "C" dgo_status dgo_assemble(const dgo_mesh *m, dgo_dtype dtype, int32_t batch,
                                   const void *d_X, const dgo_assemble_opts *opts, void *d_Kvals,
                                   void *d_Mdiag, int64_t *h_n_degenerate, dgo_stream stream) {
    clear_error();
    if (!m || !d_X || !d_Kvals || !d_Mdiag)
        return fail(DGO_ERR_INVALID_ARG, "dgo_assemble: NULL argument");
    if (dtype != DGO_F32 && dtype != DGO_F64) return fail(DGO_ERR_INVALID_ARG, "dgo_assemble: bad dtype");
    if (batch < 1 || batch > 65535) return fail(DGO_ERR_INVALID_ARG, "dgo_assemble: batch must be in [1, 65535]");
    hipStream_t s = (hipStream_t)stream;
    void *ws;
    DGO_TRY(mesh_workspace(const_cast<dgo_mesh *>(m), 256, s, &ws));
    int32_t *ndeg = (int32_t *)ws;
    k_zero_i32<<<1, 1, 0, s>>>(ndeg);
    if (dtype == DGO_F64)
        DGO_TRY(launch_assemble<double>(m, batch, d_X, opts, d_Kvals, d_Mdiag, ndeg, s));
    else
        DGO_TRY(launch_assemble<float>(m, batch, d_X, opts, d_Kvals, d_Mdiag, ndeg, s));
    if (h_n_degenerate) {
        int32_t h = 0;
        DGO_HIP(hipMemcpyAsync(&h, ndeg, sizeof h, hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        *h_n_degenerate = h;
        if (h) return fail(DGO_ERR_DEGENERATE, "dgo_assemble: zero-measure element(s)");
    }
    return DGO_OK;
}

extern "C" dgo_status dgo_assemble_vjp(const dgo_mesh *m, dgo_dtype dtype, int32_t batch,
                                       const void *d_X, const void *d_gK, const void *d_gM,
                                       void *d_gX, dgo_stream stream) {
    clear_error();
    if (!m || !d_X || !d_gX) return fail(DGO_ERR_INVALID_ARG, "dgo_assemble_vjp: NULL argument");
    if (m->dim != 2) return fail(DGO_ERR_UNSUPPORTED, "dgo_assemble_vjp: triangle meshes only");
    if (dtype != DGO_F32 && dtype != DGO_F64) return fail(DGO_ERR_INVALID_ARG, "dgo_assemble_vjp: bad dtype");
    if (batch < 1 || batch > 65535) return fail(DGO_ERR_INVALID_ARG, "dgo_assemble_vjp: bad batch");
    hipStream_t s = (hipStream_t)stream;
    int32_t nb = (int32_t)grid_for(m->nV, T);
    dim3 grid((unsigned)nb, (unsigned)batch);
    if (dtype == DGO_F64)
        DGO_LAUNCH("assemble_vjp_tri", s,
                   k_assemble_vjp_tri<double><<<grid, T, 0, s>>>(
                       m->rowptr, m->col, m->diag, m->vtptr, m->inc, m->nV, nb, m->nnz,
                       (const double *)d_X, (const double *)d_gK, (const double *)d_gM,
                       (double *)d_gX));
    else
        DGO_LAUNCH("assemble_vjp_tri", s,
                   k_assemble_vjp_tri<float><<<grid, T, 0, s>>>(
                       m->rowptr, m->col, m->diag, m->vtptr, m->inc, m->nV, nb, m->nnz,
                       (const float *)d_X, (const float *)d_gK, (const float *)d_gM,
                       (float *)d_gX));
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}
