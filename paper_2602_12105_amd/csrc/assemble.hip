// Assembly of the cotangent stiffness K and the lumped mass M, and its
// vector-Jacobian product with respect to the vertex positions.
//
// Design: a "pull" (row-centric) formulation. One thread owns one CSR row i
// and walks the elements incident to vertex i in ascending element order,
// accumulating each element's contribution to the row's off-diagonal slots in
// LDS. A workgroup owns a contiguous block of rows, so its slots form one
// contiguous span of Kvals: the span's column ids are staged in LDS on the way
// in and the finished values leave with coalesced stores. No two threads add
// into one value: every sum has a fixed order and the output is bitwise
// deterministic (the FP64 row sums use LDS add instructions, each slot only
// by the thread of its row, in that thread's order).
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

// Threads per workgroup of the assembly kernels (rows per block and block
// LDS are fixed by the mesh): measured at the icosphere L9, the 256 x L5
// batch and the Kuhn cube 160^3 against 128 / 192 / 256 / 384 / 512 threads.
// FP64: 192 (L9 triangles 226 -> 216 us cold, tets 1149 -> 1106 us against
// 256); FP32 triangles: 128 (184 -> 150 us); FP32 tets (blocks of 32 rows):
// 256 (192: 788 -> 880 us).
template <typename R, int DIM>
constexpr int asm_threads() {
    return sizeof(R) == 8 ? 192 : (DIM == 2 ? 128 : 256);
}

template <typename R, int DIM>
__global__ void __launch_bounds__((asm_threads<R, DIM>()))
k_assemble(AsmView v, int32_t nblocks, int64_t nnz, const R *__restrict__ X,
           R *__restrict__ Kvals, R *__restrict__ Mdiag, int use_clamp, R cmin,
           int32_t *__restrict__ n_degenerate, int mass_kind) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
    const int64_t bt = blockIdx.y;
    assemble_block<R, DIM>(v, tile, X + bt * 3 * (int64_t)v.nV, Kvals + bt * nnz,
                           Mdiag + bt * (int64_t)v.nV, use_clamp, cmin, n_degenerate, smem,
                           nullptr, nullptr, mass_kind);
}

// Intrinsic variant: the same row blocks with edge lengths as input.
template <typename R>
__global__ void __launch_bounds__((asm_threads<R, 2>()))
k_assemble_intrinsic(AsmView v, int32_t nblocks, int64_t nnz, int64_t nE,
                     const int32_t *__restrict__ inc_elem, const int32_t *__restrict__ elem_edge,
                     const R *__restrict__ lengths, R *__restrict__ Kvals, R *__restrict__ Mdiag,
                     int use_clamp, R cmin, int32_t *__restrict__ n_degenerate, int mass_kind) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
    const int64_t bt = blockIdx.y;
    assemble_block<R, 2, true>(v, tile, lengths + bt * nE, Kvals + bt * nnz,
                               Mdiag + bt * (int64_t)v.nV, use_clamp, cmin, n_degenerate, smem,
                               inc_elem, elem_edge, mass_kind);
}

// ------------------------------------------------------------------- VJP

// A triangle (i, a, b)'s contribution to d loss / d x_i: gia, gib, gab are the
// loss gradients of the half-cotangent weights of edges ia, ib, ab (each half
// cot the cot of the angle opposite the edge, at b, a and i), gm the summed
// lumped-mass gradients of the three vertices (their mass is area / 3). The
// corners' derivatives share the triangle's s = |e_ia x e_ib| (twice its
// area, the same at every corner) and its edge vectors e_ia = x_a - x_i,
// e_ib = x_b - x_i, e_ab = x_b - x_a. The cot of the angle between edges e1
// and e2 of a corner is d / s with d = e1.e2, and d cot / d e1 =
// e2 / s - d (|e2|^2 e1 - d e2) / s^3 (symmetrically for e2). With d the
// corner's dot product and l the squared lengths:
//   corner b (e1 = -e_ib, e2 = -e_ab, d/dx_i = d/de1):
//     -e_ab / s - d_b (-l_ab e_ib + d_b e_ab) / s^3
//   corner a (e1 = -e_ia, e2 = e_ab):
//      e_ab / s - d_a (-l_ab e_ia - d_a e_ab) / s^3
//   corner i (e1 = e_ia, e2 = e_ib, d/dx_i = -(d/de1 + d/de2)):
//     -[(e_ia + e_ib) / s - d_i W / s^3],  W = (l_ib - d_i) e_ia + (l_ia - d_i) e_ib
//   area: d(s/2)/dx_i = -W / (2 s).
template <typename R>
__device__ __forceinline__ V3<R> vjp_corner(V3<R> xi, V3<R> xa, V3<R> xb, R gia, R gib, R gab,
                                            R gm, bool has_k, bool has_m) {
    const V3<R> eia = sub(xa, xi), eib = sub(xb, xi), eab = sub(xb, xa);
    const V3<R> n = cross(eia, eib);
    const R sn = sqrt(dot(n, n));
    const R is = R(1) / sn, is3 = is * is * is;
    const R lia = dot(eia, eia), lib = dot(eib, eib), lab = dot(eab, eab);
    const R di = dot(eia, eib);
    const V3<R> W = axpy(lib - di, eia, V3<R>{(lia - di) * eib.x, (lia - di) * eib.y,
                                              (lia - di) * eib.z});
    V3<R> g = {R(0), R(0), R(0)};
    if (has_k) {
        const R db = dot(eib, eab), da = -dot(eia, eab);
        // 1/2 cot(at b) on edge ia
        const R cb1 = R(0.5) * gia * is, cb3 = R(0.5) * gia * db * is3;
        // 1/2 cot(at a) on edge ib
        const R ca1 = R(0.5) * gib * is, ca3 = R(0.5) * gib * da * is3;
        // 1/2 cot(at i) on edge ab
        const R ci1 = R(-0.5) * gab * is, ci3 = R(-0.5) * gab * di * is3;
        g.x = -cb1 * eab.x - cb3 * (db * eab.x - lab * eib.x) + ca1 * eab.x +
              ca3 * (lab * eia.x + da * eab.x) + ci1 * (eia.x + eib.x) - ci3 * W.x;
        g.y = -cb1 * eab.y - cb3 * (db * eab.y - lab * eib.y) + ca1 * eab.y +
              ca3 * (lab * eia.y + da * eab.y) + ci1 * (eia.y + eib.y) - ci3 * W.y;
        g.z = -cb1 * eab.z - cb3 * (db * eab.z - lab * eib.z) + ca1 * eab.z +
              ca3 * (lab * eia.z + da * eab.z) + ci1 * (eia.z + eib.z) - ci3 * W.z;
    }
    if (has_m) {
        const R ga = -(gm / R(3)) * (R(0.5) * is);
        g = axpy(ga, W, g);
    }
    return g;
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
        const R gm = gM ? gMi + gM[a] + gM[b] : R(0);
        const V3<R> t = vjp_corner(xi, xa, xb, gia, gib, gab, gm, gK != nullptr, gM != nullptr);
        g = {g.x + t.x, g.y + t.y, g.z + t.z};
    }
    gX[3 * (int64_t)i + 0] = g.x;
    gX[3 * (int64_t)i + 1] = g.y;
    gX[3 * (int64_t)i + 2] = g.z;
}

// Topology of the row-block VJP, built on the mesh's first VJP call: for each
// CSR slot (i, j) the slot of (j, i) and the diagonal slot of column j; for
// each incidence (vertex i, triangle (i, a, b)) the slots of (a, b) and (b, a).
__global__ void k_vjp_topo(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ diag, const int32_t *__restrict__ vtptr,
                           const uint32_t *__restrict__ inc, int32_t nV, int32_t *__restrict__ mirror,
                           int32_t *__restrict__ coldiag, int32_t *__restrict__ opp) {
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= nV) return;
    const int32_t rb = rowptr[i], re = rowptr[i + 1];
    for (int32_t t = rb; t < re; ++t) {
        const int32_t j = col[t];
        mirror[t] = find_slot(rowptr, col, j, i);
        coldiag[t] = diag[j];
    }
    for (int32_t q = vtptr[i]; q < vtptr[i + 1]; ++q) {
        const uint32_t rec = inc[q];
        const int32_t a = col[rb + (int32_t)(rec & 255u)], b = col[rb + (int32_t)((rec >> 8) & 255u)];
        opp[2 * (int64_t)q] = find_slot(rowptr, col, a, b);
        opp[2 * (int64_t)q + 1] = find_slot(rowptr, col, b, a);
    }
}

// LDS of the row-block VJP for one block of rows [r0, r1):
//   cw   : R[3][inc_max]   per-incidence gradient contributions (phase A)
//   lgd  : R[span_max]     gK at the diagonal of each entry's column
//   lsum : R[span_max]     gK_ij + gK_ji of each entry
//   lgm  : R[span_max]     gM of each entry's column
//   xo   : R[3][rpb]       the block's own positions
//   lgii : R[rpb], lgmi : R[rpb]   gK_ii and gM_i of the block's rows
//   lcol : int32[span_max], lrec : uint32[inc_max], lopp : int32[2][inc_max],
//   lrp, lvt : int32[rpb + 1]
inline int64_t vjp_lds_bytes(int s, int64_t rpb, int64_t span, int64_t ninc) {
    return ninc * (3 * s + 12) + span * (3 * s + 4) + rpb * 5 * s + 2 * (rpb + 1) * 4 + 64;
}

// Row-block VJP: the block stages its rows' CSR span, incidence records and
// the gK, gM values they need in LDS (coalesced); phase A runs one thread per
// (vertex, triangle) incidence and forms the triangle's contribution to that
// vertex's gradient (the same terms, in the same order, as the per-row form
// above); phase B runs one thread per row and adds them in element order.
// The only gathers are the two other positions and gK of the opposite edge.
template <typename R>
__global__ void __launch_bounds__(kAssembleThreads)
k_vjp_rows(AsmView v, const int32_t *__restrict__ diag, const int32_t *__restrict__ mirror,
           const int32_t *__restrict__ coldiag, const int32_t *__restrict__ opp, int32_t nblocks,
           int64_t nnz, const R *__restrict__ X, const R *__restrict__ gK,
           const R *__restrict__ gM, R *__restrict__ gX) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t nV = v.nV, rpb = v.rpb, span_max = v.span_max, inc_max = v.inc_max;
    const int64_t bt = blockIdx.y;
    X += bt * 3 * (int64_t)nV;
    gX += bt * 3 * (int64_t)nV;
    if (gK) gK += bt * nnz;
    if (gM) gM += bt * (int64_t)nV;
    R *cw = (R *)smem;
    R *lgd = cw + 3 * (size_t)inc_max;
    R *lsum = lgd + span_max;
    R *lgm = lsum + span_max;
    R *xo = lgm + span_max;
    R *lgii = xo + 3 * (size_t)rpb;
    R *lgmi = lgii + rpb;
    int32_t *lcol = (int32_t *)(lgmi + rpb);
    uint32_t *lrec = (uint32_t *)(lcol + span_max);
    int32_t *lopp = (int32_t *)(lrec + inc_max);
    int32_t *lrp = lopp + 2 * (size_t)inc_max;
    int32_t *lvt = lrp + rpb + 1;

    const uint32_t tile = xcd_tile(blockIdx.x, (uint32_t)nblocks);
    const int32_t r0 = (int32_t)tile * rpb;
    const int32_t r1 = min(r0 + rpb, nV), nrows = r1 - r0;
    const int32_t s0 = v.rowptr[r0], span = v.rowptr[r1] - s0;
    const int32_t q0 = v.vtptr[r0], ninc = v.vtptr[r1] - q0;
    const int t = threadIdx.x;
    for (int32_t j = t; j <= nrows; j += blockDim.x) {
        lrp[j] = v.rowptr[r0 + j] - s0;
        lvt[j] = v.vtptr[r0 + j] - q0;
    }
    for (int32_t j = t; j < 3 * nrows; j += blockDim.x) {
        const int32_t r = j / 3, c = j - 3 * r;
        xo[c * rpb + r] = X[3 * (int64_t)r0 + j];
    }
    for (int32_t j = t; j < nrows; j += blockDim.x) {
        lgii[j] = gK ? gK[diag[r0 + j]] : R(0);
        lgmi[j] = gM ? gM[r0 + j] : R(0);
    }
    for (int32_t j = t; j < span; j += blockDim.x) {
        const int32_t e = s0 + j, c = v.col[e];
        lcol[j] = c;
        lsum[j] = gK ? gK[e] + gK[mirror[e]] : R(0);
        lgd[j] = gK ? gK[coldiag[e]] : R(0);
        lgm[j] = gM ? gM[c] : R(0);
    }
    for (int32_t q = t; q < ninc; q += blockDim.x) {
        lrec[q] = v.inc[q0 + q];
        lopp[q] = opp[2 * (int64_t)(q0 + q)];
        lopp[inc_max + q] = opp[2 * (int64_t)(q0 + q) + 1];
    }
    __syncthreads();
    for (int32_t q = t; q < ninc; q += blockDim.x) {
        const uint32_t rec = lrec[q];
        const int32_t rr = rec_row(rec, rpb);
        const int32_t base = lrp[rr];
        const int32_t la = base + (int32_t)(rec & 255u), lb = base + (int32_t)((rec >> 8) & 255u);
        const int32_t a = lcol[la], b = lcol[lb];
        const V3<R> xi = {xo[rr], xo[rpb + rr], xo[2 * rpb + rr]};
        const V3<R> xa = ld3(X, a), xb = ld3(X, b);
        // weight gradients: w_pq enters K_pq, K_qp with -1 and K_pp, K_qq with +1
        R gia = 0, gib = 0, gab = 0;
        if (gK) {
            gia = lgii[rr] + lgd[la] - lsum[la];
            gib = lgii[rr] + lgd[lb] - lsum[lb];
            gab = lgd[la] + lgd[lb] - gK[lopp[q]] - gK[lopp[inc_max + q]];
        }
        const R gm = gM ? lgmi[rr] + lgm[la] + lgm[lb] : R(0);
        const V3<R> g = vjp_corner(xi, xa, xb, gia, gib, gab, gm, gK != nullptr, gM != nullptr);
        cw[q] = g.x;
        cw[inc_max + q] = g.y;
        cw[2 * (size_t)inc_max + q] = g.z;
    }
    __syncthreads();
    for (int32_t rr = t; rr < nrows; rr += blockDim.x) {
        R gx = 0, gy = 0, gz = 0;
        for (int32_t q = lvt[rr]; q < lvt[rr + 1]; ++q) {
            gx += cw[q];
            gy += cw[inc_max + q];
            gz += cw[2 * (size_t)inc_max + q];
        }
        const int64_t o = 3 * (int64_t)(r0 + rr);
        gX[o] = gx;
        gX[o + 1] = gy;
        gX[o + 2] = gz;
    }
}

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

template <typename R>
dgo_status launch_assemble(const dgo_mesh *m, int32_t batch, const void *X,
                           const dgo_assemble_opts *o, void *K, void *M, int32_t *ndeg,
                           hipStream_t s) {
    const bool f32 = sizeof(R) == 4;
    const AsmView v = f32 ? view_of_f32(m) : view_of(m);
    const int32_t nblocks = f32 ? m->nblocks_f32 : m->nblocks;
    const size_t lds = (size_t)assembly_lds_bytes(m->dim, (int)sizeof(R), v.rpb, v.span_max,
                                                  v.inc_max);
    dim3 grid((unsigned)nblocks, (unsigned)batch);
    const int uc = o && o->use_clamp ? 1 : 0;
    const R cm = o ? (R)o->clamp_min : R(0);
    const int mk = o ? o->mass : 0;
    if (m->dim == 2)
    {
        auto kfn = k_assemble<R, 2>;
        DGO_LAUNCH_EXT("assemble_tri", s, kfn, grid, dim3(asm_threads<R, 2>()), (uint32_t)lds, v,
                       nblocks, m->nnz, (const R *)X, (R *)K, (R *)M, uc, cm, ndeg, mk);
    }
    else
        DGO_LAUNCH("assemble_tet", s,
                   k_assemble<R, 3><<<grid, asm_threads<R, 3>(), lds, s>>>(
                       v, nblocks, m->nnz, (const R *)X, (R *)K, (R *)M, uc, cm, ndeg, 0));
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

template <typename R>
dgo_status launch_assemble_intrinsic(const dgo_mesh *m, int32_t batch, const void *lengths,
                                     const dgo_assemble_opts *o, void *K, void *M, int32_t *ndeg,
                                     hipStream_t s) {
    const size_t lds = (size_t)assembly_lds_bytes(2, (int)sizeof(R), m->rpb, m->max_block_nnz,
                                                  m->max_block_inc);
    dim3 grid((unsigned)m->nblocks, (unsigned)batch);
    const int uc = o && o->use_clamp ? 1 : 0;
    const R cm = o ? (R)o->clamp_min : R(0);
    const int mk = o ? o->mass : 0;
    DGO_LAUNCH("assemble_intrinsic", s,
               k_assemble_intrinsic<R><<<grid, asm_threads<R, 2>(), lds, s>>>(
                   view_of(m), m->nblocks, m->nnz, m->nE, m->inc_elem, m->elem_edge,
                   (const R *)lengths, (R *)K, (R *)M, uc, cm, ndeg, mk));
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
    if (opts && (opts->mass < 0 || opts->mass > 1))
        return fail(DGO_ERR_INVALID_ARG, "dgo_assemble: mass must be 0 or 1");
    if (opts && opts->mass == 1 && m->dim != 2)
        return fail(DGO_ERR_UNSUPPORTED, "dgo_assemble: the mixed-Voronoi mass is for triangle meshes");
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

extern "C" dgo_status dgo_assemble_intrinsic(const dgo_mesh *m, dgo_dtype dtype, int32_t batch,
                                             const void *d_lengths, const dgo_assemble_opts *opts,
                                             void *d_Kvals, void *d_Mdiag, int64_t *h_n_degenerate,
                                             dgo_stream stream) {
    clear_error();
    if (!m || (!d_lengths && m->nE > 0) || !d_Kvals || !d_Mdiag)
        return fail(DGO_ERR_INVALID_ARG, "dgo_assemble_intrinsic: NULL argument");
    if (dtype != DGO_F32 && dtype != DGO_F64)
        return fail(DGO_ERR_INVALID_ARG, "dgo_assemble_intrinsic: bad dtype");
    if (batch < 1 || batch > 65535)
        return fail(DGO_ERR_INVALID_ARG, "dgo_assemble_intrinsic: batch must be in [1, 65535]");
    if (m->dim != 2)
        return fail(DGO_ERR_UNSUPPORTED, "dgo_assemble_intrinsic: triangle meshes only");
    if (opts && (opts->mass < 0 || opts->mass > 1))
        return fail(DGO_ERR_INVALID_ARG, "dgo_assemble_intrinsic: mass must be 0 or 1");
    hipStream_t s = (hipStream_t)stream;
    dgo_mesh *mm = const_cast<dgo_mesh *>(m);
    DGO_TRY(mesh_inc_elem(mm, s));
    void *ws;
    DGO_TRY(mesh_workspace(mm, 256, s, &ws));
    int32_t *ndeg = (int32_t *)ws;
    k_zero_i32<<<1, 1, 0, s>>>(ndeg);
    if (dtype == DGO_F64)
        DGO_TRY(launch_assemble_intrinsic<double>(m, batch, d_lengths, opts, d_Kvals, d_Mdiag, ndeg, s));
    else
        DGO_TRY(launch_assemble_intrinsic<float>(m, batch, d_lengths, opts, d_Kvals, d_Mdiag, ndeg, s));
    if (h_n_degenerate) {
        int32_t h = 0;
        DGO_HIP(hipMemcpyAsync(&h, ndeg, sizeof h, hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        *h_n_degenerate = h;
        if (h) return fail(DGO_ERR_DEGENERATE, "dgo_assemble_intrinsic: zero-area triangle(s)");
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
    const int es = dtype == DGO_F64 ? 8 : 4;
    const int64_t lds = vjp_lds_bytes(es, m->rpb, m->max_block_nnz, m->max_block_inc);
    if (lds <= kRowBlockLdsBytes) {
        dgo_mesh *mm = const_cast<dgo_mesh *>(m);
        if (!mm->vjp_mirror) {
            mm->vjp_mirror = (int32_t *)mm->alloc.get(sizeof(int32_t) * (size_t)m->nnz, s);
            mm->vjp_coldiag = (int32_t *)mm->alloc.get(sizeof(int32_t) * (size_t)m->nnz, s);
            mm->vjp_opp = (int32_t *)mm->alloc.get(sizeof(int32_t) * 2 * (size_t)m->n_inc, s);
            if (!mm->vjp_mirror || !mm->vjp_coldiag || !mm->vjp_opp)
                return fail(DGO_ERR_NOMEM, "dgo_assemble_vjp: topology allocation failed");
            DGO_LAUNCH("vjp_topo", s,
                       k_vjp_topo<<<grid_for(m->nV, T), T, 0, s>>>(m->rowptr, m->col, m->diag,
                                                                   m->vtptr, m->inc, m->nV,
                                                                   mm->vjp_mirror, mm->vjp_coldiag,
                                                                   mm->vjp_opp));
        }
        dim3 grid((unsigned)m->nblocks, (unsigned)batch);
        if (dtype == DGO_F64)
            DGO_LAUNCH("assemble_vjp_tri", s,
                       k_vjp_rows<double><<<grid, kAssembleThreads, (size_t)lds, s>>>(
                           view_of(m), m->diag, m->vjp_mirror, m->vjp_coldiag, m->vjp_opp,
                           m->nblocks, m->nnz, (const double *)d_X, (const double *)d_gK,
                           (const double *)d_gM, (double *)d_gX));
        else
            DGO_LAUNCH("assemble_vjp_tri", s,
                       k_vjp_rows<float><<<grid, kAssembleThreads, (size_t)lds, s>>>(
                           view_of(m), m->diag, m->vjp_mirror, m->vjp_coldiag, m->vjp_opp,
                           m->nblocks, m->nnz, (const float *)d_X, (const float *)d_gK,
                           (const float *)d_gM, (float *)d_gX));
        DGO_HIP(hipGetLastError());
        return DGO_OK;
    }
    // rows too long for the row-block form: one thread per row
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
