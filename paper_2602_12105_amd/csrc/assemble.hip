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

namespace dgo {
namespace {

constexpr int T = 256;

template <typename R>
struct V3 {
    R x, y, z;
};

template <typename R>
__device__ __forceinline__ V3<R> ld3(const R *X, int32_t v) {
    const R *p = X + 3 * (int64_t)v;
    return {p[0], p[1], p[2]};
}
template <typename R>
__device__ __forceinline__ V3<R> sub(V3<R> a, V3<R> b) {
    return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename R>
__device__ __forceinline__ R dot(V3<R> a, V3<R> b) {
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename R>
__device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename R>
__device__ __forceinline__ V3<R> axpy(R s, V3<R> a, V3<R> b) {  // s a + b
    return {s * a.x + b.x, s * a.y + b.y, s * a.z + b.z};
}

// cot of the angle at xk between (xp - xk) and (xq - xk); callers pass the
// edge endpoints (p, q) sorted by vertex id.
template <typename R>
__device__ __forceinline__ R cot_at(V3<R> xp, V3<R> xq, V3<R> xk) {
    V3<R> e1 = sub(xp, xk), e2 = sub(xq, xk);
    V3<R> n = cross(e1, e2);
    return dot(e1, e2) / sqrt(dot(n, n));
}

template <typename R>
__device__ __forceinline__ R clamp_w(R w, int use_clamp, R cmin) {
    return (use_clamp && w < cmin) ? cmin : w;
}

// Finish a row held in LDS: negate (and clamp) the off-diagonal weights and
// put their sum on the diagonal, summed in column order.
template <typename R>
__device__ __forceinline__ void finish_row(R *acc, const int32_t *lcol, int32_t base, int32_t len,
                                           int32_t i, int use_clamp, R cmin) {
    R sum = 0;
    int32_t dslot = 0;
    for (int32_t t = 0; t < len; ++t) {
        if (lcol[base + t] == i) {
            dslot = t;
            continue;
        }
        R w = clamp_w(acc[base + t], use_clamp, cmin);
        sum += w;
        acc[base + t] = -w;
    }
    acc[base + dslot] = sum;
}

template <typename R>
__global__ void __launch_bounds__(T)
k_assemble_tri(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
               const int32_t *__restrict__ vtptr, const uint32_t *__restrict__ inc, int32_t nV,
               int32_t rpb, int32_t nblocks, int32_t lds_span, int64_t nnz,
               const R *__restrict__ X, R *__restrict__ Kvals, R *__restrict__ Mdiag,
               int use_clamp, R cmin, int32_t *__restrict__ n_degenerate) {
    extern __shared__ __align__(16) unsigned char smem[];
    R *acc = (R *)smem;
    int32_t *lcol = (int32_t *)(acc + lds_span);
    const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
    const int64_t bt = blockIdx.y;
    X += bt * 3 * (int64_t)nV;
    Kvals += bt * nnz;
    Mdiag += bt * (int64_t)nV;
    const int32_t r0 = (int32_t)tile * rpb;
    const int32_t r1 = min(r0 + rpb, nV);
    const int32_t s0 = rowptr[r0], span = rowptr[r1] - s0;
    for (int32_t t = threadIdx.x; t < span; t += blockDim.x) {
        lcol[t] = col[s0 + t];
        acc[t] = R(0);
    }
    __syncthreads();
    const int32_t i = r0 + (int32_t)threadIdx.x;
    int ndeg = 0;
    if (i < r1) {
        const int32_t base = rowptr[i] - s0, len = rowptr[i + 1] - rowptr[i];
        const V3<R> xi = ld3(X, i);
        R m = 0;
        const int32_t q1 = vtptr[i + 1];
        for (int32_t q = vtptr[i]; q < q1; ++q) {
            const uint32_t rec = inc[q];
            const int32_t la = rec & 255u, lb = (rec >> 8) & 255u;
            const int32_t a = lcol[base + la], b = lcol[base + lb];
            const V3<R> xa = ld3(X, a), xb = ld3(X, b);
            // edge (i, a) is opposite b, edge (i, b) is opposite a
            const R cb = i < a ? cot_at(xi, xa, xb) : cot_at(xa, xi, xb);
            const R ca = i < b ? cot_at(xi, xb, xa) : cot_at(xb, xi, xa);
            acc[base + la] += R(0.5) * cb;
            acc[base + lb] += R(0.5) * ca;
            const V3<R> n = cross(sub(xa, xi), sub(xb, xi));
            const R n2 = dot(n, n);
            m += R(0.5) * sqrt(n2) / R(3);
            if (n2 == R(0) && i < a && i < b) ++ndeg;
        }
        finish_row(acc, lcol, base, len, i, use_clamp, cmin);
        Mdiag[i] = m;
    }
    if (ndeg) atomicAdd(n_degenerate, ndeg);
    __syncthreads();
    for (int32_t t = threadIdx.x; t < span; t += blockDim.x) Kvals[s0 + t] = acc[t];
}

// P1 stiffness of one tetrahedron in its own vertex order: the rows of E^{-1},
// E = [x1 - x0, x2 - x0, x3 - x0] (as columns), are the gradients of the
// barycentric functions 1..3: grad phi_1 = (e2 x e3)/det, grad phi_2 =
// (e3 x e1)/det, grad phi_3 = (e1 x e2)/det, grad phi_0 = -(sum).
template <typename R>
__device__ __forceinline__ void tet_grads(V3<R> x0, V3<R> x1, V3<R> x2, V3<R> x3, V3<R> g[4],
                                          R &vol, R &det) {
    const V3<R> e1 = sub(x1, x0), e2 = sub(x2, x0), e3 = sub(x3, x0);
    const V3<R> c23 = cross(e2, e3), c31 = cross(e3, e1), c12 = cross(e1, e2);
    det = dot(e1, c23);
    const R inv = R(1) / det;
    g[1] = {c23.x * inv, c23.y * inv, c23.z * inv};
    g[2] = {c31.x * inv, c31.y * inv, c31.z * inv};
    g[3] = {c12.x * inv, c12.y * inv, c12.z * inv};
    g[0] = {-(g[1].x + g[2].x + g[3].x), -(g[1].y + g[2].y + g[3].y),
            -(g[1].z + g[2].z + g[3].z)};
    vol = fabs(det) / R(6);
}

template <typename R>
__device__ __forceinline__ V3<R> pick(const V3<R> g[4], int p) {
    V3<R> r = g[0];
    r = p == 1 ? g[1] : r;
    r = p == 2 ? g[2] : r;
    r = p == 3 ? g[3] : r;
    return r;
}

template <typename R>
__global__ void __launch_bounds__(T)
k_assemble_tet(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
               const int32_t *__restrict__ vtptr, const uint32_t *__restrict__ inc, int32_t nV,
               int32_t rpb, int32_t nblocks, int32_t lds_span, int64_t nnz,
               const R *__restrict__ X, R *__restrict__ Kvals, R *__restrict__ Mdiag,
               int use_clamp, R cmin, int32_t *__restrict__ n_degenerate) {
    extern __shared__ __align__(16) unsigned char smem[];
    R *acc = (R *)smem;
    int32_t *lcol = (int32_t *)(acc + lds_span);
    const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
    const int64_t bt = blockIdx.y;
    X += bt * 3 * (int64_t)nV;
    Kvals += bt * nnz;
    Mdiag += bt * (int64_t)nV;
    const int32_t r0 = (int32_t)tile * rpb;
    const int32_t r1 = min(r0 + rpb, nV);
    const int32_t s0 = rowptr[r0], span = rowptr[r1] - s0;
    for (int32_t t = threadIdx.x; t < span; t += blockDim.x) {
        lcol[t] = col[s0 + t];
        acc[t] = R(0);
    }
    __syncthreads();
    const int32_t i = r0 + (int32_t)threadIdx.x;
    int ndeg = 0;
    if (i < r1) {
        const int32_t base = rowptr[i] - s0, len = rowptr[i + 1] - rowptr[i];
        const V3<R> xi = ld3(X, i);
        R m = 0;
        const int32_t q1 = vtptr[i + 1];
        for (int32_t q = vtptr[i]; q < q1; ++q) {
            const uint32_t rec = inc[q];
            const int p = (int)(rec >> 24);
            const int32_t l0 = rec & 255u, l1 = (rec >> 8) & 255u, l2 = (rec >> 16) & 255u;
            const int32_t w0 = lcol[base + l0], w1 = lcol[base + l1], w2 = lcol[base + l2];
            const V3<R> y0 = ld3(X, w0), y1 = ld3(X, w1), y2 = ld3(X, w2);
            // element order: i sits at position p, the others follow in order
            V3<R> x0 = p == 0 ? xi : y0;
            V3<R> x1 = p == 0 ? y0 : (p == 1 ? xi : y1);
            V3<R> x2 = p <= 1 ? y1 : (p == 2 ? xi : y2);
            V3<R> x3 = p <= 2 ? y2 : xi;
            V3<R> g[4];
            R vol, det;
            tet_grads(x0, x1, x2, x3, g, vol, det);
            const V3<R> gp = pick(g, p);
            // others in element order: positions o0 < o1 < o2 (skipping p)
            const int o0 = p == 0 ? 1 : 0;
            const int o1 = p <= 1 ? 2 : 1;
            const int o2 = p <= 2 ? 3 : 2;
            acc[base + l0] += -(vol * dot(gp, pick(g, o0)));
            acc[base + l1] += -(vol * dot(gp, pick(g, o1)));
            acc[base + l2] += -(vol * dot(gp, pick(g, o2)));
            m += vol / R(4);
            if (det == R(0) && i < w0 && i < w1 && i < w2) ++ndeg;
        }
        finish_row(acc, lcol, base, len, i, use_clamp, cmin);
        Mdiag[i] = m;
    }
    if (ndeg) atomicAdd(n_degenerate, ndeg);
    __syncthreads();
    for (int32_t t = threadIdx.x; t < span; t += blockDim.x) Kvals[s0 + t] = acc[t];
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
    const int32_t span = m->max_block_nnz;
    const size_t lds = (size_t)span * (sizeof(R) + sizeof(int32_t));
    dim3 grid((unsigned)m->nblocks, (unsigned)batch);
    const int uc = o && o->use_clamp ? 1 : 0;
    const R cm = o ? (R)o->clamp_min : R(0);
    if (m->dim == 2)
        DGO_LAUNCH("assemble_tri", s,
                   k_assemble_tri<R><<<grid, m->rpb, lds, s>>>(
                       m->rowptr, m->col, m->vtptr, m->inc, m->nV, m->rpb, m->nblocks, span,
                       m->nnz, (const R *)X, (R *)K, (R *)M, uc, cm, ndeg));
    else
        DGO_LAUNCH("assemble_tet", s,
                   k_assemble_tet<R><<<grid, m->rpb, lds, s>>>(
                       m->rowptr, m->col, m->vtptr, m->inc, m->nV, m->rpb, m->nblocks, span,
                       m->nnz, (const R *)X, (R *)K, (R *)M, uc, cm, ndeg));
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
