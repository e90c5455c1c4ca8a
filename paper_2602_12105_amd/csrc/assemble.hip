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


// P1 stiffness of one tetrahedron in its own vertex order: the rows of E^{-1},
// E = [x1 - x0, x2 - x0, x3 - x0] (as columns), are the gradients of the
// barycentric functions 1..3: grad phi_1 = (e2 x e3)/det, grad phi_2 =
// (e3 x e1)/det, grad phi_3 = (e1 x e2)/det, grad phi_0 = -(sum).
template <typename R>
struct TetG {
    V3<R> g0, g1, g2, g3;
    R vol, det;
};

template <typename R>
__device__ __forceinline__ TetG<R> tet_grads(V3<R> x0, V3<R> x1, V3<R> x2, V3<R> x3) {
    const V3<R> e1 = sub(x1, x0), e2 = sub(x2, x0), e3 = sub(x3, x0);
    const V3<R> c23 = cross(e2, e3), c31 = cross(e3, e1), c12 = cross(e1, e2);
    TetG<R> t;
    t.det = dot(e1, c23);
    const R inv = R(1) / t.det;
    t.g1 = {c23.x * inv, c23.y * inv, c23.z * inv};
    t.g2 = {c31.x * inv, c31.y * inv, c31.z * inv};
    t.g3 = {c12.x * inv, c12.y * inv, c12.z * inv};
    t.g0 = {-(t.g1.x + t.g2.x + t.g3.x), -(t.g1.y + t.g2.y + t.g3.y),
            -(t.g1.z + t.g2.z + t.g3.z)};
    t.vol = fabs(t.det) / R(6);
    return t;
}

// One of four scalars by index, as a chain of conditional moves.
template <typename R>
__device__ __forceinline__ R sel4(int p, R a, R b, R c, R d) {
    R r = a;
    r = p == 1 ? b : r;
    r = p == 2 ? c : r;
    r = p == 3 ? d : r;
    return r;
}

template <typename R>
__device__ __forceinline__ V3<R> sel2v(bool c, V3<R> a, V3<R> b) {
    return {c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}

// LDS layout of the assembly kernels for one block of rows [r0, r1). Arrays
// of records are stored field-major (structure of arrays) so that lanes
// touching consecutive entries hit consecutive banks:
//   acc  : R[span]          the block's CSR values (accumulated, then finished)
//   cw   : R[CW][inc_max]   per-incidence contributions (phase A)
//   xl   : R[3][span_max]   positions of the column vertex of each CSR entry
//   xo   : R[3][rpb]        positions of the block's own vertices
//   lcol : int32[span]      the block's column ids
//   lrec : uint32[ninc]     the block's incidence records
//   lrp  : int32[rpb + 1]   row offsets into the span
//   lvt  : int32[rpb + 1]   row offsets into the incidence records
// Every position an element needs is a column of the row it is accumulated
// into, so phase A reads positions from LDS only: X is gathered once per CSR
// entry of the block (coalesced in the CSR order) instead of three times per
// incidence.
template <typename R, int CW>
struct BlockLds {
    R *acc, *cw, *xl, *xo;
    int32_t *lcol, *lrp, *lvt;
    uint32_t *lrec;
    int32_t inc_max, span_max, rpb;
    __device__ BlockLds(unsigned char *smem, int32_t span_max_, int32_t inc_max_, int32_t rpb_)
        : inc_max(inc_max_), span_max(span_max_), rpb(rpb_) {
        acc = (R *)smem;
        cw = acc + span_max;
        xl = cw + (size_t)inc_max * CW;
        xo = xl + (size_t)span_max * 3;
        lcol = (int32_t *)(xo + (size_t)rpb * 3);
        lrec = (uint32_t *)(lcol + span_max);
        lrp = (int32_t *)(lrec + inc_max);
        lvt = lrp + rpb + 1;
    }
    __device__ R &c(int f, int32_t q) { return cw[(size_t)f * inc_max + q]; }
    __device__ V3<R> pos(int32_t j) const {
        return {xl[j], xl[span_max + j], xl[2 * span_max + j]};
    }
    __device__ V3<R> own(int32_t r) const { return {xo[r], xo[rpb + r], xo[2 * rpb + r]}; }
};

// Row of incidence q within the block: the r with lvt[r] <= q < lvt[r + 1].
__device__ __forceinline__ int32_t row_of(const int32_t *lvt, int32_t nrows, int32_t q) {
    int32_t lo = 0, hi = nrows;  // invariant: lvt[lo] <= q < lvt[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (lvt[mid] <= q) lo = mid; else hi = mid;
    }
    return lo;
}

// Phase A runs one thread per (vertex, element) incidence of the block and
// stores the element's terms for that vertex's row; phase B runs one thread
// per row and adds them in incidence (ascending element) order.
template <typename R, int DIM>
__global__ void __launch_bounds__(kAssembleThreads)
k_assemble(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
           const int32_t *__restrict__ vtptr, const uint32_t *__restrict__ inc, int32_t nV,
           int32_t rpb, int32_t nblocks, int32_t span_max, int32_t inc_max, int64_t nnz,
           const R *__restrict__ X, R *__restrict__ Kvals, R *__restrict__ Mdiag, int use_clamp,
           R cmin, int32_t *__restrict__ n_degenerate) {
    constexpr int CW = DIM == 2 ? 3 : 4;
    extern __shared__ __align__(16) unsigned char smem[];
    BlockLds<R, CW> L(smem, span_max, inc_max, rpb);
    const uint32_t tile = xcd_tile(blockIdx.x, nblocks);
    const int64_t bt = blockIdx.y;
    X += bt * 3 * (int64_t)nV;
    Kvals += bt * nnz;
    Mdiag += bt * (int64_t)nV;
    const int32_t r0 = (int32_t)tile * rpb;
    const int32_t r1 = min(r0 + rpb, nV), nrows = r1 - r0;
    const int32_t s0 = rowptr[r0], span = rowptr[r1] - s0;
    const int32_t q0 = vtptr[r0], ninc = vtptr[r1] - q0;
    const int t = threadIdx.x;
    for (int32_t j = t; j <= nrows; j += blockDim.x) {
        L.lrp[j] = rowptr[r0 + j] - s0;
        L.lvt[j] = vtptr[r0 + j] - q0;
    }
    for (int32_t j = t; j < 3 * nrows; j += blockDim.x) {
        const int32_t r = j / 3, c = j - 3 * r;
        L.xo[c * rpb + r] = X[3 * (int64_t)r0 + j];
    }
    for (int32_t j = t; j < span; j += blockDim.x) {
        const int32_t c = col[s0 + j];
        L.lcol[j] = c;
        L.acc[j] = R(0);
        L.xl[j] = X[3 * (int64_t)c];
        L.xl[span_max + j] = X[3 * (int64_t)c + 1];
        L.xl[2 * span_max + j] = X[3 * (int64_t)c + 2];
    }
    for (int32_t q = t; q < ninc; q += blockDim.x) L.lrec[q] = inc[q0 + q];
    __syncthreads();
    int ndeg = 0;
    // phase A: element terms per incidence, from LDS only
    for (int32_t q = t; q < ninc; q += blockDim.x) {
        const uint32_t rec = L.lrec[q];
        const int32_t rr = row_of(L.lvt, nrows, q);
        const int32_t i = r0 + rr, base = L.lrp[rr];
        const int32_t la = base + (int32_t)(rec & 255u), lb = base + (int32_t)((rec >> 8) & 255u);
        const V3<R> xi = L.own(rr);
        if (DIM == 2) {
            const int32_t a = L.lcol[la], b = L.lcol[lb];
            const V3<R> xa = L.pos(la), xb = L.pos(lb);
            // edge (i, a) is opposite b and edge (i, b) is opposite a; the
            // endpoints go in vertex-id order so both rows compute the same value
            const R cb = i < a ? cot_at(xi, xa, xb) : cot_at(xa, xi, xb);
            const R ca = i < b ? cot_at(xi, xb, xa) : cot_at(xb, xi, xa);
            const V3<R> n = cross(sub(xa, xi), sub(xb, xi));
            const R n2 = dot(n, n);
            L.c(0, q) = R(0.5) * cb;
            L.c(1, q) = R(0.5) * ca;
            L.c(2, q) = R(0.5) * sqrt(n2) / R(3);
            if (n2 == R(0) && i < a && i < b) ++ndeg;
        } else {
            const int p = (int)(rec >> 24);
            const int32_t lc = base + (int32_t)((rec >> 16) & 255u);
            const int32_t w0 = L.lcol[la], w1 = L.lcol[lb], w2 = L.lcol[lc];
            const V3<R> y0 = L.pos(la), y1 = L.pos(lb), y2 = L.pos(lc);
            // element order: i sits at position p, the others follow in order
            const V3<R> x0 = sel2v(p == 0, xi, y0);
            const V3<R> x1 = sel2v(p == 0, y0, sel2v(p == 1, xi, y1));
            const V3<R> x2 = sel2v(p <= 1, y1, sel2v(p == 2, xi, y2));
            const V3<R> x3 = sel2v(p <= 2, y2, xi);
            const TetG<R> tg = tet_grads(x0, x1, x2, x3);
            // every pair's product in one fixed operand order, then the three
            // pairs (p, other) in element order
            const R d01 = dot(tg.g0, tg.g1), d02 = dot(tg.g0, tg.g2), d03 = dot(tg.g0, tg.g3);
            const R d12 = dot(tg.g1, tg.g2), d13 = dot(tg.g1, tg.g3), d23 = dot(tg.g2, tg.g3);
            L.c(0, q) = -(tg.vol * sel4(p, d01, d01, d02, d03));
            L.c(1, q) = -(tg.vol * sel4(p, d02, d12, d12, d13));
            L.c(2, q) = -(tg.vol * sel4(p, d03, d13, d23, d23));
            L.c(3, q) = tg.vol / R(4);
            if (tg.det == R(0) && i < w0 && i < w1 && i < w2) ++ndeg;
        }
    }
    if (ndeg) atomicAdd(n_degenerate, ndeg);
    __syncthreads();
    // phase B: one thread per row adds the row's incidence terms in incidence
    // (ascending element) order, then forms the diagonal (the sum of the
    // row's weights in column order), negates the off-diagonals and stores
    // the lumped mass
    for (int32_t rr = t; rr < nrows; rr += blockDim.x) {
        const int32_t base = L.lrp[rr], len = L.lrp[rr + 1] - base, i = r0 + rr;
        R m = 0;
        for (int32_t q = L.lvt[rr]; q < L.lvt[rr + 1]; ++q) {
            const uint32_t rec = L.lrec[q];
            L.acc[base + (rec & 255u)] += L.c(0, q);
            L.acc[base + ((rec >> 8) & 255u)] += L.c(1, q);
            if (DIM == 3) L.acc[base + ((rec >> 16) & 255u)] += L.c(2, q);
            m += L.c(CW - 1, q);
        }
        R sum = 0;
        int32_t dslot = 0;
        for (int32_t u = 0; u < len; ++u) {
            if (L.lcol[base + u] == i) {
                dslot = u;
                continue;
            }
            const R w = clamp_w(L.acc[base + u], use_clamp, cmin);
            sum += w;
            L.acc[base + u] = -w;
        }
        L.acc[base + dslot] = sum;
        Mdiag[i] = m;
    }
    __syncthreads();
    for (int32_t j = t; j < span; j += blockDim.x) Kvals[s0 + j] = L.acc[j];
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
                       m->rowptr, m->col, m->vtptr, m->inc, m->nV, m->rpb, m->nblocks,
                       m->max_block_nnz, m->max_block_inc, m->nnz, (const R *)X, (R *)K, (R *)M,
                       uc, cm, ndeg));
    else
        DGO_LAUNCH("assemble_tet", s,
                   k_assemble<R, 3><<<grid, kAssembleThreads, lds, s>>>(
                       m->rowptr, m->col, m->vtptr, m->inc, m->nV, m->rpb, m->nblocks,
                       m->max_block_nnz, m->max_block_inc, m->nnz, (const R *)X, (R *)K, (R *)M,
                       uc, cm, ndeg));
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
