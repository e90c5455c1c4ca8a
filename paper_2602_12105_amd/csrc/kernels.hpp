// Device code shared by the per-mesh kernels and the batched serving kernels:
// geometry helpers, the assembly of one row block, the SpMM row core, and the
// reduction and state-update pieces of PCG.
#pragma once

#include "internal.hpp"

namespace dgo {
namespace kern {

constexpr int T = 256;
constexpr int kMaxK = 64;
constexpr int kMaxBlocks = 4096; // workgroups of a streaming kernel
constexpr int kMaxRedBlocks = 512;  // workgroups of a kernel that stores partial sums
constexpr int TR = 1024;            // threads per workgroup of such a kernel
constexpr int kFinThreads = 1024;
constexpr int kVecUnroll = 1;     // rows per thread per step in the vector kernels (measured best)

struct CgCol {
    double rz, pq, alpha, beta, rr, bb, best, rr0;
    double alpha_prev;  // the step length of the column's previous update
    int32_t iters, since, active, converged;
    int32_t stalled, pad0;
};

struct CgParams {
    // stop at max(rtol ||b_eff||, atol) or (rtol0 > 0) at rtol0 ||r_0||
    double rtol, rtol0, atol;
    int32_t max_iter, fixed, stall;
    int32_t k;
};



inline int pow2ceil(int k) {
    int G = 1;
    while (G < k) G *= 2;
    return G;
}

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


// P1 stiffness of one tetrahedron in its own vertex order. With E =
// [x1 - x0, x2 - x0, x3 - x0] (as columns) and det = det E, the rows of
// E^{-1} are the gradients of the barycentric functions 1..3: grad phi_1 =
// (e2 x e3) / det, grad phi_2 = (e3 x e1) / det, grad phi_3 = (e1 x e2) / det,
// grad phi_0 = -(sum). K_pq = vol grad phi_p . grad phi_q with vol = |det| / 6
// is therefore (c_p . c_q) / (6 |det|) for the unscaled cross products c_p:
// one reciprocal scales the six products instead of the twelve gradient
// components.
template <typename R>
struct TetC {
    V3<R> c0, c1, c2, c3;  // det x (the barycentric gradients)
    R det;
};

template <typename R>
__device__ __forceinline__ TetC<R> tet_cross(V3<R> x0, V3<R> x1, V3<R> x2, V3<R> x3) {
    const V3<R> e1 = sub(x1, x0), e2 = sub(x2, x0), e3 = sub(x3, x0);
    TetC<R> t;
    t.c1 = cross(e2, e3);
    t.c2 = cross(e3, e1);
    t.c3 = cross(e1, e2);
    t.c0 = {-(t.c1.x + t.c2.x + t.c3.x), -(t.c1.y + t.c2.y + t.c3.y), -(t.c1.z + t.c2.z + t.c3.z)};
    t.det = dot(e1, t.c1);
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

// LDS layout of the assembly kernels for one block of rows [r0, r1):
//   cw   : R[inc_max][CW]   per-incidence contributions (phase A), an
//                           incidence's CW terms side by side, so that phase B
//                           reads them from one address (16-byte aligned:
//                           first); the records of the block's row r are
//                           shifted by r * SK values (SK = CW / 2: half a
//                           record), so that phase B's threads, one per row,
//                           whose records lie a row's incidence count apart
//                           (24 for interior tet rows: 768 bytes, one bank
//                           set), spread over the banks
//   acc  : R[span]          the block's CSR values (accumulated, then finished)
//   lcol : int32[span]      the block's column ids
//   lrec : uint32[ninc]     the block's incidence records
//   lrp  : int32[rpb + 1]   row offsets into the span
//   lvt  : int32[rpb + 1]   row offsets into the incidence records
// The element's vertex positions are gathered from X in phase A (they are
// L1/L2-resident: each is read by the few rows around it). Staging every
// span entry's position in LDS was measured slower: the larger footprint
// allowed fewer resident workgroups.
template <typename R, int CW>
struct BlockLds {
    R *acc, *cw;
    int32_t *lcol, *lrp, *lvt;
    uint32_t *lrec;
    int32_t inc_max, span_max, rpb;
    __device__ BlockLds(unsigned char *smem, int32_t span_max_, int32_t inc_max_, int32_t rpb_)
        : inc_max(inc_max_), span_max(span_max_), rpb(rpb_) {
        cw = (R *)smem;
        acc = cw + (size_t)inc_max * CW + (size_t)rpb * SK;
        lcol = (int32_t *)(acc + span_max);
        lrec = (uint32_t *)(lcol + span_max);
        lrp = (int32_t *)(lrec + inc_max);
        lvt = lrp + rpb + 1;
    }
    static constexpr int SK = CW / 2;
    // the terms of incidence q of the block's row r
    __device__ R *rec(int32_t q, int32_t r) { return cw + (size_t)q * CW + r * SK; }
};

// Copy n 32-bit words src[0, n) (4-byte aligned) into LDS dst[0, n) with the
// whole workgroup: the 16-byte aligned middle with 16-byte loads, the up to
// three words before and after it one by one (no load leaves [src, src + n)).
__device__ __forceinline__ void stage_words(const uint32_t *__restrict__ src, int32_t n,
                                            uint32_t *dst) {
    const int32_t t = threadIdx.x, nt = blockDim.x;
    const int32_t head = min(n, (int32_t)((4u - (uint32_t)(((uintptr_t)src >> 2) & 3u)) & 3u));
    const int32_t nv = (n - head) >> 2, tail = head + 4 * nv;
    if (t < head) dst[t] = src[t];
    if (t < n - tail) dst[tail + t] = src[tail + t];
    for (int32_t k = t; k < nv; k += nt) {
        const uint4 w = *reinterpret_cast<const uint4 *>(src + head + 4 * k);
        uint32_t *d = dst + head + 4 * k;
        d[0] = w.x;
        d[1] = w.y;
        d[2] = w.z;
        d[3] = w.w;
    }
}

// Row of an incidence record within its block: the record carries its
// vertex modulo 64 (bits 26-31), and blocks hold a power of two of at most
// 64 rows starting at a multiple of that size.
__device__ __forceinline__ int32_t rec_row(uint32_t rec, int32_t rpb) {
    return (int32_t)((rec >> 26) & (uint32_t)(rpb - 1));
}

// Phase A runs one thread per (vertex, element) incidence of the block and
// stores the element's terms for that vertex's row; phase B runs one thread
// per row and adds them in incidence (ascending element) order.
// Topology a row block needs (the mesh's CSR pattern and incidence records).
struct AsmView {
    const int32_t *rowptr, *col, *vtptr;
    const uint32_t *inc;
    int32_t nV, rpb, span_max, inc_max;
};

// Area of a triangle from its edge lengths: Heron's formula in Kahan's
// numerically stable arrangement (lengths sorted a >= b >= c). Sorting makes
// the result independent of the order the lengths are passed in, so every
// row that needs a triangle's area computes the same bits. Lengths that
// violate the triangle inequality give 0.
template <typename R>
__device__ __forceinline__ R heron_area(R a, R b, R c) {
    R t;
    if (a < b) { t = a; a = b; b = t; }
    if (a < c) { t = a; a = c; c = t; }
    if (b < c) { t = b; b = c; c = t; }
    const R q = (a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c));
    return q > R(0) ? R(0.25) * sqrt(q) : R(0);
}

// Half-cotangents of a triangle (i, a, b) at b and at a from the lengths li,
// la, lb of the edges opposite i, a, b (law of cosines over 8 A), and its
// area. The two squared lengths adjacent to each angle are added first: the
// sum is commutative, so the rows of both endpoints of an edge form the same
// bits, provided no product is fused into it (hence no contraction here).
// With voronoi, m is the corner's mixed-Voronoi area (the Voronoi region
// (|e_ia|^2 cot b + |e_ib|^2 cot a) / 8 when no angle is obtuse, else A/2 at
// the obtuse corner and A/4 at the others); otherwise A/3.
template <typename R>
__device__ __forceinline__ void intrinsic_terms(R li, R la, R lb, bool voronoi, R &hb, R &ha,
                                                R &A, R &m) {
#pragma clang fp contract(off)
    A = heron_area(li, la, lb);
    const R si = li * li, sa = la * la, sb = lb * lb, d = R(8) * A;
    hb = ((si + sa) - sb) / d;
    ha = ((si + sb) - sa) / d;
    if (!voronoi)
        m = A / R(3);
    else if (si > sa + sb)
        m = A / R(2);
    else if (sa > si + sb || sb > si + sa)
        m = A / R(4);
    else
        m = (sb * hb + sa * ha) / R(4);
}

// Corner mass of vertex i in triangle (i, a, b) for the mixed-Voronoi option,
// from the edge vectors at i, twice the area nn and the half-cotangents at b
// and a (hb, ha) with the dot products db, da at those corners.
template <typename R>
__device__ __forceinline__ R voronoi_corner(V3<R> eia, V3<R> eib, R nn, R hb, R ha, R db, R da) {
    if (dot(eia, eib) < R(0)) return nn / R(4);
    if (da < R(0) || db < R(0)) return nn / R(8);
    return (dot(eia, eia) * hb + dot(eib, eib) * ha) / R(4);
}

// Assemble the row block `tile` of one mesh into Kvals / Mdiag (called by the
// whole workgroup; smem holds assembly_lds_bytes of the view). INTR: X holds
// the mesh's edge lengths instead of positions (triangles only), and
// inc_elem / elem_edge give each incidence's triangle and its edges.
// mass_kind 1: mixed-Voronoi lumped mass of triangles (else barycentric).
template <typename R, int DIM, bool INTR = false>
__device__ void assemble_block(const AsmView &v, uint32_t tile, const R *__restrict__ X,
                               R *__restrict__ Kvals, R *__restrict__ Mdiag, int use_clamp,
                               R cmin, int32_t *__restrict__ n_degenerate, unsigned char *smem,
                               const int32_t *__restrict__ inc_elem = nullptr,
                               const int32_t *__restrict__ elem_edge = nullptr,
                               int mass_kind = 0) {
    static_assert(!INTR || DIM == 2, "intrinsic assembly is for triangle meshes");
    constexpr int CW = DIM == 2 ? 3 : 4;
    const int32_t *__restrict__ rowptr = v.rowptr;
    const int32_t *__restrict__ col = v.col;
    const int32_t *__restrict__ vtptr = v.vtptr;
    const uint32_t *__restrict__ inc = v.inc;
    const int32_t nV = v.nV, rpb = v.rpb, span_max = v.span_max;
    BlockLds<R, CW> L(smem, span_max, v.inc_max, rpb);
    const int32_t r0 = (int32_t)tile * rpb;
    const int32_t r1 = min(r0 + rpb, nV), nrows = r1 - r0;
    const int32_t s0 = rowptr[r0], span = rowptr[r1] - s0;
    const int32_t q0 = vtptr[r0], ninc = vtptr[r1] - q0;
    const int t = threadIdx.x;
    // intrinsic: the triangles of this thread's first two incidences are
    // loaded with the staging (they head phase A's chain of dependent loads:
    // triangle, its edges, their lengths)
    int32_t fpre0 = 0, fpre1 = 0;
    if constexpr (INTR) {
        if (t < ninc) fpre0 = inc_elem[q0 + t];
        if (t + (int32_t)blockDim.x < ninc) fpre1 = inc_elem[q0 + t + blockDim.x];
    }
    for (int32_t j = t; j <= nrows; j += blockDim.x) {
        L.lrp[j] = rowptr[r0 + j] - s0;
        L.lvt[j] = vtptr[r0 + j] - q0;
    }
    if constexpr (DIM == 2) {
        // 16-byte loads (L9 triangles 235 -> 229 us cold; the tetrahedral
        // kernel, VALU-bound, was slower with them: 1181 -> 1281 us at 160^3)
        stage_words(reinterpret_cast<const uint32_t *>(col + s0), span,
                    reinterpret_cast<uint32_t *>(L.lcol));
        stage_words(inc + q0, ninc, L.lrec);
        for (int32_t j = t; j < span; j += blockDim.x) L.acc[j] = R(0);
    } else {
        for (int32_t j = t; j < span; j += blockDim.x) {
            L.lcol[j] = col[s0 + j];
            L.acc[j] = R(0);
        }
        for (int32_t q = t; q < ninc; q += blockDim.x) L.lrec[q] = inc[q0 + q];
    }
    __syncthreads();
    int ndeg = 0;
    // phase A: element terms per incidence, from LDS only
    int32_t it = 0;  // this thread's pass over the block's incidences
    for (int32_t q = t; q < ninc; q += blockDim.x, ++it) {
        const uint32_t rec = L.lrec[q];
        const int32_t rr = rec_row(rec, rpb);
        const int32_t i = r0 + rr, base = L.lrp[rr];
        const int32_t la = base + (int32_t)(rec & 255u), lb = base + (int32_t)((rec >> 8) & 255u);
        R *cq = L.rec(q, rr);
        if constexpr (INTR) {
            // triangle (i, a, b) in cyclic order; edge ids by the rule that
            // slot j of a triangle is the edge opposite its vertex j
            const int p = (int)((rec >> 24) & 3u);
            int32_t f;
            if (it == 0)
                f = fpre0;
            else if (it == 1)
                f = fpre1;
            else
                f = inc_elem[q0 + q];
            const int32_t *fe = elem_edge + 3 * (int64_t)f;
            const int pa = p == 2 ? 0 : p + 1, pb = p == 0 ? 2 : p - 1;
            const R ei = X[fe[p]], ea = X[fe[pa]], eb = X[fe[pb]];  // opposite i, a, b
            R A;
            intrinsic_terms(ei, ea, eb, mass_kind == 1, cq[0], cq[1], A, cq[2]);
            if (A == R(0) && i < L.lcol[la] && i < L.lcol[lb]) ++ndeg;
            continue;
        }
        if (DIM == 2) {
            const int32_t a = L.lcol[la], b = L.lcol[lb];
            // |n| = 2 area is shared by the triangle's three cotangents,
            // cot = (e1 . e2) / |n|; the positions are gathered in vertex-id
            // order (the ids are sorted, not the positions), n is formed from
            // them in that order and each corner's dot product from the
            // other two in that order, so every row that needs a value
            // computes the same bits (K stays exactly symmetric)
            const bool ia = i < a, ib = i < b, ab = a < b;
            const int32_t u0 = ia ? (ib ? i : b) : (ab ? a : b);
            const int32_t u2 = ia ? (ab ? b : a) : (ib ? b : i);
            // the middle one: i if it lies between a and b, else the smaller
            // of a, b when i is the smallest and the larger when i is largest
            const int32_t u1 = ia != ib ? i : (ia == ab ? a : b);
            const V3<R> v0 = ld3(X, u0), v1 = ld3(X, u1), v2 = ld3(X, u2);
            const V3<R> n = cross(sub(v1, v0), sub(v2, v0));
            const R n2 = dot(n, n);
            const R nn = sqrt(n2);
            const R h = R(0.5) / nn;
            // the corner dot products at the sorted vertices
            const R d0 = dot(sub(v1, v0), sub(v2, v0));
            const R d1 = dot(sub(v0, v1), sub(v2, v1));
            const R d2 = dot(sub(v0, v2), sub(v1, v2));
            // edge (i, a) is opposite b, edge (i, b) is opposite a
            const int kb = (b > a) + (b > i), ka = (a > b) + (a > i);
            const R db = kb == 0 ? d0 : (kb == 1 ? d1 : d2);
            const R da = ka == 0 ? d0 : (ka == 1 ? d1 : d2);
            cq[0] = db * h;
            cq[1] = da * h;
            if (mass_kind == 1) {
                const int ki = (i > a) + (i > b);
                const V3<R> xi = sel2v(ki == 0, v0, sel2v(ki == 1, v1, v2));
                const V3<R> xa = sel2v(ka == 0, v0, sel2v(ka == 1, v1, v2));
                const V3<R> xb = sel2v(kb == 0, v0, sel2v(kb == 1, v1, v2));
                cq[2] = voronoi_corner(sub(xa, xi), sub(xb, xi), nn, db * h, da * h, db, da);
            } else {
                cq[2] = nn * (R(1) / R(6));  // area / 3
            }
            if (n2 == R(0) && ia && ib) ++ndeg;
        } else {
            const int p = (int)((rec >> 24) & 3u);
            const int32_t lc = base + (int32_t)((rec >> 16) & 255u);
            const int32_t w0 = L.lcol[la], w1 = L.lcol[lb], w2 = L.lcol[lc];
            // element order: i sits at position p, the others follow in
            // order; the ids are placed, then the positions gathered
            const int32_t id0 = p == 0 ? i : w0;
            const int32_t id1 = p == 0 ? w0 : (p == 1 ? i : w1);
            const int32_t id2 = p <= 1 ? w1 : (p == 2 ? i : w2);
            const int32_t id3 = p <= 2 ? w2 : i;
            const V3<R> x0 = ld3(X, id0), x1 = ld3(X, id1), x2 = ld3(X, id2), x3 = ld3(X, id3);
            const TetC<R> tc = tet_cross(x0, x1, x2, x3);
            const R ad = fabs(tc.det);
            const R sc = R(1) / (R(6) * ad);  // vol / det^2
            // every pair's product in one fixed operand order, then the three
            // pairs (p, other) in element order
            const R d01 = dot(tc.c0, tc.c1), d02 = dot(tc.c0, tc.c2), d03 = dot(tc.c0, tc.c3);
            const R d12 = dot(tc.c1, tc.c2), d13 = dot(tc.c1, tc.c3), d23 = dot(tc.c2, tc.c3);
            cq[0] = -(sc * sel4(p, d01, d01, d02, d03));
            cq[1] = -(sc * sel4(p, d02, d12, d12, d13));
            cq[2] = -(sc * sel4(p, d03, d13, d23, d23));
            cq[3] = ad * (R(1) / R(24));  // vol / 4
            if (tc.det == R(0) && i < w0 && i < w1 && i < w2) ++ndeg;
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
        const int32_t qe = L.lvt[rr + 1];
        int32_t q = L.lvt[rr];
        if constexpr (sizeof(R) == 8) {
            // FP64, two incidences at a time: both incidences' terms are read
            // before their adds (which read nothing back), in incidence order
            for (; q + 1 < qe; q += 2) {
                const uint32_t ra = L.lrec[q], rb = L.lrec[q + 1];
                const R *ca = L.rec(q, rr), *cb = ca + CW;
                const R a0 = ca[0], a1 = ca[1], a2 = ca[2], am = ca[CW - 1];
                const R b0 = cb[0], b1 = cb[1], b2 = cb[2], bm = cb[CW - 1];
                atomicAdd(&L.acc[base + (ra & 255u)], a0);
                atomicAdd(&L.acc[base + ((ra >> 8) & 255u)], a1);
                if (DIM == 3) atomicAdd(&L.acc[base + ((ra >> 16) & 255u)], a2);
                atomicAdd(&L.acc[base + (rb & 255u)], b0);
                atomicAdd(&L.acc[base + ((rb >> 8) & 255u)], b1);
                if (DIM == 3) atomicAdd(&L.acc[base + ((rb >> 16) & 255u)], b2);
                m += am;
                m += bm;
            }
        }
        for (; q < qe; ++q) {
            const uint32_t rec = L.lrec[q];
            // the incidence's terms are read before any add into the row's
            // slots, so that the reads go out together
            const R *cq = L.rec(q, rr);
            const R c0 = cq[0], c1 = cq[1], c2 = cq[2], cm = cq[CW - 1];
            if constexpr (sizeof(R) == 8) {
                // FP64: LDS adds without return (one LDS round trip per
                // incidence instead of two; each slot belongs to this thread
                // alone, so its adds run in this order; tets 1472 -> 1404 us
                // at the Kuhn cube 160^3). The FP32 form was measured slower.
                atomicAdd(&L.acc[base + (rec & 255u)], c0);
                atomicAdd(&L.acc[base + ((rec >> 8) & 255u)], c1);
                if (DIM == 3) atomicAdd(&L.acc[base + ((rec >> 16) & 255u)], c2);
            } else {
                L.acc[base + (rec & 255u)] += c0;
                L.acc[base + ((rec >> 8) & 255u)] += c1;
                if (DIM == 3) L.acc[base + ((rec >> 16) & 255u)] += c2;
            }
            m += cm;
        }
        // four entries at a time: their column ids and weights are read
        // before any is written back (one LDS round trip per four entries),
        // the diagonal's weight is skipped without a branch
        R sum = 0;
        int32_t dslot = 0;
        for (int32_t u0 = 0; u0 < len; u0 += 4) {
            int32_t cu[4];
            R wu[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool in = u0 + k < len;
                cu[k] = in ? L.lcol[base + u0 + k] : i;
                wu[k] = in ? L.acc[base + u0 + k] : R(0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const R w = clamp_w(wu[k], use_clamp, cmin);
                const bool dg = cu[k] == i;
                if (dg && u0 + k < len) dslot = u0 + k;
                sum = dg ? sum : sum + w;
                wu[k] = -w;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (u0 + k < len && cu[k] != i) L.acc[base + u0 + k] = wu[k];
        }
        L.acc[base + dslot] = sum;
        Mdiag[i] = m;
    }
    __syncthreads();
    for (int32_t j = t; j < span; j += blockDim.x) Kvals[s0 + j] = L.acc[j];
    __syncthreads();
}

// Contiguous chunk of tiles for this workgroup; each XCD's workgroups cover
// one contiguous range of tiles, so neighbouring rows share an L2. The
// chunks differ in length by at most one tile, so every XCD gets an equal
// share (chunks of ceil(ntiles / nb) would leave the last workgroups, and
// with them whole XCDs, without work).
__device__ __forceinline__ void tile_range(int64_t ntiles, int64_t &t0, int64_t &t1) {
    const uint32_t nb = gridDim.x;
    const uint32_t lb = xcd_tile(blockIdx.x, nb);
    t0 = (int64_t)lb * ntiles / nb;
    t1 = (int64_t)(lb + 1) * ntiles / nb;
}

// The tiles of this workgroup: t0, t0 + step, ... below t1. il = 0: the
// contiguous chunk of tile_range (step 1). il != 0: the workgroups that share
// an XCD take turns over that XCD's contiguous range (the q-th of its n
// workgroups takes tiles q, q + n, q + 2n, ... of the range), so they sweep
// the range together; rows that the gathers of nearby tiles share are then
// reused from the XCD's L2 while they are still there, where with a chunk per
// workgroup the XCD's workgroups work far apart and each chunk's rows are
// evicted by the others' before their reuse (ranges larger than the L2).
struct TileSeq {
    int64_t t0, t1, step;
};

__device__ __forceinline__ TileSeq tile_seq(int64_t ntiles, int il) {
    TileSeq q;
    if (!il) {
        tile_range(ntiles, q.t0, q.t1);
        q.step = 1;
        return q;
    }
    constexpr uint32_t NX = 8;
    const uint32_t nb = gridDim.x, per = nb / NX, rem = nb % NX;
    const uint32_t x = blockIdx.x % NX, j = blockIdx.x / NX;
    const uint32_t start = x * per + (x < rem ? x : rem), count = per + (x < rem ? 1u : 0u);
    q.t0 = (int64_t)start * ntiles / nb + j;
    q.t1 = (int64_t)(start + count) * ntiles / nb;
    q.step = count;
    return q;
}

// ------------------------------------------------------ fixed-order reduce

// Store the workgroup's W partial sums (LDS) column-major, at
// part[w * gridDim.x + blockIdx.x], so that the finalize kernel reads each
// value's partials as one contiguous run.
__device__ __forceinline__ void store_partials(const double *s_part, int W, double *part) {
    if ((int)threadIdx.x < W) part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = s_part[threadIdx.x];
}

// Finalize sums: for w < W1, tot[w] = sum over b < n1 of p1[w * n1 + b]; for
// W1 <= w < W1 + W2 the same over p2 (n2 partials per value), computed by
// the whole workgroup: value w is taken by tpw consecutive threads (tpw a
// power of two of at most 64, so they share a wavefront); thread `sub` adds
// partials sub, sub + tpw, ... in order (loads issued kFinUnroll at a time),
// and a fixed xor-shuffle tree adds the tpw subtotals. Deterministic.
constexpr int kFinUnroll = 16;

__device__ void fin_sum2(const double *__restrict__ p1, int n1, int W1,
                         const double *__restrict__ p2, int n2, int W2, double *tot) {
    const int W = W1 + W2;
    int tpw = 64;
    while (tpw > 1 && tpw * W > (int)blockDim.x) tpw >>= 1;
    const int t = threadIdx.x, w = t / tpw, sub = t % tpw;
    double s = 0.0;
    if (w < W) {
        const double *src = w < W1 ? p1 + (size_t)w * n1 : p2 + (size_t)(w - W1) * n2;
        const int n = w < W1 ? n1 : n2;
        for (int b0 = sub; b0 < n; b0 += tpw * kFinUnroll) {
            double v[kFinUnroll];
#pragma unroll
            for (int u = 0; u < kFinUnroll; ++u) {
                const int b = b0 + u * tpw;
                v[u] = b < n ? src[b] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kFinUnroll; ++u) s += v[u];
        }
    }
    for (int off = 1; off < tpw; off <<= 1) s += __shfl_xor(s, off);
    if (sub == 0 && w < W) tot[w] = s;
    __syncthreads();
}

__device__ __forceinline__ void fin_sum(const double *__restrict__ part, int nblk, int W,
                                        double *tot) {
    fin_sum2(part, nblk, W, nullptr, 0, 0, tot);
}

// Per-column sums over the workgroup of `nval` per-lane values (lanes with
// act = false give 0). Column c lives in the lanes whose index modulo CW is c
// (CW a power of two: KP in the vector kernels, the lane-group width G in the
// SpMM kernels), and c < k <= CW. Each wavefront adds its lanes of a column
// with a fixed xor-shuffle tree; thread v * k + c then adds the wavefronts'
// sums in wavefront order into s_part[v * k + c]. s_red holds
// red_scratch(blockDim.x, nval) doubles.
__host__ __device__ constexpr int red_scratch(int bt, int nval) { return (bt / 64) * nval * kMaxK; }

__device__ __forceinline__ void column_partials(const double *vals, int nval, int k, int CW,
                                                bool act, double *s_red, double *s_part) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int v = 0; v < nval; ++v) {
        double x = act ? vals[v] : 0.0;
        for (int off = CW; off < 64; off <<= 1) x += __shfl_xor(x, off);
        if (lane < k) s_red[(wv * nval + v) * k + lane] = x;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < nval * k) {
        const int v = t / k, c = t % k;
        double a = 0.0;
        for (int w = 0; w < nw; ++w) a += s_red[(w * nval + v) * k + c];
        s_part[v * k + c] = a;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ SpMM

// One row of (alpha M + beta K) x for the calling group of G lanes: row i,
// CSR entries [rb, rb + len), dterm = alpha M_i added on the diagonal entry.
// The group loads up to G entries at once (one per lane); every lane then
// takes the entries of its part (NP = G / KP parts) from its neighbours by
// cross-lane shuffles and gathers x for its column c = lane % KP, issuing the
// gathers of up to 8 entries before using any. An entry a lane does not use
// (past the row's end, or a masked column) gathers x[i, c] with coefficient
// 0. The result is meaningful in lanes lane < KP with lane < k. With NP = 1,
// *xi (if given) receives x[i, c], taken from the diagonal entry's gather.
template <typename R, int G, int KP, bool MASK>
__device__ __forceinline__ R row_apply(const int32_t *__restrict__ col, const R *__restrict__ K,
                                       R beta, R dterm, const uint8_t *__restrict__ mask,
                                       const R *__restrict__ x, int32_t i, int32_t rb,
                                       int32_t len, int k, int lane, int gbase, R *xi) {
    constexpr int NP = G / KP;
    constexpr int CH = KP < 8 ? KP : 8;  // gathers issued together
    const int c = lane % KP, part = lane / KP;
    const int cc = c < k ? c : k - 1;
    R acc = 0, self = 0;
    for (int32_t e0 = 0; e0 < len; e0 += G) {
        int32_t cj = i;
        R aj = 0;
        if (e0 + lane < len) {
            const int32_t e = rb + e0 + lane;
            const int32_t j = col[e];
            if (!MASK || !mask[j]) {
                cj = j;
                aj = beta * K[e];
                if (j == i) aj += dterm;
            }
        }
        if (KP == 1) {
            acc += aj * x[cj];
        } else {
#pragma unroll
            for (int s0 = 0; s0 < KP; s0 += CH) {
                // one lane per entry (NP = 1): a chunk past the row's end
                // holds only padding (coefficient 0), so it is skipped
                if (NP == 1 && e0 + s0 >= len) break;
                int32_t js[CH];
                R xv[CH];
#pragma unroll
                for (int s = 0; s < CH; ++s) js[s] = __shfl(cj, gbase + (s0 + s) * NP + part);
#pragma unroll
                for (int s = 0; s < CH; ++s) xv[s] = x[(int64_t)js[s] * k + cc];
#pragma unroll
                for (int s = 0; s < CH; ++s) {
                    acc += __shfl(aj, gbase + (s0 + s) * NP + part) * xv[s];
                    if (NP == 1 && js[s] == i) self = xv[s];
                }
            }
        }
    }
#pragma unroll
    for (int off = G / 2; off >= KP; off /= 2) acc += __shfl_down(acc, off, G);
    if (xi) *xi = self;
    return acc;
}

// Padded rows of at most G entries (slots [i W, i W + W), W <= G), split in
// two so that a caller can load the next row's entries while the current
// row's gathers are in flight: ell_entry loads the lane's entry (column,
// value), padding and lanes past W giving (i, 0); ell_row forms the row from
// those entries exactly as row_apply does (same operations, same order).
template <typename R>
__device__ __forceinline__ void ell_entry(const int32_t *__restrict__ col, const R *__restrict__ v,
                                          int32_t W, int32_t i, int lane, int32_t &cj, R &aj) {
    cj = i;
    aj = R(0);
    if (lane < W) {
        const int64_t e = (int64_t)i * W + lane;
        cj = col[e];
        aj = v[e];
    }
}

template <typename R, int G, int KP>
__device__ __forceinline__ R ell_row(int32_t cj, R aj, const R *__restrict__ x, int32_t i, int k,
                                     int32_t W, int lane, int gbase, R *xi) {
    constexpr int NP = G / KP;
    constexpr int CH = KP < 8 ? KP : 8;
    const int c = lane % KP, part = lane / KP;
    const int cc = c < k ? c : k - 1;
    R acc = 0, self = 0;
    if (KP == 1) {
        acc += aj * x[cj];
    } else {
#pragma unroll
        for (int s0 = 0; s0 < KP; s0 += CH) {
            if (NP == 1 && s0 >= W) break;  // only padding from here on
            int32_t js[CH];
            R xv[CH];
#pragma unroll
            for (int s = 0; s < CH; ++s) js[s] = __shfl(cj, gbase + (s0 + s) * NP + part);
#pragma unroll
            for (int s = 0; s < CH; ++s) xv[s] = x[(int64_t)js[s] * k + cc];
#pragma unroll
            for (int s = 0; s < CH; ++s) {
                acc += __shfl(aj, gbase + (s0 + s) * NP + part) * xv[s];
                if (NP == 1 && js[s] == i) self = xv[s];
            }
        }
    }
#pragma unroll
    for (int off = G / 2; off >= KP; off /= 2) acc += __shfl_down(acc, off, G);
    if (xi) *xi = self;
    return acc;
}

// 16-byte pieces of a vertex-major row: V = 16 / sizeof(R) consecutive
// columns, one dwordx4 access (the address must be 16-byte aligned).
template <typename R>
struct Piece {
    static constexpr int V = 16 / (int)sizeof(R);
    R v[V];
};

template <typename R>
__device__ __forceinline__ Piece<R> ld_piece(const R *p) {
    Piece<R> o;
    if constexpr (sizeof(R) == 8) {
        const double2 t = *reinterpret_cast<const double2 *>(p);
        o.v[0] = t.x;
        o.v[1] = t.y;
    } else {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        o.v[0] = t.x;
        o.v[1] = t.y;
        o.v[2] = t.z;
        o.v[3] = t.w;
    }
    return o;
}

template <typename R>
__device__ __forceinline__ void st_piece(R *p, const Piece<R> &o) {
    if constexpr (sizeof(R) == 8)
        *reinterpret_cast<double2 *>(p) = make_double2(o.v[0], o.v[1]);
    else
        *reinterpret_cast<float4 *>(p) = make_float4(o.v[0], o.v[1], o.v[2], o.v[3]);
}

// A row times 8 columns of x (k = 8, rows 16-byte aligned) for a group of 8
// lanes, with 16-byte gathers. The row's entries come in chunks of 8, one
// entry (cj, aj) per lane (unused lanes: a valid row and 0). In a chunk, lane
// q + LPR s (LPR = 8 / V lanes per x row) gathers columns [qV, qV + V) of
// entries s, s + NPI, s + 2 NPI, ... (NPI = 8 / LPR entries per gather
// instruction), so a chunk takes 8 / NPI gathers instead of 8; wide8_chunk
// adds them to the lane's partial sums, wide8_combine adds the NPI partial
// sums by a fixed xor tree, after which every lane of the group holds the
// row's columns [qV, qV + V), q = lane % LPR.
template <typename R>
__device__ __forceinline__ void wide8_chunk(int32_t cj, R aj, const R *__restrict__ x, int lane,
                                            int gbase, Piece<R> &acc) {
    constexpr int V = Piece<R>::V, LPR = 8 / V, NPI = 8 / LPR, NS = 8 / NPI;
    const int q = lane % LPR, sub = lane / LPR;
    int32_t js[NS];
    Piece<R> xv[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) js[s] = __shfl(cj, gbase + s * NPI + sub);
#pragma unroll
    for (int s = 0; s < NS; ++s) xv[s] = ld_piece(x + (int64_t)js[s] * 8 + q * V);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const R a = __shfl(aj, gbase + s * NPI + sub);
#pragma unroll
        for (int v = 0; v < V; ++v) acc.v[v] += a * xv[s].v[v];
    }
}

template <typename R>
__device__ __forceinline__ void wide8_combine(Piece<R> &acc) {
    constexpr int LPR = 8 / Piece<R>::V;
#pragma unroll
    for (int off = LPR; off < 8; off *= 2)
#pragma unroll
        for (int v = 0; v < Piece<R>::V; ++v) acc.v[v] += __shfl_xor(acc.v[v], off);
}

// A padded row of W <= 8 entries (loaded by ell_entry, one per lane of the
// KPW-lane group) times KPW = 8 or 16 columns of x (k = KPW, rows 16-byte
// aligned), with 16-byte gathers: lane q + LPR s (LPR = KPW / V lanes per x
// row) gathers columns [qV, qV + V) of entries s, s + NPI, ... (NPI = KPW /
// LPR entries per instruction); with 16 columns, instructions past the W
// real entries (only padding) are skipped. The NPI partial sums are added by a
// fixed xor tree;
// every lane of the group ends with the row's columns [qV, qV + V), q =
// lane % LPR. For KPW = 8 these are wide8_chunk's operations in its order.
template <typename R, int KPW>
__device__ __forceinline__ Piece<R> ell_row_wide(int32_t cj, R aj, const R *__restrict__ x,
                                                 int lane, int gbase, int32_t W) {
    constexpr int V = Piece<R>::V, LPR = KPW / V, NPI = KPW / LPR, NS = KPW / NPI;
    const int q = lane % LPR, sub = lane / LPR;
    // instructions with real entries (uniform over the group); with 8 columns
    // all are issued (a guard there slowed the 8-column iteration by 2%)
    const int ns = KPW == 8 ? NS : (W + NPI - 1) / NPI;
    int32_t js[NS];
    Piece<R> xv[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        js[s] = __shfl(cj, gbase + s * NPI + sub);
#pragma unroll
        for (int v = 0; v < V; ++v) xv[s].v[v] = R(0);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
        if (s < ns) xv[s] = ld_piece(x + (int64_t)js[s] * KPW + q * V);
    Piece<R> acc;
#pragma unroll
    for (int v = 0; v < V; ++v) acc.v[v] = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (s >= ns) break;
        const R a = __shfl(aj, gbase + s * NPI + sub);
#pragma unroll
        for (int v = 0; v < V; ++v) acc.v[v] += a * xv[s].v[v];
    }
#pragma unroll
    for (int off = LPR; off < KPW; off *= 2)
#pragma unroll
        for (int v = 0; v < V; ++v) acc.v[v] += __shfl_xor(acc.v[v], off);
    return acc;
}

// RU rows at once for one lane group, as row_apply without the mask: row u
// is i[u] with entries [rb[u], rb[u] + len[u]) and dterm[u] on the diagonal
// (PLAIN: the coefficients are the stored values as they are, beta and dterm
// unused); ok[u] = false yields 0 (i[u] must still be a valid row). The entry
// loads of all RU rows are issued before any gather, and the gathers of a
// chunk of every row before any is used, so a lane keeps RU rows in flight.
// Each row's sum is formed in the same order as row_apply's.
template <typename R, int G, int KP, int RU, bool PLAIN>
__device__ __forceinline__ void rows_apply(const int32_t *__restrict__ col,
                                           const R *__restrict__ K, R beta, const R (&dterm)[RU],
                                           const R *__restrict__ x, const int32_t (&i)[RU],
                                           const int32_t (&rb)[RU], const int32_t (&len)[RU],
                                           const bool (&ok)[RU], int k, int lane, int gbase,
                                           R (&acc)[RU], R (&xi)[RU]) {
    constexpr int NP = G / KP;
    constexpr int CH0 = KP < 8 ? KP : 8;
    constexpr int CH = CH0 / RU > 0 ? CH0 / RU : 1;  // gathers per row issued together
    const int c = lane % KP, part = lane / KP;
    const int cc = c < k ? c : k - 1;
    int32_t lmax = 0;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        acc[u] = 0;
        xi[u] = 0;
        lmax = max(lmax, ok[u] ? len[u] : 0);
    }
    for (int32_t e0 = 0; e0 < lmax; e0 += G) {
        int32_t cj[RU];
        R aj[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            cj[u] = i[u];
            aj[u] = 0;
            if (ok[u] && e0 + lane < len[u]) {
                const int32_t e = rb[u] + e0 + lane;
                const int32_t j = col[e];
                cj[u] = j;
                if (PLAIN) {
                    aj[u] = K[e];
                } else {
                    aj[u] = beta * K[e];
                    if (j == i[u]) aj[u] += dterm[u];
                }
            }
        }
        if (KP == 1) {
#pragma unroll
            for (int u = 0; u < RU; ++u) acc[u] += aj[u] * x[cj[u]];
        } else {
#pragma unroll
            for (int s0 = 0; s0 < KP; s0 += CH) {
                if (NP == 1 && e0 + s0 >= lmax) break;  // only padding from here on
                int32_t js[RU][CH];
                R xv[RU][CH];
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int s = 0; s < CH; ++s) js[u][s] = __shfl(cj[u], gbase + (s0 + s) * NP + part);
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int s = 0; s < CH; ++s) xv[u][s] = x[(int64_t)js[u][s] * k + cc];
#pragma unroll
                for (int u = 0; u < RU; ++u)
#pragma unroll
                    for (int s = 0; s < CH; ++s) {
                        acc[u] += __shfl(aj[u], gbase + (s0 + s) * NP + part) * xv[u][s];
                        if (NP == 1 && js[u][s] == i[u]) xi[u] = xv[u][s];
                    }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int off = G / 2; off >= KP; off /= 2) acc[u] += __shfl_down(acc[u], off, G);
}

// Rows of the SpMV kernels (k_spmm, k_cg_sdot) handled together by one lane
// group. Two rows in flight were measured slower on MI355X (5% on the PCG
// iteration, 4% on a 2.6M-row SpMV): the extra registers cost more than the
// overlap gains.
constexpr int kSpmvRows = 1;

// Lane layout of the vector kernels: KP lanes per row, lane c owns column c.
struct VLane {
    int c;
    bool act;
    int grp, gpb;
};

__device__ __forceinline__ VLane vlane(int k, int KP) {
    VLane v;
    v.c = threadIdx.x % KP;
    v.act = v.c < k;
    v.grp = threadIdx.x / KP;
    v.gpb = (int)blockDim.x / KP;
    return v;
}


enum FinMode {
    FIN_OUT = 3,                     // totals out (the true residual)
    FIN_SR_INIT = 4, FIN_SR_ITER = 5  // PCG state: start, after an iteration
};

// Values per column in the (first) partial-sum array of a finalize mode; the
// PCG modes read a second array of k values (w.z).
__host__ __device__ inline int fin_width(int mode, int k) {
    return (mode == FIN_SR_INIT ? 3 : (mode == FIN_SR_ITER ? 2 : 1)) * k;
}

// Stopping tests after an iteration that produced residual norm^2 rr.
__device__ inline void cg_stop_tests(CgCol &s, double rr, const CgParams &prm) {
    if (rr < s.best) {
        s.best = rr;
        s.since = 0;
    } else {
        s.since += 1;
    }
    if (!prm.fixed && (sqrt(rr) <= fmax(prm.rtol * sqrt(s.bb), prm.atol) ||
                       (prm.rtol0 > 0.0 && sqrt(rr) <= prm.rtol0 * sqrt(s.rr0)))) {
        s.converged = 1;
        s.active = 0;
    } else if (s.iters >= prm.max_iter) {
        s.active = 0;
    } else if (!prm.fixed && prm.stall > 0 && s.since >= prm.stall) {
        s.stalled = 1;
        s.active = 0;
    }
}

// One-reduction PCG (Chronopoulos and Gear's rearrangement of the same
// iteration): every iteration needs gamma = r.z, rho = r.r and delta = w.z,
// w = A z, z = D^-1 r, all of one residual, so they are reduced together:
//   beta_i = gamma_i / gamma_{i-1},
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})
// (alpha_0 = gamma_0 / delta_0, beta_0 = 0). The vector update then forms
// p = z + beta p and s = w + beta s (s = A p), r -= alpha s and the x update.
//   FIN_SR_INIT: tot = [r.z | r.r | b.b], tot2 = [w.z]
//   FIN_SR_ITER: tot = [r.z | r.r],       tot2 = [w.z]  (after one update)
__device__ inline void cg_sr_update(int mode, CgCol &s, const double *tot, const double *tot2,
                                    int c, int k, const CgParams &prm) {
    const double g = tot[c], rr = tot[k + c], dl = tot2[c];
    if (mode == FIN_SR_INIT) {
        s.bb = tot[2 * k + c];
        s.rr0 = tot[k + c];
        s.rr = rr;
        s.best = rr;
        s.iters = 0;
        s.since = 0;
        s.stalled = 0;
        const bool conv = !prm.fixed && sqrt(rr) <= fmax(prm.rtol * sqrt(s.bb), prm.atol);
        s.converged = conv ? 1 : 0;
        s.active = (!conv && prm.max_iter > 0) ? 1 : 0;
        s.rz = g;
        s.pq = dl;
        s.beta = 0.0;
        s.alpha_prev = 0.0;
        s.alpha = (s.active && dl != 0.0) ? g / dl : 0.0;
        return;
    }
    if (!s.active) return;
    s.alpha_prev = s.alpha;
    s.iters += 1;
    s.rr = rr;
    cg_stop_tests(s, rr, prm);
    const double bt = s.rz != 0.0 ? g / s.rz : 0.0;
    const double den = dl - (s.alpha != 0.0 ? bt * g / s.alpha : 0.0);
    s.beta = bt;
    s.pq = den;
    s.alpha = den != 0.0 ? g / den : 0.0;
    s.rz = g;
}

}  // namespace kern

inline kern::AsmView view_of(const dgo_mesh *m) {
    return {m->rowptr, m->col, m->vtptr, m->inc, m->nV, m->rpb, m->max_block_nnz, m->max_block_inc};
}

// The row blocks of FP32 assembly (m->rpb_f32 and its sizes).
inline kern::AsmView view_of_f32(const dgo_mesh *m) {
    return {m->rowptr, m->col, m->vtptr, m->inc, m->nV, m->rpb_f32, m->max_block_nnz_f32,
            m->max_block_inc_f32};
}

}  // namespace dgo
