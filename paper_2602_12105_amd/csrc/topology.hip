// Mesh topology on the device: validation, edge extraction by owner-vertex
// bucketing (bit-exact, canonical order), the element -> edge map and signs,
// the CSR pattern, boundary vertices and the per-vertex incidence records used
// by the row-centric assembly kernels.
//
// Edge extraction: every local edge (a, b) of every element is an occurrence
// with key (lo, hi) = (min, max) and id occ = elem * nl + slot. Occurrences are
// bucketed by their owner lo with integer atomics, then each bucket is sorted
// by (hi, occ); since (hi, occ) is unique the result does not depend on the
// order the atomics ran in. Distinct hi values in bucket lo are the edges owned
// by lo, so numbering buckets in vertex order and edges within a bucket by hi
// gives the lexicographic (min, max) rank of each edge.
#include "internal.hpp"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <new>
#include <vector>

namespace dgo {

namespace {

constexpr int T = 256;

__device__ __forceinline__ void local_pair(int dim, int slot, int &a, int &b) {
    if (dim == 2) {
        a = slot == 2 ? 0 : slot + 1;   // slot j: edge opposite vertex j
        b = slot == 0 ? 2 : (slot == 1 ? 0 : 1);
    } else {
        // 01 02 03 12 13 23
        a = slot < 3 ? 0 : (slot < 5 ? 1 : 2);
        b = slot < 3 ? slot + 1 : (slot < 5 ? slot - 1 : 3);
    }
}

__global__ void k_validate(const int32_t *elem, int64_t n_elem, int nv, int32_t nV,
                           int32_t *flags) {
    int64_t e = (int64_t)blockIdx.x * T + threadIdx.x;
    if (e >= n_elem) return;
    int32_t v[4];
    bool range = false, rep = false;
    for (int a = 0; a < nv; ++a) {
        v[a] = elem[e * nv + a];
        if (v[a] < 0 || v[a] >= nV) range = true;
        for (int b = 0; b < a; ++b)
            if (v[b] == v[a]) rep = true;
    }
    if (range) atomicOr(&flags[0], 1);
    if (rep) atomicOr(&flags[1], 1);
}

__global__ void k_owner_count(const int32_t *elem, int64_t n_elem, int dim, int32_t *cnt) {
    const int nv = dim + 1, nl = dim == 2 ? 3 : 6;
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_elem * nl) return;
    int64_t e = o / nl;
    int a, b;
    local_pair(dim, (int)(o % nl), a, b);
    int32_t va = elem[e * nv + a], vb = elem[e * nv + b];
    atomicAdd(&cnt[va < vb ? va : vb], 1);
}

__global__ void k_owner_scatter(const int32_t *elem, int64_t n_elem, int dim,
                                const int32_t *boff, int32_t *cursor, uint64_t *bucket) {
    const int nv = dim + 1, nl = dim == 2 ? 3 : 6;
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_elem * nl) return;
    int64_t e = o / nl;
    int a, b;
    local_pair(dim, (int)(o % nl), a, b);
    int32_t va = elem[e * nv + a], vb = elem[e * nv + b];
    int32_t lo = va < vb ? va : vb, hi = va < vb ? vb : va;
    int32_t pos = boff[lo] + atomicAdd(&cursor[lo], 1);
    bucket[pos] = ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)o;
}

// Insertion sort of each vertex's bucket (buckets are short on meshes).
template <typename K>
__global__ void k_segment_sort(const int32_t *off, K *keys, int32_t n_seg) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= n_seg) return;
    int32_t b = off[v], e = off[v + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        K x = keys[i];
        int32_t j = i - 1;
        while (j >= b && keys[j] > x) {
            keys[j + 1] = keys[j];
            --j;
        }
        keys[j + 1] = x;
    }
}

__global__ void k_unique_count(const int32_t *boff, const uint64_t *bucket, int32_t nV,
                               int32_t *ecnt) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    int32_t c = 0;
    uint32_t prev = 0xffffffffu;
    for (int32_t i = boff[v]; i < boff[v + 1]; ++i) {
        uint32_t hi = (uint32_t)(bucket[i] >> 32);
        if (hi != prev) ++c;
        prev = hi;
    }
    ecnt[v] = c;
}

__global__ void k_emit_edges(const int32_t *boff, const uint64_t *bucket, const int32_t *eoff,
                             int32_t nV, int32_t *EV, int32_t *elem_edge) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    int32_t e = eoff[v] - 1;
    uint32_t prev = 0xffffffffu;
    for (int32_t i = boff[v]; i < boff[v + 1]; ++i) {
        uint64_t key = bucket[i];
        uint32_t hi = (uint32_t)(key >> 32);
        if (hi != prev) {
            ++e;
            EV[2 * (int64_t)e] = v;
            EV[2 * (int64_t)e + 1] = (int32_t)hi;
        }
        prev = hi;
        elem_edge[(uint32_t)key] = e;
    }
}

__global__ void k_signs(const int32_t *elem, int64_t n_elem, int dim, int8_t *sign) {
    const int nv = dim + 1, nl = dim == 2 ? 3 : 6;
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_elem * nl) return;
    int64_t e = o / nl;
    int a, b;
    local_pair(dim, (int)(o % nl), a, b);
    sign[o] = elem[e * nv + a] < elem[e * nv + b] ? 1 : -1;
}

__global__ void k_lower_count(const int32_t *EV, int64_t nE, int32_t *lcnt) {
    int64_t e = (int64_t)blockIdx.x * T + threadIdx.x;
    if (e >= nE) return;
    atomicAdd(&lcnt[EV[2 * e + 1]], 1);
}

__global__ void k_rowlen(const int32_t *lcnt, const int32_t *ecnt, int32_t nV, int32_t *len) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    len[v] = lcnt[v] + 1 + ecnt[v];
}

__global__ void k_fill_upper(const int32_t *rowptr, const int32_t *lcnt, const int32_t *eoff,
                             const int32_t *EV, int32_t nV, int32_t *col, int32_t *diag) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    int32_t d = rowptr[v] + lcnt[v];
    col[d] = v;
    diag[v] = d;
    int32_t n = eoff[v + 1] - eoff[v];
    for (int32_t t = 0; t < n; ++t) col[d + 1 + t] = EV[2 * ((int64_t)eoff[v] + t) + 1];
}

__global__ void k_fill_lower(const int32_t *EV, int64_t nE, const int32_t *rowptr,
                             int32_t *cursor, int32_t *col) {
    int64_t e = (int64_t)blockIdx.x * T + threadIdx.x;
    if (e >= nE) return;
    int32_t lo = EV[2 * e], hi = EV[2 * e + 1];
    col[rowptr[hi] + atomicAdd(&cursor[hi], 1)] = lo;
}

// Sort the lower (j < i) part of each row: [rowptr[i], rowptr[i] + lcnt[i]).
__global__ void k_sort_lower(const int32_t *rowptr, const int32_t *lcnt, int32_t nV,
                             int32_t *col) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    int32_t b = rowptr[v], e = rowptr[v] + lcnt[v];
    for (int32_t i = b + 1; i < e; ++i) {
        int32_t x = col[i];
        int32_t j = i - 1;
        while (j >= b && col[j] > x) {
            col[j + 1] = col[j];
            --j;
        }
        col[j + 1] = x;
    }
}

__global__ void k_max_row(const int32_t *rowptr, int32_t nV, int32_t *mx) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    atomicMax(mx, rowptr[v + 1] - rowptr[v]);
}

__global__ void k_max_count(const int32_t *cnt, int32_t nV, int32_t *mx) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    atomicMax(mx, cnt[v]);
}

__global__ void k_inc_count(const int32_t *elem, int64_t n_inc, int32_t *cnt) {
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_inc) return;
    atomicAdd(&cnt[elem[o]], 1);
}

__global__ void k_inc_scatter(const int32_t *elem, int64_t n_inc, int nv, const int32_t *vtptr,
                              int32_t *cursor, int32_t *inc_elem) {
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_inc) return;
    int32_t v = elem[o];
    inc_elem[vtptr[v] + atomicAdd(&cursor[v], 1)] = (int32_t)(o / nv);
}

__device__ __forceinline__ int32_t local_col(const int32_t *col, int32_t b, int32_t e, int32_t j) {
    while (b < e) {
        int32_t m = (b + e) >> 1;
        if (col[m] < j) b = m + 1; else e = m;
    }
    return b;
}

// Incidence record of vertex v in element el (sorted by element id):
//   bits 0-7, 8-15, 16-23: row-local CSR column indices of the other vertices
//   of the element, in element order after v (triangles: cyclic (v, a, b);
//   tetrahedra: local order skipping v); bits 24-25: v's local position;
//   bits 26-31: v modulo 64 (the row within its block of rows).
__global__ void k_inc_pack(const int32_t *elem, int nv, const int32_t *vtptr,
                           const int32_t *inc_elem, const int32_t *rowptr, const int32_t *col,
                           int32_t nV, uint32_t *rec) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    int32_t rb = rowptr[v], re = rowptr[v + 1];
    for (int32_t q = vtptr[v]; q < vtptr[v + 1]; ++q) {
        const int32_t *el = elem + (int64_t)inc_elem[q] * nv;
        int p = 0;
        for (int a = 0; a < nv; ++a)
            if (el[a] == v) p = a;
        uint32_t r = ((uint32_t)p << 24) | ((uint32_t)(v & 63) << 26);
        if (nv == 3) {
            int32_t la = local_col(col, rb, re, el[(p + 1) % 3]) - rb;
            int32_t lb = local_col(col, rb, re, el[(p + 2) % 3]) - rb;
            r |= (uint32_t)la | ((uint32_t)lb << 8);
        } else {
            int sh = 0;
            for (int a = 0; a < 4; ++a) {
                if (a == p) continue;
                r |= (uint32_t)(local_col(col, rb, re, el[a]) - rb) << sh;
                sh += 8;
            }
        }
        rec[q] = r;
    }
}

// Boundary of triangle meshes: edges with one incident triangle.
__global__ void k_edge_faces(const int32_t *elem_edge, int64_t n, int32_t *cnt) {
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n) return;
    atomicAdd(&cnt[elem_edge[o]], 1);
}

__global__ void k_mark_bedges(const int32_t *EV, const int32_t *cnt, int64_t nE, uint8_t *mask,
                              int32_t *nb) {
    int64_t e = (int64_t)blockIdx.x * T + threadIdx.x;
    if (e >= nE) return;
    if (cnt[e] == 1) {
        mask[EV[2 * e]] = 1;
        mask[EV[2 * e + 1]] = 1;
        atomicAdd(nb, 1);
    }
}

// Boundary of tetrahedral meshes: triangles (face j opposite vertex j) that
// belong to one tetrahedron. Faces are bucketed by their smallest vertex,
// keyed (mid, max), sorted, and counted.
__device__ __forceinline__ void tet_face(const int32_t *el, int j, int32_t &a, int32_t &b,
                                         int32_t &c) {
    int32_t w[3];
    int t = 0;
    for (int i = 0; i < 4; ++i)
        if (i != j) w[t++] = el[i];
    int32_t x;
    if (w[0] > w[1]) { x = w[0]; w[0] = w[1]; w[1] = x; }
    if (w[1] > w[2]) { x = w[1]; w[1] = w[2]; w[2] = x; }
    if (w[0] > w[1]) { x = w[0]; w[0] = w[1]; w[1] = x; }
    a = w[0]; b = w[1]; c = w[2];
}

__global__ void k_face_count(const int32_t *elem, int64_t n_elem, int32_t *cnt) {
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_elem * 4) return;
    int32_t a, b, c;
    tet_face(elem + (o / 4) * 4, (int)(o % 4), a, b, c);
    atomicAdd(&cnt[a], 1);
}

__global__ void k_face_scatter(const int32_t *elem, int64_t n_elem, const int32_t *off,
                               int32_t *cursor, uint64_t *keys) {
    int64_t o = (int64_t)blockIdx.x * T + threadIdx.x;
    if (o >= n_elem * 4) return;
    int32_t a, b, c;
    tet_face(elem + (o / 4) * 4, (int)(o % 4), a, b, c);
    keys[off[a] + atomicAdd(&cursor[a], 1)] = ((uint64_t)(uint32_t)b << 32) | (uint32_t)c;
}

__global__ void k_mark_bfaces(const int32_t *off, const uint64_t *keys, int32_t nV,
                              uint8_t *mask, int32_t *nb) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v >= nV) return;
    int32_t b = off[v], e = off[v + 1];
    int32_t found = 0;
    for (int32_t i = b; i < e;) {
        int32_t j = i;
        while (j < e && keys[j] == keys[i]) ++j;
        if (j - i == 1) {
            mask[v] = 1;
            mask[(uint32_t)(keys[i] >> 32)] = 1;
            mask[(uint32_t)keys[i]] = 1;
            ++found;
        }
        i = j;
    }
    if (found) atomicAdd(nb, found);
}

__global__ void k_count_mask(const uint8_t *mask, int32_t nV, int32_t *n) {
    int32_t v = blockIdx.x * T + threadIdx.x;
    if (v < nV && mask[v]) atomicAdd(n, 1);
}

__global__ void k_block_nnz(const int32_t *rowptr, const int32_t *vtptr, int32_t nV, int32_t rpb,
                            int32_t *mx) {
    int32_t b = blockIdx.x * T + threadIdx.x;
    int64_t r0 = (int64_t)b * rpb;
    if (r0 >= nV) return;
    int64_t r1 = r0 + rpb < nV ? r0 + rpb : nV;
    atomicMax(&mx[0], rowptr[r1] - rowptr[r0]);
    atomicMax(&mx[1], vtptr[r1] - vtptr[r0]);
}

// Pinned host memory for the small device-to-host readbacks of a topology
// build (status flags, the edge count): one buffer per host thread, so that
// concurrent builds (the server's preparation threads) never copy into
// pageable stack memory.
struct PinnedWords {
    int32_t *p = nullptr;
    ~PinnedWords() {
        if (p) (void)hipHostFree(p);
    }
    int32_t *get() {
        if (!p && hipHostMalloc((void **)&p, 64 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        return p;
    }
};

int32_t *readback_words() {
    static thread_local PinnedWords w;
    return w.get();
}

struct Tmp {
    const Alloc &al;
    hipStream_t s;
    void *p[16] = {};
    int n = 0;
    Tmp(const Alloc &a, hipStream_t st) : al(a), s(st) {}
    template <typename X>
    X *get(int64_t count) {
        if (n == 16) return nullptr;  // the caller reports it as an allocation failure
        void *q = al.get((size_t)(count > 0 ? count : 1) * sizeof(X), s);
        if (q) p[n++] = q;
        return (X *)q;
    }
    ~Tmp() {
        for (int i = 0; i < n; ++i) al.put(p[i], s);
    }
};

}  // namespace


static dgo_status build(dgo_mesh *m, const int32_t *d_elem, hipStream_t s) {
    const int dim = m->dim, nv = m->nv_elem, nl = m->nl;
    const int32_t nV = m->nV;
    const int64_t ne = m->n_elem, nkeys = ne * nl, ninc = ne * nv;
    const Alloc &al = m->alloc;
    Tmp tmp(al, s);

    m->elem = (int32_t *)al.get(sizeof(int32_t) * (size_t)(ninc ? ninc : 1), s);
    if (!m->elem) return fail(DGO_ERR_NOMEM, "mesh: element copy allocation failed");
    if (ninc) DGO_HIP(hipMemcpyAsync(m->elem, d_elem, sizeof(int32_t) * ninc, hipMemcpyDeviceToDevice, s));

    // a1: validation, and the most elements at one vertex (the per-vertex
    // sorts below are quadratic in it: a vertex past the supported degree is
    // rejected before they run)
    int32_t *hf = readback_words();
    if (!hf) return fail(DGO_ERR_NOMEM, "mesh: pinned readback allocation failed");
    int32_t *flags = tmp.get<int32_t>(8);
    int32_t *ecnt = tmp.get<int32_t>(nV + 1);
    if (!flags || !ecnt) return fail(DGO_ERR_NOMEM, "mesh: allocation failed");
    DGO_HIP(hipMemsetAsync(flags, 0, 8 * sizeof(int32_t), s));
    DGO_HIP(hipMemsetAsync(ecnt, 0, sizeof(int32_t) * (nV + 1), s));
    if (ne) k_validate<<<grid_for(ne, T), T, 0, s>>>(m->elem, ne, nv, nV, flags);
    DGO_HIP(hipGetLastError());
    DGO_HIP(hipMemcpyAsync(hf, flags, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DGO_HIP(hipStreamSynchronize(s));
    if (hf[0]) return fail(DGO_ERR_INDEX_RANGE, "mesh: element index outside [0, nV)");
    if (hf[1]) return fail(DGO_ERR_INVALID_ARG, "mesh: repeated vertex within an element");
    if (ninc) k_inc_count<<<grid_for(ninc, T), T, 0, s>>>(m->elem, ninc, ecnt);
    if (nV) k_max_count<<<grid_for(nV, T), T, 0, s>>>(ecnt, nV, flags + 7);
    DGO_HIP(hipGetLastError());
    DGO_HIP(hipMemcpyAsync(hf + 7, flags + 7, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DGO_HIP(hipStreamSynchronize(s));
    if (hf[7] > kMaxVertexElems)
        return fail(DGO_ERR_UNSUPPORTED, "mesh: a vertex lies in more than " +
                                             std::to_string(kMaxVertexElems) + " elements");

    // a2: edges by owner-vertex bucketing
    const size_t stmp = scan_tmp_elems((int64_t)nV + 1);
    int32_t *cnt = tmp.get<int32_t>(nV + 1);
    int32_t *boff = tmp.get<int32_t>(nV + 1);
    int32_t *cursor = tmp.get<int32_t>(nV + 1);
    int32_t *lcnt = tmp.get<int32_t>(nV + 1);
    int32_t *stmpb = tmp.get<int32_t>((int64_t)stmp + 1);
    uint64_t *bucket = tmp.get<uint64_t>(nkeys);
    if (!cnt || !boff || !cursor || !lcnt || !stmpb || !bucket)
        return fail(DGO_ERR_NOMEM, "mesh: topology scratch allocation failed");
    DGO_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nV + 1), s));
    DGO_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * (nV + 1), s));
    if (nkeys) k_owner_count<<<grid_for(nkeys, T), T, 0, s>>>(m->elem, ne, dim, cnt);
    DGO_HIP(hipGetLastError());
    DGO_TRY(exclusive_scan(cnt, boff, nV, stmpb, s));
    if (nkeys) k_owner_scatter<<<grid_for(nkeys, T), T, 0, s>>>(m->elem, ne, dim, boff, cursor, bucket);
    DGO_HIP(hipGetLastError());
    if (nV) {
        k_segment_sort<uint64_t><<<grid_for(nV, T), T, 0, s>>>(boff, bucket, nV);
        k_unique_count<<<grid_for(nV, T), T, 0, s>>>(boff, bucket, nV, ecnt);
    }
    DGO_HIP(hipGetLastError());
    int32_t *eoff = cnt;  // reuse
    DGO_TRY(exclusive_scan(ecnt, eoff, nV, stmpb, s));
    DGO_HIP(hipMemcpyAsync(hf + 8, eoff + nV, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DGO_HIP(hipStreamSynchronize(s));
    m->nE = hf[8];
    m->nnz = (int64_t)nV + 2 * m->nE;
    if (m->nnz > INT32_MAX) return fail(DGO_ERR_UNSUPPORTED, "mesh: more than 2^31 CSR entries");

    m->EV = (int32_t *)al.get(sizeof(int32_t) * 2 * (size_t)(m->nE ? m->nE : 1), s);
    m->elem_edge = (int32_t *)al.get(sizeof(int32_t) * (size_t)(nkeys ? nkeys : 1), s);
    m->elem_sign = (int8_t *)al.get((size_t)(nkeys ? nkeys : 1), s);
    m->rowptr = (int32_t *)al.get(sizeof(int32_t) * ((size_t)nV + 1), s);
    m->col = (int32_t *)al.get(sizeof(int32_t) * (size_t)m->nnz, s);
    m->diag = (int32_t *)al.get(sizeof(int32_t) * (size_t)(nV ? nV : 1), s);
    m->vtptr = (int32_t *)al.get(sizeof(int32_t) * ((size_t)nV + 1), s);
    m->inc = (uint32_t *)al.get(sizeof(uint32_t) * (size_t)(ninc ? ninc : 1), s);
    m->bmask = (uint8_t *)al.get((size_t)(nV ? nV : 1), s);
    if (!m->EV || !m->elem_edge || !m->elem_sign || !m->rowptr || !m->col || !m->diag ||
        !m->vtptr || !m->inc || !m->bmask)
        return fail(DGO_ERR_NOMEM, "mesh: topology allocation failed");

    if (nV) k_emit_edges<<<grid_for(nV, T), T, 0, s>>>(boff, bucket, eoff, nV, m->EV, m->elem_edge);
    if (nkeys) k_signs<<<grid_for(nkeys, T), T, 0, s>>>(m->elem, ne, dim, m->elem_sign);
    DGO_HIP(hipGetLastError());

    // a3: CSR pattern, lower neighbours then the diagonal then upper neighbours
    DGO_HIP(hipMemsetAsync(lcnt, 0, sizeof(int32_t) * (nV + 1), s));
    DGO_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * (nV + 1), s));
    if (m->nE) k_lower_count<<<grid_for(m->nE, T), T, 0, s>>>(m->EV, m->nE, lcnt);
    if (nV) k_rowlen<<<grid_for(nV, T), T, 0, s>>>(lcnt, ecnt, nV, boff);  // boff reused as len
    DGO_HIP(hipGetLastError());
    DGO_TRY(exclusive_scan(boff, m->rowptr, nV, stmpb, s));
    if (nV) k_fill_upper<<<grid_for(nV, T), T, 0, s>>>(m->rowptr, lcnt, eoff, m->EV, nV, m->col, m->diag);
    if (m->nE) k_fill_lower<<<grid_for(m->nE, T), T, 0, s>>>(m->EV, m->nE, m->rowptr, cursor, m->col);
    if (nV) k_sort_lower<<<grid_for(nV, T), T, 0, s>>>(m->rowptr, lcnt, nV, m->col);
    DGO_HIP(hipGetLastError());

    // incidence records, sorted by element id within each vertex
    int32_t *inc_elem = tmp.get<int32_t>(ninc);
    if (!inc_elem) return fail(DGO_ERR_NOMEM, "mesh: incidence scratch allocation failed");
    DGO_HIP(hipMemsetAsync(ecnt, 0, sizeof(int32_t) * (nV + 1), s));
    DGO_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * (nV + 1), s));
    if (ninc) k_inc_count<<<grid_for(ninc, T), T, 0, s>>>(m->elem, ninc, ecnt);
    DGO_HIP(hipGetLastError());
    DGO_TRY(exclusive_scan(ecnt, m->vtptr, nV, stmpb, s));
    if (ninc) k_inc_scatter<<<grid_for(ninc, T), T, 0, s>>>(m->elem, ninc, nv, m->vtptr, cursor, inc_elem);
    if (nV) {
        k_segment_sort<int32_t><<<grid_for(nV, T), T, 0, s>>>(m->vtptr, inc_elem, nV);
        k_inc_pack<<<grid_for(nV, T), T, 0, s>>>(m->elem, nv, m->vtptr, inc_elem, m->rowptr, m->col,
                                                 nV, m->inc);
    }
    DGO_HIP(hipGetLastError());
    m->n_inc = ninc;

    // boundary
    DGO_HIP(hipMemsetAsync(m->bmask, 0, (size_t)(nV ? nV : 1), s));
    DGO_HIP(hipMemsetAsync(flags, 0, 8 * sizeof(int32_t), s));
    if (dim == 2) {
        int32_t *fc = tmp.get<int32_t>(m->nE);
        if (!fc) return fail(DGO_ERR_NOMEM, "mesh: boundary scratch allocation failed");
        DGO_HIP(hipMemsetAsync(fc, 0, sizeof(int32_t) * (size_t)(m->nE ? m->nE : 1), s));
        if (nkeys) k_edge_faces<<<grid_for(nkeys, T), T, 0, s>>>(m->elem_edge, nkeys, fc);
        if (m->nE) k_mark_bedges<<<grid_for(m->nE, T), T, 0, s>>>(m->EV, fc, m->nE, m->bmask, flags + 2);
    } else {
        uint64_t *fkeys = tmp.get<uint64_t>(ne * 4);
        if (!fkeys) return fail(DGO_ERR_NOMEM, "mesh: boundary scratch allocation failed");
        DGO_HIP(hipMemsetAsync(lcnt, 0, sizeof(int32_t) * (nV + 1), s));
        DGO_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * (nV + 1), s));
        if (ne) k_face_count<<<grid_for(ne * 4, T), T, 0, s>>>(m->elem, ne, lcnt);
        DGO_HIP(hipGetLastError());
        DGO_TRY(exclusive_scan(lcnt, boff, nV, stmpb, s));
        if (ne) k_face_scatter<<<grid_for(ne * 4, T), T, 0, s>>>(m->elem, ne, boff, cursor, fkeys);
        if (nV) {
            k_segment_sort<uint64_t><<<grid_for(nV, T), T, 0, s>>>(boff, fkeys, nV);
            k_mark_bfaces<<<grid_for(nV, T), T, 0, s>>>(boff, fkeys, nV, m->bmask, flags + 2);
        }
    }
    DGO_HIP(hipGetLastError());
    if (nV) {
        k_count_mask<<<grid_for(nV, T), T, 0, s>>>(m->bmask, nV, flags + 3);
        k_max_row<<<grid_for(nV, T), T, 0, s>>>(m->rowptr, nV, flags + 4);
    }
    DGO_HIP(hipGetLastError());

    // row blocks: the most rows per workgroup whose CSR span and incidence
    // records fit the LDS budget of the assembly kernels
    int32_t rpb = dim == 2 ? kRowsPerBlockTri : kRowsPerBlockTet;
    const int64_t budget = m->lds_budget > 0 ? m->lds_budget : kRowBlockLdsBytes;
    for (;;) {
        DGO_HIP(hipMemsetAsync(flags + 5, 0, 2 * sizeof(int32_t), s));
        int32_t nb = (int32_t)((nV + rpb - 1) / rpb);
        if (nb) k_block_nnz<<<grid_for(nb, T), T, 0, s>>>(m->rowptr, m->vtptr, nV, rpb, flags + 5);
        DGO_HIP(hipGetLastError());
        DGO_HIP(hipMemcpyAsync(hf, flags, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        if (assembly_lds_bytes(dim, 8, rpb, hf[5], hf[6]) <= budget || rpb <= 1) break;
        rpb /= 2;
    }
    m->n_bfaces = hf[2];
    m->n_boundary = hf[3];
    m->max_row = hf[4];
    m->rpb = rpb;
    m->nblocks = (int32_t)((nV + rpb - 1) / rpb);
    m->max_block_nnz = hf[5];
    m->max_block_inc = hf[6];
    if (m->max_row > 255)
        return fail(DGO_ERR_UNSUPPORTED, "mesh: a vertex has more than 254 neighbours");
    if (assembly_lds_bytes(dim, 8, rpb, hf[5], hf[6]) > budget)
        return fail(DGO_ERR_UNSUPPORTED, "mesh: a vertex's row exceeds the LDS budget");
    m->rpb_f32 = m->rpb;
    m->nblocks_f32 = m->nblocks;
    m->max_block_nnz_f32 = m->max_block_nnz;
    m->max_block_inc_f32 = m->max_block_inc;
    if (dim == 3 && nV) {
        // FP32 blocks of tetrahedral meshes: the most rows up to
        // kRowsPerBlockTetF32 whose FP32 LDS fits the budget (never fewer than
        // the FP64 blocks, which fit it with FP64 terms)
        for (int32_t r32 = kRowsPerBlockTetF32; r32 > m->rpb; r32 /= 2) {
            DGO_HIP(hipMemsetAsync(flags + 5, 0, 2 * sizeof(int32_t), s));
            const int32_t nb = (int32_t)((nV + r32 - 1) / r32);
            k_block_nnz<<<grid_for(nb, T), T, 0, s>>>(m->rowptr, m->vtptr, nV, r32, flags + 5);
            DGO_HIP(hipGetLastError());
            DGO_HIP(hipMemcpyAsync(hf + 5, flags + 5, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            DGO_HIP(hipStreamSynchronize(s));
            if (assembly_lds_bytes(dim, 4, r32, hf[5], hf[6]) <= budget) {
                m->rpb_f32 = r32;
                m->nblocks_f32 = nb;
                m->max_block_nnz_f32 = hf[5];
                m->max_block_inc_f32 = hf[6];
                break;
            }
        }
    }
    return DGO_OK;
}

namespace {
__global__ void k_row_desc(const int32_t *order, const int32_t *rowptr, int32_t nV, int2 *rdesc,
                           uint8_t *rlen) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nV) return;
    const int32_t i = order ? order[r] : (int32_t)r;
    const int32_t b = rowptr[i];
    rdesc[r] = make_int2(i, b);
    rlen[r] = (uint8_t)(rowptr[i + 1] - b);  // at most 255 (checked by build)
}

__global__ void k_inverse_perm(const int32_t *order, int32_t nV, int32_t *pos) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nV) pos[order[p]] = (int32_t)p;
}

// Slot t of position p: the row's t-th entry (column position, CSR slot), or
// padding (p, -1) past the row's end. Rows have at most W entries.
__global__ void k_build_ell(const int32_t *order, const int32_t *pos, const int32_t *rowptr,
                            const int32_t *col, int32_t nV, int32_t W, int32_t *ell_col,
                            int32_t *ell_src) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)nV * W) return;
    const int32_t p = (int32_t)(q / W), t = (int32_t)(q % W);
    const int32_t i = order ? order[p] : p;
    const int32_t b = rowptr[i], len = rowptr[i + 1] - b;
    if (t < len) {
        const int32_t j = col[b + t];
        ell_col[q] = pos ? pos[j] : j;
        ell_src[q] = b + t;
    } else {
        ell_col[q] = p;
        ell_src[q] = -1;
    }
}
}  // namespace

// Row order for the SpMV kernels. For large meshes: breadth-first search over
// the CSR pattern from the lowest-numbered unvisited vertex of each
// component, neighbours in ascending column order (a deterministic function
// of the pattern), kept when it is more local than the natural order. Each
// XCD takes a contiguous range of positions, i.e. a band of BFS levels, so
// the x rows its rows gather are mostly those of its own band and stay in its
// L2; in the natural order of a subdivided mesh a vertex's neighbours are
// spread over the whole index range. Small meshes keep the natural order
// (their x fits every L2).
static dgo_status build_row_desc(dgo_mesh *m, hipStream_t s, bool bfs) {
    const int32_t nV = m->nV;
    m->rdesc = (int2 *)m->alloc.get(sizeof(int2) * (size_t)nV, s);
    m->rlen = (uint8_t *)m->alloc.get((size_t)nV, s);
    if (!m->rdesc || !m->rlen) return fail(DGO_ERR_NOMEM, "mesh: row descriptor allocation failed");
    // Host staging of the breadth-first order: pinned memory (rowptr, col and
    // the order), released only after the stream has drained, on every return
    // path, so no copy in flight ever touches freed host memory.
    struct Staging {
        hipStream_t s;
        int32_t *h = nullptr;
        ~Staging() {
            if (h) {
                (void)hipStreamSynchronize(s);
                (void)hipHostFree(h);
            }
        }
    } stg{s};
    if (bfs && nV >= kRowOrderMinRows) {
        const size_t words = ((size_t)nV + 1) + (size_t)m->nnz + (size_t)nV;
        if (hipHostMalloc((void **)&stg.h, sizeof(int32_t) * words, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            stg.h = nullptr;
            return fail(DGO_ERR_NOMEM, "mesh: pinned staging allocation failed");
        }
        int32_t *rp = stg.h, *cl = rp + nV + 1, *order = cl + m->nnz;
        DGO_HIP(hipMemcpyAsync(rp, m->rowptr, sizeof(int32_t) * ((size_t)nV + 1), hipMemcpyDeviceToHost, s));
        DGO_HIP(hipMemcpyAsync(cl, m->col, sizeof(int32_t) * (size_t)m->nnz, hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        std::vector<uint8_t> seen((size_t)nV, 0);
        int64_t tail = 0;
        for (int32_t root = 0; root < nV; ++root) {
            if (seen[root]) continue;
            seen[root] = 1;
            int64_t head = tail;
            order[tail++] = root;
            while (head < tail) {
                const int32_t v = order[head++];
                for (int32_t t = rp[v]; t < rp[v + 1]; ++t) {
                    const int32_t j = cl[t];
                    if (!seen[j]) {
                        seen[j] = 1;
                        order[tail++] = j;
                    }
                }
            }
        }
        // Keep the breadth-first order only where it is more local than the
        // natural one: per row, the largest index distance to a neighbour
        // (natural ids, or positions in the breadth-first order), compared
        // at the 90th percentile over the rows. Structured numberings (grids,
        // the Kuhn cube) are local already: a row's neighbours lie within a
        // few lines or planes, while breadth-first fronts spread every
        // plane over the whole index range.
        std::vector<int32_t> pos((size_t)nV), dn((size_t)nV), db((size_t)nV);
        for (int32_t q = 0; q < nV; ++q) pos[order[q]] = q;
        for (int32_t v = 0; v < nV; ++v) {
            int32_t a = 0, b = 0;
            for (int32_t t = rp[v]; t < rp[v + 1]; ++t) {
                const int32_t j = cl[t];
                a = std::max(a, std::abs(j - v));
                b = std::max(b, std::abs(pos[j] - pos[v]));
            }
            dn[v] = a;
            db[v] = b;
        }
        const size_t p90 = (size_t)((int64_t)nV * 9 / 10);
        std::nth_element(dn.begin(), dn.begin() + p90, dn.end());
        std::nth_element(db.begin(), db.begin() + p90, db.end());
        if (db[p90] < dn[p90]) {
            m->order = (int32_t *)m->alloc.get(sizeof(int32_t) * (size_t)nV, s);
            if (!m->order) return fail(DGO_ERR_NOMEM, "mesh: row order allocation failed");
            DGO_HIP(hipMemcpyAsync(m->order, order, sizeof(int32_t) * (size_t)nV,
                                   hipMemcpyHostToDevice, s));
        }
    }
    k_row_desc<<<grid_for(nV, T), T, 0, s>>>(m->order, m->rowptr, nV, m->rdesc, m->rlen);
    DGO_HIP(hipGetLastError());
    if (m->max_row <= kEllMaxWidth && (int64_t)nV * kEllMaxWidth < INT32_MAX) {
        const int32_t W = m->max_row <= 8 ? 8 : kEllMaxWidth;
        const int64_t ns = (int64_t)nV * W;
        m->ell_col = (int32_t *)m->alloc.get(sizeof(int32_t) * (size_t)ns, s);
        m->ell_src = (int32_t *)m->alloc.get(sizeof(int32_t) * (size_t)ns, s);
        if (!m->ell_col || !m->ell_src) return fail(DGO_ERR_NOMEM, "mesh: padded-row allocation failed");
        Tmp tmp(m->alloc, s);
        int32_t *pos = nullptr;
        if (m->order) {
            pos = tmp.get<int32_t>(nV);
            if (!pos) return fail(DGO_ERR_NOMEM, "mesh: row position allocation failed");
            k_inverse_perm<<<grid_for(nV, T), T, 0, s>>>(m->order, nV, pos);
        }
        k_build_ell<<<grid_for(ns, T), T, 0, s>>>(m->order, pos, m->rowptr, m->col, nV, W,
                                                   m->ell_col, m->ell_src);
        DGO_HIP(hipGetLastError());
        m->ell_w = W;
    }
    DGO_HIP(hipStreamSynchronize(s));
    return DGO_OK;
}

static void release(dgo_mesh *m, hipStream_t s) {
    for (auto &e : m->poll_ev)
        if (e) (void)hipEventDestroy(e);
    if (m->poll_host) (void)hipHostFree(m->poll_host);
    m->poll_ev[0] = m->poll_ev[1] = nullptr;
    m->poll_host = nullptr;
    void *ptrs[] = {m->elem, m->EV, m->elem_edge, m->elem_sign, m->rowptr, m->col,
                    m->diag, m->vtptr, m->inc, m->bmask, m->rdesc, m->rlen, m->order,
                    m->ell_col, m->ell_src, m->vjp_mirror, m->vjp_coldiag, m->vjp_opp,
                    m->inc_elem, m->face_islot, m->conf_bslot, m->conf_bptr, m->ws};
    for (void *p : ptrs) m->alloc.put(p, s);
}

}  // namespace dgo

using namespace dgo;

// The same scatter and per-vertex sort as the topology build, so entry q of
// inc_elem is the element of incidence record q.
dgo_status dgo::mesh_inc_elem(dgo_mesh *m, hipStream_t s) {
    if (m->inc_elem) return DGO_OK;
    const int64_t ninc = m->n_inc;
    const int32_t nV = m->nV;
    int32_t *ie = (int32_t *)m->alloc.get(sizeof(int32_t) * (size_t)(ninc ? ninc : 1), s);
    int32_t *cursor = (int32_t *)m->alloc.get(sizeof(int32_t) * ((size_t)nV + 1), s);
    if (!ie || !cursor) {
        m->alloc.put(ie, s);
        m->alloc.put(cursor, s);
        return fail(DGO_ERR_NOMEM, "mesh: incidence element allocation failed");
    }
    DGO_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * ((size_t)nV + 1), s));
    if (ninc) {
        k_inc_scatter<<<grid_for(ninc, T), T, 0, s>>>(m->elem, ninc, m->nv_elem, m->vtptr, cursor, ie);
        k_segment_sort<int32_t><<<grid_for(nV, T), T, 0, s>>>(m->vtptr, ie, nV);
    }
    DGO_HIP(hipGetLastError());
    m->alloc.put(cursor, s);
    m->inc_elem = ie;
    return DGO_OK;
}

dgo_status dgo::mesh_create(int32_t dim, int32_t nV, int64_t n_elem, const int32_t *d_elem,
                            const dgo_allocator *alloc, hipStream_t s, RowsMode rows,
                            int64_t lds_budget, dgo_mesh **out) {
    clear_error();
    if (!out) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_create: out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_create: dim must be 2 or 3");
    if (nV < 1 || n_elem < 0) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_create: bad nV or n_elem");
    if (n_elem > 0 && !d_elem) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_create: d_elem is NULL");
    if (n_elem * (dim == 2 ? 3 : 6) >= INT32_MAX)
        return fail(DGO_ERR_UNSUPPORTED, "dgo_mesh_create: too many elements for int32 occurrence ids");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_create: allocator callbacks missing");
    dgo_mesh *m = new (std::nothrow) dgo_mesh();
    if (!m) return fail(DGO_ERR_NOMEM, "dgo_mesh_create: host allocation failed");
    m->dim = dim;
    m->nv_elem = dim + 1;
    m->nl = dim == 2 ? 3 : 6;
    m->nV = nV;
    m->n_elem = n_elem;
    if (alloc) {
        m->alloc.user = *alloc;
        m->alloc.has_user = true;
    }
    m->home = s;
    m->lds_budget = lds_budget;
    (void)hipGetDevice(&m->device);
    dgo_status st = build(m, d_elem, s);
    if (st == DGO_OK && rows != ROWS_NONE) st = build_row_desc(m, s, rows == ROWS_AUTO);
    if (st != DGO_OK) {
        std::string msg = dgo_last_error();
        (void)hipStreamSynchronize(s);
        release(m, s);
        (void)hipStreamSynchronize(s);
        delete m;
        set_error(msg);
        return st;
    }
    *out = m;
    return DGO_OK;
}

extern "C" dgo_status dgo_mesh_create(int32_t dim, int32_t nV, int64_t n_elem,
                                      const int32_t *d_elem, const dgo_allocator *alloc,
                                      dgo_stream stream, dgo_mesh **out) {
    return mesh_create(dim, nV, n_elem, d_elem, alloc, (hipStream_t)stream, ROWS_AUTO, 0, out);
}

extern "C" void dgo_mesh_destroy(dgo_mesh *m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->home);
    release(m, m->home);
    (void)hipStreamSynchronize(m->home);
    delete m;
}

extern "C" dgo_status dgo_mesh_sizes(const dgo_mesh *m, dgo_sizes *o) {
    clear_error();
    if (!m || !o) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_sizes: NULL argument");
    o->dim = m->dim;
    o->nV = m->nV;
    o->n_elem = m->n_elem;
    o->nE = m->nE;
    o->nnz = m->nnz;
    o->n_bfaces = m->n_bfaces;
    o->n_boundary = m->n_boundary;
    o->max_row = m->max_row;
    return DGO_OK;
}

extern "C" dgo_status dgo_mesh_edges(const dgo_mesh *m, int32_t *d_EV, int32_t *d_elem_edge,
                                     int8_t *d_elem_sign, dgo_stream stream) {
    clear_error();
    if (!m) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_edges: mesh is NULL");
    hipStream_t s = (hipStream_t)stream;
    int64_t nk = m->n_elem * m->nl;
    if (d_EV && m->nE)
        DGO_HIP(hipMemcpyAsync(d_EV, m->EV, sizeof(int32_t) * 2 * m->nE, hipMemcpyDeviceToDevice, s));
    if (d_elem_edge && nk)
        DGO_HIP(hipMemcpyAsync(d_elem_edge, m->elem_edge, sizeof(int32_t) * nk, hipMemcpyDeviceToDevice, s));
    if (d_elem_sign && nk)
        DGO_HIP(hipMemcpyAsync(d_elem_sign, m->elem_sign, (size_t)nk, hipMemcpyDeviceToDevice, s));
    return DGO_OK;
}

extern "C" dgo_status dgo_mesh_csr(const dgo_mesh *m, int32_t *d_rowptr, int32_t *d_col,
                                   dgo_stream stream) {
    clear_error();
    if (!m) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_csr: mesh is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (d_rowptr)
        DGO_HIP(hipMemcpyAsync(d_rowptr, m->rowptr, sizeof(int32_t) * ((size_t)m->nV + 1),
                               hipMemcpyDeviceToDevice, s));
    if (d_col)
        DGO_HIP(hipMemcpyAsync(d_col, m->col, sizeof(int32_t) * (size_t)m->nnz, hipMemcpyDeviceToDevice, s));
    return DGO_OK;
}

extern "C" dgo_status dgo_mesh_boundary(const dgo_mesh *m, uint8_t *d_mask, dgo_stream stream) {
    clear_error();
    if (!m || !d_mask) return fail(DGO_ERR_INVALID_ARG, "dgo_mesh_boundary: NULL argument");
    DGO_HIP(hipMemcpyAsync(d_mask, m->bmask, (size_t)m->nV, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return DGO_OK;
}
