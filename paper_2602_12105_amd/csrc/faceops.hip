// Per-face gradient G and divergence D of triangle meshes (the operators of
// the geodesic-distance ADMM loop, Sec. 7.4).
//
// G maps k vertex fields to k piecewise-constant face vector fields: on face f
// with vertices x0, x1, x2 and n = (x1 - x0) x (x2 - x0), the hat function of
// local vertex j has gradient (n x e_j) / |n|^2, e_j = x_{j+2} - x_{j+1} the
// edge opposite j. D = G^T diag(A_f) maps face fields back to vertices, so that
// D G is the cotangent stiffness K.
//
// Face fields are component-major, (k, 3, nF): component d of field c on face
// f at [(c * 3 + d) * nF + f], so the face kernels touch each plane with
// coalesced accesses. G runs one thread per face (geometry once, then the k
// fields). D runs in two launches: one thread per face forms the three corner
// terms A_f grad phi_j . y_f of each field and stores each at its corner's
// incidence record (the vertex's incidence list holds its faces in ascending
// order), then one thread per (vertex, field) adds its run of consecutive
// terms in that order. The sum has a fixed order, no atomics are used, and
// the second pass streams the terms instead of gathering them at scattered
// face ids (a pull over the faces directly was measured several times slower:
// three dependent gathers per incidence).
#include "internal.hpp"
#include <climits>
#include "kernels.hpp"

namespace dgo {
namespace {

using namespace kern;

constexpr int kFaceThreads = 256;

template <typename R>
__device__ __forceinline__ V3<R> scale(V3<R> a, R s) {
    return {a.x * s, a.y * s, a.z * s};
}

template <typename R>
__global__ void __launch_bounds__(kFaceThreads)
k_face_gradient(const int32_t *__restrict__ elem, const R *__restrict__ X, int64_t nF, int32_t k,
                const R *__restrict__ u, R *__restrict__ g) {
    const int64_t f = (int64_t)blockIdx.x * kFaceThreads + threadIdx.x;
    if (f >= nF) return;
    const int32_t v0 = elem[3 * f], v1 = elem[3 * f + 1], v2 = elem[3 * f + 2];
    const V3<R> x0 = ld3(X, v0), x1 = ld3(X, v1), x2 = ld3(X, v2);
    const V3<R> n = cross(sub(x1, x0), sub(x2, x0));
    const R nn = dot(n, n);
    const V3<R> g0 = scale(cross(n, sub(x2, x1)), R(1) / nn);
    const V3<R> g1 = scale(cross(n, sub(x0, x2)), R(1) / nn);
    const V3<R> g2 = scale(cross(n, sub(x1, x0)), R(1) / nn);
    for (int32_t c = 0; c < k; ++c) {
        const R u0 = u[(int64_t)v0 * k + c], u1 = u[(int64_t)v1 * k + c], u2 = u[(int64_t)v2 * k + c];
        R *out = g + (int64_t)c * 3 * nF + f;
        out[0] = u0 * g0.x + u1 * g1.x + u2 * g2.x;
        out[nF] = u0 * g0.y + u1 * g1.y + u2 * g2.y;
        out[2 * nF] = u0 * g0.z + u1 * g1.z + u2 * g2.z;
    }
}

// corner terms T[c * 3 nF + islot[3 f + j]] = A_f grad phi_j . y_f, at the
// incidence record of corner j of face f
template <typename R>
__global__ void __launch_bounds__(kFaceThreads)
k_face_corners(const int32_t *__restrict__ elem, const R *__restrict__ X, int64_t nF, int32_t k,
               const int32_t *__restrict__ islot, const R *__restrict__ y, R *__restrict__ T) {
    const int64_t f = (int64_t)blockIdx.x * kFaceThreads + threadIdx.x;
    if (f >= nF) return;
    const int32_t v0 = elem[3 * f], v1 = elem[3 * f + 1], v2 = elem[3 * f + 2];
    const V3<R> x0 = ld3(X, v0), x1 = ld3(X, v1), x2 = ld3(X, v2);
    const V3<R> n = cross(sub(x1, x0), sub(x2, x0));
    const R nn = dot(n, n);
    const R h = (R(0.5) * sqrt(nn)) / nn;  // A_f / |n|^2
    const V3<R> w0 = scale(cross(n, sub(x2, x1)), h);
    const V3<R> w1 = scale(cross(n, sub(x0, x2)), h);
    const V3<R> w2 = scale(cross(n, sub(x1, x0)), h);
    const int32_t q0 = islot[3 * f], q1 = islot[3 * f + 1], q2 = islot[3 * f + 2];
    for (int32_t c = 0; c < k; ++c) {
        const R *yc = y + (int64_t)c * 3 * nF + f;
        const V3<R> yf = {yc[0], yc[nF], yc[2 * nF]};
        R *out = T + (int64_t)c * 3 * nF;
        out[q0] = dot(w0, yf);
        out[q1] = dot(w1, yf);
        out[q2] = dot(w2, yf);
    }
}

// islot[3 f + p] = q for incidence record q of the vertex at corner p of face f
__global__ void k_face_islot(const int32_t *__restrict__ inc_elem, const uint32_t *__restrict__ inc,
                             int64_t n_inc, int32_t *__restrict__ islot) {
    const int64_t q = (int64_t)blockIdx.x * kFaceThreads + threadIdx.x;
    if (q >= n_inc) return;
    islot[3 * (int64_t)inc_elem[q] + ((inc[q] >> 24) & 3u)] = (int32_t)q;
}

template <typename R>
__global__ void __launch_bounds__(kFaceThreads)
k_vertex_gather(const int32_t *__restrict__ vtptr, int32_t nV, int64_t n_inc, int32_t k,
                const R *__restrict__ T, R *__restrict__ div) {
    const int64_t o = (int64_t)blockIdx.x * kFaceThreads + threadIdx.x;
    if (o >= (int64_t)nV * k) return;
    const int32_t i = (int32_t)(o / k), c = (int32_t)(o - (int64_t)i * k);
    const R *__restrict__ Tc = T + (int64_t)c * n_inc;
    const int32_t e = vtptr[i + 1];
    int32_t q = vtptr[i];
    R acc = 0;
    // four terms' loads in flight at a time, added in order
    for (; q + 4 <= e; q += 4) {
        const R t0 = Tc[q], t1 = Tc[q + 1], t2 = Tc[q + 2], t3 = Tc[q + 3];
        acc += t0;
        acc += t1;
        acc += t2;
        acc += t3;
    }
    for (; q < e; ++q) acc += Tc[q];
    div[o] = acc;
}

// X, the vertex fields and the face fields; the face fields' pointer may be
// NULL when the mesh has no faces
dgo_status check_args(const dgo_mesh *m, dgo_dtype dtype, const void *X, int32_t k, const void *vf,
                      const void *ff, const std::string &who) {
    if (!m || !X || !vf || (!ff && m->n_elem > 0)) return fail(DGO_ERR_INVALID_ARG, who + ": NULL argument");
    if (dtype != DGO_F32 && dtype != DGO_F64) return fail(DGO_ERR_INVALID_ARG, who + ": bad dtype");
    if (k < 1 || k > 64) return fail(DGO_ERR_INVALID_ARG, who + ": k must be in [1, 64]");
    if (m->dim != 2) return fail(DGO_ERR_UNSUPPORTED, who + ": triangle meshes only");
    return DGO_OK;
}

}  // namespace
}  // namespace dgo

using namespace dgo;

extern "C" dgo_status dgo_face_gradient(const dgo_mesh *m, dgo_dtype dtype, const void *d_X,
                                        int32_t k, const void *d_u, void *d_g, dgo_stream stream) {
    clear_error();
    DGO_TRY(check_args(m, dtype, d_X, k, d_u, d_g, "dgo_face_gradient"));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nF = m->n_elem;
    if (nF == 0) return DGO_OK;
    const dim3 grid(grid_for(nF, kFaceThreads)), block(kFaceThreads);
    if (dtype == DGO_F64)
        DGO_LAUNCH_EXT("face_gradient", s, k_face_gradient<double>, grid, block, 0u, m->elem,
                       (const double *)d_X, nF, k, (const double *)d_u, (double *)d_g);
    else
        DGO_LAUNCH_EXT("face_gradient", s, k_face_gradient<float>, grid, block, 0u, m->elem,
                       (const float *)d_X, nF, k, (const float *)d_u, (float *)d_g);
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

extern "C" dgo_status dgo_face_divergence(const dgo_mesh *m, dgo_dtype dtype, const void *d_X,
                                          int32_t k, const void *d_y, void *d_div,
                                          dgo_stream stream) {
    clear_error();
    DGO_TRY(check_args(m, dtype, d_X, k, d_div, d_y, "dgo_face_divergence"));
    hipStream_t s = (hipStream_t)stream;
    dgo_mesh *mm = const_cast<dgo_mesh *>(m);
    const int64_t nF = m->n_elem, n = (int64_t)m->nV * k;
    if (3 * nF > INT32_MAX) return fail(DGO_ERR_UNSUPPORTED, "dgo_face_divergence: more than 2^31 / 3 faces");
    if (!m->face_islot) {
        DGO_TRY(mesh_inc_elem(mm, s));
        int32_t *is = (int32_t *)m->alloc.get(sizeof(int32_t) * (size_t)(m->n_inc ? m->n_inc : 1), s);
        if (!is) return fail(DGO_ERR_NOMEM, "dgo_face_divergence: corner slot allocation failed");
        if (m->n_inc)
            k_face_islot<<<grid_for(m->n_inc, kFaceThreads), kFaceThreads, 0, s>>>(m->inc_elem, m->inc,
                                                                                 m->n_inc, is);
        DGO_HIP(hipGetLastError());
        mm->face_islot = is;
    }
    const size_t es = dtype == DGO_F64 ? sizeof(double) : sizeof(float);
    void *T = nullptr;
    DGO_TRY(mesh_workspace(mm, es * 3 * (size_t)k * (size_t)(nF ? nF : 1), s, &T));
    if (dtype == DGO_F64)
        DGO_LAUNCH("face_divergence", s, {
            if (nF)
                k_face_corners<double><<<grid_for(nF, kFaceThreads), kFaceThreads, 0, s>>>(
                    m->elem, (const double *)d_X, nF, k, m->face_islot, (const double *)d_y,
                    (double *)T);
            k_vertex_gather<double><<<grid_for(n, kFaceThreads), kFaceThreads, 0, s>>>(
                m->vtptr, m->nV, m->n_inc, k, (const double *)T, (double *)d_div);
        });
    else
        DGO_LAUNCH("face_divergence", s, {
            if (nF)
                k_face_corners<float><<<grid_for(nF, kFaceThreads), kFaceThreads, 0, s>>>(
                    m->elem, (const float *)d_X, nF, k, m->face_islot, (const float *)d_y,
                    (float *)T);
            k_vertex_gather<float><<<grid_for(n, kFaceThreads), kFaceThreads, 0, s>>>(
                m->vtptr, m->nV, m->n_inc, k, (const float *)T, (float *)d_div);
        });
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}
