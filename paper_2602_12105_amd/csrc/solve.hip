// Operator application y = (alpha M + beta K) x and Jacobi-preconditioned
// conjugate gradients on it.
//
// SpMV/SpMM: CSR rows are handed to groups of G lanes inside a 64-lane
// wavefront. With k >= 8 right-hand sides each lane of a group owns one
// column and walks the whole row (the row's values and column ids are
// broadcast within the group, the gathered x row is one contiguous k-vector);
// with k < 8 the group's lanes also split the row's entries into `parts`
// interleaved subsets that are combined by a fixed shuffle tree. The operator
// alpha M + beta K is never formed: the diagonal term is added on the fly.
//
// PCG (Saad, Alg. 9.1, Jacobi preconditioner) runs three kernels per
// iteration: q = A p fused with the dot p.q, then the x / r / z updates fused
// with the dots r.z and r.r, then p = z + beta p. Each dot is reduced in a
// fixed order: every workgroup stores its partial sums, and the last
// workgroup to finish (found with an integer atomic ticket) adds all partials
// in workgroup order and updates the per-column scalars. The result is
// bitwise deterministic run to run. Columns are frozen once they stop.
#include "internal.hpp"

#include <algorithm>
#include <cstdlib>

namespace dgo {
namespace {

constexpr int T = 256;
constexpr int kMaxK = 64;
constexpr int kMaxRedBlocks = 512;

struct CgCol {
    double rz, pq, alpha, beta, rr, bb, best;
    int32_t iters, since, active, converged;
    int32_t stalled, pad0;
};

struct CgParams {
    double rtol;
    int32_t max_iter, fixed, stall;
    int32_t k;
};

struct Layout {
    int G;      // lanes per row group (power of two, divides 64)
    int parts;  // interleaved subsets of a row's entries
};

Layout spmm_layout(int k) {
    if (k >= 8) {
        int G = 8;
        while (G < k) G *= 2;
        return {G, 1};
    }
    int parts = 1;
    while (parts * 2 * k <= 8) parts *= 2;
    return {8, parts};
}

int pow2ceil(int k) {
    int G = 1;
    while (G < k) G *= 2;
    return G;
}

// Contiguous chunk of row tiles for workgroup `bid` (XCD-aware: each XCD's
// workgroups cover one contiguous range of tiles).
__device__ __forceinline__ void tile_range(int64_t ntiles, int64_t &t0, int64_t &t1) {
    const uint32_t nb = gridDim.x;
    const uint32_t lb = xcd_tile(blockIdx.x, nb);
    const int64_t per = (ntiles + nb - 1) / nb;
    t0 = (int64_t)lb * per;
    t1 = t0 + per < ntiles ? t0 + per : ntiles;
}

template <typename R>
struct Acc {
    using type = R;
};

// ------------------------------------------------------ fixed-order reduce

// Store this workgroup's W partial sums (in LDS `part`, W <= T) and, if it
// is the last workgroup to finish, sum every workgroup's partials in
// workgroup order into `tot` (LDS, W values). Returns true in the last one.
__device__ bool block_then_last(const double *part, int W, double *gpart, uint32_t *ticket,
                                double *tot, double *scratch) {
    __shared__ int s_last;
    const int t = threadIdx.x;
    const uint32_t nblk = gridDim.x;
    if (t < W)
        __hip_atomic_store(&gpart[(int64_t)blockIdx.x * W + t], part[t], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    __syncthreads();
    if (t == 0) s_last = atomicAdd(ticket, 1u) == nblk - 1;
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    const int tpw = T / W;  // threads per value
    const int w = t / tpw, sub = t % tpw;
    double s = 0.0;
    if (w < W) {
        for (uint32_t b = sub; b < nblk; b += tpw)
            s += __hip_atomic_load(&gpart[(int64_t)b * W + w], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
    scratch[t] = s;
    __syncthreads();
    if (t < W) {
        double a = 0.0;
        for (int j = 0; j < tpw; ++j) a += scratch[t * tpw + j];
        tot[t] = a;
    }
    if (t == 0) *ticket = 0u;
    __syncthreads();
    return true;
}

// ------------------------------------------------------------------ SpMM

template <typename R, bool MASK>
__device__ __forceinline__ R row_apply(const int32_t *__restrict__ rowptr,
                                       const int32_t *__restrict__ col, const R *__restrict__ K,
                                       R dterm, R beta, const uint8_t *__restrict__ mask,
                                       const R *__restrict__ x, int32_t i, int k, int c, int part,
                                       int parts) {
    R acc = 0;
    const int32_t e = rowptr[i + 1];
    for (int32_t t = rowptr[i] + part; t < e; t += parts) {
        const int32_t j = col[t];
        if (MASK && mask[j]) continue;
        R a = beta * K[t];
        if (j == i) a += dterm;
        acc += a * x[(int64_t)j * k + c];
    }
    return acc;
}

template <typename R>
__global__ void __launch_bounds__(T)
k_spmm(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t nV, int64_t nnz,
       R alpha, const R *__restrict__ M, R beta, const R *__restrict__ K, int k, int G, int parts,
       const R *__restrict__ x, R *__restrict__ y) {
    const int64_t bt = blockIdx.y;
    M += bt * nV;
    K += bt * nnz;
    x += bt * (int64_t)nV * k;
    y += bt * (int64_t)nV * k;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G, gpb = T / G;
    const int c = lane % k, part = lane / k;
    const bool act = part < parts;
    int64_t t0, t1;
    tile_range(((int64_t)nV + gpb - 1) / gpb, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i = tile * gpb + grp;
        R acc = 0;
        if (i < nV && act)
            acc = row_apply<R, false>(rowptr, col, K, alpha * M[i], beta, nullptr, x, (int32_t)i, k,
                                      c, part, parts);
        for (int off = (parts / 2) * k; off >= k && off > 0; off /= 2)
            acc += __shfl_down(acc, off, G);
        if (i < nV && act && part == 0) y[i * k + c] = acc;
    }
}

// ------------------------------------------------------------------- PCG

// q = A p on the interior rows (q_B = 0), partial p.q per column; the last
// workgroup forms alpha = rz / pq for active columns.
template <typename R>
__global__ void __launch_bounds__(T)
k_cg_spmm_dot(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t nV,
              R alpha_m, const R *__restrict__ M, R beta_k, const R *__restrict__ K,
              const uint8_t *__restrict__ mask, int k, int G, int parts, const R *__restrict__ p,
              R *__restrict__ q, int mode, double *gpart, uint32_t *ticket, CgCol *st) {
    __shared__ double s_part[kMaxK];
    __shared__ double s_tot[kMaxK];
    __shared__ double s_scr[T];
    __shared__ double s_red[T];
    const int lane = threadIdx.x % G, grp = threadIdx.x / G, gpb = T / G;
    const int c = lane % k, part = lane / k;
    const bool act = part < parts;
    double dsum = 0.0;
    int64_t t0, t1;
    tile_range(((int64_t)nV + gpb - 1) / gpb, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i = tile * gpb + grp;
        R acc = 0;
        const bool row = i < nV && act && !(mask && mask[i]);
        if (row) {
            if (mask)
                acc = row_apply<R, true>(rowptr, col, K, alpha_m * M[i], beta_k, mask, p, (int32_t)i,
                                         k, c, part, parts);
            else
                acc = row_apply<R, false>(rowptr, col, K, alpha_m * M[i], beta_k, nullptr, p,
                                          (int32_t)i, k, c, part, parts);
        }
        for (int off = (parts / 2) * k; off >= k && off > 0; off /= 2)
            acc += __shfl_down(acc, off, G);
        if (i < nV && act && part == 0) {
            q[i * k + c] = acc;
            if (mode == 1) dsum += (double)p[i * k + c] * (double)acc;
        }
    }
    if (mode != 1) return;
    // workgroup partial per column, in a fixed order
    s_red[threadIdx.x] = (act && part == 0) ? dsum : 0.0;
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double a = 0.0;
        for (int t = threadIdx.x; t < T; t += G) a += s_red[t];
        s_part[threadIdx.x] = a;
    }
    __syncthreads();
    if (!block_then_last(s_part, k, gpart, ticket, s_tot, s_scr)) return;
    if ((int)threadIdx.x < k) {
        CgCol &s = st[threadIdx.x];
        const double pq = s_tot[threadIdx.x];
        s.pq = pq;
        s.alpha = (s.active && pq != 0.0) ? s.rz / pq : 0.0;
    }
}

// Columns-in-lanes layout for the vector kernels: G = pow2ceil(k) lanes per row.
struct VLane {
    int c;
    bool act;
    int grp, gpb;
};

__device__ __forceinline__ VLane vlane(int k, int G) {
    VLane v;
    v.c = threadIdx.x % G;
    v.act = v.c < k;
    v.grp = threadIdx.x / G;
    v.gpb = T / G;
    return v;
}

// Reduce per-lane sums (nval values per lane) to per-column workgroup partials.
__device__ __forceinline__ void column_partials(const double *vals, int nval, int k, int G,
                                                bool act, double *s_red, double *s_part) {
    for (int v = 0; v < nval; ++v) {
        __syncthreads();
        s_red[threadIdx.x] = act ? vals[v] : 0.0;
        __syncthreads();
        if ((int)threadIdx.x < k) {
            double a = 0.0;
            for (int t = threadIdx.x; t < T; t += G) a += s_red[t];
            s_part[v * k + threadIdx.x] = a;
        }
    }
    __syncthreads();
}

// r = beff - q, z = D^-1 r, p = z; dots r.z, r.r, beff.beff; the last
// workgroup initialises the per-column state.
template <typename R>
__global__ void __launch_bounds__(T)
k_cg_init(int32_t nV, int k, int G, const R *__restrict__ beff, const R *__restrict__ q,
          const R *__restrict__ invD, R *__restrict__ r, R *__restrict__ z, R *__restrict__ p,
          double *gpart, uint32_t *ticket, CgCol *st, CgParams prm) {
    __shared__ double s_part[3 * kMaxK];
    __shared__ double s_tot[3 * kMaxK];
    __shared__ double s_scr[T];
    __shared__ double s_red[T];
    const VLane L = vlane(k, G);
    double d[3] = {0.0, 0.0, 0.0};
    int64_t t0, t1;
    tile_range(((int64_t)nV + L.gpb - 1) / L.gpb, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i = tile * L.gpb + L.grp;
        if (i >= nV || !L.act) continue;
        const int64_t e = i * k + L.c;
        const R b = beff[e];
        const R rv = b - q[e];
        const R zv = invD[i] * rv;
        r[e] = rv;
        z[e] = zv;
        p[e] = zv;
        d[0] += (double)rv * (double)zv;
        d[1] += (double)rv * (double)rv;
        d[2] += (double)b * (double)b;
    }
    column_partials(d, 3, k, G, L.act, s_red, s_part);
    if (!block_then_last(s_part, 3 * k, gpart, ticket, s_tot, s_scr)) return;
    if ((int)threadIdx.x < k) {
        CgCol &s = st[threadIdx.x];
        s.rz = s_tot[threadIdx.x];
        s.rr = s_tot[k + threadIdx.x];
        s.bb = s_tot[2 * k + threadIdx.x];
        s.best = s.rr;
        s.iters = 0;
        s.since = 0;
        s.stalled = 0;
        s.pq = 0.0;
        s.alpha = 0.0;
        s.beta = 0.0;
        const bool conv = !prm.fixed && sqrt(s.rr) <= prm.rtol * sqrt(s.bb);
        s.converged = conv ? 1 : 0;
        s.active = (!conv && prm.max_iter > 0) ? 1 : 0;
    }
}

// x += alpha p, r -= alpha q, z = D^-1 r on active columns; dots r.z, r.r;
// the last workgroup advances the per-column state and tests for stopping.
template <typename R>
__global__ void __launch_bounds__(T)
k_cg_update(int32_t nV, int k, int G, R *__restrict__ x, R *__restrict__ r, R *__restrict__ z,
            const R *__restrict__ p, const R *__restrict__ q, const R *__restrict__ invD,
            double *gpart, uint32_t *ticket, CgCol *st, CgParams prm) {
    __shared__ double s_part[2 * kMaxK];
    __shared__ double s_tot[2 * kMaxK];
    __shared__ double s_scr[T];
    __shared__ double s_red[T];
    const VLane L = vlane(k, G);
    const bool on = L.act && st[L.c].active;
    const R a = on ? (R)st[L.c].alpha : R(0);
    double d[2] = {0.0, 0.0};
    int64_t t0, t1;
    tile_range(((int64_t)nV + L.gpb - 1) / L.gpb, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i = tile * L.gpb + L.grp;
        if (i >= nV || !on) continue;
        const int64_t e = i * k + L.c;
        x[e] += a * p[e];
        const R rv = r[e] - a * q[e];
        const R zv = invD[i] * rv;
        r[e] = rv;
        z[e] = zv;
        d[0] += (double)rv * (double)zv;
        d[1] += (double)rv * (double)rv;
    }
    column_partials(d, 2, k, G, on, s_red, s_part);
    if (!block_then_last(s_part, 2 * k, gpart, ticket, s_tot, s_scr)) return;
    if ((int)threadIdx.x < k) {
        CgCol &s = st[threadIdx.x];
        if (s.active) {
            const double rz_new = s_tot[threadIdx.x], rr = s_tot[k + threadIdx.x];
            s.beta = s.rz != 0.0 ? rz_new / s.rz : 0.0;
            s.rz = rz_new;
            s.rr = rr;
            s.iters += 1;
            if (rr < s.best) {
                s.best = rr;
                s.since = 0;
            } else {
                s.since += 1;
            }
            if (!prm.fixed && sqrt(rr) <= prm.rtol * sqrt(s.bb)) {
                s.converged = 1;
                s.active = 0;
            } else if (s.iters >= prm.max_iter) {
                s.active = 0;
            } else if (!prm.fixed && prm.stall > 0 && s.since >= prm.stall) {
                s.stalled = 1;
                s.active = 0;
            }
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(T)
k_cg_pupdate(int32_t nV, int k, int G, R *__restrict__ p, const R *__restrict__ z,
             const CgCol *st) {
    const VLane L = vlane(k, G);
    if (!L.act || !st[L.c].active) return;
    const R bt = (R)st[L.c].beta;
    int64_t t0, t1;
    tile_range(((int64_t)nV + L.gpb - 1) / L.gpb, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i = tile * L.gpb + L.grp;
        if (i >= nV) continue;
        const int64_t e = i * k + L.c;
        p[e] = z[e] + bt * p[e];
    }
}

// 1 / (alpha M_ii + beta K_ii); zero on masked rows.
template <typename R>
__global__ void k_cg_invdiag(int32_t nV, R alpha, const R *__restrict__ M, R beta,
                             const R *__restrict__ K, const int32_t *__restrict__ diag,
                             const uint8_t *__restrict__ mask, R *__restrict__ invD) {
    const int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= nV) return;
    invD[i] = (mask && mask[i]) ? R(0) : R(1) / (alpha * M[i] + beta * K[diag[i]]);
}

// Dirichlet lift: beff_I = b_I - A_IB g_B, beff_B = 0, and u_B = g_B.
template <typename R>
__global__ void k_cg_lift(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                          int32_t nV, R alpha, const R *__restrict__ M, R beta,
                          const R *__restrict__ K, const uint8_t *__restrict__ mask, int k,
                          const R *__restrict__ b, const R *__restrict__ g, R *__restrict__ beff,
                          R *__restrict__ u) {
    const int64_t e = (int64_t)blockIdx.x * T + threadIdx.x;
    if (e >= (int64_t)nV * k) return;
    const int32_t i = (int32_t)(e / k);
    const int c = (int)(e % k);
    if (mask[i]) {
        beff[e] = R(0);
        u[e] = g[e];
        return;
    }
    R s = b[e];
    for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
        const int32_t j = col[t];
        if (!mask[j]) continue;
        R a = beta * K[t];
        if (j == i) a += alpha * M[i];
        s -= a * g[(int64_t)j * k + c];
    }
    beff[e] = s;
}

// ||beff - A_II u||^2 per column with FP64 accumulation.
template <typename R>
__global__ void __launch_bounds__(T)
k_cg_trueres(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t nV,
             double alpha, const R *__restrict__ M, double beta, const R *__restrict__ K,
             const uint8_t *__restrict__ mask, int k, int G, const R *__restrict__ beff,
             const R *__restrict__ u, double *gpart, uint32_t *ticket, double *out) {
    __shared__ double s_part[kMaxK];
    __shared__ double s_tot[kMaxK];
    __shared__ double s_scr[T];
    __shared__ double s_red[T];
    const VLane L = vlane(k, G);
    double d = 0.0;
    int64_t t0, t1;
    tile_range(((int64_t)nV + L.gpb - 1) / L.gpb, t0, t1);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i = tile * L.gpb + L.grp;
        if (i >= nV || !L.act || (mask && mask[i])) continue;
        double s = (double)beff[i * k + L.c];
        for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
            const int32_t j = col[t];
            if (mask && mask[j]) continue;
            double a = beta * (double)K[t];
            if (j == i) a += alpha * (double)M[i];
            s -= a * (double)u[(int64_t)j * k + L.c];
        }
        d += s * s;
    }
    column_partials(&d, 1, k, G, L.act, s_red, s_part);
    if (!block_then_last(s_part, k, gpart, ticket, s_tot, s_scr)) return;
    if ((int)threadIdx.x < k) out[threadIdx.x] = s_tot[threadIdx.x];
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

unsigned red_blocks(int64_t ntiles) {
    int64_t b = ntiles < kMaxRedBlocks ? ntiles : kMaxRedBlocks;
    return (unsigned)(b < 1 ? 1 : b);
}

unsigned stream_blocks(int64_t ntiles) {
    const int64_t cap = 256 * 16;
    int64_t b = ntiles < cap ? ntiles : cap;
    return (unsigned)(b < 1 ? 1 : b);
}

template <typename R>
dgo_status run_pcg(const dgo_mesh *m, double alpha, const R *M, double beta, const R *K,
                   const uint8_t *mask, const R *g, int k, const R *b, R *u, const dgo_cg_opts &o,
                   dgo_cg_report *rep, hipStream_t s) {
    const int64_t nV = m->nV, n = nV * k;
    const Layout sl = spmm_layout(k);
    const int Gv = pow2ceil(k);
    // workspace: r z p q beff invD | partials | tickets | state | trueres
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t vec = al(sizeof(R) * (size_t)n);
    const size_t off_r = 0, off_z = vec, off_p = 2 * vec, off_q = 3 * vec, off_b = 4 * vec;
    const size_t off_d = 5 * vec, off_part = off_d + al(sizeof(R) * (size_t)nV);
    const size_t off_tk = off_part + al(sizeof(double) * kMaxRedBlocks * 3 * kMaxK);
    const size_t off_st = off_tk + 256;
    const size_t off_tr = off_st + al(sizeof(CgCol) * kMaxK);
    const size_t total = off_tr + al(sizeof(double) * kMaxK);
    void *wsv;
    DGO_TRY(mesh_workspace(const_cast<dgo_mesh *>(m), total, s, &wsv));
    char *ws = (char *)wsv;
    R *r = (R *)(ws + off_r), *z = (R *)(ws + off_z), *p = (R *)(ws + off_p), *q = (R *)(ws + off_q);
    R *beff = mask ? (R *)(ws + off_b) : const_cast<R *>(b);
    R *invD = (R *)(ws + off_d);
    double *gpart = (double *)(ws + off_part);
    uint32_t *ticket = (uint32_t *)(ws + off_tk);
    CgCol *st = (CgCol *)(ws + off_st);
    double *tr = (double *)(ws + off_tr);

    CgParams prm;
    prm.rtol = o.rtol;
    prm.max_iter = o.max_iter;
    prm.fixed = o.fixed_iters;
    prm.stall = o.stall_iters;
    prm.k = k;

    const int gpb_s = T / sl.G, gpb_v = T / Gv;
    const int64_t tiles_s = (nV + gpb_s - 1) / gpb_s, tiles_v = (nV + gpb_v - 1) / gpb_v;
    const unsigned nb_s = red_blocks(tiles_s), nb_v = red_blocks(tiles_v);
    const R ra = (R)alpha, rb = (R)beta;

    k_zero_u32<<<1, 64, 0, s>>>(ticket, 64);
    DGO_LAUNCH("cg_invdiag", s, k_cg_invdiag<R><<<grid_for(nV, T), T, 0, s>>>((int32_t)nV, ra, M, rb, K, m->diag, mask, invD));
    if (mask)
        DGO_LAUNCH("cg_lift", s, k_cg_lift<R><<<grid_for(n, T), T, 0, s>>>(m->rowptr, m->col, (int32_t)nV, ra, M, rb, K, mask,
                                                  k, b, g, beff, u));
    // r0 = beff - A_II x0
    DGO_LAUNCH("cg_spmm_dot", s, k_cg_spmm_dot<R><<<nb_s, T, 0, s>>>(m->rowptr, m->col, (int32_t)nV, ra, M, rb, K, mask, k, sl.G,
                                        sl.parts, u, q, 0, gpart, ticket, st));
    DGO_LAUNCH("cg_init", s, k_cg_init<R><<<nb_v, T, 0, s>>>((int32_t)nV, k, Gv, beff, q, invD, r, z, p, gpart, ticket + 1, st,
                                    prm));
    DGO_HIP(hipGetLastError());

    const int every = o.fixed_iters ? (o.max_iter > 0 ? o.max_iter : 1)
                                    : (o.check_every > 0 ? o.check_every : 8);
    CgCol hst[kMaxK];
    int32_t done_iters = 0;
    for (;;) {
        const int32_t chunk = std::min(every, o.max_iter - done_iters);
        if (chunk <= 0) break;
        for (int32_t it = 0; it < chunk; ++it) {
            DGO_LAUNCH("cg_spmm_dot", s, k_cg_spmm_dot<R><<<nb_s, T, 0, s>>>(m->rowptr, m->col, (int32_t)nV, ra, M, rb, K, mask,
                                                k, sl.G, sl.parts, p, q, 1, gpart, ticket + 2, st));
            DGO_LAUNCH("cg_update", s, k_cg_update<R><<<nb_v, T, 0, s>>>((int32_t)nV, k, Gv, u, r, z, p, q, invD, gpart,
                                              ticket + 3, st, prm));
            DGO_LAUNCH("cg_pupdate", s, k_cg_pupdate<R><<<stream_blocks(tiles_v), T, 0, s>>>((int32_t)nV, k, Gv, p, z, st));
        }
        DGO_HIP(hipGetLastError());
        done_iters += chunk;
        DGO_HIP(hipMemcpyAsync(hst, st, sizeof(CgCol) * k, hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int c = 0; c < k; ++c) any = any || hst[c].active;
        if (!any) break;
    }
    // final state and the true residual in FP64
    DGO_LAUNCH("cg_trueres", s, k_cg_trueres<R><<<nb_v, T, 0, s>>>(m->rowptr, m->col, (int32_t)nV, alpha, M, beta, K, mask, k, Gv,
                                       beff, u, gpart, ticket + 4, tr));
    DGO_HIP(hipGetLastError());
    double htr[kMaxK];
    DGO_HIP(hipMemcpyAsync(hst, st, sizeof(CgCol) * k, hipMemcpyDeviceToHost, s));
    DGO_HIP(hipMemcpyAsync(htr, tr, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    DGO_HIP(hipStreamSynchronize(s));
    bool all = true;
    for (int c = 0; c < k; ++c) all = all && hst[c].converged;
    if (rep) {
        rep->k = k;
        rep->converged_all = all ? 1 : 0;
        for (int c = 0; c < k; ++c) {
            const double bn = sqrt(hst[c].bb);
            rep->iters[c] = hst[c].iters;
            rep->relres[c] = bn > 0 ? sqrt(hst[c].rr) / bn : sqrt(hst[c].rr);
            rep->true_relres[c] = bn > 0 ? sqrt(htr[c]) / bn : sqrt(htr[c]);
        }
    }
    if (!all && !o.fixed_iters) {
        if (o.strict) return fail(DGO_ERR_NOT_CONVERGED, "dgo_pcg: a column did not reach rtol");
        if (getenv("DGO_LOG") && atoi(getenv("DGO_LOG")) > 0)
            fprintf(stderr, "dgo_pcg: warning: not every column reached rtol\n");
    }
    return DGO_OK;
}

}  // namespace
}  // namespace dgo

using namespace dgo;

extern "C" dgo_status dgo_spmv(const dgo_mesh *m, dgo_dtype dtype, int32_t batch, double alpha,
                               const void *d_Mdiag, double beta, const void *d_Kvals, int32_t k,
                               const void *d_x, void *d_y, dgo_stream stream) {
    clear_error();
    if (!m || !d_Mdiag || !d_Kvals || !d_x || !d_y)
        return fail(DGO_ERR_INVALID_ARG, "dgo_spmv: NULL argument");
    if (k < 1 || k > kMaxK) return fail(DGO_ERR_INVALID_ARG, "dgo_spmv: k must be in [1, 64]");
    if (batch < 1 || batch > 65535) return fail(DGO_ERR_INVALID_ARG, "dgo_spmv: bad batch");
    if (d_x == d_y) return fail(DGO_ERR_INVALID_ARG, "dgo_spmv: x and y alias");
    if (dtype != DGO_F32 && dtype != DGO_F64) return fail(DGO_ERR_INVALID_ARG, "dgo_spmv: bad dtype");
    hipStream_t s = (hipStream_t)stream;
    const Layout L = spmm_layout(k);
    const int gpb = T / L.G;
    const int64_t tiles = ((int64_t)m->nV + gpb - 1) / gpb;
    dim3 grid(stream_blocks(tiles), (unsigned)batch);
    if (dtype == DGO_F64)
        DGO_LAUNCH("spmm", s,
                   k_spmm<double><<<grid, T, 0, s>>>(m->rowptr, m->col, m->nV, m->nnz, alpha,
                                                     (const double *)d_Mdiag, beta,
                                                     (const double *)d_Kvals, k, L.G, L.parts,
                                                     (const double *)d_x, (double *)d_y));
    else
        DGO_LAUNCH("spmm", s,
                   k_spmm<float><<<grid, T, 0, s>>>(m->rowptr, m->col, m->nV, m->nnz, (float)alpha,
                                                    (const float *)d_Mdiag, (float)beta,
                                                    (const float *)d_Kvals, k, L.G, L.parts,
                                                    (const float *)d_x, (float *)d_y));
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

extern "C" dgo_status dgo_pcg(const dgo_mesh *m, dgo_dtype dtype, double alpha, const void *d_Mdiag,
                              double beta, const void *d_Kvals, const uint8_t *d_mask,
                              const void *d_g, int32_t k, const void *d_b, void *d_u,
                              const dgo_cg_opts *opts, dgo_cg_report *h_rep, dgo_stream stream) {
    clear_error();
    if (!m || !d_Mdiag || !d_Kvals || !d_b || !d_u)
        return fail(DGO_ERR_INVALID_ARG, "dgo_pcg: NULL argument");
    if (k < 1 || k > kMaxK) return fail(DGO_ERR_INVALID_ARG, "dgo_pcg: k must be in [1, 64]");
    if (d_mask && !d_g) return fail(DGO_ERR_INVALID_ARG, "dgo_pcg: mask given without g");
    if (dtype != DGO_F32 && dtype != DGO_F64) return fail(DGO_ERR_INVALID_ARG, "dgo_pcg: bad dtype");
    dgo_cg_opts o;
    if (opts) {
        o = *opts;
    } else {
        o.rtol = 1e-8;
        o.max_iter = 1000;
        o.fixed_iters = 0;
        o.check_every = 8;
        o.stall_iters = 0;
        o.strict = 0;
    }
    if (o.max_iter < 0 || !(o.rtol >= 0.0)) return fail(DGO_ERR_INVALID_ARG, "dgo_pcg: bad options");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == DGO_F64)
        return run_pcg<double>(m, alpha, (const double *)d_Mdiag, beta, (const double *)d_Kvals,
                               d_mask, (const double *)d_g, k, (const double *)d_b, (double *)d_u, o,
                               h_rep, s);
    return run_pcg<float>(m, alpha, (const float *)d_Mdiag, beta, (const float *)d_Kvals, d_mask,
                          (const float *)d_g, k, (const float *)d_b, (float *)d_u, o, h_rep, s);
}
