// Smallest generalized eigenpairs K u = lam M u of a mesh operator (the
// forward pass of the spectral implicit layers, Sec. 5.2): subspace iteration
// on the shift-invert operator (K - sigma M)^-1 M with Rayleigh-Ritz, whose
// fixed point is the relation U = Q((A - sigma B)^-1 B U) of Eq. eigiter
// (Q: B-orthonormalization with a canonical sign per column).
//
// One outer iteration on a block of p >= k columns:
//   1. Y = (K - sigma M)^-1 M U by Jacobi PCG (the library's solver, all p
//      columns at once), warm-started at U diag(1 / (theta - sigma)), the
//      exact solution once U holds eigenvectors;
//   2. KY by the SpMV kernel;
//   3. the p x p Gram matrices G = Y^T M Y and H = Y^T K Y (fixed-order
//      reductions, FP64 accumulation);
//   4. on the host: H c = theta G c by Cholesky and cyclic Jacobi (p <= 64);
//   5. U = Y C, KU = KY C, then the residuals ||K u_j - theta_j M u_j||_{M^-1}.
// Each inner solve stops once its residual is a tenth of the warm start's (or
// below the absolute floor): the outer iteration count stays the same while the
// inner work drops several fold (at icosphere level 7 with 9 pairs: 22k -> 2.9k
// PCG iterations, eigenvalues equal to 1e-14).
// The first iteration applies Rayleigh-Ritz to a pseudo-random start block
// (splitmix64). Every reduction has a fixed order, so the result is bitwise
// deterministic. The paper's GPU eigensolver is power iteration; on mesh
// Laplacians the smallest eigenvalues are too clustered for it (the ratio of
// consecutive eigenvalues of the unshifted operator tends to 1 as meshes grow),
// so the inverse is applied by the same PCG as the linear solves instead.
#include "internal.hpp"
#include "kernels.hpp"
#include "dense_small.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace dgo {
namespace {

constexpr int ET = 256;        // threads of the elementwise and reduction kernels
constexpr int kGramTile = 32;  // rows per LDS tile of the Gram kernel
constexpr int kEigMaxP = 64;   // largest block (the PCG's column limit)
constexpr int kMaxParts = 512; // most partial-sum blocks of a reduction

// splitmix64 (Steele, Lea and Flood 2014; the constants of Vigna's reference
// implementation): output number o of the stream that starts at `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t o) {
    uint64_t z = seed + (o + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename R>
__global__ void k_eig_random(int64_t n, uint64_t seed, R *__restrict__ Y) {
    const int64_t o = (int64_t)blockIdx.x * ET + threadIdx.x;
    if (o >= n) return;
    const double u = (double)(splitmix64(seed, (uint64_t)o) >> 11) * 0x1.0p-53;
    Y[o] = R(2.0 * u - 1.0);
}

// Partial Gram sums of the rows [blockIdx.x * chunk, ...): per pair q = a p + c
//   G_q = sum_i M_i Y_ia Y_ic,  H_q = sum_i Y_ia Z_ic.
// Rows are staged in LDS tiles; each thread owns pairs t, t + ET, ...
template <typename R>
__global__ void __launch_bounds__(ET)
k_eig_gram(int64_t n, int p, int64_t chunk, const R *__restrict__ Y, const R *__restrict__ Z,
           const R *__restrict__ M, double *__restrict__ partG, double *__restrict__ partH) {
    __shared__ double ys[kGramTile * kEigMaxP], zs[kGramTile * kEigMaxP], ms[kGramTile];
    constexpr int PPT = kEigMaxP * kEigMaxP / ET;
    const int t = threadIdx.x, pp = p * p;
    const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    double g[PPT], h[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) g[u] = h[u] = 0.0;
    for (int64_t base = r0; base < r1; base += kGramTile) {
        const int rows = (int)min((int64_t)kGramTile, r1 - base);
        __syncthreads();
        for (int e = t; e < rows * p; e += ET) {
            ys[e] = (double)Y[base * p + e];
            zs[e] = (double)Z[base * p + e];
        }
        for (int e = t; e < rows; e += ET) ms[e] = (double)M[base + e];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int q = t + u * ET;
            if (q < pp) {
                const int a = q / p, c = q - a * p;
                for (int r = 0; r < rows; ++r) {
                    const double ya = ys[r * p + a];
                    g[u] += ms[r] * ya * ys[r * p + c];
                    h[u] += ya * zs[r * p + c];
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        const int q = t + u * ET;
        if (q < pp) {
            partG[(int64_t)blockIdx.x * pp + q] = g[u];
            partH[(int64_t)blockIdx.x * pp + q] = h[u];
        }
    }
}

// Sum the partials of each pair over the blocks: one workgroup per pair,
// thread t adds blocks t, t + ET, ... in order, then a fixed-shape tree in
// LDS; the same order on every run.
__global__ void __launch_bounds__(ET)
k_eig_gram_final(int nblk, int pp, const double *__restrict__ partG,
                 const double *__restrict__ partH, double *__restrict__ GH) {
    __shared__ double sg[ET], sh[ET];
    const int q = blockIdx.x, t = threadIdx.x;
    double g = 0.0, h = 0.0;
    for (int b = t; b < nblk; b += ET) {
        g += partG[(int64_t)b * pp + q];
        h += partH[(int64_t)b * pp + q];
    }
    sg[t] = g;
    sh[t] = h;
    __syncthreads();
    for (int w = ET / 2; w > 0; w /= 2) {
        if (t < w) {
            sg[t] += sg[t + w];
            sh[t] += sh[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        GH[q] = sg[0];
        GH[pp + q] = sh[0];
    }
}

// U = Y C, KU = KY C (C: p x p, FP64, staged in LDS)
template <typename R>
__global__ void __launch_bounds__(ET)
k_eig_combine(int64_t n, int p, const R *__restrict__ Y, const R *__restrict__ KY,
              const double *__restrict__ C, R *__restrict__ U, R *__restrict__ KU) {
    __shared__ double cs[kEigMaxP * kEigMaxP];
    for (int e = threadIdx.x; e < p * p; e += ET) cs[e] = C[e];
    __syncthreads();
    const int64_t o = (int64_t)blockIdx.x * ET + threadIdx.x;
    if (o >= n * p) return;
    const int64_t i = o / p;
    const int j = (int)(o - i * p);
    double u = 0.0, ku = 0.0;
    for (int b = 0; b < p; ++b) {
        const double c = cs[b * p + j];
        u += (double)Y[i * p + b] * c;
        ku += (double)KY[i * p + b] * c;
    }
    U[o] = R(u);
    KU[o] = R(ku);
}

// Per column j, over the rows of this block: sum_i (KU_ij - theta_j M_i U_ij)^2 / M_i,
// and the largest |U_ij| with its smallest row index.
template <typename R>
__global__ void __launch_bounds__(ET)
k_eig_resid(int64_t n, int p, int64_t chunk, const R *__restrict__ U, const R *__restrict__ KU,
            const R *__restrict__ M, const double *__restrict__ theta, double *__restrict__ part) {
    __shared__ double ssum[ET], smax[ET];
    __shared__ int64_t sidx[ET];
    const int t = threadIdx.x, rstride = ET / p, j = t % p, roff = t / p;
    const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    double acc = 0.0, amax = -1.0;
    int64_t aidx = -1;
    if (roff < rstride) {
        const double th = theta[j];
        for (int64_t i = r0 + roff; i < r1; i += rstride) {
            const double mi = (double)M[i], u = (double)U[i * p + j];
            const double d = (double)KU[i * p + j] - th * mi * u;
            acc += d * d / mi;
            if (fabs(u) > amax) {
                amax = fabs(u);
                aidx = i;
            }
        }
    }
    ssum[t] = acc;
    smax[t] = amax;
    sidx[t] = aidx;
    __syncthreads();
    if (t < p) {
        double s = 0.0, mx = -1.0;
        int64_t ix = -1;
        for (int r = 0; r < rstride; ++r) {
            const int w = r * p + t;
            s += ssum[w];
            if (smax[w] > mx || (smax[w] == mx && sidx[w] >= 0 && sidx[w] < ix)) {
                mx = smax[w];
                ix = sidx[w];
            }
        }
        double *out = part + (int64_t)blockIdx.x * 3 * p;
        out[t] = s;
        out[p + t] = mx;
        out[2 * p + t] = (double)ix;
    }
}

// Reduce the per-block column results, one workgroup per column (the same
// fixed order as the Gram reduction): out[j] = residual sum, out[p + j] =
// signed value of the largest-magnitude entry (the first on ties).
template <typename R>
__global__ void __launch_bounds__(ET)
k_eig_resid_final(int nblk, int p, const double *__restrict__ part, const R *__restrict__ U,
                  double *__restrict__ out) {
    __shared__ double ss[ET], sm[ET];
    __shared__ int64_t si[ET];
    const int j = blockIdx.x, t = threadIdx.x;
    double s = 0.0, mx = -1.0;
    int64_t ix = -1;
    for (int b = t; b < nblk; b += ET) {
        const double *pb = part + (int64_t)b * 3 * p;
        s += pb[j];
        const int64_t bi = (int64_t)pb[2 * p + j];
        if (pb[p + j] > mx) {  // blocks visited in increasing row order
            mx = pb[p + j];
            ix = bi;
        }
    }
    ss[t] = s;
    sm[t] = mx;
    si[t] = ix;
    __syncthreads();
    for (int w = ET / 2; w > 0; w /= 2) {
        if (t < w) {
            ss[t] += ss[t + w];
            const double m2 = sm[t + w];
            const int64_t i2 = si[t + w];
            if (m2 > sm[t] || (m2 == sm[t] && i2 >= 0 && (si[t] < 0 || i2 < si[t]))) {
                sm[t] = m2;
                si[t] = i2;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        out[j] = ss[0];
        out[p + j] = si[0] >= 0 ? (double)U[si[0] * p + j] : 0.0;
    }
}

// B = M U (the right-hand sides) and X = U diag(s) (the warm start)
template <typename R>
__global__ void k_eig_rhs(int64_t n, int p, const R *__restrict__ U, const R *__restrict__ M,
                          const double *__restrict__ sc, R *__restrict__ B, R *__restrict__ X) {
    const int64_t o = (int64_t)blockIdx.x * ET + threadIdx.x;
    if (o >= n * p) return;
    const int64_t i = o / p;
    const int j = (int)(o - i * p);
    const R u = U[o];
    B[o] = M[i] * u;
    X[o] = R((double)u * sc[j]);
}

template <typename R>
__global__ void k_eig_out(int64_t n, int p, int k, const R *__restrict__ U,
                          const double *__restrict__ sign, R *__restrict__ out) {
    const int64_t o = (int64_t)blockIdx.x * ET + threadIdx.x;
    if (o >= n * k) return;
    const int64_t i = o / k;
    const int j = (int)(o - i * k);
    out[o] = R(sign[j] * (double)U[i * p + j]);
}

struct DevBufs {
    const dgo_mesh *m;
    hipStream_t s;
    std::vector<void *> ptrs;
    void *get(size_t bytes) {
        void *p = m->alloc.get(bytes, s);
        if (p) ptrs.push_back(p);
        return p;
    }
    ~DevBufs() {
        for (void *p : ptrs) m->alloc.put(p, s);
    }
};

template <typename R>
dgo_status run_eigs(const dgo_mesh *m, dgo_dtype dt, const R *M, const R *K, int k,
                    const dgo_eig_opts &o, R *Uout, double *lam, dgo_eig_report *rep,
                    hipStream_t s) {
    const int64_t n = m->nV;
    const int p = o.block;
    const int pp = p * p;
    const int nblk = (int)std::min<int64_t>(kMaxParts, (n + 63) / 64);
    const int64_t chunk = (n + nblk - 1) / nblk;
    DevBufs buf{m, s, {}};
    const size_t vb = sizeof(R) * (size_t)n * p;
    R *U = (R *)buf.get(vb), *Y = (R *)buf.get(vb), *KY = (R *)buf.get(vb), *KU = (R *)buf.get(vb),
      *B = (R *)buf.get(vb);
    double *partG = (double *)buf.get(sizeof(double) * (size_t)nblk * pp);
    double *partH = (double *)buf.get(sizeof(double) * (size_t)nblk * pp);
    double *small = (double *)buf.get(sizeof(double) * (size_t)(2 * pp + pp + 4 * p));
    double *partR = (double *)buf.get(sizeof(double) * (size_t)nblk * 3 * p);
    if (buf.ptrs.size() != 9) return fail(DGO_ERR_NOMEM, "dgo_eigs_smallest: workspace allocation failed");
    double *GH = small, *Cd = small + 2 * pp, *vec = small + 3 * pp, *rout = vec + p;

    double sigma = o.sigma;
    const double tol = o.tol;
    dgo_cg_opts co{};
    co.rtol = o.inner_rtol;
    co.rtol_initial = o.inner_rtol_initial > 0.0 ? o.inner_rtol_initial : 0.0;
    co.max_iter = o.inner_max_iter;
    co.check_every = 8;
    co.stall_iters = dt == DGO_F32 ? 50 : 0;
    dgo_cg_report cr{};

    std::vector<double> hGH(2 * (size_t)pp), theta, C, hr(2 * (size_t)p), hv(p);
    int it = 0;
    int64_t inner = 0;
    bool conv = false;
    std::vector<double> res(p, 0.0);
    k_eig_random<R><<<grid_for(n * p, ET), ET, 0, s>>>(n * p, o.seed, Y);
    DGO_HIP(hipGetLastError());
    for (;; ++it) {
        if (it > 0) {
            for (int j = 0; j < p; ++j) hv[j] = 1.0 / (theta[j] - sigma);
            DGO_HIP(hipMemcpyAsync(vec, hv.data(), sizeof(double) * p, hipMemcpyHostToDevice, s));
            k_eig_rhs<R><<<grid_for(n * p, ET), ET, 0, s>>>(n, p, U, M, vec, B, Y);
            DGO_HIP(hipGetLastError());
            DGO_TRY(dgo_pcg(m, dt, -sigma, M, 1.0, K, nullptr, nullptr, p, B, Y, &co, &cr,
                            (dgo_stream)s));
            int mx = 0;
            for (int j = 0; j < p; ++j) mx = std::max(mx, cr.iters[j]);
            inner += mx;
        }
        DGO_TRY(dgo_spmv(m, dt, 1, 0.0, M, 1.0, K, p, Y, KY, (dgo_stream)s));
        k_eig_gram<R><<<nblk, ET, 0, s>>>(n, p, chunk, Y, KY, M, partG, partH);
        k_eig_gram_final<<<pp, ET, 0, s>>>(nblk, pp, partG, partH, GH);
        DGO_HIP(hipGetLastError());
        DGO_HIP(hipMemcpyAsync(hGH.data(), GH, sizeof(double) * 2 * pp, hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        std::vector<double> G(hGH.begin(), hGH.begin() + pp), H(hGH.begin() + pp, hGH.end());
        if (!dense::rayleigh_ritz(G, H, p, theta, C))
            return fail(DGO_ERR_NOT_CONVERGED, "dgo_eigs_smallest: the iterated block lost rank");
        DGO_HIP(hipMemcpyAsync(Cd, C.data(), sizeof(double) * pp, hipMemcpyHostToDevice, s));
        DGO_HIP(hipMemcpyAsync(vec, theta.data(), sizeof(double) * p, hipMemcpyHostToDevice, s));
        DGO_LAUNCH("eig_rayleigh_ritz", s, {
            k_eig_combine<R><<<grid_for(n * p, ET), ET, 0, s>>>(n, p, Y, KY, Cd, U, KU);
            k_eig_resid<R><<<nblk, ET, 0, s>>>(n, p, chunk, U, KU, M, vec, partR);
            k_eig_resid_final<R><<<p, ET, 0, s>>>(nblk, p, partR, U, rout);
        });
        DGO_HIP(hipGetLastError());
        DGO_HIP(hipMemcpyAsync(hr.data(), rout, sizeof(double) * 2 * p, hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        conv = it > 0;
        for (int j = 0; j < p; ++j) {
            res[j] = std::sqrt(hr[j]) / std::max(std::fabs(theta[j]), std::fabs(sigma));
            if (j < k && !(res[j] <= tol)) conv = false;
        }
        if (conv || it >= o.max_iter) break;
    }
    // canonical signs: the largest-magnitude entry of each column positive
    for (int j = 0; j < k; ++j) hv[j] = hr[p + j] < 0.0 ? -1.0 : 1.0;
    DGO_HIP(hipMemcpyAsync(vec, hv.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    k_eig_out<R><<<grid_for(n * k, ET), ET, 0, s>>>(n, p, k, U, vec, Uout);
    DGO_HIP(hipGetLastError());
    DGO_HIP(hipStreamSynchronize(s));  // the workspace is released on return
    for (int j = 0; j < k; ++j) lam[j] = theta[j];
    if (rep) {
        rep->k = k;
        rep->block = p;
        rep->iters = it;
        rep->inner_iters = inner;
        rep->converged = conv ? 1 : 0;
        rep->sigma = sigma;
        for (int j = 0; j < k; ++j) rep->resid[j] = res[j];
    }
    return DGO_OK;
}

}  // namespace
}  // namespace dgo

using namespace dgo;

extern "C" dgo_status dgo_eigs_smallest(const dgo_mesh *m, dgo_dtype dtype, const void *d_Mdiag,
                                        const void *d_Kvals, int32_t k, const dgo_eig_opts *opts,
                                        void *d_U, double *h_lambda, dgo_eig_report *h_rep,
                                        dgo_stream stream) {
    clear_error();
    if (!m || !d_Mdiag || !d_Kvals || !d_U || !h_lambda)
        return fail(DGO_ERR_INVALID_ARG, "dgo_eigs_smallest: NULL argument");
    if (dtype != DGO_F32 && dtype != DGO_F64)
        return fail(DGO_ERR_INVALID_ARG, "dgo_eigs_smallest: bad dtype");
    dgo_eig_opts o{};
    if (opts) o = *opts;
    if (k < 1 || k > kEigMaxP || k > m->nV)
        return fail(DGO_ERR_INVALID_ARG, "dgo_eigs_smallest: k must be in [1, min(64, nV)]");
    // default block: the power of two with at least 6 guard columns (the PCG
    // pads its columns to a power of two, so other sizes cost the same lanes)
    if (o.block == 0)
        o.block = std::max<int64_t>(
            k, std::min<int64_t>({(int64_t)kEigMaxP, (int64_t)m->nV, (int64_t)kern::pow2ceil(k + 6)}));
    if (o.block < k || o.block > kEigMaxP || o.block > m->nV)
        return fail(DGO_ERR_INVALID_ARG, "dgo_eigs_smallest: block must be in [k, min(64, nV)]");
    hipStream_t s = (hipStream_t)stream;
    if (o.sigma == 0.0) {
        // default shift: minus the reciprocal of the total measure (sum of M),
        // a fraction of the smallest nonzero eigenvalue of typical domains
        const size_t es = dtype == DGO_F64 ? sizeof(double) : sizeof(float);
        std::vector<unsigned char> hm(es * (size_t)m->nV);
        DGO_HIP(hipMemcpyAsync(hm.data(), d_Mdiag, hm.size(), hipMemcpyDeviceToHost, s));
        DGO_HIP(hipStreamSynchronize(s));
        double tot = 0.0;
        for (int32_t i = 0; i < m->nV; ++i)
            tot += dtype == DGO_F64 ? ((const double *)hm.data())[i] : (double)((const float *)hm.data())[i];
        if (!(tot > 0.0)) return fail(DGO_ERR_INVALID_ARG, "dgo_eigs_smallest: M must be positive");
        o.sigma = -1.0 / tot;
    }
    if (!(o.sigma < 0.0))
        return fail(DGO_ERR_INVALID_ARG, "dgo_eigs_smallest: sigma must be negative");
    if (o.tol <= 0.0) o.tol = dtype == DGO_F64 ? 1e-8 : 1e-4;
    if (o.inner_rtol <= 0.0) o.inner_rtol = 0.1 * o.tol;
    if (o.inner_rtol_initial == 0.0) o.inner_rtol_initial = 0.1;
    if (o.inner_max_iter <= 0) o.inner_max_iter = 20000;
    if (o.max_iter <= 0) o.max_iter = 200;
    if (dtype == DGO_F64)
        return run_eigs<double>(m, dtype, (const double *)d_Mdiag, (const double *)d_Kvals, k, o,
                                (double *)d_U, h_lambda, h_rep, s);
    return run_eigs<float>(m, dtype, (const float *)d_Mdiag, (const float *)d_Kvals, k, o,
                           (float *)d_U, h_lambda, h_rep, s);
}
