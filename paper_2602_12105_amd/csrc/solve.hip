// Operator application y = (alpha M + beta K) x and Jacobi-preconditioned
// conjugate gradients on it.
//
// SpMV/SpMM. x and y are vertex-major (nV x k). A CSR row is handled by a
// group of G = max(KP, 8) lanes of a 64-lane wavefront (KP = k rounded up to a
// power of two). The group first loads G consecutive entries of the row at
// once (column id and value, one entry per lane), then every lane takes the
// entries of its part (G / KP parts) from its neighbours by cross-lane
// shuffles and gathers x for its column c = lane % KP; the gathers of one
// chunk are independent, so they are all in flight together. Parts are
// combined by a fixed shuffle tree. The operator alpha M + beta K is never
// formed: the mass term is added on the diagonal entry. Rows are visited in
// the mesh's breadth-first row order when it has one (large meshes), so that
// each XCD's contiguous share of rows gathers mostly x rows of its own share.
//
// PCG: Jacobi-preconditioned conjugate gradients (Saad, Alg. 9.1) in the
// one-reduction arrangement of Chronopoulos and Gear: the recurrence s = A p
// is carried along, so that the three dots an iteration needs (r.z, r.r of the
// new residual and w.z with w = A z) belong to one residual and are reduced
// together. An iteration is two kernels:
//   1. vector update: every workgroup first adds the previous iteration's
//      partial sums in the same fixed order and advances the per-column state
//      (beta, alpha, stopping tests), then p = z + beta p, s = w + beta s,
//      r -= alpha s, with partial sums of r.z and r.r (z = D^-1 r); x takes
//      the steps of two iterations at once every second iteration
//      (x += alpha' p' + alpha p), which saves one read and one write of x
//      per pair, and the last odd step is added when the solution is copied
//      out;
//   2. w = A z, fused with partial sums of w.z; A z is one sweep over the
//      values v_ij = A_ij d_j prepared once per solve (d = D^-1).
// Every dot is reduced in a fixed order: each workgroup stores its
// per-column partial sums with plain stores and the next kernel adds them in
// a fixed order; the kernel boundary orders the stores before the reads, so
// no device-scope fence is issued per workgroup (each such fence writes back
// the XCD's L2). Results are bitwise deterministic run to run. Columns stop
// independently and are frozen once stopped.
#include "internal.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

namespace dgo {
namespace {

using namespace kern;

// Rows are taken in the mesh's row order: position r holds row i = rdesc[r].x
// whose entries start at rdesc[r].y, rlen[r] of them (one load level instead
// of order -> row pointers).
template <typename R, int KP, int G = (KP < 8 ? 8 : KP)>
__global__ void __launch_bounds__(T, KP <= 16 ? 8 : 4)
k_spmm(const int2 *__restrict__ rdesc, const uint8_t *__restrict__ rlen,
       const int32_t *__restrict__ col, int32_t nV, int64_t nnz, R alpha,
       const R *__restrict__ M, R beta, const R *__restrict__ K, int k, const R *__restrict__ x,
       R *__restrict__ y, int wide) {
    constexpr int GPB = T / G;
    const int64_t bt = blockIdx.y;
    M += bt * nV;
    K += bt * nnz;
    x += bt * (int64_t)nV * k;
    y += bt * (int64_t)nV * k;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int gbase = (threadIdx.x & 63) - lane;
    constexpr int RU = KP <= 8 ? kSpmvRows : 1;
    int64_t t0, t1;
    tile_range(((int64_t)nV + GPB - 1) / GPB, t0, t1);
    if (KP == 8 && wide) {
        // k = 8 with x and y 16-byte aligned: 16-byte gathers
        constexpr int V = Piece<R>::V, LPR = 8 / V;
        for (int64_t tile = t0; tile < t1; ++tile) {
            const int64_t r = tile * GPB + grp;
            if (r >= nV) break;  // uniform over the lane group; later tiles are past nV too
            const int2 d = rdesc[r];
            const int32_t i = d.x, len = rlen[r];
            const R dt = alpha * M[i];
            Piece<R> acc;
#pragma unroll
            for (int c = 0; c < V; ++c) acc.v[c] = R(0);
            for (int32_t e0 = 0; e0 < len; e0 += 8) {
                int32_t cj = i;
                R aj = R(0);
                if (e0 + lane < len) {
                    const int32_t e = d.y + e0 + lane;
                    cj = col[e];
                    aj = beta * K[e];
                    if (cj == i) aj += dt;
                }
                wide8_chunk(cj, aj, x, lane, gbase, acc);
            }
            wide8_combine(acc);
            if (lane < LPR) st_piece(y + (int64_t)i * 8 + (lane % LPR) * V, acc);
        }
        return;
    }
    for (int64_t tile = t0; tile < t1; tile += RU) {
        int32_t i[RU], rb[RU], len[RU];
        bool ok[RU];
        R dt[RU], acc[RU], xi[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {  // uniform over the lane group
            const int64_t r = (tile + u) * GPB + grp;
            ok[u] = tile + u < t1 && r < nV;
            const int2 d = ok[u] ? rdesc[r] : make_int2(0, 0);
            i[u] = d.x;
            rb[u] = d.y;
            len[u] = ok[u] ? (int32_t)rlen[r] : 0;
            dt[u] = ok[u] ? alpha * M[d.x] : R(0);
        }
        if (!ok[0]) continue;
        rows_apply<R, G, KP, RU, false>(col, K, beta, dt, x, i, rb, len, ok, k, lane, gbase, acc, xi);
#pragma unroll
        for (int u = 0; u < RU; ++u)
            if (ok[u] && lane < k && lane < KP) y[(int64_t)i[u] * k + lane] = acc[u];
    }
}

// y = (alpha M_i) x_i: the operator with beta = 0 (a diagonal), one thread
// per entry of batch x nV x k.
template <typename R>
__global__ void k_diag_apply(int64_t n, int k, R alpha, const R *__restrict__ M,
                             const R *__restrict__ x, R *__restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * T + threadIdx.x;
    if (e >= n) return;
    const int64_t row = e / k;  // batch * nV + vertex
    y[e] = (alpha * M[row]) * x[e];
}

// The SpMM with 8 columns and 16-byte aligned x, y: 16-byte gathers (two
// FP64 or four FP32 columns per lane, see wide8_chunk) on 1024-thread
// workgroups, each walking its tiles in a two-stage software pipeline: while
// a tile's gathers are in flight, the next tile's row descriptor has arrived
// and its first eight entries are loaded, and the descriptor of the tile
// after that is loaded.
template <typename R>
__global__ void __launch_bounds__(TR)
k_spmm8_pipe(const int2 *__restrict__ rdesc, const uint8_t *__restrict__ rlen,
             const int32_t *__restrict__ col, int32_t nV, int64_t nnz, R alpha,
             const R *__restrict__ M, R beta, const R *__restrict__ K, const R *__restrict__ x,
             R *__restrict__ y, int il) {
    constexpr int G = 8, GPB = TR / G;
    constexpr int V = Piece<R>::V, LPR = 8 / V;
    const int64_t bt = blockIdx.y;
    M += bt * nV;
    K += bt * nnz;
    x += bt * (int64_t)nV * 8;
    y += bt * (int64_t)nV * 8;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int gbase = (threadIdx.x & 63) - lane;
    const TileSeq ts = tile_seq(((int64_t)nV + GPB - 1) / GPB, il);
    const int64_t t0 = ts.t0, t1 = ts.t1, st_ = ts.step;
    // the lane group's row of a tile (len 0: none; a row holds at least its diagonal)
    auto desc = [&](int64_t tile, int2 &d, int32_t &len) {
        const int64_t r = tile * GPB + grp;
        d = make_int2(0, 0);
        len = 0;
        if (tile < t1 && r < nV) {
            d = rdesc[r];
            len = rlen[r];
        }
    };
    // the lane's entry of a row's first eight and the row's mass
    auto first = [&](const int2 &d, int32_t len, int32_t &cj, R &kv, R &mv) {
        cj = d.x;
        kv = R(0);
        mv = R(0);
        if (len > 0) {
            mv = M[d.x];
            if (lane < len) {
                cj = col[d.y + lane];
                kv = K[d.y + lane];
            }
        }
    };
    int2 dA, dB;
    int32_t lA, lB;
    desc(t0, dA, lA);
    desc(t0 + st_, dB, lB);
    int32_t cjA;
    R kA, mA;
    first(dA, lA, cjA, kA, mA);
    for (int64_t tile = t0; tile < t1; tile += st_) {
        if (lA == 0) break;  // past nV: uniform over the lane group, and so are later tiles
        int2 dC;
        int32_t lC, cjB;
        R kB, mB;
        desc(tile + 2 * st_, dC, lC);
        first(dB, lB, cjB, kB, mB);
        const int32_t i = dA.x;
        const R dt = alpha * mA;
        Piece<R> acc;
#pragma unroll
        for (int c = 0; c < V; ++c) acc.v[c] = R(0);
        {
            R aj = R(0);
            if (lane < lA) {
                aj = beta * kA;
                if (cjA == i) aj += dt;
            }
            wide8_chunk(cjA, aj, x, lane, gbase, acc);
        }
        for (int32_t e0 = 8; e0 < lA; e0 += 8) {  // rows of more than eight entries
            int32_t cj = i;
            R aj = R(0);
            if (e0 + lane < lA) {
                const int32_t e = dA.y + e0 + lane;
                cj = col[e];
                aj = beta * K[e];
                if (cj == i) aj += dt;
            }
            wide8_chunk(cj, aj, x, lane, gbase, acc);
        }
        wide8_combine(acc);
        if (lane < LPR) st_piece(y + (int64_t)i * 8 + (lane % LPR) * V, acc);
        dA = dB;
        lA = lB;
        cjA = cjB;
        kA = kB;
        mA = mB;
        dB = dC;
        lB = lC;
    }
}

// The same pipeline for one column: a lane per entry gathers x[j], and the
// group's G lanes are added by a shuffle tree (G = 8: the same operations in
// the same order as k_spmm's row for k = 1; G = 16 for rows of up to 16
// entries, tetrahedral meshes, whose entries then come in one chunk).
template <typename R, int G = 8>
__global__ void __launch_bounds__(TR)
k_spmm1_pipe(const int2 *__restrict__ rdesc, const uint8_t *__restrict__ rlen,
             const int32_t *__restrict__ col, int32_t nV, int64_t nnz, R alpha,
             const R *__restrict__ M, R beta, const R *__restrict__ K, const R *__restrict__ x,
             R *__restrict__ y) {
    constexpr int GPB = TR / G;
    const int64_t bt = blockIdx.y;
    M += bt * nV;
    K += bt * nnz;
    x += bt * (int64_t)nV;
    y += bt * (int64_t)nV;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    int64_t t0, t1;
    tile_range(((int64_t)nV + GPB - 1) / GPB, t0, t1);
    auto desc = [&](int64_t tile, int2 &d, int32_t &len) {
        const int64_t r = tile * GPB + grp;
        d = make_int2(0, 0);
        len = 0;
        if (tile < t1 && r < nV) {
            d = rdesc[r];
            len = rlen[r];
        }
    };
    auto first = [&](const int2 &d, int32_t len, int32_t &cj, R &kv, R &mv) {
        cj = d.x;
        kv = R(0);
        mv = R(0);
        if (len > 0) {
            mv = M[d.x];
            if (lane < len) {
                cj = col[d.y + lane];
                kv = K[d.y + lane];
            }
        }
    };
    int2 dA, dB;
    int32_t lA, lB;
    desc(t0, dA, lA);
    desc(t0 + 1, dB, lB);
    int32_t cjA;
    R kA, mA;
    first(dA, lA, cjA, kA, mA);
    for (int64_t tile = t0; tile < t1; ++tile) {
        if (lA == 0) break;  // past nV: uniform over the lane group, and so are later tiles
        int2 dC;
        int32_t lC, cjB;
        R kB, mB;
        desc(tile + 2, dC, lC);
        first(dB, lB, cjB, kB, mB);
        const int32_t i = dA.x;
        const R dt = alpha * mA;
        R acc = 0;
        {
            R aj = R(0);
            if (lane < lA) {
                aj = beta * kA;
                if (cjA == i) aj += dt;
            }
            acc += aj * x[cjA];
        }
        for (int32_t e0 = G; e0 < lA; e0 += G) {  // rows of more than G entries
            int32_t cj = i;
            R aj = R(0);
            if (e0 + lane < lA) {
                const int32_t e = dA.y + e0 + lane;
                cj = col[e];
                aj = beta * K[e];
                if (cj == i) aj += dt;
            }
            acc += aj * x[cj];
        }
#pragma unroll
        for (int off = G / 2; off >= 1; off /= 2) acc += __shfl_down(acc, off, G);
        if (lane == 0) y[i] = acc;
        dA = dB;
        lA = lB;
        cjA = cjB;
        kA = kB;
        mA = mB;
        dB = dC;
        lB = lC;
    }
}

// Gradients of a linear solve with respect to K and M (see
// dgo_linear_solve_vjp): one thread per row, sums over the columns c in
// ascending order.
template <typename R>
__global__ void k_solve_vjp(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            int32_t nV, R alpha, R beta, int k, const R *__restrict__ lam,
                            const R *__restrict__ u, const R *__restrict__ f,
                            R *__restrict__ gK, R *__restrict__ gM) {
    const int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= nV) return;
    const R *li = lam + i * k;
    for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
        const R *uj = u + (int64_t)col[t] * k;
        R s = 0;
        for (int c = 0; c < k; ++c) s += li[c] * uj[c];
        gK[t] = -beta * s;
    }
    const R *ui = u + i * k;
    R m = 0;
    for (int c = 0; c < k; ++c) m += li[c] * ui[c];
    R g = -alpha * m;
    if (f) {
        const R *fi = f + i * k;
        R q = 0;
        for (int c = 0; c < k; ++c) q += li[c] * fi[c];
        g += q;
    }
    gM[i] = g;
}

// ------------------------------------------------------------------- PCG

// The start of a solve, one pass over the rows: q = A_II x0 (q_B = 0) from M
// and K, then r = beff - q, p = s = 0, and partial sums of r.z, r.r and
// beff.beff (z = D^-1 r). x0 and beff are in natural order; r, p, s and dvec
// in the loop's order (with pos_order, the rows' positions, where xp
// receives x0 as well; else natural).
template <typename R, int KP, bool MASK>
__global__ void __launch_bounds__(TR, KP <= 8 ? 8 : 4)
k_cg_start(const int2 *__restrict__ rdesc, const uint8_t *__restrict__ rlen,
           const int32_t *__restrict__ col, int32_t nV, R alpha_m, const R *__restrict__ M,
           R beta_k, const R *__restrict__ K, const uint8_t *__restrict__ mask, int k,
           const R *__restrict__ x0, const R *__restrict__ beff, int pos_order, R *__restrict__ xp,
           const R *__restrict__ dvec, R *__restrict__ r, R *__restrict__ p, R *__restrict__ sv,
           double *__restrict__ part, int il) {
    constexpr int G = KP < 8 ? 8 : KP;
    constexpr int GPB = TR / G;
    __shared__ double s_part[3 * kMaxK];
    __shared__ double s_red[red_scratch(TR, 3)];
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int gbase = (threadIdx.x & 63) - lane;
    const bool out_lane = lane < k && lane < KP;
    double d[3] = {0.0, 0.0, 0.0};
    const TileSeq ts = tile_seq(((int64_t)nV + GPB - 1) / GPB, il);
    const int64_t t0 = ts.t0, t1 = ts.t1, st_ = ts.step;
    for (int64_t tile = t0; tile < t1; tile += st_) {
        const int64_t pos = tile * GPB + grp;
        if (pos >= nV) continue;  // uniform over the lane group
        const int2 dd = rdesc[pos];
        const int32_t i = dd.x;
        const int32_t len = rlen[pos];
        R q = 0;
        if (!(MASK && mask[i]))
            q = row_apply<R, G, KP, MASK>(col, K, beta_k, alpha_m * M[i], mask, x0, i, dd.y, len,
                                          k, lane, gbase, nullptr);
        if (out_lane) {
            const int64_t vi = pos_order ? pos : (int64_t)i;
            const int64_t e = vi * k + lane, en = (int64_t)i * k + lane;
            const R b = beff[en];
            const R rv = b - q;
            const R zv = dvec[vi] * rv;
            if (xp) xp[e] = x0[en];
            r[e] = rv;
            p[e] = R(0);
            sv[e] = R(0);
            d[0] += (double)rv * (double)zv;
            d[1] += (double)rv * (double)rv;
            d[2] += (double)b * (double)b;
        }
    }
    column_partials(d, 3, k, G, out_lane, s_red, s_part);
    store_partials(s_part, 3 * k, part);
}

// The vector update adds a column's steps to x in pairs (every second
// iteration); a column whose last update had an even index still lacks
// alpha p of that update: its iteration count is odd. Completes x in place
// (xout == xp) or while copying the row-order solution back to natural order:
// x[order[p]] = xp[p] (+ alpha_prev p[p]).
template <typename R>
__global__ void k_cg_finish_x(int64_t n, int k, const int32_t *__restrict__ order,
                              const CgCol *__restrict__ st, const R *__restrict__ pdir,
                              const R *xp, R *xout) {
    const int64_t e = (int64_t)blockIdx.x * T + threadIdx.x;
    if (e >= n) return;
    const int64_t q = e / k;
    const int c = (int)(e - q * k);
    R v = xp[e];
    if (st[c].iters & 1) v += (R)st[c].alpha_prev * pdir[e];
    xout[(order ? (int64_t)order[q] : q) * k + c] = v;
}

// Padded-row values: slot q = p * W + t holds v = A_ij d_j for the entry of
// CSR slot ell_src[q] (row i = order[p], column j), 0 for padding and on
// masked rows; dp[p] = d_i (D^-1 in row order).
template <typename R>
__global__ void k_cg_values_ell(const int32_t *__restrict__ order, const int32_t *__restrict__ src,
                                const int32_t *__restrict__ col, int32_t nV, int32_t W, R alpha,
                                const R *__restrict__ M, R beta, const R *__restrict__ K,
                                const uint8_t *__restrict__ mask, const R *__restrict__ invD,
                                R *__restrict__ v, R *__restrict__ dp) {
    const int64_t q = (int64_t)blockIdx.x * T + threadIdx.x;
    if (q >= (int64_t)nV * W) return;
    const int64_t p = q / W;
    const int32_t i = order ? order[p] : (int32_t)p;
    const int32_t t = src[q];
    R val = R(0);
    if (t >= 0 && !(mask && mask[i])) {
        const int32_t j = col[t];
        R a = beta * K[t];
        if (j == i) a += alpha * M[i];
        val = a * invD[j];
    }
    v[q] = val;
    if (q - p * W == 0) dp[p] = invD[i];
}

// The operator's values scaled by the preconditioner, v_ij = A_ij d_j with
// A = alpha M + beta K and d = D^-1 (d is zero on masked rows, so masked
// columns drop out), and v = 0 on masked rows. Prepared once per solve, so
// that w = A D^-1 r is one sweep over v with no per-entry scaling.
template <typename R>
__global__ void k_cg_values(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            int32_t nV, R alpha, const R *__restrict__ M, R beta,
                            const R *__restrict__ K, const uint8_t *__restrict__ mask,
                            const R *__restrict__ invD, R *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * T + threadIdx.x;
    if (i >= nV) return;
    const bool masked = mask && mask[i];
    const R dm = alpha * M[i];
    for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
        const int32_t j = col[t];
        R a = beta * K[t];
        if (j == i) a += dm;
        v[t] = masked ? R(0) : a * invD[j];
    }
}

// w = A_II z with z = D^-1 r, as w_i = sum_j v_ij r_j, fused with per-column
// partial sums of w.z. Rows in the mesh's row order (as k_spmm).
// ELL: the padded rows in row order (vectors in row order, i = position,
// dvec = D^-1 in row order); otherwise CSR rows through the row descriptors
// (vectors in natural order).
template <typename R, int KP, bool ELL, int G = (KP < 8 ? 8 : KP)>
__global__ void __launch_bounds__(TR, KP <= 8 ? 8 : 4)
k_cg_sdot(const int2 *__restrict__ rdesc, const uint8_t *__restrict__ rlen, int32_t W,
          const int32_t *__restrict__ col, int32_t nV, const R *__restrict__ v,
          const R *__restrict__ dvec, int k, const R *__restrict__ r, R *__restrict__ w,
          const CgCol *__restrict__ st, double *__restrict__ part, int wide, int il) {
    constexpr int GPB = TR / G;
    __shared__ double s_part[kMaxK];
    __shared__ double s_red[red_scratch(TR, 1)];
    __shared__ int s_any;
    if (st) {  // nothing to do once every column has stopped
        if (threadIdx.x == 0) {
            int any = 0;
            for (int c = 0; c < k; ++c) any |= st[c].active;
            s_any = any;
        }
        __syncthreads();
        if (!s_any) return;
    }
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int gbase = (threadIdx.x & 63) - lane;
    const bool out_lane = lane < k && lane < KP;
    constexpr int RU = ELL && KP <= 8 ? kSpmvRows : 1;
    double dsum = 0.0;
    const TileSeq ts = tile_seq(((int64_t)nV + GPB - 1) / GPB, il);
    const int64_t t0 = ts.t0, t1 = ts.t1, st_ = ts.step;
    if constexpr (ELL && (KP == 8 || KP == 16)) {
      if (wide) {
        // k = KP = 8 or 16 columns over padded rows of at most 8 entries, r
        // and w 16-byte aligned: 16-byte gathers
        constexpr int V = Piece<R>::V, LPR = KP / V;
        const int q = lane % LPR;
        double ds[V];
#pragma unroll
        for (int c = 0; c < V; ++c) ds[c] = 0.0;
        // the next tile's entries are loaded while this tile's gathers are in
        // flight (measured faster once each workgroup had five tiles or so)
        int32_t cjn = 0;
        R ajn = R(0);
        if (t0 < t1 && t0 * GPB + grp < nV) ell_entry(col, v, W, (int32_t)(t0 * GPB + grp), lane, cjn, ajn);
        for (int64_t tile = t0; tile < t1; tile += st_) {
            const int64_t row = tile * GPB + grp;
            if (row >= nV) break;  // uniform over the lane group; later tiles are past nV too
            const int32_t cj = cjn;
            const R aj = ajn;
            const int64_t rown = row + st_ * GPB;
            if (tile + st_ < t1 && rown < nV) ell_entry(col, v, W, (int32_t)rown, lane, cjn, ajn);
            const Piece<R> acc = ell_row_wide<R, KP>(cj, aj, r, lane, gbase, W);
            if (lane < LPR) {
                const int64_t e = row * KP + q * V;
                st_piece(w + e, acc);
                const Piece<R> ri = ld_piece(r + e);
                const R d = dvec[row];
#pragma unroll
                for (int c = 0; c < V; ++c) ds[c] += (double)acc.v[c] * (double)(d * ri.v[c]);
            }
        }
        // column c's sum sits in lane c / V, component c % V
        double dc = 0.0;
#pragma unroll
        for (int c = 0; c < V; ++c) {
            const double t = __shfl(ds[c], gbase + lane / V);
            if (lane % V == c) dc = t;
        }
        column_partials(&dc, 1, k, G, out_lane, s_red, s_part);
        store_partials(s_part, k, part);
        return;
      }
    }
    for (int64_t tile = t0; tile < t1; tile += RU * st_) {
        int32_t i[RU], rb[RU], len[RU];
        bool ok[RU];
        R dt[RU], acc[RU], ri[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {  // uniform over the lane group
            const int64_t pos = (tile + u * st_) * GPB + grp;
            ok[u] = tile + u * st_ < t1 && pos < nV;
            if (ELL) {
                i[u] = ok[u] ? (int32_t)pos : 0;
                rb[u] = i[u] * W;
                len[u] = W;
            } else {
                const int2 d = ok[u] ? rdesc[pos] : make_int2(0, 0);
                i[u] = d.x;
                rb[u] = d.y;
                len[u] = ok[u] ? (int32_t)rlen[pos] : 0;
            }
            dt[u] = R(0);
        }
        if (!ok[0]) continue;
        rows_apply<R, G, KP, RU, true>(col, v, R(1), dt, r, i, rb, len, ok, k, lane, gbase, acc, ri);
        if (out_lane) {
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                if (!ok[u]) continue;
                const int64_t e = (int64_t)i[u] * k + lane;
                w[e] = acc[u];
                if (G != KP) ri[u] = r[e];  // rows_apply returns r[i, c] only when G == KP
                dsum += (double)acc[u] * (double)(dvec[i[u]] * ri[u]);
            }
        }
    }
    column_partials(&dsum, 1, k, G, out_lane, s_red, s_part);
    store_partials(s_part, k, part);
}

// The vector work of iteration i on the active columns: p = z + beta p,
// s = w + beta s, r -= alpha s (z = D^-1 r) and, in odd iterations, the two
// steps x += alpha' p' + alpha p, fused with partial sums of r.z and r.r of
// the new residual (stored to pout). The iteration's state S_i (alpha, beta,
// stopping) is either read from st_cur (iteration 0, whose state the start
// finalize computed) or, with reduce, computed here from S_{i-1} (st_prev)
// and the partial sums of the previous update (pin) and of w.z (pin2): every
// workgroup adds the same partials in the same fixed order, so all agree
// bitwise, and workgroup 0 stores S_i to st_cur. pin, pout and st_prev,
// st_cur are distinct buffers (alternating with the iteration's parity), so
// no workgroup reads what another writes.
// tiles of the vector update whose loads are issued before its reduction
constexpr int kVuPre = 5;

template <typename R>
__global__ void __launch_bounds__(TR)
k_cg_vupdate(int32_t nV, int k, int KP, R *__restrict__ x, R *__restrict__ r, R *__restrict__ p,
             R *__restrict__ sv, const R *__restrict__ w, const R *__restrict__ invD,
             const CgCol *__restrict__ st_prev, CgCol *__restrict__ st_cur, int reduce, int odd,
             const double *__restrict__ pin, int nbu, const double *__restrict__ pin2, int nbs,
             double *__restrict__ pout, CgParams prm) {
    __shared__ double s_part[2 * kMaxK];
    __shared__ double s_red[red_scratch(TR, 2)];
    __shared__ double s_tot[3 * kMaxK];
    __shared__ double s_ab[3 * kMaxK];
    __shared__ int s_on[kMaxK];
    __shared__ int s_any;
    const int t = threadIdx.x;
    const CgCol *sin = reduce ? st_prev : st_cur;
    // The vectors of the block's first tiles do not depend on alpha and beta:
    // their loads are all issued before the reduction below, which they
    // overlap (one workgroup per CU, so the registers are there).
    const VLane L = vlane(k, KP);
    int64_t t0, t1;
    tile_range(((int64_t)nV + L.gpb - 1) / L.gpb, t0, t1);
    R fr[kVuPre], fw[kVuPre], fp[kVuPre], fs[kVuPre], fx[kVuPre], fd[kVuPre];
#pragma unroll
    for (int u = 0; u < kVuPre; ++u) {
        const int64_t i = (t0 + u) * L.gpb + L.grp;
        fr[u] = fw[u] = fp[u] = fs[u] = fx[u] = fd[u] = R(0);
        if (L.act && t0 + u < t1 && i < nV) {
            const int64_t e = i * k + L.c;
            fr[u] = r[e];
            fw[u] = w[e];
            fp[u] = p[e];
            fs[u] = sv[e];
            if (odd) fx[u] = x[e];
            fd[u] = invD[i];
        }
    }
    if (t == 0) {
        int any = 0;
        for (int c = 0; c < k; ++c) any |= sin[c].active;
        s_any = any;
    }
    __syncthreads();
    if (!s_any) {  // every column has stopped: the state carries over
        if (reduce && blockIdx.x == 0 && t < k) st_cur[t] = st_prev[t];
        return;
    }
    if (reduce) fin_sum2(pin, nbu, 2 * k, pin2, nbs, k, s_tot);
    if (t < k) {
        CgCol c = reduce ? st_prev[t] : st_cur[t];
        if (reduce) {
            cg_sr_update(FIN_SR_ITER, c, s_tot, s_tot + 2 * k, t, k, prm);
            if (blockIdx.x == 0) st_cur[t] = c;
        }
        s_on[t] = c.active;
        s_ab[t] = c.alpha;
        s_ab[k + t] = c.beta;
        s_ab[2 * k + t] = c.alpha_prev;
    }
    __syncthreads();
    const bool on = L.act && s_on[L.c];
    const R a = on ? (R)s_ab[L.c] : R(0), bt = on ? (R)s_ab[k + L.c] : R(0);
    const R ap = on ? (R)s_ab[2 * k + L.c] : R(0);
    double d[2] = {0.0, 0.0};
    if (on) {
        auto update = [&](int64_t i, R rv, R wv, R pv, R s0, R xv, R dv) {
            const int64_t e = i * k + L.c;
            const R pn = dv * rv + bt * pv;
            const R sn = wv + bt * s0;
            const R rn = rv - a * sn;
            p[e] = pn;
            sv[e] = sn;
            // x takes two steps every second iteration: x += a' p' + a p
            // (p' the previous direction, still in p before this update)
            if (odd) x[e] = xv + ap * pv + a * pn;
            r[e] = rn;
            const R zn = dv * rn;
            d[0] += (double)rn * (double)zn;
            d[1] += (double)rn * (double)rn;
        };
#pragma unroll
        for (int u = 0; u < kVuPre; ++u) {
            const int64_t i = (t0 + u) * L.gpb + L.grp;
            if (t0 + u < t1 && i < nV) update(i, fr[u], fw[u], fp[u], fs[u], fx[u], fd[u]);
        }
        // the remaining tiles, software pipelined: the next tile's loads are
        // issued before the current tile is computed and stored
        const int64_t tb = t0 + kVuPre;
        R rv = 0, wv = 0, pv = 0, s0 = 0, xv = 0, dv = 0;
        if (tb < t1) {
            const int64_t i = tb * L.gpb + L.grp;
            if (i < nV) {
                const int64_t e = i * k + L.c;
                rv = r[e];
                wv = w[e];
                pv = p[e];
                s0 = sv[e];
                if (odd) xv = x[e];
                dv = invD[i];
            }
        }
        for (int64_t tile = tb; tile < t1; ++tile) {
            const int64_t i = tile * L.gpb + L.grp, in = i + L.gpb;
            R nr = 0, nw = 0, np = 0, ns = 0, nx = 0, nd = 0;
            if (tile + 1 < t1 && in < nV) {
                const int64_t en = in * k + L.c;
                nr = r[en];
                nw = w[en];
                np = p[en];
                ns = sv[en];
                if (odd) nx = x[en];
                nd = invD[in];
            }
            if (i < nV) update(i, rv, wv, pv, s0, xv, dv);
            rv = nr;
            wv = nw;
            pv = np;
            s0 = ns;
            xv = nx;
            dv = nd;
        }
    }
    column_partials(d, 2, k, KP, on, s_red, s_part);
    store_partials(s_part, 2 * k, pout);
}

// One workgroup: add the partial sums of the preceding kernels in a fixed
// order and advance the per-column state from st_in to st_out (FIN_SR_INIT:
// a fresh state), or store the totals to out (FIN_OUT).
template <int MODE>
__global__ void __launch_bounds__(kFinThreads)
k_cg_fin(const double *__restrict__ part, int nblk, const double *__restrict__ part2, int nblk2,
         int k, const CgCol *st_in, CgCol *st_out, CgParams prm, double *out) {
    __shared__ double s_tot[4 * kMaxK];
    constexpr bool SR = MODE == FIN_SR_INIT || MODE == FIN_SR_ITER;
    const int W = fin_width(MODE, k);
    fin_sum2(part, nblk, W, part2, nblk2, SR ? k : 0, s_tot);
    const int c = threadIdx.x;
    if (c >= k) return;
    if (!SR) {
        out[c] = s_tot[c];
        return;
    }
    CgCol st = MODE == FIN_SR_INIT ? CgCol{} : st_in[c];
    cg_sr_update(MODE, st, s_tot, s_tot + W, c, k, prm);
    st_out[c] = st;
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

// Partial sums of ||beff - A_II u||^2 per column, accumulated in FP64.
template <typename R>
__global__ void __launch_bounds__(TR)
k_cg_trueres(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, int32_t nV,
             double alpha, const R *__restrict__ M, double beta, const R *__restrict__ K,
             const uint8_t *__restrict__ mask, int k, int KP, const R *__restrict__ beff,
             const R *__restrict__ u, double *__restrict__ part) {
    __shared__ double s_part[kMaxK];
    __shared__ double s_red[red_scratch(TR, 1)];
    const VLane L = vlane(k, KP);
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
    column_partials(&d, 1, k, KP, L.act, s_red, s_part);
    store_partials(s_part, k, part);
}

// The same true residual for FP64 solves, with the lane groups of the SpMV
// kernels: rows in the mesh's row order, G lanes per row, the row's sum
// (alpha M + beta K) u formed as row_apply does, then (beff - A u)^2 added
// per column (the sum of a row is formed in a different order than above).
template <typename R, int KP, bool MASK>
__global__ void __launch_bounds__(TR, KP <= 8 ? 8 : 4)
k_cg_trueres_rows(const int2 *__restrict__ rdesc, const uint8_t *__restrict__ rlen,
                  const int32_t *__restrict__ col, int32_t nV, R alpha_m, const R *__restrict__ M,
                  R beta_k, const R *__restrict__ K, const uint8_t *__restrict__ mask, int k,
                  const R *__restrict__ beff, const R *__restrict__ u, double *__restrict__ part,
                  int il) {
    constexpr int G = KP < 8 ? 8 : KP;
    constexpr int GPB = TR / G;
    __shared__ double s_part[kMaxK];
    __shared__ double s_red[red_scratch(TR, 1)];
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;
    const int gbase = (threadIdx.x & 63) - lane;
    const bool out_lane = lane < k && lane < KP;
    double d = 0.0;
    const TileSeq ts = tile_seq(((int64_t)nV + GPB - 1) / GPB, il);
    const int64_t t0 = ts.t0, t1 = ts.t1, st_ = ts.step;
    for (int64_t tile = t0; tile < t1; tile += st_) {
        const int64_t pos = tile * GPB + grp;
        if (pos >= nV) continue;  // uniform over the lane group
        const int2 dd = rdesc[pos];
        const int32_t i = dd.x;
        if (MASK && mask[i]) continue;
        const R q = row_apply<R, G, KP, MASK>(col, K, beta_k, alpha_m * M[i], mask, u, i, dd.y,
                                              (int32_t)rlen[pos], k, lane, gbase, nullptr);
        if (out_lane) {
            const double sres = (double)beff[(int64_t)i * k + lane] - (double)q;
            d += sres * sres;
        }
    }
    column_partials(&d, 1, k, G, out_lane, s_red, s_part);
    store_partials(s_part, k, part);
}

unsigned nblocks_for(int64_t ntiles, int64_t cap = kMaxBlocks) {
    int64_t b = ntiles < cap ? ntiles : cap;
    return (unsigned)(b < 1 ? 1 : b);
}

int64_t ntiles(int64_t nV, int rows_per_tile) { return (nV + rows_per_tile - 1) / rows_per_tile; }

// Tile order of the PCG kernels that gather (tile_seq): interleaved over each
// XCD's workgroups once the gathered vector of one XCD's share of the rows is
// larger than half its 4 MB L2, else a contiguous chunk per workgroup. These
// grids hold one or two workgroups per CU with many tiles each (w = A z at
// the icosphere L9, 8 FP64 columns: 186 -> 172 us per iteration). The other
// SpMM grids are not persistent (workgroups of about five tiles, dispatched
// in order), so their resident workgroups already work on neighbouring
// chunks; interleaving them was slower (L9, 8 columns: 201 -> 210 us); the
// 8-column pipeline instead turns persistent with interleaved tiles past the
// L2 (kSpmmPersistBlocks).
constexpr int64_t kXcdL2Bytes = 4 << 20;

int gather_il(const dgo_mesh *m, int k, size_t es) {
    return (int64_t)m->nV * k * (int64_t)es / 8 > kXcdL2Bytes / 2 ? 1 : 0;
}

// Workgroups of the 8-column SpMM when its tiles are interleaved: one per CU
// (icosphere L9: 201 -> 193 us warm, 241 -> 235 us cold against the grid of
// about five tiles per workgroup; 512 workgroups: 231 / 287 us, 1024: 236 / 299)
constexpr int kSpmmPersistBlocks = 256;

// ------------------------------------------------------------- dispatch

template <typename R, int KP>
void launch_spmm_kp(const dgo_mesh *m, int32_t batch, R alpha, const R *M, R beta, const R *K,
                    int k, const R *x, R *y, hipStream_t s) {
    constexpr int G = KP < 8 ? 8 : KP;
    const int wide = KP == 8 && k == 8 && ((uintptr_t)x % 16) == 0 && ((uintptr_t)y % 16) == 0;
    // the pipelines prefetch a row's first eight entries: used when every row
    // fits them (triangle meshes); longer rows (tetrahedra) were measured
    // faster in k_spmm (Kuhn cube 64^3, one column: 19.2 vs 26.6 us)
    const bool short_rows = m->max_row <= 8;
    if (wide && short_rows) {
        // about five tiles per workgroup, and no fewer than one workgroup per
        // CU (L7: 256 workgroups, 10.2 vs 14.1 us for the k_spmm grid; L9:
        // 4096, 201 vs 206 us; 256 at L9, 80 tiles each: 267 us)
        const int64_t nt8 = ntiles(m->nV, TR / 8);
        const int il8 = gather_il(m, k, sizeof(R));
        dim3 grid8(nblocks_for(nt8, il8 ? (int64_t)kSpmmPersistBlocks : std::max<int64_t>(256, nt8 / 5)),
                   (unsigned)batch);
        auto kfn8 = k_spmm8_pipe<R>;
        DGO_LAUNCH_EXT("spmm", s, kfn8, grid8, dim3(TR), 0u, m->rdesc, m->rlen, m->col, m->nV, m->nnz,
                       alpha, M, beta, K, x, y, il8);
        return;
    }
    if (KP == 1 && short_rows) {  // one column: the same pipeline, a lane per entry
        const int64_t nt1 = ntiles(m->nV, TR / 8);
        dim3 grid1(nblocks_for(nt1, std::max<int64_t>(256, nt1 / 5)), (unsigned)batch);
        auto kfn1 = k_spmm1_pipe<R>;
        DGO_LAUNCH_EXT("spmm", s, kfn1, grid1, dim3(TR), 0u, m->rdesc, m->rlen, m->col, m->nV, m->nnz,
                       alpha, M, beta, K, x, y);
        return;
    }
    if (KP == 1 && m->max_row <= 16) {  // one column, rows of 9 to 16 entries: 16 lanes per row
        const int64_t nt1 = ntiles(m->nV, TR / 16);
        dim3 grid1(nblocks_for(nt1, std::max<int64_t>(256, nt1 / 5)), (unsigned)batch);
        auto kfn1 = k_spmm1_pipe<R, 16>;
        DGO_LAUNCH_EXT("spmm", s, kfn1, grid1, dim3(TR), 0u, m->rdesc, m->rlen, m->col, m->nV, m->nnz,
                       alpha, M, beta, K, x, y);
        return;
    }
    if (KP < 8 && m->max_row > 8 && m->max_row <= 16) {
        // rows of 9 to 16 entries (tetrahedral meshes) and few columns: 16
        // lanes per row, so that a row's entries and gathers are issued in
        // one chunk instead of two
        dim3 grid16(nblocks_for(ntiles(m->nV, T / 16)), (unsigned)batch);
        auto kfn16 = k_spmm<R, KP, 16>;
        DGO_LAUNCH_EXT("spmm", s, kfn16, grid16, dim3(T), 0u, m->rdesc, m->rlen, m->col, m->nV,
                       m->nnz, alpha, M, beta, K, k, x, y, 0);
        return;
    }
    dim3 grid(nblocks_for(ntiles(m->nV, T / G)), (unsigned)batch);
    auto kfn = k_spmm<R, KP>;
    DGO_LAUNCH_EXT("spmm", s, kfn, grid, dim3(T), 0u, m->rdesc, m->rlen, m->col, m->nV, m->nnz,
                   alpha, M, beta, K, k, x, y, wide);
}

template <typename R>
void launch_spmm(const dgo_mesh *m, int32_t batch, R alpha, const R *M, R beta, const R *K, int k,
                 const R *x, R *y, hipStream_t s) {
    switch (pow2ceil(k)) {
        case 1: launch_spmm_kp<R, 1>(m, batch, alpha, M, beta, K, k, x, y, s); break;
        case 2: launch_spmm_kp<R, 2>(m, batch, alpha, M, beta, K, k, x, y, s); break;
        case 4: launch_spmm_kp<R, 4>(m, batch, alpha, M, beta, K, k, x, y, s); break;
        case 8: launch_spmm_kp<R, 8>(m, batch, alpha, M, beta, K, k, x, y, s); break;
        case 16: launch_spmm_kp<R, 16>(m, batch, alpha, M, beta, K, k, x, y, s); break;
        case 32: launch_spmm_kp<R, 32>(m, batch, alpha, M, beta, K, k, x, y, s); break;
        default: launch_spmm_kp<R, 64>(m, batch, alpha, M, beta, K, k, x, y, s); break;
    }
}

// Returns the number of workgroups launched (the count of partial rows).
template <typename R, int KP, bool MASK>
int launch_cg_start_kp(const dgo_mesh *m, R alpha, const R *M, R beta, const R *K,
                       const uint8_t *mask, int k, const R *x0, const R *beff, int pos_order,
                       R *xp, const R *dvec, R *r, R *p, R *sv, double *part, hipStream_t s) {
    constexpr int G = KP < 8 ? 8 : KP;
    const unsigned nb = nblocks_for(ntiles(m->nV, TR / G), kMaxRedBlocks);
    DGO_LAUNCH("cg_start", s,
               k_cg_start<R, KP, MASK><<<nb, TR, 0, s>>>(m->rdesc, m->rlen, m->col, m->nV, alpha, M,
                                                        beta, K, mask, k, x0, beff, pos_order, xp,
                                                        dvec, r, p, sv, part,
                                                        gather_il(m, k, sizeof(R))));
    return (int)nb;
}

template <typename R, bool MASK>
int launch_cg_start_m(const dgo_mesh *m, R alpha, const R *M, R beta, const R *K,
                      const uint8_t *mask, int k, const R *x0, const R *beff, int pos_order, R *xp,
                      const R *dvec, R *r, R *p, R *sv, double *part, hipStream_t s) {
#define DGO_START_CASE(KPV)                                                                        \
    return launch_cg_start_kp<R, KPV, MASK>(m, alpha, M, beta, K, mask, k, x0, beff, pos_order, xp, \
                                            dvec, r, p, sv, part, s)
    switch (pow2ceil(k)) {
        case 1: DGO_START_CASE(1);
        case 2: DGO_START_CASE(2);
        case 4: DGO_START_CASE(4);
        case 8: DGO_START_CASE(8);
        case 16: DGO_START_CASE(16);
        case 32: DGO_START_CASE(32);
        default: DGO_START_CASE(64);
    }
#undef DGO_START_CASE
}

template <typename R>
int launch_cg_start(const dgo_mesh *m, R alpha, const R *M, R beta, const R *K,
                    const uint8_t *mask, int k, const R *x0, const R *beff, int pos_order, R *xp,
                    const R *dvec, R *r, R *p, R *sv, double *part, hipStream_t s) {
    if (mask)
        return launch_cg_start_m<R, true>(m, alpha, M, beta, K, mask, k, x0, beff, pos_order, xp,
                                          dvec, r, p, sv, part, s);
    return launch_cg_start_m<R, false>(m, alpha, M, beta, K, mask, k, x0, beff, pos_order, xp, dvec,
                                       r, p, sv, part, s);
}

// Returns the number of workgroups launched (the count of partial rows).
template <typename R, int KP, bool MASK>
int launch_trueres_rows_kp(const dgo_mesh *m, R alpha, const R *M, R beta, const R *K,
                           const uint8_t *mask, int k, const R *beff, const R *u, double *part,
                           hipStream_t s) {
    constexpr int G = KP < 8 ? 8 : KP;
    const unsigned nb = nblocks_for(ntiles(m->nV, TR / G), kMaxRedBlocks);
    DGO_LAUNCH("cg_trueres", s,
               k_cg_trueres_rows<R, KP, MASK><<<nb, TR, 0, s>>>(m->rdesc, m->rlen, m->col, m->nV,
                                                               alpha, M, beta, K, mask, k, beff, u,
                                                               part, gather_il(m, k, sizeof(R))));
    return (int)nb;
}

template <typename R, bool MASK>
int launch_trueres_rows_m(const dgo_mesh *m, R alpha, const R *M, R beta, const R *K,
                          const uint8_t *mask, int k, const R *beff, const R *u, double *part,
                          hipStream_t s) {
    switch (pow2ceil(k)) {
        case 1: return launch_trueres_rows_kp<R, 1, MASK>(m, alpha, M, beta, K, mask, k, beff, u, part, s);
        case 2: return launch_trueres_rows_kp<R, 2, MASK>(m, alpha, M, beta, K, mask, k, beff, u, part, s);
        case 4: return launch_trueres_rows_kp<R, 4, MASK>(m, alpha, M, beta, K, mask, k, beff, u, part, s);
        case 8: return launch_trueres_rows_kp<R, 8, MASK>(m, alpha, M, beta, K, mask, k, beff, u, part, s);
        case 16: return launch_trueres_rows_kp<R, 16, MASK>(m, alpha, M, beta, K, mask, k, beff, u, part, s);
        case 32: return launch_trueres_rows_kp<R, 32, MASK>(m, alpha, M, beta, K, mask, k, beff, u, part, s);
        default: return launch_trueres_rows_kp<R, 64, MASK>(m, alpha, M, beta, K, mask, k, beff, u, part, s);
    }
}

template <int MODE>
void launch_fin(const double *part, int nblk, const double *part2, int nblk2, int k,
                const CgCol *st_in, CgCol *st_out, CgParams prm, double *out, hipStream_t s) {
    DGO_LAUNCH("cg_fin", s,
               k_cg_fin<MODE><<<1, kFinThreads, 0, s>>>(part, nblk, part2, nblk2, k, st_in, st_out,
                                                        prm, out));
}

// w = A z with 8 or more columns runs on at most one 1024-thread workgroup
// per CU: with balanced tile shares this was measured faster than two (2.49
// vs 2.55 ms per L7 step; 128 or 384 workgroups: 2.89 / 2.67 ms), and the next
// update then adds half as many partial sums. Fewer columns make cheap rows,
// which want the two (the Dirichlet solve on the Kuhn cube 64^3, one column:
// 4.98 vs 5.57 ms).
constexpr int kSdotBlocks = 256;

template <typename R, int KP>
int launch_sdot_kp(const dgo_mesh *m, const R *v, const R *dvec, int k, const R *r, R *w,
                   const CgCol *st, double *part, hipStream_t s) {
    constexpr int G = KP < 8 ? 8 : KP;
    const unsigned nb = nblocks_for(ntiles(m->nV, TR / G), KP >= 8 ? kSdotBlocks : kMaxRedBlocks);
    const int il = gather_il(m, k, sizeof(R));
    if (m->ell_w) {
        const int wide = (KP == 8 || KP == 16) && k == KP && m->ell_w <= 8 && ((uintptr_t)r % 16) == 0 &&
                         ((uintptr_t)w % 16) == 0;
        if (KP < 8 && m->ell_w == 16) {
            // padded rows of 16 entries (tetrahedral meshes) and few columns:
            // 16 lanes per row, the row's entries and gathers in one chunk
            const unsigned nb16 = nblocks_for(ntiles(m->nV, TR / 16), kMaxRedBlocks);
            auto kfn16 = k_cg_sdot<R, KP, true, 16>;
            DGO_LAUNCH_EXT("cg_sdot", s, kfn16, dim3(nb16), dim3(TR), 0u, (const int2 *)nullptr,
                           (const uint8_t *)nullptr, m->ell_w, (const int32_t *)m->ell_col, m->nV, v,
                           dvec, k, r, w, st, part, 0, il);
            return (int)nb16;
        }
        auto kfn = k_cg_sdot<R, KP, true>;
        DGO_LAUNCH_EXT("cg_sdot", s, kfn, dim3(nb), dim3(TR), 0u, (const int2 *)nullptr,
                       (const uint8_t *)nullptr, m->ell_w, (const int32_t *)m->ell_col, m->nV, v, dvec,
                       k, r, w, st, part, wide, il);
    } else {
        auto kfn = k_cg_sdot<R, KP, false>;
        DGO_LAUNCH_EXT("cg_sdot", s, kfn, dim3(nb), dim3(TR), 0u, (const int2 *)m->rdesc,
                       (const uint8_t *)m->rlen, 0, (const int32_t *)m->col, m->nV, v, dvec, k, r, w,
                       st, part, 0, il);
    }
    return (int)nb;
}

template <typename R>
int launch_sdot(const dgo_mesh *m, const R *v, const R *dvec, int k, const R *r, R *w,
                const CgCol *st, double *part, hipStream_t s) {
    switch (pow2ceil(k)) {
        case 1: return launch_sdot_kp<R, 1>(m, v, dvec, k, r, w, st, part, s);
        case 2: return launch_sdot_kp<R, 2>(m, v, dvec, k, r, w, st, part, s);
        case 4: return launch_sdot_kp<R, 4>(m, v, dvec, k, r, w, st, part, s);
        case 8: return launch_sdot_kp<R, 8>(m, v, dvec, k, r, w, st, part, s);
        case 16: return launch_sdot_kp<R, 16>(m, v, dvec, k, r, w, st, part, s);
        case 32: return launch_sdot_kp<R, 32>(m, v, dvec, k, r, w, st, part, s);
        default: return launch_sdot_kp<R, 64>(m, v, dvec, k, r, w, st, part, s);
    }
}

}  // namespace

PcgLayout pcg_layout(int64_t nV, int64_t nvals, int k, size_t elem) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t vec = al(elem * (size_t)nV * (size_t)k);
    PcgLayout L;
    L.off_r = 0;
    L.off_p = vec;
    L.off_s = 2 * vec;
    L.off_w = 3 * vec;
    L.off_b = 4 * vec;
    L.off_x = 5 * vec;
    L.off_d = 6 * vec;
    L.off_dp = L.off_d + al(elem * (size_t)nV);
    L.off_v = L.off_dp + al(elem * (size_t)nV);
    L.off_pt = L.off_v + al(elem * (size_t)nvals);
    L.off_pt2 = L.off_pt + 2 * al(sizeof(double) * kern::kMaxRedBlocks * 3 * kern::kMaxK);
    L.off_st = L.off_pt2 + al(sizeof(double) * kern::kMaxRedBlocks * kern::kMaxK);
    L.off_tr = L.off_st + 2 * al(sizeof(kern::CgCol) * kern::kMaxK);
    L.total = L.off_tr + al(sizeof(double) * kern::kMaxK);
    return L;
}

namespace {

template <typename R>
dgo_status run_pcg(const dgo_mesh *m, double alpha, const R *M, double beta, const R *K,
                   const uint8_t *mask, const R *g, int k, const R *b, R *u, const dgo_cg_opts &o,
                   dgo_cg_report *rep, hipStream_t s, char *ws_given = nullptr) {
    const int64_t nV = m->nV, n = nV * k;
    const int KP = pow2ceil(k);
    // With a padded-row layout the iteration runs in the mesh's row order
    // (vectors permuted once in and once out); otherwise in natural order.
    const bool ell = m->ell_w > 0;
    const int64_t nvals = ell ? nV * m->ell_w : m->nnz;
    const PcgLayout L = pcg_layout(nV, nvals, k, sizeof(R));
    void *wsv = ws_given;
    if (!ws_given) DGO_TRY(mesh_workspace(const_cast<dgo_mesh *>(m), L.total, s, &wsv));
    char *ws = (char *)wsv;
    R *r = (R *)(ws + L.off_r), *p = (R *)(ws + L.off_p), *sv = (R *)(ws + L.off_s);
    R *w = (R *)(ws + L.off_w);
    R *beff = mask ? (R *)(ws + L.off_b) : const_cast<R *>(b);
    R *x = ell ? (R *)(ws + L.off_x) : u;             // iterate in the loop's order
    R *invD = (R *)(ws + L.off_d);                     // natural order
    R *dvec = ell ? (R *)(ws + L.off_dp) : invD;       // the loop's order
    R *v = (R *)(ws + L.off_v);
    // partU[i & 1]: partials of the update that precedes iteration i;
    // stt[i & 1]: the state S_i of iteration i
    const size_t pu_stride = ((sizeof(double) * kMaxRedBlocks * 3 * kMaxK + 255) & ~(size_t)255);
    const size_t st_stride = ((sizeof(CgCol) * kMaxK + 255) & ~(size_t)255);
    double *partU[2] = {(double *)(ws + L.off_pt), (double *)(ws + L.off_pt + pu_stride)};
    double *part2 = (double *)(ws + L.off_pt2);
    CgCol *stt[2] = {(CgCol *)(ws + L.off_st), (CgCol *)(ws + L.off_st + st_stride)};
    double *part = partU[0];
    double *tr = (double *)(ws + L.off_tr);

    CgParams prm;
    prm.rtol = o.rtol;
    prm.rtol0 = o.rtol_initial;
    prm.atol = o.atol;
    prm.max_iter = o.max_iter;
    prm.fixed = o.fixed_iters;
    prm.stall = o.stall_iters;
    prm.k = k;

    // the vector update runs on at most 256 workgroups (each of them adds
    // every partial sum of the previous iteration first); the true-residual
    // SpMV after the loop uses the full grid
    const unsigned nb_v = nblocks_for(ntiles(nV, TR / KP), 256);
    const unsigned nb_t = nblocks_for(ntiles(nV, TR / KP), kMaxRedBlocks);
    const R ra = (R)alpha, rb = (R)beta;

    DGO_LAUNCH("cg_invdiag", s,
               k_cg_invdiag<R><<<grid_for(nV, T), T, 0, s>>>((int32_t)nV, ra, M, rb, K, m->diag, mask,
                                                             invD));
    if (ell)
        DGO_LAUNCH("cg_values", s,
                   k_cg_values_ell<R><<<grid_for(nvals, T), T, 0, s>>>(
                       m->order, m->ell_src, m->col, (int32_t)nV, m->ell_w, ra, M, rb, K, mask, invD,
                       v, dvec));
    else
        DGO_LAUNCH("cg_values", s,
                   k_cg_values<R><<<grid_for(nV, T), T, 0, s>>>(m->rowptr, m->col, (int32_t)nV, ra,
                                                                M, rb, K, mask, invD, v));
    if (mask)
        DGO_LAUNCH("cg_lift", s,
                   k_cg_lift<R><<<grid_for(n, T), T, 0, s>>>(m->rowptr, m->col, (int32_t)nV, ra, M, rb,
                                                             K, mask, k, b, g, beff, u));
    // r0 = beff - A_II x0, p = s = 0, w0 = A D^-1 r0; alpha_0 = (r.z) / (w.z)
    const int nb_0 = launch_cg_start<R>(m, ra, M, rb, K, mask, k, u, beff, ell ? 1 : 0,
                                        ell ? x : nullptr, dvec, r, p, sv, part, s);
    int nb_s = launch_sdot<R>(m, v, dvec, k, r, w, nullptr, part2, s);
    launch_fin<FIN_SR_INIT>(part, nb_0, part2, nb_s, k, nullptr, stt[0], prm, nullptr, s);
    DGO_HIP(hipGetLastError());

    const int every = o.fixed_iters ? (o.max_iter > 0 ? o.max_iter : 1)
                                    : (o.check_every > 0 ? o.check_every : 8);
    // Iterations i0 .. i0 + count - 1. Each iteration is two kernels: the
    // vector update (which also finishes the previous iteration's reductions
    // and writes the state of iteration i to stt[i & 1]) and w = A z with w.z.
    // After iteration e - 1 the newest complete state is stt[(e - 1) & 1]: it
    // carries the stopping tests of every iteration but the last, which the
    // host's progress check may therefore see one iteration late; a single
    // finalize after the last iteration completes the state.
    int nbs = nb_s;
    auto iterate = [&](hipStream_t st_s, int32_t i0, int32_t count) {
        for (int32_t it = 0; it < count; ++it) {
            const int32_t i = i0 + it;
            DGO_LAUNCH_EXT("cg_vupdate", st_s, k_cg_vupdate<R>, dim3(nb_v), dim3(TR), 0u,
                           (int32_t)nV, k, KP, x, r, p, sv, w, dvec, stt[(i + 1) & 1], stt[i & 1],
                           i > 0 ? 1 : 0, i & 1, partU[i & 1], (int)nb_v, part2, nbs,
                           partU[(i + 1) & 1], prm);
            nbs = launch_sdot<R>(m, v, dvec, k, r, w, stt[i & 1], part2, st_s);
        }
    };
    auto unorder = [&](int32_t done) {
        if (ell)
            DGO_LAUNCH("cg_unorder", s,
                       k_cg_finish_x<R><<<grid_for(n, T), T, 0, s>>>(n, k, m->order, stt[done & 1],
                                                                     p, x, u));
        else
            DGO_LAUNCH("cg_unorder", s,
                       k_cg_finish_x<R><<<grid_for(n, T), T, 0, s>>>(n, k, nullptr, stt[done & 1],
                                                                     p, x, x));
    };
    if (ws_given) {
        // the allocation-free form (a fixed iteration count): every
        // iteration is queued at once, with no progress polling, no true
        // residual and nothing read back to the host
        const int32_t iters = std::max<int32_t>(o.max_iter, 0);
        iterate(s, 0, iters);
        if (iters > 0)
            launch_fin<FIN_SR_ITER>(partU[iters & 1], (int)nb_v, part2, nbs, k, stt[(iters + 1) & 1],
                                    stt[iters & 1], prm, nullptr, s);
        unorder(iters);
        DGO_HIP(hipGetLastError());
        return DGO_OK;
    }
    // Progress polling without idling the device: up to two chunks are in
    // flight, so the next one is queued before the host waits for the state
    // copied after the previous one. Once every column has stopped, queued
    // launches find no active column and do next to nothing; to queue few of
    // them, the host plans how far to queue from each active column's
    // residual rate (two successive polled states give its geometric rate per
    // iteration, hence the iterations it still needs). The plan only sets how
    // many launches are queued: every column stops on the device's own test,
    // and a column that runs past the plan gets further chunks.
    dgo_mesh *mm = const_cast<dgo_mesh *>(m);
    if (!mm->poll_host) {
        // two polling slots, then the final state and true residuals
        DGO_HIP(hipHostMalloc(&mm->poll_host, 3 * sizeof(CgCol) * kMaxK + sizeof(double) * kMaxK,
                              hipHostMallocDefault));
        for (auto &e : mm->poll_ev) DGO_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    CgCol *hpoll = (CgCol *)mm->poll_host;
    const int32_t cap = std::max<int32_t>(o.max_iter, 0);
    int32_t done_iters = 0, plan_end = cap;
    int flight[2], nflight = 0, next_slot = 0;
    double last_rr[kMaxK];
    int32_t last_it[kMaxK];
    for (int c = 0; c < k; ++c) {
        last_rr[c] = 0.0;
        last_it[c] = -1;
    }
    auto queue_chunk = [&](int32_t len) -> dgo_status {
        const int slot = next_slot;
        next_slot ^= 1;
        iterate(s, done_iters, len);
        done_iters += len;
        DGO_HIP(hipMemcpyAsync(hpoll + slot * kMaxK, stt[(done_iters - 1) & 1], sizeof(CgCol) * k,
                               hipMemcpyDeviceToHost, s));
        DGO_HIP(hipEventRecord(mm->poll_ev[slot], s));
        DGO_HIP(hipGetLastError());
        flight[nflight++] = slot;
        return DGO_OK;
    };
    if (cap > 0) DGO_TRY(queue_chunk(std::min(every, cap)));
    while (nflight > 0) {
        if (nflight < 2 && done_iters < plan_end) DGO_TRY(queue_chunk(std::min(every, plan_end - done_iters)));
        const int slot = flight[0];
        flight[0] = flight[1];
        --nflight;
        DGO_HIP(hipEventSynchronize(mm->poll_ev[slot]));
        const CgCol *sc = hpoll + slot * kMaxK;
        bool any = false, known = !o.fixed_iters;
        int64_t need_end = 0;
        for (int c = 0; c < k; ++c) {
            const CgCol &q = sc[c];
            if (!q.active) continue;
            any = true;
            double target = std::max(o.rtol * o.rtol * q.bb, o.atol * o.atol);
            if (o.rtol_initial > 0.0) target = std::max(target, o.rtol_initial * o.rtol_initial * q.rr0);
            if (last_it[c] >= 0 && q.iters > last_it[c] && q.rr > 0.0 && q.rr < last_rr[c] && target > 0.0) {
                // log of the residual norm^2 ratio per iteration (< 0)
                const double rate = std::log(q.rr / last_rr[c]) / (double)(q.iters - last_it[c]);
                const double more = q.rr > target ? std::ceil(std::log(target / q.rr) / rate) : 0.0;
                // the state of iteration i reaches the host after chunk end i + 1
                need_end = std::max<int64_t>(need_end, q.iters + (int64_t)std::min(more, 1e9) + 2);
            } else {
                known = false;
            }
            last_rr[c] = q.rr;
            last_it[c] = q.iters;
        }
        if (!any) break;
        plan_end = known ? (int32_t)std::min<int64_t>(cap, need_end) : cap;
        if (nflight == 0 && done_iters >= plan_end)  // a column outran the plan
            plan_end = std::min(cap, done_iters + 2);
    }
    if (done_iters > 0)
        launch_fin<FIN_SR_ITER>(partU[done_iters & 1], (int)nb_v, part2, nbs, k,
                                stt[(done_iters + 1) & 1], stt[done_iters & 1], prm, nullptr, s);
    unorder(done_iters);
    // the true residual: FP64 solves with the SpMV's lane groups, FP32 ones
    // with one thread per (row, column) accumulating in FP64
    int nb_tr = (int)nb_t;
    if constexpr (sizeof(R) == 8) {
        nb_tr = mask ? launch_trueres_rows_m<R, true>(m, ra, M, rb, K, mask, k, beff, u, part, s)
                     : launch_trueres_rows_m<R, false>(m, ra, M, rb, K, mask, k, beff, u, part, s);
    } else {
        DGO_LAUNCH("cg_trueres", s,
                   k_cg_trueres<R><<<nb_t, TR, 0, s>>>(m->rowptr, m->col, (int32_t)nV, alpha, M, beta,
                                                      K, mask, k, KP, beff, u, part));
    }
    launch_fin<FIN_OUT>(part, nb_tr, nullptr, 0, k, nullptr, nullptr, prm, tr, s);
    DGO_HIP(hipGetLastError());
    // into pinned memory (a copy to pageable memory would block the host
    // once per copy); a chunk still in flight wrote its polling slot earlier
    // in stream order
    CgCol *hst = hpoll + 2 * kMaxK;
    double *htr = (double *)(hpoll + 3 * kMaxK);
    DGO_HIP(hipMemcpyAsync(hst, stt[done_iters & 1], sizeof(CgCol) * k, hipMemcpyDeviceToHost, s));
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
        if (o.strict) return fail(DGO_ERR_NOT_CONVERGED, "dgo_pcg: a column did not reach its tolerance");
        if (getenv("DGO_LOG") && atoi(getenv("DGO_LOG")) > 0)
            fprintf(stderr, "dgo_pcg: warning: not every column reached its tolerance\n");
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
    if (!m->rdesc || !m->rlen)
        return fail(DGO_ERR_INVALID_ARG, "dgo_spmv: mesh was built without SpMV row descriptors");
    hipStream_t s = (hipStream_t)stream;
    if (beta == 0.0) {  // the diagonal alpha M: no pass over K
        const int64_t n = (int64_t)batch * m->nV * k;
        if (dtype == DGO_F64)
            DGO_LAUNCH("spmm_diag", s,
                       k_diag_apply<double><<<grid_for(n, T), T, 0, s>>>(
                           n, k, alpha, (const double *)d_Mdiag, (const double *)d_x,
                           (double *)d_y));
        else
            DGO_LAUNCH("spmm_diag", s,
                       k_diag_apply<float><<<grid_for(n, T), T, 0, s>>>(
                           n, k, (float)alpha, (const float *)d_Mdiag, (const float *)d_x,
                           (float *)d_y));
        DGO_HIP(hipGetLastError());
        return DGO_OK;
    }
    if (dtype == DGO_F64)
        launch_spmm<double>(m, batch, alpha, (const double *)d_Mdiag, beta, (const double *)d_Kvals, k,
                            (const double *)d_x, (double *)d_y, s);
    else
        launch_spmm<float>(m, batch, (float)alpha, (const float *)d_Mdiag, (float)beta,
                           (const float *)d_Kvals, k, (const float *)d_x, (float *)d_y, s);
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
    if (!m->rdesc || !m->rlen)
        return fail(DGO_ERR_INVALID_ARG, "dgo_pcg: mesh was built without SpMV row descriptors");
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
        o.rtol_initial = 0.0;
        o.atol = 0.0;
    }
    if (o.max_iter < 0 || !(o.rtol >= 0.0) || !(o.rtol_initial >= 0.0) || !(o.atol >= 0.0))
        return fail(DGO_ERR_INVALID_ARG, "dgo_pcg: bad options");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == DGO_F64)
        return run_pcg<double>(m, alpha, (const double *)d_Mdiag, beta, (const double *)d_Kvals,
                               d_mask, (const double *)d_g, k, (const double *)d_b, (double *)d_u, o,
                               h_rep, s);
    return run_pcg<float>(m, alpha, (const float *)d_Mdiag, beta, (const float *)d_Kvals, d_mask,
                          (const float *)d_g, k, (const float *)d_b, (float *)d_u, o, h_rep, s);
}

extern "C" dgo_status dgo_linear_solve_vjp(const dgo_mesh *m, dgo_dtype dtype, double alpha,
                                           double beta, int32_t k, const void *d_lambda,
                                           const void *d_u, const void *d_f, void *d_gK,
                                           void *d_gM, dgo_stream stream) {
    clear_error();
    if (!m || !d_lambda || !d_u || !d_gK || !d_gM)
        return fail(DGO_ERR_INVALID_ARG, "dgo_linear_solve_vjp: NULL argument");
    if (k < 1 || k > kMaxK) return fail(DGO_ERR_INVALID_ARG, "dgo_linear_solve_vjp: k must be in [1, 64]");
    if (dtype != DGO_F32 && dtype != DGO_F64)
        return fail(DGO_ERR_INVALID_ARG, "dgo_linear_solve_vjp: bad dtype");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == DGO_F64)
        DGO_LAUNCH("solve_vjp", s,
                   k_solve_vjp<double><<<grid_for(m->nV, T), T, 0, s>>>(
                       m->rowptr, m->col, m->nV, alpha, beta, k, (const double *)d_lambda,
                       (const double *)d_u, (const double *)d_f, (double *)d_gK, (double *)d_gM));
    else
        DGO_LAUNCH("solve_vjp", s,
                   k_solve_vjp<float><<<grid_for(m->nV, T), T, 0, s>>>(
                       m->rowptr, m->col, m->nV, (float)alpha, (float)beta, k,
                       (const float *)d_lambda, (const float *)d_u, (const float *)d_f,
                       (float *)d_gK, (float *)d_gM));
    DGO_HIP(hipGetLastError());
    return DGO_OK;
}

// ------------------------------------------------ allocation-free PCG form

namespace {

// Workspace of dgo_pcg_fixed_noalloc: one static device array per GPU the
// library runs on (held until the process ends). Host code never passes the
// array's name to a kernel: it takes the array's device address from
// hipGetSymbolAddress, once per device, and passes that.
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on
// that device, with the device current).
dgo_status scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(DGO_ERR_UNSUPPORTED, "dgo_pcg_fixed_noalloc: device ordinal above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        if (!p) return fail(DGO_ERR_DEVICE, "dgo_pcg_fixed_noalloc: no scratch address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DGO_OK;
}

}  // namespace

extern "C" size_t dgo_pcg_fixed_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

extern "C" size_t dgo_pcg_fixed_noalloc_bytes(const dgo_mesh *m, dgo_dtype dtype, int32_t k) {
    if (!m || k < 1 || k > kMaxK || (dtype != DGO_F32 && dtype != DGO_F64)) return 0;
    const int64_t nvals = m->ell_w > 0 ? (int64_t)m->nV * m->ell_w : m->nnz;
    return pcg_layout(m->nV, nvals, k, dtype == DGO_F64 ? 8 : 4).total;
}

extern "C" dgo_status dgo_pcg_fixed_noalloc(const dgo_mesh *m, dgo_dtype dtype, double alpha,
                                            const void *d_Mdiag, double beta, const void *d_Kvals,
                                            const uint8_t *d_mask, const void *d_g, int32_t k,
                                            const void *d_b, void *d_u, int32_t iters,
                                            dgo_stream stream) {
    clear_error();
    if (!m || !d_Mdiag || !d_Kvals || !d_b || !d_u)
        return fail(DGO_ERR_INVALID_ARG, "dgo_pcg_fixed_noalloc: NULL argument");
    if (k < 1 || k > kMaxK) return fail(DGO_ERR_INVALID_ARG, "dgo_pcg_fixed_noalloc: k must be in [1, 64]");
    if (iters < 0) return fail(DGO_ERR_INVALID_ARG, "dgo_pcg_fixed_noalloc: iters must be >= 0");
    if (d_mask && !d_g) return fail(DGO_ERR_INVALID_ARG, "dgo_pcg_fixed_noalloc: mask given without g");
    if (dtype != DGO_F32 && dtype != DGO_F64)
        return fail(DGO_ERR_INVALID_ARG, "dgo_pcg_fixed_noalloc: bad dtype");
    if (!m->rdesc || !m->rlen)
        return fail(DGO_ERR_INVALID_ARG, "dgo_pcg_fixed_noalloc: mesh was built without SpMV row descriptors");
    int dev = 0;
    DGO_HIP(hipGetDevice(&dev));
    if (dev != m->device)
        return fail(DGO_ERR_INVALID_ARG, "dgo_pcg_fixed_noalloc: the mesh lives on another device");
    const size_t need = dgo_pcg_fixed_noalloc_bytes(m, dtype, k);
    if (need > kNoAllocScratchBytes)
        return fail(DGO_ERR_UNSUPPORTED,
                    "dgo_pcg_fixed_noalloc: this mesh and column count need " + std::to_string(need) +
                        " bytes of workspace; the static scratch holds " +
                        std::to_string(kNoAllocScratchBytes) + " (use dgo_pcg)");
    void *ws = nullptr;
    DGO_TRY(scratch_address(dev, &ws));
    dgo_cg_opts o{};
    o.rtol = 0.0;
    o.max_iter = iters;
    o.fixed_iters = 1;
    o.check_every = iters > 0 ? iters : 1;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == DGO_F64)
        return run_pcg<double>(m, alpha, (const double *)d_Mdiag, beta, (const double *)d_Kvals,
                               d_mask, (const double *)d_g, k, (const double *)d_b, (double *)d_u, o,
                               nullptr, s, (char *)ws);
    return run_pcg<float>(m, alpha, (const float *)d_Mdiag, beta, (const float *)d_Kvals, d_mask,
                          (const float *)d_g, k, (const float *)d_b, (float *)d_u, o, nullptr, s,
                          (char *)ws);
}
