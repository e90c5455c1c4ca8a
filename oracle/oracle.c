/*
 * Oracle for the mesh-operator path (FP64, single thread, plain loops).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg. It shares nothing with the HIP library.
 *
 * What it follows:
 *  - topology: the simplex sets and incidence tensors of Sec. 4.1 (EV, VV)
 *    and the face-vertex / face-subface / subface-orientation tensors of
 *    Sec. 6.1, with subface j opposite vertex j;
 *  - operators: the cotangent Laplacian built from per-edge cotangent weights
 *    and the diagonal mass matrix of the MCF application (Sec. 7.1), and the
 *    ARAP example of Sec. 4.2 (cotan_weights -> laplacian_from_weights).
 *    Reading: weights are 1/2 (cot a + cot b) per edge (the P1 stiffness),
 *    K is exported positive semidefinite (K = -L of the MCF equation), the
 *    mass is barycentric (area/3, volume/4); for tetrahedra K is the P1
 *    stiffness vol * grad(phi_i) . grad(phi_j);
 *  - solves: textbook Jacobi-preconditioned CG (Saad, Iterative Methods for
 *    Sparse Linear Systems, 2nd ed., Alg. 9.1), standing in for the linear
 *    solves of Sec. 5.2 and the quadratic energy with fixed values used in
 *    the ARAP step;
 *  - derivatives: the vector-Jacobian product of assembly with respect to the
 *    vertex positions, the term df/dx of the adjoint method (Sec. 3.1) for the
 *    MCF relation whose matrices depend on the positions.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

static int nloc_vertices(int dim) { return dim == 2 ? 3 : (dim == 3 ? 4 : 0); }
static int nloc_edges(int dim) { return dim == 2 ? 3 : (dim == 3 ? 6 : 0); }

/* local vertex pair of each local edge slot */
static void local_pair(int dim, int slot, int *a, int *b) {
    if (dim == 2) {
        *a = (slot + 1) % 3;
        *b = (slot + 2) % 3;
    } else {
        static const int P[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        *a = P[slot][0];
        *b = P[slot][1];
    }
}

typedef struct { int32_t lo, hi; } pair_t;

static int cmp_pair(const void *pa, const void *pb) {
    const pair_t *a = (const pair_t *)pa, *b = (const pair_t *)pb;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    return 0;
}

/* index of (lo,hi) in the sorted unique edge list, or -1 */
static int64_t find_edge(const int32_t *EV, int64_t nE, int32_t lo, int32_t hi) {
    int64_t a = 0, b = nE;
    while (a < b) {
        int64_t m = (a + b) / 2;
        int32_t l = EV[2 * m], h = EV[2 * m + 1];
        if (l < lo || (l == lo && h < hi)) a = m + 1; else b = m;
    }
    if (a < nE && EV[2 * a] == lo && EV[2 * a + 1] == hi) return a;
    return -1;
}

/* CSR slot of (i,j), or -1 */
static int64_t find_slot(const int32_t *rowptr, const int32_t *col, int32_t i, int32_t j) {
    int64_t a = rowptr[i], b = rowptr[i + 1];
    while (a < b) {
        int64_t m = (a + b) / 2;
        if (col[m] < j) a = m + 1; else b = m;
    }
    if (a < rowptr[i + 1] && col[a] == j) return a;
    return -1;
}

static void sub3(const double *a, const double *b, double *o) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ----------------------------------------------------------- validation */

int orc_validate(int dim, int32_t nV, int64_t n_elem, const int32_t *elem) {
    int nv = nloc_vertices(dim);
    if (!nv || nV < 0 || n_elem < 0) return ORC_ERR_INVALID_ARG;
    for (int64_t e = 0; e < n_elem; ++e) {
        for (int a = 0; a < nv; ++a) {
            int32_t v = elem[e * nv + a];
            if (v < 0 || v >= nV) return ORC_ERR_INDEX_RANGE;
            for (int b = 0; b < a; ++b)
                if (elem[e * nv + b] == v) return ORC_ERR_INVALID_ARG;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------- topology */

int orc_edges(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
              int32_t *EV, int64_t *nE, int32_t *elem_edge, int8_t *elem_sign) {
    int st = orc_validate(dim, nV, n_elem, elem);
    if (st) return st;
    int nv = nloc_vertices(dim), ne = nloc_edges(dim);
    int64_t nkeys = n_elem * ne;
    pair_t *keys = (pair_t *)malloc(sizeof(pair_t) * (nkeys ? nkeys : 1));
    if (!keys) return ORC_ERR_NOMEM;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int s = 0; s < ne; ++s) {
            int a, b;
            local_pair(dim, s, &a, &b);
            int32_t va = elem[e * nv + a], vb = elem[e * nv + b];
            keys[e * ne + s].lo = va < vb ? va : vb;
            keys[e * ne + s].hi = va < vb ? vb : va;
        }
    qsort(keys, nkeys, sizeof(pair_t), cmp_pair);
    int64_t m = 0;
    for (int64_t i = 0; i < nkeys; ++i) {
        if (m == 0 || cmp_pair(&keys[i], &keys[m - 1]) != 0) keys[m++] = keys[i];
    }
    for (int64_t i = 0; i < m; ++i) {
        EV[2 * i] = keys[i].lo;
        EV[2 * i + 1] = keys[i].hi;
    }
    free(keys);
    *nE = m;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int s = 0; s < ne; ++s) {
            int a, b;
            local_pair(dim, s, &a, &b);
            int32_t va = elem[e * nv + a], vb = elem[e * nv + b];
            int32_t lo = va < vb ? va : vb, hi = va < vb ? vb : va;
            elem_edge[e * ne + s] = (int32_t)find_edge(EV, m, lo, hi);
            elem_sign[e * ne + s] = va < vb ? 1 : -1;
        }
    return ORC_OK;
}

int orc_csr(int32_t nV, int64_t nE, const int32_t *EV, int32_t *rowptr, int32_t *col) {
    int64_t nnz = (int64_t)nV + 2 * nE;
    pair_t *ent = (pair_t *)malloc(sizeof(pair_t) * (nnz ? nnz : 1));
    if (!ent) return ORC_ERR_NOMEM;
    int64_t n = 0;
    for (int32_t i = 0; i < nV; ++i) { ent[n].lo = i; ent[n].hi = i; ++n; }
    for (int64_t e = 0; e < nE; ++e) {
        ent[n].lo = EV[2 * e]; ent[n].hi = EV[2 * e + 1]; ++n;
        ent[n].lo = EV[2 * e + 1]; ent[n].hi = EV[2 * e]; ++n;
    }
    qsort(ent, nnz, sizeof(pair_t), cmp_pair);
    for (int32_t i = 0; i <= nV; ++i) rowptr[i] = 0;
    for (int64_t t = 0; t < nnz; ++t) {
        rowptr[ent[t].lo + 1] += 1;
        col[t] = ent[t].hi;
    }
    for (int32_t i = 0; i < nV; ++i) rowptr[i + 1] += rowptr[i];
    free(ent);
    return ORC_OK;
}

typedef struct { int32_t v[3]; } tri_t;

static int cmp_tri(const void *pa, const void *pb) {
    const tri_t *a = (const tri_t *)pa, *b = (const tri_t *)pb;
    for (int i = 0; i < 3; ++i)
        if (a->v[i] != b->v[i]) return a->v[i] < b->v[i] ? -1 : 1;
    return 0;
}

static void sort3(int32_t *v) {
    int32_t t;
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
    if (v[1] > v[2]) { t = v[1]; v[1] = v[2]; v[2] = t; }
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
}

int orc_boundary(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
                 uint8_t *mask, int64_t *n_bfaces) {
    int st = orc_validate(dim, nV, n_elem, elem);
    if (st) return st;
    memset(mask, 0, (size_t)nV);
    *n_bfaces = 0;
    if (dim == 2) {
        /* edges (as sorted pairs) that occur in exactly one triangle */
        int64_t n = n_elem * 3;
        pair_t *k = (pair_t *)malloc(sizeof(pair_t) * (n ? n : 1));
        if (!k) return ORC_ERR_NOMEM;
        for (int64_t e = 0; e < n_elem; ++e)
            for (int s = 0; s < 3; ++s) {
                int32_t a = elem[e * 3 + (s + 1) % 3], b = elem[e * 3 + (s + 2) % 3];
                k[e * 3 + s].lo = a < b ? a : b;
                k[e * 3 + s].hi = a < b ? b : a;
            }
        qsort(k, n, sizeof(pair_t), cmp_pair);
        for (int64_t i = 0; i < n;) {
            int64_t j = i;
            while (j < n && cmp_pair(&k[i], &k[j]) == 0) ++j;
            if (j - i == 1) {
                mask[k[i].lo] = 1;
                mask[k[i].hi] = 1;
                *n_bfaces += 1;
            }
            i = j;
        }
        free(k);
    } else {
        /* triangles (sorted triples), face j of a tet opposite vertex j */
        int64_t n = n_elem * 4;
        tri_t *k = (tri_t *)malloc(sizeof(tri_t) * (n ? n : 1));
        if (!k) return ORC_ERR_NOMEM;
        for (int64_t e = 0; e < n_elem; ++e)
            for (int j = 0; j < 4; ++j) {
                int t = 0;
                for (int a = 0; a < 4; ++a)
                    if (a != j) k[e * 4 + j].v[t++] = elem[e * 4 + a];
                sort3(k[e * 4 + j].v);
            }
        qsort(k, n, sizeof(tri_t), cmp_tri);
        for (int64_t i = 0; i < n;) {
            int64_t j = i;
            while (j < n && cmp_tri(&k[i], &k[j]) == 0) ++j;
            if (j - i == 1) {
                for (int a = 0; a < 3; ++a) mask[k[i].v[a]] = 1;
                *n_bfaces += 1;
            }
            i = j;
        }
        free(k);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------- operators */

/* cotangent of the angle at xk between xi - xk and xj - xk */
static double cot_at(const double *xi, const double *xj, const double *xk, int *degenerate) {
    double e1[3], e2[3], n[3];
    sub3(xi, xk, e1);
    sub3(xj, xk, e2);
    cross3(e1, e2, n);
    double s = sqrt(dot3(n, n));
    if (s == 0.0) { *degenerate = 1; return 0.0; }
    return dot3(e1, e2) / s;
}

static double tri_area(const double *x0, const double *x1, const double *x2) {
    double e1[3], e2[3], n[3];
    sub3(x1, x0, e1);
    sub3(x2, x0, e2);
    cross3(e1, e2, n);
    return 0.5 * sqrt(dot3(n, n));
}

/* P1 element stiffness of a tetrahedron: Kc[a][b] = vol grad(phi_a).grad(phi_b).
 * E has columns x_r - x_0 (r = 1..3); the rows of E^{-1} are grad(phi_1..3),
 * computed by cofactors, and grad(phi_0) = -(sum). */
static double tet_stiffness(const double *x0, const double *x1, const double *x2,
                            const double *x3, double Kc[4][4], int *degenerate) {
    double E[3][3];
    for (int r = 0; r < 3; ++r) {
        E[r][0] = x1[r] - x0[r];
        E[r][1] = x2[r] - x0[r];
        E[r][2] = x3[r] - x0[r];
    }
    double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1])
               - E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0])
               + E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    if (det == 0.0) { *degenerate = 1; memset(Kc, 0, sizeof(double) * 16); return 0.0; }
    double inv[3][3]; /* inverse by the adjugate: inv[i][j] = cof[j][i] / det */
    inv[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
    inv[0][1] = -(E[0][1] * E[2][2] - E[0][2] * E[2][1]) / det;
    inv[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
    inv[1][0] = -(E[1][0] * E[2][2] - E[1][2] * E[2][0]) / det;
    inv[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
    inv[1][2] = -(E[0][0] * E[1][2] - E[0][2] * E[1][0]) / det;
    inv[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
    inv[2][1] = -(E[0][0] * E[2][1] - E[0][1] * E[2][0]) / det;
    inv[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
    double g[4][3];
    for (int c = 0; c < 3; ++c) {
        g[1][c] = inv[0][c];
        g[2][c] = inv[1][c];
        g[3][c] = inv[2][c];
        g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    }
    double vol = fabs(det) / 6.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) Kc[a][b] = vol * dot3(g[a], g[b]);
    return vol;
}

int orc_edge_weights(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
                     const double *X, int64_t nE, const int32_t *elem_edge,
                     double *w) {
    int st = orc_validate(dim, nV, n_elem, elem);
    if (st) return st;
    int degenerate = 0;
    for (int64_t e = 0; e < nE; ++e) w[e] = 0.0;
    if (dim == 2) {
        for (int64_t f = 0; f < n_elem; ++f) {
            const int32_t *v = elem + 3 * f;
            for (int k = 0; k < 3; ++k) {
                /* corner k is opposite edge slot k = {v[k+1], v[k+2]} */
                double c = cot_at(X + 3 * v[(k + 1) % 3], X + 3 * v[(k + 2) % 3],
                                  X + 3 * v[k], &degenerate);
                w[elem_edge[3 * f + k]] += 0.5 * c;
            }
        }
    } else {
        double Kc[4][4];
        for (int64_t t = 0; t < n_elem; ++t) {
            const int32_t *v = elem + 4 * t;
            tet_stiffness(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], X + 3 * v[3], Kc,
                          &degenerate);
            for (int s = 0; s < 6; ++s) {
                int a, b;
                local_pair(3, s, &a, &b);
                w[elem_edge[6 * t + s]] -= Kc[a][b];
            }
        }
    }
    return degenerate ? ORC_ERR_DEGENERATE : ORC_OK;
}

int orc_assemble(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
                 const double *X, const int32_t *rowptr, const int32_t *col,
                 double clamp_min, double *Kvals, double *Mdiag) {
    int st = orc_validate(dim, nV, n_elem, elem);
    if (st) return st;
    int nv = nloc_vertices(dim), ne = nloc_edges(dim);
    int64_t cap = n_elem * ne;
    int32_t *EV = (int32_t *)malloc(sizeof(int32_t) * 2 * (cap ? cap : 1));
    int32_t *ee = (int32_t *)malloc(sizeof(int32_t) * (cap ? cap : 1));
    int8_t *es = (int8_t *)malloc(cap ? cap : 1);
    double *w = (double *)malloc(sizeof(double) * (cap ? cap : 1));
    if (!EV || !ee || !es || !w) { free(EV); free(ee); free(es); free(w); return ORC_ERR_NOMEM; }
    int64_t nE = 0;
    st = orc_edges(dim, nV, n_elem, elem, EV, &nE, ee, es);
    int wst = st ? st : orc_edge_weights(dim, nV, n_elem, elem, X, nE, ee, w);
    if (st == ORC_OK) {
        int64_t nnz = rowptr[nV];
        for (int64_t t = 0; t < nnz; ++t) Kvals[t] = 0.0;
        for (int64_t e = 0; e < nE; ++e) {
            double we = w[e];
            if (we < clamp_min) we = clamp_min;
            int32_t a = EV[2 * e], b = EV[2 * e + 1];
            int64_t sab = find_slot(rowptr, col, a, b), sba = find_slot(rowptr, col, b, a);
            int64_t saa = find_slot(rowptr, col, a, a), sbb = find_slot(rowptr, col, b, b);
            if (sab < 0 || sba < 0 || saa < 0 || sbb < 0) { st = ORC_ERR_INVALID_ARG; break; }
            Kvals[sab] = -we;
            Kvals[sba] = -we;
            Kvals[saa] += we;
            Kvals[sbb] += we;
        }
        for (int32_t i = 0; i < nV; ++i) Mdiag[i] = 0.0;
        for (int64_t e = 0; e < n_elem && st == ORC_OK; ++e) {
            const int32_t *v = elem + nv * e;
            double m;
            if (dim == 2) {
                m = tri_area(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2]) / 3.0;
            } else {
                double Kc[4][4];
                int dg = 0;
                m = tet_stiffness(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], X + 3 * v[3],
                                  Kc, &dg) / 4.0;
            }
            for (int a = 0; a < nv; ++a) Mdiag[v[a]] += m;
        }
    }
    free(EV); free(ee); free(es); free(w);
    if (st) return st;
    return wst;
}

/* ------------------------------------------------------------------ SpMV */

int orc_spmv(int32_t nV, const int32_t *rowptr, const int32_t *col,
             double alpha, const double *Mdiag, double beta, const double *Kvals,
             int32_t k, const double *x, double *y) {
    if (k < 1) return ORC_ERR_INVALID_ARG;
    for (int32_t i = 0; i < nV; ++i)
        for (int32_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
                int32_t j = col[t];
                double a = beta * Kvals[t];
                if (j == i) a += alpha * Mdiag[i];
                s += a * x[(int64_t)j * k + c];
            }
            y[(int64_t)i * k + c] = s;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------- PCG */

/* y_I = A_II x_I on the interior (mask == 0) rows; y_B = 0. */
static void apply_reduced(int32_t nV, const int32_t *rowptr, const int32_t *col,
                          double alpha, const double *Mdiag, double beta,
                          const double *Kvals, const uint8_t *mask,
                          const double *x, double *y) {
    for (int32_t i = 0; i < nV; ++i) {
        if (mask && mask[i]) { y[i] = 0.0; continue; }
        double s = 0.0;
        for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
            int32_t j = col[t];
            if (mask && mask[j]) continue;
            double a = beta * Kvals[t];
            if (j == i) a += alpha * Mdiag[i];
            s += a * x[j];
        }
        y[i] = s;
    }
}

static double vdot(int32_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

int orc_pcg(int32_t nV, const int32_t *rowptr, const int32_t *col,
            double alpha, const double *Mdiag, double beta, const double *Kvals,
            const uint8_t *mask, const double *g, int32_t k, const double *b,
            double *u, double rtol, int32_t max_iter, int32_t *iters,
            double *relres) {
    if (k < 1 || max_iter < 0) return ORC_ERR_INVALID_ARG;
    if (mask && !g) return ORC_ERR_INVALID_ARG;
    double *D = (double *)malloc(sizeof(double) * nV);
    double *x = (double *)malloc(sizeof(double) * nV);
    double *r = (double *)malloc(sizeof(double) * nV);
    double *z = (double *)malloc(sizeof(double) * nV);
    double *p = (double *)malloc(sizeof(double) * nV);
    double *q = (double *)malloc(sizeof(double) * nV);
    double *be = (double *)malloc(sizeof(double) * nV);
    if (!D || !x || !r || !z || !p || !q || !be) {
        free(D); free(x); free(r); free(z); free(p); free(q); free(be);
        return ORC_ERR_NOMEM;
    }
    /* Jacobi preconditioner: the diagonal of A = alpha M + beta K */
    for (int32_t i = 0; i < nV; ++i) {
        D[i] = alpha * Mdiag[i];
        for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t)
            if (col[t] == i) D[i] += beta * Kvals[t];
    }
    for (int32_t c = 0; c < k; ++c) {
        /* effective right-hand side of the reduced system */
        for (int32_t i = 0; i < nV; ++i) be[i] = b[(int64_t)i * k + c];
        if (mask) {
            for (int32_t i = 0; i < nV; ++i) {
                if (mask[i]) { be[i] = 0.0; continue; }
                for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
                    int32_t j = col[t];
                    if (!mask[j]) continue;
                    double a = beta * Kvals[t];
                    if (j == i) a += alpha * Mdiag[i];
                    be[i] -= a * g[(int64_t)j * k + c];
                }
            }
        }
        for (int32_t i = 0; i < nV; ++i) x[i] = (mask && mask[i]) ? 0.0 : u[(int64_t)i * k + c];
        double bnorm = sqrt(vdot(nV, be, be));
        /* r0 = b - A x0, z0 = D^{-1} r0, p0 = z0 */
        apply_reduced(nV, rowptr, col, alpha, Mdiag, beta, Kvals, mask, x, q);
        for (int32_t i = 0; i < nV; ++i) {
            r[i] = be[i] - q[i];
            z[i] = (mask && mask[i]) ? 0.0 : r[i] / D[i];
            p[i] = z[i];
        }
        double rz = vdot(nV, r, z);
        double rnorm = sqrt(vdot(nV, r, r));
        int32_t it = 0;
        while (it < max_iter && !(rtol > 0.0 && rnorm <= rtol * bnorm)) {
            apply_reduced(nV, rowptr, col, alpha, Mdiag, beta, Kvals, mask, p, q);
            double a = rz / vdot(nV, p, q);
            for (int32_t i = 0; i < nV; ++i) {
                x[i] += a * p[i];
                r[i] -= a * q[i];
                z[i] = (mask && mask[i]) ? 0.0 : r[i] / D[i];
            }
            double rz_new = vdot(nV, r, z);
            double bt = rz_new / rz;
            rz = rz_new;
            for (int32_t i = 0; i < nV; ++i) p[i] = z[i] + bt * p[i];
            rnorm = sqrt(vdot(nV, r, r));
            ++it;
        }
        for (int32_t i = 0; i < nV; ++i)
            u[(int64_t)i * k + c] = (mask && mask[i]) ? g[(int64_t)i * k + c] : x[i];
        if (iters) iters[c] = it;
        if (relres) relres[c] = bnorm > 0.0 ? rnorm / bnorm : rnorm;
    }
    free(D); free(x); free(r); free(z); free(p); free(q); free(be);
    return ORC_OK;
}

/* ------------------------------------------------------------ gradients */

/* d cot(angle at xk) / d(xi, xj, xk), with e1 = xi - xk, e2 = xj - xk,
 * d = e1.e2, s = |e1 x e2|, cot = d / s:
 *   dcot/de1 = e2/s - d (|e2|^2 e1 - d e2) / s^3
 *   dcot/de2 = e1/s - d (|e1|^2 e2 - d e1) / s^3
 *   dcot/dxk = -(dcot/de1 + dcot/de2). */
static void cot_grad(const double *xi, const double *xj, const double *xk,
                     double gi[3], double gj[3], double gk[3]) {
    double e1[3], e2[3], n[3];
    sub3(xi, xk, e1);
    sub3(xj, xk, e2);
    cross3(e1, e2, n);
    double s = sqrt(dot3(n, n));
    double d = dot3(e1, e2), l1 = dot3(e1, e1), l2 = dot3(e2, e2);
    double s3 = s * s * s;
    for (int c = 0; c < 3; ++c) {
        gi[c] = e2[c] / s - d * (l2 * e1[c] - d * e2[c]) / s3;
        gj[c] = e1[c] / s - d * (l1 * e2[c] - d * e1[c]) / s3;
        gk[c] = -(gi[c] + gj[c]);
    }
}

/* d area / d(x0, x1, x2): area = s/2 with e1 = x1 - x0, e2 = x2 - x0,
 *   d area/de1 = (|e2|^2 e1 - d e2) / (2 s), d area/de2 = (|e1|^2 e2 - d e1) / (2 s). */
static void area_grad(const double *x0, const double *x1, const double *x2,
                      double g0[3], double g1[3], double g2[3]) {
    double e1[3], e2[3], n[3];
    sub3(x1, x0, e1);
    sub3(x2, x0, e2);
    cross3(e1, e2, n);
    double s = sqrt(dot3(n, n));
    double d = dot3(e1, e2), l1 = dot3(e1, e1), l2 = dot3(e2, e2);
    for (int c = 0; c < 3; ++c) {
        g1[c] = (l2 * e1[c] - d * e2[c]) / (2.0 * s);
        g2[c] = (l1 * e2[c] - d * e1[c]) / (2.0 * s);
        g0[c] = -(g1[c] + g2[c]);
    }
}

int orc_loss_grad_tri(int32_t nV, int64_t nF, const int32_t *F, const double *X,
                      const double *u, double *loss, double *grad) {
    int st = orc_validate(2, nV, nF, F);
    if (st) return st;
    int degenerate = 0;
    double L = 0.0;
    for (int64_t i = 0; i < (int64_t)nV * 3; ++i) grad[i] = 0.0;
    for (int64_t f = 0; f < nF; ++f) {
        const int32_t *v = F + 3 * f;
        /* u^T K u = sum over triangles and corners k of 1/2 cot_k (u_i - u_j)^2 */
        for (int k = 0; k < 3; ++k) {
            int32_t vi = v[(k + 1) % 3], vj = v[(k + 2) % 3], vk = v[k];
            double du = u[vi] - u[vj];
            double coef = 0.5 * du * du;
            L += coef * cot_at(X + 3 * vi, X + 3 * vj, X + 3 * vk, &degenerate);
            double gi[3], gj[3], gk[3];
            cot_grad(X + 3 * vi, X + 3 * vj, X + 3 * vk, gi, gj, gk);
            for (int c = 0; c < 3; ++c) {
                grad[3 * vi + c] += coef * gi[c];
                grad[3 * vj + c] += coef * gj[c];
                grad[3 * vk + c] += coef * gk[c];
            }
        }
        L += tri_area(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2]);
        double g0[3], g1[3], g2[3];
        area_grad(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], g0, g1, g2);
        for (int c = 0; c < 3; ++c) {
            grad[3 * v[0] + c] += g0[c];
            grad[3 * v[1] + c] += g1[c];
            grad[3 * v[2] + c] += g2[c];
        }
    }
    *loss = L;
    return degenerate ? ORC_ERR_DEGENERATE : ORC_OK;
}

/* complex-valued loss, written with sqrt(dot) (analytic) rather than |.| */
static double complex cdot3(const double complex *a, const double complex *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void ccross3(const double complex *a, const double complex *b, double complex *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

int orc_loss_cstep_tri(int32_t nV, int64_t nF, const int32_t *F, const double *X,
                       const double *u, int32_t v0, int32_t c0, double h,
                       double *dloss) {
    int st = orc_validate(2, nV, nF, F);
    if (st) return st;
    if (v0 < 0 || v0 >= nV || c0 < 0 || c0 > 2 || !(h > 0.0)) return ORC_ERR_INVALID_ARG;
    double complex L = 0.0;
    for (int64_t f = 0; f < nF; ++f) {
        const int32_t *v = F + 3 * f;
        double complex x[3][3];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                x[a][c] = X[3 * v[a] + c] + ((v[a] == v0 && c == c0) ? I * h : 0.0);
        for (int k = 0; k < 3; ++k) {
            int a = (k + 1) % 3, b = (k + 2) % 3;
            double complex e1[3], e2[3], n[3];
            for (int c = 0; c < 3; ++c) { e1[c] = x[a][c] - x[k][c]; e2[c] = x[b][c] - x[k][c]; }
            ccross3(e1, e2, n);
            double du = u[v[a]] - u[v[b]];
            L += 0.5 * du * du * cdot3(e1, e2) / csqrt(cdot3(n, n));
        }
        double complex e1[3], e2[3], n[3];
        for (int c = 0; c < 3; ++c) { e1[c] = x[1][c] - x[0][c]; e2[c] = x[2][c] - x[0][c]; }
        ccross3(e1, e2, n);
        L += 0.5 * csqrt(cdot3(n, n));
    }
    *dloss = cimag(L) / h;
    return ORC_OK;
}

int orc_assemble_vjp_tri(int32_t nV, int64_t nF, const int32_t *F, const double *X,
                         const int32_t *rowptr, const int32_t *col,
                         const double *gK, const double *gM, double *gX) {
    int st = orc_validate(2, nV, nF, F);
    if (st) return st;
    for (int64_t i = 0; i < (int64_t)nV * 3; ++i) gX[i] = 0.0;
    for (int64_t f = 0; f < nF; ++f) {
        const int32_t *v = F + 3 * f;
        for (int k = 0; k < 3; ++k) {
            int32_t vi = v[(k + 1) % 3], vj = v[(k + 2) % 3], vk = v[k];
            /* w_ij enters K_ij and K_ji with -1 and K_ii, K_jj with +1 */
            double gw = 0.0;
            if (gK) {
                int64_t sij = find_slot(rowptr, col, vi, vj), sji = find_slot(rowptr, col, vj, vi);
                int64_t sii = find_slot(rowptr, col, vi, vi), sjj = find_slot(rowptr, col, vj, vj);
                if (sij < 0 || sji < 0 || sii < 0 || sjj < 0) return ORC_ERR_INVALID_ARG;
                gw = -gK[sij] - gK[sji] + gK[sii] + gK[sjj];
            }
            double coef = 0.5 * gw;
            double gi[3], gj[3], gk[3];
            cot_grad(X + 3 * vi, X + 3 * vj, X + 3 * vk, gi, gj, gk);
            for (int c = 0; c < 3; ++c) {
                gX[3 * vi + c] += coef * gi[c];
                gX[3 * vj + c] += coef * gj[c];
                gX[3 * vk + c] += coef * gk[c];
            }
        }
        if (gM) {
            double ga = (gM[v[0]] + gM[v[1]] + gM[v[2]]) / 3.0;
            double g0[3], g1[3], g2[3];
            area_grad(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], g0, g1, g2);
            for (int c = 0; c < 3; ++c) {
                gX[3 * v[0] + c] += ga * g0[c];
                gX[3 * v[1] + c] += ga * g1[c];
                gX[3 * v[2] + c] += ga * g2[c];
            }
        }
    }
    return ORC_OK;
}

/* dl/dA = -lambda u^T restricted to the pattern, split into its K and M parts
 * (A = alpha M + beta K), plus the right-hand side's dependence on M when
 * b = M f: db/dM_ii = f_i, so gM_i gains lambda_i . f_i. */
int orc_linear_solve_vjp(int32_t nV, const int32_t *rowptr, const int32_t *col, double alpha,
                         double beta, int32_t k, const double *lambda, const double *u,
                         const double *f, double *gK, double *gM) {
    if (nV < 1 || k < 1 || !rowptr || !col || !lambda || !u || !gK || !gM)
        return ORC_ERR_INVALID_ARG;
    for (int32_t i = 0; i < nV; ++i) {
        for (int32_t t = rowptr[i]; t < rowptr[i + 1]; ++t) {
            const int32_t j = col[t];
            double s = 0.0;
            for (int32_t c = 0; c < k; ++c) s += lambda[(int64_t)i * k + c] * u[(int64_t)j * k + c];
            gK[t] = -beta * s;
        }
        double m = 0.0;
        for (int32_t c = 0; c < k; ++c) m += lambda[(int64_t)i * k + c] * u[(int64_t)i * k + c];
        double g = -alpha * m;
        if (f) {
            double q = 0.0;
            for (int32_t c = 0; c < k; ++c) q += lambda[(int64_t)i * k + c] * f[(int64_t)i * k + c];
            g += q;
        }
        gM[i] = g;
    }
    return ORC_OK;
}

/* Area from three edge lengths: Heron's formula in Kahan's stable form
 * (sorted a >= b >= c, "Miscalculating Area and Angles of a Needle-like
 * Triangle"). */
static double heron_area(double a, double b, double c) {
    double t;
    if (a < b) { t = a; a = b; b = t; }
    if (a < c) { t = a; a = c; c = t; }
    if (b < c) { t = b; b = c; c = t; }
    double q = (a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c));
    return q > 0.0 ? 0.25 * sqrt(q) : 0.0;
}

int orc_assemble_intrinsic(int32_t nV, int64_t nF, const int32_t *F, const double *lengths,
                           const int32_t *rowptr, const int32_t *col, double *Kvals,
                           double *Mdiag) {
    int st = orc_validate(2, nV, nF, F);
    if (st) return st;
    if (!lengths || !rowptr || !col || !Kvals || !Mdiag) return ORC_ERR_INVALID_ARG;
    int64_t cap = nF * 3;
    int32_t *EV = (int32_t *)malloc(sizeof(int32_t) * 2 * (cap ? cap : 1));
    int32_t *ee = (int32_t *)malloc(sizeof(int32_t) * (cap ? cap : 1));
    int8_t *es = (int8_t *)malloc(cap ? cap : 1);
    double *w = (double *)malloc(sizeof(double) * (cap ? cap : 1));
    if (!EV || !ee || !es || !w) { free(EV); free(ee); free(es); free(w); return ORC_ERR_NOMEM; }
    int64_t nE = 0;
    st = orc_edges(2, nV, nF, F, EV, &nE, ee, es);
    if (st == ORC_OK) {
        for (int64_t e = 0; e < nE; ++e) w[e] = 0.0;
        for (int32_t i = 0; i < nV; ++i) Mdiag[i] = 0.0;
        for (int64_t t = 0; t < nF && st == ORC_OK; ++t) {
            double l[3];
            for (int j = 0; j < 3; ++j) l[j] = lengths[ee[3 * t + j]];
            double A = heron_area(l[0], l[1], l[2]);
            if (A == 0.0) { st = ORC_ERR_DEGENERATE; break; }
            for (int j = 0; j < 3; ++j) {
                double lj1 = l[(j + 1) % 3], lj2 = l[(j + 2) % 3];
                double cot = (lj1 * lj1 + lj2 * lj2 - l[j] * l[j]) / (4.0 * A);
                w[ee[3 * t + j]] += 0.5 * cot;
            }
            for (int j = 0; j < 3; ++j) Mdiag[F[3 * t + j]] += A / 3.0;
        }
        if (st == ORC_OK) {
            int64_t nnz = rowptr[nV];
            for (int64_t t = 0; t < nnz; ++t) Kvals[t] = 0.0;
            for (int64_t e = 0; e < nE; ++e) {
                int32_t a = EV[2 * e], b = EV[2 * e + 1];
                int64_t sab = find_slot(rowptr, col, a, b), sba = find_slot(rowptr, col, b, a);
                int64_t saa = find_slot(rowptr, col, a, a), sbb = find_slot(rowptr, col, b, b);
                if (sab < 0 || sba < 0 || saa < 0 || sbb < 0) { st = ORC_ERR_INVALID_ARG; break; }
                Kvals[sab] = -w[e];
                Kvals[sba] = -w[e];
                Kvals[saa] += w[e];
                Kvals[sbb] += w[e];
            }
        }
    }
    free(EV); free(ee); free(es); free(w);
    return st;
}

/* grad phi_j of the face's three vertices and its area */
static void face_grads(const double *x0, const double *x1, const double *x2, double g[3][3],
                       double *area) {
    const double *x[3] = {x0, x1, x2};
    double e1[3], e2[3], n[3];
    for (int c = 0; c < 3; ++c) { e1[c] = x1[c] - x0[c]; e2[c] = x2[c] - x0[c]; }
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    *area = 0.5 * sqrt(nn);
    for (int j = 0; j < 3; ++j) {
        const double *p = x[(j + 1) % 3], *q = x[(j + 2) % 3];
        double e[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        g[j][0] = (n[1] * e[2] - n[2] * e[1]) / nn;
        g[j][1] = (n[2] * e[0] - n[0] * e[2]) / nn;
        g[j][2] = (n[0] * e[1] - n[1] * e[0]) / nn;
    }
}

int orc_face_gradient(int32_t nV, int64_t nF, const int32_t *F, const double *X, int32_t k,
                      const double *u, double *g) {
    int st = orc_validate(2, nV, nF, F);
    if (st) return st;
    if (k < 1 || !X || !u || !g) return ORC_ERR_INVALID_ARG;
    for (int64_t t = 0; t < nF; ++t) {
        const int32_t *v = F + 3 * t;
        double gr[3][3], A;
        face_grads(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], gr, &A);
        for (int32_t c = 0; c < k; ++c)
            for (int d = 0; d < 3; ++d) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j) s += u[(int64_t)v[j] * k + c] * gr[j][d];
                g[((int64_t)c * 3 + d) * nF + t] = s;
            }
    }
    return ORC_OK;
}

int orc_face_divergence(int32_t nV, int64_t nF, const int32_t *F, const double *X, int32_t k,
                        const double *y, double *div) {
    int st = orc_validate(2, nV, nF, F);
    if (st) return st;
    if (k < 1 || !X || !y || !div) return ORC_ERR_INVALID_ARG;
    for (int64_t i = 0; i < (int64_t)nV * k; ++i) div[i] = 0.0;
    for (int64_t t = 0; t < nF; ++t) {
        const int32_t *v = F + 3 * t;
        double gr[3][3], A;
        face_grads(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], gr, &A);
        for (int j = 0; j < 3; ++j)
            for (int32_t c = 0; c < k; ++c) {
                const double *yc = y + (int64_t)c * 3 * nF + t;
                div[(int64_t)v[j] * k + c] +=
                    A * (gr[j][0] * yc[0] + gr[j][1] * yc[nF] + gr[j][2] * yc[2 * nF]);
            }
    }
    return ORC_OK;
}

int orc_mass_voronoi(int32_t nV, int64_t nF, const int32_t *F, const double *X, double *M) {
    int st = orc_validate(2, nV, nF, F);
    if (st) return st;
    if (!X || !M) return ORC_ERR_INVALID_ARG;
    for (int32_t i = 0; i < nV; ++i) M[i] = 0.0;
    for (int64_t t = 0; t < nF; ++t) {
        const int32_t *v = F + 3 * t;
        const double *x[3] = {X + 3 * v[0], X + 3 * v[1], X + 3 * v[2]};
        double A = tri_area(x[0], x[1], x[2]);
        if (A == 0.0) return ORC_ERR_DEGENERATE;
        /* the angle at corner j is obtuse when the dot product of its two
         * edges is negative */
        int obtuse = -1;
        for (int j = 0; j < 3; ++j) {
            double e1[3], e2[3];
            sub3(x[(j + 1) % 3], x[j], e1);
            sub3(x[(j + 2) % 3], x[j], e2);
            if (dot3(e1, e2) < 0.0) obtuse = j;
        }
        for (int j = 0; j < 3; ++j) {
            const double *P = x[j], *Q = x[(j + 1) % 3], *R = x[(j + 2) % 3];
            double a;
            if (obtuse < 0) {
                int deg = 0;
                double PR[3], PQ[3];
                sub3(R, P, PR);
                sub3(Q, P, PQ);
                a = (dot3(PR, PR) * cot_at(P, R, Q, &deg) + dot3(PQ, PQ) * cot_at(P, Q, R, &deg)) / 8.0;
            } else {
                a = obtuse == j ? A / 2.0 : A / 4.0;
            }
            M[v[j]] += a;
        }
    }
    return ORC_OK;
}

int orc_slot_map(int dim, int32_t nV, int64_t n_elem, const int32_t *elem, const int32_t *rowptr,
                 const int32_t *col, int32_t *slots) {
    int st = orc_validate(dim, nV, n_elem, elem);
    if (st) return st;
    if (!rowptr || !col || !slots) return ORC_ERR_INVALID_ARG;
    const int nv = dim + 1, nl = dim == 2 ? 3 : 6;
    for (int64_t e = 0; e < n_elem; ++e)
        for (int j = 0; j < nl; ++j) {
            int a, b;
            local_pair(dim, j, &a, &b);
            const int32_t va = elem[e * nv + a], vb = elem[e * nv + b];
            const int64_t sab = find_slot(rowptr, col, va, vb), sba = find_slot(rowptr, col, vb, va);
            if (sab < 0 || sba < 0) return ORC_ERR_INVALID_ARG;
            slots[(e * nl + j) * 2] = (int32_t)sab;
            slots[(e * nl + j) * 2 + 1] = (int32_t)sba;
        }
    return ORC_OK;
}
