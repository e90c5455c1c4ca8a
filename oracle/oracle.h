/*
 * Oracle for the mesh-operator path: a plain, slow, single-threaded FP64 CPU
 * implementation written from the paper's definitions.
 *
 * TEST INFRASTRUCTURE ONLY. It is called by the tests, by the smoke check and
 * by the benchmark's CPU-baseline leg, never by the library itself. It shares
 * no code, header, table or helper with the HIP library.
 *
 * Index arrays are int32, row-major: triangles (n_elem x 3), tetrahedra
 * (n_elem x 4). Positions are double (nV x 3). Vectors with k right-hand sides
 * are vertex-major (nV x k). All functions return 0 on success or one of the
 * ORC_ERR_* codes; no function allocates memory it hands back.
 */
#ifndef DGO_ORACLE_H
#define DGO_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_ERR_INVALID_ARG 1
#define ORC_ERR_INDEX_RANGE 2
#define ORC_ERR_DEGENERATE 3
#define ORC_ERR_NOMEM 4

/* Element indices in [0, nV) and pairwise distinct within each element. */
int orc_validate(int dim, int32_t nV, int64_t n_elem, const int32_t *elem);

/* Edges (Sec. 4.1 notation EV) and the element -> edge map (Sec. 6.1
 * face-subface and subface-orientation tensors, d = 1 level).
 *   EV        : out, capacity n_elem*nl*2, first 2*nE entries written, edges
 *               as (min, max), sorted lexicographically; edge id = rank.
 *   elem_edge : out, n_elem*nl. Triangles: slot j is the edge opposite local
 *               vertex j, i.e. {v[j+1], v[j+2]} (indices mod 3).
 *               Tetrahedra: slots are the local pairs 01,02,03,12,13,23.
 *   elem_sign : out, n_elem*nl, +1 if the slot's local pair (first, second)
 *               runs from the smaller to the larger vertex id, else -1.
 *   nl = 3 (triangles) or 6 (tetrahedra). */
int orc_edges(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
              int32_t *EV, int64_t *nE, int32_t *elem_edge, int8_t *elem_sign);

/* CSR pattern {(i,i)} U {(i,j),(j,i) : edge ij}, rows ascending, columns
 * ascending within a row. rowptr: nV+1, col: nV + 2 nE. */
int orc_csr(int32_t nV, int64_t nE, const int32_t *EV, int32_t *rowptr, int32_t *col);

/* Slot map (the CSR slots the scatter of Sec. 6.1 reaches through an
 * element's local pairs): for element e and local
 * pair slot j (the element->edge slot order of orc_edges), slots[(e*nl + j)*2]
 * is the CSR position of (a, b) in row a and slots[(e*nl + j)*2 + 1] that of
 * (b, a) in row b, (a, b) the pair's vertices in local order. */
int orc_slot_map(int dim, int32_t nV, int64_t n_elem, const int32_t *elem, const int32_t *rowptr,
                 const int32_t *col, int32_t *slots);

/* Boundary: triangle meshes mark the vertices of edges with one incident
 * triangle; tetrahedral meshes mark the vertices of triangles that belong to
 * one tetrahedron. mask: nV bytes (1 = boundary). n_bfaces: number of
 * boundary edges (dim 2) or boundary triangles (dim 3). */
int orc_boundary(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
                 uint8_t *mask, int64_t *n_bfaces);

/* Cotangent stiffness K (positive semidefinite, K_ij = -w_ij, K_ii = sum_j
 * w_ij) in CSR order and the barycentric lumped mass M (diagonal).
 * clamp_min: if > -inf, every per-edge weight w is replaced by max(w,
 * clamp_min) before the diagonal is formed. Returns ORC_ERR_DEGENERATE if an
 * element has zero measure (outputs are then unspecified). */
int orc_assemble(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
                 const double *X, const int32_t *rowptr, const int32_t *col,
                 double clamp_min, double *Kvals, double *Mdiag);

/* Per-edge weights w (indexed like EV) as the plain sum over elements. */
int orc_edge_weights(int dim, int32_t nV, int64_t n_elem, const int32_t *elem,
                     const double *X, int64_t nE, const int32_t *elem_edge,
                     double *w);

/* y = (alpha M + beta K) x for k columns (x, y: nV x k). */
int orc_spmv(int32_t nV, const int32_t *rowptr, const int32_t *col,
             double alpha, const double *Mdiag, double beta, const double *Kvals,
             int32_t k, const double *x, double *y);

/* Jacobi-preconditioned CG on (alpha M + beta K) u = b, per column, from the
 * initial guess in u. With a Dirichlet mask (may be NULL) rows and columns
 * of masked vertices are eliminated: b_I <- b_I - A_IB g_B, u_B = g_B.
 * A column stops when ||r||_2 <= rtol ||b_eff||_2 (rtol <= 0: never) or
 * after max_iter iterations. iters (k) and relres (k, recursive residual over
 * ||b_eff||) are outputs and may be NULL. */
int orc_pcg(int32_t nV, const int32_t *rowptr, const int32_t *col,
            double alpha, const double *Mdiag, double beta, const double *Kvals,
            const uint8_t *mask, const double *g, int32_t k, const double *b,
            double *u, double rtol, int32_t max_iter, int32_t *iters,
            double *relres);

/* Triangle meshes: loss = u^T K(X) u + sum_T area_T and its gradient with
 * respect to X (nV x 3), summed per element in ascending element order. */
int orc_loss_grad_tri(int32_t nV, int64_t nF, const int32_t *F, const double *X,
                      const double *u, double *loss, double *grad);

/* Complex-step derivative of the same loss with respect to X[v, c]:
 * Im(loss(X + i h e_vc)) / h. */
int orc_loss_cstep_tri(int32_t nV, int64_t nF, const int32_t *F, const double *X,
                       const double *u, int32_t v, int32_t c, double h,
                       double *dloss);

/* Vector-Jacobian product of triangle assembly:
 * gX = (dKvals/dX)^T gK + (dMdiag/dX)^T gM; gK (CSR-aligned) or gM may be
 * NULL (treated as zero). Unclamped weights. */
int orc_assemble_vjp_tri(int32_t nV, int64_t nF, const int32_t *F, const double *X,
                         const int32_t *rowptr, const int32_t *col,
                         const double *gK, const double *gM, double *gX);

/* Gradients of a linear solve with respect to its operators (the adjoint
 * method of Sec. 3.1, Eq. implicit-full, for the linear relation
 * f(u; K, M) = (alpha M + beta K) u - b of Sec. 5.2; the MCF step of Sec. 7.1
 * is the case alpha = 1, beta = tau, b = M x). With u solving
 * (alpha M + beta K) u = b and lambda solving the same (symmetric) system with
 * the loss gradient dl/du on the right-hand side, dl/dA = -lambda u^T, so on
 * the CSR pattern:
 *   gK[t] = -beta * sum_c lambda[i,c] u[j,c]          (slot t = (i, j))
 *   gM[i] = -alpha * sum_c lambda[i,c] u[i,c]
 *           + sum_c lambda[i,c] f[i,c]                (only when b = M f, f != NULL)
 * lambda, u, f: nV x k. */
int orc_linear_solve_vjp(int32_t nV, const int32_t *rowptr, const int32_t *col, double alpha,
                         double beta, int32_t k, const double *lambda, const double *u,
                         const double *f, double *gK, double *gM);

/* Intrinsic assembly (Sec. 7.2, the intrinsic cotangent weights of the SCP
 * example): K and M of a triangle mesh from its edge lengths alone. lengths
 * is indexed like EV (the sorted (min, max) edges of orc_edges). For a
 * triangle with edge lengths l_j (edge opposite local vertex j) and area A
 * (Heron's formula in Kahan's stable form), the angle at vertex j has
 * cot = (l_{j+1}^2 + l_{j+2}^2 - l_j^2) / (4 A); K and M then follow as in
 * orc_assemble (w_ij = sum of 1/2 cot over the triangles on edge ij,
 * M_ii = sum of A / 3). */
int orc_assemble_intrinsic(int32_t nV, int64_t nF, const int32_t *F, const double *lengths,
                           const int32_t *rowptr, const int32_t *col, double *Kvals,
                           double *Mdiag);

/* Per-face gradient G (Sec. 7.4: the gradient operator of the geodesic
 * example) of k vertex fields u (nV x k, row-major): (G u)_f = sum_j u[v_j]
 * grad phi_j, grad phi_j = (n x e_j) / |n|^2 with n = (x1 - x0) x (x2 - x0)
 * and e_j = x_{j+2} - x_{j+1} the edge opposite local vertex j. g is
 * component-major like the (3, nF) face fields of that example: component d
 * of field c on face f at g[(c * 3 + d) * nF + f]. */
int orc_face_gradient(int32_t nV, int64_t nF, const int32_t *F, const double *X, int32_t k,
                      const double *u, double *g);

/* Divergence D = G^T diag(A_f): (D y)_i = sum over the faces f of i of
 * A_f grad phi_i . y_f, for k face vector fields y in the layout of g above;
 * div: nV x k. The sign is the one the u-update of the geodesic ADMM loop
 * (Sec. 7.4) needs with an SPD Laplacian: D G = K, the cotangent stiffness. */
int orc_face_divergence(int32_t nV, int64_t nF, const int32_t *F, const double *X, int32_t k,
                        const double *y, double *div);

/* Mixed-Voronoi lumped mass of a triangle mesh (the "vertex areas" variant
 * of the lumped mass, Sec. 7.1 and 7.4; the mixed area of Meyer et al. 2003):
 * per triangle and corner P with other corners Q, R: if no angle of the
 * triangle is obtuse, (|PR|^2 cot Q + |PQ|^2 cot R) / 8 (the corner's Voronoi
 * region); else A/2 for the obtuse corner and A/4 for the other two. */
int orc_mass_voronoi(int32_t nV, int64_t nF, const int32_t *F, const double *X, double *M);

#endif
