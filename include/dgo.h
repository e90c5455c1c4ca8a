/*
 * dgo -- discrete geometry operators on simplicial meshes for MI355X (gfx950).
 *
 * C ABI of the library libdgo.so. It follows the statement of the problem in
 * the paper "iskra: A System for Inverse Geometry Processing" (arXiv
 * 2602.12105): a mesh is a set of simplices with unique indices and a
 * canonical orientation (Sec. 4.1); its topology is the hierarchy of
 * face-subface tensors (Sec. 6.1); per-element quantities are scattered down
 * the hierarchy into vertex-indexed sparse operators (Sec. 5.1), the
 * cotangent Laplacian and diagonal mass matrix of the MCF application
 * (Sec. 7.1), which are then applied inside linear solves (Sec. 5.2) and
 * differentiated with respect to the vertex positions (the df/dx term of the
 * adjoint method, Sec. 3.1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named d_* are device pointers (HBM of the current HIP device);
 *   h_* are host pointers. The caller owns every pointer it passes and keeps
 *   it alive until the work enqueued on the stream has finished. The library
 *   owns the storage inside dgo_mesh and dgo_server objects.
 * - dgo_stream is a hipStream_t (NULL = the legacy default stream). Numeric
 *   calls only enqueue work on that stream and return; they synchronise the
 *   stream only when a host-side result pointer (h_*) is non-NULL or when
 *   stated below.
 * - Indices are int32; element arrays are row-major (n_elem x 3) for
 *   triangles (dim = 2) and (n_elem x 4) for tetrahedra (dim = 3).
 * - Vertex positions are (batch x nV x 3), row-major, in the call's dtype.
 *   Vectors with k columns are vertex-major: (nV x k).
 * - Operators use the CSR pattern of the mesh (dgo_mesh_csr): the stiffness
 *   values Kvals are (batch x nnz) aligned with that pattern, the lumped mass
 *   Mdiag is (batch x nV).
 * - Sign convention: K is positive semidefinite, K_ij = -w_ij for an edge ij
 *   and K_ii = sum_j w_ij, with w_ij = 1/2 (cot a_ij + cot b_ij) on triangle
 *   meshes and the P1 stiffness on tetrahedra. The paper's Laplacian L of the
 *   MCF equation (M - tau L) v' = M v is -K.
 * - Every call returns a dgo_status. On failure nothing is enqueued, except
 *   where noted, and dgo_last_error() returns a message for the calling
 *   thread. No C++ exception crosses this boundary.
 * - A mesh object may be used from one host thread at a time: the numeric
 *   calls share a scratch workspace stored inside it.
 */
#ifndef DGO_H
#define DGO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *dgo_stream; /* hipStream_t */

typedef enum {
    DGO_OK = 0,
    DGO_ERR_INVALID_ARG = 1,   /* bad pointer, size, dtype or option */
    DGO_ERR_INDEX_RANGE = 2,   /* an element index outside [0, nV) */
    DGO_ERR_DEGENERATE = 3,    /* an element of zero measure */
    DGO_ERR_NOMEM = 4,         /* device allocation failed */
    DGO_ERR_DEVICE = 5,        /* a HIP runtime error */
    DGO_ERR_NOT_CONVERGED = 6, /* solver stopped early and strict was set */
    DGO_ERR_BUDGET = 7,        /* request larger than the server's HBM budget */
    DGO_ERR_UNSUPPORTED = 8,   /* valid input outside what the library handles */
    DGO_ERR_TIMEOUT = 9,       /* a wait ran out of time */
    DGO_ERR_SHUTDOWN = 10      /* server is shutting down */
} dgo_status;

typedef enum { DGO_F32 = 0, DGO_F64 = 1 } dgo_dtype;

/* Optional device allocator; NULL means hipMallocAsync / hipFreeAsync on the
 * stream given to the call that allocates. alloc returns NULL on failure. */
typedef struct {
    void *(*alloc)(size_t bytes, dgo_stream stream, void *ctx);
    void (*free)(void *ptr, dgo_stream stream, void *ctx);
    void *ctx;
} dgo_allocator;

typedef struct dgo_mesh dgo_mesh;

typedef struct {
    int32_t dim;        /* 2 triangles, 3 tetrahedra */
    int32_t nV;         /* vertices */
    int64_t n_elem;     /* triangles or tetrahedra */
    int64_t nE;         /* edges */
    int64_t nnz;        /* CSR entries = nV + 2 nE */
    int64_t n_bfaces;   /* boundary edges (dim 2) or boundary triangles (dim 3) */
    int64_t n_boundary; /* boundary vertices */
    int32_t max_row;    /* longest CSR row (1 + vertex degree) */
} dgo_sizes;

/* ---------------------------------------------------------------- topology */

/* Build the topology of a simplicial mesh (Sec. 4.1 simplex sets and EV, VV;
 * Sec. 6.1 face-subface and subface-orientation tensors):
 *   - edges EV as (min, max) vertex pairs sorted lexicographically, edge id =
 *     rank (the canonical orientation is min -> max);
 *   - the element -> edge map and its orientation signs;
 *   - the CSR pattern {(i,i)} U VV with ascending columns per row;
 *   - boundary vertices (edges of one triangle / triangles of one tetrahedron);
 *   - the per-vertex incidence lists the assembly kernels read.
 * d_elem: device, (n_elem x (dim+1)) int32, read during the call only (the
 * library keeps its own copy). Every index must lie in [0, nV) and the
 * vertices of an element must be distinct: otherwise DGO_ERR_INDEX_RANGE or
 * DGO_ERR_INVALID_ARG. A vertex touched by no element is allowed (an isolated
 * row holding only its diagonal). Rows longer than 255 entries (vertex degree
 * above 254) return DGO_ERR_UNSUPPORTED.
 * Synchronises the stream (sizes are needed on the host). On success *out is
 * a new mesh owned by the caller, released with dgo_mesh_destroy. */
dgo_status dgo_mesh_create(int32_t dim, int32_t nV, int64_t n_elem, const int32_t *d_elem,
                           const dgo_allocator *alloc, dgo_stream stream, dgo_mesh **out);

/* Release a mesh and its device storage (after synchronising its last
 * stream). NULL is accepted. */
void dgo_mesh_destroy(dgo_mesh *mesh);

/* Sizes of the mesh's simplex sets and operators (the element, edge and
 * vertex counts of the simplex hierarchy, Sec. 4.1 and 6.1, and the nonzero
 * count of the vertex-indexed operators of Sec. 5.1), read on the host: no
 * device work, no synchronisation. DGO_ERR_INVALID_ARG for NULL arguments. */
dgo_status dgo_mesh_sizes(const dgo_mesh *mesh, dgo_sizes *out);

/* Copy out the edge topology (any pointer may be NULL to skip it):
 *   d_EV (nE x 2), d_elem_edge (n_elem x nl), d_elem_sign (n_elem x nl),
 * nl = 3 for triangles (slot j = edge opposite local vertex j, the paper's
 * rule that subface j is opposite vertex j) and 6 for tetrahedra (local pairs
 * 01, 02, 03, 12, 13, 23). sign = +1 when the slot's local pair runs from the
 * smaller to the larger vertex id. */
dgo_status dgo_mesh_edges(const dgo_mesh *mesh, int32_t *d_EV, int32_t *d_elem_edge,
                          int8_t *d_elem_sign, dgo_stream stream);

/* Copy out the CSR pattern of the vertex-indexed operators: the diagonal and
 * the vertex adjacency VV (Sec. 4.1; the vertex_adjacency of the ARAP
 * example, Sec. 4.2), rows sorted by column. d_rowptr (nV + 1) and d_col
 * (nnz) are caller-owned device buffers sized from dgo_mesh_sizes; either
 * may be NULL. Enqueued on the stream (device-to-device copies). */
dgo_status dgo_mesh_csr(const dgo_mesh *mesh, int32_t *d_rowptr, int32_t *d_col,
                        dgo_stream stream);

/* COO form of the CSR pattern (the coordinate sparse format of Sec. 5.1):
 * d_row (nnz) receives the row of every CSR slot, d_col (nnz) its column, so
 * values stored in CSR order (Kvals) are already in this COO order. Either
 * pointer may be NULL, not both. */
dgo_status dgo_mesh_coo(const dgo_mesh *mesh, int32_t *d_row, int32_t *d_col, dgo_stream stream);

/* Per-element CSR slot map (the slots the scatter of Sec. 6.1 reaches through
 * an element's local pairs): d_slots (n_elem x nl x 2 int32) receives, for
 * local pair j of element e (the slot order of dgo_mesh_edges), the CSR
 * position of (a, b) in row a and of (b, a) in row b, (a, b) the pair's
 * vertices in local order. */
dgo_status dgo_mesh_slots(const dgo_mesh *mesh, int32_t *d_slots, dgo_stream stream);

/* Copy out the boundary-vertex mask: the vertices of edges with one incident
 * triangle, or of triangles with one incident tetrahedron. These are where
 * the boundary conditions a geometric solver takes as input are imposed
 * (Sec. 4, the programming model) and the kind of fixed-value set the quadratic-energy solve of the
 * ARAP example takes (Sec. 4.2); dgo_pcg accepts such a mask. d_mask (nV
 * bytes, 1 = boundary), caller-owned device memory. DGO_ERR_INVALID_ARG for
 * NULL arguments; enqueued on the stream. */
dgo_status dgo_mesh_boundary(const dgo_mesh *mesh, uint8_t *d_mask, dgo_stream stream);

/* ----------------------------------------------------------------- assembly */

typedef struct {
    /* Clamp of the per-edge weights (the clamp_min argument of the paper's
     * cotan_weights, Sec. 4.2): when use_clamp != 0 every summed edge weight
     * w is replaced by max(w, clamp_min) and the diagonal is formed from the
     * clamped weights. */
    int32_t use_clamp;
    double clamp_min;
    /* Lumped mass: 0 = barycentric (A/3 per triangle corner, vol/4 per tet
     * corner); 1 = mixed Voronoi (the "vertex areas" variant, triangles only:
     * per corner the Voronoi region (|e_ij|^2 cot k + |e_ik|^2 cot j) / 8 when
     * the triangle has no obtuse angle, else A/2 at the obtuse corner and A/4
     * at the others; Meyer et al. 2003). */
    int32_t mass;
} dgo_assemble_opts;

/* Edge-weight clamp of the ARAP example (Sec. 4.2): its cotan_weights call
 * clamps the weights from below at this value. */
#define DGO_ARAP_CLAMP_MIN 1e-5

/* Assemble the stiffness K and lumped mass M of `batch` meshes that share
 * this topology (the cotangent Laplacian of the ARAP example, Sec. 4.2, and
 * the Laplacian and diagonal mass matrix of the MCF application, Sec. 7.1):
 *   triangles: w_ij = sum over triangles on edge ij of 1/2 cot(opposite angle),
 *              M_ii = sum over incident triangles of area/3;
 *   tetrahedra: w_ij = -sum over tets on edge ij of vol grad(phi_i).grad(phi_j),
 *              M_ii = sum over incident tets of vol/4.
 * d_X (batch x nV x 3), d_Kvals (batch x nnz), d_Mdiag (batch x nV) in dtype.
 * opts may be NULL (no clamp). The result is bitwise deterministic and
 * bitwise symmetric (K_ij == K_ji). If h_n_degenerate is non-NULL the call
 * synchronises, stores the number of zero-measure elements (over the batch)
 * and returns DGO_ERR_DEGENERATE when it is not zero; otherwise such elements
 * silently produce non-finite values. */
dgo_status dgo_assemble(const dgo_mesh *mesh, dgo_dtype dtype, int32_t batch, const void *d_X,
                        const dgo_assemble_opts *opts, void *d_Kvals, void *d_Mdiag,
                        int64_t *h_n_degenerate, dgo_stream stream);

/* Vector-Jacobian product of dgo_assemble (unclamped) with respect to the
 * vertex positions, for triangle meshes: the df/dx factor of the adjoint
 * method (Sec. 3.1, Eq. implicit-full) for a relation whose matrices depend on
 * the positions, as in the MCF application (Sec. 7.1):
 *   d_gX = (dKvals/dX)^T gK + (dMdiag/dX)^T gM,
 * d_gK (batch x nnz) and d_gM (batch x nV) may each be NULL (= zero);
 * d_gX (batch x nV x 3) is overwritten. Deterministic. dim 3 meshes return
 * DGO_ERR_UNSUPPORTED. */
dgo_status dgo_assemble_vjp(const dgo_mesh *mesh, dgo_dtype dtype, int32_t batch,
                            const void *d_X, const void *d_gK, const void *d_gM, void *d_gX,
                            dgo_stream stream);

/* Intrinsic assembly (the intrinsic cotangent weights of the SCP example,
 * Sec. 7.2): K and M of a triangle mesh from its edge lengths alone. For a
 * triangle with edge lengths l_j (edge opposite local vertex j) and area A
 * (Heron's formula in Kahan's stable form), the weight of the angle at vertex
 * j is 1/2 cot = (l_{j+1}^2 + l_{j+2}^2 - l_j^2) / (8 A); K and M then follow
 * as in dgo_assemble (w_ij summed over the triangles on edge ij, M_ii = sum of
 * A / 3). d_lengths (batch x nE) is indexed like the mesh's edges
 * (dgo_mesh_edges order; may be NULL when the mesh has no edges); d_Kvals (batch x nnz), d_Mdiag (batch x nV). opts
 * and h_n_degenerate as in dgo_assemble (lengths that violate the triangle
 * inequality count as zero-area triangles). Bitwise deterministic and
 * symmetric. The first call on a mesh allocates its per-incidence face list
 * (4 bytes per vertex-face incidence). dim 3 meshes return
 * DGO_ERR_UNSUPPORTED. */
dgo_status dgo_assemble_intrinsic(const dgo_mesh *mesh, dgo_dtype dtype, int32_t batch,
                                  const void *d_lengths, const dgo_assemble_opts *opts,
                                  void *d_Kvals, void *d_Mdiag, int64_t *h_n_degenerate,
                                  dgo_stream stream);

/* Conformal Laplacian of the spectral conformal parameterization (Sec. 7.2)
 * from a stiffness K of this triangle mesh (d_Kvals, nnz, from dgo_assemble
 * or dgo_assemble_intrinsic): the 2 nV x 2 nV matrix
 *   L_C = [[K, -S], [S, K]]   (unknowns: all x, then all y),
 * with 1/2 u^T L_C u = E_D(u) - A(u) the conformal energy of a planar map u:
 * E_D its Dirichlet energy and A(u) = x^T S y its signed area over the
 * boundary edges, S_ij = 1/2 and S_ji = -1/2 for a boundary edge running
 * i -> j in its triangle's orientation. CSR output, columns sorted: row x_i
 * is K's row i then -S_ij at columns nV + j; row y_i is S_ij at columns j then
 * K's row i at columns nV + j. d_rowptr2 (2 nV + 1) and d_col2 (nnz2) may be
 * NULL (the pattern depends on the topology only); d_vals2 (nnz2) in dtype,
 * nnz2 = 2 nnz + 4 n_bfaces (n_bfaces: boundary edges, dgo_mesh_sizes).
 * Exact (entries are copies of K or +-1/2). The first call on a mesh caches
 * the boundary orientation of its CSR slots (nnz bytes + 4 (nV + 1)). */
dgo_status dgo_conformal_laplacian(const dgo_mesh *mesh, dgo_dtype dtype, const void *d_Kvals,
                                   int32_t *d_rowptr2, int32_t *d_col2, void *d_vals2,
                                   dgo_stream stream);

/* ------------------------------------------------ face gradient, divergence */

/* Per-face gradient G (the gradient operator of the geodesic example,
 * Sec. 7.4) of k vertex fields: (G u)_f = sum_j u[v_j] grad phi_j with
 * grad phi_j = (n x e_j) / |n|^2, n = (x1 - x0) x (x2 - x0), e_j = x_{j+2} -
 * x_{j+1} the edge opposite local vertex j. d_X (nV x 3), d_u (nV x k,
 * row-major), 1 <= k <= 64; d_g (k x 3 x nF, component-major: component d of
 * field c on face f at [(c * 3 + d) * nF + f], the (3, nF) face-field layout
 * of that example) is overwritten; it may be NULL when the mesh has no
 * faces (then nothing is done). Triangle meshes only (else
 * DGO_ERR_UNSUPPORTED). Zero-area faces give non-finite values. */
dgo_status dgo_face_gradient(const dgo_mesh *mesh, dgo_dtype dtype, const void *d_X, int32_t k,
                             const void *d_u, void *d_g, dgo_stream stream);

/* Divergence D = G^T diag(A_f) (the divergence operator of Sec. 7.4, with the
 * sign its u-update needs when the Laplacian is the SPD stiffness: D G = K):
 * (D y)_i = sum over the faces f of vertex i of A_f grad phi_i . y_f. d_y
 * (k x 3 x nF, the layout of dgo_face_gradient's output; may be NULL when
 * the mesh has no faces: then every sum is 0), d_div (nV x k) is
 * overwritten. Each sum runs over the vertex's faces in ascending face order:
 * deterministic. The per-face corner terms are staged in the mesh's
 * workspace (3 k nF values, grown on demand and shared with the mesh's other
 * calls, so calls on one mesh must not overlap); the first call on a mesh
 * also allocates its per-incidence face lists (8 bytes per vertex-face
 * incidence). Triangle meshes with fewer than 2^31 / 3 faces only. */
dgo_status dgo_face_divergence(const dgo_mesh *mesh, dgo_dtype dtype, const void *d_X, int32_t k,
                               const void *d_y, void *d_div, dgo_stream stream);

/* --------------------------------------------------------- operator apply */

/* y = (alpha M + beta K) x for `batch` operator instances and k columns:
 * d_Mdiag (batch x nV), d_Kvals (batch x nnz), d_x and d_y (batch x nV x k),
 * 1 <= k <= 64. d_y must not alias d_x. This is the operator application
 * repeated inside the solves of Sec. 5.2. With beta == 0 the operator is the
 * diagonal alpha M and y = (alpha M_i) x_i is formed without reading K (the
 * same bits as the full product for finite x; d_Kvals must still be given). */
dgo_status dgo_spmv(const dgo_mesh *mesh, dgo_dtype dtype, int32_t batch, double alpha,
                    const void *d_Mdiag, double beta, const void *d_Kvals, int32_t k,
                    const void *d_x, void *d_y, dgo_stream stream);

/* Options of dgo_pcg. The relative and absolute tolerances follow the
 * paper's solver conventions (Sec. 6.2: absolute and relative tolerances, an
 * iteration cap, a warning or, with strict, an error when the cap is reached
 * with the tolerances unmet): a column stops as soon as
 *   ||r||_2 <= max(rtol ||b_eff||_2, atol),
 * r the recursive residual, b_eff the right-hand side after Dirichlet
 * elimination. Every dot product is accumulated in FP64 in both dtypes (there
 * is no option to turn that off). */
typedef struct {
    double rtol;          /* relative tolerance (see above), >= 0 */
    int32_t max_iter;     /* iteration cap per column */
    int32_t fixed_iters;  /* != 0: run exactly max_iter iterations, no test */
    int32_t check_every;  /* host convergence poll period (iterations), >= 1 */
    int32_t stall_iters;  /* > 0: also stop a column after this many
                             iterations without a new smallest residual */
    int32_t strict;       /* != 0: return DGO_ERR_NOT_CONVERGED if a column
                             stops without meeting rtol (the paper's strict
                             flag of its GMRES, Sec. 6.2) */
    double rtol_initial;  /* > 0: a column also stops (and counts as
                             converged) when ||r||_2 <= rtol_initial ||r_0||_2,
                             r_0 the residual of the initial guess; 0: off */
    double atol;          /* absolute tolerance on ||r||_2 (see above), >= 0;
                             0: relative test only */
} dgo_cg_opts;

typedef struct {
    int32_t k;
    int32_t converged_all;  /* 1 if every column met its tolerance */
    int32_t iters[64];      /* iterations per column */
    double relres[64];      /* recursive residual / ||b_eff|| per column */
    double true_relres[64]; /* ||b_eff - A u|| / ||b_eff|| evaluated in FP64 */
} dgo_cg_report;

/* Jacobi-preconditioned conjugate gradients (Saad, Alg. 9.1) on
 * (alpha M + beta K) u = b for k independent columns (1 <= k <= 64), standing
 * in for the linear solves of Sec. 5.2 and for the quadratic energy with
 * fixed values of the ARAP step (Sec. 4.2). Columns stop independently and
 * are frozen once stopped. d_Mdiag (nV), d_Kvals (nnz), d_b and d_u (nV x k);
 * d_u holds the initial guess on entry and the solution on exit.
 * Dirichlet data: when d_mask (nV bytes) is non-NULL, rows and columns of
 * masked vertices are eliminated (b_I <- b_I - A_IB g_B) and u_B = g_B on
 * exit, with d_g (nV x k). Vectors are in dtype; with F32 every dot product
 * is accumulated in FP64. Reductions are in a fixed order: the result is
 * bitwise deterministic. Polls the device every check_every iterations
 * (synchronising the stream); h_rep (may be NULL) receives the report.
 * Non-convergence returns DGO_OK unless opts->strict is set. */
dgo_status dgo_pcg(const dgo_mesh *mesh, dgo_dtype dtype, double alpha, const void *d_Mdiag,
                   double beta, const void *d_Kvals, const uint8_t *d_mask, const void *d_g,
                   int32_t k, const void *d_b, void *d_u, const dgo_cg_opts *opts,
                   dgo_cg_report *h_rep, dgo_stream stream);

/* Allocation-free form of dgo_pcg with a fixed iteration count, for callers
 * that cannot allocate device or host memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. It runs exactly
 * `iters` Jacobi-PCG iterations (the fixed_iters mode of dgo_pcg: the same
 * kernels, the same iterate bit for bit) on (alpha M + beta K) u = b with
 * optional Dirichlet data (d_mask, d_g as in dgo_pcg), and only enqueues work
 * on the stream: no host synchronisation, no progress polling, no report and
 * no true-residual pass. Arguments, layouts and ownership are those of
 * dgo_pcg (d_u holds the initial guess on entry, the iterate on exit).
 * Its workspace (the PCG vectors, partial sums and per-column state) is a
 * static device array of dgo_pcg_fixed_noalloc_max_bytes() = 128 MiB that
 * each GPU the library runs on holds until the process ends; a mesh and
 * column count needing more (dgo_pcg_fixed_noalloc_bytes) return
 * DGO_ERR_UNSUPPORTED without enqueuing anything (about 78 MB for the
 * icosphere of level 7 with 8 FP64 columns). The mesh must live on the
 * current device (else DGO_ERR_INVALID_ARG). Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller. Nothing in the array needs to
 * start at zero. The mesh itself is created (and allocates) beforehand. */
dgo_status dgo_pcg_fixed_noalloc(const dgo_mesh *mesh, dgo_dtype dtype, double alpha,
                                 const void *d_Mdiag, double beta, const void *d_Kvals,
                                 const uint8_t *d_mask, const void *d_g, int32_t k, const void *d_b,
                                 void *d_u, int32_t iters, dgo_stream stream);
/* Workspace bytes dgo_pcg_fixed_noalloc needs for this mesh, dtype and k (0
 * for invalid arguments), and the size of its static array. Host only. */
size_t dgo_pcg_fixed_noalloc_bytes(const dgo_mesh *mesh, dgo_dtype dtype, int32_t k);
size_t dgo_pcg_fixed_noalloc_max_bytes(void);

/* Gradients of a linear solve with respect to its operators: the adjoint
 * method (Sec. 3.1, Eq. implicit-full) applied to the linear relation
 * (alpha M + beta K) u - b = 0 of the solves of Sec. 5.2 (the implicit MCF
 * step of Sec. 7.1 is alpha = 1, beta = tau, b = M x). Given the solution u
 * and the adjoint solution lambda of the same symmetric system with the loss
 * gradient dl/du on the right-hand side (a second dgo_pcg call), dl/dA =
 * -lambda u^T restricted to the CSR pattern:
 *   d_gK[t] = -beta  sum_c lambda[i,c] u[j,c]       for CSR slot t = (i, j)
 *   d_gM[i] = -alpha sum_c lambda[i,c] u[i,c] + sum_c lambda[i,c] f[i,c]
 * where the last term (the right-hand side b = M f depends on M) is present
 * only when d_f is given. d_lambda, d_u, d_f: nV x k; d_gK: nnz; d_gM: nV;
 * the outputs are overwritten. Sums run over c in ascending order
 * (deterministic). DGO_ERR_INVALID_ARG for NULL outputs or inputs (other than
 * d_f), k outside [1, 64] or a bad dtype. */
dgo_status dgo_linear_solve_vjp(const dgo_mesh *mesh, dgo_dtype dtype, double alpha, double beta,
                                int32_t k, const void *d_lambda, const void *d_u, const void *d_f,
                                void *d_gK, void *d_gM, dgo_stream stream);

/* ------------------------------------------------------------ eigenpairs */

typedef struct {
    double sigma;           /* shift, < 0; 0 selects -1 / sum(M) (minus the
                               reciprocal of the total measure) */
    double tol;             /* stop when every requested pair has
                               ||K u - lam M u||_{M^-1} <= tol max(|lam|, |sigma|)
                               with u^T M u = 1 (0: 1e-8 FP64, 1e-4 FP32) */
    double inner_rtol;      /* PCG rtol of each inner solve (0: tol / 10) */
    double inner_rtol_initial; /* each inner solve also stops at this fraction
                               of its warm start's residual (0: 0.1; < 0: off) */
    int32_t block;          /* subspace size p, k <= p <= 64 (0: the power of
                               two >= k + 6, at most min(64, nV), at least k) */
    int32_t max_iter;       /* outer iterations (0: 200) */
    int32_t inner_max_iter; /* PCG iteration cap per solve (0: 20000) */
    int32_t reserved;
    uint64_t seed;          /* start block: splitmix64 stream from this seed */
} dgo_eig_opts;

typedef struct {
    int32_t k, block;
    int32_t iters;          /* outer iterations (solves) performed */
    int32_t converged;      /* 1 if every requested pair met tol */
    int64_t inner_iters;    /* PCG iterations summed over the solves (the
                               longest column of each) */
    double sigma;           /* shift used */
    double resid[64];       /* relative residual of each requested pair */
} dgo_eig_report;

/* The k smallest eigenpairs of K u = lam M u (the forward pass of the
 * spectral implicit layers, Sec. 5.2: A U = B U diag(lam), U^T B U = I with
 * A = K, B = M diagonal positive): subspace iteration on (K - sigma M)^-1 M
 * with Rayleigh-Ritz, the fixed point U = Q((A - sigma B)^-1 B U) of
 * Eq. eigiter, each inverse applied by dgo_pcg to all p columns. d_Mdiag
 * (nV), d_Kvals (nnz) in dtype; d_U (nV x k, row-major) receives the
 * M-orthonormal eigenvectors, each column signed so that its entry of
 * largest magnitude (the first on ties) is positive; h_lambda (k, host)
 * the eigenvalues ascending. 1 <= k <= min(64, nV). Synchronises the stream
 * once per outer iteration; deterministic. Returns DGO_ERR_NOT_CONVERGED
 * only if the iterated block loses rank; otherwise non-convergence is
 * reported in h_rep (may be NULL). opts may be NULL (defaults). */
dgo_status dgo_eigs_smallest(const dgo_mesh *mesh, dgo_dtype dtype, const void *d_Mdiag,
                             const void *d_Kvals, int32_t k, const dgo_eig_opts *opts, void *d_U,
                             double *h_lambda, dgo_eig_report *h_rep, dgo_stream stream);

/* ----------------------------------------------------------------- tracing */

/* Kernel timing for measurement (not part of the method). While enabled,
 * every kernel the library launches whose name contains `filter` (NULL or ""
 * = every kernel) is bracketed by a pair of hipEvents recorded on the stream
 * it is launched on. dgo_trace_read synchronises those events and returns,
 * per kernel name, the launch count and the summed and extreme durations.
 * Process-wide and thread-safe. Disabling keeps the collected records. */
typedef struct {
    char name[48];
    int64_t count;
    double total_ms, min_ms, max_ms;
} dgo_trace_entry;

dgo_status dgo_trace_enable(int32_t on, const char *filter);
/* Fill up to cap entries (sorted by total time, largest first); *n receives
 * the number of distinct kernels seen. Pending records are consumed. */
dgo_status dgo_trace_read(dgo_trace_entry *h_out, int32_t cap, int32_t *n);
void dgo_trace_reset(void);

/* ------------------------------------------------------------------ errors */

/* Message of the last failing call on this host thread ("" if none). */
const char *dgo_last_error(void);

/* Library version string. */
const char *dgo_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DGO_H */
