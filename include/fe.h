/*
 * fe.h -- C ABI of the MI355X finite element hot path: cell-wise Galerkin
 * integration on Lagrangian Q_k quadrilaterals/hexahedra, deterministic
 * scatter into a CSR matrix and right-hand side with strong Dirichlet
 * elimination, and the CSR SpMV inside a Jacobi-preconditioned CG solve.
 *
 * The method follows arXiv 1708.01773 (FEMPAR): the weak problem and its
 * affine operator F_h(u) = A u - f (Sect. 3.1-3.2), cell-wise assembly
 * A_[a][b] = sum_K A^K_ab (Sect. 3.6 eq. assembly), numerical integration on
 * the reference cell (Sect. 3.7 eqs. fematrix and shape_grad), Lagrangian
 * Q_k elements (Sect. 3.4 eqs. lagbas/lagbasmd, Sect. 3.8), strong Dirichlet
 * elimination with lifting (Sect. 10.4 eq. dirichlet_bc_discrete_problem),
 * CSR storage reused across assemblies (Sect. 11.1), and CG among the
 * library's iterative solvers (Sect. 12).
 *
 * General conventions
 *  - Every call returns fe_status; FE_OK == 0.  No exception crosses the ABI.
 *    On a non-OK status the output buffers are unspecified and
 *    fe_last_error() returns a text for the calling thread.
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library borrows them for the stream-ordered duration of the
 *    call and never frees them.  Library-owned device memory (mesh arrays,
 *    cached patterns and tables) lives until fe_destroy_mesh.
 *  - fe_stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that only enqueue work return as soon as it is enqueued.
 *  - Index types: row pointers and nnz counts are int64, column indices and
 *    cell-to-DOF entries int32 (a single system holds < 2^31 rows).
 *
 * Data layout and numbering (fixed, so that results are reproducible)
 *  - Mesh: structured brick of n0 x n1 (x n2) cells; vertex (i,j,l) has id
 *    i + (n0+1)(j + (n1+1) l) (x fastest); cell (i,j,l) has id
 *    i + n0 (j + n1 l); local vertex v = v0 + 2 v1 + 4 v2.
 *  - Reference cell [0,1]^d, equidistant nodes (Sect. 3.15), local node
 *    a = a0 + (k+1) a1 + (k+1)^2 a2, geometry map of order 1 for every k.
 *  - Global node lattice (n_r k + 1 nodes per axis).  A node is fixed when
 *    it lies on a Dirichlet face (bit 2r: x_r = 0, bit 2r+1: x_r = 1).  Free
 *    nodes are ranked lexicographically (x fastest); vector problems
 *    interleave components: DOF = ncomp * rank + c, local DOF ncomp * a + c.
 *  - CSR: rows are free DOFs, columns sorted ascending, every pair of free
 *    DOFs sharing a cell is stored (structural zeros included).
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *fe_stream; /* hipStream_t */

typedef enum {
    FE_OK = 0,
    FE_EINVAL = 1,      /* invalid argument (order, dim, sizes, null pointer, too small workspace) */
    FE_ENOMEM = 2,      /* device allocation failed or a budget was exceeded */
    FE_EMESH = 3,       /* a cell has det J <= 0 (at a corner on the host, at a quadrature point on the device) */
    FE_ENOTCONV = 4,    /* iterative solve reached maxit */
    FE_EBREAKDOWN = 5,  /* CG breakdown: p.Ap <= 0 or not finite */
    FE_EDEVICE = 6      /* a HIP runtime call failed */
} fe_status;

/* Text of the last non-OK status set on the calling thread ("" if none). */
const char *fe_last_error(void);

/* ABI version (incremented on incompatible changes). */
int32_t fe_version(void);

/* ------------------------------------------------------------------------ */
/* Mesh (Sect. 7: triangulation; the structured brick generator of Sect. 7.4) */
/* ------------------------------------------------------------------------ */
typedef struct fe_mesh_s *fe_mesh; /* opaque, library-owned */

typedef struct {
    int32_t dim;              /* 2 or 3 */
    int32_t n[3];             /* cells per axis (n[2] ignored for dim 2); each >= 1 */
    const double *vertex_xyz; /* host, (n0+1)(n1+1)[(n2+1)] x dim, AoS, x fastest; NULL = uniform grid on [0,1]^d */
    const double *cell_coeff; /* host, one coefficient per cell; NULL = 1.0 */
} fe_mesh_desc;

/* Copies the host arrays to the device (the caller may free them on return),
 * validates the geometry and returns a handle.  Synchronous.
 * FE_EMESH if det J <= 0 at any cell corner; FE_EINVAL on bad sizes. */
fe_status fe_create_mesh(const fe_mesh_desc *desc, fe_mesh *out);

/* Frees the mesh and everything cached in it.  Waits for pending work. */
fe_status fe_destroy_mesh(fe_mesh mesh);

/* Replaces the per-cell coefficients (host array, one per cell).  Synchronous.
 * Cached patterns and tables stay valid. */
fe_status fe_set_coefficients(fe_mesh mesh, const double *cell_coeff);

/* ------------------------------------------------------------------------ */
/* Problem description                                                       */
/* ------------------------------------------------------------------------ */
enum { FE_POISSON = 0, FE_ELASTICITY = 1 };
/* Precision of the element GEMM only.  Geometry (J, det J, J^-1), the load
 * vector, the scatter accumulation, the CSR values and every solver quantity
 * stay FP64.  FE_FP16/FE_BF16 round the GEMM inputs and accumulate in FP32. */
enum { FE_FP64 = 0, FE_FP32 = 1, FE_FP16 = 2, FE_BF16 = 3 };
enum { FE_SOURCE_NONE = 0, FE_SOURCE_CONST = 1, FE_SOURCE_SINPROD = 2 };
enum { FE_DIRICHLET_ZERO = 0, FE_DIRICHLET_AFFINE = 1 };

typedef struct {
    int32_t problem;           /* FE_POISSON: int k grad u . grad v ;
                                  FE_ELASTICITY: int k (2 mu eps(u):eps(v) + lambda div u div v),
                                  lambda, mu from young / poisson_ratio; ncomp = dim */
    int32_t precision;         /* FE_FP64 ... FE_BF16 */
    double young;              /* elasticity only */
    double poisson_ratio;      /* elasticity only, in (-1, 0.5) */
    int32_t source_kind;       /* NONE; CONST: f_c = source[c]; SINPROD: f_c = source[c] d pi^2 prod_r sin(pi x_r) */
    double source[3];
    uint32_t dirichlet_faces;  /* bitmask of the 2 dim faces; 0 = no fixed DOFs */
    int32_t dirichlet_kind;    /* ZERO, or AFFINE: u_D,c(x) = aff[4c] + sum_r aff[4c+1+r] x_r */
    double dirichlet_affine[12];
} fe_coeff;

/* CSR of the free-free system.  All pointers are device memory owned by the
 * caller: rowptr n_rows+1 (int64), colind nnz (int32), values nnz, rhs n_rows,
 * dinv n_rows (Jacobi: 1 / diagonal). */
typedef struct {
    int64_t n_rows;
    int64_t nnz;
    int64_t *rowptr;
    int32_t *colind;
    double *values;
    double *rhs;
    double *dinv;
} fe_csr;

/* ------------------------------------------------------------------------ */
/* Assembly                                                                  */
/* ------------------------------------------------------------------------ */
/* Sizes of the free-free system of (mesh, order, coeff) and the device
 * workspace fe_assemble / fe_integrate need (element matrices and loads).
 * Builds and caches the order-dependent set-up on first use (synchronous).
 * FE_EINVAL for order outside 1..4 or a bad coeff. */
fe_status fe_assemble_query(fe_mesh mesh, int32_t order, const fe_coeff *coeff,
                            int64_t *n_rows, int64_t *nnz, size_t *ws_bytes);

/* Symbolic phase (Sect. 11.1: the pattern is built once and reused by every
 * later assembly): writes out->rowptr and out->colind.  out->n_rows and
 * out->nnz must equal the query's values.  Enqueues only. */
fe_status fe_pattern(fe_mesh mesh, int32_t order, const fe_coeff *coeff, fe_csr *out, fe_stream stream);

/* Numeric phase: element integration (K3) into the workspace, then the
 * deterministic scatter (K5) of the free-free entries into out->values, of
 * loads and Dirichlet lifting into out->rhs, and out->dinv = 1 / diagonal.
 * Requires the pattern written by fe_pattern in out->rowptr/colind (it is
 * not read: the scatter evaluates the same positions).  No float atomics:
 * every value is a sum of its contributions in ascending cell order, so the
 * result is bitwise reproducible.  Enqueues only; a det J <= 0 found at a
 * quadrature point is reported by the next fe_get_status. */
fe_status fe_assemble(fe_mesh mesh, int32_t order, const fe_coeff *coeff, fe_csr *out,
                      void *ws, size_t ws_bytes, fe_stream stream);

/* K3 alone: element matrices and loads (with lifting) into the workspace.
 * Layout of the workspace (elements of type double for FE_FP64, float
 * otherwise, then the loads as double), cb and packed from fe_element_layout:
 *   E[((c / cb) * ne + e) * cb + c % cb]
 *     packed = 0: e = a * nloc + b, ne = nloc * nloc;
 *     packed = 1 (Q1 scalar; element matrices are symmetric): only a <= b is
 *       stored, e = a * nloc - a (a - 1) / 2 + (b - a), ne = nloc (nloc + 1) / 2;
 *   F[c * nloc + a]  starting at byte offset *load_offset. */
fe_status fe_integrate(fe_mesh mesh, int32_t order, const fe_coeff *coeff, void *ws, size_t ws_bytes,
                       fe_stream stream);
fe_status fe_element_layout(fe_mesh mesh, int32_t order, const fe_coeff *coeff, int32_t *nloc,
                            int32_t *cell_block, int32_t *elem_bytes, size_t *load_offset, int32_t *packed);

/* K5 alone: scatter of a workspace filled by fe_integrate into out. */
fe_status fe_scatter(fe_mesh mesh, int32_t order, const fe_coeff *coeff, fe_csr *out, const void *ws,
                     size_t ws_bytes, fe_stream stream);

/* Batched numeric phase: the assembly of fe_assemble (Sect. 3.6 eq. assembly,
 * Sect. 3.7) for nprob problems of different meshes, orders, problems and
 * precisions in one call.  Problems are grouped by kernel class (dimension,
 * order, components, precision); each class is one integration launch and
 * one scatter launch in which every problem owns its own range of
 * workgroups.  Classes without a batched kernel (2D orders >= 2, Q1
 * elasticity) and the Dirichlet lifting are launched per problem.  Each
 * problem's output is bitwise that of fe_assemble on it alone.
 *   meshes, orders, coeffs, out: host arrays of nprob entries.  A mesh may
 *   appear more than once only with the same order, problem and faces.
 *   out[i]: device CSR with the pattern of fe_pattern, sizes from the query.
 *   ws: device workspace of the size fe_assemble_batch_query reports (job
 *   tables plus every problem's element workspace).
 * Waits for the stream's earlier work before enqueueing (the job table is
 * staged from host memory), then enqueues only. */
fe_status fe_assemble_batch_query(int32_t nprob, const fe_mesh *meshes, const int32_t *orders,
                                  const fe_coeff *coeffs, int64_t *n_rows, int64_t *nnz, size_t *ws_bytes);
fe_status fe_assemble_batch(int32_t nprob, const fe_mesh *meshes, const int32_t *orders, const fe_coeff *coeffs,
                            fe_csr *out, void *ws, size_t ws_bytes, fe_stream stream);

/* Cell-to-DOF map (Sect. 10.1 lst_dofs_gids): out[c * nloc + ncomp * a + comp]
 * = free DOF id, or -1 - fixed DOF id.  out: device, ncells * nloc int32. */
fe_status fe_cell_dofs(fe_mesh mesh, int32_t order, const fe_coeff *coeff, int32_t *out, fe_stream stream);

/* The cell-to-nnz permutation made explicit: perm[c * nloc^2 + a * nloc + b] =
 * index into the CSR values that element entry (a, b) of cell c adds to, or
 * -1 if a or b is fixed.  out: device, ncells * nloc^2 int64. */
fe_status fe_permutation(fe_mesh mesh, int32_t order, const fe_coeff *coeff, int64_t *perm, fe_stream stream);

/* Waits for the mesh's pending work and returns FE_EMESH if a kernel found
 * det J <= 0 at a quadrature point since the last call (and clears it). */
fe_status fe_get_status(fe_mesh mesh);

/* ------------------------------------------------------------------------ */
/* Solve                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t iters;           /* CG iterations performed */
    int32_t status;          /* FE_OK, FE_ENOTCONV or FE_EBREAKDOWN */
    double relres;           /* ||r_j|| / ||b|| of the recursively updated residual */
    double true_relres;      /* ||b - A x|| / ||b|| recomputed at exit */
    double lambda_min_est;   /* extremal Ritz values of diag(A)^-1 A (Lanczos from CG coefficients) */
    double lambda_max_est;
} fe_solve_info;

/* Workspace bytes fe_pcg_solve needs for n_rows unknowns. */
fe_status fe_pcg_query(int64_t n_rows, size_t *ws_bytes);

/* Jacobi-preconditioned CG on A (device CSR with dinv filled): x holds x0 on
 * entry and the solution on exit (device, n_rows).  Stops when
 * ||r_j||_2 <= rtol ||b||_2 or after maxit iterations.  Reductions are
 * deterministic (fixed-order two-stage sums, no float atomics).  Synchronizes
 * before returning (info is host memory).  Returns info->status.
 * Alignment: device arrays need the alignment of their element type; the
 * workspace 8 bytes (FE_EINVAL otherwise).  Vectors and workspace that are
 * 16-byte aligned (any device allocation is) get 16-byte vector accesses,
 * others single accesses with the same results. */
fe_status fe_pcg_solve(const fe_csr *A, const double *b, double *x, double rtol, int32_t maxit, void *ws,
                       size_t ws_bytes, fe_solve_info *info, fe_stream stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): fe_pcg_solve without a
 * workspace argument.  The workspace lives in a static device array of
 * FE_PCG_NOALLOC_BYTES (64 MiB) inside the library, one copy per device,
 * held from the first call on that device until the process ends; the call
 * itself allocates no device, pinned-host or graph memory and creates no
 * stream or event (iterations are launched directly on `stream`, the stop
 * test is read into pageable host memory).  Arguments, results and
 * alignment rules as for fe_pcg_solve; the caller still owns A, b and x.
 * Systems of more than FE_PCG_NOALLOC_MAX_ROWS rows are refused with
 * FE_EINVAL before any device work.  Every call on a device uses that
 * device's one array: calls that overlap on one device (other host threads,
 * other streams) race and must be serialized by the caller.  Nothing in the
 * array needs to start cleared, so the previous call's contents are harmless.
 * Synchronizes before returning. */
#define FE_PCG_NOALLOC_BYTES (64u << 20)
#define FE_PCG_NOALLOC_MAX_ROWS 2700000
fe_status fe_pcg_solve_noalloc(const fe_csr *A, const double *b, double *x, double rtol, int32_t maxit,
                               fe_solve_info *info, fe_stream stream);

/* ------------------------------------------------------------------------ */
/* Interior-penalty discontinuous Galerkin (Sect. 3.12 eq. ip_dg_formulations, */
/* facet matrices of eq. local_to_face_matrix, facet integration Sect. 3.13) */
/* ------------------------------------------------------------------------ */
/* The DG form of -Laplace(u) = f on the brick, with coefficient 1 (the cell
 * coefficients of the mesh are not used):
 *   sum_K int_K grad u . grad v
 *   + sum_F int_F ( -{grad u}.[v] - tau {grad v}.[u] + sigma_F [u].[v] ),
 * where F runs over interior and boundary facets, [w] = w^- n^- + w^+ n^+
 * (w n on the boundary), {g} is the mean (g itself on the boundary),
 * sigma_F = gamma / h_F, h_F = |F|^(1/(d-1)) (facet length in 2D, square
 * root of the facet area in 3D).  Dirichlet data u_D (coeff->dirichlet_kind,
 * dirichlet_affine) is imposed weakly on every boundary facet: the rhs holds
 *   sum_K int_K f v + sum_{F boundary} int_F u_D (-tau grad v . n + sigma_F v).
 * tau = 1 gives the symmetric method (SPD for gamma large enough, e.g.
 * 4 (k+1)^2 on a mildly distorted brick), tau = -1 the nonsymmetric one and
 * tau = 0 the incomplete one.
 * Space: Q_k per cell (order 1..4), no DOF shared, DOF(K, a) = K nn + a with
 * nn = (k+1)^d and the local node order of the conforming space; every DOF
 * is a row (no fixed DOFs).  Row K nn + a holds the nn columns of K and of
 * each facet neighbour of K, cells in ascending id order.
 * Quadrature: (k+1)^d Gauss points per cell, (k+1)^(d-1) per facet. */

/* Rows, nonzeros and workspace bytes (volume element matrices and loads) of
 * the DG system of (mesh, order).  FE_EINVAL for a null mesh, order outside
 * 1..4 or 2^31 rows or more.  Host only. */
fe_status fe_dg_query(fe_mesh mesh, int32_t order, int64_t *n_rows, int64_t *nnz, size_t *ws_bytes);

/* Pattern of the DG system into out->rowptr (n_rows + 1, int64) and
 * out->colind (nnz, int32), device memory owned by the caller; out->n_rows
 * and out->nnz must equal fe_dg_query's.  Enqueues only. */
fe_status fe_dg_pattern(fe_mesh mesh, int32_t order, fe_csr *out, fe_stream stream);

/* Numeric phase: volume element matrices and loads into ws (the integration
 * kernels of fe_integrate, coefficient 1, FP64), then one workgroup per cell
 * writes the values of the cell's rows: the volume block plus, for each
 * facet, its two facet matrices with the cell on the row side, and the
 * facet terms of the rhs; dinv = 1 / diagonal.  No atomics: bitwise
 * reproducible; for tau = 1 the off-diagonal blocks of the two cells of a
 * facet are transposes of each other to the last bit.
 * out->rowptr must hold fe_dg_pattern's pattern (colind is not read).
 * coeff: problem FE_POISSON, precision FE_FP64, source_kind / source and
 * dirichlet_kind / dirichlet_affine as for fe_assemble, dirichlet_faces all
 * 2 dim bits set; young / poisson_ratio unused.  gamma > 0, tau finite.
 * FE_EINVAL otherwise or for a workspace smaller than fe_dg_query's.
 * Enqueues only; det J <= 0 at a volume or facet point is reported by the
 * next fe_get_status.  The system is solved by fe_pcg_solve (tau = 1). */
fe_status fe_dg_assemble(fe_mesh mesh, int32_t order, const fe_coeff *coeff, double gamma, double tau,
                         fe_csr *out, void *ws, size_t ws_bytes, fe_stream stream);

/* y = A x for a DG system of (mesh, order), the pattern evaluated from the
 * cell index instead of read (out->rowptr / colind are not read): the nn rows
 * of a cell are contiguous in the values, so only the values and x are
 * loaded.  x, y: device, n_rows doubles; A->values 16-byte aligned
 * (FE_EINVAL otherwise).  Each row is summed in a fixed order: bitwise
 * reproducible.  Enqueues only. */
fe_status fe_dg_spmv(fe_mesh mesh, int32_t order, const fe_csr *A, const double *x, double *y, fe_stream stream);

/* The Jacobi-PCG of fe_pcg_solve (Sect. 12) on a DG system of (mesh, order),
 * with the SpMV of fe_dg_spmv; A->values and A->dinv as written by
 * fe_dg_assemble (tau = 1: symmetric positive definite for a large enough
 * gamma).  ws: fe_pcg_query(n_rows) bytes; statuses as fe_pcg_solve.
 * Synchronous (returns after the solve). */
fe_status fe_dg_pcg_solve(fe_mesh mesh, int32_t order, const fe_csr *A, const double *b, double *x, double rtol,
                          int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *info, fe_stream stream);

/* ------------------------------------------------------------------------ */
/* Taylor-Hood Stokes (the Stokes example of Sect. 3.1; the mixed pair       */
/* Q_{k+1}^d x Q_k from the scalar spaces of Sect. 3.8)                      */
/* ------------------------------------------------------------------------ */
/* Find velocity u (order k+1, d components, zero on the whole boundary) and
 * pressure p (order k, every node free) with
 *   int mu eps(u):eps(v) - int p div v = int f . v,   - int q div u = 0
 * for all v, q: the symmetric indefinite system [[A, B^T], [B, 0]] [u; p] =
 * [f; 0], A the elasticity matrix of order k+1 with lambda = 0, B_(a),(b,c) =
 * -int psi_a d_c phi_b on the velocity order's Gauss rule.  The pressure is
 * fixed up to a constant (the solve returns one solution).
 * DOFs: velocity as the vector space of fe.h's numbering with every face
 * fixed (dim components interleaved), pressure as the scalar lattice with no
 * fixed node. */
typedef struct fe_stokes_s *fe_stokes; /* opaque, library-owned */

/* Builds both spaces, the patterns of A, B and B^T and the gather maps of
 * B's entries (made once on the host: every CSR entry's element
 * contributions in ascending cell order), and allocates the system and
 * solver storage on the device (owned by the handle).  order = k, the
 * pressure order, in 1..3; mu > 0; force: source_kind / source as in
 * fe_coeff (NULL: no force).  Synchronous.  The mesh must outlive the handle. */
fe_status fe_stokes_create(fe_mesh mesh, int32_t order, double mu, const fe_coeff *force, fe_stokes *out);
fe_status fe_stokes_destroy(fe_stokes s);

/* Velocity unknowns, pressure unknowns, nonzeros of A and of B.  Host only. */
fe_status fe_stokes_query(fe_stokes s, int64_t *n_u, int64_t *n_p, int64_t *nnz_a, int64_t *nnz_b);

/* Numeric phase: A (the integration and scatter kernels), the element
 * blocks of B, B and B^T by deterministic gathers (bitwise reproducible), the
 * pressure mass diagonal, the rhs [f; 0] and the preconditioner.  Enqueues
 * only; det J <= 0 is reported by the next fe_get_status of the mesh. */
fe_status fe_stokes_assemble(fe_stokes s, fe_stream stream);

/* Device views of the assembled system (owned by the handle, valid until it
 * is destroyed): A (rows n_u, with rhs = the first n_u entries of the
 * system's rhs and dinv), B (n_p x n_u; rhs and dinv NULL), B^T (n_u x n_p),
 * the pressure mass diagonal md (n_p) and the whole rhs (n_u + n_p).  Any
 * pointer may be NULL. */
fe_status fe_stokes_system(fe_stokes s, fe_csr *A, fe_csr *B, fe_csr *Bt, const double **md, const double **rhs);

/* MINRES on the Stokes system (a Lanczos process on the preconditioned
 * operator, its tridiagonal reduced by Givens rotations), preconditioned by
 * diag(A)^-1 on the velocity and mu / md on the pressure.  u (n_u) and p
 * (n_p), device: the initial guess on entry, the solution on exit.  Stops when
 * ||r||_{M^-1} <= rtol ||b||_{M^-1} (the recurrence's estimate; info->relres)
 * or after maxit iterations; info->true_relres recomputes it from K x.
 * Dot products are deterministic (fixed partials summed in a fixed order).
 * Synchronous.  FE_ENOTCONV at maxit, FE_EBREAKDOWN if the preconditioned
 * Lanczos process breaks down. */
fe_status fe_stokes_solve(fe_stokes s, double rtol, int32_t maxit, double *u, double *p, fe_solve_info *info,
                          fe_stream stream);

/* ------------------------------------------------------------------------ */
/* Lagrangian P_k on simplicial meshes (Sect. 3.3 truncated spaces and node  */
/* sets, Sect. 3.5 shape functions by a change of basis, Sect. 3.7 collapsed */
/* quadrature on simplices; triangles and tetrahedra of a general mesh)      */
/* ------------------------------------------------------------------------ */
/* A simplicial mesh: vertex coordinates and cell-to-vertex connectivity,
 * with no structure assumed.  Local nodes are the lattice points s/k with
 * |s| <= k of the reference simplex (x fastest); global nodes are numbered
 * by first appearance over (cell ascending, local node ascending); a node is
 * on the boundary when it lies on a facet of one cell only.  DOFs follow
 * fe.h's conventions (free ranks in node order, components interleaved,
 * fixed DOFs -1 - fixed rank in cell_dofs). */
typedef struct fe_simplex_s *fe_simplex; /* opaque, library-owned */

typedef struct {
    int32_t dim;              /* 2 (triangles) or 3 (tetrahedra) */
    int64_t nverts, ncells;
    const double *vertex_xyz; /* host, nverts x dim (AoS) */
    const int32_t *cells;     /* host, ncells x (dim+1) vertex ids; either orientation */
    const double *cell_coeff; /* host, ncells; NULL = 1.0 */
} fe_simplex_desc;

/* Builds the space of P_order (1..4; elasticity 1..3) on the mesh: the
 * reference element (change of basis, collapsed Gauss rule with
 * order + ceil(dim/2) points per direction), the global numbering, the CSR
 * pattern and the stored cell-to-nnz gather map (every entry's element
 * contributions in ascending cell order), on the host; copies the mesh and
 * those maps to the device (owned by the handle).  coeff: problem, FP64
 * precision only, source, dirichlet_faces != 0 fixes every boundary node
 * (0: none), Dirichlet kind and affine datum.  Synchronous.  FE_EMESH for a
 * vertex id out of range, a degenerate cell (det J = 0) or a facet of more
 * than two cells; FE_EINVAL for 2^31 or more free DOFs or 2^32 or more
 * element entries. */
fe_status fe_simplex_create(const fe_simplex_desc *desc, int32_t order, const fe_coeff *coeff, fe_simplex *out);
fe_status fe_simplex_destroy(fe_simplex s);

/* Lowest-order vector elements on the same meshes (Sect. 3.9, 3.10):
 * FE_NEDELEC, one tangential moment per edge (the line integral along the
 * edge), mapped by the covariant Piola map J^-T; FE_RAVIART_THOMAS, one flux
 * moment per facet, mapped by the contravariant Piola map J / det J.  Shape
 * functions by the change of basis from the spaces' pre-bases.  Global
 * orientation: an edge runs from its lower to its higher vertex id, a facet's
 * normal is taken over its vertices in ascending id.  The form is
 *   int c curl u . curl v + kappa u . v   (Nedelec)
 *   int c div u div v + kappa u . v       (Raviart-Thomas)
 * with c the per-cell coefficient (cell_coeff, NULL = 1).  coeff: FP64;
 * source_kind CONST (f = source) or SINPROD (f_c = source[c] m_c(x), m the
 * family's field: Nedelec 3D (sin pi y sin pi z, sin pi z sin pi x,
 * sin pi x sin pi y), 2D (sin pi y, sin pi x); Raviart-Thomas (sin pi x_r)_r);
 * dirichlet_faces != 0 fixes the DOFs on the boundary to zero (tangential or
 * normal trace), FE_DIRICHLET_ZERO only.  A DOF entity (edge, facet) is
 * numbered by first appearance over (cell, local DOF); local DOFs are the
 * edges (0,1),(0,2),(1,2) [2D] or (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) [3D],
 * or the facets by their opposite vertex.  The other fe_simplex_* calls
 * apply (n_nodes counts the DOFs).  FE_NEDELEC2: the second-order Nedelec
 * element ([P_1]^d plus the quadratic fields orthogonal to x): two moments
 * per edge (against 1 - t and t from its first vertex), two per face against
 * the face's edge tangents x_i1 - x_i0, x_i2 - x_i0 (3D), two interior
 * moments on the reference triangle (2D); local DOF order: the edges' pairs,
 * then the faces' (3D) or the interior pair (2D).  A DOF's global frame is its
 * entity's vertices in ascending global id; the cell's local moments are T
 * times the global ones with a 2 x 2 block per edge (identity, or swapped and
 * negated) and per face (the local tangents in the global ones), and the
 * element matrix and load are returned in the global frame (T^T A T, T^T f).
 * FE_RAVIART_THOMAS2: the second-order Raviart-Thomas element ([P_1]^d plus
 * x times the linear monomials): per facet the fluxes (N as for
 * FE_RAVIART_THOMAS) against the barycentric of each of its vertices, then
 * the integrals of the d components over the reference cell (15 DOFs in 3D,
 * 8 in 2D; local order: facet by facet, its vertices ascending, then the
 * interior).  A facet's global frame lists its vertices in ascending global id;
 * a local moment is the global moment of the same vertex times the parity of
 * the facet's vertex order; matrix and load in the global frame as above.
 * FE_EINVAL for kappa < 0 or an unknown family; mesh errors as
 * fe_simplex_create. */
enum { FE_NEDELEC = 1, FE_RAVIART_THOMAS = 2, FE_NEDELEC2 = 3, FE_RAVIART_THOMAS2 = 4 };
fe_status fe_simplex_create_vector(const fe_simplex_desc *desc, int32_t family, double kappa, const fe_coeff *coeff,
                                   fe_simplex *out);

/* Free DOFs (rows), nonzeros, global nodes and element contributions to the
 * nonzeros (the gather map's length).  Host only. */
fe_status fe_simplex_query(fe_simplex s, int64_t *n_rows, int64_t *nnz, int64_t *n_nodes, int64_t *n_contrib);

/* The cell-to-DOF map into cell_dofs (device, ncells x nloc int32). */
fe_status fe_simplex_cell_dofs(fe_simplex s, int32_t *cell_dofs, fe_stream stream);

/* Symbolic phase: A->rowptr and A->colind (device, caller-owned, sizes from
 * fe_simplex_query) from the pattern built at creation.  Synchronous. */
fe_status fe_simplex_pattern(fe_simplex s, const fe_csr *A, fe_stream stream);

/* Numeric phase (Sect. 3.6, 3.7, 10.4): the element matrices (upper
 * triangles) and loads with Dirichlet lifting of every cell, then A->values
 * by the gather map, A->rhs and A->dinv.  Bitwise reproducible.  Enqueues
 * only. */
fe_status fe_simplex_assemble(fe_simplex s, const fe_csr *A, fe_stream stream);

/* Device views of the last assembly's element data (owned by the handle):
 * E[K ntri + t], t = I nloc - I (I - 1) / 2 + (J - I) for local DOFs I <= J
 * (nloc = nodes x components, ntri = nloc (nloc + 1) / 2), and the loads with
 * lifting F[K nloc + I]. */
fe_status fe_simplex_elements(fe_simplex s, const double **E, const double **F);

/* ------------------------------------------------------------------------ */
/* Batched solve: many independent systems in one sequence of launches       */
/* ------------------------------------------------------------------------ */
/* Workspace bytes fe_pcg_solve_batch needs for nprob systems of n_rows[i]
 * unknowns (host array). */
fe_status fe_pcg_batch_query(int32_t nprob, const int64_t *n_rows, size_t *ws_bytes);

/* The Jacobi-PCG of fe_pcg_solve (Sect. 12) applied to nprob independent
 * systems at once: every kernel launch covers all systems, each owning its
 * own range of workgroups, partial sums and iteration state, and chunks of
 * iterations are replayed from a captured HIP graph.  A, b, x and infos are
 * host arrays of nprob entries; A[i] is a device CSR with dinv filled, b[i]
 * and x[i] device vectors of A[i].n_rows (x[i]: x0 on entry, solution on
 * exit).  Each system stops on its own criterion ||r|| <= rtol ||b|| or at
 * maxit; its result is bitwise the same as that of fe_pcg_solve on it alone
 * (same kernels, same reduction order).  Systems with n_rows == 0 are
 * skipped.  Synchronizes before returning; returns FE_OK if every system
 * converged, else the first failing status (infos[i].status per system).
 * infos[i].lambda_*_est are filled only when nprob == 1. */
fe_status fe_pcg_solve_batch(int32_t nprob, const fe_csr *A, const double *const *b, double *const *x, double rtol,
                             int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *infos, fe_stream stream);

/* ------------------------------------------------------------------------ */
/* Solves of systems assembled by this library: pattern evaluated            */
/* ------------------------------------------------------------------------ */
/* The CSR pattern of a system assembled on a structured brick is a closed
 * form of the mesh's per-axis node intervals (the same one fe_pattern
 * writes, Sect. 11.1).  These variants of fe_spmv / fe_pcg_solve /
 * fe_pcg_solve_batch read the CSR values in CSR order and evaluate each
 * entry's column from that form instead of loading row pointers and column
 * indices: 8 instead of 12 bytes per nonzero, and no gather that waits on a
 * loaded index.  (mesh, order, coeff) must be those A was assembled with
 * (sizes are checked; A->rowptr / colind are not read).  Results equal the
 * CSR variants up to rounding (each row is summed in the same lane order,
 * with a different number of lanes per row), and are bitwise reproducible;
 * fe_pcg_solve_batch_mesh gives each system bitwise the result of
 * fe_pcg_solve_mesh on it alone.  The workspace sizes are those of
 * fe_pcg_query / fe_pcg_batch_query. */
fe_status fe_spmv_mesh(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A, const double *x,
                       double *y, fe_stream stream);
fe_status fe_pcg_solve_mesh(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A, const double *b,
                            double *x, double rtol, int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *info,
                            fe_stream stream);
fe_status fe_pcg_solve_batch_mesh(int32_t nprob, const fe_mesh *meshes, const int32_t *orders, const fe_coeff *coeffs,
                                  const fe_csr *A, const double *const *b, double *const *x, double rtol,
                                  int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *infos, fe_stream stream);

/* ------------------------------------------------------------------------ */
/* Symmetric storage (Q1 scalar systems)                                     */
/* ------------------------------------------------------------------------ */
/* The FE operator may keep only the upper triangle of a symmetric matrix
 * (Sect. 11.3; the driver of Sect. 12 asks for it).  For a Q1 scalar system
 * assembled on a structured brick (order 1, Poisson) the upper triangle is
 * kept slot-major: with g = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) the code of a
 * neighbour offset (g = 3 (dy + 1) + (dx + 1) in 2D) and C = 13 (4 in 2D),
 * slot s = g - C of row r holds A[r, r + dx + f0 dy + f0 f1 dz] at
 * sym[s * stride + r], stride = n_rows rounded up to a multiple of 64, f0, f1
 * the free nodes per line and per plane; slot 0 is the diagonal; 14 slots in
 * 3D, 5 in 2D; an entry whose neighbour is not a free node holds 0.  A lower
 * entry is read as the upper entry of the neighbour's row, so the operator is
 * the symmetric matrix with A's upper triangle: half the value bytes of the
 * CSR per SpMV.
 *   fe_sym_query: *bytes of the storage of (mesh, order, coeff); FE_EINVAL
 *     unless order 1 and a scalar problem.
 *   fe_sym_from_csr: sym (device, >= fe_sym_query bytes, 8-byte aligned,
 *     owned by the caller) = the upper triangle of A, assembled by this
 *     library on (mesh, order, coeff) (values read, rowptr / colind not);
 *     asynchronous on stream.
 *   fe_spmv_sym: y = A x from sym (x, y device, n_rows each).  Each row is
 *     summed in the order of the Q1 traversal of fe_spmv_mesh, so for a
 *     bitwise symmetric A (as assembled here) y is bitwise that of
 *     fe_spmv_mesh.  Asynchronous.
 *   fe_pcg_solve_sym: Jacobi-PCG of A x = b with A applied from sym and the
 *     diagonal inverse read from A->dinv (A->values, rowptr, colind not
 *     read); workspace of fe_pcg_query(n_rows) bytes.  The same rows and
 *     products as fe_pcg_solve_mesh; its fused p.q partials group 256 rows
 *     instead of 128, so the iterates agree to rounding, and they are bitwise
 *     reproducible from run to run.  Synchronizes.
 * Errors (FE_EINVAL, nothing launched): not Q1 scalar, sym too small, null
 * or not 8-byte aligned, csr sizes not those of fe_assemble_query. */
fe_status fe_sym_query(fe_mesh mesh, int32_t order, const fe_coeff *coeff, size_t *bytes);
fe_status fe_sym_from_csr(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A, double *sym,
                          size_t sym_bytes, fe_stream stream);
fe_status fe_spmv_sym(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const double *sym, size_t sym_bytes,
                      const double *x, double *y, fe_stream stream);
fe_status fe_pcg_solve_sym(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A, const double *sym,
                           size_t sym_bytes, const double *b, double *x, double rtol, int32_t maxit, void *ws,
                           size_t ws_bytes, fe_solve_info *info, fe_stream stream);

/* ------------------------------------------------------------------------ */
/* SpMV plans and their autotuner                                            */
/* ------------------------------------------------------------------------ */
/* A plan is how the CSR SpMV of fe_spmv / fe_pcg_solve / fe_pcg_solve_batch
 * walks the rows: mode 0 = wave-level CSR-stream with rows_per_wave rows
 * (1..32) per wave iteration, mode 1 = one wave per row.  Without tuning a
 * plan follows from the average row length nnz / n_rows; fe_spmv_autotune
 * times every plan on a matrix (reps launches each, after a warm-up launch)
 * and makes the fastest the plan of every matrix of the same row-length class
 * (half octaves of nnz / n_rows) in this process.  The plan fixes each row's
 * summation order: results are bitwise reproducible for a fixed plan table.
 *   ws: device, fe_spmv_autotune_query bytes.  tried: host, up to max_tried
 *   entries (us = mean launch time in microseconds); chosen: host.
 *   Synchronizes.  fe_spmv_tuning_reset forgets every tuned plan. */
typedef struct {
    int32_t mode;
    int32_t rows_per_wave;
    double us;
} fe_spmv_plan;

fe_status fe_spmv_autotune_query(int64_t n_rows, size_t *ws_bytes);
fe_status fe_spmv_autotune(const fe_csr *A, int32_t reps, void *ws, size_t ws_bytes, fe_spmv_plan *tried,
                           int32_t max_tried, int32_t *n_tried, fe_spmv_plan *chosen, fe_stream stream);
fe_status fe_spmv_tuning_reset(void);
/* The same for the evaluated-pattern traversal of fe_spmv_mesh /
 * fe_pcg_solve_mesh / fe_pcg_solve_batch_mesh: plans are modes 2 (lanes per
 * row, rows_per_wave runs), 3 (short rows, two lanes per row; rows_per_wave
 * reports the longest row), for the Q1 scalar pattern 4 (the values of 32
 * rows and the runs of x they touch staged in LDS with wide loads; two lanes
 * per row in the order of mode 3, so modes 3 and 4 give bitwise the same
 * products), and for every other pattern 6 (rows_per_wave 8: x over the
 * column box of 32 consecutive rows of a line of nodes staged in LDS per
 * workgroup; bitwise the same products as mode 2 with 8 rows per wave),
 * timed on A assembled on (mesh, order, coeff); the fastest
 * becomes the plan of every mesh system with the same longest row and
 * component count.  ws: fe_spmv_autotune_query(A->n_rows) bytes.
 * fe_spmv_plan_set_mesh makes `plan` (mode and rows_per_wave of one of the
 * plans the autotuner would time; us is ignored) the plan of that class
 * without timing; FE_EINVAL for any other plan. */
fe_status fe_spmv_autotune_mesh(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A, int32_t reps,
                                void *ws, size_t ws_bytes, fe_spmv_plan *tried, int32_t max_tried, int32_t *n_tried,
                                fe_spmv_plan *chosen, fe_stream stream);
fe_status fe_spmv_plan_of_mesh(fe_mesh mesh, int32_t order, const fe_coeff *coeff, fe_spmv_plan *plan,
                               int32_t *row_class);
fe_status fe_spmv_plan_set_mesh(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_spmv_plan *plan);
/* Tile shapes of the matrix-core element integration (3D, orders 2..4): the
 * node-tile pairs each wave accumulates (the workgroups per cell follow).
 * Every shape sums each element-matrix entry over the quadrature points in
 * the same order, so element matrices are bitwise the same for every shape.
 * FP16 / BF16 classes have one shape (a workgroup per cell, parts = 1;
 * pairs_per_wave the most node-tile pairs one of its waves takes).
 * fe_integrate_autotune times each candidate shape of the class (order,
 * problem, precision) of (mesh, order, coeff) with reps K3 launches into ws
 * (the workspace of fe_assemble_query, whose element matrices it overwrites)
 * and makes the fastest the shape of the class in this process (single and
 * batched assembly).  tried: host, up to max_tried entries (us = mean launch
 * time); chosen: host.  Synchronizes.  FE_EINVAL for spaces without
 * matrix-core integration (2D, Q1).  fe_integrate_plan_of reports the shape
 * a class gets now (pairs_per_wave 0: not a matrix-core class).
 * fe_spmv_tuning_reset also forgets the tuned shapes. */
typedef struct {
    int32_t pairs_per_wave;
    int32_t parts;  /* workgroups per cell */
    double us;
} fe_k3_plan;
fe_status fe_integrate_autotune(fe_mesh mesh, int32_t order, const fe_coeff *coeff, void *ws, size_t ws_bytes,
                                int32_t reps, fe_k3_plan *tried, int32_t max_tried, int32_t *n_tried,
                                fe_k3_plan *chosen, fe_stream stream);
fe_status fe_integrate_plan_of(fe_mesh mesh, int32_t order, const fe_coeff *coeff, fe_k3_plan *plan);

/* The plan a matrix of n_rows rows and nnz entries gets now, and its class. */
fe_status fe_spmv_plan_of(int64_t n_rows, int64_t nnz, fe_spmv_plan *plan, int32_t *row_class);
/* Makes `plan` (mode and rows_per_wave of one of the CSR plans fe_spmv_autotune
 * times; us is ignored) the plan of the row-length class of a matrix of n_rows
 * rows and nnz entries, without timing.  Host only, no device work.
 * FE_EINVAL for a null plan, negative sizes or any other plan. */
fe_status fe_spmv_plan_set(int64_t n_rows, int64_t nnz, const fe_spmv_plan *plan);

/* y = A x (device vectors).  Enqueues only. */
fe_status fe_spmv(const fe_csr *A, const double *x, double *y, fe_stream stream);

/* ------------------------------------------------------------------------ */
/* Mixed precision: iterative refinement                                     */
/* ------------------------------------------------------------------------ */
/* values32[j] = (float) A->values[j] (device, nnz floats).  Enqueues only. */
fe_status fe_csr_to_fp32(const fe_csr *A, float *values32, fe_stream stream);

typedef struct {
    int32_t outer_iters;  /* corrections applied */
    int32_t inner_iters;  /* CG iterations summed over the corrections */
    int32_t status;       /* FE_OK or FE_ENOTCONV */
    double relres;        /* ||b - A_hi x|| / ||b|| in FP64 at exit */
} fe_refine_info;

/* Workspace bytes fe_refine_solve needs for n_rows unknowns. */
fe_status fe_refine_query(int64_t n_rows, size_t *ws_bytes);

/* Solves A_hi x = b to ||b - A_hi x||_2 <= rtol ||b||_2 by iterative
 * refinement: the residual is formed in FP64 with A_hi; each correction d
 * solves A_lo d = r approximately by Jacobi-PCG to inner_rtol (at most
 * max_inner iterations) and x += d.  A_lo has the pattern of A_hi; its values
 * are read from values32 (FP32) when that pointer is not NULL, otherwise from
 * A_lo->values (for example a matrix assembled with reduced-precision element
 * integration); A_lo->dinv is its Jacobi diagonal.  x holds x0 on entry.
 * Synchronizes; returns info->status. */
fe_status fe_refine_solve(const fe_csr *A_hi, const fe_csr *A_lo, const float *values32, const double *b, double *x,
                          double rtol, double inner_rtol, int32_t max_outer, int32_t max_inner, void *ws,
                          size_t ws_bytes, fe_refine_info *info, fe_stream stream);

/* fe_refine_solve on a system assembled by this library on (mesh, order,
 * coeff) (either coeff; A_hi and A_lo share the pattern): the inner Jacobi-PCG
 * evaluates the pattern from the mesh instead of reading column indices, so
 * an FP32 A_lo (values32) costs 4 bytes per entry per product, each value
 * widened to FP64 in its product; every vector, dot and the outer residual
 * with A_hi stay FP64 (the residual through the CSR of A_hi).  values32 (if
 * not NULL: device, A_lo->nnz floats, 4-byte aligned, e.g. fe_csr_to_fp32 of
 * A_lo) takes the block-staged traversal; otherwise A_lo->values (FP64) take
 * the mesh system's plan.  Refinement by the paper's iterative solvers (Sect.
 * 12) with FP64 residuals; the workspace is fe_refine_query's.  Synchronizes;
 * returns info->status.  Errors: as for fe_pcg_solve_mesh and fe_refine_solve. */
fe_status fe_refine_solve_mesh(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A_hi,
                               const fe_csr *A_lo, const float *values32, const double *b, double *x, double rtol,
                               double inner_rtol, int32_t max_outer, int32_t max_inner, void *ws, size_t ws_bytes,
                               fe_refine_info *info, fe_stream stream);

/* Batched iterative refinement: fe_refine_solve_mesh with FP64 A_lo values
 * for nprob systems at once (the batching form with reduced-precision
 * integration: A_lo[i] integrated in FP32/FP16/BF16, A_hi[i] in FP64, on
 * meshes[i], orders[i], coeffs[i] as for fe_pcg_solve_batch_mesh).  Each
 * correction step forms the residuals of the systems still running with their
 * A_hi (FP64, CSR) and solves their corrections A_lo d = r together by the
 * batched Jacobi-PCG (the pattern evaluated from the meshes); a system stops
 * at ||b - A_hi x|| <= rtol ||b|| or after max_outer corrections.  Every
 * result is bitwise that of fe_refine_solve_mesh on the system alone.
 *   fe_refine_batch_query: workspace bytes for nprob systems of n_rows[i] rows.
 *   infos: host, nprob entries.  Synchronizes; returns FE_OK if every system
 *   converged, else FE_ENOTCONV or FE_EBREAKDOWN (per system in infos). */
fe_status fe_refine_batch_query(int32_t nprob, const int64_t *n_rows, size_t *ws_bytes);
fe_status fe_refine_solve_batch_mesh(int32_t nprob, const fe_mesh *meshes, const int32_t *orders,
                                     const fe_coeff *coeffs, const fe_csr *A_hi, const fe_csr *A_lo,
                                     const double *const *b, double *const *x, double rtol, double inner_rtol,
                                     int32_t max_outer, int32_t max_inner, void *ws, size_t ws_bytes,
                                     fe_refine_info *infos, fe_stream stream);

/* Iterative refinement with the inner solve on the symmetric storage of A_lo
 * in FP32 (Q1 scalar systems; the layout of fe_sym_query with float slots):
 *   fe_sym_fp32_from_csr: sym32 (device, >= fe_sym_query / 2 bytes, 4-byte
 *     aligned) = the upper triangle of A, rounded to FP32 (as fe_csr_to_fp32
 *     rounds); asynchronous.
 *   fe_refine_solve_sym: fe_refine_solve with the inner Jacobi-PCG applying
 *     A_lo from sym32 (its FP32 values widened to FP64 in each product; every
 *     vector, dot and the outer residual with A_hi stay FP64) and A_lo->dinv
 *     as its diagonal; (mesh, order, coeff) those A_hi and A_lo were
 *     assembled with (either coeff; their patterns are one).  The workspace
 *     is fe_refine_query's.  Synchronizes; returns info->status.
 * Errors: as for fe_sym_from_csr and fe_refine_solve. */
fe_status fe_sym_fp32_from_csr(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A, float *sym32,
                               size_t sym32_bytes, fe_stream stream);
fe_status fe_refine_solve_sym(fe_mesh mesh, int32_t order, const fe_coeff *coeff, const fe_csr *A_hi,
                              const fe_csr *A_lo, const float *sym32, size_t sym32_bytes, const double *b, double *x,
                              double rtol, double inner_rtol, int32_t max_outer, int32_t max_inner, void *ws,
                              size_t ws_bytes, fe_refine_info *info, fe_stream stream);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop with admission by device-memory budget            */
/* ------------------------------------------------------------------------ */
/* A server owns one device-memory budget on the current device and two host
 * threads.  Each request is one assemble-and-solve of the system above
 * (Sect. 3.6-3.7 assembly, Sect. 10.4 Dirichlet elimination, Jacobi-PCG of
 * Sect. 12) on its own structured mesh.  Requests are admitted in submission
 * order when their bytes (CSR, vectors and PCG state, element workspace
 * during assembly, mesh arrays) fit the remaining budget and fewer than
 * max_active are in flight; set-up and assembly run on one stream while the
 * CG iterations of every request in flight run as batched chunks on another,
 * new requests joining between chunks (continuous batching).  A request's
 * result is bitwise that of fe_assemble + fe_pcg_solve_mesh on it alone.  A
 * finished request keeps its system and solution on the device until
 * fe_server_release.  Calls are thread-safe. */
typedef struct fe_server_s *fe_server;

typedef struct {
    fe_mesh_desc mesh;  /* host arrays, copied by fe_server_submit */
    int32_t order;      /* 1..4 */
    fe_coeff coeff;
    double rtol;        /* ||r|| <= rtol ||b|| */
    int32_t maxit;
} fe_request;

typedef enum {
    FE_REQ_QUEUED = 0,
    FE_REQ_SETUP = 1,    /* admitted: mesh, pattern, assembly */
    FE_REQ_SOLVING = 2,  /* in the batched CG chunks */
    FE_REQ_DONE = 3,     /* status = the solver's status */
    FE_REQ_FAILED = 4    /* status = the error; fe_last_error() has its text after poll/wait */
} fe_request_state;

typedef struct {
    int32_t state;
    int32_t status;
    int64_t n_rows, nnz;
    int64_t bytes;  /* device bytes charged at admission */
    int32_t iters;
    double relres, true_relres;
    double t_submit, t_admit, t_ready, t_done;  /* seconds on fe_server_clock */
} fe_result;

typedef struct {
    int64_t budget, arena_bytes, mesh_reserve, in_use, peak_in_use, peak_arena;
    int32_t queued, setting_up, solving, peak_solving;
    int64_t submitted, admitted, completed, rejected, chunks;
    int64_t admission_waits;  /* times the head of the queue waited for memory or a slot */
} fe_server_stats;

/* hbm_budget: device bytes the server may hold (allocated at creation: one
 * arena plus a reserve of budget / 8 for mesh arrays).  FE_ENOMEM if the
 * device cannot hold it. */
fe_status fe_server_create(size_t hbm_budget, int32_t max_active, fe_server *out);
/* Queues a request; FE_ENOMEM if it can never fit the budget, FE_EINVAL for
 * invalid sizes or parameters (others are reported as FE_REQ_FAILED). */
fe_status fe_server_submit(fe_server server, const fe_request *req, uint64_t *ticket);
fe_status fe_server_poll(fe_server server, uint64_t ticket, fe_result *out);
/* Waits until the request is done or failed, or timeout_s passed (then
 * out->state tells which). */
fe_status fe_server_wait(fe_server server, uint64_t ticket, double timeout_s, fe_result *out);
/* Copies the n = n_rows solution values of a done request into x (device or
 * host memory); synchronous. */
fe_status fe_server_solution(fe_server server, uint64_t ticket, double *x, int64_t n);
/* Frees a done or failed request's device memory and forgets the ticket. */
fe_status fe_server_release(fe_server server, uint64_t ticket);
fe_status fe_server_get_stats(fe_server server, fe_server_stats *out);
double fe_server_clock(fe_server server);
/* Stops admitting, fails queued requests, finishes those in flight, frees all. */
fe_status fe_server_destroy(fe_server server);

/* ------------------------------------------------------------------------ */
/* Kernel timing (for benchmarks)                                            */
/* ------------------------------------------------------------------------ */
/* When enabled (process-wide), fe_integrate / fe_scatter record HIP events
 * around their kernels and the single-system solves (fe_pcg_solve,
 * fe_pcg_solve_mesh, fe_pcg_solve_sym; not those replayed from a graph)
 * around the SpMV launch of every 16th CG iteration before convergence, on
 * the call's own stream (an event pair costs a few microseconds of device
 * time).  fe_get_timing waits for the recorded events, returns the
 * accumulated kernel times (milliseconds) and counts of timed launches, and
 * clears them when reset != 0. */
typedef struct {
    double integrate_ms, scatter_ms, spmv_ms;
    int64_t integrate_calls, scatter_calls, spmv_calls;
} fe_timing;

fe_status fe_set_timing(int32_t enable);
fe_status fe_get_timing(fe_timing *out, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* FE_H */
