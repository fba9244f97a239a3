/*
 * tetmf — matrix-free Galerkin operators on unstructured tetrahedral meshes
 * for AMD Instinct MI355X (gfx950).
 *
 * The operator is the cell-by-cell evaluation of eq. (5) (continuous
 * Galerkin) and eq. (7) (SIPG discontinuous Galerkin) of Still, Fehn, Wall,
 * Kronbichler, "Matrix-Free Evaluation Strategies for Continuous and
 * Discontinuous Galerkin Discretizations on Unstructured Tetrahedral Grids"
 * (arXiv 2509.10226):
 *
 *     A(u) = sum_e G_e^T E^T D_e E G_e u   (+ sum_f G_f^T E_f^T D_f E_f G_f u)
 *
 * G_e gathers the cell's DoF values, E tabulates reference gradients (and
 * values) of the nodal basis at the quadrature points (eq. (6)), D_e applies
 * the per-point geometry J^{-1} J^{-T} |det J| w_q and the coefficient
 * kappa_q, E^T integrates against the test functions and G_e^T scatters back.
 * The bilinear forms are eq. (2) (Poisson), eq. (3) (SIPG) and the
 * Helmholtz-type form of eq. (19) (stiffness plus sigma times mass).
 *
 * Conventions shared by every entry point
 *  - Status codes: 0 = OK, > 0 = non-fatal status, < 0 = error.  No entry
 *    point throws or aborts; tetmf_last_error() describes the last failure
 *    of the calling thread.
 *  - "host" pointers are CPU memory, "device" pointers are GPU memory of the
 *    op's device.  Device buffers passed in are owned by the caller.
 *  - Work is enqueued on the given HIP stream (NULL = default stream) and
 *    returns asynchronously unless stated otherwise; only launch errors are
 *    reported by the return code.
 *  - An op is not thread-safe: concurrent calls on one op race on its
 *    internal scratch (the interface partial sums).  Use one op per stream.
 *  - Library order: the op renumbers cells for locality (a Morton order of
 *    cell centroids) and numbers DoFs by first touch in that order.
 *    tetmf_op_numbering() exports the maps back to the user's order.
 *  - Cell quadrature data (coefficients, coefficient gradients, source
 *    samples) use the library layout [ceil(n_cell / 16)][n_q][16]: library
 *    cells in tiles of 16, and the value at point q of library cell i at
 *    index ((i / 16) n_q + q) 16 + i % 16, so that one tile's data is one
 *    contiguous run (tetmf_info.n_cell_data = 16 n_q ceil(n_cell / 16)
 *    entries; the padding entries of a partly used last tile are ignored on
 *    input and written as zero by the library).  Point q of a cell is
 *    X0 + J x_q with J = [X1-X0 | X2-X0 | X3-X0] built from the cell's
 *    vertices in the user's order (vertices are never reordered).
 *  - Face quadrature data use [n_qf][n_face] with faces in canonical order
 *    (lexicographic order of the sorted global vertex triples) and point q
 *    at a + s_q (b - a) + t_q (c - a) for the sorted vertices a < b < c.
 */
#ifndef TETMF_H
#define TETMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tetmf_mesh tetmf_mesh;
typedef struct tetmf_op tetmf_op;

enum tetmf_status {
  TETMF_OK = 0,
  TETMF_NOT_CONVERGED = 1,
  TETMF_ERR_INVALID_ARGUMENT = -1,
  TETMF_ERR_DEGENERATE_CELL = -2,
  TETMF_ERR_NONCONFORMING_MESH = -3,
  TETMF_ERR_UNSUPPORTED = -4,
  TETMF_ERR_ALIAS = -5,
  TETMF_ERR_OUT_OF_MEMORY = -6,
  TETMF_ERR_DEVICE = -7
};

enum tetmf_kind { TETMF_CG = 0, TETMF_DG = 1 };
enum tetmf_bc { TETMF_NEUMANN = 0, TETMF_DIRICHLET = 1 };
/* arithmetic of the operator: FP64; FP32 (MFMA f32); BF16 operands of both
 * products with FP32 accumulation and FP32 vectors */
enum tetmf_precision { TETMF_F64 = 0, TETMF_F32 = 1, TETMF_BF16IN = 2 };
enum tetmf_ordering { TETMF_ORDER_LOCALITY = 0, TETMF_ORDER_AS_GIVEN = 1 };

/* Operator description (all host memory, copied by tetmf_op_create). */
typedef struct {
  int32_t kind;        /* tetmf_kind */
  int32_t degree;      /* polynomial degree p, 1..3 (nodal equispaced Lagrange) */
  int32_t bc;          /* CG: DIRICHLET constrains boundary DoFs (rows act as
                          identity, v_c = u_c); DG: DIRICHLET adds the mirror
                          boundary terms, NEUMANN adds none */
  int32_t precision;   /* tetmf_precision */
  int32_t ordering;    /* tetmf_ordering */
  int32_t n_q;         /* cell rule: points [n_q][3] on the reference tet  */
  const double* q_points;   /* (0,0,0),(1,0,0),(0,1,0),(0,0,1); weights sum */
  const double* q_weights;  /* to 1/6 */
  int32_t n_qf;        /* face rule (DG only): points [n_qf][2] on the      */
  const double* qf_points;  /* reference triangle (0,0),(1,0),(0,1);        */
  const double* qf_weights; /* weights sum to 1/2 */
  double sigma;        /* mass coefficient of the Helmholtz-type form (0 = Poisson) */
  double eta;          /* SIPG penalty factor: tau_F = eta (p+1)^2 |F| / min|K| */
  int32_t device;      /* HIP device ordinal */
  /* Curved cells (Sec. 3.2), CG only: NULL for straight-sided cells (the
   * affine map of each tetrahedron's vertices), or the Jacobian of each
   * cell's reference-to-physical map at each cell rule point, host
   * [n_cell][n_q][3][3] in user cell order, J[a][b] = d x_a / d xi_b.  The
   * operator then stores G_q = |det J_q| J_q^-1 J_q^-T (and |det J_q| with a
   * mass term) per point and reads it in every apply: 6 n_q (7 n_q) values
   * per cell instead of 6 (7).  The vertex mesh still defines the DoF
   * connectivity and tetmf_op_numbering's coordinates.  DG: UNSUPPORTED.
   * DEGENERATE_CELL when some |det J_q| <= 1e-12 |J_q|_F^3 or is not finite. */
  const double* q_jacobians;
  /* Components of the field (Sec. 3.2, vector-valued problems without
   * coupling between the components): 0 or 1 scalar; 3 a vector field, CG or
   * DG, in F64 or F32 only (else UNSUPPORTED).  Every vector of the operator then
   * holds the components one after another, [n_components][n_dofs], and
   * A acts on each with the same coefficient; the kappa gradient of the
   * backward is the sum over the components.  tetmf_load_vector is
   * UNSUPPORTED for vector fields. */
  int32_t n_components;
} tetmf_op_desc;

typedef struct {
  int64_t n_dofs;      /* global DoFs (CG: continuous nodes; DG: 20 n_cell at p=3) */
  int64_t n_free;      /* CG: unconstrained DoFs, numbered 0..n_free-1 */
  int64_t n_cell, n_face, n_interior_face;
  int32_t n_q, n_qf, n_dof_cell, precision;
  int64_t n_blocks;    /* CG: cell blocks of one workgroup */
  int64_t n_shared;    /* CG: free DoFs touched by more than one block */
  int64_t n_partials;  /* CG: (block, shared DoF) pairs */
  double flops_per_apply;  /* algorithmic work of one apply (method's count) */
  double bytes_per_apply;  /* algorithmic HBM bytes of one apply */
  int64_t device_bytes;    /* device memory held by the op */
  int32_t n_components;    /* 1, or 3 for a vector field (vectors hold n_components * n_dofs values) */
  double flops_per_backward; /* algorithmic work of one tetmf_apply_backward with every output */
  double bytes_per_backward;
  int64_t n_cell_data;     /* entries of a cell-data array in library layout: 16 n_q ceil(n_cell / 16) */
} tetmf_info;

/* Mesh setup (Sec. 2.2 geometry; faces for eq. (7)).
 * xyz: host [n_vert][3]; tets: host [n_cell][4] vertex ids.
 * Errors: INVALID_ARGUMENT (NULL pointers; sizes outside 4 <= n_vert < 2^31
 * and 1 <= n_cell <= (2^31 - 1) / 4, so an empty mesh is rejected; ids out
 * of range; non-finite coordinates), DEGENERATE_CELL
 * (|det J| <= 1e-12 (mean edge length)^3), NONCONFORMING_MESH (a triangle in
 * more than two cells).  Inputs are copied; free with tetmf_mesh_destroy. */
int tetmf_mesh_create(int64_t n_vert, const double* xyz, int64_t n_cell, const int32_t* tets,
                      tetmf_mesh** out);
void tetmf_mesh_destroy(tetmf_mesh* mesh);
/* Number of faces (canonical order) and of interior faces. */
int tetmf_mesh_faces(const tetmf_mesh* mesh, int64_t* n_face, int64_t* n_interior);

/* Operator setup (Sec. 2.2: the precomputed geometry of each cell, J^{-1}
 * and |det J| folded into G_e = |det J| J^{-1} J^{-T} as the factor of eq.
 * (5); the tabulated basis matrices E of eq. (6); for SIPG the face data of
 * eq. (7)): DoF numbering, cell blocks, geometry computed in FP64 and rounded
 * to the op precision, basis tables, face data.  Allocates device memory
 * (OUT_OF_MEMORY on failure).  UNSUPPORTED for a (degree, n_q, n_qf,
 * precision, kind) combination with no compiled kernel, and for meshes
 * beyond the kernels' 32-bit indexing: n_dof_cell x n_cell, rounded up to
 * whole 256-cell blocks for CG and to 16-cell tiles for DG, must stay below
 * 2^31 (about 107 million cells at P3); CG also needs at most 2^27 cells
 * (rounded up to blocks) and n_dofs x element size below 2^32.  The mesh may
 * be destroyed afterwards. */
int tetmf_op_create(const tetmf_mesh* mesh, const tetmf_op_desc* desc, tetmf_op** out);
void tetmf_op_destroy(tetmf_op* op);
/* Sizes of the op and the algorithmic work of one apply and one backward:
 * the flop count of eq. (9) extended by the per-point coefficient (and the
 * mass term), with the DG face terms of eq. (11) counted per face, and the
 * HBM bytes of eq. (8) for the stored geometry, indices, coefficients and
 * vectors (each read or written once).  info: host, caller-owned. */
int tetmf_op_info(const tetmf_op* op, tetmf_info* info);

/* Host-only set-up check: runs the set-up of tetmf_op_create (numbering,
 * blocks, face data) without touching any device and verifies the
 * invariants the kernels rely on for every memory access (all indices in
 * range, every (cell, node) slot used exactly once, every partial sum
 * written exactly once).  Returns the status tetmf_op_create would return,
 * or TETMF_ERR_DEVICE with a description if an invariant fails.  n_dofs and
 * n_free (may be NULL) receive the sizes the op would have. */
int tetmf_op_check(const tetmf_mesh* mesh, const tetmf_op_desc* desc, int64_t* n_dofs, int64_t* n_free);

/* Maps from library order to user order (host buffers, any may be NULL):
 *  cell_perm [n_cell]: user cell id of library cell i
 *  dof_xyz   [n_dofs][3]: coordinates of each DoF (library numbering)
 *  dof_cell  [n_dofs]: DG: user cell owning the DoF; CG: one user cell containing it */
int tetmf_op_numbering(const tetmf_op* op, int32_t* cell_perm, double* dof_xyz, int32_t* dof_cell);

/* Reorder per-point cell data from user layout [n_cell][n_q] (user cell
 * order, FP64, device) to the library layout (n_cell_data entries, see the
 * top of this file) in the op precision (FP32 for F32 and BF16IN), or back
 * (to_user != 0; library layout in the op precision to user layout in
 * FP64). */
int tetmf_cell_data_layout(const tetmf_op* op, const void* src, void* dst, int to_user, void* stream);

/* v = A(kappa) u  (eq. (5) CG / eq. (7) DG), deterministic: the result is
 * bitwise reproducible for fixed inputs.
 *  u, v: device [n_components * n_dofs] in the op precision (FP32 for BF16IN); must not
 *        alias (ALIAS).
 *  kappa_cell: device, library cell-data layout (n_cell_data entries), or NULL (kappa = 1).
 *  kappa_face: DG only, device [n_qf][n_face] or NULL (kappa = 1).
 *  CG DIRICHLET: constrained entries v_c = u_c; constrained u_c do not enter
 *  the free rows (masked gather, Sec. 2.4). */
int tetmf_apply(tetmf_op* op, const void* u, const void* kappa_cell, const void* kappa_face, void* v,
                void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): v =
 * A(kappa) u exactly as tetmf_apply computes it (the same kernels; the
 * result is bitwise equal), with the CG interface partial sums (the
 * op's only per-apply scratch) kept in a fixed device array of the library
 * instead of the op's buffer.  The call allocates nothing and takes no
 * profiling events.  The array is TETMF_NOALLOC_SCRATCH_BYTES long; every
 * GPU the library runs on holds its own copy until the process ends, and
 * its device address is resolved at tetmf_op_create.
 *  Arguments, layouts and errors as for tetmf_apply, and UNSUPPORTED (no
 *  kernel launched) when n_partials * n_components * element size exceeds
 *  the array (the 64^3 x 6 P3 FP64 scalar operator needs 40 MB; its
 *  three-component form 120 MB does not fit).
 *  All calls on one GPU share the array and it keeps the last call's
 *  contents: calls whose execution overlaps on one GPU (other streams, other
 *  host threads) race and give wrong results; serialise them.  SIPG
 *  operators use no scratch and run tetmf_apply's kernels. */
#define TETMF_NOALLOC_SCRATCH_BYTES (64u << 20)
int tetmf_apply_noalloc(tetmf_op* op, const void* u, const void* kappa_cell, const void* kappa_face, void* v,
                        void* stream);

/* Backward of v = A(kappa) u for an upstream gradient g = dL/dv: the
 * derivatives of the bilinear forms of eq. (5) / eq. (7) (the paper gives no
 * backward; these follow from differentiating the forms):
 *  du = A^T g (= A g, both forms are symmetric) and the derivatives of
 *  g^T A(kappa) u with respect to the coefficients:
 *  dkappa_cell(q, e) = w_q |det J_e| (grad u . grad g)(x_q)            (CG, DG)
 *  dkappa_face[q][F] (DG only) = omega_q (tau [[u]][[g]] - {{d_n u}}[[g]]
 *        - [[u]]{{d_n g}}) on an interior face, omega_q (2 tau u g - g d_n u
 *        - u d_n g) on a Dirichlet boundary face, 0 on a Neumann one.
 * du, dkappa_cell or dkappa_face may be NULL; kappa_face and dkappa_face must
 * be NULL for CG (INVALID_ARGUMENT).  Outputs must not alias each other or an
 * input (ALIAS).  Layouts as for tetmf_apply (dkappa_cell in the library
 * cell-data layout, its padding entries set to zero).  UNSUPPORTED for
 * BF16IN. */
int tetmf_apply_backward(tetmf_op* op, const void* u, const void* g, const void* kappa_cell,
                         const void* kappa_face, void* du, void* dkappa_cell, void* dkappa_face,
                         void* stream);

/* d = diag(A(kappa)) (CG), constrained entries 1: the point Jacobi
 * preconditioner of the conjugate-gradient and Chebyshev iterations of Sec.
 * 4.1, from the diagonal entries of the cell matrices of eq. (5) summed per
 * DoF.  kappa_cell as for tetmf_apply; kappa_face must be NULL (SIPG:
 * UNSUPPORTED).  d: device [n_components * n_dofs] in the op precision. */
int tetmf_diagonal(tetmf_op* op, const void* kappa_cell, const void* kappa_face, void* d, void* stream);

/* Load vector: the right-hand side b(phi_i) of eq. (2) for the source f of
 * eq. (1), b_i = (f, phi_i) =
 * sum_e sum_q w_q |det J| f_{e,q} phi_i(x_q) (CG), with the cell rule of the
 * operator; zero on constrained rows.  f: device, library cell-data layout
 * in the op precision, or NULL (f = 1).  b: device [n_dofs].  UNSUPPORTED for SIPG and
 * for vector fields. */
int tetmf_load_vector(tetmf_op* op, const void* f, void* b, void* stream);

typedef struct {
  double rtol;         /* stop when ||b - A x|| <= rtol ||b|| (FP64 true residual) */
  double inner_rtol;   /* inner solve reduction per outer step (mixed precision) */
  int32_t max_outer;
  int32_t max_inner;   /* also the iteration cap of the plain FP64 PCG */
  int32_t precond;     /* 0 = none, 1 = Jacobi (point diagonal of the operator) */
  int32_t method;      /* with op_inner: 0 = iterative refinement, 1 = reliable updates (below) */
} tetmf_solve_opts;

typedef struct {
  int32_t outer_its, inner_its;
  double final_relres;  /* ||b - A64 x|| / ||b||, FP64 */
  double seconds;
} tetmf_solve_stats;

/* Solve A64 x = b (CG, SPD operator) on the GPU.
 *  op_inner == NULL: Jacobi-preconditioned conjugate gradients in FP64.
 *  op_inner (F32 or BF16IN op on the same mesh), mixed precision as in Sec.
 *  4.1 (the bulk of the work in the inner precision, every residual that
 *  decides convergence in FP64; dot products accumulated in FP64):
 *   method 0, iterative refinement: the FP64 residual r = b - A64 x, an
 *    inner Jacobi-PCG on A_inner d = r down to inner_rtol ||r||, x += d in
 *    FP64, repeated (max_outer steps);
 *   method 1, reliable updates: one inner-precision Jacobi-PCG whose iterate
 *    is added to x in FP64 and whose residual is replaced by the FP64 true
 *    residual b - A64 x whenever its recursively updated residual has fallen
 *    by inner_rtol since the previous replacement (or below rtol ||b|| / 2);
 *    with an F32 inner op the search direction is kept across a replacement
 *    while the true and the recursive residual agree (squared norms within a
 *    factor 4), so no Krylov information is discarded; it is restarted
 *    otherwise and always with a BF16IN inner op (max_outer caps the
 *    replacements, max_inner the inner iterations).
 *  b, x: device FP64 [n_components * n_dofs]; x holds x0 on entry (warm start) and the
 *  solution on exit.  kappa: device, library cell-data layout, for each op's
 *  precision, or NULL.  Synchronises the stream.  Returns NOT_CONVERGED when the caps are
 *  reached. */
int tetmf_solve(tetmf_op* op64, const void* kappa64, tetmf_op* op_inner, const void* kappa_inner,
                const double* b, double* x, const tetmf_solve_opts* opts, tetmf_solve_stats* stats,
                void* stream);

/* Chebyshev iteration preconditioned by the point Jacobi diagonal: the
 * smoother of the multigrid V-cycle of Sec. 4.1 (five pre- and five
 * post-smoothing steps per level there, run in single precision).  With
 * D = diag(A), theta = (lambda_max + lambda_min) / 2 and
 * delta = (lambda_max - lambda_min) / 2:
 *   r_0 = b - A x_0 (b when zero_guess), d_0 = D^-1 r_0 / theta,
 *   x_1 = x_0 + d_0, rho_0 = delta / theta, and for k = 1 .. degree - 1:
 *   r_k = b - A x_k, rho_k = 1 / (2 theta / delta - rho_{k-1}),
 *   d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D^-1 r_k,
 *   x_{k+1} = x_k + d_k.
 * The error x* - x is multiplied by p(D^-1 A) with
 * p(t) = T_degree((theta - t) / delta) / T_degree(theta / delta); one
 * operator application per step (degree - 1 with zero_guess).
 *  inv_diag: device [n_components * n_dofs], 1 / tetmf_diagonal (constrained entries 1).
 *  b, x: device [n_components * n_dofs], x_0 on entry unless zero_guess,
 *  the smoothed vector on exit.  All in the op precision (FP32 for BF16IN).
 *  kappa_cell as for tetmf_apply.
 *  degree >= 1, 0 <= lambda_min < lambda_max (INVALID_ARGUMENT otherwise);
 *  x may not alias b or inv_diag (ALIAS).  CG only (UNSUPPORTED for DG).
 *  Two work vectors are allocated by the op on the first call and kept.
 *  Asynchronous on the stream. */
int tetmf_chebyshev(tetmf_op* op, const void* kappa_cell, const void* inv_diag, const void* b, void* x,
                    int degree, double lambda_min, double lambda_max, int zero_guess, void* stream);

/* Estimate of the largest eigenvalue of D^-1 A (D = diag(A)), the upper end
 * of the smoother's interval: n_iter steps of Jacobi-preconditioned
 * conjugate gradients on A y = r_0 from a fixed pseudo-random r_0, and the
 * largest eigenvalue of the Lanczos tridiagonal matrix formed from their
 * step lengths (a lower bound of the true value that converges from below;
 * smoothers commonly scale it by 1.1-1.2).  n_iter in 1..500.  inv_diag as
 * for tetmf_chebyshev.  Allocates and frees temporaries; synchronises. */
int tetmf_estimate_lambda_max(tetmf_op* op, const void* kappa_cell, const void* inv_diag, int n_iter,
                              double* lambda_max, void* stream);

/* Measurement aid.  While enabled, every launch of the op's main kernel (the
 * cell kernel of apply, backward, diagonal and load vector; the
 * cell-and-face kernel for DG) carries a HIP event pair attached to its
 * dispatch on the caller's stream, which records the dispatch's start and
 * end timestamps (no extra packet between launches).  tetmf_op_profile(op,
 * 1) starts a new measurement (events are created on demand and reused),
 * tetmf_op_profile(op, 0) stops recording.
 * tetmf_op_profile_read synchronises on the recorded events and returns the
 * summed kernel time in milliseconds and the number of launches recorded. */
int tetmf_op_profile(tetmf_op* op, int enable);
int tetmf_op_profile_read(tetmf_op* op, double* total_ms, int64_t* launches);
/* The same measurement launch by launch: ms (host [capacity]) receives the
 * duration of each of the first min(capacity, launches) recorded launches
 * in recording order; *launches the number recorded.  Synchronises. */
int tetmf_op_profile_times(tetmf_op* op, double* ms, int64_t capacity, int64_t* launches);

const char* tetmf_status_string(int status);
const char* tetmf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TETMF_H */
