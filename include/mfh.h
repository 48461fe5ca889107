/*
 * mfh.h -- C ABI of the MI355X matrix-free finite-strain hyperelasticity library.
 *
 * The library applies the Newton tangent of a compressible Neo-Hookean body
 * without assembling it (the matrix-free vmult of Sec. 5, built on the
 * linearisation of Sec. 2.2 and the material law of Sec. 2.3), evaluates the
 * residual of the weak form (Sec. 2.1, Sec. 3), and solves the Newton system
 * with a CG preconditioned by the geometric multigrid V-cycle of Sec. 6 whose
 * level operators are linearised about the displacement interpolated onto each
 * level.  Smoother and solver settings follow Sec. 7: Chebyshev of degree 4
 * on the operator diagonal, two pre- and two post-smoothing steps, the
 * interval [0.6, 1.2] x lambda_max, lambda_max from 30 CG iterations.
 *
 * Geometry and numbering.  The body is the unit box [0,1]^dim (dim = 2 is
 * plane strain) split into n_cells^dim equal cells; the displacement is a
 * continuous vector Lagrange field of degree p (Gauss-Lobatto-Legendre
 * support points) integrated with the (p+1)^dim Gauss rule (Tables 1-2).  The
 * lattice has L = p*n_cells + 1 nodes per direction; every vector is
 * component-blocked with the first lattice index fastest (the tensor
 * multi-index of Sec. 5):  dof = c * L^dim + i + L * (j + L * k).
 *
 * Ownership and memory.  All vector arguments are DEVICE pointers owned by
 * the caller; the library never frees them.  Every device buffer the library
 * uses lives in the caller-supplied workspace passed to mfh_create (size from
 * mfh_workspace_size); after mfh_create returns the library allocates no
 * device memory.  Host arrays inside mfh_desc are copied at mfh_create.
 *
 * Streams and synchronisation.  Work is enqueued on the HIP stream given to
 * mfh_create (NULL = the null stream).  Calls documented as "async" return
 * after enqueueing; calls that return host scalars synchronise the stream.
 *
 * Errors.  Every call returns an mfh_status; nothing throws or exits.  After
 * an error, mfh_last_error(problem) (or mfh_last_error(NULL) for failures
 * before a problem exists) gives a message.  A problem stays usable after any
 * error other than MFH_ERR_HIP.  A problem is not thread-safe.
 *
 * Dirichlet conditions fix whole components on whole faces.  Bit
 * ((2*axis + side) * dim + comp) of dirichlet_mask fixes component comp on the
 * face x_axis = side.  Operators carry identity rows and columns on
 * constrained DoFs:  tangent_vmult returns K_c x with
 * K_c = (I - C) K (I - C) + C (C = indicator of constrained DoFs); residual
 * returns zero on constrained rows; cg_solve expects b = 0 on constrained
 * rows and returns x = 0 there.
 */
#ifndef MFH_H
#define MFH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MFH_OK = 0,
  MFH_ERR_INVALID_ARG = -1,   /* bad descriptor, level, dtype, pointer, or call order   */
  MFH_ERR_HIP = -2,           /* a HIP runtime call failed; the problem is unusable      */
  MFH_ERR_WORKSPACE = -3,     /* workspace smaller than mfh_workspace_size reported      */
  MFH_ERR_INVERTED = -4,      /* a quadrature point has J = det F <= 0 (Sec. 2.1)       */
  MFH_ERR_NOT_CONVERGED = -5, /* CG / Newton hit its iteration limit; outputs still set */
  MFH_ERR_BREAKDOWN = -6,     /* CG: p^T A p <= 0 or a NaN appeared                     */
  MFH_ERR_NOT_SPD = -7        /* coarse-level tangent numerically singular (zero or
                                 non-finite pivot); see mfh_coarse_inertia               */
} mfh_status;

enum { MFH_F64 = 0, MFH_F32 = 1 };

/* Quadrature-point policies of the tangent vmult (Sec. 5, Algorithms 1-3):
 *  RECOMPUTE  re-evaluates Grad u, F, J, F^-1, ln J and the stresses at every
 *             quadrature point from the displacement (the recompute end of
 *             the caching trade-off; Algorithm 1 without its scalar cache);
 *  CACHE_F    reads the cached deformation gradient F and recomputes the rest;
 *  CACHE_T2   reads cached F^-1 and c1 = mu - 2 lambda ln J: the
 *             referential counterpart of Algorithm 2's cached tau/J, c1, c2
 *             (for this law the geometric term Grad x S equals
 *             mu Grad x - c1 Grad x F^-1 F^-T, so the stress need not be
 *             stored);
 *  CACHE_T4   reads cached F^-1, S and the material part of the spatial
 *             tangent J c (21 symmetric words in 3-D, 6 in 2-D): the
 *             referential counterpart of Algorithm 3 ("tensor4"); the
 *             quadrature-point stage evaluates no constitutive law, so it
 *             serves any law (the only policy for MFH_LAW_MOONEY_RIVLIN).
 * Cache words per quadrature point: 0, d^2, d^2 + 1,
 * d^2 + d(d+1)/2 + (d(d+1)/2)(d(d+1)/2 + 1)/2 (36 in 3-D), in the V-cycle
 * precision and in FP64 on every level.                                     */
enum { MFH_QP_RECOMPUTE = 0, MFH_QP_CACHE_F = 1, MFH_QP_CACHE_T2 = 2, MFH_QP_CACHE_T4 = 3 };

/* Material law.  NEO_HOOKE is the compressible Neo-Hookean energy of Sec. 2.3,
 *   psi = mu/2 [I1 - 3 - 2 ln J] + lambda ln^2 J.
 * MOONEY_RIVLIN adds a second-invariant term (a second law for the tensor4
 * route, whose operator does not depend on the law):
 *   psi = mu/2 [I1 - 3 - 2 ln J] + mu2/2 [I2 - 3 - 4 ln J] + lambda ln^2 J,
 * stress-free at F = I, small-strain Lame pair (mu + mu2, 2 lambda + 2 mu2);
 * invariants of the 3-D tensors (plane strain: C_33 = 1).  It needs
 * qp_policy CACHE_T4; the residual, diagonal and coarse / CSR assembly
 * evaluate it directly. */
enum { MFH_LAW_NEO_HOOKE = 0, MFH_LAW_MOONEY_RIVLIN = 1 };

/* Scatter of cell results into the output vector: ATOMIC (one hardware float
 * atomic per cell node; summation order varies run to run), COLOR (2^dim
 * launches over cells of equal coordinate parity, plain read-modify-write,
 * deterministic), TILE (one block per tile of cells: tile nodes staged in
 * LDS, contributions summed there, global atomics only on tile faces shared
 * with a neighbouring tile; order varies) or ELEMENT (the cell kernel stores
 * every cell's nodal results in an element buffer, the shared face nodes of
 * x-neighbours in one cell block already summed, and a second kernel sums
 * the remaining contributions of every node in a fixed order and writes each
 * output entry once: deterministic, no atomics, no separate output fill; the
 * workspace grows by dim * (p+1)^dim * cells of the finest level doubles).
 * AUTO takes, for every level and precision, the mode measured
 * fastest on gfx950 for the problem's dimension, degree, qp policy and the
 * level's cell count (a table built by the package's autotuner and compiled
 * into the library).  The choice affects tangent_vmult only; all other cell
 * kernels use ATOMIC when TILE or ELEMENT is selected. */
enum {
  MFH_SCATTER_AUTO = -1,
  MFH_SCATTER_ATOMIC = 0,
  MFH_SCATTER_COLOR = 1,
  MFH_SCATTER_TILE = 2,
  MFH_SCATTER_ELEMENT = 3
};

/* Tile shape of the TILE scatter: two shapes (cells per axis) are compiled
 * for every dimension, degree and precision; AUTO takes the one the
 * autotuner measured faster for the level (same table as the scatter mode),
 * 0 or 1 forces one.  mfh_tile_shape reports the shape a level uses. */
enum { MFH_TILE_SHAPE_AUTO = -1 };

/* Cells per workgroup of the tangent vmult's pencil kernels (ATOMIC, COLOR,
 * ELEMENT): two lengths are compiled for every dimension and degree (0: the
 * length that keeps the most FP64 blocks resident, 1: about half of it, or
 * for 3-D Q4 the ten cells 256 threads hold); AUTO takes the one the
 * autotuner measured faster with the level's scatter mode, 0 or 1 forces one.
 * mfh_cell_block reports the choice of a level. */
enum { MFH_CELL_BLOCK_AUTO = -1 };

/* Displacement the coarser level operators are linearised about (Sec. 6
 * restricts the fine displacement to every level without saying how):
 * NODAL interpolates the finer level's field at the coarser support points,
 * level by level; VERTEX takes the fine field's values at the coarser level's
 * cell vertices and fills each coarse cell multilinearly.  The two agree for
 * degree 1; for higher degrees NODAL reproduces more of the field, while
 * VERTEX cannot overshoot between vertices, which keeps the coarse tangents of
 * strongly heterogeneous bodies positive definite for longer under load. */
enum { MFH_LEVEL_FIELD_NODAL = 0, MFH_LEVEL_FIELD_VERTEX = 1 };

/* Coarsest-level solve inside the V-cycle: DIRECT (dense FP64 inverse of the
 * coarse tangent on the free DoFs, exact; coarse levels up to 20,000 DoFs) or
 * CHEBYSHEV (Sec. 7: the Chebyshev iteration used as a solver that reduces the
 * residual by three orders of magnitude: Jacobi-preconditioned, on the
 * interval [lambda_min, cheb_hi * lambda_max] of the coarse level's CG-Lanczos
 * estimates, degree = ceil(acosh(1000) / acosh((b + a) / (b - a))), at most
 * 1000; a fixed polynomial, so the V-cycle stays a symmetric linear operator;
 * needs a definite coarse tangent and allows coarse levels of any size). */
enum { MFH_COARSE_DIRECT = 0, MFH_COARSE_CHEBYSHEV = 1 };

typedef struct mfh_problem mfh_problem;

typedef struct {
  int dim;                   /* 2 or 3                                                   */
  int n_cells;               /* cells per direction on the finest level (>= 1)            */
  int degree;                /* polynomial degree p, 1..4                                */
  int n_levels;              /* multigrid levels >= 1; n_cells % 2^(n_levels-1) == 0      */
  int n_materials;           /* 1 or 2 (material 0 = matrix)                             */
  const double* mu;          /* host [n_materials] shear moduli, > 0                     */
  const double* lambda;      /* host [n_materials] parameter lambda of the energy         */
  int n_inclusions;          /* >= 0                                                     */
  const double* inclusions;  /* host [n_inclusions][dim + 2]: centre, radius, material id;
                                a quadrature point X is in an inclusion when
                                |X - centre|^2 <= radius^2 (later rows win)               */
  unsigned dirichlet_mask;   /* face-component bits, see above                           */
  int qp_policy;             /* MFH_QP_*                                                  */
  int scatter;               /* MFH_SCATTER_*                                              */
  int vcycle_dtype;          /* MFH_F32: mixed precision V-cycle; MFH_F64: all FP64        */
  int cheb_degree;           /* Chebyshev degree (paper: 4), 1..16                       */
  int n_smooth;              /* Chebyshev applications pre and post (paper: 2), 1..8      */
  int eig_iters;             /* CG iterations for lambda_max (paper: 30), 1..200          */
  double cheb_lo, cheb_hi;   /* smoother interval factors (paper: 0.6, 1.2)              */
  int level_field;           /* MFH_LEVEL_FIELD_*: displacement on the coarser levels     */
  int coarse_solver;         /* MFH_COARSE_*                                             */
  int eig_refresh;           /* eigenvalue estimates: 1 every linearisation, k every k-th,
                                0 only the first (then reused)                           */
  int law;                   /* MFH_LAW_*                                                 */
  const double* mu2;         /* host [n_materials] second-invariant moduli >= 0 (law
                                MOONEY_RIVLIN; ignored, may be NULL, otherwise)           */
  int tile_shape;            /* MFH_TILE_SHAPE_AUTO, 0 or 1 (TILE scatter only)          */
  int cell_block;            /* MFH_CELL_BLOCK_AUTO, 0 or 1 (tangent vmult, pencil modes)  */
} mfh_desc;

/* Fills *desc with the paper's solver settings (degree 4, 2 steps, 30
 * iterations, [0.6, 1.2]), RECOMPUTE, AUTO scatter, tile shape and cell
 * block, F32 V-cycle, NODAL level fields, DIRECT coarse solve, eigenvalue estimates at
 * every linearisation, the Neo-Hookean law; geometry fields are zeroed and
 * must be set by the caller. */
void mfh_desc_defaults(mfh_desc* desc);

/* Device bytes the problem needs.  Errors: MFH_ERR_INVALID_ARG. */
mfh_status mfh_workspace_size(const mfh_desc* desc, size_t* bytes);

/* Creates a problem inside `workspace` (device, >= mfh_workspace_size bytes,
 * 256-byte aligned, owned by the caller and kept alive until mfh_destroy).
 * `hip_stream` is a hipStream_t or NULL.  Builds the level lattices, 1-D
 * tables, per-quadrature-point material ids, transfer tables and Dirichlet
 * masks.  Synchronises.  Errors: INVALID_ARG, WORKSPACE, HIP. */
mfh_status mfh_create(const mfh_desc* desc, void* workspace, size_t bytes,
                      void* hip_stream, mfh_problem** out);

/* Releases host state (never the workspace).  NULL is accepted. */
mfh_status mfh_destroy(mfh_problem* problem);

/* Number of DoFs of level `level` (0 = coarsest, n_levels-1 = finest). */
mfh_status mfh_n_dofs(const mfh_problem* problem, int level, long long* n);

/* Linearisation point (Sec. 6): copies the finest-level displacement u
 * (device FP64, n_dofs), interpolates it at the support points of every
 * coarser level, and builds each level operator's quadrature data.  Writes
 * the smallest J over all levels to *min_J_host (may be NULL).  The
 * preconditioner data (operator diagonals, Chebyshev intervals with
 * lambda_max from eig_iters CG iterations, FP64 coarse-level inverse) are
 * built on the first V-cycle / CG / Chebyshev / diagonal query that follows.
 * Synchronises.  Errors: INVALID_ARG, INVERTED (min J <= 0; the problem then
 * has no valid linearisation point until the next successful call), HIP. */
mfh_status mfh_set_deformation(mfh_problem* problem, const double* u_dev, double* min_J_host);

/* y = K_c x on `level` in precision `dtype` (MFH_F64: double*, MFH_F32:
 * float*), linearised about the level displacement of the last
 * mfh_set_deformation (eq. mf_vmult / eq. algebraic_tangent).  x and y are
 * device vectors of n_dofs(level) entries and must not overlap.  Async.
 * Errors: INVALID_ARG (also when no deformation was set), HIP. */
mfh_status mfh_tangent_vmult(mfh_problem* problem, int level, int dtype,
                             const void* x_dev, void* y_dev);

/* ---- Matrix-based baseline: K_c in CSR form ---- */

/* Sizes of the CSR form of a level's constrained tangent K_c (the matrix of
 * eq. algebraic_tangent with the constraints of Sec. 3), the operator of the
 * matrix-based approach that Sec. 4 and Sec. 7.1 compare against.
 * n_rows = dim * nodes, DoF numbering as the vectors.
 * A free row lists every DoF of the cells that hold its node, component-major
 * and by ascending node index within a component (constrained columns stay as
 * stored zeros); a constrained row holds its diagonal only.  Host outputs, no
 * device work.  Errors: INVALID_ARG. */
mfh_status mfh_csr_size(mfh_problem* problem, int level, long long* n_rows_host, long long* nnz_host);

/* Fills caller-allocated device arrays with K_c of the level at the current
 * linearisation point: row_ptr (n_rows + 1 int64), col (nnz int32, sorted
 * within each row), val (nnz FP64).  Element matrices are added with atomics,
 * so values may differ from run to run in the last bits.  Synchronises.
 * Errors: INVALID_ARG (also for n_rows >= 2^31), HIP. */
mfh_status mfh_csr_assemble(mfh_problem* problem, int level, long long* row_ptr_dev, int* col_dev,
                            double* val_dev);

/* y = A x (FP64) for the CSR arrays written by mfh_csr_assemble for this
 * level; each row is summed by a group of 16 lanes (mean rows of at most
 * 100 entries) or 8 lanes (longer rows), each lane keeping 4 or 8 entries in
 * flight.  Async on the problem's stream.
 * Errors: INVALID_ARG, HIP. */
mfh_status mfh_csr_spmv(mfh_problem* problem, int level, const long long* row_ptr_dev, const int* col_dev,
                        const double* val_dev, const double* x_dev, double* y_dev);

/* r = residual of the weak form at displacement u on the finest level
 * (eq. linear_system, volume term; FP64), zero on constrained rows.  u is any
 * device FP64 displacement (not necessarily the linearisation point).  Async.
 * Errors: INVALID_ARG, HIP. */
mfh_status mfh_residual(mfh_problem* problem, const double* u_dev, double* r_dev);

/* z = one multigrid V-cycle applied to r on the finest level (Sec. 6, Sec. 7),
 * FP64 in and out; the cycle itself runs in vcycle_dtype, the coarse solve in
 * FP64.  The V-cycle, CG and Newton entry points need a coarsest level of at
 * most 20000 DoFs (the dense direct solve); larger coarsest levels give
 * INVALID_ARG there while operator application keeps working.  The first
 * call after set_deformation builds the preconditioner data and synchronises;
 * later calls are async.  Errors: INVALID_ARG, NOT_SPD (coarse-level tangent
 * numerically singular), BREAKDOWN (eigenvalue estimate), HIP. */
mfh_status mfh_gmg_vcycle(mfh_problem* problem, const double* r_dev, double* z_dev);

/* Solves K_c x = b on the finest level with FP64 CG preconditioned by the
 * V-cycle, x0 = 0, until |r|_2 <= rtol |b|_2 or max_it iterations.  Writes the
 * iteration count and the final relative residual (recomputed explicitly as
 * |b - K_c x| / |b|) to the host pointers (may be NULL).  Synchronises.
 * Errors: INVALID_ARG, NOT_CONVERGED, BREAKDOWN, NOT_SPD, HIP. */
mfh_status mfh_cg_solve(mfh_problem* problem, const double* b_dev, double* x_dev,
                        double rtol, int max_it, int* iters_host, double* relres_host);

/* Message for the last error of `problem` (or of the calling thread's last
 * failed mfh_create / mfh_workspace_size when problem is NULL). */
const char* mfh_last_error(const mfh_problem* problem);

/* ---- Newton load stepping (Sec. 3 Newton-Raphson, Sec. 7 tolerances) ---- */

typedef struct {
  int load_step, newton_iter, cg_iters;   /* load_step counts attempted increments */
  double residual_norm;      /* |rhs| of this Newton step (free rows)                   */
  double residual_after;     /* |R(u)| on free rows after the update                    */
  double du_norm;            /* |du|_2                                                  */
  double cg_relres;
  double min_J;
  double setup_ms, residual_ms, solve_ms;   /* host wall time of each phase         */
  int coarse_negative;       /* negative eigenvalues of the coarse-level tangent          */
  double load_fraction;      /* fraction of the prescribed values this increment reaches  */
  int cutbacks;              /* load-increment halvings so far in the solve               */
  double step_length;        /* alpha of the accepted update (NaN: none accepted)         */
} mfh_newton_record;

/* Sets u on constrained DoFs to scale * face_values[2*axis + side][comp]
 * (host array of 2*dim*dim doubles; where faces meet, the later face in
 * axis-major order wins).  Async.  Errors: INVALID_ARG, HIP. */
mfh_status mfh_apply_dirichlet(mfh_problem* problem, double* u_dev,
                               const double* face_values, double scale);

/* Full Newton solve under displacement control and dead face tractions.
 * The prescribed values (as for mfh_apply_dirichlet) and the tractions
 * face_traction (host array of 2*dim*dim doubles, traction vector per face,
 * constant per unit reference area; NULL for none; the Neumann term of
 * Sec. 3, R = F_int(u) - s f_ext with the load fraction s) are applied in
 * n_steps equal increments.  While the prescribed values g of the increment
 * are not yet met (its first Newton step, and after a shortened step), a
 * Newton step carries the rest dg = g - u linearly (K_c d = -(R(u) + K(u) dg),
 * du = dg + d); otherwise it solves K_c du = -R(u).  The update is
 * u <- u + alpha du with alpha = 1, 1/2, ... (at most 12 halvings), the first
 * that keeps J > 0 at every quadrature point and, once g is met, lowers
 * |R|^2 by the factor 1 - 2e-4 alpha; a full step sets the constrained
 * entries to g exactly.  An increment converges when g is met, |du| <= du_tol
 * and |R| <= r_tol or |R| <= r_tol |R0| (R0: first right-hand side of the
 * increment), R on free rows.  An increment fails when the CG breaks down
 * (p^T K p <= 0: the tangent is indefinite at the iterate; also when a level
 * tangent stops the smoother's eigenvalue estimate at its first step, or the
 * coarse tangent is numerically singular) or does not reach
 * cg_rtol in cg_max_it steps, when no step length is accepted, or when
 * max_newton steps do not converge; then u is restored to the start of the
 * increment and the failed increment is halved, down to 1/256 of a load step
 * (the solve fails when an increment of that size fails); after a converged
 * cut increment the step doubles again up to 1/n_steps.  max_seconds > 0 is a
 * wall-time budget: when it is exhausted at the start of a Newton step, u is
 * restored to the last converged load and the call returns NOT_CONVERGED
 * (the records tell the load reached).  The record of a
 * Newton step whose update was not taken carries NaN in residual_after and
 * step_length (and in cg_relres after a CG breakdown).
 * u (device FP64) is the initial state and receives the solution.  Up to
 * max_records records are written to the host array; *n_records receives the
 * number of Newton steps taken.  With MFH_NEWTON_LOG=1 in the environment
 * every Newton step is also printed as one line on stderr.  Synchronises.
 * Errors: INVALID_ARG, INVERTED, NOT_CONVERGED, BREAKDOWN, NOT_SPD, HIP. */
mfh_status mfh_newton_solve(mfh_problem* problem, double* u_dev, const double* face_values,
                            const double* face_traction, int n_steps, double cg_rtol, int cg_max_it,
                            double du_tol, double r_tol, int max_newton, double max_seconds,
                            mfh_newton_record* records, int max_records, int* n_records);

/* f = nodal forces of dead face tractions on the finest level (as for
 * mfh_newton_solve: f_a = sum over loaded faces of the face integral of
 * T_f N_a), zero on constrained rows.  f is a device FP64 vector.  Async.
 * Errors: INVALID_ARG, HIP. */
mfh_status mfh_external_force(mfh_problem* problem, const double* face_traction, double* f_dev);

/* The scatter mode tangent_vmult uses on `level` in precision dtype (the
 * descriptor's mode, or the tuned choice under MFH_SCATTER_AUTO) into *mode.
 * Host only.  Errors: INVALID_ARG. */
mfh_status mfh_scatter_mode(const mfh_problem* problem, int level, int dtype, int* mode);

/* The TILE scatter's tile shape on `level` in precision dtype (the
 * descriptor's, or the tuned one under MFH_TILE_SHAPE_AUTO) into *shape (0 or
 * 1) and its cells per axis into cells[0..2] (cells[2] = 1 in 2-D).  Reported
 * whatever the scatter mode; it is used only when the level runs TILE.  Host
 * only.  Errors: INVALID_ARG. */
mfh_status mfh_tile_shape(const mfh_problem* problem, int level, int dtype, int* shape, int* cells);

/* The cell-block variant (0 or 1) the tangent vmult's pencil kernels use on
 * `level` in precision dtype into *variant and its cells per workgroup into
 * *cells.  Host only.  Errors: INVALID_ARG. */
mfh_status mfh_cell_block(const mfh_problem* problem, int level, int dtype, int* variant, int* cells);

/* Coordinates of the support points along one axis of `level` (all axes
 * are alike): the L = degree * N + 1 lattice positions in [0, 1], the
 * Gauss-Lobatto-Legendre points of every cell (the paper names no point
 * family; this is the library's choice, equispaced for degree <= 2), into the host array
 * x (L doubles).  Node (i, j, k) sits at (x[i], x[j], x[k]).  Host only.
 * Errors: INVALID_ARG. */
mfh_status mfh_node_coords_1d(mfh_problem* problem, int level, double* x_host);

/* ---- Access to multigrid pieces, for verification against a reference ---- */

/* Copies the FP64 level displacement of the last set_deformation. Sync. */
mfh_status mfh_level_displacement(mfh_problem* problem, int level, double* u_dev);
/* Copies the FP64 operator diagonal of `level` (1 on constrained DoFs). Sync. */
mfh_status mfh_level_diagonal(mfh_problem* problem, int level, double* d_dev);
/* lambda_max estimate of D^-1 A on `level` >= 1 (host). */
mfh_status mfh_level_lambda_max(mfh_problem* problem, int level, double* lam_host);
/* Fixes the eigenvalue estimates of `level` that the smoother (Sec. 7: the
 * Chebyshev interval [cheb_lo, cheb_hi] * lam_max on levels >= 1) or, on level
 * 0, the Chebyshev coarse solver ([lam_min, cheb_hi * lam_max]) is built from,
 * in place of the Lanczos estimates; for comparing smoothers and V-cycles
 * across implementations on one interval.  lam_max = 0 clears the override
 * (the next solver call re-estimates).  lam_max must be finite and > 0
 * otherwise; lam_min is read only on level 0 with the Chebyshev coarse solver
 * and must then satisfy 0 < lam_min < lam_max (MFH_ERR_INVALID_ARG).  Kept
 * across set_deformation calls; takes effect at the next solver call. */
mfh_status mfh_set_level_eigenvalues(mfh_problem* problem, int level, double lam_min, double lam_max);
/* y_fine = P x_coarse (coarse level = level-1, fine = level, 1 <= level),
 * constrained fine entries zeroed; dtype as for tangent_vmult.  Async. */
mfh_status mfh_prolongate(mfh_problem* problem, int level, int dtype, const void* x_dev, void* y_dev);
/* y_coarse = P^T x_fine, constrained coarse entries zeroed.  Async. */
mfh_status mfh_restrict(mfh_problem* problem, int level, int dtype, const void* x_dev, void* y_dev);
/* One degree-cheb_degree Chebyshev application on `level` >= 1 in the
 * V-cycle's precision (vcycle_dtype): x <- x + p(D^-1 A)(D^-1 (f - A x)).  Async. */
mfh_status mfh_chebyshev(mfh_problem* problem, int level, const void* f_dev, void* x_dev);

/* The coarse level's dense direct solver (the exact FP64 coarse solve that
 * replaces the paper's Chebyshev coarse iteration, Sec. 7) on a caller's
 * matrix, for any nonsingular symmetric matrix, definite or not: block
 * Gauss-Jordan in plain diagonal order first, kept when every pivot is
 * positive and above 1e-12 max |A_ii| (A positive definite: no element
 * growth without exchanges); otherwise symmetric block Gauss-Jordan with
 * symmetric pivoting (each block of 64 takes the unswept indices of largest
 * |diagonal| of the current Schur complement and is inverted with
 * Bunch-Kaufman 1x1/2x2 pivots).  The choice is made on the device.
 * a_dev: n x n FP64 row-major symmetric matrix (device), work space of the
 * pivoted pass: unchanged when the plain pass is kept, else overwritten
 * by the inverse in the pivoted basis; inv_dev: receives A^-1 in the original
 * order (device, n x n, must not overlap a_dev); work_dev: at least
 * mfh_dense_inverse_workspace(n) bytes of device memory, 256-byte aligned;
 * stream: HIP stream (NULL: default).  *negative receives the number of
 * negative eigenvalues of A (Sylvester: signs of the kept pass's 1x1 and 2x2
 * pivots).
 * 1 <= n <= 20000.  Synchronises.  Errors: INVALID_ARG, WORKSPACE, NOT_SPD
 * (numerically singular: a pivot, or a 2x2 pivot's determinant against its
 * largest entry, at most 1e-12 max |A_ii| or not finite), HIP. */
mfh_status mfh_dense_inverse_workspace(long long n, size_t* bytes);
mfh_status mfh_dense_inverse(double* a_dev, double* inv_dev, long long n, void* work_dev, size_t work_bytes,
                             void* stream, int* negative);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * dense inverse with its work arrays in a static device array of the library
 * (2.25 MiB per GPU, held until the process ends) instead of a caller
 * workspace.  Allocates nothing.  Runs on the calling thread's current
 * device (stream must belong to it; NULL: default stream); 1 <= n <= 2048
 * (INVALID_ARG otherwise).  All calls on one GPU share the array, so calls
 * that overlap in time on one GPU (other threads, other streams) race and
 * must be serialised by the caller.  Arguments, results and errors as for
 * mfh_dense_inverse.  Synchronises. */
mfh_status mfh_dense_inverse_static(double* a_dev, double* inv_dev, long long n, void* stream, int* negative);

/* Number of negative eigenvalues of the coarse-level tangent about the current
 * linearisation point (the signs of its elimination pivots).  The V-cycle's
 * coarse solve is exact for any nonsingular coarse tangent; a nonzero count
 * means the coarse mesh does not resolve the material well enough for the
 * level linearised about the interpolated displacement to stay positive
 * definite (the assumption of Sec. 6), and the preconditioner is then
 * indefinite.  Builds the preconditioner data if needed (synchronises).
 * DIRECT coarse solver only.  Errors: INVALID_ARG, NOT_SPD, HIP. */
mfh_status mfh_coarse_inertia(mfh_problem* problem, int* negative);

/* ---- Graph capture ---- */

/* enable != 0: the CG replays its V-cycle from a HIP graph captured on the
 * problem's stream (captured at the first V-cycle after each
 * set_deformation, since the Chebyshev coefficients are kernel arguments).
 * Has no effect for problems created on the null stream, which cannot be
 * captured.  Default off. */
mfh_status mfh_enable_graphs(mfh_problem* problem, int enable);

/* ---- Batches of independent problems (many meshes, degrees, materials) ---- */

typedef struct mfh_batch mfh_batch;

/* All calls on one batch, and on the problems it holds while it exists, must
 * come from one host thread (the batch drives the problems' streams itself);
 * concurrent calls from several threads are not supported. */

/* Device bytes for a batch over n existing problems (all with one qp_policy). */
mfh_status mfh_batch_workspace_size(int n, mfh_problem* const* problems, size_t* bytes);

/* Builds the device work lists of a batch: problems are binned by (dim,
 * degree); each bin's tangent vmult is one launch with one workgroup per
 * (problem, cell block) item of all its problems.  The problems keep their
 * own workspaces and streams and must outlive the batch; the batch workspace
 * (device, 256-byte aligned) holds the per-problem argument tables and the
 * item lists; the batch also allocates a small pinned host buffer (a few
 * hundred bytes per problem) for the scalars its solves read back.  Batched
 * vmults are enqueued on `hip_stream`.  Synchronises.
 * Errors: INVALID_ARG, WORKSPACE, HIP. */
mfh_status mfh_batch_create(int n, mfh_problem* const* problems, void* workspace, size_t bytes,
                            void* hip_stream, mfh_batch** out);
mfh_status mfh_batch_destroy(mfh_batch* batch);
const char* mfh_batch_last_error(const mfh_batch* batch);

/* mfh_set_deformation of every problem (host array u of device pointers):
 * the level data of all problems are enqueued on their own streams first and
 * drained once; min J per problem into the host array min_J (may be NULL; NaN
 * for a failed problem).  Synchronises.  Returns the first failing problem's
 * status (INVERTED, HIP, INVALID_ARG); the other problems are set. */
mfh_status mfh_batch_set_deformation(mfh_batch* batch, const double* const* u, double* min_J);

/* y[i] = K_c,i x[i] for every problem i, on the finest levels (host arrays of
 * device pointers, dtype as for mfh_tangent_vmult): one batched output fill
 * and one launch per (dim, degree) bin.  Async on the batch stream, except
 * that a pointer set different from the previous call's is uploaded and the
 * batch stream synchronised first; every problem must have a linearisation
 * point. */
mfh_status mfh_batch_tangent_vmult(mfh_batch* batch, int dtype, const void* const* x, void* const* y);

/* The 1-D contraction stage of the sum factorisation (Sec. 5) alone, for the
 * autotuner's choice between VALU and MFMA at degrees 3 and 4 in FP32:
 * `blocks` workgroups of 256 lines of degree + 1 values in LDS, `sweeps`
 * dependent applications of a pair of (degree + 1)^2 tables; mfma = 0: one
 * line per thread with FMAs, 1: v_mfma_f32_16x16x4f32 on 16 lines at a time
 * (the tables stacked as A, the lines' values as B).  out (device, blocks *
 * (degree + 1) * 256 floats) receives the final values (both forms agree up
 * to rounding).  Async on `stream`.  Errors: INVALID_ARG, HIP. */
mfh_status mfh_contraction_stage(int degree, int mfma, int sweeps, int blocks, float* out_dev, void* stream);

/* Launch form of mfh_batch_tangent_vmult: one launch per (dim, degree) bin
 * (PER_DEGREE: each degree's kernel at its own occupancy), or one persistent
 * launch over the cell blocks of every problem (FUSED: a grid of the
 * workgroups the GPU holds at once walks XCD-local ranges of the item list,
 * heaviest degree first, each running its item's degree; 3-D batches of
 * degrees 1 to 3 only), followed in both by the node sums of the problems on
 * the ELEMENT scatter.  AUTO (default): the form the autotuner measured
 * faster on gfx950.  Errors: INVALID_ARG (unknown mode; FUSED for a batch
 * it does not cover). */
enum { MFH_BATCH_LAUNCH_AUTO = -1, MFH_BATCH_LAUNCH_PER_DEGREE = 0, MFH_BATCH_LAUNCH_FUSED = 1 };
mfh_status mfh_batch_set_launch(mfh_batch* batch, int mode);

/* mfh_cg_solve of every problem (host arrays of device pointers) from one
 * host thread, in lockstep: the preconditioner set-ups of all problems are
 * enqueued and drained together, then every round issues one PCG iteration of
 * every unfinished problem on its own stream (V-cycles replayed from graphs
 * when enabled) and judges them all after one drain.  Each problem follows
 * the same sequence of operations as mfh_cg_solve.  Per-problem iterations,
 * relative residuals (|b - K_c x| / |b| at the end) and the time (ms, from the
 * call's start) at which the problem finished, into the host arrays (may be
 * NULL).  Synchronises.  Returns the first failing problem's status
 * (NOT_CONVERGED, BREAKDOWN, NOT_SPD, HIP); the others are solved. */
mfh_status mfh_batch_cg_solve(mfh_batch* batch, const double* const* b, double* const* x, double rtol,
                              int max_it, int* iters, double* relres, double* solve_ms);

/* ---- Kernel timers (measurement of the operator kernel) ---- */

/* enable != 0: from now on the cell kernels of every mfh_tangent_vmult are
 * bracketed by HIP events on the problem's stream (the output fill of the
 * atomic, colour and tile scatters is not included; with the ELEMENT scatter
 * the bracket holds the cell kernel and the node-sum kernel); enable == 0
 * stops recording.  Either call resets the totals. */
mfh_status mfh_timer_enable(mfh_problem* problem, int enable);
/* Synchronises and returns the summed duration (ms) and the number of the
 * timed cell-kernel launches since the last mfh_timer_enable. */
mfh_status mfh_timer_read(mfh_problem* problem, double* total_ms, long long* launches);

#ifdef __cplusplus
}
#endif

#endif /* MFH_H */
