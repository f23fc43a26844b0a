/*
 * libfsi: one time step of the distributed-Lagrange-multiplier fictitious-domain FSI
 * method (Boffi, Credali, Gastaldi, Scacchi, "A parallel solver for FSI problems with
 * fictitious domain approach"), on one AMD Instinct MI355X (gfx950).
 *
 * The library solves, at each step, the saddle-point system of Sec. 4, eq. (matrix):
 *
 *   [ A_f   -B^T    0            C_f^T ] [u]     [g1]
 *   [ -B     pin    0            0     ] [p]  =  [0 ]
 *   [ 0      0      A_s         -C_s   ] [X]     [0 ]
 *   [ C_f    0     -(1/dt) C_s   0     ] [lam]   [g2]
 *
 * with A_f = (rho/dt) M_f + K_f, K_f the form nu (eps(u), eps(v)), B the divergence,
 * A_s = kappa (grad, grad)_B, C_s the solid mass, C_f(X^n) the coupling (chi_l, phi_j(X^n))_B,
 * g1 = (rho/dt) M_f u^n, g2 = -(1/dt) C_s X^n.  GMRES is right-preconditioned by the
 * block-diagonal or block-triangular preconditioner of Sec. 5.
 *
 * Discretisation (readings where the paper leaves a choice):
 *  - fluid: [0,1]^2, n x n squares split along (i,j)->(i+1,j+1); P2 velocity, continuous
 *    P1 pressure; P2 node (I,J), 0<=I,J<=2n, has index J(2n+1)+I; P1 node (i,j) has
 *    index j(n+1)+i; homogeneous Dirichlet velocity on the whole boundary, imposed by
 *    value (rows/columns zeroed, 1 on the A_f diagonal); pressure pinned at P1 node 0
 *    ("pin" is 1 at (p0,p0), row 0 of B is zero);
 *  - solid: P1 triangles (CCW), X and lam both P1 on the solid mesh; A_s, C_s, C_f act on
 *    the two components separately.
 *
 * Unknown vector (FP64, N entries, structure of arrays):
 *   x = [u_x (N2) | u_y (N2) | p (Np) | X_x (Ns) | X_y (Ns) | lam_x (Ns) | lam_y (Ns)]
 * with N2 = (2n+1)^2, Np = (n+1)^2, Ns = number of solid nodes.
 *
 * Conventions of every call:
 *  - the return value is an fsi_status (0 = FSI_OK, negative = error); no C++ exception
 *    crosses this interface; fsi_last_error(ctx) gives a message for the last error;
 *  - host arrays given to fsi_create are copied and stay owned by the caller;
 *  - vector arguments are DEVICE pointers (FP64), owned by the caller, which keeps them
 *    valid until the work enqueued on the context's stream completes;
 *  - work is enqueued on the context's HIP stream (fsi_set_stream); calls that return
 *    statistics or counts synchronise that stream;
 *  - a context serves one host thread and one stream at a time;
 *  - on error outputs are unspecified, except FSI_E_NOCONV (x holds the last iterate and
 *    the statistics are filled in);
 *  - 32-bit indices: every matrix of a context must have fewer than 2^31 entries
 *    (n <= 4096 for the fluid blocks).
 */
#ifndef FSI_H
#define FSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsi_ctx fsi_ctx;

enum fsi_status {
  FSI_OK = 0,
  FSI_E_ARG = -1,        /* null pointer, size mismatch, unsupported value */
  FSI_E_MESH = -2,       /* degenerate/clockwise reference triangle, X^n(E) inverted or outside [0,1]^2 */
  FSI_E_NOMEM = -3,      /* device memory (or the given budget) exhausted */
  FSI_E_NOCONV = -4,     /* Krylov solve reached maxit */
  FSI_E_NONFINITE = -5,  /* NaN/Inf met in a residual */
  FSI_E_HIP = -6,        /* HIP runtime error */
  FSI_E_CAPACITY = -7,   /* a fixed capacity was exceeded (the allocation-free coupling assembly) */
  FSI_E_STATE = -8       /* call order: e.g. operator apply before fsi_assemble_coupling */
};

/* Arithmetic of a solve.  FSI_FP64: everything FP64.  FSI_FP32 (mixed): the inner block
 * solves' multigrid V-cycles, Chebyshev mass solves and Schur approximation in FP32 with
 * FP32 accumulation (the bulk of the bytes); Arnoldi, the operator, the A11 product of
 * the inner Krylov recurrence, A22, residuals and clipping in FP64.  FSI_FP32_IR: as
 * FSI_FP32 and the operator of the Arnoldi process in FP32 too, with iterative refinement
 * on the FP64 residual (an FP32 product loses about kappa * 6e-8 to cancellation on smooth
 * vectors, so each cycle gains only a few digits on fine grids).  fsi_apply_operator
 * takes FSI_FP64 or FSI_FP32 (operator in FP32 arithmetic). */
enum fsi_prec { FSI_FP64 = 0, FSI_FP32 = 1, FSI_FP32_IR = 2 };
enum fsi_pc { FSI_PC_DIAG = 0, FSI_PC_TRI = 1 };/* Sec. 5: block-diagonal / block-triangular */

/* Fluid: n x n grid on [0,1]^2 (n >= 2), viscosity nu, density rho (= solid density,
 * Sec. 3, Problem 2), time step dt. */
typedef struct {
  int32_t n;
  double nu, rho, dt;
} fsi_fluid_desc;

/* Solid reference mesh (host arrays, copied): xy = [x (n_nodes) | y (n_nodes)],
 * tri = 3 node ids per triangle, counter-clockwise; kappa of the law P(F) = kappa F. */
typedef struct {
  int32_t n_nodes, n_tris;
  const double *xy;
  const int32_t *tri;
  double kappa;
} fsi_solid_desc;

typedef struct {
  int64_t N2, Np, Ns, Nt, N;
  int64_t off_ux, off_uy, off_p, off_Xx, off_Xy, off_lx, off_ly;
  int64_t nnz_Af;   /* P2-P2 pattern entries (each carries xx, xy, yx, yy) */
  int64_t nnz_B;    /* P1-P2 pattern entries of B (each carries B_x, B_y) */
  int64_t nnz_s;    /* solid P1 pattern entries (A_s and C_s share it) */
  int64_t nnz_Cf;   /* C_f entries after the last fsi_assemble_coupling (0 before) */
  int64_t n_pairs;  /* intersection pieces after the last fsi_assemble_coupling */
  int64_t device_bytes;
  int32_t mg_levels_u, mg_levels_p;
} fsi_sizes_t;

typedef struct {
  int64_t n_pairs;  /* kept (solid triangle, fluid triangle) intersection pieces */
  int64_t nnz;      /* entries of the scalar C_f pattern */
} fsi_coupling_info;

/* The inner A11^{-1} (the paper inverts A11 exactly with a direct solver; here A11 =
 * [A_f, -B^T; -B, 0] is solved iteratively to inner_rtol, the outer solve being flexible, or
 * approximated at a fixed cost).  The building blocks: V, one P2 geometric-multigrid V-cycle
 * on A_f; S~^{-1} = nu M_p^{-1} + (rho/dt) L_p^{-1}, the Cahouet-Chabard approximation of the
 * inverse Schur complement (B A_f^{-1} B^T)^{-1}.
 *   FSI_INNER_MINRES (default): MINRES to inner_rtol (its preconditioned residual estimate)
 *     with the symmetric positive definite block-diagonal diag(V, S~^{-1}).
 *   FSI_INNER_GMRES: right-preconditioned restarted GMRES on A11 to
 *     ||D (r - A11 z)|| <= inner_rtol ||D r||, with the block upper-triangular approximation
 *     P^{-1}: z_p = -S~^{-1} r_p, z_u = V (r_u + B^T z_p) (the pinned pressure row: the
 *     identity); D weights the pressure rows by sqrt(a_u s_p), a_u the diagonal scale of
 *     A_f and s_p that of S~^{-1}, so that the norm weighs both blocks like MINRES's.
 *   FSI_INNER_FIXED_DIAG: one application of diag(V, -S~^{-1}), no inner Krylov steps.
 *   FSI_INNER_FIXED_TRI: inner_cycles steps of the stationary iteration
 *     z <- z + P^{-1} (r - A11 z) from z = 0, no inner Krylov steps.
 * The fixed-cost forms take more outer steps than the oracle's exact blocks. */
enum fsi_inner { FSI_INNER_MINRES = 0, FSI_INNER_FIXED_DIAG = 1, FSI_INNER_FIXED_TRI = 2, FSI_INNER_GMRES = 3 };

typedef struct {
  int32_t restart;      /* outer FGMRES restart length m (default 30) */
  int32_t maxit;        /* outer Arnoldi steps over all restarts (default 10000) */
  double rtol;          /* ||b - A x||_2 <= rtol ||b||_2 (default 1e-8, Sec. 6) */
  int32_t pc;           /* fsi_pc */
  int32_t prec;         /* fsi_prec */
  double inner_rtol;    /* relative tolerance of the inner A11 solve (0: default, 1e-2 with the
                           block-triangular, 1e-6 with the block-diagonal preconditioner) */
  int32_t inner_maxit;  /* inner Krylov steps per A11 solve (default 1000; 300 in FP32) */
  double cycle_rtol;    /* FSI_FP32_IR: residual reduction asked of each FGMRES cycle
                           (default 1e-5); ignored otherwise */
  int32_t inner_mode;   /* fsi_inner: how A11^{-1} is applied inside the block
                           preconditioners of Sec. 5.  Other values: FSI_E_ARG. */
  int32_t inner_cycles; /* FSI_INNER_FIXED_TRI: cycles per A11 application (0: 1; at most 100,
                           else FSI_E_ARG); ignored otherwise */
} fsi_solve_opts;

typedef struct {
  int32_t its;          /* outer Arnoldi steps, summed over restarts (and refinement cycles) */
  int32_t restarts;     /* outer cycles */
  int64_t inner_its;    /* inner MINRES steps, summed */
  int32_t converged;
  int32_t refinements;  /* FP64 true-residual cycles (mixed precision) */
  double relres_true;   /* ||b - A x|| / ||b|| recomputed in FP64 */
  double relres_est;
  double t_coup, t_rhs, t_solve;  /* seconds (stream-synchronised wall time) */
} fsi_solve_stats;

/* Blocks exported by fsi_export_csr (host copies, for tests). */
enum fsi_block {
  FSI_BLK_AF = 0,   /* A_f, BC applied: width 4 (xx, xy, yx, yy) on the P2-P2 pattern */
  FSI_BLK_MF = 1,   /* M_f, no BC: width 1, same pattern */
  FSI_BLK_B = 2,    /* B, BC + pin applied: width 2 (B_x, B_y), rows P1, columns P2 */
  FSI_BLK_BT = 3,   /* B^T stored explicitly: width 2, rows P2, columns P1 */
  FSI_BLK_AS = 4,   /* A_s = kappa K_s: width 1, solid pattern */
  FSI_BLK_CS = 5,   /* C_s: width 1, solid pattern */
  FSI_BLK_CF = 6,   /* C_f(X^n): width 1, rows solid nodes, columns P2 nodes */
  FSI_BLK_CFT = 7,  /* C_f^T: width 1, rows P2 nodes, columns solid nodes */
  FSI_BLK_MP = 8,   /* pressure mass (used by the preconditioner): width 1, P1-P1 */
  FSI_BLK_KT = 9    /* solid tangent K(X) of the last fsi_solid_tangent: width 4 (xx, xy, yx, yy) on
                       the solid pattern; FSI_E_STATE before one */
};

/* Build the time-independent blocks (Sec. 4: A_f, B, A_s, C_s), the multigrid
 * hierarchies of the preconditioner and all work space on the current HIP device.
 * hip_stream: a hipStream_t (NULL = default stream).  hbm_budget: maximum device
 * bytes the context may hold (0 = no limit); FSI_E_NOMEM if the footprint exceeds it.
 * The hierarchies halve n while it is even and above 4 and solve their last level densely
 * (from n = 512 the velocity levels end on the first of 16 x 16 cells or fewer instead).
 * Errors: FSI_E_ARG (n outside [2, 4096], or a dense coarsest level of more than 6,000
 * unknowns, 8,192 for the velocity levels from n = 512, such as the single level of an odd
 * n above 25), FSI_E_MESH (a reference triangle with area <= 0), FSI_E_NOMEM, FSI_E_HIP. */
int fsi_create(const fsi_fluid_desc *fluid, const fsi_solid_desc *solid, void *hip_stream,
               size_t hbm_budget, fsi_ctx **out);

/* The paper's own element pair (Sec. 4, the discrete spaces).  fsi_create_q2 makes a context
 * of the Q2 / P1-disc fluid and the Q1 solid; every later call of this interface takes it
 * except those that name the triangle pair's kernels (fsi_set_solid, fsi_set_smoother with
 * FSI_SMOOTH_STENCIL, fsi_set_coupling_mode with FSI_COUPLING_INCREMENTAL,
 * fsi_assemble_coupling_noalloc, fsi_step_batch, fsi_set_law with another law,
 * fsi_solid_residual, fsi_solid_tangent, fsi_newton_step, inner modes other than
 * FSI_INNER_MINRES), which return FSI_E_STATE.
 *  - fluid: the n x n squares (no diagonal), Q2 velocity on the same node lattice as the P2
 *    velocity (node (I,J) has index J(2n+1)+I); discontinuous P1 pressure with Np = 3 n^2
 *    unknowns: on cell (i,j), k = j n + i, the unknowns 3k, 3k+1, 3k+2 are the coefficients
 *    of 1, (x - x_c)/h, (y - y_c)/h (x_c, y_c the cell centre); pinned at unknown 0;
 *    boundary conditions as for the triangle pair;
 *  - solid: solid->tri holds 4 node indices per quadrilateral (counter-clockwise, strictly
 *    convex) and n_tris counts the quadrilaterals; X and lam are bilinear on each (S_h = Lambda_h);
 *  - C_f(X^n): each mapped quadrilateral X^n(E) (strictly convex and counter-clockwise, else
 *    FSI_E_MESH) clipped against the cells of its bounding box; the integral over a piece by
 *    the inverse of the bilinear map, on the fan of the piece with 4 x 4 conical Gauss points
 *    per fan triangle (exact when X^n is affine on E); fsi_export_pairs gives (E, cell j n + i);
 *  - the A11 preconditioner: V-cycles on the assembled operators (no matrix-free form):
 *    velocity on the Q2 A_f of every level, and the Cahouet-Chabard approximation
 *    nu M_p^{-1} + (rho/dt) L^{-1} with L = B D^{-1} B^T (D the row sums of M_f) re-formed on
 *    every level and the P1-disc prolongation between levels.
 * hbm_budget: checked against the device footprint after creation (0: none).
 * Errors as for fsi_create; FSI_E_MESH also for a reference quadrilateral that is not
 * strictly convex and counter-clockwise. */
enum fsi_pair { FSI_PAIR_P2P1 = 0, FSI_PAIR_Q2P1DISC = 1 };
int fsi_create_q2(const fsi_fluid_desc *fluid, const fsi_solid_desc *solid, void *hip_stream, size_t hbm_budget,
                  fsi_ctx **out);
void fsi_destroy(fsi_ctx *ctx);

/* Replace the solid mesh of an existing context (fluid blocks and multigrid are kept).
 * Device buffers only grow, so re-meshing with a solid no larger than any earlier one
 * allocates nothing: this lets a request loop keep one context per slot resident.  The
 * coupling must be assembled again afterwards.  Errors: FSI_E_ARG, FSI_E_MESH, FSI_E_NOMEM. */
int fsi_set_solid(fsi_ctx *ctx, const fsi_solid_desc *solid);
int fsi_set_stream(fsi_ctx *ctx, void *hip_stream);

/* Device bytes a context for this fluid grid and a solid of n_nodes / n_tris would hold
 * (the estimate fsi_create checks against its budget); for admission control. */
int fsi_footprint(const fsi_fluid_desc *fluid, int64_t n_nodes, int64_t n_tris, size_t *bytes);
int fsi_sizes(const fsi_ctx *ctx, fsi_sizes_t *out);

/* C_f(X^n) and its transpose (Sec. 4, the coupling assembly): the mapped solid triangles
 * X^n(E) are clipped (Sutherland-Hodgman) with the fluid triangles of the cells in their
 * bounding box; each kept piece is integrated exactly (the integrand is cubic).
 * Xn: device, 2 Ns doubles [x | y].  info may be NULL (then no synchronisation).
 * Each C_f row (solid node) is assembled in a window of the P2 lattice nodes its pieces touch:
 * in LDS up to 4,096 nodes, in device memory above (a solid much coarser than the fluid
 * grid; one wavefront per such row), with the same fixed order of the sums.
 * Errors: FSI_E_MESH if some X^n(E) has area <= 0 or leaves [0,1]^2 (detected on the
 * device, reported at the next synchronising call or here when info != NULL). */
int fsi_assemble_coupling(fsi_ctx *ctx, const double *Xn, fsi_coupling_info *info);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * allocation): fsi_assemble_coupling without any device allocation or release.  It builds the
 * same C_f(X^n) and C_f^T, bitwise, but carves every work array of the assembly (candidate
 * offsets, piece counters, scan partials, the piece list with its local matrices, transpose
 * staging and counters, deferred-row lists, the device-memory window of rows above 4,096
 * lattice nodes, error flags) from one static device array of
 * FSI_COUPLING_SCRATCH_BYTES per GPU, whose address the library takes once per device in
 * fsi_create.  Outputs go to the context's coupling storage: reserved by fsi_create and
 * fsi_set_solid for 64 entries per solid node, grown only by fsi_assemble_coupling.
 * Xn, info: as fsi_assemble_coupling.  The call synchronises the context's stream (it reads
 * the piece and entry counts), like fsi_assemble_coupling.
 * Errors: those of fsi_assemble_coupling, and FSI_E_CAPACITY when the work space exceeds the
 * scratch array or C_f has more entries than the context's storage holds (nothing is
 * allocated; the context then has no C_f until the next successful assembly).
 * The scratch array is shared by every context on the GPU and keeps the last call's contents:
 * calls that overlap on one GPU (other streams or host threads) race, so the caller
 * serialises them.  fsi_export_pairs after this call returns FSI_E_STATE (the piece list stays
 * in the scratch array). */
#define FSI_COUPLING_SCRATCH_BYTES (32u << 20)
int fsi_assemble_coupling_noalloc(fsi_ctx *ctx, const double *Xn, fsi_coupling_info *info);

/* How fsi_assemble_coupling (and the steps that call it) finds the intersections.  The paper
 * detects them anew at every step and proposes, against the cost of that search, to keep track
 * of the solid's position at the previous time step (Sec. 7).
 *  FSI_COUPLING_FULL: every call detects, clips and builds the pattern from scratch (default).
 *  FSI_COUPLING_INCREMENTAL: the context keeps, from one call to the next, each solid
 *    triangle's candidate box (its bounding box in fluid cells grown by one cell in x and y, two
 *    piece slots per cell), the positions of the last call, the C_f pattern and the
 *    permutation of C_f^T.  A call re-clips only the triangles with a vertex that moved (any
 *    coordinate differs from the last call's), into their own slots; it keeps C_f when nothing
 *    moved, refills only the values (pattern, C_f^T order kept) when every moved triangle kept
 *    the same pieces, builds rows and transpose anew when one did not, and rebuilds boxes and
 *    slots when a triangle outgrew its box (and on the first call, after fsi_set_solid, after a
 *    call that failed, or after fsi_assemble_coupling_noalloc).  The result is bitwise that of FSI_COUPLING_FULL:
 *    the same pieces in the same order, the same sums in the same order.  Extra device memory:
 *    the slots hold (w + 1)(h + 1) cells per triangle instead of w h, their previous pieces,
 *    2 Ns doubles, 3 Nt ints and two ints per C_f entry.
 * Errors: FSI_E_ARG (unknown mode).  A change of mode drops the kept state. */
enum fsi_coupling_mode { FSI_COUPLING_FULL = 0, FSI_COUPLING_INCREMENTAL = 1 };
int fsi_set_coupling_mode(fsi_ctx *ctx, int mode);

/* What the FSI_COUPLING_INCREMENTAL calls of a context did (cumulative, host-side counts). */
typedef struct {
  int64_t calls;           /* assemblies in the incremental mode */
  int64_t rebuilds;        /* boxes and slots built (first call, overflow, after fsi_set_solid...) */
  int64_t pattern_builds;  /* moved triangles re-clipped, some pieces changed: rows and transpose anew */
  int64_t value_refills;   /* moved triangles re-clipped, the same pieces: values only */
  int64_t unchanged;       /* nothing moved: C_f kept */
} fsi_coupling_counts;
int fsi_get_coupling_counts(const fsi_ctx *ctx, fsi_coupling_counts *out);

/* (g1, 0, 0, g2) of eq. (matrix): g1 = (rho/dt) M_f u^n with boundary rows zero (u^n is
 * taken as zero on the boundary), g2 = -(1/dt) C_s X^n.  u_n: device 2 N2, X_n: device
 * 2 Ns, b: device N. */
int fsi_build_rhs(fsi_ctx *ctx, const double *u_n, const double *X_n, double *b);

/* y = A x with the full operator of eq. (matrix) (needs fsi_assemble_coupling).
 * prec = FSI_FP32 rounds x and the matrix values to FP32, accumulates in FP32 and
 * writes FP64.  FSI_FP64 with the structured-grid products on (fsi_set_smoother,
 * default) computes the fluid rows matrix-free (A_f, B, B^T from the element matrices;
 * C_f^T from its CSR).  x, y: device N (no aliasing). */
int fsi_apply_operator(fsi_ctx *ctx, int prec, const double *x, double *y);

/* z = P^{-1} r, P = diag(A11, A22) or [[A11, 0], [A21, A22]] (Sec. 5).  A22^{-1} in
 * closed form (two solid mass solves and one A_s product); A11^{-1} by the context's inner
 * mode (fsi_set_inner_mode, default FSI_INNER_MINRES) to its inner tolerance
 * (fsi_set_inner).  r, z: device N (no aliasing). */
int fsi_apply_precond(fsi_ctx *ctx, int pc, int prec, const double *r, double *z);
/* The context's inner tolerance (<= 0: the default of the preconditioner) and step limit
 * (0: unchanged; negative: FSI_E_ARG). */
int fsi_set_inner(fsi_ctx *ctx, double inner_rtol, int32_t inner_maxit);
/* The context's inner mode (fsi_inner) and FSI_INNER_FIXED_TRI cycles (0: 1; at most 100),
 * used by fsi_apply_precond; a solve takes both from its options.  Errors: FSI_E_ARG. */
int fsi_set_inner_mode(fsi_ctx *ctx, int32_t mode, int32_t cycles);

/* Right-preconditioned flexible GMRES(m) on eq. (matrix) from the initial guess in x,
 * stopping when ||b - A x||_2 <= rtol ||b||_2 (Sec. 6, recomputed in FP64); precision
 * forms as in fsi_prec.  b, x: device N.  stats may be NULL.
 * Errors: FSI_E_NOCONV, FSI_E_NONFINITE, FSI_E_STATE. */
int fsi_gmres_solve(fsi_ctx *ctx, const fsi_solve_opts *opts, const double *b, double *x,
                    fsi_solve_stats *stats);

/* One semi-implicit step (Sec. 4, Problem 3): fsi_assemble_coupling(X_n), fsi_build_rhs,
 * then fsi_gmres_solve from x = 0.  u_n: device 2 N2, X_n: device 2 Ns, state: device N
 * (u, p, X, lam at n+1). */
int fsi_step(fsi_ctx *ctx, const fsi_solve_opts *opts, const double *u_n, const double *X_n,
             double *state, fsi_solve_stats *stats);

/* K independent steps in lockstep (a batch of small requests): system k is
 * fsi_step(ctxs[k], opts, u_n[k], X_n[k], state[k], &stats[k]), and its result is bitwise
 * the result of that call.  The contexts share the fluid grid and fluid parameters (n, nu,
 * rho, dt) and have their own solids.  Every kernel runs on ctxs[0]'s stream (the other
 * contexts' streams are synchronised, set to it for the call and restored); the inner A11
 * solves of all systems run as K lanes of the same launches (lane = second grid dimension)
 * on ctxs[0]'s inner work space and with its inner and smoother settings, so a batch issues
 * about as many launches as one step.  ctxs[0] keeps inner work space for K systems
 * (grow-only; growing it drops its captured graphs).
 * K: 1..FSI_MAX_LANES; ctxs: host array of K distinct contexts; u_n, X_n, state: host arrays
 * of K device pointers (sizes as in fsi_step); stats: host array of K (may be NULL); rc: host
 * array of K per-system statuses, FSI_OK / FSI_E_NOCONV / FSI_E_NONFINITE (may be NULL).
 * Returns FSI_OK when every system converged, else the status of the first system that did
 * not (its message in fsi_last_error(ctxs[0])).  Any other error (FSI_E_ARG, FSI_E_MESH,
 * FSI_E_CAPACITY, FSI_E_HIP, ...) fails the whole batch; outputs are then unspecified. */
#define FSI_MAX_LANES 32
int fsi_step_batch(int32_t K, fsi_ctx *const *ctxs, const fsi_solve_opts *opts, const double *const *u_n,
                   const double *const *X_n, double *const *state, fsi_solve_stats *stats, int32_t *rc);

/* ---- nonlinear solid (Sec. 4, last paragraph: a nonlinear law P(F) is solved by Newton's
 * method; Sec. 6.2: the exponential law of the nonlinear test).
 * FSI_LAW_LINEAR: P(F) = kappa F (kappa of the solid descriptor), the law of eq. (matrix).
 * FSI_LAW_EXP: W(F) = (gamma / (2 eta)) exp(eta (tr F^T F - 2)), P(F) = dW/dF =
 *   gamma exp(eta (|F|^2 - 2)) F (the paper's gamma = 1.333, eta = 9.242; eta = 0 is the linear
 *   law with kappa = gamma).
 * The solid row of a step becomes (P(F_h^{n+1}), grad_s Y_h)_B - (lam_h^{n+1}, Y_h)_B = (f, Y_h):
 * with P1 triangles the residual R(X)_{l,a} = sum_E |E| P_ab(F_E) (grad chi_l)_b and its tangent
 * K(X) = dR/dX (2 x 2 blocks on the solid pattern) replace A_s X and A_s.  Vectors [x | y]. */
enum fsi_law { FSI_LAW_LINEAR = 0, FSI_LAW_EXP = 1 };

/* Select the solid law of the context (default FSI_LAW_LINEAR).  gamma > 0, eta >= 0 for
 * FSI_LAW_EXP (ignored for the linear law).  Errors: FSI_E_ARG. */
int fsi_set_law(fsi_ctx *ctx, int law, double gamma, double eta);

/* R(X) of the context's law at the solid position X (device, 2 Ns) into R (device, 2 Ns).
 * Errors: FSI_E_ARG. */
int fsi_solid_residual(fsi_ctx *ctx, const double *X, double *R);

/* Assemble the tangent K(X) (X device, 2 Ns) and use it in place of A_s in fsi_apply_operator,
 * fsi_apply_precond, fsi_gmres_solve and fsi_step (the Jacobian of a Newton iteration) until the
 * next call; X = NULL returns to A_s.  Batched steps (fsi_step_batch) always use A_s. */
int fsi_solid_tangent(fsi_ctx *ctx, const double *X);

typedef struct {
  double rtol;      /* stop when ||G(x_k)|| <= rtol ||G(x_0)|| (Sec. 6: 1e-6) */
  int32_t maxit;    /* Newton iterations at most (default 50) */
} fsi_newton_opts;

typedef struct {
  int32_t nit;          /* Newton iterations (Jacobian solves) */
  int32_t converged;
  int32_t its_total;    /* outer GMRES steps summed over the Jacobian solves */
  int64_t inner_its;    /* inner MINRES steps, summed */
  double res0, res;     /* ||G(x_0)||, ||G(x_nit)|| */
  double t_coup, t_res, t_solve;   /* seconds: C_f assembly, residuals, Jacobian solves */
} fsi_newton_stats;

/* One step of Problem 3 with the context's law by Newton's method (Sec. 4): the system
 * G(x) = 0, eq. (matrix) with A_s X replaced by R(X), C_f(X^n) assembled once, right-hand side
 * (g1, 0, f_X, g2); each iteration solves J(x_k) d = -G(x_k) with J the matrix of eq. (matrix)
 * whose A_s block is K(X_k), by fsi_gmres_solve with opts (the Jacobian tolerance opts->rtol,
 * Sec. 6: 1e-8), and sets x_{k+1} = x_k + d, until ||G(x_k)|| <= nopts->rtol ||G(x_0)||.
 * u_n: device 2 N2; X_n: device 2 Ns; f_X: device 2 Ns load on the solid nodes, or NULL;
 * state: device N, in: the initial guess x_0 (e.g. (u^n, 0, X^n, 0) or the previous step), out:
 * x at n+1.  The solid block returns to what it was before the call.  stats may be NULL.
 * Errors: FSI_E_NOCONV (Newton or a Jacobian solve did not converge; state holds the last
 * iterate), FSI_E_NONFINITE, FSI_E_MESH, FSI_E_ARG. */
int fsi_newton_step(fsi_ctx *ctx, const fsi_solve_opts *opts, const fsi_newton_opts *nopts, const double *u_n,
                    const double *X_n, const double *f_X, double *state, fsi_newton_stats *stats);

/* Test exports (host copies; synchronising).  fsi_export_pairs writes up to cap pieces
 * (solid triangle E, fluid triangle T) in the canonical order (by E, then cell j-major,
 * then T) and stores the total in *count.  fsi_export_csr: call with NULL arrays to get
 * nrows, nnz and width (values per entry); then rowptr (nrows+1), col (nnz) and
 * val (nnz*width) are filled. */
int fsi_export_pairs(fsi_ctx *ctx, int32_t *E, int32_t *T, int64_t cap, int64_t *count);
int fsi_export_csr(fsi_ctx *ctx, int block, int64_t *nrows, int64_t *nnz, int32_t *width,
                   int32_t *rowptr, int32_t *col, double *val);

/* Test export, host only (no context, no device): the coefficient tables of the
 * matrix-free products on an n x n grid (fsi_set_smoother), built as the library builds
 * them, so tests can compare them with independently assembled matrices.  rdt = rho / dt
 * (FSI_LAT_AF only), nu the viscosity (FSI_LAT_AF only).  Output, row-major over
 * (class, entry) with FSI_LAT_MAX_ENTRIES entries per class and unused entries zero:
 * counts[9] entries per class; offs[9 * 81 * 2] lattice offsets (dI, dJ); vals[9 * 81 * 4].
 *   FSI_LAT_AF: A_f = (rho/dt) M_f + K_f at interior P2 nodes, classes by parity
 *               (bit 0: I odd, bit 1: J odd); offsets in P2 lattice units; vals = the 2x2
 *               block (xx, xy, yx, yy).
 *   FSI_LAT_LP, FSI_LAT_MP: P1 Laplacian with node 0 pinned (identity row, zero column) and
 *               P1 mass; classes 3 cj + ci by position (0: first, 1: interior, 2: last index);
 *               7 entries each at offsets (0,0), (-1,0), (1,0), (0,-1), (0,1), (-1,-1), (1,1);
 *               vals[.][0] = coefficient (zero where the neighbour is outside the lattice).
 *   FSI_LAT_BT: rows of B^T (Dirichlet BC, pin) at interior P2 nodes by parity class;
 *               offsets of P1 nodes from (I >> 1, J >> 1); vals = (B_x, B_y).
 *   FSI_LAT_B:  the B row of a P1 node (i, j) (class 0 only); offsets of P2 nodes from
 *               (2i, 2j); vals = (B_x, B_y); Dirichlet columns are applied by the caller.
 *   FSI_LAT_R:  P2 restriction R = P^T at interior coarse nodes by parity class; offsets of
 *               fine nodes from (2 Ic, 2 Jc) in fine lattice units; vals[.][0] = weight.
 *   FSI_LAT_Q2AF: A_f of the paper's element pair (Q2 on squares, fsi_create_q2) at interior
 *               nodes by parity class (vertex, x-edge, y-edge, centre: 25, 15, 15, 9 entries);
 *               offsets and vals as FSI_LAT_AF.
 * Errors: FSI_E_ARG (n outside [2, 4096], unknown table, null buffer). */
enum fsi_lattice_table { FSI_LAT_AF = 0, FSI_LAT_LP = 1, FSI_LAT_MP = 2, FSI_LAT_BT = 3, FSI_LAT_B = 4,
                         FSI_LAT_R = 5, FSI_LAT_Q2AF = 6 };
#define FSI_LAT_MAX_ENTRIES 81
int fsi_export_lattice(int32_t n, double nu, double rdt, int32_t table, int32_t *counts, int32_t *offs,
                       double *vals);

/* Products inside the A11 preconditioner (both multigrid hierarchies and the pressure
 * mass solve): FSI_SMOOTH_STENCIL (default) applies them matrix-free on the structured
 * grid: A_f from four translation-invariant 2x2-block stencils (boundary rows identity,
 * boundary columns zero), L_p and M_p from 7-point stencils in nine position classes
 * (L_p: pinned node identity row, zero column), and the P2 / P1 prolongations and
 * restrictions from the nested refinement, all with the same element matrices and
 * interpolation weights as the assembled operators.  FSI_SMOOTH_CSR reads the assembled
 * matrices.  The same switch selects the matrix-free fluid rows of the FP64 operator
 * (A11 in the inner solves and fsi_apply_operator).  Both settings give the same results
 * up to the order of the sums. */
enum fsi_smoother { FSI_SMOOTH_CSR = 0, FSI_SMOOTH_STENCIL = 1 };
int fsi_set_smoother(fsi_ctx *ctx, int kind);

/* Replay the A11 preconditioner (V-cycles, Chebyshev mass solve, pressure V-cycle) and the
 * inner MINRES steps as captured HIP graphs.  Default: off.  A graph keeps the pressure part
 * on the context's stream (without it, that part runs on a second stream beside the velocity
 * cycle) and the inner solve checks convergence every 2 steps (frozen steps past
 * convergence); with the coarse ends of both multigrid cycles in one launch each, the two
 * streams measured faster at every grid size.  The graph holds kernel nodes only; results
 * are the same as without it. */
int fsi_set_graphs(fsi_ctx *ctx, int enable);

/* When the inner MINRES solve learns that it has converged (without graphs).
 *  FSI_CHECK_AUTO (default): FSI_CHECK_LAGGED on grids of n <= 256, FSI_CHECK_EVERY_STEP above.
 *  FSI_CHECK_EVERY_STEP: the state of each step is copied back and the host waits for it
 *    before it enqueues the next step (the device idles for that round trip).
 *  FSI_CHECK_LAGGED: the state of step k - 1 is read after step k has been enqueued, so the
 *    device does not wait for the host; the step enqueued past convergence is frozen by the
 *    device-side done flag (the same results, bitwise; one extra step of work per solve).
 *    Faster for one solve on an idle device (32^2-256^2: 4-15% per step), slower where other
 *    streams keep the device busy (the request loop of serve.py measured 141-147 against 151
 *    requests/s), where the extra step takes time from the other work.
 * Errors: FSI_E_ARG (unknown mode). */
enum fsi_check_mode { FSI_CHECK_AUTO = 0, FSI_CHECK_EVERY_STEP = 1, FSI_CHECK_LAGGED = 2 };
int fsi_set_inner_check(fsi_ctx *ctx, int mode);

/* Measurement of the dominant kernel, the finest-level Chebyshev smoothing on A_f
 * (d = c1 d + c2 D^{-1}(b - A_f x), y = x + d on the 2x2-block system): with the
 * structured-grid products (default) the launch that takes the post-smoothing steps at
 * once (three for the default degree 3, temporal blocking); with FSI_SMOOTH_CSR every
 * single-step launch.
 * fsi_profile(ctx, 1) starts (and resets) timing every such launch with a pair of HIP
 * events on the context's stream; fsi_profile(ctx, 0) stops.  fsi_profile_read
 * synchronises and returns, for precision prec, the number of timed launches, their summed
 * duration in milliseconds and the algorithmic bytes one launch must move, with w = 8
 * (FP64) or 4 (FP32) bytes: structured form 6 w N2 for the default degrees 2 and 3 (x and
 * b read, y written, two components each: the first step has c1 = 0 and reads no d, and
 * the last direction is not stored when no single step follows; 8 w N2 when one does),
 * in FP32 with three steps (4 w + 16) N2 (y is stored straight into the FP64
 * preconditioner output); with three or more steps the launch also reads the coarse
 * correction, 2 w N2c (N2c = (n + 1)^2 nodes of the next level).  Inside the inner MINRES
 * the FP32 launch also reads the FP64 residual for its tile sums of r . z (16 N2 bytes,
 * not counted here: the figure is that of the smoothing itself); CSR form
 * nnz (4 w + 4) + N2 (4 + 14 w) + 4 (values and column indices once; per node the row
 * pointer, x, b, d read and written, the inverse 2x2 diagonal block and y). */
int fsi_profile(fsi_ctx *ctx, int enable);
int fsi_profile_read(fsi_ctx *ctx, int prec, int64_t *launches, double *total_ms,
                     double *bytes_per_launch);

const char *fsi_strerror(int status);
const char *fsi_last_error(const fsi_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
