/*
 * mfpsi -- matrix-free multi-body stream-function solver for AMD MI355X (gfx950).
 *
 * C ABI of libmfpsi.so.  The method is that of Sadasivan & Yadav, "A Computational
 * Approach for Multi-Body Potential-Flow Interaction Effects Using Matrix-Free FEM and
 * Body-Conforming Grids":
 *
 *   mfp_mesh_conform   section "Body-Conforming Grid Generation" (projection of
 *                      just-inside nodes, displacement d_ik = x_ik - x_gk, Laplacian
 *                      propagation of d, x_new = x_old + d);
 *   mfp_psi_solve      sections "Governing Equation", "Boundary Conditions",
 *                      "Weak formulation", "Matrix-Free Conjugate Gradient with Multiple
 *                      Constraint Enforcement", Algorithm 1 (appendix), "Velocity Field
 *                      and Surface Tangential Velocity", and the CoPFI definition of
 *                      "Effect of Gap Ratio";
 *   mfp_phi_solve      section "Governing Equation": the velocity potential phi
 *                      (u = grad phi, Laplace equation), whose contours and those of
 *                      psi form the flow net, on the same mesh and operator;
 *   mfp_cubic_fit      the cubic fit of CoPFI over the gap ratio ("Effect of Gap
 *                      Ratio");
 *   mfp_contour        contour lines of psi or phi: the flow net and the stagnation
 *                      streamlines of the transverse cylinders ("Effect of Gap Ratio");
 *   mfp_element_apply  the matrix-free element product of Algorithm 1 on its own;
 *   mfp_psi_solve_kutta  the trailing-edge (Kutta) constraint of section "Boundary
 *                      Conditions": psi at an added fluid point equals psi_b;
 *   mfp_mixed_*        the mixed-cell variant of the body-conforming grid (cut points
 *                      on the grid lines, triangles and quadrilaterals) with its
 *                      element product and constrained solve;
 *   mfp_psi_grad / mfp_mesh_conform_grad
 *                      the adjoint of that map (the automated sensitivity analysis named
 *                      in the Conclusions as the next step).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - Background grid: nx x ny cells, (nx+1)(ny+1) nodes; node (i, j) sits at
 *   x0 + i*hx, y0 + j*hy with hx = (x1-x0)/nx, hy = (y1-y0)/ny; flat node id
 *   j*(nx+1) + i (x fastest).
 * - Pointers named *_h are HOST memory.  Every other array pointer is DEVICE memory
 *   owned by the caller; the library never allocates, frees or keeps them.
 * - Displacements are stored component-major: disp[0 .. n) = x, disp[n .. 2n) = y,
 *   n = (nx+1)(ny+1).
 * - Scratch memory comes from the caller's workspace (ws, ws_bytes), at least the
 *   size reported by the matching *_workspace_size call, 256-byte aligned.  Its
 *   contents on entry are ignored.
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  All device work is
 *   enqueued on it.  Calls that report host-side results (psi_b_h, stats_h, ...)
 *   synchronise that stream before returning; mfp_mesh_conform and mfp_element_apply
 *   synchronise it only to read their error flags.
 * - Return value: 0 = MFP_OK, > 0 = warning (results written), < 0 = error (outputs
 *   unspecified).  mfp_last_error() returns a thread-local message for the last
 *   non-zero status of the calling thread.  No C++ exception crosses the ABI.
 * - One call at a time per workspace; calls with distinct workspaces may overlap on
 *   different streams.
 */
#ifndef MFPSI_H
#define MFPSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
#define MFP_OK 0
#define MFP_W_NOCONV 1      /* kmax reached before the tolerance                     */
#define MFP_W_STAGNATION 2  /* FP32 inner solves stalled; FP64 iterations finished it */
#define MFP_E_ARG -1        /* invalid argument (NULL pointer, bad size, bad code)    */
#define MFP_E_HIP -2        /* a HIP runtime call failed                              */
#define MFP_E_GEOMETRY -3   /* circles overlap, touch the outer band or are < 2 cells */
#define MFP_E_TANGLED -4    /* a Gauss-point Jacobian of an active cell is <= 0       */
#define MFP_E_BREAKDOWN -5  /* CG breakdown: p.Ap <= 0 or not finite                  */
#define MFP_E_WORKSPACE -6  /* workspace too small                                    */

/* ---- node kinds written by mfp_mesh_conform ---------------------------------------- */
#define MFP_FLUID 0   /* not inside any body                                           */
#define MFP_SNAPPED 1 /* body node with a fluid node among its 8 neighbours: on Gamma_i */
#define MFP_DEEP 2    /* body node with no fluid neighbour: stays put                    */

/* ---- side boundary conditions (side order: left, right, bottom, top) -------------- */
#define MFP_BC_NATURAL 0       /* zero normal derivative of the field: nodes stay unknowns */
#define MFP_BC_DIRICHLET_UY 1  /* psi = U * y                                            */
#define MFP_BC_DIRICHLET_CYL 2 /* psi = U (y-cy)(1 - a^2/rho^2) about circle 0 (tests)   */
#define MFP_BC_DIRICHLET_UX 3  /* phi = U * x (free-stream potential)                    */
#define MFP_BC_DIRICHLET_CYLPHI 4 /* phi = U (x-cx)(1 + a^2/rho^2) about circle 0 (tests) */

/* ---- solver precisions ------------------------------------------------------------ */
#define MFP_FP64 0    /* FP64 vectors and FP64 element apply                           */
#define MFP_FP32 1    /* FP32 vectors and apply; FP64 scalars and body sums            */
#define MFP_FP32_IR 2 /* FP32 CG with FP64 residual recomputation and FP64 accumulation
                         of the solution (iterative refinement, Krylov space kept)      */

#define MFP_MAX_BODIES 64

typedef struct {
  int32_t nx, ny;         /* cells in x and y, each >= 2                                */
  double x0, x1, y0, y1;  /* domain, x1 > x0, y1 > y0                                   */
} mfp_grid;

typedef struct {
  double cx, cy, r;       /* circle centre and radius                                   */
} mfp_circle;

typedef struct {
  double U;               /* free-stream speed                                          */
  int32_t side_bc[4];     /* MFP_BC_* for left, right, bottom, top                      */
} mfp_flow;

typedef struct {
  int32_t precision;      /* MFP_FP64 / MFP_FP32 / MFP_FP32_IR                          */
  double rtol;            /* stop when ||r_k|| <= rtol ||b|| (unknowns incl. bodies)    */
  int64_t kmax;           /* CG iteration cap (all inner iterations together)           */
  int32_t check_every;    /* iterations per enqueued batch (0 -> 16); the host reads a
                             batch's stop flag while the next batch runs, so an outcome
                             costs at most one batch of launches that return at once    */
  double inner_rtol;      /* MFP_FP32_IR: residual reduction of the FP32 iteration between
                             FP64 residual recomputations (0 < delta < 1; 0 -> 0.1)     */
  int32_t max_outer;      /* MFP_FP32_IR: cap on FP64 residual recomputations (0 -> 1000) */
  const double* psi0;     /* optional DEVICE warm start: nodal psi (free nodes) and the
                             first node of each body (row-major) for psi_b; may be NULL.
                             rtol stays relative to ||b|| (the residual of a zero start),
                             so a better start means fewer iterations to the same target,
                             unless rtol_from_start is set                             */
  int32_t profile_every;  /* > 0: time every n-th batch of iteration launches with HIP
                             events (between the events that end it and the batch
                             before it) -> stats.apply_ms                              */
  int32_t estimate_kappa; /* != 0: fill stats.kappa_est (see mfp_stats); costs one copy
                             of the CG scalars to the host and a host eigenvalue search */
  int32_t rtol_from_start;/* != 0 with psi0: stop at rtol ||b - A psi0|| instead (a
                             correction solve: from a nearby solution, e.g. one step of a
                             parameter sweep or a finite difference, this reaches an
                             absolute accuracy below what rtol ||b|| allows)            */
  /* Schedule of the iteration kernel; 0 = automatic: the entry for this device, grid
   * and precision in the tuning cache (written by the package's tuner): the file named
   * by the environment variable MFP_TUNE_CACHE, else tune_cache.txt beside
   * libmfpsi.so ("none" switches the cache off), else built-in rules.  The result
   * does not depend on the schedule beyond rounding.                                 */
  int32_t task_rows;      /* node rows per task: 4, 5 or 8                              */
  int32_t element_mode;   /* 1: element geometry on the fly from the displacements every
                             iteration; 2: each distorted cell's element matrix evaluated
                             once per solve (same 2x2 Gauss rule) and its six
                             off-diagonal entries read by the iteration (more bytes, far
                             fewer operations)                                          */
  int32_t store_mode;     /* 1: cached vector stores; 2: streaming (non-temporal) stores */
  int32_t launch_blocks;  /* work-groups per iteration launch (multiple of 8, <= 1024)  */
  int32_t batch_tasks_per_wave; /* mfp_psi_solve_batched: tasks per wavefront of the
                             batched iteration (1..64; its launch holds many systems)   */
} mfp_solver_opts;

typedef struct {
  int64_t iters;          /* CG iterations (inner + FP64)                               */
  int64_t outer_iters;    /* refinement steps (MFP_FP32_IR), else 0                     */
  int64_t applies;        /* element-operator applications (all precisions)             */
  int64_t n_dof;          /* N_int + N_N + N_b                                          */
  int64_t n_free;         /* N_int + N_N                                                */
  double relres_true;     /* ||b - A x|| / ||b|| recomputed in FP64 at the end          */
  double rnorm0;          /* ||b|| (the residual of a zero start)                       */
  double solve_ms;        /* device time of the iteration phase (HIP events)            */
  double apply_ms;        /* mean time per iteration launch in the timed batches        */
  int64_t apply_samples;  /* launches behind apply_ms                                   */
  int64_t n_plain_tiles;  /* tasks (node tiles) on the constant-stencil path             */
  int64_t n_tiles;        /* all tasks                                                  */
  int64_t inner_iters;    /* MFP_FP32 / MFP_FP32_IR: FP32 iterations among `iters`      */
  /* Condition estimate (opts.estimate_kappa): the CG step lengths alpha_k and direction
   * factors beta_k of Algorithm 1 define the Lanczos tridiagonal T of A on the Krylov
   * space of the right-hand side (T_11 = 1/alpha_1, T_kk = 1/alpha_k + beta_k/alpha_(k-1),
   * T_k,k-1 = sqrt(beta_k)/alpha_(k-1)); its extreme eigenvalues (Ritz values, found by
   * Sturm bisection on the host) approach the extreme eigenvalues of A on that space.
   * kappa_est = ritz_max / ritz_min.  A lower bound on cond_2(A): eigenvectors the
   * right-hand side barely touches show late or not before the stop (for a mirror-
   * symmetric layout b is odd in y, and only rounding reaches the even eigenvectors,
   * that of lambda_min among them).  Taken from the last CG run (FP32 runs for the
   * refined solve, joined
   * across its residual replacements), at most the first 16384 iterations; 0 when not
   * requested or fewer than 2 iterations ran.                                        */
  double kappa_est;
  double ritz_min, ritz_max;
  int64_t kappa_steps;    /* order of T                                                 */
  /* Launch shape of the last CG run's iteration kernel: work-groups per launch and
   * wavefronts per work-group (8: one task per wavefront from a table that puts the
   * tasks with element geometry on distinct SIMDs; 4: wavefront w takes tasks w,
   * w + W, ...).                                                                     */
  int64_t step_blocks;
  int64_t step_block_waves;
  int64_t step_element_mode;  /* 1: element geometry on the fly; 2: stored entries      */
} mfp_stats;

/* Message for the last non-zero status returned on this thread ("" if none). */
const char* mfp_last_error(void);

/* Host-only geometry check (no device work): MFP_OK or MFP_E_GEOMETRY / MFP_E_ARG.
 * Rejects: nbody outside [0, MFP_MAX_BODIES]; nx or ny < 2; any radius below
 * 2 max(hx, hy); a circle closer than one cell to a side; two circles whose centre
 * distance is not above the sum of their radii. */
int mfp_check_geometry(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody);

/* Workspace bytes for mfp_mesh_conform. */
size_t mfp_conform_workspace_size(const mfp_grid* grid, int32_t nbody);

/* Body-conforming mesh (section "Body-Conforming Grid Generation").
 *   kind[n]  MFP_FLUID / MFP_SNAPPED / MFP_DEEP, body[n] = body index or -1, where a
 *            node is inside body b iff (x-cx)^2 + (y-cy)^2 <= r^2 in FP64;
 *   disp     radial projection c + (r/rho)(x - c) - x on snapped nodes, zero on deep and
 *            outer-boundary nodes, and `nsweeps` Jacobi sweeps
 *            d <- wx (d_E + d_W) + wy (d_N + d_S), wx = hy^2/(2(hx^2+hy^2)),
 *            wy = hx^2/(2(hx^2+hy^2)), on the remaining fluid nodes (start 0).
 * All outputs are (nx+1)(ny+1) node arrays (disp twice that), device memory.
 * Returns MFP_E_TANGLED if an active cell has a non-positive Gauss-point Jacobian.
 * Results are bit-for-bit reproducible (no fused multiply-add in this step). */
int mfp_mesh_conform(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                     int32_t nsweeps, double* disp, int8_t* kind, int8_t* body,
                     void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for mfp_psi_solve / mfp_phi_solve / mfp_element_apply with this
 * precision and the automatic schedule (see mfp_solver_opts). */
size_t mfp_solve_workspace_size(const mfp_grid* grid, int32_t nbody, int32_t precision);

/* Workspace bytes for a solve with these options (precision and any explicit schedule
 * fields); 0 for invalid options. */
size_t mfp_solve_workspace_size_opts(const mfp_grid* grid, int32_t nbody,
                                     const mfp_solver_opts* opts);

/* Matrix-free element product q = K p (Algorithm 1's element loop, section "Weak
 * formulation": K_e = int (grad N)^T (grad N) dOmega, bilinear quads, 2x2 Gauss),
 * summed over active cells (cells whose four nodes are not all in one body), on the
 * mesh X = background + disp.  No boundary conditions are applied: q is the full
 * nodal product.  precision MFP_FP64: p, q are double[(nx+1)(ny+1)];
 * MFP_FP32: float[(nx+1)(ny+1)] (geometry rounded to FP32 relative to the cell).
 * `repeat` >= 1 launches the same kernel that many times (timing); apply_ms_h, if
 * non-NULL, receives the mean kernel duration in milliseconds. */
int mfp_element_apply(const mfp_grid* grid, const double* disp, const int8_t* body,
                      int32_t precision, const void* p, void* q, int32_t repeat,
                      double* apply_ms_h, void* ws, size_t ws_bytes, void* stream);

/* Scratch of mfp_element_apply_noalloc: one file-scope device array per GPU. */
#define MFP_NOALLOC_SCRATCH_BYTES (32u * 1024u * 1024u)

/* mfp_element_apply without allocation, for callers that cannot allocate device or
 * pinned memory: code being captured into a HIP graph, tight serving loops, harnesses
 * that forbid hipMalloc.  Same product q = K p (same kernels, same result bit for bit)
 * with no workspace argument, no timing and no repeat: its scratch is a file-scope
 * device array of MFP_NOALLOC_SCRATCH_BYTES (32 MiB) that each GPU the library runs on
 * holds until the process ends; its address is looked up once per device.  Tags,
 * displacements, the padded input and output and the task tables take about 33 bytes
 * per padded node (FP64 and FP32), so grids up to about 1e6 nodes fit (1300 x 650
 * cells do, 1390 x 695 do not); larger grids return MFP_E_WORKSPACE before any device
 * work.  Calls no hipMalloc, hipFree, event or other
 * allocating routine, clears what must start at zero with kernels (no memset), and does
 * not synchronise: the work is enqueued on `stream` and q is valid once it completes.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Arguments as for mfp_element_apply. */
int mfp_element_apply_noalloc(const mfp_grid* grid, const double* disp, const int8_t* body,
                              int32_t precision, const void* p, void* q, void* stream);

/* Constrained stream-function solve on a conformed mesh.
 * Unknowns: free nodes (interior and natural-boundary nodes) plus one psi_b per body
 * (all of a body's nodes tied to it); Dirichlet sides prescribed by `flow`.  Solves
 * A y = b with A = T^T K T, b = -T^T K g by conjugate gradients (Algorithm 1), to
 * ||r_k|| <= rtol ||b|| (= rtol ||r_0|| from the default zero start).
 * Outputs:
 *   psi         device double[(nx+1)(ny+1)]: nodal psi (body nodes carry psi_b);
 *   psi_b_h     host double[nbody];
 *   Q_h         host: psi_b[pair_hi] - psi_b[pair_lo]          (may be NULL);
 *   copfi_h     host: Q / (U (cy[pair_hi] - cy[pair_lo]))      (may be NULL);
 *               pair indices < 0 skip Q and CoPFI;
 *   samples     device double[2*sample_cap]: (theta, u_t) pairs, u_t = (psi_c - psi_b)/d_nc
 *               on every edge joining two nodes snapped to the same body, in each active
 *               cell with a fluid node; ordered by (body, cell id, local edge); may be
 *               NULL when sample_cap == 0;
 *   sample_body device int8[sample_cap];
 *   n_samples_h host: number of samples that exist (may exceed sample_cap);
 *   stats_h     host (may be NULL).
 * Returns MFP_W_NOCONV if kmax was reached, MFP_E_BREAKDOWN on CG breakdown (p.Ap <= 0
 * or a non-finite value, e.g. from a non-finite warm start; every kernel still ends
 * normally), MFP_E_ARG for a non-finite U or bad arguments (before any device work). */
int mfp_psi_solve(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                  const double* disp, const int8_t* kind, const int8_t* body,
                  const mfp_flow* flow, const mfp_solver_opts* opts,
                  int32_t pair_lo, int32_t pair_hi,
                  double* psi, double* psi_b_h, double* Q_h, double* copfi_h,
                  double* samples, int8_t* sample_body, int32_t sample_cap,
                  int32_t* n_samples_h, mfp_stats* stats_h,
                  void* ws, size_t ws_bytes, void* stream);

/* Velocity-potential solve on a conformed mesh (section "Governing Equation": the
 * velocity is also grad phi, phi satisfies the Laplace equation, and the contours of
 * phi and psi form the flow net), with the operator, solver and options of
 * mfp_psi_solve.  The paper gives no boundary conditions for phi; these are the
 * potential-flow ones:
 *   - sides flagged Dirichlet in `flow` carry their value (for the channel:
 *     MFP_BC_DIRICHLET_UX on inlet and outlet), natural sides (the walls) and every
 *     body surface have zero normal velocity (natural boundaries);
 *   - no body constraint: every node of an active cell (a cell whose four nodes are
 *     not all in one body) that is not Dirichlet is an unknown, body nodes included;
 *     nodes of no active cell lie inside a body and carry no equation.
 * Arguments as for mfp_psi_solve (same workspace size query, mfp_solve_workspace_size
 * with this nbody and precision); opts->psi0, if set, is a nodal warm start for phi
 * (its values at the unknowns are used, others ignored).  Output:
 *   phi      device double[(nx+1)(ny+1)]: nodal potential, NaN at nodes of no active
 *            cell;
 *   stats_h  host (may be NULL); n_dof = n_free = the number of unknowns.
 * Returns MFP_W_NOCONV if kmax was reached, MFP_E_BREAKDOWN on CG breakdown. */
int mfp_phi_solve(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                  const double* disp, const int8_t* kind, const int8_t* body,
                  const mfp_flow* flow, const mfp_solver_opts* opts, double* phi,
                  mfp_stats* stats_h, void* ws, size_t ws_bytes, void* stream);

/* Cubic least-squares fit of a gap-ratio sweep (section "Effect of Gap Ratio" fits
 * CoPFI as a cubic in delta and reports R^2 and the mean square error):
 *   y ~ coef_h[0] x^3 + coef_h[1] x^2 + coef_h[2] x + coef_h[3]   (ordinary least
 *   squares, Householder QR), r2_h = 1 - SS_res / SS_tot, mse_h = SS_res / n.
 * x_h, y_h: HOST double[n] (e.g. delta and the copfi_h of mfp_psi_solve_batched),
 * n >= 4; coef_h host double[4]; r2_h, mse_h may be NULL.  Host arithmetic only.
 * Returns MFP_E_ARG for n < 4, a non-finite value or fewer than 4 distinct x. */
int mfp_cubic_fit(const double* x_h, const double* y_h, int32_t n, double* coef_h,
                  double* r2_h, double* mse_h);

/* Workspace bytes for mfp_contour. */
size_t mfp_contour_workspace_size(const mfp_grid* grid);

/* Contour line field = level on the conformed mesh: the flow net (contours of psi and
 * phi, section "Governing Equation") and the stagnation streamlines psi = psi_b of the
 * transverse cylinders (section "Effect of Gap Ratio").  The paper does not say how its
 * lines were drawn; marching squares over the active cells, in the displaced node
 * coordinates X = background + disp: a node is above the level when field >= level;
 * on each cell edge a -> b (node order (i,j), (i+1,j), (i+1,j+1), (i,j+1); edges 0-1,
 * 1-2, 2-3, 3-0) whose end nodes differ, the crossing is X_a + t (X_b - X_a),
 * t = (level - f_a) / (f_b - f_a); two crossings make one segment (lower edge first),
 * four (a saddle) two, paired by the mean of the four values (on node 0's side: edges
 * 0,1 then 2,3, else 3,0 then 1,2).  Cells inside a body (all four nodes in one body)
 * or with a non-finite value (phi outside the domain) give none.
 *   field   device double[(nx+1)(ny+1)] (e.g. psi of mfp_psi_solve, phi of
 *           mfp_phi_solve); disp, body as for the solvers;
 *   seg     device double[4*cap]: (x0, y0, x1, y1) per segment, ordered by cell id
 *           j nx + i, then as above; only the first cap are written;
 *   n_seg_h host: number of segments that exist (may exceed cap).
 * Synchronises the stream (to read the count). */
int mfp_contour(const mfp_grid* grid, const double* disp, const int8_t* body,
                const double* field, double level, double* seg, int64_t cap,
                int64_t* n_seg_h, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for mfp_psi_grad. */
size_t mfp_grad_workspace_size(const mfp_grid* grid, int32_t nbody, int32_t precision);

/* Adjoint of mfp_psi_solve with respect to the node displacements (the automated
 * sensitivity analysis named in the paper's Conclusions as the next step).
 * For a loss L(psi_b, CoPFI) with the node classification frozen:
 *   adjoint solve   A lambda = dL/dy, A = T^T K T (the same symmetric operator, same
 *                   solver and precision options), right-hand side non-zero only in
 *                   the body rows: dL/dpsi_b = dL_dpsib_h[b] + dL_dcopfi dCoPFI/dpsi_b;
 *   shape term      dL_ddisp = -d/dX [ lambda_full^T K(X) psi ] at every node
 *                   (component-major like disp, device memory, overwritten);
 *   explicit term   dL_dcentre_h[2b+1] (host, overwritten; x entries set to 0) holds
 *                   dL_dcopfi times the derivative of CoPFI = Q / (U (cy_hi - cy_lo))
 *                   with respect to the pair's centre heights;
 *   free stream     dL_dU_h (host, may be NULL): dL/dU.  Every side datum is U times a
 *                   fixed function, so b = U b1 and y = U y1; the adjoint identity
 *                   lambda^T db/dU = (dL/dy)^T y / U, less the explicit U in CoPFI's
 *                   denominator, gives sum_b dL_dpsib_h[b] psi_b[b] / U (CoPFI itself
 *                   does not depend on U).
 * psi / psi_b_h are the outputs of mfp_psi_solve for the same inputs.  dL_dpsib_h may be
 * NULL; pair indices < 0 or dL_dcopfi == 0 skip the CoPFI terms.  opts->psi0 is ignored
 * (the adjoint solve always starts from zero; a forward warm start would not fit its
 * right-hand side).  Add the mesh part with mfp_mesh_conform_grad. */
int mfp_psi_grad(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                 const double* disp, const int8_t* kind, const int8_t* body,
                 const mfp_flow* flow, const mfp_solver_opts* opts, const double* psi,
                 const double* psi_b_h, const double* dL_dpsib_h, double dL_dcopfi,
                 int32_t pair_lo, int32_t pair_hi, double* dL_ddisp, double* dL_dcentre_h,
                 double* dL_dU_h, mfp_stats* stats_h, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for mfp_mesh_conform_grad. */
size_t mfp_conform_grad_workspace_size(const mfp_grid* grid, int32_t nbody);

/* Adjoint of mfp_mesh_conform (frozen classification): given dL/d(disp) at every node
 * (device, component-major), back-propagates through the nsweeps Jacobi sweeps
 * (transposed sweeps) and the radial projection of the snapped nodes, and ADDS
 * dL/d(cx_b, cy_b) to dL_dcentre_h[2b], [2b+1] and dL/dr_b to dL_dradius_h[b] (host;
 * dL_dradius_h may be NULL).  kind/body are the outputs of mfp_mesh_conform. */
int mfp_mesh_conform_grad(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                          int32_t nsweeps, const int8_t* kind, const int8_t* body,
                          const double* dL_ddisp, double* dL_dcentre_h, double* dL_dradius_h,
                          void* ws, size_t ws_bytes, void* stream);

/* One system of a batched solve: its grid and the outputs of mfp_mesh_conform for it
 * (device), and an optional device psi output ((nx+1)(ny+1) doubles, may be NULL). */
typedef struct {
  mfp_grid grid;
  const double* disp;
  const int8_t* kind;
  const int8_t* body;
  double* psi;
} mfp_variant;

/* Workspace bytes for mfp_psi_solve_batched (automatic schedule), and for these options
 * (precision, task_rows, element_mode, batch_tasks_per_wave; 0 for invalid options). */
size_t mfp_batched_workspace_size(int32_t nvar, const mfp_variant* vars_h, int32_t nbody,
                                  int32_t precision);
size_t mfp_batched_workspace_size_opts(int32_t nvar, const mfp_variant* vars_h, int32_t nbody,
                                       const mfp_solver_opts* opts);

/* Many independent solves of the same body layout on different meshes (the repeated
 * evaluations and design sweeps the paper's Practical Applications and Introduction
 * name), advanced together: every kernel launch covers all systems (one CG iteration
 * each), a fixed block of `iters_per_launch` iterations (0 -> the tuning cache's value,
 * else 64; rounded up to even) is
 * captured once as a hipGraph and replayed until every system has stopped.  circles_h
 * holds nvar * nbody circles (system-major), psi_b_h receives nvar * nbody values,
 * copfi_h (may be NULL) nvar values, stats_h (may be NULL) nvar entries.
 * opts->precision: MFP_FP64 (CG, each system stops on its own residual) or MFP_FP32_IR
 * (FP32 CG; after every block, at most 256 iterations, the FP32 correction is folded
 * into the FP64 iterate, the FP64 residual replaces the FP32 one and the iteration
 * restarts from it with its last direction kept; systems stop on that FP64 residual).
 * Schedule: opts->task_rows (4 or 5), opts->element_mode and opts->batch_tasks_per_wave
 * (or the tuning cache's batched entry) choose the rows per task, the element mode and
 * the tasks per wavefront of every system; other task_rows values are MFP_E_ARG.
 * Returns the worst status over the systems. */
int mfp_psi_solve_batched(int32_t nvar, const mfp_variant* vars_h, const mfp_circle* circles_h,
                          int32_t nbody, const mfp_flow* flow, const mfp_solver_opts* opts,
                          int32_t iters_per_launch, int32_t pair_lo, int32_t pair_hi,
                          double* psi_b_h, double* copfi_h, mfp_stats* stats_h, void* ws,
                          size_t ws_bytes, void* stream);

/* ---- Kutta constraints ------------------------------------------------------------
 * Section "Boundary Conditions" (trailing-edge paragraph): where the flow must leave a
 * body at a given place, a point is added in the fluid and the dividing streamline
 * psi = psi_b is made to pass through it.  For each body b with a Kutta point, the
 * equation psi(K_b) = psi_b replaces the body's zero-circulation row of the
 * constrained system (psi_b stays one unknown shared by the body's nodes; the body
 * then carries the circulation the flow needs); other bodies keep zero circulation.
 * K_b is the grid node nearest to the given point in undisplaced coordinates,
 * i = floor((x - x0)/hx + 1/2), j likewise; it must be a fluid node off the
 * Dirichlet sides (no node is moved: place the point on a grid node to have it
 * exactly).  The system is no longer symmetric; it is solved by superposition of
 * constrained CG solves (mfp_psi_solve's kernels and options): S0 with every Kutta
 * body held at 0, and per Kutta body k one solve without side data (U = 0) with body
 * k held at 1 and the others at 0; psi = S0 + sum_k c_k S_k with the nk x nk system
 * S0(K_j) + sum_k c_k S_k(K_j) = c_j solved on the host (psi_b of Kutta body k is
 * c_k).  Costs nk + 1 solves. */

/* Workspace bytes for mfp_psi_solve_kutta with nkutta Kutta points (0 if invalid). */
size_t mfp_kutta_workspace_size(const mfp_grid* grid, int32_t nbody, int32_t nkutta,
                                const mfp_solver_opts* opts);

/* Stream-function solve with Kutta constraints.  kutta_xy_h: host double[2 nbody],
 * (x, y) of body b's Kutta point, or (NaN, NaN) for a body without one.  Other
 * arguments and outputs as mfp_psi_solve (no surface samples, no warm start);
 * kutta_node_h (host int64[nbody], may be NULL) receives each body's Kutta node or -1.
 * stats: iterations, applications and solve time summed over the sub-solves,
 * relres_true their largest, kappa_est that of S0 (if requested).  MFP_E_ARG for a
 * Kutta point whose node is outside the grid, on a Dirichlet side or inside a body. */
int mfp_psi_solve_kutta(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                        const double* disp, const int8_t* kind, const int8_t* body,
                        const mfp_flow* flow, const mfp_solver_opts* opts,
                        const double* kutta_xy_h, int32_t pair_lo, int32_t pair_hi,
                        double* psi, double* psi_b_h, double* Q_h, double* copfi_h,
                        int64_t* kutta_node_h, mfp_stats* stats_h, void* ws, size_t ws_bytes,
                        void* stream);

/* ---- mixed-cell mesh ---------------------------------------------------------------
 * The mesh of section "Body-Conforming Grid Generation" that keeps the grid lines:
 * each grid edge joining a node inside a body to a fluid node is cut where it crosses
 * the circle (cut point I + t (O - I) with |I + t (O - I) - c| = r, t in [0, 1), I the
 * inside end, O the fluid end); inside nodes leave the mesh; every cut cell becomes the
 * polygon of its fluid corners and cut points walked counter-clockwise from corner
 * (i, j): a triangle (one fluid corner), a quadrilateral (two) or a pentagon (three),
 * the pentagon split into the triangle (P_a, C1, C2) and the quadrilateral
 * (P_a, C2, C3, P_b), P_a the cut point after the inside corner, C1..C3 the fluid
 * corners that follow, P_b the cut point before it.  A triangle whose two cut points
 * lie within 1e-12 max(hx, hy) of each other (max norm) has no area and is not meshed.
 * Fluid nodes are then moved by `nsweeps` Jacobi sweeps of the displacement (weights
 * as for mfp_mesh_conform, start 0, outer-boundary nodes fixed) in which an inside
 * neighbour contributes its cut point's displacement P - I.  A cell whose inside and
 * fluid corners alternate (a thin part of a body, e.g. a trailing edge, crosses it)
 * gets a triangle at each fluid corner (cut point of the edge before it, the corner,
 * cut point of the edge after it), in corner order, slivers dropped.  Cells with
 * corners in two bodies and grid edges joining two bodies are rejected
 * (MFP_E_GEOMETRY).
 * Mixed-node numbering: background nodes j (nx+1) + i (inside ones unused), then the
 * cut points, numbered in edge order: horizontal edges (edge j nx + i joins (i, j) and
 * (i+1, j)), then vertical ones (edge (ny+1) nx + j (nx+1) + i joins (i, j), (i, j+1)).
 * Elements are numbered cell by cell (cell j nx + i), a pentagon's triangle first.
 * Every floating-point expression of the mesh is evaluated without fused
 * multiply-add, so the mesh is reproducible bit for bit. */
typedef struct {
  /* caller-owned device arrays, sizes in elements */
  double* disp;          /* 2 (nx+1)(ny+1): displacements of background nodes (x, then y) */
  int8_t* body;          /* (nx+1)(ny+1): body of each background node, -1 fluid           */
  int32_t* hpt;          /* (ny+1) nx: cut point of each horizontal edge, -1 none          */
  int32_t* vpt;          /* ny (nx+1): cut point of each vertical edge, -1 none            */
  int32_t* cell_first;   /* nx ny + 1: first element of each cell, then the element count  */
  double* pxy;           /* 2 cap_points: (x, y) of each cut point                          */
  int8_t* pbody;         /* cap_points: body of each cut point                              */
  int32_t* pedge;        /* cap_points: grid edge of each cut point                         */
  int32_t* elem;         /* 4 cap_elems: mixed node ids, counter-clockwise, -1 past nne     */
  int8_t* nne;           /* cap_elems: 3 (triangle) or 4 (quadrilateral)                    */
  int64_t cap_points;    /* capacity of pxy / pbody / pedge (may be 0)                      */
  int64_t cap_elems;     /* capacity of elem / nne (may be 0)                               */
  int64_t n_points;      /* out: cut points                                                 */
  int64_t n_elems;       /* out: elements                                                   */
  int64_t n_tri;         /* out: triangles among them                                       */
} mfp_mixed_mesh_t;

/* Bodies of the mixed-cell mesh beyond circles (section "Boundary Conditions": bodies
 * with corners and trailing edges; "Practical Applications": airfoil clusters).
 * MFP_BODY_JOUKOWSKI: the Joukowski map z' = zeta + c^2/zeta of the circle
 * |zeta - zeta0| = R through zeta = c (R^2 = (c - xi0)^2 + eta0^2): an airfoil with a
 * cusped trailing edge at z' = 2c (chord about 4c; xi0 < 0 thickness, eta0 > 0
 * camber), placed as z = (x, y) + e^{-i alpha} z' (angle of attack alpha against the
 * horizontal free stream).  A point is inside (boundary included) iff both roots of
 * zeta^2 - w zeta + c^2 = 0, w = e^{i alpha}(z - (x, y)), lie in the closed circle,
 * i.e. |zeta - zeta0|^2 - R^2 <= 0 for the root farther from zeta0 (the map is one to
 * one from outside the circle onto outside the airfoil).  A grid edge from an inside
 * node I to a fluid node O is cut at I + t (O - I): t from the first sign change of
 * that level among t = k/64, then 60 bisections (the inside end kept).  A trailing
 * edge thinner than the grid is not resolved (an edge with two fluid ends is never
 * cut).  All in FP64 without fused multiply-add; cos alpha and sin alpha from the C
 * library. */
#define MFP_BODY_CIRCLE 0
#define MFP_BODY_JOUKOWSKI 1

typedef struct {
  int32_t kind;       /* MFP_BODY_CIRCLE or MFP_BODY_JOUKOWSKI                          */
  double x, y;        /* circle centre; airfoil: position of the image of zeta = 0      */
  double r;           /* circle radius; airfoil: the map constant c > 0                 */
  double xi0, eta0;   /* airfoil: centre of the generating circle, -c <= xi0 < 0        */
  double alpha;       /* airfoil: angle of attack (radians)                             */
} mfp_body;

/* Host only: for each body a circle that holds it (the circle itself; an airfoil:
 * about (x, y), 1.01 x the largest distance of 4097 boundary samples).  The mixed
 * mesh's geometry checks and the solves' circle arguments (Q, CoPFI, the
 * isolated-cylinder side data) use these.  MFP_E_ARG for an invalid body. */
int mfp_body_bounds(const mfp_body* bodies_h, int32_t nbody, mfp_circle* bounds_h);

/* Workspace bytes for mfp_mixed_mesh (0 for an invalid grid or body count). */
size_t mfp_mixed_workspace_size(const mfp_grid* grid, int32_t nbody);

/* Builds the mixed-cell mesh into *m.  body, hpt, vpt and cell_first are always
 * written; the cut points and elements are copied up to cap_points / cap_elems (the
 * counts are reported in full, so a first call with zero capacities sizes a second).
 * disp holds the smoothed displacements, except after a call with both capacities
 * zero, which skips the sweeps (counts do not depend on them) and leaves disp zero.
 * Sweep k updates only the node box of the bodies' bounding circles widened by k + 1
 * nodes: the displacement spreads one node per sweep, so the result is the same.
 * Synchronises `stream`.  MFP_E_GEOMETRY as mfp_check_geometry, for the mesh
 * rejections above, and for a body that holds no grid node (too thin for the grid;
 * the message names which). */
int mfp_mixed_mesh(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                   int32_t nsweeps, mfp_mixed_mesh_t* m, void* ws, size_t ws_bytes,
                   void* stream);

/* mfp_mixed_mesh for general bodies (circles and airfoils, see mfp_body): the same
 * mesh (for circles bit for bit), the geometry checks on mfp_body_bounds' circles. */
int mfp_mixed_mesh_bodies(const mfp_grid* grid, const mfp_body* bodies_h, int32_t nbody,
                          int32_t nsweeps, mfp_mixed_mesh_t* m, void* ws, size_t ws_bytes,
                          void* stream);

/* Workspace bytes for mfp_mixed_element_apply / mfp_mixed_psi_solve on a mixed mesh of
 * n_points cut points and n_elems elements with these solver options (NULL: FP64 and
 * the automatic schedule); 0 for invalid arguments. */
size_t mfp_mixed_solve_workspace_size(const mfp_grid* grid, int64_t n_points, int64_t n_elems,
                                      int32_t nbody, const mfp_solver_opts* opts);

/* q = K p on the mixed mesh (section "Weak formulation": P1 triangles exactly, Q1
 * quadrilaterals with 2x2 Gauss points, summed over the elements), p and q device
 * double[(nx+1)(ny+1) + n_points] in mixed-node numbering; nodes in no element get 0.
 * The element matrices are evaluated once per call into the workspace; the product is
 * a gather (each node sums its rows of the elements of the cells around it in a fixed
 * order), so it is deterministic.  `repeat` >= 1 launches the product that many times;
 * apply_ms_h (may be NULL) receives the mean product time in milliseconds.
 * Synchronises `stream`. */
int mfp_mixed_element_apply(const mfp_grid* grid, const mfp_mixed_mesh_t* m, const double* p,
                            double* q, int32_t repeat, double* apply_ms_h, void* ws,
                            size_t ws_bytes, void* stream);

/* Constrained stream-function solve on the mixed mesh (Algorithm 1): the unknowns are
 * the fluid nodes on no Dirichlet side plus one psi_b per body, shared by all its cut
 * points; Dirichlet sides as in mfp_psi_solve.  A y = b with A = T^T K T, b = -T^T K g.
 * Every element lies in one grid cell and the inside corners of a cut cell are tied
 * to the same psi_b as its cut points, so A is also the sum of 4 x 4 corner matrices,
 * one per cell (a cut cell's elements condensed onto its corners): the solve runs the
 * one-kernel CG of mfp_psi_solve on those matrices as stored element entries, with the
 * same options (precisions MFP_FP64, MFP_FP32, MFP_FP32_IR; tolerance, schedule fields
 * except element_mode, which is always the stored form; no warm start: psi0 must be
 * NULL) and the same statistics (n_free counts every fluid node off the Dirichlet
 * sides).  psi: device double[(nx+1)(ny+1) + n_points]: free values, Dirichlet values,
 * psi_b at the cut points and 0 at the inside nodes.  psi_b_h, Q_h, copfi_h, stats_h
 * as in mfp_psi_solve.  Synchronises `stream`.  Returns as mfp_psi_solve. */
int mfp_mixed_psi_solve(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                        const mfp_mixed_mesh_t* m, const mfp_flow* flow,
                        const mfp_solver_opts* opts, int32_t pair_lo, int32_t pair_hi,
                        double* psi, double* psi_b_h, double* Q_h, double* copfi_h,
                        mfp_stats* stats_h, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for mfp_mixed_psi_solve_kutta with nkutta Kutta points. */
size_t mfp_mixed_kutta_workspace_size(const mfp_grid* grid, int64_t n_points, int64_t n_elems,
                                      int32_t nbody, int32_t nkutta,
                                      const mfp_solver_opts* opts);

/* mfp_mixed_psi_solve with the Kutta constraints of mfp_psi_solve_kutta (kutta_xy_h:
 * (x, y) or (NaN, NaN) per body; the Kutta node must be a fluid node of the mesh off
 * the Dirichlet sides; kutta_node_h may be NULL).  circles_h: for airfoils the circles
 * of mfp_body_bounds.  Outputs as mfp_mixed_psi_solve. */
int mfp_mixed_psi_solve_kutta(const mfp_grid* grid, const mfp_circle* circles_h, int32_t nbody,
                              const mfp_mixed_mesh_t* m, const mfp_flow* flow,
                              const mfp_solver_opts* opts, const double* kutta_xy_h,
                              int32_t pair_lo, int32_t pair_hi, double* psi, double* psi_b_h,
                              double* Q_h, double* copfi_h, int64_t* kutta_node_h,
                              mfp_stats* stats_h, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MFPSI_H */
