/*
 * poromech.h -- C ABI of the MI355X (gfx950) solver for one backward-Euler
 * step of hybridized three-field poromechanics: Q1 displacement u, P0 cell
 * pressure p, face traces pi of the hybridized lowest-order Raviart-Thomas
 * Darcy velocity, with macro-element pressure-jump stabilization.
 *
 * The linear system solved per step is the stabilized, statically condensed
 * block system (paper: Frigo, Castelletto, Ferronato, White, "Efficient
 * solvers for hybridized three-field mixed finite element coupled
 * poromechanics", eq. stab_A):
 *
 *     [ A_uu   A_up              0        ] [u ]   [f_u ]
 *     [ A_pu   Abar_pp + A_stab  dt A_ppi ] [p ] = [f_p ]
 *     [ 0      A_pip             A_pipi   ] [pi]   [f_pi]
 *
 * solved by right-preconditioned flexible GMRES with the block upper
 * triangular preconditioner of eq. hybridPrec (B~_p diagonal of eq. app_Bp,
 * aggregation-AMG V-cycles for A_uu and C~_pi).
 *
 * Mesh: structured nx x ny x nz hexahedra (each count even: the stabilization
 * works on aligned 2x2x2 macro-elements), trilinear geometry given by node
 * coordinates.  Numbering:
 *   node (i,j,k)   i + (nx+1)*(j + (ny+1)*k)
 *   cell (i,j,k)   i + nx*(j + ny*k)
 *   faces          x-normal (i<=nx,j<ny,k<nz) i+(nx+1)*(j+ny*k), then y-normal
 *                  (offset n_fx) i+nx*(j+(ny+1)*k), then z-normal
 *                  (offset n_fx+n_fy) i+nx*(j+ny*k)
 *   u dof          3*node + component
 *   system vector  [u (n_u) ; p (n_p = cells) ; pi (n_pi = faces)]
 * Boundary conditions: bottom (k=0) nodes fixed (u = 0); top (k=nz) faces
 * drained (pi = p_top) and loaded by a uniform traction; all other boundary
 * parts traction-free and no-flow.  PM_BC_ROLLERS additionally fixes the
 * normal displacement of the four lateral sides.  PM_BC_CANTILEVER (the
 * paper's cantilever test, Sec. 5.2): the nodes of the face x = x_min (i=0)
 * fixed, the top loaded by the traction, no-flow on the whole boundary (no
 * drained face; p_top unused).  Dirichlet dofs stay in the
 * system as identity rows and columns, so sizes match the paper's table
 * tab:grids.
 *
 * Conventions for every entry point:
 *   - return 0 on success or a negative PM_E* code; the message of the last
 *     error is returned by pm_last_error(ctx).  No C++ exception crosses it.
 *   - "device" pointers are HIP device (or managed) memory owned by the
 *     caller; "host or device" inputs are copied (hipMemcpyDefault).
 *   - kernels are enqueued on the stream passed to pm_setup, except that
 *     pm_setup, pm_assemble and pm_update_material build B~_p, C~_pi and the
 *     C~_pi hierarchy on a second, library-owned stream (non-blocking,
 *     default priority) from a helper thread, concurrently with the A_uu
 *     hierarchy on the caller's stream.  These calls, pm_set_dt, pm_solve
 *     and pm_solve_transpose synchronize the caller's stream on entry and
 *     return after all their work has completed; the others are
 *     asynchronous.
 *   - a context is not thread-safe; use one context per host thread.
 */
#ifndef POROMECH_H
#define POROMECH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PM_OK = 0,
  PM_EINVAL = -1,       /* invalid argument (odd dims, non-positive field, det J <= 0, null) */
  PM_ENOMEM = -2,       /* device allocation failed */
  PM_EHIP = -3,         /* HIP runtime error (message in pm_last_error) */
  PM_ENOCONV = -4,      /* max_it reached; outputs hold the last iterate, info filled */
  PM_EBREAKDOWN = -5,   /* NaN/Inf in a reduction or Krylov breakdown */
  PM_ESTATE = -6,       /* call out of order (e.g. solve before assemble) */
  PM_EINTERNAL = -7     /* internal capacity exceeded (e.g. AMG row too wide) */
};

enum { PM_BC_COLUMN = 0, PM_BC_ROLLERS = 1, PM_BC_CANTILEVER = 2 };

typedef struct pm_ctx pm_ctx;

typedef struct {
  int32_t nx, ny, nz;        /* cells per axis, each >= 2 and even */
  const double* coords;      /* host or device, (nx+1)(ny+1)(nz+1) x 3, node order; NULL: uniform box */
  double Lx, Ly, Lz;         /* box size used when coords == NULL */
} pm_mesh;

typedef struct {
  const double* E;           /* host or device, n_cells, Young's modulus > 0 */
  const double* kappa;       /* host or device, n_cells x 3, diagonal permeability > 0 */
  double nu;                 /* Poisson ratio in (0, 0.5) */
  double biot;               /* Biot coefficient b */
  double S_eps;              /* constrained specific storage >= 0 */
  double mu;                 /* fluid viscosity > 0 */
} pm_material;

typedef struct {
  double traction_top[3];    /* traction on the top face (e.g. {0,0,-1}) */
  double p_top;              /* prescribed face pressure on the top face */
  int32_t kind;              /* PM_BC_COLUMN, PM_BC_ROLLERS or PM_BC_CANTILEVER */
} pm_bc;

typedef struct {
  double rtol;               /* FGMRES stop: ||b - A x||_2 <= rtol ||b||_2 */
  int32_t restart;           /* FGMRES restart length m (>= 1) */
  int32_t max_it;            /* iteration cap */
  int32_t precond_fp32;      /* 1: AMG hierarchies, V-cycles and Schur apply in FP32 (the set-up's
                                lambda_max power iterations on those FP32 operators) */
  int32_t stabilize;         /* 1: add the macro-element pressure-jump term */
  int32_t increment_stab;    /* 1: stabilization acts on p_n - p_{n-1} (RHS term A_stab p_{n-1}) */
  int32_t cheb_degree;       /* Chebyshev smoother degree per pre/post smoothing, A_uu (>= 1) */
  int32_t coarse_max;        /* AMG: stop coarsening below this many block rows */
  int32_t cheb_degree_pi;    /* Chebyshev smoother degree, C~_pi hierarchy (>= 1) */
  int32_t cycles_u;          /* V-cycles per application of the A_uu block (>= 1) */
  int32_t cycles_pi;         /* V-cycles per application of the C~_pi block, and of the MFE C~_p block (>= 1) */
  int32_t orth_passes;       /* classical Gram-Schmidt passes per Arnoldi step: 1 or 2 */
  double theta_u;            /* AMG strength threshold, displacement block */
  double theta_pi;           /* AMG strength threshold, face-pressure Schur block */
  int32_t agg_dist_u;        /* AMG aggregation: roots form a distance-1 or distance-2 independent set */
  int32_t agg_dist_pi;
  double cheb_lower;         /* Chebyshev interval [cheb_lower, 1.1] x lambda_max(D^-1 A), in (0, 1) */
  double rtol_transpose;     /* stopping tolerance of pm_solve_transpose (0: use rtol) */
  int32_t restart_transpose; /* restart length of pm_solve_transpose (0: use restart) */
  int32_t orth_passes_transpose; /* Gram-Schmidt passes of pm_solve_transpose (0: use orth_passes) */
  int32_t lattice_uu;        /* 1: if every cell is a translate of the first (to 1e-12 of the edge
                                length), apply the finest A_uu level from E_T and one element
                                matrix instead of the assembled matrix; 0: always assembled */
  double p_trunc_pi;         /* C~_pi hierarchy: drop prolongator entries below this fraction of
                                their row's largest, rescaling to the row sum (0: keep all) */
  int32_t cell_pi;           /* 1: apply the finest C~_pi level cell by cell from packed symmetric
                                6x6 element matrices; 0: assembled matrix */
  double p_trunc_u;          /* A_uu hierarchy: drop prolongator blocks below this fraction of
                                their row's largest (Frobenius norms), keeping the block row sum */
  double cheb_lower_pi;      /* Chebyshev interval lower end for C~_pi (0: use cheb_lower) */
  int32_t block_minv;        /* 1: if every cell's M_T^-1 couples only the two faces of each direction
                                (off-block entries within 1e-12 of the geometric mean of the
                                diagonals: axis-aligned boxes, diagonal permeability), apply
                                M_T^-1 and C~_T in the solve from the 9 block entries, leaving
                                the rounding-level rest out; 0: always the full 6x6 matrices */
  int32_t rbm_u;             /* 1: the A_uu hierarchy's tentative prolongators span the six
                                rigid-body modes of each aggregate on every level (a translation
                                and a rotation about the aggregate's centroid: two 3x3 coarse
                                block rows per aggregate, not orthonormalised, so the coarse
                                near kernel stays the unit vectors); prolongator truncation
                                compares translation and rotation blocks each with its own kind
                                and does not rescale (the M_III^(h) variant of Sec. 5);
                                0: translations only (M_II^(h)) */
} pm_opts;

typedef struct {
  int32_t iters;             /* FGMRES iterations of the last solve */
  int32_t levels_u, levels_pi;
  double relres_est;         /* Givens residual estimate / ||b|| */
  double relres_true;        /* ||b - A x|| / ||b|| recomputed in FP64 */
  double t_asm, t_setup, t_solve;   /* seconds: assembly (element kernels, condensation,
                                       stabilization, Dirichlet rows and the A_uu values: the
                                       kernel time of the value fill, which overlaps the C~_pi
                                       set-up), preconditioner set-up (B~_p, C~_pi, both AMG
                                       hierarchies: the rest of the wall time; T_p of Sec. 5),
                                       Krylov solve (T_s of Sec. 5) */
  double opcx_u, opcx_pi;    /* AMG operator complexities */
  int32_t lattice_uu;        /* 1 if the finest A_uu level runs on the lattice operator */
  int32_t block_minv;        /* 1 if M_T^-1 is stored and applied by direction blocks */
  int32_t ncoarse_u, ncoarse_pi;  /* unknowns of the coarsest level (dense FP64 inverse) of each hierarchy */
  int32_t lattice_form;      /* unit element matrix the lattice stencils read: 0 no lattice operator;
                                1 its 576 entries; 2 box cells (mirror symmetry): 48 values in the
                                FP32 stencils, 576 entries in the FP64 ones; 3 cubic cells (mirror
                                and axis-permutation symmetry): 12 values in all stencils */
} pm_info;

/* Default options: rtol 1e-8, restart 100, max_it 1000, FP64, stabilize,
 * increment form, Chebyshev degree 2 (A_uu) / 2 (C~_pi), coarse_max 64, one
 * V-cycle per block, two Gram-Schmidt passes, strength thresholds theta
 * 0 (A_uu) / 0.08 (C~_pi), distance-2 aggregation roots, Chebyshev interval
 * from 0.3 lambda_max; transposed solves: rtol, restart 100 and two
 * Gram-Schmidt passes (restarted GMRES on the transposed preconditioned
 * operator stagnates with short restarts or one pass on strongly
 * heterogeneous permeability); lattice operator on; C~_pi prolongator
 * truncation 0.02 (C~_pi) and 0.02 (A_uu); cell-by-cell finest C~_pi level;
 * M_T^-1 by direction blocks where the cells allow it; translation-only
 * near kernel for A_uu. */
void pm_default_opts(pm_opts* opts);

/* Create a context: validates and copies mesh coordinates and material
 * fields to the device and allocates the operator storage.  dt > 0.
 * stream: a hipStream_t (NULL = default stream).  On error *out is NULL. */
int pm_setup(const pm_mesh* mesh, const pm_material* mat, const pm_bc* bc, double dt,
             const pm_opts* opts, void* stream, pm_ctx** out);

/* Element kernels (Q1 stiffness and coupling: Appendix A eq. MFE_matrix; RT0
 * mass and its static condensation: eq. hmfeSys/A_33H), macro-element
 * stabilization (eq. J_def, 3D beta_M of Sec. 3), global assembly with the
 * Dirichlet identity rows, B~_p (eq. app_Bp), C~_pi (Sec. 4) and both AMG
 * hierarchies.  Fails with PM_EINVAL on an inverted hexahedron. */
int pm_assemble(pm_ctx* ctx);

/* Change dt (backward Euler, Sec. 2.1: dt scales the condensed pressure
 * block Abar_pp and the coupling dt A_ppi of eq. stab_A): rebuilds the
 * dt-dependent blocks, B~_p (eq. app_Bp), C~_pi (Sec. 4) and the C~_pi
 * hierarchy; the A_uu hierarchy, independent of dt, is reused.  dt > 0. */
int pm_set_dt(pm_ctx* ctx, double dt);

/* Replace E (n_cells) and/or kappa (n_cells x 3) (host or device; NULL keeps
 * the current field) and assemble everything (as pm_assemble). */
int pm_update_material(pm_ctx* ctx, const double* E, const double* kappa);

/* Right-hand side of the step (Appendix A eq. MHFE_vector with the f~_n of
 * Sec. 2.1, no fluid source): traction load, A_pu u_prev + S_eps|T| p_prev
 * (+ A_stab p_prev in increment form), Dirichlet values and lifting.
 * u_prev (n_u), p_prev (n_p) device, may be NULL (state at rest);
 * b device, N = n_u + n_p + n_pi. */
int pm_build_rhs(pm_ctx* ctx, const double* u_prev, const double* p_prev, double* b);

/* Solve A_H x = b (eq. stab_A; device b, N) by flexible GMRES with the block
 * upper triangular preconditioner of eq. hybridPrec applied by back
 * substitution pi -> p -> u (C~_pi V-cycle, B~_p^-1, A_uu V-cycle), zero
 * initial guess, stopping at ||b - A x|| <= rtol ||b|| on the recomputed FP64
 * residual (the solver settings of Sec. 5).  Outputs (device, caller-owned):
 * u (n_u), pi (n_pi), p (n_p); any may be NULL.  info may be NULL.  Returns
 * PM_ENOCONV if max_it is reached (outputs = last iterate), PM_EBREAKDOWN on
 * a non-finite value in the iteration. */
int pm_solve(pm_ctx* ctx, const double* b, double* u, double* pi, double* p, pm_info* info);

/* pm_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same FGMRES and preconditioner kernels, with the Krylov workspace (basis,
 * preconditioned vectors, reduction partials, device scalars) in a static
 * device array of 256 MiB per GPU that the library holds until the process
 * ends, and the host side of the Givens process on the call's stack.  This
 * call never calls hipMalloc, hipFree or any other allocating routine; the
 * context's own buffers come from pm_setup / pm_assemble.  Limits: restart
 * <= 64 and (restart+1) FP64 plus restart FP64 (or, with the FP32
 * preconditioner and one Gram-Schmidt pass, FP32) vectors of N unknowns
 * plus 8 MiB of partial sums within the 256 MiB (restart 24: N up to about
 * 660,000, or 880,000 with the FP32 preconditioner); larger problems return
 * PM_EINVAL before any work.  Arguments, outputs and return codes as
 * pm_solve.  Every call on one GPU uses that GPU's one array and leaves its
 * contents behind: calls that overlap on one GPU (several host threads or
 * streams) race and must be serialized by the caller. */
int pm_solve_noalloc(pm_ctx* ctx, const double* b, double* u, double* pi, double* p, pm_info* info);

/* Right-hand side [f_u; f_q; f_p] of the step in the non-hybridized mixed
 * (MFE) form (Sec. 2.1 eq. mfeSys, Appendix A eq. MFE_vector), order
 * [u; q; p] as PM_OP_MFE: the traction load; f_q = -s p_top on each drained
 * face (s = +1 for a cell's +x/+y/+z face), 0 elsewhere; f_p = A_pu u_prev +
 * S_eps|T| p_prev (+ A_stab p_prev in increment form).  u_prev, p_prev device
 * or NULL; b device, N. */
int pm_build_rhs_mfe(pm_ctx* ctx, const double* u_prev, const double* p_prev, double* b);

/* Solve A_M x = b, the MFE form of the step (the comparison system of Sec.
 * 5), by FP64 FGMRES right-preconditioned with PM_OP_BTP (eq. prec), zero
 * initial guess, with the context's rtol, restart, max_it and Gram-Schmidt
 * passes.  b device, N, order [u; q; p]; outputs (device, caller-owned, any
 * may be NULL): u (n_u), q (n_pi face fluxes), p (n_p).  The first call after
 * pm_assemble or pm_set_dt builds C~_p and its hierarchy (info->t_setup;
 * info->levels_pi, opcx_pi and ncoarse_pi describe that hierarchy).
 * Returns PM_ENOCONV if max_it is reached. */
int pm_solve_mfe(pm_ctx* ctx, const double* b, double* u, double* q, double* p, pm_info* info);

/* Solve A_H^T lam = g (the adjoint of the step: the transposed system of eq.
 * stab_A) with FGMRES right-preconditioned by M^T, the transpose of eq.
 * hybridPrec (block lower triangular: forward substitution u -> p -> pi with
 * the same, symmetric V-cycles), with rtol_transpose, restart_transpose and
 * orth_passes_transpose.  g device, N; outputs and return codes as pm_solve. */
int pm_solve_transpose(pm_ctx* ctx, const double* g, double* lu, double* lpi, double* lp,
                       pm_info* info);

/* Accumulate per-cell gradients of a scalar loss L:
 *   dlogk[T] += -lam^T (dA/dlog kappa_T) x
 *   dlogE[T] += -lam^T (dA/dlog E_T) x + lam^T (db/dlog E_T)
 * where lam solves A_H^T lam = dL/dx (Dirichlet rows of lam ignored), x is
 * the step solution [u;p;pi] and p_prev the previous pressure (NULL = 0;
 * it enters only through the increment-form stabilization).  All device;
 * lam, x: N; p_prev: n_p; dlogk, dlogE: n_p (accumulated, not cleared). */
int pm_grad(pm_ctx* ctx, const double* lam, const double* x, const double* p_prev,
            double* dlogk, double* dlogE);

/* Adjoint coupling of consecutive steps: c_u += -A_up lam_p, c_p +=
 * (S_eps|T| + A_stab) lam_p (increment form), i.e. (d b_{n+1}/d x_n)^T lam
 * for lam = lam_{n+1}; lam device N, c device N (accumulated). */
int pm_rhs_adjoint(pm_ctx* ctx, const double* lam, double* c);

/* Cell fluxes w_T = M_T^-1 (p_T 1 - pi_T), outward per local face
 * (-x,+x,-y,+y,-z,+z); p (n_p), pi (n_pi, holding the drained values), w
 * (n_p x 6, cell-major) device. */
int pm_reconstruct_w(pm_ctx* ctx, const double* p, const double* pi, double* w);

/* Operator applications for testing and benchmarking, all device, FP64:
 *   PM_OP_AH       y = A_H x            (N -> N)
 *   PM_OP_AHT      y = A_H^T x          (N -> N)
 *   PM_OP_MINV     y = M^-1 x           (N -> N, AMG inner solves)
 *   PM_OP_MINVT    y = M^-T x           (N -> N)
 *   PM_OP_CPI      y = C~_pi x          (n_pi -> n_pi, assembled, Dirichlet rows identity)
 *   PM_OP_BP       y = B~_p x           (n_p -> n_p, diagonal)
 *   PM_OP_AUU      y = A_uu x           (n_u -> n_u, assembled, Dirichlet rows identity)
 *   PM_OP_VCYCLE_U y = one V-cycle for A_uu applied to x (zero initial guess)
 *   PM_OP_VCYCLE_PI y = one V-cycle for C~_pi applied to x
 *   PM_OP_MFE      y = A_M x            (N -> N) the non-hybridized mixed system of
 *                  Sec. 2.1 (eq. mfeSys, Appendix A eq. MFE_matrix) with the stabilized
 *                  pressure block A_pp + A_stab of Sec. 3, in the order [u; q; p]: q has one
 *                  flux per face (n_pi of them, same face numbering), oriented by the face's
 *                  global +x/+y/+z normal; p one pressure per cell.  Fixed displacements and
 *                  faces on the no-flow boundary are identity rows with zero columns; drained
 *                  faces carry a free flux.  The first call after pm_assemble stores the
 *                  per-cell RT0 mass (36 doubles per cell, owned by the context).
 *   PM_OP_CP       y = C~_p x           (n_p -> n_p) the Schur complement approximation of the
 *                  MFE block triangular preconditioner (Sec. 5, eq. prec): A_stab + A_pp +
 *                  the fixed-stress diagonal of B~_p + dt A_qp^T L_qq^-1 A_qp, with L_qq the
 *                  absolute row sums of A_qq (no-flow faces excluded).  Assembled as a
 *                  7-point CSR held by the context on the first MFE call after pm_assemble
 *                  or pm_set_dt, together with the hierarchy below.
 *   PM_OP_VCYCLE_CP y = cycles_pi V-cycles for C~_p applied to x (zero initial guess), on
 *                  the context's smoothed-aggregation hierarchy of C~_p (C~_pi settings, FP64),
 *                  built once per assembly and dt (the inner C~_p solve of the MFE
 *                  preconditioner).
 *   PM_OP_BTP      y = M^-1 x           (N -> N, order [u; q; p]) the block lower triangular
 *                  preconditioner of the MFE system (Sec. 5, eq. prec, GPU analogue of
 *                  variant M_II^(m)): y_u = cycles_u A_uu V-cycles (the pm_assemble
 *                  hierarchy, FP64 levels) on x_u; y_q = five Chebyshev-Jacobi sweeps on
 *                  A_qq y_q = x_q from zero (in place of the paper's incomplete Cholesky
 *                  factor, whose triangular solves are sequential); y_p = cycles_pi C~_p
 *                  V-cycles on x_p - A_pu y_u - dt A_pq y_q. */
enum { PM_OP_AH = 0, PM_OP_AHT = 1, PM_OP_MINV = 2, PM_OP_MINVT = 3, PM_OP_CPI = 4,
       PM_OP_BP = 5, PM_OP_AUU = 6, PM_OP_VCYCLE_U = 7, PM_OP_VCYCLE_PI = 8, PM_OP_MFE = 9,
       PM_OP_CP = 10, PM_OP_VCYCLE_CP = 11, PM_OP_BTP = 12 };
int pm_apply(pm_ctx* ctx, int which, const double* x, double* y);

/* Kernel timing for roofline measurements.  pm_profile_begin clears the
 * records and, for every kernel whose bit (1 << id) is set in mask, records a
 * pair of HIP events on the launching stream around each later launch, with
 * the algorithmic bytes that launch must move (stored values and indices,
 * each input vector read once, each output written once) and, for the
 * matrix-free lattice stencils on the finest A_uu level, whose arithmetic
 * bounds them, the flops of their multiply-adds (576 per node: three rows of
 * the 24x24 element matrix for each of the 8 cells around it; 0 for the
 * memory-bound kernels).  pm_profile_end synchronizes the recorded events and
 * returns, for kernel id, the number of launches, their summed duration (ms),
 * summed algorithmic bytes and summed flops (flops may be NULL); it does not
 * stop the recording (call pm_profile_begin(ctx, 0) for that).  Ids:
 *   1 u-rows of A_H (FP64; lattice operator or assembled A_uu, with the coupling)
 *   2 fused Chebyshev smoothing step on the finest A_uu level
 *   3 fused Chebyshev smoothing step on the finest C~_pi level
 *   4 FGMRES multi-dot (Gram-Schmidt projections)
 *   5 FGMRES Gram-Schmidt update of the new basis vector (orthogonalise and
 *     normalise in one pass, or the multi-AXPY of the two-pass variant)
 *   6 restriction from the finest A_uu level
 *   7 p-rows of A_H
 *   8 pi-rows of A_H
 *   9 prolongation onto the finest A_uu level (added to the smoothed iterate)
 *  10 restriction from the finest C~_pi level
 *  11 prolongation onto the finest C~_pi level
 *  12 residual on the finest A_uu level
 *  13 residual on the finest C~_pi level
 * The recorder is process-wide (one context at a time). */
enum { PM_PROF_AH_U = 1, PM_PROF_CHEB_U0 = 2, PM_PROF_CHEB_PI0 = 3, PM_PROF_MULTIDOT = 4,
       PM_PROF_MULTIAXPY = 5, PM_PROF_RESTRICT_U0 = 6, PM_PROF_AH_P = 7, PM_PROF_AH_PI = 8,
       PM_PROF_PROLONG_U0 = 9, PM_PROF_RESTRICT_PI0 = 10, PM_PROF_PROLONG_PI0 = 11,
       PM_PROF_RESID_U0 = 12, PM_PROF_RESID_PI0 = 13 };
int pm_profile_begin(pm_ctx* ctx, uint32_t mask);
int pm_profile_end(pm_ctx* ctx, int id, int64_t* launches, double* ms, double* bytes, double* flops);

/* Sizes: out[0..5] = n_u, n_p, n_pi, N, n_nodes, n_macro. */
int pm_sizes(const pm_ctx* ctx, int64_t* out);

/* Info of the last solve and the last assembly timings. */
int pm_get_info(const pm_ctx* ctx, pm_info* info);

/* Message of the last error of ctx (or of the last failed pm_setup if ctx
 * is NULL).  Never NULL. */
const char* pm_last_error(const pm_ctx* ctx);

/* Free every device buffer of ctx (after synchronizing its stream). */
void pm_destroy(pm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* POROMECH_H */
