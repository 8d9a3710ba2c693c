/*
 * cellfft: periodic linear-elastic cell problem on a voxel grid, solved on
 * an AMD Instinct MI355X (gfx950) by conjugate gradients preconditioned with
 * the Fourier-diagonalised inverse of a homogeneous reference stiffness.
 *
 * Problem (static, periodic special case of the elastic system of the
 * paper's Sec. 2.1, eq. TimeHarmonicSystem with k = 0): on the cell
 * Y = [0,L_x) x [0,L_y) (x [0,L_z)) with N_x x N_y (x N_z) voxels, nodes at
 * the voxel corners (periodic), find the nodal fluctuation u minimising
 *     sum over voxels v, simplices s of v:  |s| W_v(eps_bar + eps(u)),
 * with W(eps) = lambda/2 tr(eps)^2 + mu eps:eps (Sec. 2.2, eq.
 * LinearElastEnergy), lambda = nu E / ((1+nu)(1-2nu)), mu = E / (2(1+nu))
 * (Sec. 6.3), and u linear on each simplex of the Kuhn subdivision (6
 * tetrahedra per voxel sharing the main diagonal; 2 triangles per pixel).
 * 2D is plane strain.  The effective stiffness is
 *     C*_IJ = (1/|Y|) sum |s| (eps_bar^I + B u^I) : D (eps_bar^J + B u^J).
 *
 * Conventions
 *   - Arrays over voxels/nodes are colexicographic, x fastest (Sec. 3.1):
 *     index = i_x + N_x (i_y + N_y i_z).  Displacements are [d][n].
 *   - Voigt order (11,22,33,23,13,12) in 3D, (11,22,12) in 2D; strains use
 *     engineering shear (a unit shear load is gamma = 1).  C_out[3][3] is
 *     the tensor component C*_2323.
 *   - Every array passed in or out is owned by the caller.  Inputs are
 *     copied before the call returns; the library keeps no caller pointer.
 *     on_device = 1 means a device pointer on the handle's device, consumed
 *     in order on the handle's stream; 0 means host memory.
 *   - Calls that return host results synchronise the handle's stream.
 *   - A handle is not thread-safe; different handles are independent.
 *   - No C++ exception crosses this interface.  Negative status: nothing
 *     was written.  CELL_NOT_CONVERGED: the best iterate and its results
 *     were written and cell_info holds the residuals.  cell_last_error()
 *     returns a thread-local message for the last failure.
 *   - A linear solve ends CELL_NOT_CONVERGED when a load reaches max_iter
 *     or stagnates: CELLFFT_STAG_WINDOW iterations (environment, read at
 *     create; default 256, 0 = never) without halving the smallest
 *     ||r||^2 seen so far.  The first stagnation refreshes the residual in
 *     FP64 and restarts CG there (beta = 0 at the next direction update);
 *     the second ends that load, and cell_last_error() names it.
 *   - Grid sizes: N_a in {4,6,8,12,16,24,32,48,64,96,128,192,256} (even,
 *     radix 2/3 FFTs); others return CELL_E_UNSUPPORTED.
 */
#ifndef CELLFFT_H
#define CELLFFT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cell_s* cell_t;
typedef struct cell_batch_s* cell_batch_t;

typedef enum {
  CELL_OK = 0,
  CELL_NOT_CONVERGED = 1,
  CELL_E_ARG = -1,         /* invalid argument (null pointer, bad size, nu out of range) */
  CELL_E_NOMEM = -2,       /* device allocation failed */
  CELL_E_DEVICE = -3,      /* HIP runtime error */
  CELL_E_STATE = -4,       /* call order violated (no material / no solve yet) */
  CELL_E_NONFINITE = -5,   /* non-finite or non-positive Young's modulus */
  CELL_E_BREAKDOWN = -6,   /* CG breakdown: p.Kp <= 0, r.z <= 0 or non-finite scalar */
  CELL_E_UNSUPPORTED = -7  /* grid size without an FFT plan */
} cell_status;

enum { CELL_FP64 = 0, CELL_MIXED = 1 };

typedef struct {
  int dim;           /* 2 or 3 */
  int n[3];          /* N_x, N_y, N_z (n[2] ignored in 2D) */
  double len[3];     /* cell edge lengths; 0 means 1 */
  int precision;     /* CELL_FP64: every kernel in FP64.  CELL_MIXED: stencil,
                        FFT and vector updates in FP32, all reductions, CG
                        scalars and residual recomputation in FP64 */
  double tol;        /* stop when ||f - K u||_2 <= tol ||f||_2; 0 -> 1e-10 (FP64) / 1e-6 (mixed) */
  int max_iter;      /* CG iteration cap; 0 -> 10000 */
  int max_loads;     /* simultaneous load cases; 0 -> 3 (2D) / 6 (3D) */
  void* stream;      /* hipStream_t to run on; NULL -> a library-owned stream */
  int device;        /* HIP device ordinal; -1 -> the current device */
} cell_config;

typedef struct {
  int nload;
  int iters[6];            /* CG iterations per load */
  int refinements[6];      /* FP64 residual recomputations per load */
  double relres[6];        /* final ||f - K u|| / ||f||, recomputed in FP64 */
  double hill_mandel_gap;  /* max_J |<sigma:eps>^J - sigma_bar^J . eps_bar^J| / max|C| (effective stiffness) */
  double sym_gap;          /* max |S_IJ - S_JI| / max|S|, S = mean-stress form (effective stiffness) */
  double seconds;          /* wall time of the call */
} cell_info;

/* Create a solver for one cell grid.  Allocates all device buffers for
 * max_loads simultaneous loads.  *out receives the handle. */
cell_status cell_create(const cell_config* cfg, cell_t* out);

/* Per-voxel Young's modulus E (> 0, finite) and Poisson ratio nu in
 * (-1, 0.5), n values each, colexicographic.  Copies the data (host arrays
 * through a temporary device buffer), validates it and converts it to the
 * Lame parameters on the device; also fixes the preconditioner's reference
 * medium (geometric means of the extreme bulk and shear moduli).  The first
 * invalid voxel is reported (CELL_E_NONFINITE for E, CELL_E_ARG for nu; E
 * first at one voxel) and the previous material, if any, stays in place. */
cell_status cell_set_material(cell_t c, const double* E, const double* nu, int on_device);

/* Solve the cell problem for nload (<= max_loads) macro strains
 * macro_strain[nload][nv] (host, Voigt, engineering shear).  Writes the
 * mean stress sigma_bar[nload][nv] (host, may be NULL).  The solutions are
 * kept for cell_get_displacement / cell_adjoint. */
cell_status cell_solve(cell_t c, int nload, const double* macro_strain, double* mean_stress_out,
                       cell_info* info);

/* Solve the nv unit loads and write C*[nv][nv] (host, row-major, energy
 * form; symmetric by construction).  info->sym_gap reports the asymmetry of
 * the mean-stress form, info->hill_mandel_gap the energy mismatch. */
cell_status cell_effective_stiffness(cell_t c, double* C_out, cell_info* info);

/* Derivative of J = sum_IJ dJ_dC[I][J] C*_IJ with respect to the Young's
 * modulus of every voxel (nu fixed), from the solutions of the last
 * cell_effective_stiffness call: the problem is self-adjoint, so the adjoint
 * states are the primal solutions and dC*_IJ/dE_v =
 * (1/|Y|) sum_{s in v} |s| eps^I : (D_v / E_v) eps^J.  dJ_dC is host
 * [nv][nv]; dJ_dE_out has n values.  CELL_E_STATE before any solve. */
cell_status cell_adjoint(cell_t c, const double* dJ_dC, double* dJ_dE_out, int on_device);

/* Strain-based Fourier projection variant of the solve (3D, FP64, a
 * cross-check of the iteration; not built for speed): conjugate gradients
 * on compatible strain fields e = B u (one Voigt strain per simplex) with
 * the operator B M^-1 B^T D (M the Fourier-inverted reference operator of
 * the preconditioner) in the inner product sum_s |s| a_s . D0 b_s of the
 * reference medium.  Its iterates are the strains of the displacement PCG's
 * iterates: the same step lengths and, stopped on the same residual
 * ||f - K u|| <= tol ||f|| (the handle's tol and max_iter), the same
 * iteration counts.  nload (1..6) macro strains [nload][6] (host, Voigt,
 * engineering shear); writes the mean stresses [nload][6] (host, may be
 * NULL) and per-load iterations and relative residuals into info.  Allocates
 * its strain fields (about 1.2 KB per voxel) for the call; leaves no
 * solution for the getters.  CELL_E_UNSUPPORTED in 2D or for a batch;
 * CELL_E_STATE without a material or while a surrogate operator is set. */
cell_status cell_solve_projection(cell_t c, int nload, const double* macro_strain, double* mean_stress_out,
                                  cell_info* info);

/* Initial guess of load case `load` (0 <= load < max_loads) for the
 * linear solves that follow (cell_solve, cell_effective_stiffness): u0
 * [d][n], host or device (on_device); NULL clears it.  The values are
 * copied before the call returns (the handle's stream is synchronised).
 * The guess stays set across cell_set_material calls, so that a solve on a
 * perturbed material starts from an earlier solution, until it is cleared
 * or the handle destroyed.  The solve then starts from x = u0 with
 * r = f - K u0 recomputed in FP64 and stops on the same test as a cold
 * start (||f - K u|| <= tol ||f||); a guess that already passes it ends
 * that load with 0 iterations.  The per-component mean of u0 does not
 * matter (displacements are returned mean-free; C* and the gradient depend
 * on strains only).  Not used by cell_solve_hyper nor while a surrogate
 * stencil operator is set.  Errors: CELL_E_ARG for a load out of range or
 * non-finite host values (device values are checked through their residual:
 * the next solve returns CELL_E_ARG); CELL_E_NOMEM if the guess storage
 * ([max_loads][d][n] doubles, allocated at the first guess) cannot be
 * allocated. */
cell_status cell_set_initial_guess(cell_t c, int load, const double* u0, int on_device);

/* Displacement fluctuation of load `load` of the last solve, [d][n], each
 * component with zero nodal mean. */
cell_status cell_get_displacement(cell_t c, int load, double* u_out, int on_device);

/* Energy-form matrix (1/|Y|) sum |s| eps^I : D eps^J among the nload loads of
 * the last cell_solve / cell_effective_stiffness, host [nload][nload]
 * (for unit loads it is C*).  CELL_E_STATE before any solve. */
cell_status cell_energy_matrix(cell_t c, double* C_out);

/* Final residual f - K u of load `load` of the last solve, [d][n], as
 * recomputed from the FP64 solution (mixed precision: rounded to FP32 on the
 * device).  CELL_E_STATE before any solve. */
cell_status cell_get_residual(cell_t c, int load, double* r_out, int on_device);

/* Residual history of load `load` in the last linear solve (the PCG of
 * Sec. 2.1's static problem; for cell_solve_hyper, its last inner PCG):
 * hist_out[k] = ||r_k||_2 / ||f||_2 after k iterations, k = 0 the initial
 * residual, as the iteration tracks it (mixed precision: the FP32 iterated
 * residual between FP64 refreshes; the stopping test itself uses the FP64
 * recomputation).  *count_out receives the number of entries, min(iterations
 * + 1, min(max_iter + 1, 4096)) (a longer solve keeps its last entry in the
 * final slot); min(count, capacity) values are written to hist_out (host;
 * may be NULL when capacity is 0).  CELL_E_STATE before any solve of that
 * load, CELL_E_ARG for a load outside [0, max_loads) or a negative
 * capacity. */
cell_status cell_get_residual_history(cell_t c, int load, double* hist_out, int capacity, int* count_out);

void cell_destroy(cell_t c);

const char* cell_last_error(void);

/* Debugging aid.  The bounds-checked build of this library (compiled with
 * -DCELLFFT_BOUNDS_CHECK: paper_2004_05197_amd/build.py build_checked(),
 * libcellfft_checked.so) compares every field, spectrum, material and
 * reduction-partial access of the PCG iteration kernels (operator, x/y/z
 * FFT passes, finalize) and every partial written by the neo-Hookean and
 * surrogate kernels with the extent of the slot's buffer; an access out of
 * range is skipped (a load yields zero) and counted.  Returns the number
 * counted on the current device since the last call and clears the
 * counters (synchronises the device first); -2 if the device could not be
 * read.  The normal build checks nothing and returns -1. */
int cell_debug_bounds_violations(void);

/* ---- kernel-level entry points (parity checks of single steps) ---------- */

/* q = K u with the stencil kernel of the given precision (CELL_FP64 or
 * CELL_MIXED = FP32 arithmetic); u, q host [d][n]. */
cell_status cell_apply_operator(cell_t c, int precision, const double* u, double* q_out);

/* q = K u like cell_apply_operator in FP64, for callers that cannot
 * allocate device memory: code recorded under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc.  u and q are device arrays of d n
 * doubles ([d][n]) on the handle's device; uKu_out (device, one double, may
 * be NULL) receives u . K u.  The call allocates nothing, neither through
 * the handle nor otherwise: the reduction's per-block partials and its
 * scalar block use a library-owned static device array of 1 MiB (held by
 * each device the library runs on until the process ends); a stencil launch
 * with more blocks than it holds (131040) would return CELL_E_ARG, which no
 * supported grid reaches (256^3 in FP64 with z extent 8: 8192 blocks).
 * Asynchronous on the handle's stream (no synchronisation, no memset);
 * results are ready once that stream has reached them.  Every handle on one
 * device shares the array: calls that may overlap on one device (several
 * streams, several threads) race, calls ordered on one stream do not.
 * CELL_E_UNSUPPORTED while a surrogate stencil operator is set, CELL_E_STATE
 * without a material, CELL_E_ARG for null u or q. */
cell_status cell_apply_operator_noalloc(cell_t c, const double* u, double* q_out, double* uKu_out);

/* z = K_ref^{-1} r through the FFT passes of the given precision (the
 * zero-frequency component of z is 0); r, z host [d][n]; r should have zero
 * mean per component. */
cell_status cell_apply_preconditioner(cell_t c, int precision, const double* r, double* z_out);

/* Reference medium (lambda_0, mu_0) used by the preconditioner. */
cell_status cell_reference_medium(cell_t c, double* lam0, double* mu0);

/* ---- per-kernel timing --------------------------------------------------- */

/* Kernel kinds timed by cell_profile (HIP events on the handle's stream
 * around every launch). */
enum {
  CELL_K_APPLY = 0,     /* q = K p (fused stencil) */
  CELL_K_XFWD = 1,      /* r -= alpha q, FFT along x */
  CELL_K_YFWD = 2,      /* FFT along y (3D) */
  CELL_K_LAST = 3,      /* FFT, K_ref^{-1}, inverse FFT along the last axis */
  CELL_K_YINV = 4,      /* inverse FFT along y (3D) */
  CELL_K_XINV = 5,      /* inverse FFT along x, x and p updates */
  CELL_K_RESIDUAL = 6,  /* FP64 residual f - K u */
  CELL_K_MERGE = 7,     /* FP64 solution += FP32 correction */
  CELL_K_HOMOG = 8,     /* effective stiffness / mean stress */
  CELL_NKERNEL = 9
};

/* enable = 1: time every launch from now on (counters reset); 0: stop. */
cell_status cell_profile(cell_t c, int enable);

/* Accumulated milliseconds and launch counts per kernel kind
 * (CELL_NKERNEL entries each, host). */
cell_status cell_profile_read(cell_t c, double* ms_out, long long* launches_out);

/* ---- neo-Hookean cell problem (Newton's method) ----------------------------
 *
 * Compressible neo-Hookean energy density (Sec. 2.2, eq. NeoHookeanEnergy),
 * J = det F:  W(F) = lambda/2 (ln J)^2 - mu ln J + mu/2 (tr(F^T F) - tr I),
 * with F = F_bar + grad u on every simplex (2D: plane strain, F the in-plane
 * block).  For each macroscopic deformation gradient F_bar the periodic
 * fluctuation u minimising sum |s| W is found by Newton's method (Sec. 4,
 * nonlinear problems: the tangent is re-evaluated at every iterate).  Each
 * Newton step solves K_T(u) du = f(u) = -grad Pi by the same preconditioned
 * CG (Fourier reference medium, mixed or FP64 as configured, tolerance
 * cfg.tol on the step), then takes the largest step 1, 1/2, 1/4, ... that
 * keeps every J > 0 and decreases Pi by at least 1e-4 t f.du.  Residuals,
 * energies and stresses are evaluated in FP64. */
typedef struct {
  int nload;
  int newton_iters[6];   /* Newton steps per load */
  int cg_iters[6];       /* PCG iterations summed over the steps */
  double resnorm[6];     /* final ||f|| / max(||f_0||, |Y| max(|lambda| + 2 mu) max(|F_bar|, 1)) */
  double energy[6];      /* Pi / |Y| */
  int indefinite_steps[6]; /* Newton steps on an indefinite K_T: the inner PCG
                              met p.K_T p <= 0, or returned no descent direction */
  double seconds;
} cell_hyper_info;

/* nload (<= max_loads) macroscopic deformation gradients F_bar[nload][d][d]
 * (host, row-major; det > 0).  tol: stop when ||f|| <= tol times the scale
 * above (0 -> 1e-10); max_newton: 0 -> 50.  P_out (host, may be NULL):
 * [nload][d][d] mean first Piola-Kirchhoff stress.  Afterwards
 * cell_get_displacement returns the fluctuation of each load; the linear
 * results (cell_energy_matrix, cell_get_residual, cell_adjoint) are
 * CELL_E_STATE until the next linear solve.  Where K_T is not positive
 * definite, the inner PCG stops at the first direction with p.K_T p <= 0
 * and the step is the iterate reached so far, or the preconditioned
 * residual if that is the first direction (a descent direction either
 * way); a converged step that is no descent direction is replaced by one
 * PCG iteration.  CELL_E_BREAKDOWN if the line search finds no admissible
 * step. */
cell_status cell_solve_hyper(cell_t c, int nload, const double* F_bar, double tol, int max_newton, double* P_out,
                             cell_hyper_info* info);

/* Single steps of the Newton path (parity checks), on host arrays [d][n]:
 * q = K_T(u) p, the tangent at F = F_bar + grad u, in the given precision
 * (CELL_MIXED needs a mixed-precision handle); and f = -grad Pi(u) in FP64
 * with sums_out[10] (may be NULL) = sum |s| W, then sum |s| P (3 x 3
 * row-major; 2D uses the leading 2 x 2).  Invalidate the last solve. */
cell_status cell_apply_hyper_tangent(cell_t c, int precision, const double* F_bar, const double* u, const double* p,
                                     double* q_out);
cell_status cell_hyper_residual(cell_t c, const double* F_bar, const double* u, double* f_out, double* sums_out);

/* ---- surrogate stencil operator (Sec. 3.3, 3.4) ----------------------------
 * Replaces the operator of later cell_solve / cell_effective_stiffness calls
 * by its surrogate: the stencil functions K_delta(x_i) (the 3 x 3 blocks of K
 * coupling node i with node i + delta, delta in the seven nonzero 0/1
 * offsets x, y, z, xy, yz, xz, xyz) are computed exactly at every M-th node
 * along each axis and interpolated everywhere by periodic cardinal
 * B-splines of degree q (1 or 3) with knots at those nodes; the off-diagonal
 * blocks at -delta are the transposes, the diagonal block is minus the
 * symmetric part of the block row sum (eq.
 * DefinitionOfSurrogateMatrixSymmetricKernel).  The PCG then solves the
 * surrogate system over fluctuations with zero nodal mean, with the exact
 * load vectors; the reported C* is the exact energy form of the surrogate
 * solutions' strain fields (>= the exact C*, by the quadratic consistency
 * error), the mean stresses and residuals those of the exact operator at
 * them.  M = 0 switches the surrogate off (as does cell_set_material).
 * 3D single-cell handles; M must divide every grid size.  The stencil takes
 * 63 FP64 + 63 FP32 values per node of device memory.  cell_adjoint returns
 * CELL_E_STATE while a surrogate is set.  setup_seconds (may be NULL): time
 * of the sampling, the spline coefficients and the expansion. */
cell_status cell_set_surrogate(cell_t c, int M, int q, double* setup_seconds);
/* the interpolated stencil blocks, host [7][3][3][n] (FP64), offset order above */
cell_status cell_get_surrogate_stencil(cell_t c, double* blocks_out);

/* ---- autotuner ------------------------------------------------------------
 *
 * A schedule picks the compiled variant of each iteration kernel; all
 * variants compute the same operator (sums inside a block may be ordered
 * differently).  Six ints: stencil tile (0..4: fp32 64x4, 32x8, 16x16,
 * 64x8, 32x16; fp64 32x8, 16x16, 64x4, 32x16, 16x32 threads; 5: the fp32
 * row-wave operator, one wave per x-row of N_x = 64, 128 or 256 nodes; a
 * tile that does not fit the grid falls back to the first one that does,
 * or to the runtime tile), stencil z
 * extent (8, 16, 32, 64), x-pass rows per block (0: 2048/(N_x/2) complex
 * values, 1: half; fp64 half of these; 2, 3: the same with radix 16 first),
 * y-pass columns per block (0: 16, 1: 8; fp64 8, 4; 2, 3: the same with
 * radix 16 first), last pass columns x threads per block (0: 8 x 512,
 * 1: 4 x 512, 3D also 2: 8 x 768, 3: 16 x 1024; fp64 half the columns; 2D
 * takes 2, 3 as 0, 1), last-pass
 * radix order (0: radix 8 first, 1: radix 16 first).  Default
 * {0, 32, 0, 0, 0, 0}.
 *
 * cell_autotune times every variant on the handle's own buffers (material
 * must be set; the last solve is discarded) and keeps the fastest.  If the
 * environment variable CELLFFT_TUNE_CACHE names a file, schedules are
 * cached there (JSON object: key "arch|dim|grid|precision|slots" -> six
 * ints); force = 0 takes a cached schedule when one exists, and handles
 * created later with a cached key start from it. */
cell_status cell_autotune(cell_t c, int force);
cell_status cell_get_schedule(cell_t c, int* sched_out /* [6] */);
/* CELL_E_ARG for values outside the ranges above. */
cell_status cell_set_schedule(cell_t c, const int* sched /* [6] */);

/* ---- batches of independent cells ---------------------------------------
 *
 * ncell independent cells (microstructures), possibly of different grid
 * sizes, each solved for the same macro strains.  Cells of the same grid
 * (n and len) share one set of kernel launches: with lpc = max_loads slots
 * per cell, a launch covers ncell_g * lpc independent load cases, each with
 * its own material, reference medium and CG scalars.  Groups of different
 * grids advance in lockstep on one stream: one captured HIP graph holds a
 * chunk of iterations of every unfinished group (captured again when a
 * group finishes), with one host synchronisation per chunk for all groups.
 * Results equal those of one single-cell handle per cell (the same kernels
 * on the same data). */

/* cfgs[ncell]: per-cell configurations; dim, precision, tol, max_iter,
 * max_loads, stream and device must agree (else CELL_E_ARG). */
cell_status cell_batch_create(const cell_config* cfgs, int ncell, cell_batch_t* out);

/* Material of cell i (0 <= i < ncell), as cell_set_material. */
cell_status cell_batch_set_material(cell_batch_t b, int i, const double* E, const double* nu, int on_device);

/* Solve every cell for macro_strain[nload][nv]; mean_stress_out (host, may
 * be NULL) receives [ncell][nload][nv]; infos (may be NULL) [ncell]. */
cell_status cell_batch_solve(cell_batch_t b, int nload, const double* macro_strain, double* mean_stress_out,
                             cell_info* infos);

/* C* of every cell, C_out host [ncell][nv][nv]; infos (may be NULL) [ncell]. */
cell_status cell_batch_effective_stiffness(cell_batch_t b, double* C_out, cell_info* infos);

/* Displacement / final residual of load `load` of cell i after the last
 * batched solve, as cell_get_displacement / cell_get_residual ([d][n_i]). */
cell_status cell_batch_get_displacement(cell_batch_t b, int i, int load, double* u_out, int on_device);
cell_status cell_batch_get_residual(cell_batch_t b, int i, int load, double* r_out, int on_device);

/* Per-kernel timing summed over the batch's groups (as cell_profile). */
cell_status cell_batch_profile(cell_batch_t b, int enable);
cell_status cell_batch_profile_read(cell_batch_t b, double* ms_out, long long* launches_out);

/* Number of distinct grids (kernel-launch groups) in the batch. */
int cell_batch_groups(cell_batch_t b);

/* cell_autotune for every group of the batch. */
cell_status cell_batch_autotune(cell_batch_t b, int force);

void cell_batch_destroy(cell_batch_t b);

#ifdef __cplusplus
}
#endif

#endif /* CELLFFT_H */
