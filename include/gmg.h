/*
 * gmg.h -- C ABI of the MI355X (gfx950) geometric-multigrid-preconditioned
 * FGMRES solver for the variable-coefficient Poisson-type equation
 *
 *     -div(a grad phi) = f   on a uniform nx x ny x nz cell grid,
 *     phi = phi_bot on the plate z = 0, phi = phi_top on the plate z = 1,
 *     d phi / dn = 0 on the four x and y sides,
 *
 * the elliptic problem solved once per time step of the paper's semi-implicit
 * streamer scheme (Lin, Zhuang, Cai, Zeng, Bao, "An efficient and accurate
 * MPI-based parallel simulator for streamer discharges in three dimensions":
 * problem statement Sec. 1; discretisation eq. e18, Sec. 2.2; solver
 * Algorithm 1, Sec. 3.1; preconditioner Sec. 3.2; stopping rule eq. criterion,
 * Sec. 5.2).
 *
 * Discretisation (eq. e18): cell-centred finite volumes; the face coefficient
 * is the arithmetic mean of the two adjacent cells' a; the plates act through
 * a ghost cell mirrored through the plate (phi_g = 2 phi_b - phi_c) whose face
 * coefficient is the cell's own a; the sides carry no flux.  The linear system
 * is A phi = b with b = f + 2 a_c phi_b / hz^2 on the first and last z-layers.
 *
 * Layout of every field: float64, C order (nz, ny, nx), x fastest; cell
 * (i, j, k) is element (k*ny + j)*nx + i; cell centre ((i+1/2)hx, ...).
 * Every pointer named *_dev is a device pointer on the current HIP device.
 *
 * Ownership: the caller allocates and frees every device buffer, including
 * the workspace.  The context keeps the pointers a_dev (until the next
 * gmg_update_coefficient or gmg_destroy) and workspace_dev (until
 * gmg_destroy); it keeps no pointer to f, phi, x, y, lam or dLda after a call
 * returns.  gmg_destroy frees only host-side state.
 *
 * Streams: every kernel is enqueued on the stream given to gmg_setup (or
 * gmg_set_stream).  Calls block the host only where they must read a scalar
 * back (one read per Arnoldi step in fgmres_solve) and before returning.
 *
 * Threads: a context is not re-entrant; calls on one context must not
 * overlap.  Distinct contexts with distinct workspaces are independent.
 *
 * Errors: functions return a status code (never throw); gmg_status_string
 * gives its text.
 */
#ifndef GMG_H
#define GMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmg_ctx gmg_ctx;

enum {
  GMG_OK = 0,
  GMG_NOT_CONVERGED = 1, /* max_iter Arnoldi steps taken; phi holds the last iterate */
  GMG_ERR_ARG = -1,      /* null pointer, bad option, a <= 0, tol < 0 */
  GMG_ERR_SHAPE = -2,    /* grid does not coarsen to <= coarse_max_cells cells */
  GMG_ERR_NONFINITE = -3,/* NaN or Inf in a, f, phi (x0) or during the iteration */
  GMG_ERR_WORKSPACE = -4,/* workspace null, too small or misaligned (256 B) */
  GMG_ERR_HIP = -5,      /* a HIP runtime call failed */
  GMG_ERR_BREAKDOWN = -6 /* gmg_krylov_solve: a zero denominator in a method's recurrences */
};

enum { GMG_FP64 = 0, GMG_MIXED = 1 };

/* Finest-level smoother kernels (both run the same red-black Gauss-Seidel
 * arithmetic, so the choice changes speed only, and results at the level of
 * float32 rounding). */
enum { GMG_SWEEP_AUTO = 0, GMG_SWEEP_HALF = 1, GMG_SWEEP_FUSED = 2 };

/* Multigrid cycle applied by the preconditioner (Sec. 3.2: FMG on the first
 * time step, which starts from zero; V-cycles once the previous solution is
 * the guess). */
enum { GMG_CYCLE_V = 0, GMG_CYCLE_FMG = 1 };

/* Smoother of every level but the coarsest (Sec. 3.2).  GMG_SMOOTH_RBGS:
 * red-black symmetric Gauss-Seidel, nu_pre sweeps red-black before the coarse
 * correction and nu_post black-red after it.  GMG_SMOOTH_CHEBYSHEV: the
 * paper's own smoother, the degree-2 Chebyshev polynomial of eq. qntn in the
 * SSOR-preconditioned level operator M^{-1} A_l (M: one symmetric red-black
 * sweep from zero, red, black, red), nu_pre applications before and nu_post
 * after the coarse correction, with bounds lambda* = 0.1 lambda and
 * lambda_max = 1.1 lambda from lambda, the largest real part of the Ritz
 * values of 10 Arnoldi steps on M^{-1} A_l (estimated when the coefficient
 * is set; the start vector of level l is drawn by SplitMix64 seeded with l,
 * cell c taking output c + 1 mapped to [-1, 1) as 2 (z >> 11) 2^-53 - 1).
 * Chebyshev smoothing runs every level through per-level kernels (no
 * one-workgroup bottom kernel) and needs cold_cycle = warm_cycle =
 * GMG_CYCLE_V. */
enum { GMG_SMOOTH_RBGS = 0, GMG_SMOOTH_CHEBYSHEV = 1 };

/* Restriction of the V-cycle (Sec. 3.2; the paper's figure of the transfer
 * operators is missing, so both are readings).  GMG_RESTRICT_MEAN: the
 * residual averaged over the 8 children of a coarse cell (default).
 * GMG_RESTRICT_TRANSPOSE: R = P^T / 8, the transpose of the trilinear
 * prolongation with its ghost rules folded back (full weighting over the
 * 4 x 4 x 4 fine cells around a coarse cell); with nu_pre = nu_post the
 * V-cycle is then a symmetric positive definite operator, which the
 * conjugate gradient method of the comparison in Sec. 5.3 assumes.  The
 * transpose restriction runs as a residual pass and a restriction pass on
 * every level (no one-workgroup bottom kernel) and needs cold_cycle =
 * warm_cycle = GMG_CYCLE_V and the red-black smoother. */
enum { GMG_RESTRICT_MEAN = 0, GMG_RESTRICT_TRANSPOSE = 1 };

/* Solver options.  gmg_default_options fills the defaults given below. */
typedef struct gmg_options {
  int restart;          /* Krylov dimension m of FGMRES(m), 1..32 (default 10)   */
  int max_iter;         /* cap on Arnoldi steps over all restarts (default 200)  */
  int nu_pre;           /* pre-smoothing sweeps (Chebyshev: applications), 0..8
                           (default 2)                                           */
  int nu_post;          /* post-smoothing sweeps (applications), 0..8 (default 2) */
  int precision;        /* GMG_FP64: whole solve in float64; GMG_MIXED: V-cycle
                           (coefficients, smoother, transfers, coarse solve) in
                           float32, FGMRES in float64 (default GMG_MIXED)       */
  int coarse_max_cells; /* largest coarsest level solved directly (default 4096) */
  int fine_sweep;       /* red-black Gauss-Seidel smoothing kernels:
                           GMG_SWEEP_HALF: one kernel per red or black half-sweep;
                           GMG_SWEEP_FUSED: one kernel per symmetric sweep
                           (nu_pre, nu_post >= 1; on the finest level of a grid
                           of at least two levels, and on coarse levels above
                           the one-workgroup bottom with rows of at most 256
                           x-pairs in float32, 128 in float64; half-sweeps
                           elsewhere);
                           GMG_SWEEP_AUTO (default): fused where it was
                           measured faster (finest level: long z-chunks;
                           coarse levels: at least 128^3 cells) */
  int cold_cycle;       /* preconditioner of a solve with use_x0 = 0: GMG_CYCLE_FMG
                           (default) one full multigrid cycle per step,
                           GMG_CYCLE_V one V-cycle per step. */
  int graphs;           /* 1: each preconditioner application is captured
                           once into a HIP graph and replayed; 0 (default):
                           its kernels are launched one by one.  Results are
                           the same (the replays were not faster here: the
                           coarse-level kernels wait on the GPU's dispatch
                           latency, not on the host). */
  int smoother;         /* GMG_SMOOTH_RBGS (default) or GMG_SMOOTH_CHEBYSHEV */
  int warm_cycle;       /* preconditioner of a solve with use_x0 = 1:
                           GMG_CYCLE_V (default, the paper's choice) or
                           GMG_CYCLE_FMG (full multigrid cycles: fewer steps
                           on the time loops measured; the cycle acts on the
                           Krylov vectors, so either serves a warm start) */
  int restriction;      /* GMG_RESTRICT_MEAN (default) or GMG_RESTRICT_TRANSPOSE */
} gmg_options;

void gmg_default_options(gmg_options* opt);

/* Bytes of device workspace a grid needs (0 if the shape or options are
 * invalid).  The workspace must be 256-byte aligned. */
size_t gmg_workspace_bytes(int nx, int ny, int nz, const gmg_options* opt);

/* Build the multigrid hierarchy for coefficient a (float64, > 0, finite)
 * on an nx x ny x nz grid with spacings hx, hy, hz (Sec. 2.2).  Levels halve
 * every dimension while all are even and >= 4 (Sec. 3.2, 2x2x2 agglomeration);
 * the coarsest level (<= coarse_max_cells cells) is solved directly (Sec. 3.2,
 * coarsest-mesh direct solver).  hip_stream is a hipStream_t (NULL = default
 * stream).  On success *out receives the context. */
int gmg_setup(int nx, int ny, int nz, double hx, double hy, double hz,
              const double* a_dev, const gmg_options* opt, void* workspace_dev,
              size_t workspace_bytes, void* hip_stream, gmg_ctx** out);

/* Replace the coefficient (same grid) and rebuild the hierarchy: the
 * per-time-step renewal of operator and preconditioner (Sec. 2.1, last
 * paragraphs). */
int gmg_update_coefficient(gmg_ctx* ctx, const double* a_dev);

/* Change the stream later calls enqueue on. */
int gmg_set_stream(gmg_ctx* ctx, void* hip_stream);

/* FGMRES(m) (Algorithm 1), right-preconditioned by one multigrid cycle per
 * step (Sec. 3.2; opt->cold_cycle or opt->warm_cycle picks the full
 * multigrid cycle or the V-cycle from a zero guess), on A phi = b.  Stops when the relative
 * residual ||b - A phi|| / ||b|| < tol (eq. criterion; the in-cycle least-
 * squares estimate triggers the check, the true residual decides it) or after
 * opt->max_iter Arnoldi steps.
 *   f_dev        right side f (nz*ny*nx float64), read only.
 *   phi_bot/top  plate values.
 *   tol          relative tolerance >= 0 (tol = 0 runs exactly max_iter steps).
 *   phi_dev      output phi; if use_x0 != 0 it holds the initial guess on
 *                entry (warm start), otherwise it is overwritten.
 *   iterations   (may be NULL) Arnoldi steps taken over all restarts.
 *   res_hist     (may be NULL) res_hist[0] = ||b - A x0|| / ||b||, then one
 *                least-squares estimate per step; at most res_hist_cap
 *                entries are written, *res_hist_len (may be NULL) gets the
 *                number written.
 *   final_true_relres (may be NULL) recomputed ||b - A phi|| / ||b||.
 * b = 0 gives phi = 0, 0 steps, GMG_OK.
 * Returns GMG_OK, GMG_NOT_CONVERGED or an error. */
int fgmres_solve(gmg_ctx* ctx, const double* f_dev, double phi_bot,
                 double phi_top, double tol, double* phi_dev, int use_x0,
                 int* iterations, double* res_hist, int res_hist_cap,
                 int* res_hist_len, double* final_true_relres);

/* Largest workspace (gmg_workspace_bytes) fgmres_solve_static accepts: 64 MiB,
 * enough for a 64^3 grid in either precision.  The library holds this much
 * device memory on every GPU it runs fgmres_solve_static on, from the first
 * such call until the process ends. */
#define GMG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): gmg_setup followed by fgmres_solve and
 * gmg_destroy in one call, whose workspace is a device array of
 * GMG_STATIC_SCRATCH_BYTES the library holds per GPU instead of a
 * caller-allocated one.  It allocates no device or pinned host memory and
 * calls no allocating HIP or torch routine (its host bookkeeping uses the C++
 * heap).  Arguments: those of gmg_setup without the workspace (the grid,
 * spacings, coefficient a_dev, options, stream), then those of fgmres_solve
 * without the context; results, the initial guess (use_x0) and every status
 * as there.  opt->graphs must be 0 (GMG_ERR_ARG otherwise: capturing a graph
 * allocates).  GMG_ERR_WORKSPACE, with nothing launched, when the grid's
 * workspace exceeds GMG_STATIC_SCRATCH_BYTES; GMG_ERR_HIP when the array's
 * device address cannot be obtained.  Every call on one GPU uses the same
 * array and nothing in it needs clearing (each buffer is written before it is
 * read), which the next call overwrites: calls that overlapped on one GPU
 * would race on it, so the library runs them one at a time (a lock per GPU,
 * held until the call has synchronised its stream). */
int fgmres_solve_static(int nx, int ny, int nz, double hx, double hy, double hz, const double* a_dev,
                        const gmg_options* opt, void* hip_stream, const double* f_dev, double phi_bot,
                        double phi_top, double tol, double* phi_dev, int use_x0, int* iterations, double* res_hist,
                        int res_hist_cap, int* res_hist_len, double* final_true_relres);

/* Krylov methods with the same multigrid preconditioner, for the comparison
 * of Sec. 5.3 (Table t1).  GMRES is right-preconditioned (Arnoldi on A M, the
 * update applies M to V y); CG is the preconditioned conjugate gradient; FCG
 * its flexible form with the new direction made A-orthogonal to the last one;
 * CGS and BiCGSTAB are right-preconditioned. */
enum {
  GMG_KRYLOV_FGMRES = 0,
  GMG_KRYLOV_GMRES = 1,
  GMG_KRYLOV_CG = 2,
  GMG_KRYLOV_FCG = 3,
  GMG_KRYLOV_CGS = 4,
  GMG_KRYLOV_BICGSTAB = 5
};

/* Solve A phi = b (as fgmres_solve) with `method`, one V-cycle from zero per
 * preconditioner application whatever the initial guess (the comparison uses
 * the same preconditioner for every method).  Stops on the relative residual
 * of eq. criterion: the recursively updated residual triggers the check, the
 * true residual b - A phi decides it (a method restarts from phi when it
 * fails), or after opt->max_iter iterations.  iterations (may be NULL): the
 * method's iterations (CGS and BiCGSTAB apply the preconditioner twice per
 * iteration); precond_apps (may be NULL): preconditioner applications;
 * final_true_relres (may be NULL).  CG and FCG use basis slots 0-3, CGS and
 * BiCGSTAB 0-7 of the workspace: they need restart >= 3 and >= 7
 * (GMG_ERR_ARG otherwise).  Returns GMG_OK, GMG_NOT_CONVERGED,
 * GMG_ERR_BREAKDOWN (a zero denominator in the recurrences) or an error. */
int gmg_krylov_solve(gmg_ctx* ctx, int method, const double* f_dev, double phi_bot, double phi_top, double tol,
                     double* phi_dev, int use_x0, int* iterations, int* precond_apps, double* final_true_relres);

/* y = A x - lifting: the left side of e18 on cell values x with plate values
 * phi_bot, phi_top (so y = f exactly when x solves the problem).  x and y
 * must not overlap. */
int gmg_apply_operator(gmg_ctx* ctx, const double* x_dev, double* y_dev,
                       double phi_bot, double phi_top);

/* One V-cycle from a zero guess with right side v (Sec. 3.2, last
 * paragraph): z = M v, in the context's precision (in GMG_MIXED, v is rounded
 * to float32 and the float32 result is promoted exactly).  v and z must not
 * overlap. */
int gmg_vcycle(gmg_ctx* ctx, const double* v_dev, double* z_dev);

/* One full multigrid cycle with right side v (Sec. 3.2, FMG for a solve
 * without an initial guess): the right side restricted (mean of the 8
 * children) to every level, the coarsest level solved directly, then on each
 * finer level one V-cycle from the interpolated coarser result.  z = F v, a
 * fixed linear map; precision, layout, overlap and errors as gmg_vcycle. */
int gmg_fmg(gmg_ctx* ctx, const double* v_dev, double* z_dev);

/* Gradient with respect to the coefficient of a loss L(phi) through the
 * solve, given phi (the solution for plate values phi_bot, phi_top) and the
 * adjoint lam (the solution of A lam = dL/dphi with zero plate values):
 *   dLda_c = -1/2 * sum over the faces of cell c of (d phi)_f (d lam)_f,
 * with (d u)_f = (u_nb - u_c)/h on interior faces, the half-cell quotients
 * (phi_c - phi_b)/(hz/2) and lam_c/(hz/2) on plate faces, and no term on the
 * sides (derived from e18).  dL/df is lam itself. */
int gmg_face_flux_grad(gmg_ctx* ctx, const double* phi_dev,
                       const double* lam_dev, double phi_bot, double phi_top,
                       double* dLda_dev);

/* Parameters of the elliptic problem of one semi-implicit step (Sec. 2.1,
 * eq. semi2 / e15; Sec. 2.2, definition of P^n and eq. e18). */
typedef struct gmg_step_params {
  double eps0_over_e; /* eps0 / e: the vacuum part of the coefficient         */
  double tau_eff;     /* tau_n / 2 for the predictor of the second-order scheme
                         (eq. semi2), tau_n for the first-order scheme (e15)   */
  double mu_e, mu_p;  /* electron and ion mobilities                           */
  double De[3];       /* electron diffusion coefficients D_x, D_y, D_z         */
} gmg_step_params;

/* Coefficient and right side of the elliptic problem of a semi-implicit step
 * from the densities (Sec. 2.2): a = P = eps0/e + tau_eff (mu_p n_p + mu_e n_e)
 * and f = n_p - n_e - tau_eff sum_d D_d / h_d^2 delta_d^2 n_e (eq. e18), the
 * second differences with ghost cells equal to the boundary cells (the
 * homogeneous Neumann condition of n_e, Sec. 1).  ne, np, a, f: nz*ny*nx
 * float64 on the context's grid (x fastest); a and f must not overlap ne or
 * np.  a then goes to gmg_update_coefficient and f to fgmres_solve.  Errors:
 * GMG_ERR_ARG for null pointers or non-finite parameters. */
int gmg_assemble_elliptic(gmg_ctx* ctx, const double* ne_dev, const double* np_dev, const gmg_step_params* prm,
                          double* a_dev, double* f_dev);

/* Electric field E = -grad phi by central differences (Sec. 2.2, after eq.
 * e18) and |E|: ghost cells equal to the boundary cells on the x and y sides
 * (Neumann), mirrored through the plates (2 phi_b - phi_c) with plate values
 * phi_bot, phi_top.  All arrays nz*ny*nx float64; the outputs must not overlap
 * phi.  Errors: GMG_ERR_ARG for null pointers or non-finite plate values. */
int gmg_electric_field(gmg_ctx* ctx, const double* phi_dev, double phi_bot, double phi_top, double* ex_dev,
                       double* ey_dev, double* ez_dev, double* emag_dev);

/* The elliptic half of one time step of the semi-implicit schemes (Sec.
 * 2.1): from the densities at t_n, the coefficient and right side
 * (gmg_assemble_elliptic, into the caller's a_dev and f_dev: prm->tau_eff =
 * tau/2 for eq. semi2 of the second-order scheme, tau for eq. e15 of the
 * first-order one), the coefficient renewal (gmg_update_coefficient with
 * a_dev, which the context keeps), the solve (fgmres_solve, warm-started
 * from phi_dev when use_x0 != 0, Sec. 3.2) and the field E = -grad phi and
 * |E| of the solution (gmg_electric_field), in one call with one wait at
 * the end.  ne, np, a, f, phi, ex, ey, ez, emag: nz*ny*nx float64 on the
 * context's grid, a and f distinct from ne, np; phi_dev holds phi^{n+1/2}
 * (second order) or phi^{n+1} (first order) on return.  iterations and
 * final_true_relres (may be NULL) as in fgmres_solve.  Returns the solve's
 * status (GMG_OK or GMG_NOT_CONVERGED) or an error of any of the steps. */
int gmg_elliptic_step(gmg_ctx* ctx, const double* ne_dev, const double* np_dev, const gmg_step_params* prm,
                      double phi_bot, double phi_top, double tol, double* a_dev, double* f_dev, double* phi_dev,
                      int use_x0, double* ex_dev, double* ey_dev, double* ez_dev, double* emag_dev, int* iterations,
                      double* final_true_relres);

/* The density half of the time step (Sec. 2.1): n_out = n + dt L for both
 * species, L the time derivatives the caller's transport operator (drift,
 * diffusion and source of the density equations, which this library does not
 * discretise) gives for the field of gmg_elliptic_step: dt = tau/2 with L at
 * t_n for the predictor of eq. e1, dt = tau with L at t_n + tau/2 for the
 * corrector of eq. e2 (both from n at t_n), dt = tau with L at t_n for the
 * first-order scheme.  All arrays nz*ny*nx float64; the outputs may be the
 * inputs ne_dev, np_dev.  Errors: GMG_ERR_ARG for null pointers or a
 * non-finite dt. */
int gmg_density_update(gmg_ctx* ctx, const double* ne_dev, const double* np_dev, const double* le_dev,
                       const double* lp_dev, double dt, double* ne_out, double* np_out);

/* Hierarchy description: number of levels and, for level l < cap, its
 * (nx, ny, nz) in shapes[3l..3l+2]. */
int gmg_get_levels(gmg_ctx* ctx, int* nlevels, int* shapes, int cap);

/* Chebyshev smoother (options.smoother = GMG_SMOOTH_CHEBYSHEV): the
 * Arnoldi estimate lambda of each smoothed level (the coarsest is solved
 * directly), from the coefficient last given to gmg_setup or
 * gmg_update_coefficient; the bounds of eq. qntn are 0.1 and 1.1 lambda.
 * Writes *nlevels (levels minus one) and the first min(cap, *nlevels)
 * values to lam (host).  GMG_ERR_ARG for a context with the red-black
 * smoother or null pointers. */
int gmg_chebyshev_estimates(gmg_ctx* ctx, double* lam, int cap, int* nlevels);

/* Host step of the estimate above (no GPU work): the largest real part of
 * the eigenvalues of the m x m upper Hessenberg matrix H (row-major, row
 * stride ldh >= m; entries below the subdiagonal are ignored), by the Francis
 * double-shift QR iteration, into *out.  H is not modified.  GMG_ERR_ARG
 * for null pointers, m < 1 or m > 64, ldh < m, or non-finite entries;
 * GMG_NOT_CONVERGED if the iteration did not converge. */
int gmg_ritz_max_real(const double* H, int m, int ldh, double* out);

/* Per-kernel timing with HIP events on the context's stream.  While enabled,
 * every kernel launch is bracketed by events; gmg_profile_read sums the
 * elapsed times per kernel name since the last reset (it synchronises the
 * stream).  names[i] point to static strings. */
int gmg_profile_enable(gmg_ctx* ctx, int enable);
int gmg_profile_reset(gmg_ctx* ctx);
int gmg_profile_read(gmg_ctx* ctx, const char** names, double* total_ms,
                     long long* launches, int cap, int* count);

void gmg_destroy(gmg_ctx* ctx);

const char* gmg_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* GMG_H */
