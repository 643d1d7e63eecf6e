/*
 * imexhdg.h -- C ABI of the MI355X (gfx950) engine for the geometry-split
 * additive Runge-Kutta IMEX scheme with explicit DG-IP and implicit HDG-IP /
 * HDG-MX of Ellmenreich, Shehadi and Lederer ("IMEX Schemes for Compressible
 * Flow using Hybridizable Discontinuous Galerkin Methods").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: imex_status; 0 on success, < 0 on error.  No entry point
 *   throws or aborts; on error imex_last_error() holds a message and no output
 *   has been modified unless stated otherwise.
 * - Pointers named "dev" are device pointers (hipMalloc'd or from torch) on the
 *   device the context was created on; all work is queued on the context's
 *   stream and the call returns once that work is complete.  Pointers named
 *   "host" are host memory.  The caller owns every pointer it passes; the
 *   library owns its workspaces (allocated in imex_create / imex_set_regions,
 *   freed in imex_destroy).
 * - Mesh (Sec. 3.1): 2D tensor-product mesh of nx x ny axis-aligned quads;
 *   element e = i + nx*j covers [x_i, x_{i+1}] x [y_j, y_{j+1}].
 * - Element state layout: U[e][v][n], e over ALL elements, v = 0..3 for
 *   (rho, rho u, rho v, rho E), n = a + (k+1) b the nodal index of the
 *   Gauss-Legendre node (xi_a, xi_b), x fastest.  FP64.
 * - Facet state layout: Uhat[f][v][m], f over the HDG facets (facets touching
 *   an implicit element) in the library's order (vertical facets first, then
 *   horizontal, each lexicographic), m = facet node in increasing coordinate.
 * - A context is not safe for concurrent use from several threads.
 */
#ifndef IMEXHDG_H
#define IMEXHDG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IMEX_OK = 0,
  IMEX_EINVAL = -1,      /* bad argument: sizes, flags, null pointer            */
  IMEX_ENOMEM = -2,      /* device allocation failed                             */
  IMEX_EDEVICE = -3,     /* a HIP call failed                                    */
  IMEX_ENOCONV = -4,     /* Newton did not converge; state left at last iterate  */
  IMEX_ENONFINITE = -5,  /* a non-finite value appeared in the Newton iteration  */
  IMEX_ENOTIMPL = -6,    /* option combination not implemented                   */
  IMEX_ESTATE = -7       /* call order violated (e.g. solve before set_regions)  */
} imex_status;

enum { IMEX_BC_PERIODIC = 0, IMEX_BC_FARFIELD = 1, IMEX_BC_WALL = 2 };
enum { IMEX_FLUX_VIJAYASUNDARAM = 0, IMEX_FLUX_LAX_FRIEDRICHS = 1 };   /* DG convective flux        */
enum { IMEX_HDG_FLUX_FVS = 0, IMEX_HDG_FLUX_LF = 1 };                  /* HDG stabilisation S_c     */
enum { IMEX_HDG_IP = 0, IMEX_HDG_MX = 1 };                             /* implicit formulation      */
enum { IMEX_FP64 = 0, IMEX_FP32_REFINE = 1 };                          /* implicit linear algebra   */

typedef struct imex_ctx imex_ctx;

/* Mesh and degree (Sec. 3.1).  bc[] for the sides -x, +x, -y, +y; periodic must
 * be set on both sides of an axis.  degree k in 1..4; the volume and facet rules
 * use ceil((3k+1)/2) Gauss points per direction (over-integration, Sec. 5). */
typedef struct {
  int nx, ny;
  const double* xgrid;   /* host, nx+1 strictly increasing */
  const double* ygrid;   /* host, ny+1 strictly increasing */
  int bc[4];
  int degree;
} imex_mesh_desc;

/* Gas model (Sec. 2): ideal gas p = rho R theta, constant mu, kappa = c_p mu / Pr,
 * lambda = -2 mu / 3.  viscous = 0 gives the Euler equations.  u_inf is the
 * conservative far-field state (App. B). */
typedef struct {
  double gamma, R, mu, Pr;
  int viscous;
  double u_inf[4];
} imex_physics;

typedef struct {
  int dg_flux;           /* IMEX_FLUX_*                                                     */
  int hdg_flux;          /* IMEX_HDG_FLUX_*                                                 */
  int hdg_variant;       /* IMEX_HDG_IP | IMEX_HDG_MX                                       */
  double alpha_dg;       /* IP penalty factor of DG (1 in the paper, Sec. 3.3)              */
  double alpha_hdg;      /* IP penalty factor of HDG-IP (10 in the paper, Sec. 3.4)         */
  int precision;         /* IMEX_FP64 | IMEX_FP32_REFINE                                    */
  double newton_rtol;    /* stop when max|dU| <= rtol max|U| and max|dUhat| <= rtol max|Uhat| */
  int newton_maxit;
  double gmres_rtol;     /* relative residual of the condensed facet solve                  */
  int gmres_restart;     /* 1..64                                                           */
  int gmres_maxit;
  /* Newton corrections that reuse the last Jacobian (simplified Newton steps: the
   * condensed factors of the previous iterate with a fresh FP64 residual, one facet
   * solve, no assembly or condensation).  Convergence is still certified by the
   * increment test above, on the measured contraction of each correction.
   *   0  every correction assembles and condenses the Jacobian at the current iterate
   *   1  after two full iterations, while the last correction contracted by < 1/20
   *   2  after the first full iteration, under the same contraction bound (the Jacobian
   *      is frozen within a stage, a variant the paper leaves out)
   * A simplified correction that contracts more slowly hands back to full iterations. */
  int newton_simplified;
  /* Forcing term of the facet solves (inexact Newton): 0 solves every correction to
   * gmres_rtol; 1 solves correction k to max(gmres_rtol, min(1e-4, dz_{k-1} / 100)), with
   * dz_{k-1} the relative size of the previous correction of the stage (1e-4 for the
   * first); 2 solves the first full correction of each stage loosely, to
   * max(gmres_rtol, min(1e-5, q / 100)) with q the contraction of the second correction
   * against the first in the previous stage of this context (gmres_rtol until one has
   * been measured), and the later full corrections to gmres_rtol; 3 (the recommended
   * setting) solves the first two full corrections so.  The first correction's linear
   * error stays a hundredth of the second correction; the second's is removed by the
   * correction that follows it, or is below newton_rtol when the stage stops there.  The
   * corrections and Jacobians are those of 0 on the workloads measured.  Convergence is certified by the increment
   * test either way.  (The facet solve of a simplified correction, which only certifies
   * convergence, always stops at 1e-4.) */
  int gmres_forcing;
} imex_options;

/* ARK pair synchronised by padding (Sec. 4.2.2): explicit (s+1)x(s+1) tableau Ae
 * (row-major in a 4x4 array), weights be[s+1]; implicit s x s tableau Ai (row-major
 * in a 3x3 array), weights bi[s].  s in 1..3. */
typedef struct {
  int s;
  double Ae[16];
  double be[4];
  double Ai[9];
  double bi[3];
  int fsal;              /* be == last row of Ae and c = 1: U^ex_{n+1} = y^ex_{s+1}       */
  int stiffly_accurate;  /* bi == last row of Ai and c = 1: U^im_{n+1} = y^im_s           */
} imex_tableau;

typedef struct {
  int newton_its;        /* Newton iterations (summed over stages for a step)             */
  int gmres_its;         /* GMRES iterations (summed)                                     */
  double newton_last_du; /* last max|dU| / max|U|                                         */
  double t_assemble_ms;  /* device time in assembly + condensation                        */
  double t_solve_ms;     /* device time in the facet solve                                */
  int n_jacobians;       /* Newton corrections that assembled a Jacobian (the rest reused one) */
  int n_hist;            /* entries of du_hist in use                                     */
  double du_hist[24];    /* per Newton iteration, in order over the stages of a step:
                            max(max|dU|/max|U|, max|dUhat|/max|Uhat|) of its increment   */
} imex_stats;

/* Create a context for one mesh on the current HIP device.  stream: hipStream_t
 * or NULL for the default stream.  Errors: EINVAL (bad mesh, degree, options),
 * ENOMEM, EDEVICE. */
imex_status imex_create(const imex_mesh_desc* mesh, const imex_physics* phys, const imex_options* opt,
                        void* stream, imex_ctx** out);

/* A batch of n_inst independent meshes of the same degree advanced together
 * (one context over their disjoint union: every kernel runs over all instances
 * in one launch, Newton and GMRES treat the block-diagonal union system).
 * meshes host [n_inst]; dt_scale host [n_inst] or NULL: instance k steps with
 * dt * dt_scale[k] wherever a call takes dt or dt_aii.  Elements are numbered
 * instance by instance (instance k starts after the elements of instances
 * 0..k-1), each instance lexicographically as in imex_create; HDG facets and
 * the flags of imex_set_regions follow the same instance order.  Physics and
 * options are shared.  Errors as imex_create, EINVAL for mixed degrees. */
imex_status imex_create_batch(int n_inst, const imex_mesh_desc* meshes, const double* dt_scale,
                              const imex_physics* phys, const imex_options* opt, void* stream, imex_ctx** out);

/* Geometry split T = T^im U T^ex (Sec. 4, eq. union_mesh): implicit_flag[e] != 0
 * marks element e implicit.  host, n_elem bytes.  Builds the HDG facet set and
 * allocates the implicit workspaces.  Errors: EINVAL (explicit element on a wall
 * boundary), ENOMEM. */
imex_status imex_set_regions(imex_ctx* ctx, const unsigned char* implicit_flag);

/* out[0..7] = n_elem, n_implicit, n_explicit, nodes per element, n_hdg_facets,
 *             unknowns per facet (4(k+1)), quadrature points per direction,
 *             workspace bytes.  host. */
imex_status imex_query_sizes(const imex_ctx* ctx, long long out[8]);

/* Physical coordinates of the element nodes, host arrays x[n_elem*nn], y[n_elem*nn]. */
imex_status imex_node_coords(const imex_ctx* ctx, double* x_host, double* y_host);

/* Facet state from element traces: mean of the adjacent traces at the facet nodes,
 * the explicit trace on interface facets (their Dirichlet value, eq.
 * interface_bilinearform_implicit_facet).  U dev (all elements), Uhat dev (out). */
imex_status imex_init_facets(imex_ctx* ctx, const double* U, double* Uhat);

/* Transpose of imex_init_facets (a linear map): Ubar += (dUhat/dU)^T Uhatbar, for
 * runs whose facet state starts from the element traces.  Uhatbar dev [n_hf][4][k+1]
 * (read); Ubar dev [E][4][(k+1)^2] (accumulated).  Deterministic (no atomics).
 * Errors: EINVAL (null argument), ESTATE (regions not set). */
imex_status imex_vjp_init_facets(imex_ctx* ctx, const double* Uhatbar, double* Ubar);

/* Wall shear of the HDG-MX region: J = sum over adiabatic-wall faces of implicit
 * elements of the integral of 2 mu eps_12 = mu (du/dy + dv/dx), with eps_12 the
 * stored strain component of the mixed variables (Sec. 3.5) lifted from (U, Uhat).
 * It is the integrand of a time-averaged wall-shear objective.  U, Uhat dev (read);
 * J host out.  Errors: ENOTIMPL without an HDG-MX region (viscous), EINVAL, ESTATE. */
imex_status imex_wall_shear(imex_ctx* ctx, const double* U, const double* Uhat, double* J);

/* Adjoint of imex_wall_shear: Ubar += Jbar dJ/dU, Uhatbar += Jbar dJ/dUhat (through the
 * lifting of the mixed variables).  Ubar dev [E][4][(k+1)^2], Uhatbar dev
 * [n_hf][4][k+1], both accumulated.  Errors as imex_wall_shear. */
imex_status imex_vjp_wall_shear(imex_ctx* ctx, const double* U, const double* Uhat, double Jbar, double* Ubar,
                                double* Uhatbar);

/* Explicit DG-IP residual R^DG (Sec. 3.3, eq. bilinear_form_interior_sdg with the
 * far-field form of App. B.1.1 and the interface form of eq.
 * interface_bilinearform_explicit), with M dU/dt = -R.  U dev, all elements
 * (implicit entries supply the interface traces y^im); Uhat dev, used only for
 * HDG-MX coupling (the implicit side's mixed variables are lifted from U, Uhat),
 * may be NULL otherwise; R dev out, rows of explicit elements written, rows of
 * implicit elements set to zero. */
imex_status imex_dg_residual(imex_ctx* ctx, const double* U, const double* Uhat, double* R);

/* imex_dg_residual for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same result from
 * the same kernels, with its scratch (face traces, and the lifted mixed variables of an
 * HDG-MX region) in a static device array of 96 MiB per device (12 582 912 doubles) that
 * the library holds until the process ends, instead of the context's workspace.  It
 * calls no hipMalloc / hipFree and no allocating library routine; R is cleared by a
 * kernel, not a memset.  Limit: E * 4 * NQ * 8 doubles of face traces (NQ Gauss points
 * per face) plus, with HDG-MX coupling, E * 5 * (k+1)^2 doubles of mixed variables must
 * fit in the array (the 256 x 128, k = 4 boundary layer needs 11 436 032); larger meshes
 * get EINVAL and nothing runs.  Every call on a device shares that device's array, which keeps the
 * last call's contents: calls that overlap on one device (several contexts or streams)
 * race and must be serialised by the caller.  U dev (all elements), Uhat dev (required
 * with an HDG-MX region, else may be NULL), R dev out as imex_dg_residual.
 * Errors: EINVAL (null argument, Uhat missing, mesh above the limit), ESTATE (regions
 * not set), EDEVICE (the array's device address could not be resolved). */
imex_status imex_dg_residual_noalloc(imex_ctx* ctx, const double* U, const double* Uhat, double* R);

/* One SDIRK stage of the implicit region (eqs. dirk_stage_update_solution /
 * _facet / _mixed) solved by Newton (Sec. 4.3) with static condensation
 * (eqs. statically_condensed_system, SchurCompliment, local_solve_static_condensation)
 * and a GMRES facet solve:
 *   M y + dt_aii R^HDG(y, yhat) - rhs = 0,  Rhat(y, yhat, U^ex) = 0.
 * rhs dev [e][v][n] (implicit rows read); U dev inout: explicit rows are the
 * interface data y^ex_{i+1} (read), implicit rows the initial guess on entry and
 * the stage solution on exit; Uhat dev inout; R_out dev (nullable): R^HDG at the
 * converged state in implicit rows.  st host (nullable).
 * Convergence is certified only by corrections whose facet solve reached gmres_rtol; a
 * solve stopped by gmres_maxit is followed by another full correction.
 * Errors: ESTATE (no implicit region), ENOCONV (newton_maxit corrections without a
 * certified increment; U, Uhat hold the last iterate), ENONFINITE (a non-finite residual
 * or increment: NaN or Inf in the inputs or a diverging iteration). */
imex_status imex_implicit_stage_solve(imex_ctx* ctx, double dt_aii, const double* rhs, double* U,
                                      double* Uhat, double* R_out, imex_stats* st);

/* One time step of Alg. imex_scheme_update (App. C) from t_n to t_n + dt:
 * U dev inout (all elements), Uhat dev inout.  st host (nullable).
 * The tableau is checked before any work: s in 1..3, Ae strictly and Ai lower
 * triangular, fsal and stiffly_accurate equal to what the coefficients say.
 * Errors: EINVAL (bad tableau, flags that disagree with it, dt <= 0, Uhat NULL with
 * an implicit region), ENOTIMPL (an implicit region with an implicit tableau that is
 * not stiffly accurate), ESTATE (regions not set), and the errors of
 * imex_implicit_stage_solve, after which U is unchanged and Uhat holds the failed
 * stage's last iterate. */
imex_status imex_ark_step(imex_ctx* ctx, const imex_tableau* tab, double dt, double* U, double* Uhat,
                          imex_stats* st);

/* Manufactured-solution source (Sec. 5.1.1, method of manufactured solutions): with on != 0
 * every imex_ark_step adds S = dU_e/dt + div(F^c(U_e) - F^nu(U_e, grad U_e)) of the exact
 * solution U_e = (s, s, s, s^2), s = sin(pi (kx x + ky y) - omega pi t) + 4, to the equations:
 * the explicit residual of stage i takes R^DG - b(t_n + cbar_i dt), the implicit stage i solves
 * M y + dt a_ii (R^HDG(y) - b(t_n + c_i dt)) = rhs and passes R^HDG - b to later stages, with
 * b[e][v][n] = int_T S_v phi_n.  params host [3] = kx, ky, omega; t0 = the time of the state the
 * next step starts from; each successful imex_ark_step advances that clock by dt.  on = 0
 * removes the source (and sets the clock to t0).  The adjoint entry points return ENOTIMPL
 * while a source is set.  Errors: EINVAL (null or non-finite parameters; a batch with
 * per-instance time-step scales), ENOMEM. */
imex_status imex_set_mms_source(imex_ctx* ctx, const double params[3], double t0, int on);

/* The source's load vector at time t: b[e][v][n] = int_T S_v(x, t) phi_n dx over all
 * elements (dev out [E][4][(k+1)^2]), with the volume Gauss rule.  Errors: ESTATE (no source
 * set), EINVAL. */
imex_status imex_mms_load(imex_ctx* ctx, double t, double* b);

/* out[v] = sum over elements of int_T U_v (host, 4 doubles); U dev. */
imex_status imex_conservation_sums(imex_ctx* ctx, const double* U, double out[4]);

/* Element-local Newton system of the implicit stage (inspection of the assembly):
 * for each implicit element (in increasing element index) the residual rows f
 * [NU], facet rows h [NF] and the blocks K [NU x NU], C [NU x NF], D [NF x NU],
 * E [NF x NF] (row-major) of the linearisation in (U_T, Uhat on dT), with the
 * mixed variables eliminated for HDG-MX.  NU = 4 (k+1)^2, NF = 16 (k+1), facet
 * unknowns of an element ordered face 0..3 (x-, x+, y-, y+), then variable, then
 * node.  All pointers dev, sized for n_implicit elements. */
imex_status imex_local_system(imex_ctx* ctx, double dt_aii, const double* rhs, const double* U,
                              const double* Uhat, double* f, double* h, double* K, double* C, double* D,
                              double* E);

/* Accumulated device time per phase, measured with hipEvents on the context's
 * stream: out[2t] = milliseconds, out[2t+1] = number of timed launches for
 * t = 0 explicit DG residual (trace + residual kernels), 1 element assembly
 * (point-wise Jacobians + block contraction), 2 mixed-block elimination (one
 * batched GEMM launch), 3 K^-1 + condensation, 4 facet right-hand side and
 * preconditioner factorisation, 5 GMRES (including 7), 6 back-substitution and
 * update, 7 facet preconditioner applications, and single kernels inside these:
 * 8 point-wise Jacobians (assembly launches that build a Jacobian), 9 block
 * contraction, 10 Gauss-Jordan K^-1.  Launches inside replayed graphs are not
 * timed.  host out[2 * IMEX_NTIMERS]; reset != 0 clears the counters after reading. */
#define IMEX_NTIMERS 11
imex_status imex_kernel_times(imex_ctx* ctx, double out[2 * IMEX_NTIMERS], int reset);

/* Which of the phases above record their hipEvents: bit t of mask for phase t (all by
 * default, mask = 2^IMEX_NTIMERS - 1).  Each timed launch adds two event records to the
 * stream, a few microseconds of idle device time each, so a run measured by its wall
 * clock keeps only the phases it reads.  The counters of masked phases stay unchanged.
 * IMEX_EINVAL for bits at or above IMEX_NTIMERS. */
imex_status imex_set_timer_mask(imex_ctx* ctx, unsigned mask);

/* Graph mode (on != 0): imex_ark_step replays the explicit sequence of every stage
 * (explicit residual, stage combination and implicit right-hand side) from a
 * hipGraph captured on first use on a private stream and captured again when dt
 * or the tableau changes; the Newton solves, which decide on the host when they
 * have converged, run eagerly between the replays.  on = 0 returns to eager
 * launches.  Results are identical either way.  Errors: EDEVICE. */
imex_status imex_set_graphs(imex_ctx* ctx, int on);

/* Launch-shape autotuner: times the explicit residual kernel for each feasible
 * number of elements per workgroup (at state U, all elements; Uhat needed for
 * HDG-MX coupling, else nullable) and each batched GEMM of the implicit stage for
 * its output tiles (64x64, 32x32, and in FP32 the full-inner-dimension variants
 * 1064, 1032 and the whole-matrix shapes 2001..2010 of imex_set_launch_shapes that
 * apply to the matrix), and keeps the fastest for this context.
 * out (host [4]): elements per residual workgroup (0 = built-in default), then
 * the tiles of the mixed-block elimination, K^-1 [C f] and Schur-update GEMMs
 * (0 = not used).  Call after imex_set_regions and before stepping: it
 * overwrites the implicit-stage workspaces and resets the kernel timers. */
imex_status imex_autotune(imex_ctx* ctx, const double* U, const double* Uhat, int out[4]);

/* Set the launch shapes that imex_autotune picks, e.g. a table kept from an earlier
 * run: in (host [4]) = elements per residual workgroup (0 = default, else one the
 * residual kernel supports for the degree), then the tiles of the elimination,
 * K^-1 [C f] and Schur-update GEMMs: 0 (default), 32, 64 (output tile edge), or
 * 1032, 1064 (the same edges with the whole inner dimension staged in LDS; FP32 and
 * inner dimension <= 128, else the plain edge), or 2001..2006 (FP32, one workgroup
 * per element holding the whole output: up to 192 x 192 with 4 x 4 or 2 x 4 waves,
 * up to 128 x 96 with 2 x 2 or 4 x 2 waves, up to 80 x 96 with 5 x 2 waves, up to
 * 112 x 96 with 1 x 2 waves; else edge 64), or 2007, 2008 (FP32, the output split
 * into parts of 96 x 192 with 2 x 4 waves or 96 x 96 with 2 x 2 waves, one
 * workgroup per part; any size), or 2010, 2009, 2011 (parts of 96 x 192, 96 x 96 and
 * 128 x 96 with each FP32 product formed from three-way bf16 splits of both factors on the
 * bf16 matrix cores, six partial products accumulated in FP32: FP32 accuracy).  Results do
 * not depend on the shapes beyond rounding.  Errors: EINVAL. */
imex_status imex_set_launch_shapes(imex_ctx* ctx, const int in[4]);

/* The element inverse K^-1 of the static condensation (eq. local_solve_static_condensation):
 * *method 0 is the register-tiled Gauss-Jordan with partial pivoting (FP64 and FP32), 1 the
 * blocked Gauss-Jordan with partial pivoting whose rank-16 updates run on the matrix cores
 * (FP32 only: IMEX_FP32_REFINE).  set != 0 selects *method (EINVAL for other values, or for
 * 1 in FP64); on return *method holds the method in use.  imex_autotune times both in FP32
 * and keeps the faster.  host method. */
imex_status imex_element_inverse(imex_ctx* ctx, int set, int* method);

/* Vector-Jacobian product of the explicit residual (reverse mode of Sec. 3.3):
 * Ubar = (dR^DG/dU)^T Rbar, with R^DG as in imex_dg_residual.  U dev (all
 * elements); Rbar dev [e][v][n], rows of implicit elements ignored; Ubar dev out,
 * all elements (implicit elements receive the adjoint of their interface traces).
 * With viscous HDG-MX coupling the implicit side's mixed variables are lifted
 * from (U, Uhat) (Uhat dev, required) and Uhatbar (dev out, facets) receives
 * their adjoint through the lifting; otherwise Uhat, Uhatbar may be NULL.
 * Point-wise flux Jacobians by forward-mode dual numbers, contracted with the
 * transposed basis; deterministic (no atomics).  The first call allocates the
 * transposed-product buffers (kept by the context).  Errors: EINVAL, ENOMEM. */
imex_status imex_vjp_dg_residual(imex_ctx* ctx, const double* U, const double* Uhat, const double* Rbar,
                                 double* Ubar, double* Uhatbar);

/* Reverse mode of one explicit ARK step (Sec. 4.2.2, explicit tableau of tab):
 * given the state U_n (dev, unchanged) and the adjoint Ubar_next of U_{n+1} (dev),
 * writes Ubar = (dU_{n+1}/dU_n)^T Ubar_next (dev out).  The stage states are
 * recomputed from U_n.  Errors: ENOTIMPL with an implicit region. */
imex_status imex_vjp_ark_step(imex_ctx* ctx, const imex_tableau* tab, double dt, const double* U,
                              const double* Ubar_next, double* Ubar);

/* Reverse mode of one IMEX step (Alg. imex_scheme_update) with implicit region:
 * given the state (U dev, Uhat dev; unchanged) at t_n and the adjoints Ubar_next
 * (dev, all elements) and Uhatbar_next (dev, facets; nullable = 0) of the state
 * after the step, writes Ubar = adjoint of U_n (dev out, all elements) and
 * Uhatbar = adjoint of Uhat_n (dev out, facets, nullable; zero except for HDG-MX,
 * whose first explicit residual reads the mixed variables lifted from
 * (U_n, Uhat_n); Uhat_n otherwise only seeds Newton).  The step is recomputed
 * from (U, Uhat) recording the stage values; each implicit stage is reversed
 * with the transposed condensed system at its converged state (K^-T, S^T by
 * GMRES with a facet block-Jacobi preconditioner, tolerance min(gmres_rtol,
 * 1e-12)), the explicit parts with imex_vjp_dg_residual.  Without an implicit
 * region this is imex_vjp_ark_step.  duinf host [4] and pbar host [1] (both
 * nullable): the derivative of <Ubar_next, U_{n+1}> + <Uhatbar_next, Uhat_{n+1}>
 * along a change u_inf + p duinf of the far-field state (App. B.1.1, B.2.1) at p = 0,
 * with U_n, Uhat_n fixed: the sum over the step's residual evaluations of their
 * adjoint times the residual's exact derivative in p (the far-field face integrand of
 * R^DG differentiated by a dual number seeded in u_inf, and A^-(Uhat) du_inf for the
 * far-field facet rows).  st host (nullable): gmres_its of the transposed solves.
 * The first reverse-mode call on a context allocates its adjoint workspaces (the
 * step's stage tape, the facet block-Jacobi factors and the transposed-product
 * buffers); later calls reuse them and allocate nothing.  Errors: ENOMEM (that first
 * allocation), ENOTIMPL for implicit tableaux that are not stiffly accurate, or for
 * duinf without an implicit region; as imex_ark_step. */
imex_status imex_vjp_imex_step(imex_ctx* ctx, const imex_tableau* tab, double dt, const double* U,
                               const double* Uhat, const double* Ubar_next, const double* Uhatbar_next, double* Ubar,
                               double* Uhatbar, const double* duinf, double* pbar, imex_stats* st);

const char* imex_status_str(imex_status s);
const char* imex_last_error(const imex_ctx* ctx);
void imex_destroy(imex_ctx* ctx);

/* ------------------------------------------------------------------------- *
 * Three dimensions: the explicit DG residual on hexahedra (the explicit part of
 * the 3D channel).  The paper's forms are two-dimensional; the 3D residual is
 * eq. bilinear_form_interior_sdg with a third direction and five conservative
 * variables (rho, rho u, rho v, rho w, rho E): convective and viscous fluxes of
 * Sec. 2 (lambda = -2 mu / 3), Vijayasundaram or Lax-Friedrichs faces, the
 * interior-penalty consistency, adjoint and penalty terms, far-field faces as in
 * App. B.1.1.  All elements are explicit; the implicit wall layers are 2D only.
 * ------------------------------------------------------------------------- */
typedef struct imex3d_ctx imex3d_ctx;

/* Cartesian hexahedral mesh: element (i, j, l) at index i + nx (j + ny l) covers
 * [x_i, x_i+1] x [y_j, y_j+1] x [z_l, z_l+1]; bc[] for the sides -x, +x, -y, +y,
 * -z, +z, each IMEX_BC_PERIODIC (paired) or IMEX_BC_FARFIELD; degree 1..3. */
typedef struct {
  int nx, ny, nz;
  const double* xgrid;   /* host, nx+1 strictly increasing */
  const double* ygrid;   /* host, ny+1 */
  const double* zgrid;   /* host, nz+1 */
  int bc[6];
  int degree;
} imex3d_mesh_desc;

/* Create a 3D residual context.  phys: gamma, R, mu, Pr, viscous (its u_inf is not
 * used); dg_flux: IMEX_FLUX_*; alpha_dg: penalty factor (tau = alpha (k+1)^2 / l,
 * l = |T| / |dT|, the smaller l of the two sides on interior faces); u_inf: host,
 * the five-variable far-field state.  Allocates the face-trace records
 * (E x 6 x Q^2 x 10 doubles).  Errors: EINVAL, ENOMEM, EDEVICE. */
imex_status imex3d_create(const imex3d_mesh_desc* mesh, const imex_physics* phys, int dg_flux, double alpha_dg,
                          const double u_inf[5], void* stream, imex3d_ctx** out);

/* out[0..3] = n_elem, nodes per element (k+1)^3, quadrature points per
 * direction, workspace bytes.  host. */
imex_status imex3d_query_sizes(const imex3d_ctx* ctx, long long out[4]);

/* Node coordinates, host out [E][(k+1)^3] each (node a + N b + N^2 c at the
 * Gauss-Legendre points of the element's three axes). */
imex_status imex3d_node_coords(const imex3d_ctx* ctx, double* x, double* y, double* z);

/* R^DG (eq. bilinear_form_interior_sdg in 3D) so that M dU/dt = -R: U and R dev
 * [E][5][(k+1)^3], on the context's stream (asynchronous).  Errors: EINVAL, EDEVICE. */
imex_status imex3d_residual(imex3d_ctx* ctx, const double* U, double* R);

const char* imex3d_last_error(const imex3d_ctx* ctx);
void imex3d_destroy(imex3d_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* IMEXHDG_H */
