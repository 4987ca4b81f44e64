/*
 * osam.h -- C ABI of libosam: the overlapping Schwarz alternating method (O-SAM)
 * coupling linear-elastodynamics subdomains that are hex8 finite-element
 * models (FOM) or Operator-Inference reduced models (OpInf), with OpInf
 * learning, on one AMD Instinct MI355X (gfx950).
 *
 * Method: "Hybrid coupling with operator inference and the overlapping Schwarz
 * alternating method" (arXiv 2511.20687).  Sec. 2 (FE model, Eq.
 * matrix_vector_form_with_dbcs), Sec. 3 (POD, OpInf least squares), Sec. 4.1
 * (multiplicative Schwarz, Alg. 1, Eq. schwarz_discrete, Eq. conv_criterion),
 * Sec. 4.2 (OpInf-FOM / OpInf-OpInf coupling, Eq. opinf_schwarz_inference,
 * Alg. 2, Alg. 3).
 *
 * Conventions shared by every call
 *   - Every call returns an osam_status (0 = OK, negative = error) and never
 *     throws or aborts.  On error, osam_last_error() describes the failure; the
 *     context is left as it was before the call unless stated otherwise.
 *   - The context owns every device buffer it allocates and frees them in
 *     osam_ctx_destroy().  Host pointers passed in are read (or written) only
 *     during the call.  Device pointers passed in (e.g. torch tensors'
 *     data_ptr) are borrowed for the call only, except record buffers, which
 *     are borrowed until replaced or the context is destroyed.
 *   - A context is not thread-safe.  Separate contexts are independent.
 *   - Geometry: every subdomain is a set of node layers [z_lo, z_hi] of a
 *     structured nx x ny x nz hex8 grid of the box [0,Lx]x[0,Ly]x[0,Lz].
 *     Node (i, j, k) of a subdomain has local id i + (nx+1)(j + (ny+1)(k - z_lo)).
 *     A z-face at the bar's end (z_lo == 0 or z_hi == nz) is exterior: clamped
 *     when clamp_ends != 0, traction-free otherwise.  Any other z-face is a
 *     Schwarz (overlap) boundary whose values come from the neighbouring
 *     subdomain that contains it.  Lateral faces (x = 0, Lx or y = 0, Ly) are
 *     traction-free, or hold the displacement components selected by
 *     lateral_fix at zero (the effectively-1D bar of Sec. 5.1 fixes x and y).
 *   - Vector fields on the host are float64 structure-of-arrays [3][n_nodes].
 *   - Free-DOF vectors (snapshots, records) use the library layout
 *     [3][free nodes], free nodes = layers z_lo+1 .. z_hi-1 in node order.
 *     Schwarz-DOF vectors use [3][schwarz nodes], low face first.
 *   - "batch" independent instances share all subdomain descriptions; every
 *     per-instance device array is instance-major.
 */
#ifndef OSAM_H
#define OSAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OSAM_OK = 0,
  OSAM_E_INVALID = -1,   /* bad argument, size or unsupported option */
  OSAM_E_OOM = -2,       /* device allocation failed */
  OSAM_E_HIP = -3,       /* HIP runtime error */
  OSAM_E_NONFINITE = -4, /* a state or norm became NaN/Inf (run stops) */
  OSAM_E_SINGULAR = -5,  /* least-squares system not positive definite */
  OSAM_E_OUTSIDE = -6,   /* a Schwarz node lies in no neighbouring subdomain */
  OSAM_E_ORDER = -7      /* call-order violation (e.g. run before set_initial) */
} osam_status;

/* OSAM_FP32_BF16H: as OSAM_FP32, except that the reduced operator contraction
 * [A | H] [q; q (x) q] of OpInf subdomains takes BF16 operands with FP32
 * accumulation on the matrix cores (Eq. opinf_model_schwarz; the rounding of the
 * operands is the only difference, so results differ from OSAM_FP32 by about
 * 2^-9 relative in that term). */
typedef enum { OSAM_FP64 = 0, OSAM_FP32 = 1, OSAM_FP32_BF16H = 2 } osam_precision;
typedef enum { OSAM_GUESS_HOLD = 0, OSAM_GUESS_PREDICTOR = 1 } osam_guess;
typedef enum { OSAM_LINEAR = 0, OSAM_QUADRATIC = 1, OSAM_CUBIC = 2 } osam_form;
typedef enum { OSAM_LINEAR_ELASTIC = 0, OSAM_SVK = 1 } osam_material;

typedef struct osam_ctx osam_ctx;

/* Library version (major*10000 + minor*100 + patch). */
int32_t osam_version(void);

/* Create a context on HIP device `device` computing in `precision` with `batch`
 * independent instances.  `hip_stream` (hipStream_t) is used for all work; NULL
 * selects the library's own stream.  *out receives the context. */
int32_t osam_ctx_create(osam_ctx **out, int32_t device, int32_t precision, int32_t batch,
                        void *hip_stream);
/* Free every library-owned device buffer and the context itself.  NULL is ignored. */
void osam_ctx_destroy(osam_ctx *ctx);
/* Text of the last error on this context ("" if none); valid until the next call. */
const char *osam_last_error(const osam_ctx *ctx);

/* One subdomain = one mesh + material + BCs + time integrator: the input of
 * Alg. 1 (overlapping subdomains, each with a mesh, initial condition, time
 * integrator and uniform time step).  Linear elasticity (App. A.1), 2x2x2-Gauss
 * hex8 stiffness, row-sum lumped mass, textbook Newmark-beta (Sec. 4.1; the
 * printed Eq. schwarz_discrete is garbled in its scaling): beta = 0 is the
 * explicit central-difference scheme, beta > 0 the implicit one, whose free DOFs
 * solve (M + beta dt^2 K_ff) a+ = -K [u~; u_c] (conjugate gradients on the GPU;
 * an OpInf subdomain solves its reduced equation by Newton's method).  Each
 * subdomain advances a controller step dt in n_sub Newmark steps of dt / n_sub
 * (Sec. 4.1, mixed time steps; its Schwarz data at the intermediate times come
 * from the source's trajectory through the temporal interpolant Xi, linear in
 * time).  All subdomains share dt.  material = OSAM_SVK replaces the linear
 * internal force K u by the Saint Venant-Kirchhoff force f(u) (App. A.2: Green-
 * Lagrange strain, S = lam tr(E) I + 2 mu E, P = F S, total Lagrangian, the same
 * 2x2x2 Gauss rule), a cubic polynomial of the nodal displacements.  Contexts
 * whose subdomains are all linear elastic and explicit with gamma = 1/2 and
 * n_sub = 1 run the single-step path of run; any other context runs the window
 * engine (osam_set_engine). */
typedef struct {
  int32_t nx, ny, nz;          /* global grid, elements per axis (>= 1)     */
  double Lx, Ly, Lz;           /* box size                                  */
  int32_t z_lo, z_hi;          /* node-layer range, 0 <= z_lo, z_lo+2 <= z_hi <= nz */
  double E, nu, rho;           /* Young's modulus, Poisson ratio, density   */
  int32_t clamp_ends;          /* exterior z-faces clamped (chi = 0)        */
  int32_t lateral_fix;         /* components held at zero on lateral faces:
                                  bit 0 = x, bit 1 = y, bit 2 = z (0 = traction-free);
                                  the same value for every subdomain          */
  double dt;                   /* controller step (shared by all subdomains) */
  double beta, gamma;          /* Newmark parameters: 0 <= beta <= 1/2,
                                  1/2 <= gamma <= 1                         */
  int32_t n_sub;               /* Newmark steps per controller step (0 or 1:
                                  one; at most 64)                          */
  int32_t material;            /* OSAM_LINEAR_ELASTIC (App. A.1) or OSAM_SVK:
                                  Saint Venant-Kirchhoff (App. A.2), explicit
                                  scheme only (beta = 0)                    */
} osam_subdomain_desc;

/* Append a FOM subdomain; *sd_id receives its index (0, 1, ...).  The
 * multiplicative Schwarz order is the index order.  Must precede osam_couple. */
int32_t create_subdomain(osam_ctx *ctx, const osam_subdomain_desc *desc, int32_t *sd_id);

/* Build the pointwise projections Pi (Sec. 4.1: trilinear interpolation of the
 * neighbour's FE field at each Schwarz node) for every subdomain.  Called
 * implicitly by the first call that needs it; OSAM_E_OUTSIDE if a Schwarz node
 * lies strictly inside no other subdomain. */
int32_t osam_couple(osam_ctx *ctx);

/* Initial condition of instance `inst` from the global fields u0, v0
 * (host float64 [3][(nx+1)(ny+1)(nz+1)] of subdomain 0's grid): every subdomain
 * restricts them, zeroes its clamped DOFs, keeps the IC on its Schwarz DOFs and
 * forms a0 = M^-1(-K u0) on free DOFs (FOM) or q0 = Phi^T u0, q'0 = Phi^T v0,
 * q''0 = f(q0, g^0) (OpInf, Sec. 4.2).  Resets the instance's step counter. */
int32_t osam_set_initial(osam_ctx *ctx, int32_t inst, const double *u0, const double *v0);

/* Replace the reduced initial state (q0, q'0) of OpInf subdomain sd, instance
 * inst, after osam_set_initial and before the first step (OSAM_E_ORDER otherwise):
 * q''0 = f(q0, g^0) is recomputed with the g^0 of the initial condition, and the
 * FOM neighbours' faces at t_1 with it.  Host float64 [r] each. */
int32_t osam_set_reduced(osam_ctx *ctx, int32_t sd, int32_t inst, const double *q0, const double *qd0);

/* Current accepted state of subdomain sd, instance inst, as host float64
 * [3][n_nodes] arrays (any may be NULL).  OpInf subdomains return the lifted
 * fields Phi q, Phi q', Phi q'' (Sec. 4.2), lifted on the device, on free DOFs and
 * zero on Schwarz and Dirichlet DOFs. */
int32_t osam_get_state(osam_ctx *ctx, int32_t sd, int32_t inst, double *u, double *v, double *a);
/* Set the accepted state of subdomain sd, instance inst, at the instance's current
 * step (restart from stored fields; Alg. 1 advances from the accepted state at
 * t_{k-1}).  FOM: x, xd, xdd = u, v, a as host float64 [3][n_nodes] in the layout
 * osam_get_state returns (the values on Schwarz faces are the data last imposed;
 * held and clamped components must be zero).  OpInf: q, q', q'' host float64 [r]
 * (osam_get_reduced).  Set every subdomain of the instance before the next step.
 * The window engine advances from the accepted state alone, so a state saved with
 * osam_get_state / osam_get_reduced continues bit for bit there.  The single-step
 * path derives the next predictor and the values pushed to neighbours from it before
 * the next step (the acceleration of a FOM subdomain is recomputed as M^-1(-K u),
 * which is what the explicit step produced); the push of an OpInf subdomain into a
 * FOM face is formed on the host in FP64 and may differ from the kernel's in the
 * last bit (osam_save_checkpoint restores such contexts exactly).  The step counter
 * is not changed.  OSAM_E_ORDER before osam_set_initial. */
int32_t osam_set_state(osam_ctx *ctx, int32_t sd, int32_t inst, const double *x, const double *xd,
                       const double *xdd);

/* Raw checkpoint of one instance: every device range that carries state from one
 * controller step to the next (the accepted state in all its buffer roles, the
 * values pushed for the next step, OpInf predictors) and the instance's step
 * counters.  osam_checkpoint_size gives the bytes of one instance (the same for
 * every instance); osam_save_checkpoint copies instance inst into host memory of
 * that size; osam_load_checkpoint restores it into instance inst of this or another
 * context with the same subdomains, precision and engine, after which run continues
 * bit for bit as the saved instance would have.  Records are not part of it.
 * OSAM_E_ORDER before osam_set_initial. */
int32_t osam_checkpoint_size(osam_ctx *ctx, int64_t *bytes);
int32_t osam_save_checkpoint(osam_ctx *ctx, int32_t inst, void *host);
int32_t osam_load_checkpoint(osam_ctx *ctx, int32_t inst, const void *host);

/* Reduced state (q, q', q'') of an OpInf subdomain, host float64 [r] each. */
int32_t osam_get_reduced(osam_ctx *ctx, int32_t sd, int32_t inst, double *q, double *qd,
                         double *qdd);

/* Sizes of subdomain sd: nodes, free DOFs, Schwarz DOFs, reduced dimension
 * (0 for a FOM), boundary reduced dimension.  Any pointer may be NULL. */
int32_t osam_sizes(osam_ctx *ctx, int32_t sd, int64_t *n_nodes, int64_t *n_free, int64_t *n_sch,
                   int32_t *r, int32_t *r_s);

/* Recording (training snapshots, outputs).  Every `every` accepted steps (and at
 * step 0, written by osam_set_initial... or the first run step), column
 * c = step/every of each non-NULL buffer is written; steps beyond n_cols
 * columns are not recorded.  Device buffers in the context precision,
 * layout [batch][n_cols][len]: u and a have len = free DOFs (FOM; for OpInf u
 * holds q, len = r), s has len = Schwarz DOFs.  every = 0 disables. */
typedef struct {
  int64_t every, n_cols;
  void *u, *a, *s;
} osam_record;
int32_t osam_set_record(osam_ctx *ctx, int32_t sd, const osam_record *rec);

/* Operator Inference for subdomain sd (Sec. 3, 4.2; Alg. 2 steps 3-4, Alg. 3).
 * Snapshots of n_traj trajectories, T columns each, device arrays in the
 * context precision, layout [n_traj][T][len]: U free-DOF displacements, Udd the
 * FOM's Newmark accelerations at the same times (the D_t^2 data), S Schwarz-DOF
 * values, V0 [n_traj][n_free] initial velocities (for the Alg. 3 rollout start).
 * POD bases by the method of snapshots (FP64 Gram, symmetric eigensolver) with
 * r (or the energy criterion Eq. pod_energy when r <= 0) and r_s (energy_bnd
 * when r_s <= 0); least squares in FP64 (normal or dual form) for each lambda
 * in `lambdas`; Alg. 3 picks lambda* (frozen-boundary rollout error, smallest
 * lambda on ties, non-finite = +inf) and the operators are refit with it.  On
 * success sd becomes an OpInf subdomain.  The POD computes only the leading
 * eigenpairs of the Gram (block subspace iteration with Rayleigh-Ritz; a full
 * Jacobi eigen-decomposition when that does not converge).  Outputs (host, may
 * be NULL): sigma (singular values of U, min(n_free, n_traj*T) entries: the
 * leading max(r, 16) or more, the entries beyond those computed are 0), E_lambda [n_lambda],
 * lambda_star, r_out, rs_out.  stride: time steps between consecutive snapshots
 * (0 or 1: every step).  The fit is pointwise in time (Udd holds the Newmark
 * accelerations of the snapshot times); the Alg. 3 rollout takes `stride`
 * steps between snapshots with the boundary input interpolated linearly
 * between the two snapshots.  form: OSAM_LINEAR, OSAM_QUADRATIC (q (x) q columns)
 * or OSAM_CUBIC (also the q (x) q (x) q columns of COpInf, the ansatz of the Saint
 * Venant-Kirchhoff model, App. A.2; the cubic operator is read back with
 * osam_get_opinf_cubic). */
typedef struct {
  int32_t form, with_c;
  int32_t r, r_s;
  double energy, energy_bnd;
  int32_t n_lambda;
  const double *lambdas;
  int32_t n_traj;
  int64_t T;
  const void *U, *Udd, *S, *V0;
  double *sigma_out, *E_lambda_out, *lambda_star_out;
  int32_t *r_out, *rs_out;
  int32_t stride;
} osam_opinf_desc;
int32_t learn_opinf(osam_ctx *ctx, int32_t sd, const osam_opinf_desc *desc);

/* Install given OpInf data on subdomain sd (host float64, column-major):
 * Phi [n_free x r], PhiS [n_sch x r_s], A [r x r], H [r x r(r+1)/2] or NULL,
 * B [r x r_s] or NULL, c [r] or NULL.  Columns of Phi and PhiS should be
 * orthonormal (the convergence norm is taken in reduced coordinates). */
int32_t osam_set_opinf(osam_ctx *ctx, int32_t sd, int32_t r, int32_t r_s, const double *Phi,
                       const double *PhiS, const double *A, const double *H, const double *B,
                       const double *c);
/* Read back the OpInf data of subdomain sd into host float64 buffers of the
 * sizes above (any may be NULL). */
int32_t osam_get_opinf(osam_ctx *ctx, int32_t sd, double *Phi, double *PhiS, double *A, double *H,
                       double *B, double *c);
/* Cubic operator of an OpInf subdomain (COpInf, Eq. opinf_rom: the term
 * C (q (x) q (x) q) of the Saint Venant-Kirchhoff ansatz), host float64
 * column-major [r x r(r+1)(r+2)/6] over the compressed cubic power q_a q_b q_c,
 * a <= b <= c in lexicographic order; NULL removes it.  Call after
 * osam_set_opinf (or learn_opinf) and before osam_set_initial (the instances
 * need their initial condition again).  OpInf subdomains with a cubic term run
 * in the window engine.  OSAM_E_ORDER for a FOM subdomain. */
int32_t osam_set_opinf_cubic(osam_ctx *ctx, int32_t sd, const double *C);
/* Read back the cubic operator (zeros when there is none). */
int32_t osam_get_opinf_cubic(osam_ctx *ctx, int32_t sd, double *C);

/* Schwarz options (Eq. conv_criterion): converged when n >= min_iter and
 * sum_i ||du_i + dt_i dv_i||^2 < tol_abs^2 or that sum < tol_rel^2 sum_i
 * ||u_i + dt_i v_i||^2 (free DOFs; reduced coordinates for OpInf).  At most
 * max_iter iterations per controller step; reaching the cap is not an error.
 * guess: initial data of a neighbour not yet advanced in the step.
 * additive: 0 = multiplicative sweeps (Alg. 1: each subdomain takes the newest
 * iterate of its neighbours), 1 = the additive variant of Remark additive_sam
 * (each subdomain takes its neighbours' iterates of the previous iteration, so
 * the first iteration of a step starts every face from `guess`). */
typedef struct {
  double tol_abs, tol_rel;
  int32_t min_iter, max_iter;
  int32_t guess;
  int32_t additive;
} osam_schwarz_opts;

/* Per-instance progress and statistics. */
typedef struct {
  int64_t steps;          /* accepted controller steps since osam_set_initial */
  int32_t last_iters;     /* Schwarz iterations of the last step              */
  int32_t last_converged; /* 1 if the last step met the criterion             */
  double abs2, den2;      /* numerator / denominator of the last test         */
  int64_t total_iters;    /* sum of iterations over all steps                 */
  int32_t max_iters;      /* largest iteration count of any step              */
  int64_t unconverged;    /* steps that hit max_iter                          */
  int32_t status;         /* OSAM_OK or OSAM_E_NONFINITE                      */
} osam_instance_info;

/* One controller step of Alg. 1 for every instance (multiplicative sweeps over
 * the subdomains in index order, or the additive variant, until Eq.
 * conv_criterion).  info: [batch] or NULL.  The sweeps are launched from the host
 * even in graph mode (osam_set_graph), so the call does no more sweeps than the step
 * needs; results equal those of run(ctx, 1, ...). */
int32_t schwarz_step(osam_ctx *ctx, const osam_schwarz_opts *opts, osam_instance_info *info);

/* n_steps controller steps for every instance; the host does not wait on
 * individual steps (each instance iterates at its own pace on the device).
 * Returns OSAM_E_NONFINITE if any instance went non-finite (that instance stops
 * at its last finite step; the others complete).  info: [batch] or NULL. */
int32_t run(osam_ctx *ctx, int64_t n_steps, const osam_schwarz_opts *opts, osam_instance_info *info);

/* run without any device allocation, for callers that cannot allocate device
 * memory (work under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels, results and iteration counts as run, except
 * that the per-workgroup partial sums of Eq. conv_criterion live in a static
 * device array of the library (32 MiB per GPU, held until the process ends)
 * instead of the context's buffers, and graph mode and kernel timing are off for
 * the call.  The context must be wired (osam_set_initial done for every instance)
 * and, for a context the window engine runs (osam_set_engine), that engine set up
 * by a first run call: OSAM_E_ORDER otherwise.  OSAM_E_INVALID when the partial
 * sums need more than 32 MiB (16 bytes x batch x the FOM subdomains' workgroups).
 * Every call on one GPU shares the array, so calls that overlap on the same GPU
 * (other threads, other contexts) race: serialise them. */
int32_t run_noalloc(osam_ctx *ctx, int64_t n_steps, const osam_schwarz_opts *opts, osam_instance_info *info);

/* Trajectory misfit of the coupled rollout and its gradient (discrete adjoint).
 *
 * Not a passage of the paper: a calibration tool around its method.  With the
 * explicit scheme (Sec. 4.1, beta = 0) every accepted step of the multiplicative
 * Schwarz loop (Alg. 1) is the explicit map in which each subdomain advances
 * with the neighbours' displacements at t_k (their Newmark predictors) as
 * Schwarz data (Sec. 4.2: Pi Phi q for an OpInf source, Phi_S^T s for an OpInf
 * destination).  run_adjoint differentiates that map exactly (the iteration
 * counts and the convergence test do not enter it).
 *
 *   J = 1/2 sum_{k = every, 2 every, ... <= n_steps} [ sum_FOM ||u_k - u_obs,k||^2
 *                                                     + sum_OpInf ||q_k - q_obs,k||^2 ]
 *
 * over the free DOFs of FOM subdomains and the reduced coordinates of OpInf
 * subdomains (for an orthonormal Phi, ||Phi q - u||^2 = ||q - Phi^T u||^2 + const).
 * The rollout starts from instance 0's current accepted state (batch must be 1)
 * and leaves the context's state unchanged.  Gradients are taken with respect to
 * the OpInf operators A, H, B, c and the initial state (q0, q'0 of OpInf, u0, v0 on
 * FOM free DOFs); the initial accelerations are functions of these, the Schwarz
 * data at t_0 are constants.  The state is stored every checkpoint_every steps
 * and each segment is recomputed once. */
typedef struct {
  int64_t every;              /* observed steps k = every, 2 every, ... (every >= 1) */
  const void *obs[8];         /* per subdomain id, device, context precision, or NULL:
                                 FOM [n_obs][n_free] (free-DOF layout), OpInf [n_obs][r],
                                 n_obs = n_steps / every */
} osam_misfit;
typedef struct {
  double *dA[8], *dH[8], *dB[8], *dc[8];  /* OpInf subdomains: host float64, layouts of
                                             osam_set_opinf (column-major); NULL = skip */
  double *dq0[8], *dqd0[8];               /* OpInf: host float64 [r] */
  void *du0[8], *dv0[8];                  /* FOM: device [n_free], context precision; 0 on
                                             components held by lateral_fix (not parameters) */
} osam_grads;
/* *J receives the misfit.  OSAM_E_INVALID for batch != 1 or bad sizes. */
int32_t run_adjoint(osam_ctx *ctx, int64_t n_steps, int64_t checkpoint_every, const osam_misfit *misfit,
                    double *J, const osam_grads *grads);

/* Kernel timing: with enable != 0, every Schwarz-step kernel launch of every
 * subdomain records a pair of HIP events stamped with that kernel's own start
 * and end (hipExtLaunchKernel; a little host overhead, off by default).
 * Enabling (again) clears the accumulated times. */
int32_t osam_set_timing(osam_ctx *ctx, int32_t enable);
/* Device time (ms) summed over the timed launches of subdomain sd's step
 * kernel and their number (synchronises the stream). */
int32_t osam_get_timing(osam_ctx *ctx, int32_t sd, double *ms, int64_t *launches);

/* Launch shape of FOM subdomain sd's step kernel: `block` threads per workgroup
 * (64, 128 or 256; 0 = automatic) and `kc` z-layers marched per thread
 * (>= 1; 0 = automatic).  block = 1024 selects the layer-staged variant (FP32
 * contexts, at most 4535 nodes per layer): workgroups of 1024 threads stage
 * whole layers in LDS and take kc layers each, the boundary columns run in a
 * second launch.  Affects speed only, never results (the FP64 convergence sums
 * are added in another order).  OSAM_E_INVALID for other values, an OpInf
 * subdomain, or the layer-staged variant where it does not apply. */
int32_t osam_set_fe_launch(osam_ctx *ctx, int32_t sd, int32_t block, int32_t kc);
/* Interior layout of the FE step kernel of FOM subdomain sd (Sec. 2 explicit
 * step; results are the same bits either way: every interior path adds the
 * stencil in the same x-resolved order).  enable = 1: a wave covers 62
 * consecutive nodes of the rows 1 .. ny-1 (their boundary columns included),
 * loads for each of the 9 (y, z) rows of the 27-point neighbourhood only the
 * value at its own x (a third of the neighbour loads; the default); with one
 * layer per thread each lane forms the x-offset partial sums of its own column
 * and only those 3-vectors cross lanes, otherwise the x-neighbours come from
 * the adjacent lanes; enable = 0: 64 interior columns per wave, every
 * neighbour loaded.  Applies to the column kernel; fused sweeps
 * and the layer-staged variant's interior always use their own layouts.  OSAM_E_INVALID
 * for a bad id or an OpInf subdomain. */
int32_t osam_set_fe_xshare(osam_ctx *ctx, int32_t sd, int32_t enable);

/* Current launch shape of FOM subdomain sd (any pointer may be NULL). */
int32_t osam_get_fe_launch(osam_ctx *ctx, int32_t sd, int32_t *block, int32_t *kc);

/* Evaluation path of OpInf subdomain sd's step in FP32 contexts (Sec. 4.2,
 * Eq. opinf_model_schwarz): 0 automatic (batched for batch >= 8 or
 * r(r+1)/2 >= 1024), 1 fused (one kernel per Schwarz iteration; every
 * workgroup of an instance re-evaluates the reduced right-hand side), 2 batched
 * (f0 = A q + H (q (x) q) + c once per controller step on the matrix cores over
 * tiles of 16 instances, g^ of FOM-fed faces split over the face DOFs).  The
 * explicit predictor q(t_k) is fixed within a step, so both paths compute the
 * same map; they differ by FP32 rounding order only.  OSAM_FP32_BF16H contexts
 * always use the batched path; FP64 contexts always the fused one.  Takes
 * effect for the following steps.  OSAM_E_INVALID for other values. */
int32_t osam_set_rom_path(osam_ctx *ctx, int32_t sd, int32_t path);
/* The path subdomain sd's step uses once wired: 1 fused, 2 batched (0 for a FOM). */
int32_t osam_get_rom_path(osam_ctx *ctx, int32_t sd, int32_t *path);

/* Graph mode of run (rounds > 0, even): run captures `rounds` Schwarz sweeps
 * (Alg. 1) into a HIP graph and replays it, which saves the host's launch work
 * and part of the dispatch latency per kernel.  streams = 1 captures the
 * sweeps as they are launched otherwise.  streams = 2 runs the FOM kernels of
 * a sweep on the context stream and the OpInf kernels on a second stream:
 * every source pushes its next-step displacement into the buffer role of the
 * next step, which no kernel of the sweep reads, so the streams only meet at a
 * finisher kernel, which takes the decision of Eq. conv_criterion; this pays
 * where the kernels are long next to a cross-stream dependency.  Results and
 * iteration counts are those of the sequential launch in both cases (the data
 * each subdomain reads are the same).  A replay may run up to rounds - 1 sweeps
 * past the last step; sweeps of finished instances change nothing.  Ignored
 * while kernel timing is on.  rounds = 0 (the default) launches every sweep
 * from the host.  OSAM_E_INVALID for odd or negative rounds, more than 4096,
 * or streams other than 1 and 2. */
int32_t osam_set_graph(osam_ctx *ctx, int32_t rounds, int32_t streams);

/* Fused sweeps (enable = 1): each Schwarz sweep of Alg. 1 runs as one kernel
 * launch in which every subdomain's step (FOM explicit step, or OpInf step of
 * Eq. opinf_model_schwarz) takes its own range of workgroups.  The decision of
 * Eq. conv_criterion on a sweep's sums is taken by every workgroup of the next
 * sweep (the same fixed-order reduction in each), and a finisher kernel takes it
 * after the last sweep of each chunk of launches; with the batched OpInf parts of
 * osam_set_rom_path 2 (launched before each sweep) the finisher follows every
 * sweep.  Within a sweep no
 * step reads what another writes: sources push the displacement of the next
 * step into buffers the sweep does not read, and an OpInf face fed by another
 * OpInf subdomain forms the source's displacement at t_k (its explicit
 * predictor) from the source's accepted state.  Results and iteration counts
 * equal those of the sequential launches.  FOM steps run the column kernel
 * with 512 threads per workgroup and kc (>= 1; 0 means 1) node layers per
 * thread, whatever osam_set_fe_launch chose (that
 * choice still serves the initial acceleration).  Combines with osam_set_graph (its streams setting is
 * then unused).  At most 4 subdomains, 3 FOM and 2 OpInf: OSAM_E_INVALID here
 * when the context already has more, and from run when a sweep does not fit
 * (also when an OpInf step needs more than 64 KB of LDS).  enable = 0 (the
 * default) returns to one launch per subdomain. */
int32_t osam_set_fusion(osam_ctx *ctx, int32_t enable, int32_t kc);

/* Launch-configuration autotuner.  Times trial runs of trial_steps and
 * 2 trial_steps controller steps (after 2 warm-up steps) from the context's
 * current state with `opts`, takes their difference per step (what every run
 * pays once, such as graph capture, cancels), and keeps, one coordinate at a time, the fastest: the FE launch shape of each
 * FOM subdomain (osam_set_fe_launch: 256/1, 128/1, 64/1, 64/2, 256/8, 64/8 and,
 * where it applies, the layer-staged 1024 with 4, 8, 16 layers; the column
 * kernel shapes with both interior layouts of osam_set_fe_xshare), the OpInf
 * path of each OpInf subdomain of an FP32 context (osam_set_rom_path 1 or 2)
 * the launch mode (osam_set_graph: none, 32 or 128 sweeps on one stream,
 * 32 on two) and sweep fusion (osam_set_fusion with 1, 2 or 4 layers per thread,
 * host launches or graphs of 32 or 128 sweeps).  None of these changes results.  The choice is cached for the
 * process per configuration (precision, batch, subdomain and reduced sizes) and
 * applied without trials on a later call (from_cache = 1).  The trials advance
 * the state: set the initial condition again before the production run.
 * *out (may be NULL) receives the choice per subdomain id and the trial time of
 * the winner.  OSAM_E_ORDER if an instance has no initial condition. */
typedef struct {
  int32_t fe_block[8], fe_kc[8];   /* FOM subdomains (0 for OpInf) */
  int32_t rom_path[8];             /* OpInf subdomains (0 for FOM) */
  int32_t graph_rounds, graph_streams;
  double ms_per_step;              /* wall time per step of the chosen configuration's trial */
  int32_t from_cache;
  int32_t fusion_kc;               /* fused sweeps with this many layers per FE thread, 0: off */
  int32_t fe_xs[8];                /* FOM subdomains: interior layout of osam_set_fe_xshare */
} osam_tuning;
int32_t osam_autotune(osam_ctx *ctx, int64_t trial_steps, const osam_schwarz_opts *opts, osam_tuning *out);

/* Wait for all queued work of the context (host synchronisation). */
int32_t osam_sync(osam_ctx *ctx);

/* Controller engine of run and schwarz_step (Alg. 1).  engine = 0 (default):
 * the single-step path (explicit central difference, one Newmark step per
 * controller step: fused sweeps, graphs, batched OpInf path, autotuner, adjoint)
 * when every subdomain has beta = 0, gamma = 1/2 and n_sub = 1 and no cubic
 * operator, otherwise the window engine.  engine = 1: the window engine for
 * every context.  The window engine runs each Schwarz iteration as every
 * subdomain's whole window of n_sub Newmark steps from the accepted state at
 * t_{k-1} (Sec. 4.1), with the Schwarz data at each sub-step interpolated in time
 * from the source's trajectory of the newest iterate (the temporal interpolant
 * Xi; the initial guess while the source has not run in the step), and the
 * implicit solves of beta > 0; one workgroup per instance and subdomain.  Both
 * engines compute the same iterates for explicit single-step contexts (up to
 * rounding order).  The launch settings (osam_set_fe_launch, osam_set_fusion,
 * osam_set_graph, osam_set_rom_path) do not apply to it; osam_autotune and
 * run_adjoint return OSAM_E_INVALID for contexts it runs.  OSAM_E_INVALID for
 * other values.  engine = 2: the persistent OpInf engine, for contexts whose
 * subdomains are all explicit single-step OpInf models (at most 4, r <= 128,
 * multiplicative Schwarz): one kernel launch runs every controller step of a run
 * call, one workgroup per instance holding every subdomain's reduced state in LDS
 * (the operators too, where they fit; else they are read from global memory); no
 * workgroup waits for another.  Its iterates, sums, iteration counts and records
 * are those of the single-step path with osam_set_rom_path 1, bit for bit.  run
 * returns OSAM_E_INVALID for other contexts. */
int32_t osam_set_engine(osam_ctx *ctx, int32_t engine);

/* Iteration statistics of the window engine's solves for subdomain sd: iters
 * [batch] receives, per instance, the most conjugate-gradient iterations (FOM)
 * or Newton iterations (OpInf) any implicit sub-step took since the engine was
 * set up (0 for explicit subdomains or before the first run). */
int32_t osam_get_solver_stats(osam_ctx *ctx, int32_t sd, int32_t *iters);

#ifdef __cplusplus
}
#endif
#endif /* OSAM_H */
