/*
 * tpf.h -- C ABI of the MI355X (gfx950) two-phase phase-field step library.
 *
 * Method: Mirjalili, Khanwale & Mani, "Assessment of an energy-based surface
 * tension model for simulation of two-phase flows using second-order phase
 * field methods" (arXiv 2205.05835).  One time step advances the phase field
 * phi (Eq. 1 with a regularisation g of Table 1: CDI, SB or ISODI) and the
 * incompressible velocity u with a surface tension force on cell faces
 * (energy-based F = mu grad phi of Eq. 4 with mu of Eq. 2, or CSF, or the
 * localized CSF of Eq. 11), momentum advection and viscous diffusion, and a
 * variable-density pressure projection D(beta G p) = D f*, integrated with
 * classical RK4 on a uniform staggered grid, periodic or (batched calls)
 * closed by free-slip walls per axis (Sec. 3, opening; Secs. 3.1, 3.2).
 *
 * Grid and layout (every array handed across this ABI):
 *   cells (nx, ny, nz), nz = 1 in 2D, equal spacing h = length / nx on all
 *   axes; cell c = (k*ny + j)*nx + i, x fastest (C order [z][y][x]).
 *   phi, p live at cell centres; velocity component u_a[c] lives on the LOWER
 *   a-face of cell c (between c - e_a and c).  Phase 1 is phi = 1.
 *
 * Memory and streams:
 *   The caller owns all device memory.  tpf_workspace_bytes() sizes one
 *   device buffer that the caller allocates and passes to tpf_create(); the
 *   library carves every field, multigrid level and reduction scratch out of
 *   it and never allocates device memory itself (each context holds one
 *   small pinned host buffer, through which the kernels hand the solver's
 *   convergence scalars to the host).  All work is issued on the
 *   hip_stream given at creation (NULL = the legacy default stream).
 *   Host-side arrays passed to set/get functions are read or written before
 *   the call returns and are never retained.  Arrays exchanged across the ABI
 *   are always FP64, whatever the internal precision.
 *
 * Errors: every call returns a tpf_status; nothing throws, nothing aborts.
 * tpf_last_error() returns a thread-local message for the last failure.
 * One context must not be used from two host threads at once.
 */
#ifndef TPF_H
#define TPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TPF_OK = 0,
    TPF_EINVAL = -1,     /* invalid argument or parameter set                   */
    TPF_ENOMEM = -2,     /* workspace smaller than tpf_workspace_bytes()        */
    TPF_EDEVICE = -3,    /* a HIP runtime call failed                           */
    TPF_ENOCONV = -4,    /* pressure solve hit poisson_maxit; state rolled back */
    TPF_ENONFINITE = -5, /* NaN/Inf produced by a step; state rolled back       */
    TPF_ESTATE = -6      /* call not valid in the current context state         */
} tpf_status;

typedef enum { TPF_CDI = 0, TPF_SB = 1, TPF_ISODI = 2 } tpf_model;  /* Table 1 */
typedef enum { TPF_EB = 0, TPF_CSF = 1, TPF_LCSF = 2 } tpf_force;   /* Eq. 4, CSF, Eq. 11 */
typedef enum {
    TPF_FP64 = 0,        /* everything in FP64                                   */
    TPF_FP32_MIXED = 1   /* FP32 state, stencils and smoothers; FP64 pressure,
                            Poisson right-hand side, outer residual (defect
                            correction) and all diagnostics                     */
} tpf_precision;

/* Parameters of one case.  Non-dimensional throughout. */
typedef struct {
    int32_t dim;              /* 2 or 3                                           */
    int32_t n[3];             /* cells per axis (>= 2); n[2] = 1 when dim = 2;
                                 at most 2^29 cells in total                      */
    double length;            /* box edge along x; h = length / n[0]              */
    int32_t model;            /* tpf_model                                        */
    int32_t force;            /* tpf_force                                        */
    int32_t precision;        /* tpf_precision                                    */
    int32_t clamp_properties; /* 1: clamp phi to [0,1] in the density/viscosity laws */
    double sigma;             /* surface tension coefficient (sigma_hat = 6 sigma, Eq. 2) */
    double eps;               /* interface thickness epsilon                      */
    double gamma;             /* regularisation velocity scale gamma (Table 1)    */
    double rho1, rho2;        /* densities of phase phi=1 and phi=0               */
    double visc1, visc2;      /* dynamic viscosities of phase phi=1 and phi=0     */
    double normal_delta;      /* n = g / sqrt(g.g + delta^2); 0 -> 1e-12          */
    double poisson_rtol;      /* stop at ||r|| <= rtol ||rhs||; 0 -> 1e-13 (FP64) or 1e-9 (mixed) */
    double poisson_rtol_inner;/* mixed: smallest relative tolerance asked of an FP32
                                 inner PCG (each inner solve aims at the outer
                                 tolerance, but not below this); 0 -> 1e-6       */
    int32_t poisson_maxit;    /* PCG iteration cap per solve; 0 -> 400            */
    int32_t mg_levels;        /* multigrid levels; 0 -> as deep as the grid allows */
    int32_t adjoint;          /* 1: the workspace also holds the scratch of the
                                 adjoint calls (11 + 8 dim FP64 fields of N
                                 values); 0: those calls return TPF_EINVAL   */
    int32_t walls;            /* bit a (x = bit 0) set: free-slip walls at both
                                 ends of axis a instead of periodicity (the box
                                 of Sec. 3.1, the top and bottom of Sec. 3.2).
                                 A wall is a mirror plane: no flow through it
                                 (u_a on the wall faces a-index 0 is taken as
                                 0 whatever the array holds, and the step
                                 leaves it unchanged), no normal gradient of
                                 phi, p or the tangential velocity, no shear.
                                 Batched calls only; single-case contexts
                                 return TPF_EINVAL for walls != 0            */
} tpf_params;

/* Scalar diagnostics of the current state (FP64; t and step count included). */
typedef struct {
    double t;
    int64_t step;
    double mass;          /* h^d sum phi                                          */
    double mass0;         /* mass when the state was last set                     */
    double phi_min, phi_max;
    double umax;          /* max over cells of |cell-averaged u|                  */
    double ca_inf;        /* umax * visc1 / sigma (Sec. 3.1)                      */
    double ke;            /* 1/2 h^d sum_a sum_c rho_a u_a^2 (face densities)     */
    double se;            /* h^d sum [sigma_hat/eps psi + 1/2 sigma_hat eps |G phi|^2] */
    double dp;            /* mean(p | phi > 0.99) - mean(p | phi < 0.01)          */
    double div_max;       /* max |D u|                                            */
    double poisson_relres;/* relative residual of the last pressure solve         */
    int32_t poisson_outer;/* outer (defect-correction) iterations, last solve     */
    int32_t poisson_inner;/* PCG iterations, last solve (summed over outer)       */
} tpf_diag;

typedef struct tpf_ctx tpf_ctx;

/* Size in bytes of the device workspace for params (validated first). */
tpf_status tpf_workspace_bytes(const tpf_params* params, size_t* bytes);

/* Create a context on the current HIP device.  workspace: device pointer,
 * 256-byte aligned, at least tpf_workspace_bytes(); owned by the caller and
 * not freed by tpf_destroy().  hip_stream: a hipStream_t (may be NULL). */
tpf_status tpf_create(const tpf_params* params, void* workspace, size_t ws_bytes,
                      void* hip_stream, tpf_ctx** out);
tpf_status tpf_destroy(tpf_ctx* ctx);

/* Set the state.  phi: N = nx*ny*nz values; u: dim arrays of N values (u[2]
 * ignored in 2D).  on_device = 1: device pointers read on the context's stream;
 * 0: host pointers, copied before return.  Resets t, step and the pressure
 * warm start, and records mass0. */
tpf_status tpf_set_state(tpf_ctx* ctx, const double* phi, const double* u0,
                         const double* u1, const double* u2, int32_t on_device);

/* phi = [1 + tanh(s / 2 eps)] / 2 (Eq. 2 footnote) for an ellipse/ellipsoid
 * with the given centre and semi-axes (s = first-order signed distance,
 * minimum image in the periodic box); u = 0, p = 0. */
tpf_status tpf_init_droplet(tpf_ctx* ctx, const double center[3], const double semi_axes[3]);

/* Advance nsteps classical RK4 steps of size dt (> 0).  Each step is
 * transactional: on TPF_ENOCONV / TPF_ENONFINITE the state stays at the last
 * completed step. */
tpf_status tpf_step(tpf_ctx* ctx, double dt, int32_t nsteps);

/* Zero-copy access to the state inside the caller's workspace.  The state is
 * the (phi, u) of the problem statement (Sec. 3.1: given phi and u, advance
 * and report) and the projection pressure p.
 *
 * tpf_field_offset: byte offset from the workspace base of field `field`
 * (tpf_state_field below) and its element type (tpf_dtype: TPF_DTYPE_F32
 * for phi and u of a TPF_FP32_MIXED context, TPF_DTYPE_F64 otherwise; p is
 * always TPF_DTYPE_F64).  The array has N = nx*ny*nz elements in the layout
 * above, contiguous.  Offsets are multiples of 256.  The state alternates
 * between two slots of the workspace each RK4 step, and the pressure between
 * two arrays (the projection of a stage writes the next stage's starting
 * guess beside it), so the offsets of phi, u and p hold until the next
 * tpf_step or tpf_step_adjoint (ask again after either; tpf_load_checkpoint
 * and tpf_implicit_phase_step write the current slot in place).  p holds the zero-mean
 * projection pressure of the current state once tpf_get_state (with p),
 * tpf_diagnostics or tpf_eval_field has run since the state last changed;
 * otherwise it holds the last solve's iterate.  Returns TPF_EINVAL for an
 * unknown field or a velocity component beyond dim.
 *
 * tpf_state_changed: after the caller wrote phi and/or u in place (stream
 * ordered before this call), do what tpf_set_state does after its copy:
 * reset t, the step count, the pressure and its warm start, and record mass0.
 * Synchronises the stream. */
typedef enum {
    TPF_STATE_PHI = 0, TPF_STATE_U0 = 1, TPF_STATE_U1 = 2, TPF_STATE_U2 = 3, TPF_STATE_P = 4
} tpf_state_field;
typedef enum { TPF_DTYPE_F64 = 0, TPF_DTYPE_F32 = 1 } tpf_dtype;
tpf_status tpf_field_offset(const tpf_ctx* ctx, int32_t field, size_t* byte_offset, int32_t* dtype);
tpf_status tpf_state_changed(tpf_ctx* ctx);

/* Copy the state out (any pointer may be NULL to skip it).  p is the
 * projection pressure of the current state (computed on demand by one stage
 * evaluation, zero mean). */
tpf_status tpf_get_state(tpf_ctx* ctx, double* phi, double* u0, double* u1, double* u2,
                         double* p, int32_t on_device);

/* Diagnostics of the current state; synchronises the stream.  dp uses the
 * projection pressure of the current state (one stage evaluation). */
tpf_status tpf_diagnostics(tpf_ctx* ctx, tpf_diag* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics of tpf_diagnostics for a state held in the caller's own device
 * arrays, with no context and no workspace.  params describes the grid and
 * properties (validated as for tpf_create).  phi, u0, u1 (u2 in 3D; ignored
 * in 2D) are FP64 device arrays of N = nx*ny*nz values in the layout above;
 * p (FP64, N values, may be NULL: dp is then NaN) is the pressure to measure
 * dp with.  Work is issued on hip_stream (NULL = legacy default stream) and
 * the call synchronises it before filling *out (host memory).  mass0 and
 * poisson_relres are NaN and t, step and the Poisson counters 0: they belong
 * to a context.  The reduction's block partials live in a static device
 * array of the library (5.5 MiB on every device the library runs on, held
 * until the process ends), so the grid may have at most 65536 tiles of
 * 64 x 4 cells, ceil(nx/64) * ceil(ny/4) * nz <= 65536 (256^3 and 4096^2
 * fit); larger grids return TPF_EINVAL.  The call allocates nothing.  Calls
 * that overlap on one device (from two host threads or two streams) share
 * that array and race. */
tpf_status tpf_diagnostics_noalloc(const tpf_params* params, const double* phi, const double* u0,
                                   const double* u1, const double* u2, const double* p, void* hip_stream,
                                   tpf_diag* out);

/* Fields of one stage evaluation at the current state, for verification of
 * each operator.  out: N doubles (host if on_device = 0). */
typedef enum {
    TPF_FIELD_NORMAL0 = 0, TPF_FIELD_NORMAL1, TPF_FIELD_NORMAL2,   /* n_a at cells      */
    TPF_FIELD_MU,                                                  /* mu (Eq. 2)        */
    TPF_FIELD_KAPPA,                                               /* kappa (Eq. 3)     */
    TPF_FIELD_CDIFLUX0, TPF_FIELD_CDIFLUX1, TPF_FIELD_CDIFLUX2,    /* CDI face flux r_a */
    TPF_FIELD_MASSFLUX0, TPF_FIELD_MASSFLUX1, TPF_FIELD_MASSFLUX2, /* m_a              */
    TPF_FIELD_DPHI,                                                /* dphi/dt (Eq. 1)   */
    TPF_FIELD_FORCE0, TPF_FIELD_FORCE1, TPF_FIELD_FORCE2,          /* surface force F_a */
    TPF_FIELD_FSTAR0, TPF_FIELD_FSTAR1, TPF_FIELD_FSTAR2,          /* f*_a              */
    TPF_FIELD_DIVFSTAR,                                            /* D f*              */
    TPF_FIELD_PRESSURE,                                            /* p                 */
    TPF_FIELD_DU0, TPF_FIELD_DU1, TPF_FIELD_DU2,                   /* du_a/dt           */
    TPF_FIELD_COUNT
} tpf_field;
tpf_status tpf_eval_field(tpf_ctx* ctx, int32_t field, double* out, int32_t on_device);

/* Solve D(beta G x) = b - mean(b), mean(x) = 0, with beta from the current
 * phi, by the library's multigrid-preconditioned CG.  b, x: N doubles; x is
 * the initial guess on entry.  iters/relres may be NULL. */
tpf_status tpf_poisson_solve(tpf_ctx* ctx, const double* b, double* x, int32_t on_device,
                             int32_t* iters, double* relres);

/* Pressure-solve counters since creation or the last reset: out[0] solves,
 * out[1] outer (defect-correction) iterations, out[2] PCG iterations,
 * out[3..6] PCG iterations of the last four solves, oldest first (-1: none).
 * reset = 1 zeroes the counters after reading. */
tpf_status tpf_solver_stats(tpf_ctx* ctx, int64_t out[7], int32_t reset);

/* Per-kernel-class device timing: HIP events recorded on the context stream
 * around every launch of the selected classes (the class list is fixed; see
 * tpf_profile_read for names).  enable = bit mask of classes (bit q selects
 * class q; -1 selects all; 0 stops recording); enabling clears the totals.
 * Events are read back when the pool of 8192 pairs fills or on read.
 * tpf_profile_read reports, per class, the name, total device time, launch
 * count and the algorithmic bytes one launch moves (mean over launches). */
tpf_status tpf_profile_enable(tpf_ctx* ctx, int32_t enable);
tpf_status tpf_profile_read(tpf_ctx* ctx, int32_t kernel_class, const char** name,
                            double* total_ms, int64_t* launches, double* bytes_per_launch);
int32_t tpf_profile_classes(void);

/* ------------------------------------------------------------------ checkpoints
 * A checkpoint holds the current state (phi, u), the pressure warm start, t
 * and the step count, in a caller-owned device buffer of
 * tpf_checkpoint_bytes(); loading it into a context of the same grid and
 * precision restores that state. */
tpf_status tpf_checkpoint_bytes(const tpf_ctx* ctx, size_t* bytes);
tpf_status tpf_save_checkpoint(tpf_ctx* ctx, void* dev_dst);
tpf_status tpf_load_checkpoint(tpf_ctx* ctx, const void* dev_src);

/* ------------------------------------------------------------------ adjoint
 * Reverse-mode derivative of the discrete step, written by hand for every
 * stage operator: 2D and 3D, the CDI, SB and ISODI models of Table 1, and the
 * energy-based (Eq. 4), CSF and localized CSF (Eq. 11) forces.  The context
 * must be created with params.adjoint = 1.  Cotangents are FP64 arrays of N
 * values laid out as the state (phi at cells, u_a on the lower a-faces; the
 * u2 arguments are ignored in 2D and may be NULL there); parameter cotangents
 * are those of sigma and eps (holding the state fixed).  The SB term
 * eps |C phi| kappa is differentiated with d|g|/dg = g/|g|, taken as 0 where
 * g = 0.
 *
 * tpf_stage_adjoint: for one stage evaluation F(y) = (dphi/dt, du/dt) at the
 * current state y, given the cotangent (lphi, lu) of F(y), write
 * (gphi, gu) = F'(y)^T (lphi, lu) and ADD dF/d(sigma, eps)^T (lphi, lu) to
 * grad_params[0..1].  The state is not changed.
 *
 * tpf_step_adjoint: for nsteps steps of size dt starting from the current
 * state y_0: runs them forward (the context ends at y_nsteps), recording
 * every stage's input state and pressure on the caller's device buffer
 * `tape` (tpf_adjoint_tape_bytes(nsteps) bytes), then sweeps back.  On entry
 * (gphi, gu) hold dL/dy_nsteps; on return dL/dy_0, and dL/d(sigma, eps) over
 * these steps is ADDED to grad_params.  For long rollouts, checkpoint every K
 * steps and call this once per segment, last segment first (each from its
 * loaded checkpoint).
 * on_device: 1 if the cotangent pointers are device pointers. */
tpf_status tpf_adjoint_tape_bytes(const tpf_ctx* ctx, int32_t nsteps, size_t* bytes);
tpf_status tpf_stage_adjoint(tpf_ctx* ctx, const double* lphi, const double* lu0, const double* lu1,
                             const double* lu2, double* gphi, double* gu0, double* gu1, double* gu2,
                             double grad_params[2], int32_t on_device);
tpf_status tpf_step_adjoint(tpf_ctx* ctx, void* tape, size_t tape_bytes, double dt, int32_t nsteps,
                            double* gphi, double* gu0, double* gu1, double* gu2, int32_t on_device,
                            double grad_params[2]);

/* ------------------------------------------------------------------ implicit ISODI step
 * Backward-Euler step of the phase-field equation (Eq. 1) with the ISODI
 * regularisation of Table 1, the model the paper introduces so that a fully
 * implicit step can be solved by Newton's method (the paragraph after
 * Table 1; the paper gives no implicit scheme, this is the plain backward
 * Euler reading of one).  With the face velocity u of the current state held
 * fixed, one step solves
 *     F(phi) = phi - phi_old - dt R(phi) = 0,
 * R the right-hand side of Eq. 1 with the same discrete operators as the RK4
 * stage, by Newton's method with the Jacobian of F (including the
 * derivative of the regularised normals, taken with |C phi| floored at
 * 1e-10 / h where it is smaller; F itself is exact), each linear system solved by
 * BiCGStab with a diagonal preconditioner to a relative residual that
 * follows Newton's progress (Eisenstat-Walker) or a fixed krylov_rtol, and
 * the Newton step shortened by halving until ||F||_2 decreases (Armijo
 * backtracking, at most 10 halvings).  The context must be FP64 (precision TPF_FP64) with model
 * TPF_ISODI.
 *
 * tpf_implicit_phase_step: advances phi of the context's state by nsteps such
 * steps of size dt >= 0, in place; u, the pressure, t and the step counter
 * are unchanged.  opts may be NULL (all defaults).  A step succeeds when
 * max_c |F| <= newton_tol.  If Newton does not get there within newton_maxit
 * iterations the call returns TPF_ENOCONV, and TPF_ENONFINITE if F becomes
 * NaN/Inf; either way phi is rolled back to its value at the start of the
 * failing step (earlier steps of the call are kept).  info (may be NULL)
 * receives the iteration counts.  For dt >= 2 eps / gamma the pointwise part
 * of F stops being monotone and the root reached from phi_old need not be
 * unique.  Uses the stage scratch of
 * the context: no other call on the same context may run concurrently. */
typedef struct {
    double newton_tol;     /* stop at max |F| <= newton_tol (units of phi); 0 -> 1e-12      */
    double krylov_rtol;    /* relative residual of each linear solve, in [0, 1); 0 -> adaptive */
    int32_t newton_maxit;  /* Newton iterations per step; 0 -> 30                           */
    int32_t krylov_maxit;  /* BiCGStab iterations per Newton iteration; 0 -> 400            */
} tpf_implicit_opts;

typedef struct {
    int32_t newton_iters;  /* Newton iterations of the last step                            */
    int32_t krylov_iters;  /* BiCGStab iterations of the last step (summed over Newton)     */
    double residual;       /* max |F| when the last step stopped                            */
    int64_t newton_total;  /* over all steps of the call                                    */
    int64_t krylov_total;
} tpf_implicit_info;

tpf_status tpf_implicit_phase_step(tpf_ctx* ctx, double dt, int32_t nsteps, const tpf_implicit_opts* opts,
                                   tpf_implicit_info* info);

/* ------------------------------------------------------------------ batches
 * Batched persistent form: many independent 2D cases (each its own grid,
 * properties, model, force and time step; one precision for the whole batch)
 * advance together, one GPU launch per RK4 step in which one workgroup owns
 * one case for the whole step, including its pressure solve.  Cases do not
 * wait for each other: each converges, fails or finishes on its own.  Steps
 * are replayed from a captured HIP graph (8 launches per replay).
 *
 * Workspace: tpf_batch_workspace_bytes() sizes one device buffer (caller
 * owned, 256-byte aligned) that holds every case's fields.  Case q is
 * cases[q] of the array given at creation; cases run longest first.
 */
typedef struct tpf_batch tpf_batch;

tpf_status tpf_batch_workspace_bytes(const tpf_params* cases, int32_t ncases, size_t* bytes);
tpf_status tpf_batch_create(const tpf_params* cases, int32_t ncases, void* workspace, size_t ws_bytes,
                            void* hip_stream, tpf_batch** out);
tpf_status tpf_batch_destroy(tpf_batch* b);

/* State of case q (FP64 arrays of nx*ny values; host pointers when
 * on_device = 0).  Resets the case's time, step count, status and pressure
 * warm start. */
tpf_status tpf_batch_set_state(tpf_batch* b, int32_t q, const double* phi, const double* u0,
                               const double* u1, int32_t on_device);
/* phi of a tanh ellipse (as tpf_init_droplet) for case q, u = 0. */
tpf_status tpf_batch_init_droplet(tpf_batch* b, int32_t q, const double center[2],
                                  const double semi_axes[2]);
/* phi, u of case q and its last projection pressure (any may be NULL). */
tpf_status tpf_batch_get_state(tpf_batch* b, int32_t q, double* phi, double* u0, double* u1,
                               double* p, int32_t on_device);

/* nsteps RK4 steps of every live case with its own dt (host array of ncases
 * values, each > 0).  A case whose step fails (pressure solve not converged,
 * or a non-finite value) keeps its last completed state and stops; the call
 * then returns that failure after all steps, and tpf_batch_status() names the
 * cases.  The other cases are not affected. */
tpf_status tpf_batch_step(tpf_batch* b, const double* dt, int32_t nsteps);
/* Per case (arrays of ncases, any may be NULL): status (TPF_OK or the
 * failure that stopped it), completed steps and time. */
tpf_status tpf_batch_status(tpf_batch* b, int32_t* status, int64_t* steps, double* t);
/* Let a stopped case run again (after its state or parameters were fixed). */
tpf_status tpf_batch_clear_status(tpf_batch* b, int32_t q);
/* Diagnostics of every case (out: ncases entries), as tpf_diagnostics. */
tpf_status tpf_batch_diagnostics(tpf_batch* b, tpf_diag* out);

/* Launch shapes: configuration c has `threads` threads per case-workgroup and
 * keeps the coarsest multigrid levels of each case in up to `lds_bytes` of
 * LDS (some configurations reserve their whole LDS budget so that a large
 * case gets a CU to itself).  tpf_batch_tune() times every configuration on
 * uncommitted RK4 steps of every live case with the time steps dt (the state,
 * the pressures and their history and the statuses are left as they were;
 * the pressures pass through host memory meanwhile), keeps the fastest, and records it
 * in the text file cache_path (may be NULL) under a key made of a hash of the
 * library's sources, the precision and the grid sizes; a later call with the
 * same key reads the choice back instead.  If a case's pressure solve fails
 * during the timing, the fastest configuration is still set and the call
 * returns TPF_ENOCONV naming the case (which keeps running). */
int32_t tpf_batch_configs(void);
tpf_status tpf_batch_config_info(int32_t config, int32_t* threads, int32_t* lds_bytes);
tpf_status tpf_batch_set_config(tpf_batch* b, int32_t config);
tpf_status tpf_batch_tune(tpf_batch* b, const double* dt, const char* cache_path, int32_t* chosen);

/* Pressure-solve counters of every case since creation or the last reset
 * (arrays of ncases values, any may be NULL): solves, outer
 * (defect-correction) iterations and PCG iterations, summed over the solves.
 * reset = 1 zeroes them after reading. */
tpf_status tpf_batch_solver_stats(tpf_batch* b, int64_t* solves, int64_t* outer, int64_t* inner, int32_t reset);

const char* tpf_last_error(void);
const char* tpf_version(void);

#ifdef __cplusplus
}
#endif
#endif
