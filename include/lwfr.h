/*
 * lwfr.h - C ABI of the MI355X (gfx950) time step of the single-stage,
 * time-averaged flux reconstruction scheme for hyperbolic systems with
 * non-conservative products (Babbar & Ranocha, "Compact Runge-Kutta flux
 * reconstruction methods for non-conservative hyperbolic equations").
 *
 * Problem (paper §3 eq. flux.and.non.cons, 2-D form in §5 above eq.
 * time.step.2d):   u_t + sum_d [ f_d(u)_{x_d} + B_d(u) u_{x_d} ] = 0
 * on a uniform Cartesian mesh of tensor-product elements with the N+1
 * Gauss-Legendre solution points per direction (§2 eq. soln.points),
 * periodic or with the side kinds of lwfr_config.bc.
 *
 * Conventions shared by every call
 *  - All floating point data are IEEE FP64.
 *  - State layout u[var][elem][node]: elements x-fastest (e = ex + nx*ey),
 *    nodes x-fastest inside an element (p = i + (N+1)*j).  Variables:
 *      SW1D    (h, h v, b)                SW2D (h, h v1, h v2, b)
 *      GLMMHD2D (rho, rho v1, rho v2, rho v3, E, B1, B2, B3, psi)
 *      LINADV1D (u)                       VARADV1D (v, a)
 *  - Pointers named d_* are device pointers on the device current when
 *    lwfr_bind was called; the caller owns and allocates every buffer
 *    (state, outputs, workspace).  The library never allocates device memory.
 *  - Calls that take device pointers only enqueue work on the bound stream and
 *    return at once; their status covers argument checks and launch errors.
 *    Numerical trouble inside a step is reported per element through d_flags
 *    and accumulated in the context; lwfr_query reads it back.
 *  - Functions return lwfr_status; lwfr_last_error() gives a thread-local
 *    message for the last failing call.
 */
#ifndef LWFR_H
#define LWFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LWFR_ABI_VERSION 3u

typedef struct lwfr_ctx lwfr_ctx;

typedef enum {
  LWFR_OK = 0,
  LWFR_E_INVALID_ARG = 1,   /* bad pointer, size, aliasing or configuration value */
  LWFR_E_UNSUPPORTED = 2,   /* valid request the library does not implement */
  LWFR_E_HIP = 3,           /* a HIP runtime call failed */
  LWFR_E_INADMISSIBLE = 4,  /* lwfr_query: a lower order update was not admissible */
  LWFR_E_NONFINITE = 5,     /* lwfr_query: a step produced a non-finite value */
  LWFR_E_WORKSPACE = 6,     /* workspace missing, too small or misaligned */
  LWFR_E_STATE = 7          /* call out of order (e.g. step before bind) */
} lwfr_status;

typedef enum {
  LWFR_EQ_SW1D = 1,      /* shallow water, bed b carried as a variable, B u_x = (0, g h b_x, 0) */
  LWFR_EQ_SW2D = 2,
  LWFR_EQ_GLMMHD2D = 3,  /* ideal GLM-MHD with Godunov-Powell and GLM terms (§5.5 eq. glm.mhd) */
  LWFR_EQ_LINADV1D = 4,  /* u_t + u_x = 0 (test system) */
  LWFR_EQ_VARADV1D = 5,  /* v_t + a v_x = 0 as a non-conservative system (§5.1 eq. var.coeff.adv.non.cons) */
  LWFR_EQ_JINXIN1D = 6   /* Jin-Xin relaxation (§5.1 eqs. jinxin1, jinxin2): u = (u, v), flux (v, a^2 u),
                            stiff source (0, -(v - f(u))/eps), f(u) = l u + q u^2/2; needs an IMEX flag */
} lwfr_equation;

typedef enum {
  LWFR_BLEND_OFF = 0,        /* pure high order step (alpha_e = 0, no limiting) */
  LWFR_BLEND_INDICATOR = 1,  /* subcell blend with the smoothness indicator (§4 eq. blended.scheme) */
  LWFR_BLEND_ADMISSIBLE = 2  /* blend + Algorithm 1 (face fluxes) + Algorithm 2 (element blend) */
} lwfr_blending;

/* Kinds of the sides of the domain (lwfr_config.bc).  The paper leaves the
 * boundary conditions to the problem (§2 after eq. con.law.source) and its
 * tests use periodic sides, reflective walls, inflow and outflow boundaries
 * (§5.2, shock diffraction).  A non-periodic side takes a ghost state at each
 * boundary face point and the face flux of the interior faces from it; the
 * face blends with the inside element's alpha_e, Algorithm 1 keeps only the
 * inside subcell admissible, and the smoothing of alpha_e skips the missing
 * neighbour. */
typedef enum {
  LWFR_BC_PERIODIC = 0,   /* both sides of the direction; the default */
  LWFR_BC_OUTFLOW = 1,    /* ghost = the inside face data */
  LWFR_BC_WALL = 2,       /* mirror image: normal momentum reversed (shallow water only) */
  LWFR_BC_DIRICHLET = 3   /* ghost face data given by lwfr_set_boundary_data */
} lwfr_boundary;

/* Per-element flag bits written to d_flags. */
#define LWFR_FLAG_ALG2 1u          /* Algorithm 2 limited the element */
#define LWFR_FLAG_LOW_INADM 2u     /* the lower order update is not admissible in the element */
#define LWFR_FLAG_ALG1 4u          /* Algorithm 1 limited a flux on one of the element's faces */
#define LWFR_FLAG_NONFINITE 8u     /* the new state holds a non-finite value */
#define LWFR_FLAG_ALG1_GUARD 16u   /* Algorithm 1 met an inadmissible lower order candidate */

typedef struct {
  uint32_t abi_version;  /* LWFR_ABI_VERSION */
  int32_t equation;      /* lwfr_equation */
  int32_t degree;        /* N, 1..4 */
  int32_t nelem[2];      /* elements per direction; nelem[1] ignored in 1-D; at most
                            2^26 elements in all (element, node and face-point indices
                            stay in 32 bits), else LWFR_E_INVALID_ARG */
  double lo[2], hi[2];   /* domain box */
  double gamma;          /* GLM-MHD ratio of specific heats (5/3) */
  double gravity;        /* shallow water g (9.81) */
  double cfl_safety;     /* C_s of eq. time.step.2d (the paper's default 0.9) */
  double cfl_number;     /* CFL(N) of eq. time.step.2d; <= 0: the library's own Fourier value */
  int32_t blending;      /* lwfr_blending */
  double alpha_max;      /* cap of the blending coefficient (0.5) */
  double alpha_min;      /* indicator clip threshold (1e-3) */
  double alpha_force;    /* >= 0: every alpha_e is this value; < 0: smoothness indicator */
  uint32_t flags;        /* LWFR_CFG_* bits */
  int32_t bc[4];         /* lwfr_boundary of the sides x lo, x hi, y lo, y hi (y ignored in
                            1-D); a direction is periodic on both sides or on neither */
  double source[4];      /* LWFR_EQ_JINXIN1D: a > 0, eps > 0, l, q (the paper's Burgers case:
                            3, eps, 0, 1); ignored by the other systems */
} lwfr_config;

/* lwfr_config.flags: reserve the workspace of lwfr_adjoint_step */
#define LWFR_CFG_ADJOINT 1u
/* lwfr_config.flags: Gauss-Lobatto-Legendre solution points with the g_2
 * correction functions (App. B, the variant after eq. fr.form.non.cons: GLL
 * points on [0,1], g_R'(xi_p) = delta_pN/w_p, g_L'(xi_p) = -delta_p0/w_p) in
 * place of Gauss-Legendre points with the Radau correction.  Subcell widths
 * are the GLL weights; cfl_number = 0 takes the Fourier limit of this scheme. */
#define LWFR_CFG_GLL 2u
/* lwfr_config.flags: the IMEX pair of App. C that a system with a stiff source
 * (LWFR_EQ_JINXIN1D, which needs one of them) takes in its inner stages (§2
 * eq. crkfr.inner: explicit part on the local flux terms, pointwise implicit
 * solves for the source), with the averaged source of eq. avg.source in the
 * update and the source taken implicitly in the subcell update (eq.
 * low.order.update).  HT(1,1,2): second order (eq. ht112.butcher);
 * SSP3-IMEX(4,3,3): third order, L-stable (eq. ssp33.butcher, with the
 * implicit rows (alpha), (-alpha, alpha), (0, 1-alpha, alpha),
 * (beta, eta, 1/2-beta-eta-alpha, alpha), whose sums are the nodes).
 * cfl_number = 0 takes the Fourier limit of the pair's explicit part. */
#define LWFR_CFG_IMEX_HT112 4u
#define LWFR_CFG_IMEX_SSP3 8u
/* lwfr_config.flags: element-local time averages by the approximate Lax-Wendroff
 * procedure instead of the cRK inner stages: F_d, U and B^loc as Taylor series
 * in time up to dt^N, the time derivatives of f_d and of B(u) u_x by central
 * differences (3 points for N <= 2, 5 for N >= 3) along Taylor-extrapolated
 * states, d_t^{k+1} u from the local operator.  The paper's cRK stages are
 * linearly equivalent to this Lax-Wendroff form (§5); the stencils are this
 * library's.  Not with an IMEX pair, LWFR_CFG_ADJOINT or in batches
 * (LWFR_E_UNSUPPORTED). */
#define LWFR_CFG_ALW 16u

/* Statistics of one step (filled on the device by lwfr_step when d_stats is
 * not NULL; the caller owns the device buffer of sizeof(lwfr_stats) bytes,
 * 8-byte aligned).  The paper's diagnostics are the time step (§5 eq.
 * time.step.2d), conservation of the variables whose non-conservative row is
 * zero (§4 after eq. numflux.args), the blending coefficients (§4 eq.
 * blended.scheme) and the positivity of the constraints of the admissible set
 * (§2 eq. uad.form, §4.1).  Reductions run in a fixed order: the same step
 * gives the same bits. */
typedef struct lwfr_stats {
  double dt;                  /* the step's time step */
  double ch;                  /* its GLM cleaning speed (0 without GLM) */
  double mass[9];             /* sum_e sum_p w_p |Omega_e| u^{n+1}_{v,e,p} per variable v (first M used) */
  double min_constraint[2];   /* min over nodes of P_k(u^{n+1}) (first K used: depth; density, pressure) */
  uint32_t alpha_hist[11];    /* elements by alpha_e: [0] alpha = 0, [k] alpha in ((k-1)/10, k/10] */
  uint32_t n_alg1;            /* elements with LWFR_FLAG_ALG1 */
  uint32_t n_alg2;            /* elements with LWFR_FLAG_ALG2 */
  uint32_t n_low_inadm;       /* elements with LWFR_FLAG_LOW_INADM */
  uint32_t n_nonfinite;       /* elements with LWFR_FLAG_NONFINITE */
  uint32_t n_alg1_guard;      /* elements with LWFR_FLAG_ALG1_GUARD */
  uint32_t reserved;
} lwfr_stats;

/* Validates cfg and builds the reference element, tableau and launch shapes on
 * the host.  No device work.  *out receives a context owned by the caller
 * until lwfr_destroy.  Errors: LWFR_E_INVALID_ARG (bad value, null pointer,
 * ABI mismatch, a direction periodic on one side only, a wall for a system
 * other than shallow water), LWFR_E_UNSUPPORTED (degree outside 1..4;
 * LWFR_CFG_ADJOINT with a non-periodic side). */
lwfr_status lwfr_init(const lwfr_config* cfg, lwfr_ctx** out);

/* Device workspace bytes the context needs (traces, face fluxes, indicator,
 * reductions).  256-byte alignment is required for the workspace pointer. */
lwfr_status lwfr_workspace_bytes(const lwfr_ctx* ctx, size_t* bytes);

/* Number of doubles of one state u (M * E * (N+1)^d). */
lwfr_status lwfr_state_size(const lwfr_ctx* ctx, size_t* ndouble);

/* Reference solution points xi_p on [0,1] and weights w_p (host arrays of N+1). */
lwfr_status lwfr_reference_nodes(const lwfr_ctx* ctx, double* xi, double* w);

/* The library's Fourier (von Neumann) CFL(N) of the linearised scheme. */
lwfr_status lwfr_cfl_number(int32_t degree, double* cfl);
/* As lwfr_cfl_number for the scheme that lwfr_config.flags cfg_flags select
 * (LWFR_CFG_GLL, LWFR_CFG_IMEX_*; LWFR_CFG_ALW has the limit of the cRK stages:
 * both are the Lax-Wendroff scheme for linear problems). */
lwfr_status lwfr_cfl_number_for(int32_t degree, uint32_t cfg_flags, double* cfl);

/* Doubles of the Dirichlet data of the context: for each side b = 2 d + s
 * (x lo, x hi[, y lo, y hi]; every side has its block, used or not) a block
 * [quantity 3][variable M][position along the side], quantity 0 = u^n at the
 * boundary face point (also the outside subcell state of the lower order
 * flux), 1 = U (the time average of the solution over the step), 2 = F_d (the
 * time-averaged flux normal to the side); positions: line index (the other
 * direction's element index) * nfp + q, nfp = N+1 in 2-D, 1 in 1-D. */
lwfr_status lwfr_boundary_data_size(const lwfr_ctx* ctx, size_t* ndouble);

/* Device pointer to the Dirichlet data (lwfr_boundary_data_size doubles) read
 * by every following step until replaced; the caller keeps it valid and
 * fills it for each step before enqueuing it (U and F_d depend on dt, so steps
 * of a context with a Dirichlet side need dt > 0).  Errors:
 * LWFR_E_INVALID_ARG (null), LWFR_E_STATE (the context has no Dirichlet side). */
lwfr_status lwfr_set_boundary_data(lwfr_ctx* ctx, const double* d_ghost);

/* Attaches caller-owned device workspace and a HIP stream (hipStream_t passed as
 * void*; NULL = default stream).  The workspace must stay valid until the next
 * bind or lwfr_destroy.  Errors: LWFR_E_WORKSPACE. */
lwfr_status lwfr_bind(lwfr_ctx* ctx, void* d_workspace, size_t bytes, void* stream);

/* One time step u^n -> u^{n+1} (paper §3 eq. crkfr.non.cons.final with the
 * blend of §4 and Algorithms 1-2).
 *   d_u_in   state u^n (read only)
 *   d_u_out  state u^{n+1}; must not alias d_u_in (LWFR_E_INVALID_ARG)
 *   dt       > 0: time step used as given; <= 0: eq. time.step.2d on the device
 *   d_dt_ch  nullable; receives {dt, c_h} (c_h = GLM cleaning speed, 0 otherwise)
 *   d_alpha  nullable; receives the blending coefficient alpha_e of each element
 *   d_flags  nullable; receives LWFR_FLAG_* bits of each element
 *   d_stats  nullable; receives the step's lwfr_stats (two extra launches)
 * Asynchronous on the bound stream; LWFR_E_STATE if not bound, or if the
 * context has a Dirichlet side without data; LWFR_E_INVALID_ARG for dt <= 0
 * with a Dirichlet side, or a d_stats not 8-byte aligned. */
lwfr_status lwfr_step(lwfr_ctx* ctx, const double* d_u_in, double* d_u_out, double dt, double* d_dt_ch,
                      double* d_alpha, uint32_t* d_flags, lwfr_stats* d_stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): one step as
 * lwfr_step with d_alpha and d_stats NULL, whose workspace is a static device
 * array of the library, LWFR_STATIC_SCRATCH_BYTES on each GPU it runs on (held
 * until the process ends), instead of the bound workspace.  The context needs
 * no lwfr_bind; the work is enqueued on hip_stream (hipStream_t as void*, NULL
 * = the default stream) on the current device, whose array address is resolved
 * by the first call on that device (make that first call outside a graph
 * capture).  The call allocates nothing.  Every array the step reads from the
 * scratch is written earlier in the same call, so nothing has to start at zero.
 * All calls on one GPU share its array: calls that overlap in time on one GPU
 * (concurrent streams or threads) race and give wrong results; calls in one
 * stream order are safe.  Errors: LWFR_E_WORKSPACE when the step needs more
 * than LWFR_STATIC_SCRATCH_BYTES (GLM-MHD at N = 3: up to about 300,000
 * solution points, e.g. 137 x 137 elements), and those of lwfr_step. */
#define LWFR_STATIC_SCRATCH_BYTES (64u << 20)
lwfr_status lwfr_step_noalloc(lwfr_ctx* ctx, const double* d_u_in, double* d_u_out, double dt, double* d_dt_ch,
                              uint32_t* d_flags, void* hip_stream);

/* One time step with both dt > 0 and the GLM cleaning speed ch >= 0 given
 * (ignored by systems without GLM), e.g. to replay a step sequence with the
 * values of an earlier run.  Otherwise as lwfr_step. */
lwfr_status lwfr_step_fixed(lwfr_ctx* ctx, const double* d_u_in, double* d_u_out, double dt, double ch,
                            double* d_alpha, uint32_t* d_flags);

/* Residual R = (u^n - u^{n+1})/dt of one step with the given dt > 0: the
 * right-hand side of the final update of §3 eq. crkfr.non.cons.final (the
 * divergence of the time-averaged flux, the averaged non-conservative term and
 * the correction-function terms), blended with the subcell residual of §4
 * eq. low.order.update as the mode says.
 * mode 0: high order only (alpha = 0, no limiting); 1: lower order subcell
 * scheme only (alpha = 1, no limiting); 2: as configured.  d_R must not alias d_u. */
lwfr_status lwfr_residual(lwfr_ctx* ctx, const double* d_u, double dt, int32_t mode, double* d_R);

/* Bytes of one step's tape: the values a forward step hands to the adjoint
 * (dt and c_h, alpha_e, the thetas of Algorithms 1 and 2, the face traces of
 * the time-averaged solution U).  256-byte alignment required. */
lwfr_status lwfr_tape_bytes(const lwfr_ctx* ctx, size_t* bytes);

/* A forward step like lwfr_step (dt > 0 given, <= 0 from eq. time.step.2d)
 * that writes its tape to d_tape (caller-owned device memory of
 * lwfr_tape_bytes), for a later lwfr_adjoint_step of the same step. */
lwfr_status lwfr_step_taped(lwfr_ctx* ctx, const double* d_u_in, double* d_u_out, double dt, double* d_dt_ch,
                            void* d_tape);

/* Adjoint of one step (reverse mode, hand-written): d_lam_n = (d u^{n+1}/d u^n)^T
 * d_lam_np1 for the step from d_u_n with the time step dt > 0 (the one the
 * forward step used), holding c_h, every alpha_e, the thetas of Algorithms 1
 * and 2 and every max/abs branch at their values in that forward step
 * (frozen switches).  d_tape: the tape lwfr_step_taped wrote for this very
 * step, or NULL, in which case the call re-runs the forward step internally
 * first.  All arrays have the state layout; d_lam_n must not alias d_u_n or
 * d_lam_np1.  Needs a context created with LWFR_CFG_ADJOINT (else LWFR_E_STATE). */
lwfr_status lwfr_adjoint_step(lwfr_ctx* ctx, const double* d_u_n, double dt, const double* d_lam_np1,
                              double* d_lam_n, const void* d_tape);

/* Synchronises the bound stream and returns the OR of the flags of every
 * element of every step since the previous query (then clears it; all
 * LWFR_FLAG_* bits, so limiter activity shows too): LWFR_E_NONFINITE if a non-finite
 * value appeared, LWFR_E_INADMISSIBLE if a lower order update was inadmissible,
 * LWFR_OK otherwise.  flags_or (nullable) receives the raw OR. */
lwfr_status lwfr_query(lwfr_ctx* ctx, uint32_t* flags_or);

/* Per-kernel timing with HIP events recorded on the bound stream around every
 * launch of the following calls, for at most max_launches launches (the rest
 * are not timed).  lwfr_timing_end synchronises the stream and fills, for each
 * kernel id (0 per-element means/indicator, 1 time step, 2 GLM speed candidates,
 * 3 GLM speed, 4 element stages, 5 faces, 6 update, 7 residual, 8 update adjoint,
 * 9 face adjoint, 10 stage adjoint; batches: 11 means/indicator, 12 time steps,
 * 13 element stages, 14 faces, 15 update; 16 boundary faces of non-periodic
 * sides, single problems and batches), the summed milliseconds ms[k] and the
 * number of timed launches launches[k]; both arrays hold LWFR_TIMING_KERNELS
 * entries.  Events are created on the host by the library and released by
 * lwfr_destroy.  Launches inside a graph capture are not timed. */
#define LWFR_TIMING_KERNELS 17
lwfr_status lwfr_timing_begin(lwfr_ctx* ctx, int32_t max_launches);
lwfr_status lwfr_timing_end(lwfr_ctx* ctx, double* ms, uint32_t* launches);

/* Captures nsteps consecutive steps (dt from eq. time.step.2d on the device each
 * step, as lwfr_step with dt <= 0) into a HIP graph owned by the context,
 * replacing any earlier one: step k reads d_u_a and writes d_u_b for even k,
 * the reverse for odd k, so the result is in d_u_a for even nsteps.
 * d_dt_ch_hist (nullable, device, nsteps x 2) receives each step's (dt, c_h).
 * Inside the sequence each step's update kernel also forms the next step's
 * element means, wave speeds and raw indicator, so that kernel of its own runs
 * for the first step only; the results equal nsteps lwfr_step calls bit for bit.
 * The graph holds kernel launches only (no memory set or copy nodes).  Needs a
 * bound non-default stream (else LWFR_E_STATE).  Nothing runs until
 * lwfr_graph_launch, which enqueues the whole sequence on the bound stream;
 * the pointers are baked into the graph and must stay valid.
 * LWFR_E_UNSUPPORTED for a context with a Dirichlet side (dt is not known
 * when the graph is built). */
lwfr_status lwfr_graph_capture(lwfr_ctx* ctx, double* d_u_a, double* d_u_b, int32_t nsteps, double* d_dt_ch_hist);
lwfr_status lwfr_graph_launch(lwfr_ctx* ctx);

lwfr_status lwfr_destroy(lwfr_ctx* ctx);

/* ---- Batches -------------------------------------------------------------
 * Many independent problems of one equation system (currently the 2-D shallow
 * water system), of any mix of sizes and degrees 1..4, advanced together with
 * one launch per phase of the step (means and indicator, per-problem time
 * steps, element stages, faces, update).  Each problem takes its own time step
 * from eq. time.step.2d.  The batch state is the concatenation of the
 * problems' states, problem i starting at offsets[i] doubles
 * (lwfr_batch_state_offsets fills count+1 entries; offsets[count] is the
 * total), each in the layout of lwfr_state_size.  Results equal those of
 * lwfr_step on each problem alone. */
typedef struct lwfr_batch lwfr_batch;

/* Phases whose launch shape can be set (lwfr_batch_set_launch) */
enum {
  LWFR_PHASE_PRE = 0,    /* element means, indicator (and the per-problem time steps) */
  LWFR_PHASE_STAGES = 1, /* element-local stages */
  LWFR_PHASE_FACES = 2,  /* interface fluxes and Algorithm 1 */
  LWFR_PHASE_UPDATE = 3  /* update, subcell FV, blend, Algorithm 2 */
};

/* cfgs[0..count) as for lwfr_init (same equation for all, no
 * LWFR_CFG_ADJOINT).  Errors: those of lwfr_init (message names the problem),
 * LWFR_E_UNSUPPORTED for another equation system or a Dirichlet side (the
 * per-problem time steps are computed on the device). */
lwfr_status lwfr_batch_init(const lwfr_config* cfgs, int32_t count, lwfr_batch** out);
lwfr_status lwfr_batch_workspace_bytes(const lwfr_batch* batch, size_t* bytes);
lwfr_status lwfr_batch_state_offsets(const lwfr_batch* batch, int64_t* offsets);
/* The context of problem i (owned by the batch; use it for lwfr_state_size,
 * lwfr_reference_nodes; it is bound to the batch workspace and stream). */
lwfr_status lwfr_batch_problem(lwfr_batch* batch, int32_t i, lwfr_ctx** ctx);
/* Caller-owned device workspace (256-byte aligned, lwfr_batch_workspace_bytes)
 * and stream; uploads the problem table synchronously. */
lwfr_status lwfr_batch_bind(lwfr_batch* batch, void* d_ws, size_t bytes, void* hip_stream);
/* One step of every problem; d_dt (nullable, device, count doubles) receives
 * each problem's dt.  d_u_out must not overlap d_u_in. */
lwfr_status lwfr_batch_step(lwfr_batch* batch, const double* d_u_in, double* d_u_out, double* d_dt);
/* Launch shape of a phase: tile_threads 256 or 128 threads per tile of
 * elements (floor(tile_threads/P) elements each; faces: 256 face points),
 * grid workgroups walking the tiles (0: one workgroup per tile), xcd 1 to give
 * each XCD a contiguous range of tiles, xcd 2, 3 or 4 to deal the tiles out to
 * the XCDs in chunks of 16, 64 or 256 consecutive tiles (0: no XCD grouping;
 * other values are an error).  Results do not depend on the shape. */
lwfr_status lwfr_batch_set_launch(lwfr_batch* batch, int32_t phase, int32_t tile_threads, int32_t grid, int32_t xcd);
lwfr_status lwfr_batch_get_launch(const lwfr_batch* batch, int32_t phase, int32_t* tile_threads, int32_t* grid,
                                  int32_t* xcd);
/* Autotuner: times every launch shape of every phase (tile_threads x grid in
 * {one per tile, 1024, 2048, 4096, 8192} x xcd, best of reps launches) on the
 * state d_u_in and keeps the fastest; d_u_out is used as scratch and holds one
 * step from d_u_in on return.  Synchronises the stream. */
lwfr_status lwfr_batch_autotune(lwfr_batch* batch, const double* d_u_in, double* d_u_out, int32_t reps);
/* As lwfr_graph_capture for the batch: d_dt_hist (nullable, nsteps x count). */
lwfr_status lwfr_batch_graph_capture(lwfr_batch* batch, double* d_u_a, double* d_u_b, int32_t nsteps,
                                     double* d_dt_hist);
lwfr_status lwfr_batch_graph_launch(lwfr_batch* batch);
/* As lwfr_query, over every problem of the batch. */
lwfr_status lwfr_batch_query(lwfr_batch* batch, uint32_t* flags_or);
lwfr_status lwfr_batch_timing_begin(lwfr_batch* batch, int32_t max_launches);
lwfr_status lwfr_batch_timing_end(lwfr_batch* batch, double* ms, uint32_t* launches);
lwfr_status lwfr_batch_destroy(lwfr_batch* batch);

/* Thread-local message of the last failing call ("" if none). */
const char* lwfr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LWFR_H */
