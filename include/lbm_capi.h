/*
 * lbm_capi.h -- C ABI of the MI355X (gfx950) preconditioned GLBE library.
 *
 * What the library computes (Premnath, Pattison & Banerjee, "Steady state
 * convergence acceleration of the generalized lattice Boltzmann equation with
 * forcing term through preconditioning"):
 *
 *   * the preconditioned generalized (multiple-relaxation-time) lattice
 *     Boltzmann equation with forcing on the D3Q19 lattice: effective collision
 *     in moment space with gamma-preconditioned equilibrium moments, moment
 *     source terms S^* = P_S S^ and preconditioned rates (Sec. 3, eqs.
 *     ppostcollision, pstreaming, prelax_term, precondsourceterm), followed by
 *     streaming along e_alpha (Sec. 2, eq. streaming);
 *   * optionally coupled to the preconditioned, chi-scaled vector lattice
 *     kinetic equation for the magnetic induction on the D3Q7 lattice, whose
 *     Lorentz force J x B enters the GLBE force (Sec. 4, Sec. 4.1);
 *   * the steady-state residual ||u(t) - u(t-10)||_2 (Sec. 5), relative, in FP64;
 *   * FP64 global mass and flow-rate reductions;
 *   * a discrete adjoint of the step for d(steady flow rate)/d(force field);
 *   * the two-dimensional variants (D2Q9 flow, D2Q5 induction; Sec. 2-4);
 *   * moving walls and an induction lattice extending beyond the fluid box
 *     (the MHD lid-driven cavity of Sec. 5);
 *   * batched marches of many small independent lattices with per-lattice
 *     stability verdicts (the stability map of Sec. 5).
 *
 * Conventions (all entry points):
 *   - Every function returns an lbm_status; no exception crosses the ABI.
 *   - Device memory is owned by the caller.  The library allocates no device
 *     memory: the caller provides one workspace (size from lbm_workspace_bytes)
 *     and, for the adjoint, one adjoint workspace.  The library owns only the
 *     host-side context object and, with it, 4 KB of pinned host memory
 *     (hipHostMalloc) that history reads copy through; lbm_destroy frees
 *     both.
 *   - All device work is enqueued on the caller's HIP stream given at
 *     lbm_create.  Calls documented as "synchronizes" wait for that stream.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Grid layout: nodes are indexed (x, y, z) with x the unit-stride axis,
 *     linear index n = x + nx*(y + ny*z), N = nx*ny*nz.  Population arrays
 *     exchanged through the ABI are structure-of-arrays [q][N] (direction
 *     outermost, unpadded).  Every node is a fluid node (unless mag_pad
 *     extends the induction lattice): walls sit half a link outside the first
 *     and last node of a wall axis (halfway bounce-back, Sec. 5).
 *   - State: the stored populations are the post-collision values of the last
 *     completed step, held as deviations from the rest state,
 *     f~_alpha - w_alpha rho0.  The hydrodynamic fields "at the current time"
 *     are those of the streamed populations, i.e. of the next collision.
 *   - Direction ordering is given by lbm_lattice_velocities.
 */
#ifndef LBM_CAPI_H
#define LBM_CAPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument (message in lbm_last_error)            */
  LBM_ENOWS = -2,      /* workspace missing, misaligned or too small              */
  LBM_EHIP = -3,       /* a HIP runtime call failed (hipGetErrorString text kept) */
  LBM_EUNSTABLE = -4,  /* non-finite values or residual blow-up detected          */
  LBM_ESTATE = -5,     /* call not valid in the context's current state           */
  LBM_EUNSUPPORTED = -6 /* valid request the library does not implement          */
} lbm_status;

/* Population storage type.  F64 storage computes in FP64; F32, BF16 and F16
 * storage compute in FP32 (deviation storage, round-to-nearest-even on store). */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_BF16 = 2, LBM_F16 = 3 } lbm_dtype;

/* Per-axis boundary: periodic wrap, or a no-slip wall on both faces of the axis
 * (halfway/link bounce-back for the flow, Sec. 5; anti-bounce-back Dirichlet
 * B = B0 for the magnetic populations). */
typedef enum { LBM_PERIODIC = 0, LBM_WALL = 1 } lbm_bc;

typedef enum { LBM_FORCE_UNIFORM = 0, LBM_FORCE_FIELD = 1 } lbm_force_mode;

/* Velocity sets: D3Q19 flow with D3Q7 induction, or the two-dimensional D2Q9
 * flow with D2Q5 induction (Sec. 2 eq. velocityd2q9, Sec. 4 eq. velocityd2q5). */
typedef enum { LBM_D3Q19 = 0, LBM_D2Q9 = 1 } lbm_lattice;

typedef struct {
  int32_t n[3];   /* nx, ny, nz >= 1; N = nx*ny*nz < 2^31 */
  int32_t bc[3];  /* lbm_bc per axis */
} lbm_grid;

/* Launch shape of the step kernels.  None of these changes a result: they
 * decide which workgroup updates which nodes, the cache policy of the
 * population stores and the width of the address arithmetic, and every
 * combination gives bitwise the same states and histories (tested).  All zero
 * (the default) lets the library choose (see lbm_create). */
typedef struct {
  int32_t xcd_chunk;  /* 0: library's choice; n > 0: the XCDs take n consecutive
                         workgroups of the node range in turn (n >= the
                         workgroups per XCD: one contiguous slab per XCD) */
  int32_t store;      /* 0: library's choice; 1: cacheable stores; 2: streaming
                         (non-temporal) stores of the populations */
  int32_t offsets;    /* 0: 32-bit byte offsets wherever they fit, else 64-bit
                         element offsets; 1: 64-bit element offsets always */
  int32_t load;       /* 0: library's choice; 1: cacheable loads; 2: streaming
                         (non-temporal) loads of the populations and the force
                         field, D3Q19 steps with streaming stores only */
  int32_t waves;      /* 0: library's choice; 3..7: at most this many waves per
                         SIMD run the step kernels (each workgroup reserves an
                         unused share of the compute unit's LDS); 8: no cap
                         beyond the kernels' own register use */
} lbm_launch;

typedef struct {
  int32_t storage;        /* lbm_dtype */
  double gamma;           /* preconditioning parameter, 0 < gamma <= 1 (Sec. 3) */
  double s[19];           /* preconditioned rates s*_k in moment order (Sec. 3);
                             entries 0, 3, 5, 7 (conserved moments) are ignored;
                             the others must lie in (0, 2).  lbm_default_rates fills them. */
  double rho0;            /* reference density (1.0) */
  int32_t force_mode;     /* lbm_force_mode */
  double force_const[3];  /* uniform force (force_mode = UNIFORM) */
  int32_t mhd;            /* 1: couple the D3Q7 vector induction LKE (Sec. 4) */
  double gamma_m;         /* induction preconditioning parameter, 0 < gamma_m <= 1 */
  double chi;             /* low-Pm scaling factor chi > 0 (Sec. 4.1) */
  double eta;             /* magnetic diffusivity; tau_m* = eta/(gamma_m theta_m) + 1/2 */
  double mu;              /* magnetic permeability (1 in lattice units) */
  double B0[3];           /* applied field: initial state and wall value */
  int32_t check_every;    /* residual / reductions every this many steps (10) */
  int32_t history_len;    /* entries of the device residual history ring (>= 1) */
  int32_t source_mode;    /* 0: preconditioned sources S^* = P_S S^ (Sec. 3, eq.
                             precondsourceterm); 1: the naive S^/gamma for every
                             moment (Sec. 3.1, eq. precondsourceincorrect), kept
                             only to exhibit its spurious steady-state error */
  double wall_u[6][3];    /* velocity of each wall face (x-low, x-high, y-low,
                             y-high, z-low, z-high) for link bounce-back with wall
                             momentum (the moving lid of Sec. 5's cavity): a link
                             reflected at a moving face gains 6 w_a rho0 (e_a . u_w);
                             a link crossing two walls at an edge takes the mean of
                             the two faces' terms.  Zero for fixed walls; ignored on
                             periodic axes and by the magnetic populations. */
  int32_t mag_pad[3];     /* extended induction lattice (Sec. 5, MHD cavity): with
                             mhd = 1 and wall axes only, the grid is the induction
                             lattice and the fluid occupies the box
                             [mag_pad[a], n[a] - mag_pad[a]) on each axis a.  The
                             flow has no-slip walls (moving as wall_u says) at the
                             box faces; the induced field B - B0 is zero at the
                             lattice faces; outside the box u = 0, rho = rho0, f is
                             not updated, and the induction populations only
                             diffuse.  Residual, mass and flow sums cover the box.
                             All zero: fluid and induction lattices coincide. */
  int32_t lattice;        /* lbm_lattice.  LBM_D2Q9: n[2] must be 1 (bc[2] is
                             ignored); s[0..8] are the rates in D2Q9 moment order
                             (rho, e, e2, j_x, q_x, j_y, q_y, p_xx, p_xy; conserved
                             0, 3, 5 ignored; lbm_default_rates_d2q9 fills them);
                             forces and B0 use their x and y components (B0[2]
                             and force_const[2] must be 0); wall_u and mag_pad
                             must be zero; no adjoint.  Force fields, u and B
                             keep their [3][N] layout (z components unused on
                             input, zero on output); the state blob holds f as
                             [9][N] and (mhd) g as [2][5][N]. */
  int32_t rounding;       /* lbm_rounding: how the step rounds the populations it
                             stores.  LBM_ROUND_STOCHASTIC needs LBM_BF16 or LBM_F16
                             storage and the flow step alone (no mhd); see below. */
  uint32_t seed;          /* stochastic rounding: seed of the counter-based
                             random bits (any value; the same seed gives the
                             same march bit for bit) */
  lbm_launch launch;      /* launch shape (all zero: the library's choice) */
} lbm_params;

/* Rounding of stored populations.  LBM_ROUND_NEAREST: nearest, ties to even.
 * LBM_ROUND_STOCHASTIC (16-bit storage): each FP32 result v is rounded to
 * the 16-bit value above it in magnitude with probability equal to its
 * distance from the value below (in units of their spacing, resolved to
 * 2^-16 for BF16 and 2^-13 for FP16), so that the stored value is unbiased
 * and per-step changes smaller than the spacing still accumulate.  With r the
 * 16 random bits of that value:
 *   BF16: stored bits = the upper 16 bits of (FP32 bits of v + r);
 *   FP16: with s = |v| (|v| >= 2^-14) or s = |v| + 2^-14 rounded to FP32
 *     (|v| < 2^-14, FP16's subnormal range), the FP32 bits of s plus (r >> 3)
 *     with their low 13 bits cleared, minus the 2^-14 offset if added (an
 *     exact subtraction), converted exactly (Inf on overflow);
 * Inf and NaN are kept.  The random bits are counter-based:
 * for node n, directions 2k and 2k+1 (k = 0..9 for D3Q19, 0..4 for D2Q9, in
 * the order of lbm_lattice_velocities), and the step number t being
 * computed, h = fmix32(n*0x9E3779B1 + t*0x85EBCA77 + k*0xC2B2AE3D + seed)
 * (32-bit wrap-around; fmix32 is the 32-bit finalizer of MurmurHash3:
 * h ^= h >> 16; h *= 0x85EBCA6B; h ^= h >> 13; h *= 0xC2B2AE35; h ^= h >> 16);
 * direction 2k takes the low 16 bits of h, direction 2k+1 the high 16. */
typedef enum { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 } lbm_rounding;

typedef struct lbm_ctx lbm_ctx;

/* One residual-history record (all FP64), written on device every
 * check_every steps.  residual = sqrt(du2 / u2), with du2 = sum |u(t)-u(t-k)|^2
 * and u2 = sum |u(t)|^2 over all fluid nodes and components (u(t-k) = 0 at
 * the first check).  mass = sum (rho - rho0); flow = (1/nx) sum j_x with nx the
 * fluid box's x extent (j includes F/(2 gamma)); nonfinite = count of nodes
 * with a non-finite rho or j.  All of these are taken from the populations
 * entering the collision of `step`. */
typedef struct {
  double step, residual, du2, u2, mass, flow, nonfinite, reserved;
} lbm_record;

/* Fill s_out[19] with the preconditioned D3Q19 rates of Sec. 3:
 * shear modes 9, 11, 13, 14, 15: 1/s = 3 nu/gamma + 1/2; s1 = 1.19,
 * s2 = s10 = s12 = 1.4; mode 0 ("paper"): s4 = s6 = s8 = 1.2, s16..18 = 1.98;
 * mode 1 ("fixed Lambda"): s4 = s6 = s8 = s16 = s17 = s18 = s_q with
 * (3 nu/gamma)(1/s_q - 1/2) = Lambda.  Conserved entries are set to 1.
 * Errors: LBM_EINVAL for nu <= 0, gamma outside (0,1], Lambda <= 0 in mode 1. */
lbm_status lbm_default_rates(double nu, double gamma, int32_t mode, double Lambda,
                             double s_out[19]);

/* Fill s_out[9] with the preconditioned D2Q9 rates of Sec. 3 (moment order
 * rho, e, e2, j_x, q_x, j_y, q_y, p_xx, p_xy): p_xx, p_xy: 1/s = 3 nu/gamma + 1/2;
 * s_e = 1.63, s_e2 = 1.14; mode 0: s_q = 1.92; mode 1: s_q from
 * (3 nu/gamma)(1/s_q - 1/2) = Lambda.  Conserved entries are set to 1.
 * Errors as lbm_default_rates. */
lbm_status lbm_default_rates_d2q9(double nu, double gamma, int32_t mode, double Lambda,
                                  double s_out[9]);

/* Velocity set in the library's direction order: q = 19 (D3Q19, flow), q = 9
 * (D2Q9, flow), q = 5 (D2Q5, induction; both with e_z = 0) or q = 7
 * (D3Q7, induction); writes q*3 integers (ex, ey, ez per direction) to e_out
 * (host memory).  Errors: LBM_EINVAL for another q or a NULL pointer. */
lbm_status lbm_lattice_velocities(int32_t q, int32_t* e_out);

/* Bytes of device workspace lbm_create needs for this grid and parameter set
 * (host pointers in, host size_t out).  The workspace must be 256-byte aligned. */
lbm_status lbm_workspace_bytes(const lbm_grid* grid, const lbm_params* params, size_t* bytes);

/* Validate, lay out the workspace, initialise the rest state (populations
 * f = w rho0, i.e. zero deviations; magnetic g = W B0, Sec. 4) and, for
 * force_mode = FIELD, copy the force field (device pointer `force`, layout
 * [3][N], FP64 for F64 storage, FP32 otherwise) into the workspace.
 * `workspace` is a device pointer owned by the caller that must outlive the
 * context; `hip_stream` is a hipStream_t (NULL = default stream).
 * Launch shape (params->launch, all zero: the library's choice): lattices
 * whose two population buffers fit the 256 MB last-level cache get one
 * contiguous slab per XCD and cacheable stores; up to 512 MB, slabs and
 * streaming stores; above that (lattices that stream from HBM) streaming
 * stores, a cap on the waves per SIMD (D3Q19: 5 for FP32 storage, 6 for
 * 16-bit storage, 3 for FP64 storage and for the coupled step; D2Q9: 6 for
 * FP32, 4 for FP64, 5 for the coupled FP32 step, none otherwise) and, for
 * D3Q19, streaming loads (of the flow step's force field only while that
 * field is larger than 80% of the last-level cache; a smaller one keeps
 * cacheable loads and stays in that cache from step to step),
 * and lbm_create times a few dozen plain steps on the stream for each
 * of five XCD workgroup mappings (chunks of 1, 2, 4 and 8 workgroups, slabs), keeps
 * the fastest and restores the rest state; it then synchronizes (a few ms to
 * a few tens of ms).  A non-zero launch.xcd_chunk skips the timing.  The
 * mapping decides only which workgroup updates which nodes: results are the
 * same whichever is chosen.
 * Errors: LBM_EINVAL (grid, rates, gamma, mhd parameters, unsupported
 * combination), LBM_ENOWS, LBM_EHIP.  On error *out is NULL and the message
 * is available from lbm_last_error(NULL). */
lbm_status lbm_create(const lbm_grid* grid, const lbm_params* params, const void* force,
                      void* workspace, size_t workspace_bytes, void* hip_stream,
                      lbm_ctx** out);

/* The launch shape the context uses (after lbm_create's choice): the XCD
 * chunk in workgroups, store and load 1 (cacheable) or 2 (streaming), offsets
 * 0 (32-bit byte offsets) or 1 (64-bit element offsets) of the flow step, and
 * the cap on waves per SIMD (8: none).  Host only.
 * Errors: LBM_EINVAL for a NULL argument. */
lbm_status lbm_get_launch(const lbm_ctx* ctx, lbm_launch* out);

/* Release the host-side context (no device memory is freed). */
void lbm_destroy(lbm_ctx* ctx);

/* Replace the force field (device pointer, [3][N] in the compute type); only
 * for force_mode = FIELD (else LBM_ESTATE).  Enqueued on the stream. */
lbm_status lbm_set_force(lbm_ctx* ctx, const void* force);

/* Enqueue n >= 0 time steps (stream, then collide).  Every check_every-th
 * step also writes one lbm_record to the device history ring.  Asynchronous:
 * does not synchronize and does not report instability (see lbm_residual). */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Like lbm_step, but times every step kernel with a HIP event attached to its
 * own dispatch on the stream (hipExtLaunchKernel), synchronizes, and returns
 * the mean step duration in microseconds and the wall time of the whole call
 * in milliseconds.  A step's duration runs from the end of the previous step
 * kernel to the end of its own: the kernel plus the dispatch gap before it (a
 * fraction of a microsecond).  The first step of every 512, and a step that
 * first reduces pending residual checks, is timed from a start event on its
 * own dispatch instead (the kernel alone).  No marker packets sit between the
 * steps otherwise, so the call marches at the rate of lbm_step.  Before it
 * returns, the call also reduces the pending residual checks into the history
 * (the records are the same as when lbm_history does it). */
lbm_status lbm_step_timed(lbm_ctx* ctx, int64_t n, double* mean_kernel_us, double* wall_ms);

/* Like lbm_step_timed, but writes every step's duration in
 * microseconds to the host array kernel_us[n] (step i of the call is the
 * context's step t0 + i + 1, a residual-check step when that number is a
 * multiple of check_every).  Synchronizes. */
lbm_status lbm_step_times(lbm_ctx* ctx, int64_t n, double* kernel_us, double* wall_ms);

/* Latest history record: residual and the step it was taken at.  Synchronizes.
 * Returns LBM_ESTATE if no check has run yet, LBM_EUNSTABLE (after filling
 * the outputs) if that record counted non-finite values. */
lbm_status lbm_residual(lbm_ctx* ctx, double* residual, int64_t* at_step);

/* Copy up to max_records most recent history records, oldest first, to host
 * memory `out`; *n_out receives the count.  Synchronizes. */
lbm_status lbm_history(lbm_ctx* ctx, lbm_record* out, int64_t max_records, int64_t* n_out);

/* March until a record has residual < tol (finite), or max_steps steps have
 * been taken in this call.  Steps are enqueued in chunks of at most
 * poll_every steps (rounded to check_every) and the history is read after
 * each chunk, so the crossing step is exact but up to one chunk of extra
 * steps may run after it.  *steps_to_tol = step count (since create) of the
 * first record below tol, or -1; *final_residual = that record's residual
 * (or the last one).  Returns LBM_EUNSTABLE on non-finite values or when the
 * residual exceeds 1e3 times its running minimum.  Synchronizes. */
lbm_status lbm_run_to_residual(lbm_ctx* ctx, double tol, int64_t max_steps, int64_t poll_every,
                               int64_t* steps_to_tol, double* final_residual);

/* March until the relative change of the kinetic-energy sum |u|^2 (the u2
 * field of the history records) over `window` steps falls below tol, or
 * max_steps steps have been taken in this call.  Unlike the residual, this
 * global sum averages out the rounding noise of 16-bit storage (stochastic
 * rounding included), so it can end a 16-bit march once the flow itself has
 * converged.  For a slow mode of relative amplitude a decaying at rate lambda
 * per step the change per window is about 2 a (1 - exp(-lambda window)).
 * window must be a positive multiple of check_every; steps are enqueued one
 * window at a time and the first window only sets the reference.
 * *step_out = the step of the record at which the change fell below tol, or
 * -1; *change_out = the last change computed (NaN before two windows).
 * Returns LBM_EUNSTABLE on non-finite values.  Synchronizes. */
lbm_status lbm_run_to_energy_change(lbm_ctx* ctx, double tol, int64_t max_steps, int64_t window,
                                    int64_t* step_out, double* change_out);

/* FP64 mass drift sum(rho - rho0) and flow rate (1/nx) sum j_x of the
 * current state (streamed populations; j includes F/(2 gamma); with mhd the
 * Lorentz force is included).  Synchronizes. */
lbm_status lbm_reductions(lbm_ctx* ctx, double* mass_drift, double* flow_rate);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * reductions of lbm_reductions for a population state the caller holds, with
 * no context and no workspace.  state: device [q][N] in the storage type
 * (q = 19, or 9 for D2Q9), as lbm_get_state writes it (deviations from
 * w rho0, post-collision values of the last step); force: device [3][N] in the
 * compute type for force_mode = FIELD (ignored for UNIFORM); grid and params
 * as for lbm_create (mhd = 0 only: LBM_EUNSUPPORTED otherwise).  Enqueues on
 * hip_stream, which must belong to the current device, and writes
 * out[0] = sum (rho - rho0), out[1] = (1/nx) sum j_x of the streamed state
 * (FP64, device pointer).  Does not synchronize and allocates nothing: the
 * partial sums live in a 4 MiB scratch array in device memory that each GPU
 * holds for the life of the process, so lattices are limited to 26,841,856
 * nodes (LBM_ENOWS beyond).  All calls on one GPU share that scratch: calls
 * that overlap in time on one GPU (several host threads, or several streams
 * of one GPU) race and must be serialized by the caller.  Errors: LBM_EINVAL,
 * LBM_ENOWS, LBM_EUNSUPPORTED, LBM_EHIP (lbm_last_error(NULL)). */
lbm_status lbm_reductions_noalloc(const lbm_grid* grid, const lbm_params* params,
                                  const void* state, const void* force, void* hip_stream,
                                  double* out);

/* Hydrodynamic fields of the current state into caller device buffers:
 * rho [N], u [3][N] (physical velocity, F/(2 gamma) included), B [3][N]
 * (mhd only; may be NULL).  out_dtype is LBM_F64 or LBM_F32.  Enqueued. */
lbm_status lbm_moments(lbm_ctx* ctx, int32_t out_dtype, void* rho, void* u, void* B);

/* Number of bytes of the state blob: populations [19][N] in the storage type,
 * followed (mhd) by the magnetic populations [3][7][N] (field component
 * outermost) in the compute type, held as deviations g_{a j} - W_a B0_j from the
 * applied field's rest equilibrium (so that FP32 keeps the small induced field). */
lbm_status lbm_state_bytes(const lbm_ctx* ctx, size_t* bytes);

/* Copy the state blob to / from caller device memory, and read / set the step
 * counter.  lbm_set_state also clears the residual snapshot and history.  With
 * mag_pad, f outside the fluid box keeps the values last set here (zero
 * deviations after lbm_create). */
lbm_status lbm_get_state(lbm_ctx* ctx, void* dst);
/* Continue src's march in dst's precision: dst's state becomes src's current
 * state converted to dst's storage type on the device (through FP64; rounding
 * to nearest even when narrowing, whatever dst's rounding option; the option
 * applies to the steps dst then takes), its step counter becomes src's, and its
 * residual snapshot and history are cleared as by lbm_set_state.  Both contexts
 * need the same grid, boundaries, lattice, rho0, mhd, B0 and mag_pad.  Enqueued
 * on dst's stream after the work already enqueued on src's stream.  Errors:
 * LBM_EINVAL (mismatch), LBM_EHIP. */
lbm_status lbm_convert_state(lbm_ctx* dst, const lbm_ctx* src);
lbm_status lbm_set_state(lbm_ctx* ctx, const void* src, int64_t step);
lbm_status lbm_get_step(const lbm_ctx* ctx, int64_t* step);

/* ---------------------------------------------------------------- adjoint ---
 * Discrete adjoint of one step Phi(f~; F) = Collide(Stream(f~); F) for the
 * flow rate Q = (1/nx) sum_x j_x of the streamed state (F64 or F32 storage,
 * no mhd; LBM_EUNSUPPORTED otherwise).  Gradients are written to a caller
 * device buffer dQdF [3][N] in the compute type. */

/* Adjoint workspace bytes.  mode 0: steady (fixed-point) adjoint;
 * mode 1: unrolled over n_steps with a checkpoint every ckpt_every steps. */
lbm_status lbm_adjoint_workspace_bytes(const lbm_ctx* ctx, int32_t mode, int64_t n_steps,
                                       int64_t ckpt_every, size_t* bytes);

/* Steady adjoint at the current state (meant to be a converged steady state):
 * iterates the transposed linearised step to its own fixed point (relative
 * change of the adjoint below tol, checked every check_every iterations, at
 * most max_iter iterations), then writes dQ/dF.  The mass direction, along
 * which the steady state is not unique, is projected out.  Synchronizes. */
lbm_status lbm_adjoint_steady(lbm_ctx* ctx, void* adj_ws, size_t adj_ws_bytes, double tol,
                              int64_t max_iter, void* dQdF, int64_t* iters,
                              double* final_change);

/* Unrolled adjoint: marches n_steps forward from the current state
 * (the state advances, as lbm_step would, storing a checkpoint every
 * ckpt_every steps), then sweeps backwards recomputing each segment from its
 * checkpoint, and writes dQ_N/dF for Q_N = Q of the state after n_steps.
 * Synchronizes. */
lbm_status lbm_adjoint_unrolled(lbm_ctx* ctx, void* adj_ws, size_t adj_ws_bytes, int64_t n_steps,
                                int64_t ckpt_every, void* dQdF);

/* Text of the last error on ctx, or (ctx = NULL) of the last failed
 * lbm_create on this thread.  Never NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* ------------------------------------------------------------- batches --
 * Many independent small lattices marched together, one launch per step: the
 * stability map of Sec. 5 classifies many (viscosity, velocity, gamma) points
 * on small Poiseuille lattices.  All members share the grid (no induction);
 * each has its own gamma, rates and uniform force. */
typedef struct {
  double gamma;     /* 0 < gamma <= 1 */
  double s[19];     /* D3Q19 rates as in lbm_params */
  double force[3];  /* uniform force */
} lbm_member;

typedef struct {
  int32_t verdict;   /* 0: undecided after max_steps; 1: residual below tol;
                        2: unstable (non-finite values, or the residual above
                        1e-2 and 1e3 times its running minimum) */
  int32_t reserved;
  int64_t step;      /* step of the verdict (-1 when undecided) */
  double residual;   /* last residual computed (NaN before the first check) */
} lbm_member_result;

/* Device workspace bytes for `count` members on `grid` with storage type
 * `storage` (each member's nodes rounded up to whole 256-node workgroups).
 * Errors: LBM_EINVAL for a bad grid or storage, count < 1, or 2^31 or more
 * padded nodes. */
lbm_status lbm_batch_workspace_bytes(const lbm_grid* grid, int32_t storage, int32_t count,
                                     size_t* bytes);

/* March all members from rest (deviations zero) on `stream` until each is
 * decided or max_steps is reached, with the residual every check_every steps
 * (the rules of lbm_run_to_residual, per member); the host polls the verdicts
 * every poll_every steps and stops early once all are decided.  members and
 * results are host arrays of `count`; workspace is caller device memory
 * (256-byte aligned, lbm_batch_workspace_bytes).  Blocks the calling thread
 * until the march ends.  launch may be NULL (the library's choice); only its
 * offsets field applies (members are laid out in whole workgroups, one slab
 * per XCD, cacheable stores).  Errors: LBM_EINVAL (arguments, with the member
 * index), LBM_ENOWS (workspace), LBM_EHIP. */
lbm_status lbm_batch_run(const lbm_grid* grid, int32_t storage, double rho0, int32_t count,
                         const lbm_member* members, void* workspace, size_t workspace_bytes,
                         void* stream, double tol, int64_t max_steps, int32_t check_every,
                         int64_t poll_every, const lbm_launch* launch,
                         lbm_member_result* results);

/* ---------------------------------------------------------- calibration --
 * The bandwidth the HBM delivers for copies of FP32 data, timed by the caller
 * around the launch (the step kernels' roofline fractions are read against
 * these as well as against the nominal peak).  The lattice is nx * ny * nz
 * nodes (x fastest); src and dst are device buffers of at least 22 * nodes
 * (patterns 2 and 4: 40 * nodes) FP32 values each, 16-byte aligned, planes of
 * `nodes` values.
 * pattern 0: 22 * nodes values copied as 16-byte vectors, one per thread,
 *            streaming loads and stores (moves 2 * 88 * nodes bytes);
 * pattern 1: at each node 22 planes read and 19 written, one value per plane
 *            and thread, streaming loads and stores, workgroups dealt to the
 *            XCDs in chunks of xcd_chunk (moves 164 * nodes bytes);
 * pattern 2: the same with 40 planes read and 40 written (320 * nodes bytes);
 * pattern 3: the row-aligned FP32 flow step's exact memory traffic without its
 *            arithmetic (Sec. 2 eq. streaming): planes 0-18 are the D3Q19
 *            populations in the library's direction order
 *            (lbm_lattice_velocities), each read at the upstream node with
 *            periodic wrap, or in the opposite direction's plane at the node
 *            itself where the link crosses a wall (walls: bit 0 x, bit 1 y,
 *            bit 2 z); planes 19-21 (the force field) read at the node; dst
 *            planes 0-18 receive the gathered values, plane 0 plus 0 times the
 *            sum of the force planes (164 * nodes bytes);
 * pattern 4: the coupled step's (Sec. 4): planes 0-18 as in pattern 3, planes
 *            19-39 the D3Q7 populations (component-major, 7 directions per
 *            component) gathered the same way from the D3Q7 directions, all 40
 *            written (320 * nodes bytes); the sign of anti-bounce-back, being
 *            arithmetic, is left out.
 * Patterns 3 and 4 need nx a multiple of 64 and 21 * nodes * 4 < 2^32.
 * waves: at most this many waves per SIMD (3..7, as lbm_launch.waves), or 8
 * for no cap.  Enqueued on hip_stream.  Errors: LBM_EINVAL, LBM_EHIP. */
lbm_status lbm_bandwidth_probe(int32_t pattern, const void* src, void* dst, int32_t nx, int32_t ny,
                               int32_t nz, int32_t walls, int32_t xcd_chunk, int32_t waves,
                               void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CAPI_H */
