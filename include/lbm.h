/*
 * lbm.h -- C ABI of the MI355X (gfx950) coupled phase-field / hydrodynamic
 * lattice Boltzmann solver.
 *
 * The solver advances the conservative Allen-Cahn phase-field LBM on D3Q15
 * and the velocity-based hydrodynamic LBM on D3Q27 of Holzer et al.,
 * "Highly efficient lattice Boltzmann multiphase simulations of immiscible
 * fluids at high-density ratios on CPUs and GPUs through code generation"
 * (IJHPCA 2020), Section 3 (model) and Section 4.2 (the improved algorithm:
 * one fused phase-field sweep and one fused hydrodynamic sweep per step).
 *
 * Conventions shared by every call:
 *   - Grid: nx * ny * nz cells, x fastest: cell = x + nx*(y + ny*z).
 *     x and z are periodic; y is periodic unless walls_y, in which case rows
 *     y = 0 and y = ny-1 are solid no-slip walls (halfway bounce-back for both
 *     PDF sets, mirrored phase field in the finite-difference stencils).
 *   - Field arrays passed in or out are dense planes of nx*ny*nz values
 *     (a vector field is 3 consecutive planes x, y, z; a PDF set is q
 *     consecutive planes in the canonical direction order of
 *     lbm_velocity_set).  Values at wall cells are zero on output and
 *     ignored on input.
 *   - Unless stated otherwise a pointer argument is a DEVICE pointer, owned
 *     by the caller; the library keeps no reference to it after the call
 *     returns, except the workspace given to lbm_create.
 *   - Every call returns an lbm_status; lbm_last_error() then holds a text
 *     for the calling thread.  No call aborts or exits the process.
 *   - Work is enqueued on the HIP stream given to lbm_create (the calling
 *     framework's current stream); calls are asynchronous unless they
 *     return host values (reductions), which synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EARG = -1,       /* bad argument or parameter set                  */
    LBM_EHIP = -2,       /* a HIP runtime call or kernel launch failed      */
    LBM_ESTATE = -3,     /* call out of order (e.g. step before init)       */
    LBM_ENONFINITE = -4, /* a reduction produced NaN or Inf                 */
    LBM_ESIZE = -5       /* workspace too small / grid too large           */
} lbm_status;

/* PDF storage formats.  Collision arithmetic is FP64 for LBM_F64 and FP32
 * for the others; phi and u are stored in the arithmetic type.  The 16-bit
 * formats store shifted / scaled populations of order u instead of the
 * populations: h_i - phi w_i with phi of the cell the value is stored at, and
 * g_i / w_i (the velocity-based g_i ~ w_i (p* + 3 e_i.u + ...) is already a
 * deviation). */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 } lbm_storage;

/* Element types of the field arrays exchanged by the get/set calls. */
typedef enum { LBM_DTYPE_F64 = 0, LBM_DTYPE_F32 = 1 } lbm_dtype;

/* Model parameters in lattice units (dx = dt = 1, c_s^2 = 1/3).
 *   phi_L, phi_H   bulk phase-field values of the light / heavy fluid (Sec. 3.1)
 *   xi             interface thickness; beta = 12 sigma/xi, kappa = 3 sigma xi/2
 *   mobility       M = tau_phi c_s^2 (eq. mobility); the phase-field relaxation
 *                  rate is 1/(tau_phi + 1/2)
 *   sigma          surface tension
 *   rho_L, rho_H   densities, interpolated linearly in phi (eq. density)
 *   tau_L, tau_H   hydrodynamic relaxation times with nu = tau c_s^2,
 *                  interpolated linearly in phi; the second-order moments
 *                  relax with 1/(tau + 1/2), all others with 1 (Sec. 3.2)
 *   body_accel     body acceleration a; the body force is
 *   buoyancy_rho_ref   F_b = (rho - buoyancy_rho_ref) a.  0 gives the buoyancy
 *                  rho g of Sec. 6.1 literally; rho_H removes the hydrostatic
 *                  part of the pressure (same flow between the y walls, the
 *                  pressure differs by a linear field), which keeps p* small
 *                  in tall domains
 *   normal_eps     interface normal n = grad phi / (|grad phi| + normal_eps)
 *   storage        an lbm_storage value
 *   density_literal  0: phi is clamped to [min(phi_L, phi_H), max(phi_L, phi_H)]
 *                  before the density and tau interpolations (the default;
 *                  the conservative phase field over- and undershoots the
 *                  interval by ~1e-3, which at rho_H/rho_L = 1000 would give
 *                  a near-zero density in small bubble cores); 1: eq. density
 *                  and the tau interpolation as printed, for every phi
 *   lattice_phase  velocity set of the phase-field step: 15 (0 = the default
 *                  D3Q15), 19 or 27
 *   lattice_hydro  velocity set of the hydrodynamic step: 27 (0 = the default
 *                  D3Q27), 19 or 15; its moment set is the weighted-orthogonal
 *                  Gram-Schmidt of the monomials independent on the set
 *   phase_mrt      0: single-rate phase-field collision (the benchmarks of
 *                  Sec. 5); 1: raw-moment MRT, first-order moments relaxed
 *                  with the phase-field rate, all others with one (Sec. 3.1)
 *                  Built combinations (phase, hydro, MRT): (15, 27, 0) for every
 *                  storage; with FP64 and FP32 storage also (15, 27, 1),
 *                  (19, 19, 0), (19, 19, 1), (27, 27, 0) and (15, 15, 0), the
 *                  stencil study of Sec. 5.1 and the D3Q19 lattice of Sec. 6.1;
 *                  others give LBM_EARG */
typedef struct {
    int32_t nx, ny, nz;
    int32_t walls_y;
    double phi_L, phi_H, xi, mobility, sigma;
    double rho_L, rho_H, tau_L, tau_H;
    double body_accel[3];
    double buoyancy_rho_ref;
    double normal_eps;
    int32_t storage;
    int32_t density_literal;
    int32_t lattice_phase;
    int32_t lattice_hydro;
    int32_t phase_mrt;
} lbm_params;

/* FP64 diagnostics over fluid cells (one deterministic two-pass reduction).
 * chi = (phi_H - phi)/(phi_H - phi_L) marks the light phase.
 *   mass           sum phi                     (conserved by the scheme)
 *   momentum       sum rho u
 *   gas_volume     sum chi
 *   centroid       sum chi x / sum chi         (x, y, z in cell units)
 *   rise_velocity  sum chi u_y / sum chi
 *   interface_sum  sum 4 chi (1 - chi)
 *   grad_sum       sum |grad phi| / (phi_H - phi_L)   (D3Q27 isotropic gradient)
 *   xi_eff         interface_sum / grad_sum   (= xi for the planar profile)
 *   max_speed      max |u| */
typedef struct {
    double mass;
    double momentum[3];
    double gas_volume;
    double centroid[3];
    double rise_velocity;
    double interface_sum;
    double grad_sum;
    double xi_eff;
    double max_speed;
} lbm_stats;

/* Host call.  Writes the canonical velocity set with q = 15 (D3Q15) or
 * q = 27 (D3Q27): e is q*3 int32 (host), w is q doubles (host).  Order: rest,
 * axis pairs, then (q = 27) edge pairs, then corner pairs; the opposite of
 * every odd index i is i+1.  Returns LBM_EARG for other q. */
lbm_status lbm_velocity_set(int32_t q, int32_t *e, double *w);

/* Host call.  Bytes of device workspace lbm_create needs for these
 * parameters (two PDF grids per set, two phase fields, velocity, reduction
 * scratch).  Returns 0 if the parameters are invalid (then lbm_last_error
 * says why). */
size_t lbm_workspace_bytes(const lbm_params *p);

/* Creates a solver context.  dev_workspace: caller-owned device memory of
 * at least lbm_workspace_bytes(p) bytes, 256-byte aligned, that must stay
 * allocated until lbm_destroy.  hip_stream: a hipStream_t (NULL = default
 * stream).  The context owns no device memory.  *out receives the context.
 * Sweep kernels: the environment variable LBM_ZMARCH, read here, selects the
 * z-marching sweeps that stage the phase field of three planes in LDS
 * ("1") or the one-cell-per-thread sweeps ("0"); unset, the library's
 * default.  With 16-bit storage and even nz the sweeps process cells z and
 * z + nz/2 together from shared 32-bit words; LBM_PAIR=0 selects the
 * one-cell-per-thread sweeps instead.  With FP32 and FP64 storage and the
 * one-cell-per-thread sweeps, lbm_step runs the hydrodynamic sweep of each
 * step and the phase-field sweep of the next in one kernel; LBM_FUSE=0
 * keeps them separate.  All variants compute the same numbers (same
 * operation order). */
lbm_status lbm_create(const lbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                      lbm_ctx **out);

/* Changes the stream later calls enqueue on. */
lbm_status lbm_set_stream(lbm_ctx *ctx, void *hip_stream);

/* Initial state (Sec. 4.2, "initialisation of all fields"): from device FP64
 * arrays phi (1 plane), u (3 planes) and p* = p/(rho c_s^2) (1 plane):
 * phase-field PDFs h_i = phi Gamma_i(u) taken as post-collision, hydrodynamic
 * PDFs g_i = p* w_i + Gamma_i(u) - w_i taken as pre-collision, phase field and
 * velocity copied. */
lbm_status lbm_init_fields(lbm_ctx *ctx, const double *phi, const double *u, const double *p_star);

/* Enqueues n >= 1 coupled time steps: per step the phase-field sweep
 * (pull-stream h, phi = sum h, gradient and normal of the previous phi,
 * forcing, collision) then the hydrodynamic sweep (pull-stream g, moments,
 * forces from the new phi, velocity update, moment-space collision), then a
 * buffer swap.  Both sweeps store post-collision populations at their own
 * cell and pull from the neighbours in the next sweep, which streams the
 * same values the paper's push of g does (Sec. 4.2).  With n >= 2 the
 * hydrodynamic sweep of each step and the phase-field sweep of the next run
 * as one kernel (same numbers).  Asynchronous. */
lbm_status lbm_step(lbm_ctx *ctx, int32_t n);

/* Same work as lbm_step(ctx, n), with a HIP event recorded on the context
 * stream before and after every sweep; waits for the stream and writes the
 * mean duration of one phase-field sweep and of one hydrodynamic sweep in
 * milliseconds (host outputs).  1 <= n <= 4096.  For measurement only. */
lbm_status lbm_step_timed(lbm_ctx *ctx, int32_t n, double *phase_ms, double *hydro_ms);

/* Measurement only: n (2..4096) steps exactly as lbm_step runs them with the
 * fused kernel (one phase-field sweep, n - 1 fused kernels, one
 * hydrodynamic sweep), with HIP events around every fused launch; the mean
 * fused-kernel time in ms (host output); synchronises.  LBM_EARG for 16-bit
 * storage and the z-marching sweeps, which have no fused kernel. */
lbm_status lbm_step_timed_fused(lbm_ctx *ctx, int32_t n, double *fused_ms);

/* Enqueues n >= 1 time steps of the straightforward algorithm (Alg.
 * naiveAlgorithm, Sec. 4.2) in place of the improved one: per step six
 * kernels, each a pass over the grid -- stream h, phi = sum h (eq.
 * updatePhaseField), stream g, velocity update (eq. updateVelocityField),
 * collision of h, collision of g -- so every population set is read three
 * times per step.  Time-consistent: both collisions take phi, its gradient
 * and u of the new time (the improved step takes the phase field's gradient
 * and u of the previous one in its phase-field collision); the velocity
 * update keeps the stored velocity inside the viscous force, and the
 * collision of g recomputes the force with the updated velocity.  Starts
 * from and leaves the same kind of state as lbm_step (populations
 * post-collision at their cell), so the getters, reductions and lbm_step
 * apply unchanged.  FP64 and FP32 storage only (LBM_EARG otherwise).
 * Asynchronous.  An ablation of the kernel fusion of Sec. 4.2. */
lbm_status lbm_step_straightforward(lbm_ctx *ctx, int32_t n);

/* sum of phi over fluid cells in FP64 (host output); synchronises. */
lbm_status lbm_reduce_mass(lbm_ctx *ctx, double *sum_phi);

/* All diagnostics of lbm_stats (host output); synchronises. */
lbm_status lbm_reduce_stats(lbm_ctx *ctx, lbm_stats *out);

/* Macroscopic fields into caller device arrays of element type dtype
 * (lbm_dtype): phi (1 plane), u (3 planes), p = p* rho c_s^2 (1 plane).  Any
 * pointer may be NULL. */
lbm_status lbm_get_macroscopic(lbm_ctx *ctx, int32_t dtype, void *phi, void *u, void *p);

/* Replaces the state by the equilibrium state of the given macroscopic
 * fields (same rule as lbm_init_fields, with p* = p/(rho c_s^2)). */
lbm_status lbm_set_macroscopic(lbm_ctx *ctx, int32_t dtype, const void *phi, const void *u,
                               const void *p);

/* Moves the state to the given macroscopic fields (device arrays as in
 * lbm_set_macroscopic) while keeping every population's non-equilibrium
 * part: each population gains the change of its equilibrium (the
 * equilibria of Section 3: h^eq = phi Gamma(u), g^eq(p*, u)),
 *   H_i += phi' Gamma_i(u') - phi Gamma_i(u),
 *   G_i += g^eq_i(p*', u') - g^eq_i(p*, u)   (canonical pre-collision G),
 * where phi, u are the current fields, p* = sum_i G_i the current
 * normalised pressure and p*' = p'/(rho(phi') c_s^2).  Unlike
 * lbm_set_macroscopic, the viscous stress and the interface flux carried by
 * the populations survive, so no start-up transient follows.  Wall cells
 * are unchanged.  Requires an initialised state; asynchronous. */
lbm_status lbm_shift_equilibrium(lbm_ctx *ctx, int32_t dtype, const void *phi, const void *u,
                                 const void *p);

/* Canonical state as FP64 device arrays, independent of the storage format:
 * H = post-collision phase-field PDFs (15 planes, not yet streamed),
 * G = pre-collision hydrodynamic PDFs (27 planes, already streamed).  The
 * phase field and velocity come from lbm_get_macroscopic.  Either pointer
 * may be NULL. */
lbm_status lbm_get_pdfs(lbm_ctx *ctx, double *H, double *G);

/* Loads a canonical state (FP64 device arrays as in lbm_get_pdfs, plus the
 * phase field and velocity); rounds to the storage format. */
lbm_status lbm_set_pdfs(lbm_ctx *ctx, const double *H, const double *G, const double *phi,
                        const double *u);

/* Bytes of one saved state: the current PDFs in storage format, the phase
 * field and the velocity. */
size_t lbm_state_bytes(const lbm_ctx *ctx);

/* Copies the current state into `dst` (device, lbm_state_bytes(ctx) bytes,
 * 256-byte aligned); asynchronous. */
lbm_status lbm_save_state(lbm_ctx *ctx, void *dst);

/* Makes a state saved by lbm_save_state from a context with the same
 * parameters the current state; asynchronous. */
lbm_status lbm_restore_state(lbm_ctx *ctx, const void *src);

/* STREAM-copy probe a_i = b_i over `bytes` bytes (multiple of 16) between
 * two device buffers on `hip_stream`; measures the copy bandwidth b_s used
 * by the paper's roofline P_max = b_s / n_b (Sec. 5.1). */
lbm_status lbm_stream_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

/* Number of completed steps since the last init / set call. */
int64_t lbm_steps_done(const lbm_ctx *ctx);

/* Releases the context (not the workspace). */
void lbm_destroy(lbm_ctx *ctx);

/* Text of the last error on the calling thread ("" if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
