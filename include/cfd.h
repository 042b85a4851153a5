/*
 * libcfd - FP64 finite-volume right-hand side of the compressible
 * Navier-Stokes equations on a structured Cartesian grid, hand-written HIP
 * for gfx950 (MI355X). C ABI, C99 header.
 *
 * The method is the "HLLC" setup of Bezgin, Buhendwa & Adams, JAX-FLUIDS
 * (arXiv:2203.13760): WENO5-JS reconstruction of the primitive variables,
 * HLLC Riemann flux with Einfeldt signal speeds per axis (§3.3), fourth-order
 * central viscous and heat fluxes (§3.4), the finite-volume flux divergence
 * (§3.1, Eq. FVD), and TVD-RK3 time integration with a CFL time step (§3.2).
 *
 * Conventions shared by every entry point
 *  - State layout (§2, §4.1): a state U holds the conservative variables
 *    (rho, rho*u, rho*v, rho*w, E) as 5 contiguous FP64 blocks; each block is
 *    [Z][Y][X] with x fastest, where an active axis of n cells is padded with
 *    nh halo cells on each side and an inactive axis (n == 1) has extent 1.
 *    cfd_state_numel() gives the element count. Interior cell (i,j,k) of
 *    variable v lives at v*Nz*Ny*Nx + (k+hz)*Ny*Nx + (j+hy)*Nx + (i+hx).
 *  - Memory: every array argument is device memory owned by the caller,
 *    FP64 and contiguous unless stated. The solver owns only its scratch.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream). Every call only enqueues work on that stream and returns; none
 *    synchronises except cfd_create, cfd_destroy and cfd_check. A solver
 *    handle must be used from one stream at a time.
 *  - Errors: every function returns cfd_status and never throws; on failure
 *    cfd_last_error() returns a message (thread-local).
 */
#ifndef LIBCFD_CFD_H
#define LIBCFD_CFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CFD_OK = 0,
  CFD_EINVAL = -1,      /* invalid argument or configuration */
  CFD_ENOMEM = -2,      /* device allocation failed */
  CFD_EHIP = -3,        /* a HIP runtime call failed */
  CFD_ENONFINITE = -4,  /* reserved: reported through cfd_check */
  CFD_EUNSUPPORTED = -5 /* valid request that this build does not implement */
} cfd_status;

/* Boundary types (§3.7): periodic (in pairs) and zero gradient, the paper's
 * "neumann" without a value; and the reflecting (slip) wall at which the
 * implosion of §7.4 reflects its shock: the halo mirrors the interior about
 * the boundary face with the wall-normal momentum negated. */
typedef enum { CFD_BC_PERIODIC = 0, CFD_BC_ZERO_GRADIENT = 1, CFD_BC_REFLECT = 2 } cfd_bc;

/* Physics switches, after the paper's is_inviscid_flux / is_viscous_flux /
 * is_heat_flux (Appendix A), and the convective scheme. By default the
 * high-order Godunov approach of §3.3 with WENO5-JS on the primitives and
 * HLLC (the paper's HLLC setup, §5); CFD_F_WENOZ reconstructs with WENO5-Z
 * instead (Borges et al. 2008; listed beside WENO5-JS in the paper's table of
 * methods, §3.3). CFD_F_ROE selects the flux-splitting approach of §3.3 with
 * the paper's ROE setup (§5): Roe-averaged eigen-decomposition at each face,
 * the stencil's states and fluxes projected on its characteristic fields,
 * split with the moduli of the Roe eigenvalues (no entropy fix), WENO5-JS per
 * field, transformed back. The implosion of §7.4 adds CFD_F_WENO3 (WENO3-JS
 * reconstruction of the primitives), CFD_F_RUSANOV (the Rusanov flux
 * (F_L + F_R)/2 - alpha (U_R - U_L)/2, alpha the largest |u -+ c| of the two
 * states, in place of HLLC) and CFD_F_RK2 (TVD-RK2 steps in place of TVD-RK3).
 * CFD_F_RUSANOV_NN selects the Rusanov-NN flux of §7.4: the Rusanov form
 * with alpha = exp(NN(|u_R - u_L|, (u_L + u_R)/2, (c_L + c_R)/2, |s_R - s_L|)),
 * u normal to the face, c the speed of sound, s = (ln p - gamma ln rho)/
 * (gamma - 1), NN a perceptron with three hidden ReLU layers of 32 units whose
 * weights cfd_set_nn_weights supplies; it needs CFD_F_WENO3.
 * CFD_F_ROE combines with none of WENOZ, WENO3, RUSANOV, and CFD_F_WENOZ with
 * neither WENO3 nor RUSANOV; CFD_F_RUSANOV_NN with none of ROE, WENOZ,
 * RUSANOV (CFD_EINVAL). CFD_F_SAFE_RECON is the safe reconstruction the
 * paper's setup file switches on (Appendix A, is_safe_reconstruction; not
 * defined in the paper; reading): at a face where a reconstructed state has
 * rho <= 0 or p <= 0, both states take the values of the two cells next to the
 * face (first order); not with ROE (CFD_EINVAL). Without the flag such faces
 * keep their states (the Riemann solver's sound speed is then undefined);
 * either way cfd_check reports them. The adjoint covers the default scheme
 * and WENO3-JS with the Rusanov-NN flux (inviscid), each with TVD-RK3 or
 * TVD-RK2, without safe reconstruction; the serving batch the default scheme
 * with any boundaries. */
enum {
  CFD_F_INVISCID = 1u, CFD_F_VISCOUS = 2u, CFD_F_HEAT = 4u, CFD_F_WENOZ = 8u, CFD_F_ROE = 16u, CFD_F_WENO3 = 32u,
  CFD_F_RUSANOV = 64u, CFD_F_RK2 = 128u, CFD_F_RUSANOV_NN = 256u, CFD_F_SAFE_RECON = 512u
};

/* Number of Rusanov-NN weights: W1 (32 x 4, row-major), b1 (32), W2 (32 x 32),
 * b2, W3 (32 x 32), b3, W4 (1 x 32), b4 (1); a layer maps h -> W h + b. */
#define CFD_NN_PARAMS 2305

typedef struct {
  int32_t n[3];      /* interior cells (x,y,z); n[d] == 1 marks an inactive axis */
  int32_t nh;        /* halo width on active axes; >= 3 (WENO5 and the C4 stencils) */
  double lo[3];      /* box lower corner */
  double hi[3];      /* box upper corner; dx_d = (hi_d - lo_d)/n_d */
  double gamma;      /* ratio of specific heats, > 1 (ideal gas, §2 with B = 0) */
  double mu;         /* dynamic viscosity, >= 0, constant (§2) */
  double prandtl;    /* > 0; heat conductivity = mu c_p / Pr */
  double cfl;        /* CFL number in (0, 1] (§3.2) */
  int32_t bc[6];     /* x-, x+, y-, y+, z-, z+ (cfd_bc); periodic only in pairs */
  uint32_t flags;    /* CFD_F_* */
} cfd_config;

typedef struct cfd_solver cfd_solver; /* opaque; owns the stage buffers and scratch */

/* Validate `cfg` and allocate the solver on the current HIP device: two stage
 * states, three primitive buffers (one per stage input of a step), a
 * right-hand-side accumulator and a small device control block (the adjoint
 * entry points add their scratch on first use). Active axes need n >= nh.
 * Returns CFD_EINVAL (bad config), CFD_ENOMEM or CFD_EHIP. Synchronises. */
cfd_status cfd_create(const cfd_config* cfg, cfd_solver** out);

/* Free everything the solver owns. NULL is accepted. Synchronises. */
void cfd_destroy(cfd_solver* s);

/* Number of FP64 elements of one padded state (5 * Nz * Ny * Nx), or -1. */
int64_t cfd_state_numel(const cfd_solver* s);

/* Conservative state from primitive point values (§2): W holds
 * (rho, u, v, w, p) as 5 blocks of interior cells [nz][ny][nx] (no halo);
 * U receives the padded conservative state with its halos filled. */
cfd_status cfd_state_init(cfd_solver* s, const double* W, double* U, void* stream);

/* Discrete adjoint of cfd_state_init (§2): with U = S(W) the padded state
 * cfd_state_init makes from W (halos filled), Wbar += (dS/dW)^T Ubar. Each
 * halo entry of Ubar is first added to the interior cell it is an image of
 * (the transpose of the halo fill; a reflecting wall's normal momentum with
 * its sign), in a fixed order, then the transposed primitive-to-conservative
 * map at W gives, per interior cell,
 *   rho_bar += Ubar_rho + u . Ubar_m + |u|^2/2 Ubar_E,
 *   u_bar_d += rho (Ubar_m_d + u_d Ubar_E),   p_bar += Ubar_E / (gamma - 1).
 * W and Wbar hold 5 blocks of interior cells [nz][ny][nx] (the layout of W in
 * cfd_state_init); Ubar is a padded state (device memory, not modified).
 * Wbar must not alias W or Ubar (CFD_EINVAL). The result is deterministic. */
cfd_status cfd_state_init_adjoint(cfd_solver* s, const double* W, const double* Ubar, double* Wbar, void* stream);

/* Refresh the halo cells of U in place from its interior, per the boundary
 * types (§3.7): periodic images, zero-gradient copies or mirror images with
 * the wall-normal momentum negated (reflecting walls), x then y then z. */
cfd_status cfd_fill_halo(cfd_solver* s, double* U, void* stream);

/* Right-hand side of the semi-discrete scheme (§3.1, Eq. FVD):
 *   R_i = - sum_d (G_{i+1/2} - G_{i-1/2}) / dx_d,  G = F - F^d,
 * F the WENO5-JS/HLLC convective flux (§3.3) and F^d the viscous and heat
 * flux (§3.4), per the physics flags. U's halos are refreshed in place. R is
 * a padded state; its halo entries are set to zero. */
cfd_status cfd_rhs(cfd_solver* s, double* U, double* R, void* stream);

/* CFL time step of state U (§3.2): dt = cfl / max over interior cells of
 * max(sum_d (|u_d| + c)/dx_d, 2 (mu/rho) max(4/3, gamma/Pr) sum_d dx_d^-2).
 * Writes one double to dt_dev (device memory). */
cfd_status cfd_compute_dt(cfd_solver* s, const double* U, double* dt_dev, void* stream);

/* One TVD-RK3 step (§3.2, Gottlieb & Shu):
 *   U1 = Un + dt R(Un);  U2 = 3/4 Un + 1/4 (U1 + dt R(U1));
 *   Un+1 = 1/3 Un + 2/3 (U2 + dt R(U2)),
 * in place on U (halos refreshed on return). dt > 0 fixes the step; dt <= 0
 * uses the CFL step of Un. dt_used_dev (device, nullable) receives the step. */
cfd_status cfd_rk3_step(cfd_solver* s, double* U, double dt, double* dt_used_dev, void* stream);

/* n_steps CFL steps (Algorithm 1's time loop) on U in place, with the time
 * kept on the device in *t_dev (device memory, read and updated). With
 * t_end > 0 the last step is clipped to end exactly at t_end, and steps
 * after that are device-side no-ops, so no host synchronisation is needed.
 * The step sequence is replayed from a captured HIP graph. */
cfd_status cfd_advance(cfd_solver* s, double* U, int32_t n_steps, double t_end, double* t_dev,
                       void* stream);

/* n_steps steps with a fixed dt (the paper's fixed-step rollout used for
 * differentiation, §4.5), graph-replayed like cfd_advance. */
cfd_status cfd_advance_fixed(cfd_solver* s, double* U, int32_t n_steps, double dt, void* stream);

/* Rusanov-NN weights (§7.4) of a solver created with CFD_F_RUSANOV_NN.
 * theta: device memory, CFD_NN_PARAMS doubles in the order of CFD_NN_PARAMS,
 * owned by the caller and read by every later launch of the solver (the
 * values may change between calls; the address must stay valid while the
 * solver may use it). theta_bar: device memory of CFD_NN_PARAMS doubles or
 * NULL; every later adjoint call (cfd_rhs_adjoint, cfd_rk3_step_adjoint,
 * cfd_rk3_step_adjoint_stages) adds its weight gradient to it (the caller
 * clears it). The sum over faces runs in a fixed order, so for a given Rbar
 * cfd_rhs_adjoint's weight gradient repeats bitwise; through a step it
 * inherits the last-bit variation of the state adjoint's atomics.
 * theta NULL unsets both. Solves with the flag and no weights fail with
 * CFD_EINVAL. CFD_EINVAL for a solver without the flag. Synchronises the
 * device when the solver holds a captured step (which it then discards). */
cfd_status cfd_set_nn_weights(cfd_solver* s, const double* theta, double* theta_bar);

/* Discrete adjoint of cfd_rhs: Ubar += (dR/dU)^T Rbar, evaluated at U
 * (interior cells of Rbar are read; its halo is ignored). The transposed halo
 * fill folds halo contributions back into their source cells, so the halo
 * entries of Ubar are left unchanged. U is not modified. With the Rusanov-NN
 * flux, the theta_bar of cfd_set_nn_weights (if any) receives
 * += (dR/dtheta)^T Rbar. CFD_EUNSUPPORTED for a scheme the adjoint does not
 * cover (see the physics switches). */
cfd_status cfd_rhs_adjoint(cfd_solver* s, const double* U, const double* Rbar, double* Ubar,
                           void* stream);

/* Discrete adjoint of one fixed-dt step (TVD-RK3, or TVD-RK2 with CFD_F_RK2):
 * with U^{n+1} = S(U^n), Ubar_n = (dS/dU^n)^T Ubar_np1 (interior cells;
 * Ubar_n's halo is zeroed); with the Rusanov-NN flux, theta_bar (see
 * cfd_set_nn_weights) += (dS/dtheta)^T Ubar_np1. The stage states are
 * recomputed from Un. Ubar_n must not alias the others. CFD_EUNSUPPORTED for
 * a scheme the adjoint does not cover. */
cfd_status cfd_rk3_step_adjoint(cfd_solver* s, const double* Un, double dt, const double* Ubar_np1,
                                double* Ubar_n, void* stream);

/* One fixed-dt TVD-RK3 step on U in place (§3.2; as cfd_rk3_step with dt > 0)
 * that also leaves its two stage states U1 = Un + dt R(Un) and
 * U2 = 3/4 Un + 1/4 (U1 + dt R(U1)) in U1_out and U2_out: caller-owned device
 * buffers of cfd_state_numel doubles, distinct from U and each other; their
 * interior cells are written, their halo entries are unspecified. For
 * checkpointed reverse passes that keep the stages of a recomputed segment
 * instead of recomputing them in every step adjoint. CFD_EUNSUPPORTED with
 * CFD_F_RK2. */
cfd_status cfd_rk3_step_stages(cfd_solver* s, double* U, double dt, double* U1_out, double* U2_out, void* stream);

/* cfd_rk3_step_adjoint with the stage states U1, U2 of the step from Un
 * supplied (as cfd_rk3_step_stages leaves them; interior cells are read)
 * instead of recomputed: the same result up to the summation order of the
 * atomics, without the two forward stages. Ubar_n must not alias any input.
 * CFD_EUNSUPPORTED with CFD_F_RK2 or a scheme the adjoint does not cover. */
cfd_status cfd_rk3_step_adjoint_stages(cfd_solver* s, const double* Un, const double* U1, const double* U2, double dt,
                                       const double* Ubar_np1, double* Ubar_n, void* stream);

/* One fixed-dt TVD-RK3 step on U in place (§3.2; as cfd_rk3_step with dt > 0)
 * that also leaves the primitive states of its three stage inputs Un, U1, U2
 * in P_out: a caller-owned device buffer of 3 * 6 * cfd_state_numel / 5
 * doubles, not aliasing U, holding three primitive blocks (P of Un, U1, U2 in
 * turn) of six components (rho, u, v, w, p, T~; component stride the padded
 * cell count) each. rho, u, v, w, p are written at every padded cell (halos
 * through the boundary map); T~ is written for Un only. These are everything
 * cfd_rk3_step_adjoint_prims needs: the stage passes write the primitives of
 * their outputs anyway, so keeping them costs no extra pass. For checkpointed
 * reverse passes (§4.5) that keep a recomputed segment. CFD_EUNSUPPORTED with
 * CFD_F_RK2. */
cfd_status cfd_rk3_step_prims(cfd_solver* s, double* U, double dt, double* P_out, void* stream);

/* cfd_rk3_step_adjoint of the step whose stage primitives P (as
 * cfd_rk3_step_prims leaves them) are supplied: Ubar_n = (dU^{n+1}/dU^n)^T
 * Ubar_np1 (interior cells; halo entries zero), the same result as
 * cfd_rk3_step_adjoint up to the summation order of the atomics, without the
 * forward stages and without primitive passes. Ubar_n must not alias P or
 * Ubar_np1. CFD_EUNSUPPORTED with CFD_F_RK2 or a scheme the adjoint does not
 * cover. */
cfd_status cfd_rk3_step_adjoint_prims(cfd_solver* s, const double* P, double dt, const double* Ubar_np1,
                                      double* Ubar_n, void* stream);

/* Measurement aid: enqueue the kernels of TVD-RK3 stages on U as a run of
 * steps runs them (stage r % 3 + 1 in repetition r, with dt = 1e-12, written to
 * solver scratch, so U is not modified; the third stage also forms the CFL
 * maxima and health bits of its output): the primitive pass, the x/y/z sweeps
 * (the last one also storing the primitives of the updated cells), and the
 * halo refresh of those primitives. Runs them `reps` times (1..4096) back to
 * back, each kernel bracketed by HIP events on `stream`, synchronises once,
 * and writes the average duration in milliseconds of each kernel to
 * ms_out[0..4] in that order (0 for sweeps the configuration does not launch).
 * Within a run of steps the primitive pass runs once, before the first step. */
cfd_status cfd_profile_stage(cfd_solver* s, const double* U, int32_t reps, double* ms_out, void* stream);

/* Synchronise the solver's last stream use and report its health word since
 * the previous cfd_check (which clears it): bit 0 a non-finite conservative
 * value, bit 1 rho <= 0, bit 2 p <= 0, in a state a step started from or
 * produced (its stage states included); bit 3 a face whose reconstructed
 * state had rho <= 0 or p <= 0 (any step or right-hand side; the Roe flux
 * splitting reconstructs characteristic fields and reports none). */
cfd_status cfd_check(cfd_solver* s, int32_t* status_out);

/* Allocation-free TVD-RK3 step, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): cfd_rk3_step of U in place for the configuration cfg,
 * with no solver handle and no device allocation or free. Its scratch (CFL
 * slots, control block, two stage states, two right-hand-side accumulators and
 * three primitive buffers: 38 doubles per padded cell) is one static device
 * array of 112 MiB, allocated with the library on every device it runs on and
 * held until the process ends; the grid may have at most
 * CFD_NOALLOC_MAX_PADDED_CELLS padded cells (CFD_EINVAL otherwise, before any
 * device work). dt > 0 fixes the step, dt <= 0 takes the CFL step of U;
 * dt_used_dev (device, nullable) receives it. The results equal
 * cfd_rk3_step's bitwise. Every call on a device uses that device's one
 * array: calls that overlap on one device (other streams, other threads)
 * race and give undefined results. The Rusanov-NN flux is not taken
 * (CFD_EUNSUPPORTED). */
#define CFD_NOALLOC_MAX_PADDED_CELLS 386309
cfd_status cfd_rk3_step_noalloc(const cfd_config* cfg, double* U, double dt, double* dt_used_dev, void* stream);

/* Message of the last failure on this thread ("" if none). */
const char* cfd_last_error(void);

/* ---------------------------------------------------------------------------
 * Serving batch: many independent solves (mixed sizes, 2D and 3D, different
 * physics) resident on the device at once, advanced together. Each TVD-RK3
 * step is one replay of a captured HIP graph whose launches are persistent
 * kernels, one per phase of each stage (primitives, CFL step, y/z/x
 * sweeps, halo refresh of the next primitives), each covering the work of
 * the resident grids of its sub-batch (up to four, run as concurrent
 * branches) through a device descriptor table. Every grid keeps its own state, scratch
 * and CFL step, so its result does not depend on the other grids in the batch.
 * A batch is used from one stream at a time. */
typedef struct cfd_batch cfd_batch; /* opaque */

/* Create a batch for up to max_grids resident grids (<= 512) whose buffers are
 * carved from one device arena of arena_bytes. Synchronises. */
cfd_status cfd_batch_create(int32_t max_grids, int64_t arena_bytes, cfd_batch** out);

/* Free the batch and its arena. NULL is accepted. Synchronises. */
void cfd_batch_destroy(cfd_batch* b);

/* Arena bytes one grid of this configuration occupies (its admission cost). */
cfd_status cfd_batch_footprint(const cfd_config* cfg, int64_t* bytes);

/* Admit a grid: validate cfg, take a slot and arena space, and enqueue the
 * conservative initial state from W (device, 5 x interior primitives, as for
 * cfd_state_init). Returns CFD_ENOMEM, with nothing changed, when no slot or
 * arena space is free; the caller retries after removing finished grids.
 * CFD_EUNSUPPORTED for a WENO5-Z, ROE, WENO3, RUSANOV or RK2 configuration
 * (the batch runs the default scheme). */
cfd_status cfd_batch_add(cfd_batch* b, const cfd_config* cfg, const double* W, int32_t* slot_out, void* stream);

/* Retire a grid and free its slot and arena space. The caller must have
 * synchronised the stream after the last step that used the grid. */
cfd_status cfd_batch_remove(cfd_batch* b, int32_t slot);

/* Device pointer to a resident grid's padded state and its element count. */
cfd_status cfd_batch_state(cfd_batch* b, int32_t slot, double** U_out, int64_t* numel);

/* One CFL TVD-RK3 step of every resident grid (uploads the descriptor table
 * first when grids were added or removed since the last step). The step graph
 * leaves out the phases a sub-batch has no blocks in and sizes each launch to
 * its blocks; a pattern of phases and widths not met before is captured on
 * that step (a few milliseconds of host time) and kept, up to 16 patterns;
 * with 16 kept the next new pattern first synchronises `stream` and drops
 * them, so `stream` must not be under graph capture then. */
cfd_status cfd_batch_step(cfd_batch* b, void* stream);

/* Refresh the halo cells of a resident grid's state (for read-out). */
cfd_status cfd_batch_finish(cfd_batch* b, int32_t slot, void* stream);

/* Enqueue a device-to-device copy of a resident grid's padded state into dst
 * (caller-owned device memory of cfd_batch_state's element count). */
cfd_status cfd_batch_copy_state(cfd_batch* b, int32_t slot, double* dst, void* stream);

/* Number of resident grids, or -1 for NULL. */
int32_t cfd_batch_count(const cfd_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* LIBCFD_CFD_H */
