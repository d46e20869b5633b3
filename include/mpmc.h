/*
 * mpmc.h -- C ABI of the MI355X (gfx950) library for the finite-volume hot
 * path of the four-equation multi-phase multi-component model of Collis,
 * Bezgin, Mirjalili & Mani (arXiv 2504.14063): the right-hand side of
 * Eq. DiscreteGoverningEquations advanced by SSP-RK3 (Eq. SSPRK3).
 *
 * Conventions shared by every entry point
 *  - State U: FP64 device array, structure-of-arrays [nv][nz][ny][nx]
 *    (interior cells only, x fastest), nv = ns + dim + 1, in the order
 *    rhoY_1..rhoY_ns, rho u_1..rho u_dim, E  (conserved vector of Sec. 2.1;
 *    E is total energy per unit volume).
 *  - All state, right-hand-side, adjoint and mask buffers are DEVICE pointers
 *    owned by the caller; the context owns only the scratch it allocates in
 *    mpmc_init and frees in mpmc_free.
 *  - stream is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work; nothing synchronizes except mpmc_stats.  The adjoint
 *    entry points run part of their work on a second stream of the
 *    context's (default priority), forked from and joined back into
 *    `stream` by events, so to the caller all of it is ordered as work on
 *    `stream`.
 *  - Return value: MPMC_OK or a negative error code.  Argument errors are
 *    detected on the host before anything is enqueued.  Device-side trouble
 *    -- a stage input cell that is not admissible (Eqs. PositivityReqs1-2:
 *    a negative partial density, rho <= 0, rho (e - q) <= 0,
 *    1 - sum rhoY_c b_c <= 0, or NaN anywhere in its state) or a face whose
 *    first-order fallback flux still fails the flux limiter's test (Sec.
 *    3.3.2) -- is counted on the device and sets a failure flag.  The flag
 *    is reported, once, as MPMC_EINADMISSIBLE by the return of the first
 *    call on the context that enqueues work and returns after the kernel
 *    that set it has completed: the launching call itself when that kernel
 *    finished before the call returned, else a later one (its own work is
 *    enqueued normally).  The host reads the flag without synchronizing and
 *    clears it when it reports it; a later kernel that meets trouble sets it
 *    again.  mpmc_stats synchronizes and reports the totals.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef MPMC_H
#define MPMC_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpmc_ctx mpmc_ctx; /* opaque */

enum {
  MPMC_OK = 0,
  MPMC_EINVAL = -1,        /* bad argument                                 */
  MPMC_ENOMEM = -2,        /* device allocation failed                     */
  MPMC_EHIP = -3,          /* a HIP runtime call failed                    */
  MPMC_EINADMISSIBLE = -4, /* an inadmissible cell or unrecoverable face
                              was met (see the conventions above)          */
  MPMC_EUNSUPPORTED = -5   /* valid but not built (see mpmc_init)          */
};

enum { MPMC_BC_PERIODIC = 0, MPMC_BC_OUTFLOW = 1, MPMC_BC_REFLECT = 2, MPMC_BC_CHARACTERISTIC = 3 };

/* Structured grid (Sec. 3.1).  Inactive directions (d >= dim) must have
 * n[d] = 1.  At most 2^29 cells, and at most 2^29 faces normal to each
 * direction (the kernels address an array row with 32-bit byte offsets;
 * MPMC_EINVAL otherwise).  Boundaries: periodic wrap, zero-gradient outflow (copy of the
 * nearest interior cell), reflective mirror (wall-normal momentum negated),
 * or characteristic (non-reflecting in- and outflow, a reading of the
 * Navier-Stokes characteristic boundary conditions of Sec. 3.5; see
 * mpmc_set_boundary_target).  A reflective direction needs n >= 3. */
typedef struct {
  int dim;
  int n[3];
  double dx[3];
  int bc_lo[3];
  int bc_hi[3];
} mpmc_grid;

/* Component table: NASG parameters of Eq. NASG_EOS per component and its
 * phase (0 = liquid, the paper's p = 1; 1 = gas, p = 2), plus transport
 * data of Sec. 2.2 (viscosity, Schmidt number, molar mass).  When all
 * components with a non-zero P_inf share one value the pressure is the
 * closed form of Eq. NASG_P; with several distinct values it is found
 * iteratively (the temperatures of Eqs. NASG_T1 and NASG_T2 equated, the
 * largest root above -min P_inf of the components present), in FP64 forward
 * contexts only.  Up to 8 components; with more than 3 only the FP64 forward
 * is built (mpmc_init_state, mpmc_compute_dt, mpmc_rhs, mpmc_rk3_step; the
 * other entry points return MPMC_EUNSUPPORTED for such contexts). */
typedef struct {
  int n_species;           /* 1..8 (above 3: FP64 forward only)            */
  int phase[8];
  double cv[8];            /* C_v [J/(kg K)]                               */
  double gamma[8];         /* C_P / C_v                                    */
  double pinf[8];          /* P_inf [Pa]                                   */
  double b[8];             /* co-volume [m^3/kg]                           */
  double q[8];             /* reference energy [J/kg]                      */
  double molar_mass[8];    /* [kg/mol]                                     */
  double mu[8];            /* [Pa s]                                       */
  double Sc[8];
  double lambda[8];        /* heat conductivity of a liquid component
                              [W/(m K)] (Sec. 2.2.1: constant in the liquid
                              phase; the gas phase takes mu_g / Pr sum_c
                              (Y_c / Y_g) C_P,c)                            */
} mpmc_eos;

/* User parameters of the method. */
typedef struct {
  double cfl;          /* Sec. 3.4, 0 < cfl <= 1                            */
  int cdi;             /* interface regularization flux (Sec. 3.2) on/off   */
  double eps_cdi;      /* epsilon [m] (interface thickness)                 */
  double phi_min;      /* volume-fraction floor (paper: 1e-8)               */
  double delta;        /* offset of the psi transform (paper: 1e-100)       */
  double gamma_scale;  /* Gamma = gamma_scale * max |u_d|                   */
  int diffusion;       /* phase-confined species diffusion on/off           */
  int positivity;      /* interpolation, flux and CDI limiters (Sec. 3.3)   */
  int precision;       /* 0: FP64; 1: mixed (FP32 face pipeline, FP64
                          equilibrium, limiter tests and accumulation)      */
  int weno;            /* 0: WENO5-Z (the paper's default); the variants
                          cited beside it (Sec. 4, Table
                          DropAdvectionIECResults): 1 WENO5-JS, weights
                          d_k/(beta_k+eps)^p; 2 TENO5 (C = 1, q = 6,
                          C_T = 1e-5); 3 TENO6 (six-point, C_T = 1e-7).
                          Variants: FP64 forward only                     */
  double weno_eps;     /* epsilon of the weights (every scheme)            */
  int weno_p;          /* exponent p of WENO5-Z and WENO5-JS (1 or 2)      */
  int viscous;         /* viscous stress and heat conduction (Eq.
                          DiffusionTerms, second-order central) on/off;
                          the adjoint entry points reject it (unsupported) */
  double prandtl;      /* gas-phase Prandtl number (> 0 with viscous on)    */
  int basis;           /* interpolation basis: 0 characteristic variables of
                          W = [T, Y, u, P] (Sec. 3.1.2, the method); 1 the
                          five-equation model's W = [rho Y, u, P], one
                          variable at a time, face T from the equilibrium
                          (the negative control of Sec. 4.2.2, Table
                          DropAdvectionNoIECResults).  1: FP64 forward
                          only                                            */
  int step_layout;     /* execution layout of the RK steps, not a method
                          option; every layout gives the same bits.
                          1 split: the face sweeps write face flux arrays
                          and a separate pass combines them (the layout of
                          mpmc_rhs); 2 fused: each direction's sweep also
                          takes the divergence of its fluxes and the last
                          one the RK combination (no face flux arrays);
                          0 (default) the faster of the two on MI355X
                          (split)                                        */
} mpmc_opts;

/* Limiter activity (Sec. 3.3) accumulated since the last reset. */
typedef struct {
  uint64_t faces_T;        /* faces with a temperature fallback            */
  uint64_t faces_P;        /* faces with a pressure fallback               */
  uint64_t fallback;       /* faces using the first-order HLLC flux        */
  uint64_t cdi_drop;       /* faces whose regularization flux was dropped  */
  uint64_t unrecoverable;  /* faces whose fallback flux still fails        */
  uint64_t faces;          /* faces evaluated                              */
  uint64_t inadmissible_cells; /* stage input cells of the forward entry
                              points (mpmc_rhs, mpmc_rk3_step and its
                              variants) that are not admissible            */
} mpmc_stats_t;

/* Face decision bits in mask arrays (one uint16 per face). */
enum {
  MPMC_M_TL = 1, MPMC_M_TR = 2, MPMC_M_PL = 4, MPMC_M_PR = 8,
  MPMC_M_FALLBACK = 16, MPMC_M_CDI_DROP = 32, MPMC_M_UNRECOVERABLE = 64
};

/* Create a context for one grid, component table and option set; allocates
 * the device scratch (cell quantities, face fluxes, two stage states) on the
 * current device.  *out receives the context.  Errors: EINVAL (bad sizes or
 * options), EUNSUPPORTED (weno > 3, basis > 1, several distinct P_inf,
 * weno != 0 or basis != 0 with the mixed form; more than 3 components with
 * the mixed form or the fused step layout), ENOMEM. */
int mpmc_init(const mpmc_grid* grid, const mpmc_eos* eos, const mpmc_opts* opts,
              mpmc_ctx** out);

/* Free a context and its scratch (synchronizes the device). */
int mpmc_free(mpmc_ctx* ctx);

/* Number of uint16 entries of a mask array for one stage: the sum over the
 * active directions d of prod_k (n_k + [k == d]).  Faces of direction d are
 * indexed by the cell on their high side, 0..n_d. */
long mpmc_mask_size(const mpmc_ctx* ctx);

/* Conserved state from primitive fields (Sec. 2.2 mixing rules): per cell,
 * phase volume fractions phi[2][cells] (liquid, gas), intraphase mass
 * fractions y[ns][cells], P, T [cells], velocity vel[dim][cells] (all device
 * FP64): rho_p = 1 / sum_c y_c v_c(P,T), rhoY_c = phi_p rho_p y_c,
 * E = sum_c rhoY_c e_c(P,T) + rho |u|^2 / 2. */
int mpmc_init_state(mpmc_ctx* ctx, const double* phi, const double* y, const double* P,
                    const double* T, const double* vel, double* U, void* stream);

/* Time step and regularization velocity from a state (Sec. 3.4, Sec. 3.2):
 * dt = cfl / max over cells and directions of (|u_d| + a)/dx_d and, with
 * diffusion on, 4 mu/(rho dx_d^2); Gamma = gamma_scale * max |u_d|.
 * dt_dev, gamma_dev: device scalars written by the call. */
int mpmc_compute_dt(mpmc_ctx* ctx, const double* U, double* dt_dev, double* gamma_dev,
                    void* stream);

/* Right-hand side L(U_k) of Eq. DiscreteGoverningEquations for one RK
 * stage.  U_n and the stage coefficients (rk0, rk1, rk2) enter only the
 * limiter pseudo-states of Sec. 3.3.2; dt_dev and gamma_dev are device
 * scalars.  L_out: device [nv][cells].  mask_out (nullable): device uint16
 * [mpmc_mask_size]. */
int mpmc_rhs(mpmc_ctx* ctx, const double* U_k, const double* U_n, double rk0, double rk1,
             double rk2, const double* dt_dev, const double* gamma_dev, double* L_out,
             uint16_t* mask_out, void* stream);

/* One SSP-RK3 step (Eq. SSPRK3) of U in place.  dt_in_dev / gamma_in_dev:
 * nullable device scalars; NULL means "computed from U^n" (as
 * mpmc_compute_dt), non-NULL freezes them (adjoint, finite differences).
 * dt_out_dev / gamma_out_dev: nullable device scalars receiving the values
 * used.  masks_out (nullable): device uint16 [3][mpmc_mask_size], the face
 * decisions of the three stages. */
int mpmc_rk3_step(mpmc_ctx* ctx, double* U, const double* dt_in_dev,
                  const double* gamma_in_dev, double* dt_out_dev, double* gamma_out_dev,
                  uint16_t* masks_out, void* stream);

/* Frozen-decision forward step: as mpmc_rk3_step at the given dt and Gamma,
 * with the limiter decisions of Sec. 3.3 (T/P fallback, first-order flux,
 * dropped regularization flux) of the three stages read from masks_in
 * (device uint16 [3][mpmc_mask_size], as written by mpmc_rk3_step's
 * masks_out) instead of tested.  The map this step computes is the one
 * mpmc_adjoint_step differentiates; it serves finite-difference checks of
 * the adjoint.  FP64 contexts with at most 3 components, WENO5-Z, the
 * characteristic basis and one distinct P_inf only (MPMC_EUNSUPPORTED
 * otherwise). */
int mpmc_rk3_step_replay(mpmc_ctx* ctx, double* U, const double* dt_dev, const double* gamma_dev,
                         const uint16_t* masks_in, void* stream);

/* One SSP-RK3 step (Eq. SSPRK3) of U in place at the given dt and Gamma,
 * exactly as mpmc_rk3_step with dt_in_dev / gamma_in_dev set, that also hands
 * back what its adjoint needs: stage1_out, stage2_out (device [nv][cells],
 * caller-owned) receive the intermediate states U1 = U^n + dt L(U^n) and
 * U2 = 3/4 U^n + 1/4 (U1 + dt L(U1)); masks_out (device uint16
 * [3][mpmc_mask_size]) the face decisions of Sec. 3.3 of the three stages.
 * Together with U^n they are the record that mpmc_adjoint_step_stages takes
 * in place of recomputing the step (the stage states and masks stored per
 * step of a checkpoint segment).  stage1_out, stage2_out and U must be three
 * distinct buffers (MPMC_EINVAL otherwise).  FP64 contexts with at most 3
 * components only (MPMC_EUNSUPPORTED otherwise). */
int mpmc_rk3_step_stages(mpmc_ctx* ctx, double* U, const double* dt_dev, const double* gamma_dev,
                         double* stage1_out, double* stage2_out, uint16_t* masks_out, void* stream);

/* Target of a characteristic boundary (MPMC_BC_CHARACTERISTIC) on side
 * `side` (0 low, 1 high) of direction d.  Sec. 3.5 uses the Navier-Stokes
 * characteristic boundary conditions of Thompson and of Poinsot & Lele for
 * non-reflecting inflow and outflow without giving formulas; reading: the
 * face state of the boundary face is built in the characteristic variables
 * of App. A linearized at the boundary cell (T - cT P, Y_c, u_t with speed
 * u_n; P/2 + (z/2) u_n with u_n + a; P/2 - (z/2) u_n with u_n - a).  Where a
 * wave leaves the domain the variable keeps the cell's value; where it
 * enters, the cell's value moves by the factor sigma toward the value of the
 * target state (P [Pa], T [K], mass fractions Y[ns], velocity vel[dim]):
 * sigma = 0 lets no wave enter (non-reflecting), sigma = 1 imposes the target
 * (e.g. a supersonic inflow), values between relax toward it.  The face's
 * flux is the convective flux of that state; no regularization, diffusion
 * or viscous flux crosses a characteristic boundary, and the limiters of
 * Sec. 3.3 are not applied to it (mask 0).  Every characteristic side starts
 * at sigma = 0.  Y, vel: host arrays, copied.  Errors: EINVAL (side not
 * characteristic, sigma outside [0, 1], T <= 0, non-finite values, Y negative
 * or not summing to 1 within 1e-12, P + P_inf <= 0 for a component with
 * Y > 0).  The adjoint entry points return MPMC_EUNSUPPORTED for a context
 * with a characteristic boundary. */
int mpmc_set_boundary_target(mpmc_ctx* ctx, int dir, int side, double P, double T, const double* Y,
                             const double* vel, double sigma);

/* Inflow cells held at fixed conserved values (the water inlet of the
 * Mach-100 water column, Sec. 4.2.4, Table Mach100WaterColumnSetup: the
 * paper's non-reflecting NSCBC inflow of Sec. 3.5 is defined only in its
 * references; here an inflow is a set of cells, typically the first cells
 * inside a zero-gradient boundary, whose state is prescribed).  After the
 * update of every RK stage of mpmc_rk3_step, mpmc_rk3_step_replay and
 * mpmc_rk3_step_stages, the cells idx[0..count) take the values
 * values[v * count + k] (variable-major [nv][count], the conserved variables
 * of Sec. 2.1); the stage right-hand side mpmc_rhs is not affected.
 * idx, values: host arrays, copied (the caller keeps ownership); the indices
 * must be distinct and in [0, cells), the values finite with non-negative
 * partial densities (MPMC_EINVAL otherwise; the previous set is then kept).
 * count = 0 clears (idx, values may then be NULL).  The call synchronizes the
 * device and allocates count (nv + 1) * 8 bytes.  While cells are held the
 * adjoint entry points return MPMC_EUNSUPPORTED. */
int mpmc_set_held_cells(mpmc_ctx* ctx, long count, const long* idx, const double* values);

/* Discrete adjoint of one mpmc_rk3_step (Eq. SSPRK3) at fixed dt and Gamma:
 * lam_n = (d U^{n+1} / d U^n)^T lam_np1, with every decision frozen as the
 * forward step from U_n takes it (limiter masks of Sec. 3.3 recorded by a
 * recompute of the three stages, Y-limiter branch, min/max/abs arms).  The
 * WENO-Z weights are differentiated.  Conventions where rounding decides:
 *  - a WENO-Z substencil flat to round-off (differences within 1e-7 of the
 *    stencil's largest magnitude) has smoothness indicator eps without
 *    derivative (all three flat: ideal weights);
 *  - a Y-limiter correction with |1 - sum| <= 1e-13 is not differentiated, nor
 *    a component whose |Y_face - Y_cell| <= 1e-10;
 *  - HLLC: a wave-speed arm within 1e-9 of the speed scale of a tie takes the
 *    averaged-state speed; s* within 1e-9 of zero takes the mean of the two
 *    star fluxes;
 *  - an absent phase (phi == 0 exactly) contributes no derivative of the
 *    interface transform psi.
 * The pull-back writes one record per face and then gathers per cell in a
 * fixed order (no floating-point atomics): the result is bitwise
 * reproducible.  dt_dev, gamma_dev: device scalars.  U_n, lam_np1, lam_n:
 * device [nv][cells]; lam_n may alias neither.  The first call allocates the
 * adjoint scratch: R doubles per face of every direction (rounded up to
 * whole tiles of 64 faces), R = 6 (2 + ns + dim) + 2 (5 + ns) + 4 ns + 3 + nv
 * + dim - 1; the hand-over between the face pull-back's two halves,
 * 9 + 2 ns + 2 (dim - 1) doubles per face of the largest direction and again
 * of the y direction (whose pull-back runs on a second stream of the
 * library's, beside the others); 2 nv doubles per cell; 3 masks.  FP64
 * contexts with at most 3 components, WENO5-Z, the characteristic basis, one
 * distinct P_inf, without viscous terms and without held cells only
 * (MPMC_EUNSUPPORTED otherwise). */
int mpmc_adjoint_step(mpmc_ctx* ctx, const double* U_n, const double* dt_dev,
                      const double* gamma_dev, const double* lam_np1, double* lam_n,
                      void* stream);

/* mpmc_adjoint_step from a recorded step: stage1, stage2 and masks are what
 * mpmc_rk3_step_stages wrote for the step from U_n at the same dt_dev and
 * gamma_dev (Eq. SSPRK3); no stage is recomputed, only the cell quantities of
 * each stage state.  Same result and derivative conventions as
 * mpmc_adjoint_step (which records the same decisions by recomputing the
 * step).  All arrays are device memory owned by the caller; lam_n may alias
 * none of the inputs (MPMC_EINVAL).  Adjoint scratch and FP64 restriction as
 * for mpmc_adjoint_step. */
int mpmc_adjoint_step_stages(mpmc_ctx* ctx, const double* U_n, const double* stage1,
                             const double* stage2, const uint16_t* masks, const double* dt_dev,
                             const double* gamma_dev, const double* lam_np1, double* lam_n,
                             void* stream);

/* Adjoint of mpmc_rhs (Eq. DiscreteGoverningEquations): Ubar = (dL(U_k)/dU_k)^T Lbar
 * with U^n, the stage coefficients, dt and Gamma held fixed and every decision
 * frozen: the limiter decisions are read from mask, the face-decision mask
 * that mpmc_rhs wrote for the same (U_k, U^n, rk, dt, Gamma) (device uint16
 * [mpmc_mask_size]); min/max/abs arms are recomputed from U_k.  Derivative
 * conventions as for mpmc_adjoint_step.  Uk, Lbar, Ubar: device [nv][cells];
 * Ubar is overwritten and may alias neither Uk nor Lbar.  FP64 contexts
 * with at most 3 components, WENO5-Z, the characteristic basis, one distinct
 * P_inf, without viscous terms and without held cells only
 * (MPMC_EUNSUPPORTED otherwise). */
int mpmc_rhs_vjp(mpmc_ctx* ctx, const double* Uk, const uint16_t* mask, const double* dt_dev,
                 const double* gamma_dev, const double* Lbar, double* Ubar, void* stream);

/* Per-variable sums over all cells in a fixed order (conservation checks):
 * sums_dev device [nv]. */
int mpmc_conserve_sum(mpmc_ctx* ctx, const double* U, double* sums_dev, void* stream);

/* mpmc_conserve_sum for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sums, bit for bit, with the per-block partial sums kept in a fixed scratch
 * array of the library (1024 blocks x 8 variables of FP64, 64 KiB, one per
 * device, held until the process ends) instead of context memory.  The call
 * allocates nothing.  Limits: nv <= 8 (MPMC_EINVAL otherwise).  Every call on
 * one device shares that device's array: calls that overlap on one device
 * (several streams or contexts without ordering between them) race and may
 * return wrong sums; calls ordered on a stream do not (each call rewrites
 * every partial it reads).  U, sums_dev: device, as for
 * mpmc_conserve_sum. */
int mpmc_conserve_sum_static(mpmc_ctx* ctx, const double* U, double* sums_dev, void* stream);

/* Copy the limiter and failure counters to *out (synchronizes the
 * context's last stream); reset != 0 clears them and the failure flag
 * afterwards.  Returns MPMC_EINADMISSIBLE if an unrecoverable face or an
 * inadmissible cell was counted, else MPMC_OK. */
int mpmc_stats(mpmc_ctx* ctx, mpmc_stats_t* out, int reset);

/* Kernel timing for measurement: when enabled, every kernel the context
 * launches is bracketed by HIP events on its stream.  Classes: 0 cell
 * equilibrium, 1..3 face fluxes along x, y, z, 4 divergence + RK update,
 * 5 reductions and small kernels, 6 adjoint.  mpmc_profile_read synchronizes
 * the last stream and returns, per class, the summed kernel time [ms] and
 * the number of launches (arrays of 8); reset != 0 clears them. */
int mpmc_profile(mpmc_ctx* ctx, int enable);
int mpmc_profile_read(mpmc_ctx* ctx, double* ms, long* launches, int reset);

const char* mpmc_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
