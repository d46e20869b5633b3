/*
 * oracle.h -- C ABI of the CPU oracle (test infrastructure only).
 *
 * A plain, slow FP64 implementation of one finite-volume right-hand side and
 * one SSP-RK3 step of the four-equation multi-phase multi-component model of
 * Collis, Bezgin, Mirjalili & Mani (arXiv 2504.14063).  Only the test-suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source with the GPU library.
 *
 * All arrays are host memory owned by the caller.  A state U is FP64,
 * structure-of-arrays [nv][nz][ny][nx] (interior cells only, x fastest) in
 * the order rhoY_1..rhoY_ns, rho*u_1..rho*u_dim, E   (Sec. 2.1).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int dim;            /* 1, 2 or 3 active directions (x, then y, then z) */
  int n[3];           /* interior cells per direction (1 for inactive)   */
  double dx[3];       /* cell widths [m]                                   */
  int bc_lo[3];       /* 0 periodic, 1 zero-gradient outflow, 2 reflective,
                         3 characteristic (see oracle_set_boundary_target) */
  int bc_hi[3];
} oracle_grid;

typedef struct {
  int n_species;      /* components, at most 8                             */
  int phase[8];       /* 0 liquid (p = 1), 1 gas (p = 2)                   */
  double cv[8];       /* C_v [J/kg/K]                                      */
  double gamma[8];    /* C_P / C_v                                         */
  double pinf[8];     /* stiffening pressure P_inf [Pa]                    */
  double b[8];        /* co-volume [m^3/kg]                                */
  double q[8];        /* reference energy [J/kg]                           */
  double molar_mass[8];
  double mu[8];       /* dynamic viscosity [Pa s]                          */
  double Sc[8];       /* Schmidt number                                    */
  double lambda[8];   /* heat conductivity of a liquid component [W/m/K]   */
} oracle_eos;

typedef struct {
  double cfl;
  int cdi;            /* interface regularization on/off                   */
  double eps_cdi;     /* interface length scale epsilon [m]                */
  double phi_min;     /* volume-fraction floor                             */
  double delta;       /* offset of the psi transform                       */
  double gamma_scale; /* Gamma = gamma_scale * max |u_d|                   */
  int diffusion;      /* phase-confined species diffusion on/off           */
  int positivity;     /* interpolation, flux and CDI limiters on/off       */
  int precision;      /* ignored by the oracle (always FP64)               */
  int weno;           /* 0 = WENO5-Z, 1 = WENO5-JS, 2 = TENO5, 3 = TENO6   */
  double weno_eps;
  int weno_p;
  int viscous;        /* viscous stress and heat conduction on/off         */
  double prandtl;     /* gas-phase Prandtl number                          */
  int basis;          /* interpolation basis: 0 = characteristic variables
                         of W = [T, Y, u, P] (the method); 1 = W = [rho Y,
                         u, P] component-wise (the five-equation model's
                         basis, the paper's negative control)            */
} oracle_opts;

/* Counters accumulated by a step (indices). */
enum {
  ORACLE_CNT_T = 0,         /* faces with a temperature fallback          */
  ORACLE_CNT_P = 1,         /* faces with a pressure fallback             */
  ORACLE_CNT_FALLBACK = 2,  /* faces using the first-order HLLC flux      */
  ORACLE_CNT_CDI_DROP = 3,  /* faces whose CDI flux was dropped           */
  ORACLE_CNT_UNRECOVERABLE = 4,
  ORACLE_CNT_FACES = 5,     /* faces evaluated                            */
  ORACLE_CNT_BAD_CELLS = 6, /* stage input cells that are not admissible
                               (Eqs. PositivityReqs1-2: a negative partial
                               density, rho <= 0, rho (e - q) <= 0,
                               1 - sum rhoY_c b_c <= 0, or NaN)          */
  ORACLE_NCNT = 7
};

/* Status of oracle_rhs and oracle_rk3_step: 0, or ORACLE_EINADMISSIBLE when
 * that call met an inadmissible stage input cell or a face whose first-order
 * fallback flux still fails the flux limiter's test (the step is still
 * completed; the counters say how often). */
enum { ORACLE_EINADMISSIBLE = -4 };

/* Face decision mask bits (one uint16 per face). */
enum {
  ORACLE_M_TL = 1, ORACLE_M_TR = 2, ORACLE_M_PL = 4, ORACLE_M_PR = 8,
  ORACLE_M_FALLBACK = 16, ORACLE_M_CDI_DROP = 32, ORACLE_M_UNRECOVERABLE = 64
};

void* oracle_create(const oracle_grid* g, const oracle_eos* e, const oracle_opts* o, int* status);
void oracle_destroy(void* h);

/* Initial state from phase volume fractions phi[2][cells] (phase 0 liquid,
 * 1 gas), intraphase mass fractions y[ns][cells], P, T [cells] and velocity
 * vel[dim][cells]:  rho_p = 1/sum y_c v_c(P,T),  rhoY_c = phi_p rho_p y_c,
 * E = sum rhoY_c e_c(P,T) + rho|u|^2/2.                                      */
int oracle_init_state(void* h, const double* phi, const double* y, const double* P,
                      const double* T, const double* vel, double* U);

/* dt = CFL / max(...) and Gamma from U (Sec. 3.4 and 3.2). */
int oracle_compute_dt(void* h, const double* U, double* dt, double* gamma);

/* L(U_k) of one stage: U_n and (rk0, rk1, rk2) enter only the limiter
 * pseudo-states.  mask (nullable) receives one uint16 per face, blocks per
 * direction d of size prod_k (n_k + [k==d]).  counters (nullable,
 * ORACLE_NCNT) are incremented.  Returns 0 or ORACLE_EINADMISSIBLE. */
int oracle_rhs(void* h, const double* Uk, const double* Un, double rk0, double rk1,
               double rk2, double dt, double gamma, double* L, uint16_t* mask,
               uint64_t* counters);

/* The flux limiter's pseudo-states of one stage (Sec. 3.3.2): L(U_k) as
 * oracle_rhs, and for every interior cell and active direction d the
 * pseudo-state at its low face (lo) and at its high face (hi), formed from
 * the face's final flux F as rk0 U_n + rk1 U_k + s lam (F - F_d(U_k)) with
 * lam = 2 D rk2 dt / dx_d, s = +1 at the low face and -1 at the high face,
 * F_d(U_k) the cell's physical convective flux along d.  lo, hi:
 * [dim][nv][cells].  F (nullable): the final face fluxes, directions in
 * order, each [nv][prod_k (n_k + [k==d])].  Returns as oracle_rhs. */
int oracle_pseudo_states(void* h, const double* Uk, const double* Un, double rk0, double rk1,
                         double rk2, double dt, double gamma, double* L, double* lo, double* hi,
                         double* F);

/* One SSP-RK3 step in place.  dt_in/gamma_in nullable (null: from U^n).
 * Returns 0 or ORACLE_EINADMISSIBLE (any of the three stages). */
int oracle_rk3_step(void* h, double* U, const double* dt_in, const double* gamma_in,
                    double* dt_out, double* gamma_out, uint16_t* masks, uint64_t* counters);

/* Complex-step directional derivative of one RK3 step at fixed dt, Gamma:
 * U_out = step(U), dU_out = d step(U)[dU] with every branch decided by the
 * unperturbed state (frozen decisions). */
int oracle_jvp_rk3_step(void* h, const double* U, const double* dU, double dt, double gamma,
                        double* U_out, double* dU_out);

/* Inflow cells held at fixed conserved values: after every stage of
 * oracle_rk3_step (and oracle_jvp_rk3_step, where their derivative is then
 * zero) the count distinct cells idx take the values U [nv][count] (Sec.
 * 4.2.4's water inlet; reading of the inflow boundary).  count 0 clears.
 * Returns -1 on an index out of range or repeated. */
int oracle_set_held(void* h, long count, const long* idx, const double* U);

/* Characteristic boundary (a reading of the Navier-Stokes characteristic
 * boundary conditions cited in Sec. 3.5): at the boundary face of side `side`
 * (0 low, 1 high) of direction d, the face state is built from the
 * characteristic variables of App. A linearized at the boundary cell; those
 * whose waves leave the domain take the cell's values, the entering ones the
 * cell's values moved by the factor sigma toward the target state (P, T,
 * Y[ns], vel[dim]); the face's flux is the convective flux of that state.
 * sigma = 0 (the default of every characteristic side): no entering wave;
 * sigma = 1: the target imposed (supersonic inflow).  Returns -1 on a bad
 * argument (side not characteristic, sigma outside [0, 1], T <= 0, Y
 * negative or not summing to 1, P + P_inf <= 0 for a component present). */
int oracle_set_boundary_target(void* h, int d, int side, double P, double T, const double* Y,
                               const double* vel, double sigma);

/* Complex-step directional derivative of one stage right-hand side: L and
 * dL = dL(U_k)/dU_k [dU_k] at fixed U_n, (rk0..2), dt, Gamma, every branch
 * decided by the unperturbed state. */
int oracle_jvp_rhs(void* h, const double* Uk, const double* dUk, const double* Un, double rk0,
                   double rk1, double rk2, double dt, double gamma, double* L, double* dL);

/* Threads the oracle's parallel loops use, and a setter (n >= 1). */
int oracle_num_threads(void);
void oracle_set_num_threads(int n);

/* Floating-point operations of one right-hand side of U (stage 1), counted
 * by a counting scalar type, single-threaded: out[0] cell quantities (over
 * out[5] padded cells), out[1..3] face fluxes of x, y, z, out[4] divergence. */
int oracle_count_ops(void* h, const double* U, double dt, double gamma, long* out8);

/* ---- pieces, for unit pins ---- */
/* Equilibrium of one cell state u[nv]: out = P, T, a, rho, beta, alpha, cT, z, e */
int oracle_cell_equilibrium(void* h, const double* u, double* out9);
/* Conserved state and sound speed from (P, T, Y[ns], vel[dim]). */
int oracle_state_from_PT(void* h, double P, double T, const double* Y, const double* vel,
                         double* u_out, double* a_out);
/* WENO5-JS and TENO5 face values from f[0..4], TENO6 from f[0..5]
 * (scheme variants). */
double oracle_weno5js(const double* f, double eps, int p);
double oracle_teno5(const double* f, double eps);
double oracle_teno6(const double* f, double eps, double* tau_out /* nullable: tau6 */);
/* Jiang-Shu indicator of the polynomial matching n (1..6) cell averages on
 * cells off..off+n-1 (target cell [-1/2, 1/2]); *face = its value at 1/2. */
double oracle_js_indicator(const double* f, int off, int n, double* face);

double oracle_weno5z(const double* f5, double eps, int p);
/* Mass-fraction limiter of one face side: Ys[ns] in/out against Ycell[ns].
 * Returns 0 (sum == 1), 1 (sum > 1 branch) or 2 (sum < 1 branch). */
int oracle_ylimit(int ns, double* Ys, const double* Ycell);
/* HLLC flux along x from two conserved states (dim-dependent layout). */
int oracle_hllc(void* h, const double* uL, const double* uR, double* F);
/* Physical convective flux along x of a conserved state. */
int oracle_euler_flux(void* h, const double* u, double* F);
int oracle_admissible(void* h, const double* u);
/* Per-cell auxiliaries: out = phi[2], psi[2], rho_p[2], hrho_p[2], mu_mix */
int oracle_cell_aux(void* h, const double* u, double* out9);
/* Wilke mixture viscosity of phase p at intraphase mass fractions y[ns]. */
double oracle_wilke(void* h, int p, const double* y);

#ifdef __cplusplus
}
#endif
#endif
