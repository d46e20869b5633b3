// oracle.cpp -- CPU oracle for the four-equation multi-phase multi-component
// finite-volume step (Collis, Bezgin, Mirjalili & Mani, arXiv 2504.14063).
//
// TEST INFRASTRUCTURE ONLY.  Plain loops, FP64, explicit ghost layers, no
// blocking or fusion: every function follows one passage of the paper and
// says which.  It is templated on the scalar type so that the same source
// also runs with std::complex<double> for complex-step derivatives; every
// branch is decided on the real part, which freezes the decisions of the
// unperturbed state.  Built with -ffp-contract=off.  The GPU library never
// includes, links or calls this file.
//
// Readings of passages that are garbled, ambiguous or silent are marked
// "reading:" and are listed in the design notes of the repository.
//
// Parity unpinned: the cut-off C_T of TENO6 (teno6).  Its substencils,
// weights and indicators are pinned; no case at hand tells C_T = 1e-7 from
// 1e-2 (the paper's droplet advection gives the same errors for every value
// in that range).

#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef std::complex<double> cplx;

inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }

template <class S> inline S vmin(const S& a, const S& b) { return re(b) < re(a) ? b : a; }
template <class S> inline S vmax(const S& a, const S& b) { return re(b) > re(a) ? b : a; }
template <class S> inline S vabs(const S& a) { return re(a) < 0.0 ? S(-a) : a; }
template <class S> inline double vsgn(const S& a) {
  return re(a) > 0.0 ? 1.0 : (re(a) < 0.0 ? -1.0 : 0.0);
}
using std::log;
using std::sqrt;
using std::tanh;

// Counting scalar: a double that counts the floating-point operations made on
// it (+ - * / sqrt log tanh, one each), used to state the algorithmic work
// per face and per cell.  Negation and comparisons are not counted.
struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}
};
long* g_ops = nullptr;
inline void tick() {
  if (g_ops) ++*g_ops;
}
inline double re(const Cnt& x) { return x.v; }
inline Cnt operator+(const Cnt& a, const Cnt& b) { tick(); return Cnt(a.v + b.v); }
inline Cnt operator-(const Cnt& a, const Cnt& b) { tick(); return Cnt(a.v - b.v); }
inline Cnt operator*(const Cnt& a, const Cnt& b) { tick(); return Cnt(a.v * b.v); }
inline Cnt operator/(const Cnt& a, const Cnt& b) { tick(); return Cnt(a.v / b.v); }
inline Cnt operator-(const Cnt& a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, const Cnt& b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, const Cnt& b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, const Cnt& b) { a = a * b; return a; }
inline Cnt sqrt(const Cnt& a) { tick(); return Cnt(std::sqrt(a.v)); }
inline Cnt log(const Cnt& a) { tick(); return Cnt(std::log(a.v)); }
inline Cnt tanh(const Cnt& a) { tick(); return Cnt(std::tanh(a.v)); }

// Operation buckets of the counting scalar (no-op for the other types).
long g_bucket[8];
template <class S> inline void bucket(int) {}
template <> inline void bucket<Cnt>(int b) { g_ops = b < 0 ? nullptr : &g_bucket[b]; }

// ---------------------------------------------------------------------------
// Configuration
// ---------------------------------------------------------------------------
struct Conf {
  // held inflow cells (reading of the inflow of Sec. 4.2.4): cell indices and
  // their conserved values, variable-major [nv][held.size()]
  std::vector<long> held;
  std::vector<double> held_U;
  // characteristic boundaries (reading of the NSCBC of Sec. 3.5): per
  // direction and side (0 low, 1 high) the target state (P, T, Y, u) and the
  // relaxation factor sigma of the incoming characteristic variables
  struct Target {
    double P = 0.0, T = 0.0, Y[8] = {0, 0, 0, 0, 0, 0, 0, 0}, vel[3] = {0, 0, 0}, sigma = 0.0;
  } target[3][2];
  int dim = 1;
  int n[3] = {1, 1, 1};
  double dx[3] = {1, 1, 1};
  int bclo[3] = {0, 0, 0}, bchi[3] = {0, 0, 0};
  int ns = 0;
  int ph[8];
  double cv[8], gam[8], pinf[8], b[8], q[8], W[8], mu[8], Sc[8], lamc[8];
  double Pst = 0.0;  // the single distinct non-zero P_inf (0 if none)
  int multi = 0;     // several distinct non-zero P_inf: iterative pressure
  int np = 0;        // phases present (1 or 2)
  int pid[2];        // phase id (0 liquid, 1 gas) of each present phase
  int pn[2];         // number of components in each present phase
  int pc[2][8];      // component indices of each present phase
  double cfl = 0.5;
  int cdi = 0;
  double eps = 0, phimin = 1e-8, delta = 1e-100, gscale = 1.0;
  int diffusion = 0, positivity = 1;
  int viscous = 0;
  int weno = 0;  // 0 WENO5-Z, 1 WENO5-JS, 2 TENO5, 3 TENO6
  int basis = 0;  // 0 characteristic [T, Y, u, P]; 1 component-wise [rho Y, u, P]
  double Pr = 0.71;
  double weps = 1e-40;
  int wp = 1;
  int nv = 0;
  int g[3] = {0, 0, 0};  // ghost layers per direction
  int N[3] = {1, 1, 1};  // padded extents
  long ncell = 0, npad = 0;

  long pidx(int i, int j, int k) const {  // padded index of interior coords
    return ((long)(k + g[2]) * N[1] + (j + g[1])) * N[0] + (i + g[0]);
  }
  long cidx(int i, int j, int k) const { return ((long)k * n[1] + j) * n[0] + i; }
};

// ---------------------------------------------------------------------------
// NASG equation of state of one component (Eq. NASG_EOS) written with
//   kappa_c(P) = (gamma_c - 1) C_v,c / (P + P_inf,c)     so v_c - b_c = kappa_c T
//   eps_c(P)   = C_v,c (P + gamma_c P_inf,c)/(P + P_inf,c) so e_c - q_c = eps_c T
// ---------------------------------------------------------------------------
template <class S> S kappa(const Conf& c, int k, const S& P) {
  return (c.gam[k] - 1.0) * c.cv[k] / (P + c.pinf[k]);
}
template <class S> S epsT(const Conf& c, int k, const S& P) {
  if (c.pinf[k] == 0.0) return S(c.cv[k]);  // ideal gas: (P+0)/(P+0) = 1
  return c.cv[k] * (P + c.gam[k] * c.pinf[k]) / (P + c.pinf[k]);
}
template <class S> S spec_vol(const Conf& c, int k, const S& P, const S& T) {
  return kappa(c, k, P) * T + c.b[k];
}
template <class S> S spec_energy(const Conf& c, int k, const S& P, const S& T) {
  return epsT(c, k, P) * T + c.q[k];
}
template <class S> S spec_enthalpy(const Conf& c, int k, const S& P, const S& T) {
  return c.gam[k] * c.cv[k] * T + c.b[k] * P + c.q[k];
}

// Equilibrium sound speed (Eq. SpeedOfSound with the NASG beta, alpha).
template <class S>
void sound(const Conf& c, const S& rho, const S* Y, const S& P, const S& T, S& a, S& beta,
           S& alpha) {
  S sb = 0.0, sa = 0.0, Cp = 0.0;
  for (int k = 0; k < c.ns; ++k) {
    S kp = kappa(c, k, P);
    sb += Y[k] * kp * T / (P + c.pinf[k]);
    sa += Y[k] * kp;
    Cp += Y[k] * (c.gam[k] * c.cv[k]);
  }
  beta = rho * sb;
  alpha = rho * sa;
  S a2 = Cp / (rho * beta * Cp - alpha * alpha * T);
  a = sqrt(a2);
}

// ---------------------------------------------------------------------------
// Pressure-temperature equilibrium of a conserved state (Sec. 2.3):
// closed form Eq. NASG_P, then T from Eq. NASG_T1.
// reading: R1 = sum over stiffened components of Y (C_P - C_v), Rg = the same
// over ideal-gas components, computed directly (not as C_P - C_v - R1);
// a2 < 0 uses the cancellation-free form 2 a3/(sqrt(D) - a2) of the same root;
// with no gas (Rg == 0) the quadratic degenerates to P = a2/a1.
// ---------------------------------------------------------------------------
template <class S> struct Thermo {
  S rho, Y[8], vel[3], e, P, T, a, beta, alpha, cT, z;
};

// ---------------------------------------------------------------------------
// Pressure of the general mixture (several distinct P_inf; Sec. 2.3: the two
// temperatures of Eqs. NASG_T1 and NASG_T2 equal, solved iteratively).
// Written out, T1 = T2 is
//   F(P) = (v - b) C_v - sum_c A_c / (P + P_inf,c) = 0,
//   A_c = Y_c (gamma_c - 1) C_v,c (e - q - (v - b) P_inf,c).
// reading: the pressure is the largest root above P_lo = max over components
// present of -P_inf,c (the closed form of the single-P_inf case is the larger
// root of its quadratic).  Found by scanning down from a point above which F
// stays positive (sum |A_c| / (P + P_inf,c) < C/2 there), in steps of 10 % of
// the distance to P_lo, to the first negative F, then bisection to round-off.
// The tangent of a complex-step argument follows from one Newton step in S at
// the real root (implicit function theorem).
// ---------------------------------------------------------------------------
template <class S> S pressure_general(const Conf& c, const S* Y, const S& emq, const S& vmb) {
  S A[8], Cv = 0.0;
  double Plo = -1e300;
  for (int k = 0; k < c.ns; ++k) {
    Cv += Y[k] * c.cv[k];
    A[k] = Y[k] * ((c.gam[k] - 1.0) * c.cv[k]) * (emq - vmb * c.pinf[k]);
    if (re(Y[k]) > 0.0) Plo = std::max(Plo, -c.pinf[k]);
  }
  const double C = re(S(vmb * Cv));
  auto F = [&](double P) {
    double s = C;
    for (int k = 0; k < c.ns; ++k) s -= re(A[k]) / (P + c.pinf[k]);
    return s;
  };
  double d = std::max(1.0, std::fabs(Plo));  // distance above P_lo
  for (;;) {
    double tail = 0.0;
    for (int k = 0; k < c.ns; ++k) tail += std::fabs(re(A[k])) / (Plo + d + c.pinf[k]);
    if (tail < 0.5 * C || !(d < 1e300)) break;
    d *= 2.0;
  }
  double hi = Plo + d, lo = hi;
  for (;;) {
    d *= 0.9;
    lo = Plo + d;
    if (F(lo) < 0.0) break;
    hi = lo;
    if (!(d > 1e-300)) return S(std::nan(""));
  }
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (F(mid) < 0.0)
      lo = mid;
    else
      hi = mid;
  }
  const double Pr = 0.5 * (lo + hi);
  S Fs = vmb * Cv;
  double dF = 0.0;
  for (int k = 0; k < c.ns; ++k) {
    const double w = Pr + c.pinf[k];
    Fs -= A[k] / w;
    dF += re(A[k]) / (w * w);
  }
  return S(Pr) - (Fs - re(Fs)) / dF;
}

template <class S> void equilibrium(const Conf& c, const S* u, Thermo<S>& t) {
  S rho = 0.0;
  for (int k = 0; k < c.ns; ++k) rho += u[k];
  t.rho = rho;
  for (int k = 0; k < c.ns; ++k) t.Y[k] = u[k] / rho;
  S ke = 0.0;
  for (int d = 0; d < 3; ++d) t.vel[d] = 0.0;
  for (int d = 0; d < c.dim; ++d) {
    t.vel[d] = u[c.ns + d] / rho;
    ke += 0.5 * u[c.ns + d] * t.vel[d];
  }
  const S E = u[c.ns + c.dim];
  t.e = (E - ke) / rho;
  const S v = 1.0 / rho;
  S qm = 0.0, bm = 0.0, Cv = 0.0, R1 = 0.0, Rg = 0.0;
  for (int k = 0; k < c.ns; ++k) {
    qm += t.Y[k] * c.q[k];
    bm += t.Y[k] * c.b[k];
    Cv += t.Y[k] * c.cv[k];
    if (c.pinf[k] != 0.0)
      R1 += t.Y[k] * ((c.gam[k] - 1.0) * c.cv[k]);
    else
      Rg += t.Y[k] * ((c.gam[k] - 1.0) * c.cv[k]);
  }
  const double Pinf = c.Pst;
  const S Ep = (t.e - qm) / (v - bm);
  const S a1 = Cv;
  const S a2 = Ep * (R1 + Rg) - Pinf * (Cv + R1);
  const S a3 = Ep * Pinf * Rg;
  S P;
  if (c.multi) {
    P = pressure_general(c, t.Y, S(t.e - qm), S(v - bm));
  } else if (re(Rg) == 0.0) {
    P = a2 / a1;
  } else {
    S sD = sqrt(a2 * a2 + 4.0 * a1 * a3);
    if (re(a2) >= 0.0)
      P = (a2 + sD) / (2.0 * a1);
    else
      P = 2.0 * a3 / (sD - a2);
  }
  t.P = P;
  S den = 0.0;
  for (int k = 0; k < c.ns; ++k) den += t.Y[k] * epsT(c, k, P);
  t.T = (t.e - qm) / den;
  sound(c, rho, t.Y, P, t.T, t.a, t.beta, t.alpha);
  const S a2s = t.a * t.a;
  // Left/right eigenvector coefficients (App. A): (rho a^2 beta - 1)/(alpha a^2 rho)
  // and the acoustic impedance a rho.
  t.cT = (rho * a2s * t.beta - 1.0) / (t.alpha * a2s * rho);
  t.z = t.a * rho;
}

// Conserved state and sound speed of (P, T, Y, u) (Godunov steps 4-5).
template <class S>
void state_from_PT(const Conf& c, const S& P, const S& T, const S* Y, const S* vel, S* u,
                   S& rho, S& a) {
  S vm = 0.0, em = 0.0;
  for (int k = 0; k < c.ns; ++k) {
    vm += Y[k] * spec_vol(c, k, P, T);
    em += Y[k] * spec_energy(c, k, P, T);
  }
  rho = 1.0 / vm;
  S ke = 0.0;
  for (int k = 0; k < c.ns; ++k) u[k] = rho * Y[k];
  for (int d = 0; d < c.dim; ++d) {
    u[c.ns + d] = rho * vel[d];
    ke += vel[d] * vel[d];
  }
  u[c.ns + c.dim] = rho * em + 0.5 * rho * ke;
  S beta, alpha;
  sound(c, rho, Y, P, T, a, beta, alpha);
}

// ---------------------------------------------------------------------------
// Per-cell quantities: equilibrium plus the phase quantities of the
// regularization (Sec. 3.2) and the diffusion model (Sec. 2.1-2.2).
// ---------------------------------------------------------------------------
// reading (linearization): the interface transform psi is differentiated
// only in mixed cells, where both phases' volume fractions exceed the floor
// phi_min of the regularization (Sec. 3.2); in a pure region of either phase
// psi follows tails of the initial profile down to delta = 1e-100, its
// gradient is set by rounding, and the derivative of the normal grows
// without bound.  psi_arg returns the volume fraction phi of a cell whose
// other phase has volume fraction other, without tangent outside mixed
// cells.  Values are unchanged.
template <class S> inline S psi_arg(const Conf& c, const S& phi, const S& other) {
  if constexpr (std::is_same<S, cplx>::value) {
    if (!(re(phi) > c.phimin && re(other) > c.phimin)) return cplx(phi.real(), 0.0);
  }
  (void)other;
  return phi;
}

template <class S> struct Cellq {
  Thermo<S> th;
  S u[16];                  // the conserved state itself
  S phi[2], psi[2], rhop[2], hrho[2], yrho[8];
  S chi[8], K[8], h[8];     // diffusion: X_c/X_p, D_c W_c/W_p, h_c
  S mu;                     // mixture viscosity sum_p phi_p mu_p
  S lam;                    // mixture heat conductivity sum_p phi_p lambda_p
};

// Wilke's rule (Sec. 2.2.2), mass-fraction form.
// reading: the standard Phi_ij = (1+W_i/W_j)^(-1/2) [1+(mu_i/mu_j)^(1/2)
// (W_j/W_i)^(1/4)]^2 / sqrt(8), with y_j W_i/W_j in the denominator sum.
template <class S> S wilke(const Conf& c, int p, const S* y) {
  S num = 0.0;
  for (int a = 0; a < c.pn[p]; ++a) {
    const int i = c.pc[p][a];
    S den = 0.0;
    for (int b2 = 0; b2 < c.pn[p]; ++b2) {
      const int j = c.pc[p][b2];
      const double r = c.W[i] / c.W[j];
      const double br = 1.0 + std::sqrt(c.mu[i] / c.mu[j]) * std::sqrt(std::sqrt(c.W[j] / c.W[i]));
      const double Phi = br * br / (std::sqrt(8.0) * std::sqrt(1.0 + r));
      den += y[j] * (r * Phi);
    }
    num += y[i] * c.mu[i] / den;
  }
  return num;
}

template <class S> void cell_quantities(const Conf& c, const S* u, Cellq<S>& q) {
  for (int v = 0; v < c.nv; ++v) q.u[v] = u[v];
  equilibrium(c, u, q.th);
  const S P = q.th.P, T = q.th.T;
  S y[8], mup[2], lamp[2];
  for (int p = 0; p < c.np; ++p) {
    // reading: y_c = Y_c / Y_p; where the phase is absent (rhoY_p <= 1e-300)
    // y_c = 1 / N_p so that rho_p, h_p stay defined.
    S rYp = 0.0;
    for (int a = 0; a < c.pn[p]; ++a) rYp += u[c.pc[p][a]];
    for (int a = 0; a < c.pn[p]; ++a) {
      const int k = c.pc[p][a];
      y[k] = re(rYp) > 1e-300 ? S(u[k] / rYp) : S(1.0 / c.pn[p]);
    }
    S vp = 0.0, hp = 0.0, ph = 0.0;
    for (int a = 0; a < c.pn[p]; ++a) {
      const int k = c.pc[p][a];
      const S vk = spec_vol(c, k, P, T);
      vp += y[k] * vk;
      hp += y[k] * spec_enthalpy(c, k, P, T);
      ph += u[k] * vk;  // phi_p = rho Y_p v_p (App. E, identity 3)
    }
    q.rhop[p] = 1.0 / vp;
    q.hrho[p] = q.rhop[p] * hp;
    q.phi[p] = ph;
    for (int a = 0; a < c.pn[p]; ++a) {
      const int k = c.pc[p][a];
      q.yrho[k] = y[k] * q.rhop[p];
    }
    // viscosity of the phase: Wilke for several components, else the constant
    if (c.pn[p] >= 2)
      mup[p] = wilke(c, p, y);
    else
      mup[p] = S(c.mu[c.pc[p][0]]);
    // diffusion quantities (Eq. SpeciesMassDiffusion, last form)
    if (c.pn[p] >= 2) {
      S winv = 0.0;
      for (int a = 0; a < c.pn[p]; ++a) winv += y[c.pc[p][a]] / c.W[c.pc[p][a]];
      const S Wp = 1.0 / winv;
      for (int a = 0; a < c.pn[p]; ++a) {
        const int k = c.pc[p][a];
        q.chi[k] = (y[k] / c.W[k]) * Wp;            // X_c/X_p
        const S Dk = mup[p] / (q.rhop[p] * c.Sc[k]);  // D_p^c = mu_p/(rho_p Sc)
        q.K[k] = Dk * c.W[k] / Wp;
      }
    } else {
      const int k = c.pc[p][0];
      q.chi[k] = 1.0;
      q.K[k] = 0.0;
    }
    for (int a = 0; a < c.pn[p]; ++a) {
      const int k = c.pc[p][a];
      q.h[k] = spec_enthalpy(c, k, P, T);
    }
    // heat conductivity of the phase (Sec. 2.2.1): gas mu_g / Pr sum_c
    // (Y_c/Y_g) C_P,c; reading: a liquid phase takes sum_c (Y_c/Y_l) lambda_c
    // (its one component's constant)
    lamp[p] = 0.0;
    if (c.pid[p] == 1) {
      S cp = 0.0;
      for (int a = 0; a < c.pn[p]; ++a) cp += y[c.pc[p][a]] * (c.gam[c.pc[p][a]] * c.cv[c.pc[p][a]]);
      lamp[p] = mup[p] / c.Pr * cp;
    } else {
      for (int a = 0; a < c.pn[p]; ++a) lamp[p] += y[c.pc[p][a]] * c.lamc[c.pc[p][a]];
    }
  }
  // psi transform (Eq. psi_transformation) of the first phase.
  // reading: 1 - phi_1 is the volume fraction of the other phase (>= 0 even
  // where phi_1 rounds above 1); psi_2 = -psi_1.
  if (c.np == 2) {
    q.psi[0] = c.eps * log((psi_arg(c, q.phi[0], q.phi[1]) + c.delta) /
                           (psi_arg(c, q.phi[1], q.phi[0]) + c.delta));
    q.psi[1] = -q.psi[0];
  } else {
    q.psi[0] = q.psi[1] = 0.0;
  }
  S mu = 0.0, lam = 0.0;
  for (int p = 0; p < c.np; ++p) {
    mu += q.phi[p] * mup[p];
    lam += q.phi[p] * lamp[p];
  }
  q.mu = mu;
  q.lam = lam;
}

// ---------------------------------------------------------------------------
// WENO5-Z (Borges et al. 2008, cited for the default scheme): value at the
// face i+1/2 from f_{i-2..i+2}.
// reading: epsilon = 1e-40, exponent p = 1 unless set otherwise.
// ---------------------------------------------------------------------------
// Substencils flat to round-off: both undivided differences of substencil k
// within 1e-7 of the stencil's largest magnitude plus the variable's own
// scale (1 for a mass fraction, the face sound speed for a velocity, 0 for
// the temperature- and pressure-like rows).
inline void flat_substencils(double f0, double f1, double f2, double f3, double f4, double scale, bool* fl) {
  const double m = std::max(std::max(std::fabs(f0), std::fabs(f1)),
                            std::max(std::max(std::fabs(f2), std::fabs(f3)), std::fabs(f4)));
  const double tol = 1e-7 * (m + scale);
  fl[0] = std::fabs(f0 - 2.0 * f1 + f2) <= tol && std::fabs(f0 - 4.0 * f1 + 3.0 * f2) <= tol;
  fl[1] = std::fabs(f1 - 2.0 * f2 + f3) <= tol && std::fabs(f1 - f3) <= tol;
  fl[2] = std::fabs(f2 - 2.0 * f3 + f4) <= tol && std::fabs(3.0 * f2 - 4.0 * f3 + f4) <= tol;
}

template <class S>
S weno5z(const S& f0, const S& f1, const S& f2, const S& f3, const S& f4, double eps, int p,
         double scale = 0.0) {
  const S q0 = (2.0 * f0 - 7.0 * f1 + 11.0 * f2) / 6.0;
  const S q1 = (-f1 + 5.0 * f2 + 2.0 * f3) / 6.0;
  const S q2 = (2.0 * f2 + 5.0 * f3 - f4) / 6.0;
  const S t0 = f0 - 2.0 * f1 + f2, s0 = f0 - 4.0 * f1 + 3.0 * f2;
  const S t1 = f1 - 2.0 * f2 + f3, s1 = f1 - f3;
  const S t2 = f2 - 2.0 * f3 + f4, s2 = 3.0 * f2 - 4.0 * f3 + f4;
  const S b0 = (13.0 / 12.0) * t0 * t0 + 0.25 * s0 * s0;
  const S b1 = (13.0 / 12.0) * t1 * t1 + 0.25 * s1 * s1;
  const S b2 = (13.0 / 12.0) * t2 * t2 + 0.25 * s2 * s2;
  auto combine = [&](const S& c0, const S& c1, const S& c2) {
    const S tau = vabs(S(c0 - c2));
    S r0 = tau / (c0 + eps), r1 = tau / (c1 + eps), r2 = tau / (c2 + eps);
    if (p == 2) {
      r0 = r0 * r0;
      r1 = r1 * r1;
      r2 = r2 * r2;
    }
    const S a0 = 0.1 * (1.0 + r0), a1 = 0.6 * (1.0 + r1), a2 = 0.3 * (1.0 + r2);
    return S((a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2));
  };
  S out = combine(b0, b1, b2);
  if constexpr (std::is_same<S, cplx>::value) {
    // reading (linearization): a substencil flat to round-off has a
    // smoothness indicator set by rounding noise (and two such substencils
    // split their weight by noise); its derivative is taken as in exact
    // arithmetic for constant data, indicator 0 without derivative.  All
    // three flat gives the ideal weights.  The value is kept.
    bool fl[3];
    flat_substencils(re(f0), re(f1), re(f2), re(f3), re(f4), scale, fl);
    if (fl[0] || fl[1] || fl[2]) {
      const S z(0.0);
      const S lin = combine(fl[0] ? z : b0, fl[1] ? z : b1, fl[2] ? z : b2);
      out = cplx(out.real(), lin.imag());
    }
  }
  return out;
}

// ---------------------------------------------------------------------------
// Mass-fraction interpolation limiter (Sec. 3.3.1, after Baumgart et al.).
// reading of the garbled min/max: sum > 1 uses d_c = min(Y_s, Y_cell) - Y_s,
// sum < 1 uses max; Y_s += (1 - sum)/sum(d) * d_c; no-op if the denominator
// vanishes.  Returns the branch taken (0 none, 1 sum>1, 2 sum<1).
// ---------------------------------------------------------------------------
// Value of a with the tangent (imaginary part) of b.
// ---------------------------------------------------------------------------
// WENO5-JS (Jiang and Shu 1996, cited as a scheme variant): the same
// substencil values and smoothness indicators as WENO5-Z, weights
// alpha_k = d_k / (beta_k + eps)^p, omega_k = alpha_k / sum alpha.
// reading: eps and p are the weno_eps / weno_p options (the customary 1e-6
// and 2 are the caller's to pass).
// ---------------------------------------------------------------------------
template <class S>
S weno5js(const S& f0, const S& f1, const S& f2, const S& f3, const S& f4, double eps, int p) {
  const S q0 = (2.0 * f0 - 7.0 * f1 + 11.0 * f2) / 6.0;
  const S q1 = (-f1 + 5.0 * f2 + 2.0 * f3) / 6.0;
  const S q2 = (2.0 * f2 + 5.0 * f3 - f4) / 6.0;
  const S t0 = f0 - 2.0 * f1 + f2, s0 = f0 - 4.0 * f1 + 3.0 * f2;
  const S t1 = f1 - 2.0 * f2 + f3, s1 = f1 - f3;
  const S t2 = f2 - 2.0 * f3 + f4, s2 = 3.0 * f2 - 4.0 * f3 + f4;
  S g0 = (13.0 / 12.0) * t0 * t0 + 0.25 * s0 * s0 + eps;
  S g1 = (13.0 / 12.0) * t1 * t1 + 0.25 * s1 * s1 + eps;
  S g2 = (13.0 / 12.0) * t2 * t2 + 0.25 * s2 * s2 + eps;
  if (p == 2) {
    g0 = g0 * g0;
    g1 = g1 * g1;
    g2 = g2 * g2;
  }
  const S a0 = 0.1 / g0, a1 = 0.6 / g1, a2 = 0.3 / g2;
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// ---------------------------------------------------------------------------
// TENO5 (Fu et al. 2016, cited as a scheme variant): smoothness measures
// gamma_k = (C + tau5 / (beta_k + eps))^q, tau5 = |beta_0 - beta_2|; a
// substencil whose share chi_k = gamma_k / sum gamma falls below C_T is cut
// off (delta_k = 0), the others keep their linear weights: omega_k = d_k
// delta_k / sum d delta.  reading: the paper prints no parameters; the cited
// defaults C = 1, q = 6, C_T = 1e-5 are taken, eps = weno_eps.  The shares are
// evaluated with every measure divided by the largest (the same values; no
// overflow of the sixth powers).
// ---------------------------------------------------------------------------
template <class S>
S teno5(const S& f0, const S& f1, const S& f2, const S& f3, const S& f4, double eps) {
  const S q0 = (2.0 * f0 - 7.0 * f1 + 11.0 * f2) / 6.0;
  const S q1 = (-f1 + 5.0 * f2 + 2.0 * f3) / 6.0;
  const S q2 = (2.0 * f2 + 5.0 * f3 - f4) / 6.0;
  const S t0 = f0 - 2.0 * f1 + f2, s0 = f0 - 4.0 * f1 + 3.0 * f2;
  const S t1 = f1 - 2.0 * f2 + f3, s1 = f1 - f3;
  const S t2 = f2 - 2.0 * f3 + f4, s2 = 3.0 * f2 - 4.0 * f3 + f4;
  const S b0 = (13.0 / 12.0) * t0 * t0 + 0.25 * s0 * s0;
  const S b1 = (13.0 / 12.0) * t1 * t1 + 0.25 * s1 * s1;
  const S b2 = (13.0 / 12.0) * t2 * t2 + 0.25 * s2 * s2;
  const S tau = vabs(S(b0 - b2));
  const double C = 1.0, CT = 1e-5;
  const int q = 6;
  const double a[3] = {re(C + tau / (b0 + eps)), re(C + tau / (b1 + eps)), re(C + tau / (b2 + eps))};
  const double m = std::max(a[0], std::max(a[1], a[2]));
  double g[3], sg = 0.0;
  for (int k = 0; k < 3; ++k) {
    g[k] = std::pow(a[k] / m, q);
    sg += g[k];
  }
  const double d[3] = {0.1, 0.6, 0.3};
  const S qk[3] = {q0, q1, q2};
  double sd = 0.0;
  S num = 0.0;
  for (int k = 0; k < 3; ++k)
    if (g[k] / sg >= CT) {
      sd += d[k];
      num += d[k] * qk[k];
    }
  return num / sd;
}

// ---------------------------------------------------------------------------
// The polynomial of degree n-1 whose averages over the n unit cells centred
// at off, off+1, ..., off+n-1 are f[0..n-1] (the target cell is [-1/2, 1/2]):
// its monomial coefficients a[0..n-1], from the averaging conditions solved
// by Gauss-Jordan elimination in double (the inverse of each (off, n)
// averaging matrix is formed once, for off in [-5, 5] and n <= 6).
// ---------------------------------------------------------------------------
struct AvgInverse {
  double Mi[6][6];
};
inline AvgInverse averaging_inverse(int off, int n) {
  AvgInverse r;
  double M[6][6], (&Mi)[6][6] = r.Mi;
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      const double x1 = off + j + 0.5, x0 = off + j - 0.5;
      M[j][k] = (std::pow(x1, k + 1) - std::pow(x0, k + 1)) / (k + 1);
      Mi[j][k] = j == k ? 1.0 : 0.0;
    }
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
    for (int k = 0; k < n; ++k) {
      std::swap(M[col][k], M[piv][k]);
      std::swap(Mi[col][k], Mi[piv][k]);
    }
    const double inv = 1.0 / M[col][col];
    for (int k = 0; k < n; ++k) {
      M[col][k] *= inv;
      Mi[col][k] *= inv;
    }
    for (int r = 0; r < n; ++r)
      if (r != col) {
        const double m = M[r][col];
        for (int k = 0; k < n; ++k) {
          M[r][k] -= m * M[col][k];
          Mi[r][k] -= m * Mi[col][k];
        }
      }
  }
  return r;
}

template <class S> void poly_from_averages(const S* f, int off, int n, S* a) {
  static const std::vector<AvgInverse> table = [] {
    std::vector<AvgInverse> t(11 * 7);
    for (int o = -5; o <= 5; ++o)
      for (int m = 1; m <= 6; ++m) t[(o + 5) * 7 + m] = averaging_inverse(o, m);
    return t;
  }();
  const AvgInverse inv = (off >= -5 && off <= 5) ? table[(off + 5) * 7 + n] : averaging_inverse(off, n);
  for (int k = 0; k < n; ++k) {
    a[k] = 0.0;
    for (int j = 0; j < n; ++j) a[k] += inv.Mi[k][j] * f[j];
  }
}

// Value at the face x = 1/2 of the polynomial with coefficients a[0..n-1].
template <class S> S poly_at_face(const S* a, int n) {
  S v = 0.0;
  for (int k = n - 1; k >= 0; --k) v = v * 0.5 + a[k];
  return v;
}

// Smoothness indicator of Jiang and Shu: the sum over l = 1..n-1 of the
// integral over the target cell of the square of the l-th derivative (unit
// cell width), from the monomial coefficients.
// The integrals of products of derivatives of x^j and x^k are gathered once
// into G[j][k] = sum over l of (d^l x^j)(d^l x^k) integrated over the cell
// (terms with l > min(j, k) vanish).
template <class S> S js_indicator(const S* a, int n) {
  static const std::vector<double> G = [] {
    auto fall = [](int k, int l) {  // k! / (k-l)!
      double r = 1.0;
      for (int t = 0; t < l; ++t) r *= k - t;
      return r;
    };
    std::vector<double> g(36, 0.0);
    for (int j = 1; j < 6; ++j)
      for (int k = 1; k < 6; ++k)
        for (int l = 1; l <= std::min(j, k); ++l) {
          const int m = j + k - 2 * l;  // integral of x^m over [-1/2, 1/2]
          if (m % 2) continue;
          g[j * 6 + k] += fall(j, l) * fall(k, l) * 2.0 * std::pow(0.5, m + 1) / (m + 1);
        }
    return g;
  }();
  S beta = 0.0;
  for (int j = 1; j < n; ++j)
    for (int k = 1; k < n; ++k) beta += a[j] * a[k] * G[j * 6 + k];
  return beta;
}

// ---------------------------------------------------------------------------
// TENO6 (Fu et al. 2016, cited as a scheme variant), from f_{i-2..i+3}: the
// candidate stencils {i-1,i,i+1}, {i,i+1,i+2}, {i-2,i-1,i} and
// {i,i+1,i+2,i+3}, each the polynomial matching its cell averages, evaluated
// at the face; indicators beta_k of Jiang and Shu over cell i; the reference
// tau6 = |beta_6 - (beta_up + beta_down + 4 beta_central)/6| with beta_6 the
// indicator of the six-point polynomial (the combination whose Taylor
// expansion starts at the sixth power of the cell width); measures
// gamma_k = (C + tau6/(beta_k + eps))^q, cut-off of substencils whose share
// falls below C_T; the kept ones take the linear weights (central 9/20,
// downwind 3/10, upwind 1/20, four-point 1/5), which recombine the
// six-point polynomial's face value.  reading: the paper prints no
// parameters; C = 1, q = 6, C_T = 1e-7, eps = weno_eps (C_T: parity
// unpinned).
// ---------------------------------------------------------------------------
template <class S>
S teno6(const S& f0, const S& f1, const S& f2, const S& f3, const S& f4, const S& f5, double eps,
        double* tau_out = nullptr) {
  const S f[6] = {f0, f1, f2, f3, f4, f5};
  const int off[4] = {-1, 0, -2, 0}, first[4] = {1, 2, 0, 2}, np[4] = {3, 3, 3, 4};
  const double d[4] = {9.0 / 20.0, 3.0 / 10.0, 1.0 / 20.0, 1.0 / 5.0};
  S qk[4], bk[4], a[6];
  for (int k = 0; k < 4; ++k) {
    poly_from_averages(f + first[k], off[k], np[k], a);
    qk[k] = poly_at_face(a, np[k]);
    bk[k] = js_indicator(a, np[k]);
  }
  poly_from_averages(f, -2, 6, a);
  const S b6 = js_indicator(a, 6);
  const S tau = vabs(S(b6 - (bk[1] + bk[2] + 4.0 * bk[0]) / 6.0));
  if (tau_out) *tau_out = re(tau);
  const double C = 1.0, CT = 1e-7;
  const int q = 6;
  double g[4], m = 0.0, sg = 0.0;
  for (int k = 0; k < 4; ++k) {
    g[k] = re(C + tau / (bk[k] + eps));
    m = std::max(m, g[k]);
  }
  for (int k = 0; k < 4; ++k) {
    g[k] = std::pow(g[k] / m, q);
    sg += g[k];
  }
  double sd = 0.0;
  S num = 0.0;
  for (int k = 0; k < 4; ++k)
    if (g[k] / sg >= CT) {
      sd += d[k];
      num += d[k] * qk[k];
    }
  return num / sd;
}

// Face value from f_{i-2..i+3} with the configured scheme (0 WENO5-Z,
// 1 WENO5-JS, 2 TENO5: these use f_{i-2..i+2}; 3 TENO6).
template <class S>
S reconstruct(const Conf& c, const S& f0, const S& f1, const S& f2, const S& f3, const S& f4, const S& f5,
              double scale) {
  if (c.weno == 1) return weno5js(f0, f1, f2, f3, f4, c.weps, c.wp);
  if (c.weno == 2) return teno5(f0, f1, f2, f3, f4, c.weps);
  if (c.weno == 3) return teno6(f0, f1, f2, f3, f4, f5, c.weps);
  return weno5z(f0, f1, f2, f3, f4, c.weps, c.wp, scale);
}

template <class S> inline S with_tangent_of(const S& a, const S&) { return a; }
inline cplx with_tangent_of(const cplx& a, const cplx& b) { return cplx(a.real(), b.imag()); }

template <class S> int ylimit(int ns, S* Ys, const S* Yc) {
  S sum = 0.0;
  for (int k = 0; k < ns; ++k) sum += Ys[k];
  S d[8];
  int br;
  if (re(sum) > 1.0) {
    br = 1;
    for (int k = 0; k < ns; ++k) d[k] = vmin(Ys[k], Yc[k]) - Ys[k];
  } else if (re(sum) < 1.0) {
    br = 2;
    for (int k = 0; k < ns; ++k) d[k] = vmax(Ys[k], Yc[k]) - Ys[k];
  } else {
    return 0;
  }
  // reading (linearization): a min/max decided by a difference of round-off
  // size (at most 1e-10) is a tie; the correction keeps its value but is not
  // differentiated
  for (int k = 0; k < ns; ++k)
    if (std::fabs(re(Ys[k]) - re(Yc[k])) <= 1e-10) d[k] = with_tangent_of(d[k], S(0.0));
  S sd = 0.0;
  for (int k = 0; k < ns; ++k) sd += d[k];
  if (std::fabs(re(sd)) < 1e-300) return 0;
  const S f = (1.0 - sum) / sd;
  // reading (linearization): a correction of round-off size (|1 - sum| at
  // most 1e-13) is applied to the value but not differentiated
  const bool noise = std::fabs(1.0 - re(sum)) <= 1e-13;
  for (int k = 0; k < ns; ++k) {
    const S y = Ys[k] + f * d[k];
    Ys[k] = noise ? S(with_tangent_of(y, Ys[k])) : y;
  }
  return br;
}

// ---------------------------------------------------------------------------
// One side of a face in the frame (n, t1, t2) of the sweep direction.
// ---------------------------------------------------------------------------
template <class S> struct Side {
  S rho, un, ut[2], P, E, a, rY[8];
};

// Admissibility of a conserved state (Eqs. PositivityReqs1-2).
// reading: rhoY_c >= 0 (pure regions hold exact zeros), rho > 0,
// rho (e - q) > 0 and rho (v - b) = 1 - sum rhoY_c b_c > 0; NaN fails.
template <class S> bool admissible(const Conf& c, const S* u) {
  S rho = 0.0, rq = 0.0, rb = 0.0;
  for (int k = 0; k < c.ns; ++k) {
    if (!(re(u[k]) >= 0.0)) return false;
    rho += u[k];
    rq += u[k] * c.q[k];
    rb += u[k] * c.b[k];
  }
  if (!(re(rho) > 0.0)) return false;
  S m2 = 0.0;
  for (int d = 0; d < c.dim; ++d) m2 += u[c.ns + d] * u[c.ns + d];
  const S rhoe = u[c.ns + c.dim] - 0.5 * m2 / rho - rq;
  if (!(re(rhoe) > 0.0)) return false;
  if (!(re(S(1.0 - rb)) > 0.0)) return false;
  return true;
}

// HLLC (App. B) in the face frame; U and F have the layout
// [rhoY_1..ns, rho u_n, rho u_t1.., E].
template <class S> void side_UF(const Conf& c, const Side<S>& s, S* U, S* F) {
  const int nt = c.dim - 1;
  for (int k = 0; k < c.ns; ++k) {
    U[k] = s.rY[k];
    F[k] = s.rY[k] * s.un;
  }
  U[c.ns] = s.rho * s.un;
  F[c.ns] = s.rho * s.un * s.un + s.P;
  for (int t = 0; t < nt; ++t) {
    U[c.ns + 1 + t] = s.rho * s.ut[t];
    F[c.ns + 1 + t] = s.rho * s.un * s.ut[t];
  }
  U[c.ns + c.dim] = s.E;
  F[c.ns + c.dim] = s.un * (s.E + s.P);
}

template <class S> void star_state(const Conf& c, const Side<S>& s, const S& sK, const S& ss, S* U) {
  const int nt = c.dim - 1;
  const S fac = (sK - s.un) / (sK - ss);
  for (int k = 0; k < c.ns; ++k) U[k] = fac * s.rY[k];
  U[c.ns] = fac * (s.rho * ss);
  for (int t = 0; t < nt; ++t) U[c.ns + 1 + t] = fac * (s.rho * s.ut[t]);
  U[c.ns + c.dim] = fac * (s.E + (ss - s.un) * (s.rho * ss + s.P / (sK - s.un)));
}

template <class S> void hllc(const Conf& c, const Side<S>& L, const Side<S>& R, S* F) {
  const int nv = c.nv;
  // reading: u-bar, a-bar are arithmetic means of the two face states
  const S ub = 0.5 * (L.un + R.un), ab = 0.5 * (L.a + R.a);
  S sL = vmin(S(ub - ab), S(L.un - L.a));
  S sR = vmax(S(ub + ab), S(R.un + R.a));
  bool both = false;
  if constexpr (std::is_same<S, cplx>::value) {
    // reading (linearization): a choice decided by rounding -- a near-tie of
    // the wave-speed arms within 1e-9 of the speed scale, or s* within 1e-9
    // of zero -- is differentiated as at the exact tie: the averaged-state
    // speed, the mean of the two star fluxes.  Values are kept.
    const double tS = 1e-9 * (re(ab) + std::fabs(re(ub)));
    if (std::fabs(re(L.un - L.a) - re(ub - ab)) <= tS) sL = with_tangent_of(sL, S(ub - ab));
    if (std::fabs(re(R.un + R.a) - re(ub + ab)) <= tS) sR = with_tangent_of(sR, S(ub + ab));
  }
  const S sm = vmin(S(0.0), sL), sp = vmax(S(0.0), sR);
  const S ss = (R.P - L.P + L.rho * L.un * (sL - L.un) - R.rho * R.un * (sR - R.un)) /
               (L.rho * (sL - L.un) - R.rho * (sR - R.un));
  const double sg = vsgn(ss);
  if constexpr (std::is_same<S, cplx>::value)
    both = std::fabs(re(ss)) <= 1e-9 * std::max(std::fabs(re(sL)), std::fabs(re(sR)));
  S UL[16], FL[16], UR[16], FR[16], Us[16];
  // sign(0) = 0 (reading): both halves with weight 1/2
  if (sg >= 0.0 || both) {
    side_UF(c, L, UL, FL);
    star_state(c, L, sL, ss, Us);
    for (int v = 0; v < nv; ++v) FL[v] = FL[v] + sm * (Us[v] - UL[v]);
  }
  if (sg <= 0.0 || both) {
    side_UF(c, R, UR, FR);
    star_state(c, R, sR, ss, Us);
    for (int v = 0; v < nv; ++v) FR[v] = FR[v] + sp * (Us[v] - UR[v]);
  }
  for (int v = 0; v < nv; ++v) {
    if (sg > 0.0)
      F[v] = FL[v];
    else if (sg < 0.0)
      F[v] = FR[v];
    else
      F[v] = 0.5 * FL[v] + 0.5 * FR[v];
    if (both) F[v] = with_tangent_of(F[v], S(0.5 * FL[v] + 0.5 * FR[v]));
  }
}

// ---------------------------------------------------------------------------
// Grid: ghost filling (periodic / zero-gradient / reflective mirror).
// reading: the boundary types named by the workloads; ghosts are copies of
// mapped interior cells, the wall-normal momentum negated at a mirror.
// ---------------------------------------------------------------------------
// Boundary types: 0 periodic, 1 zero-gradient outflow, 2 reflective mirror,
// 3 characteristic (the stencils see zero-gradient ghosts; the boundary
// face's flux is replaced, see characteristic_flux).
inline int map_index(int i, int n, int lo, int hi, int& flip) {
  if (i < 0) {
    if (lo == 0) return ((i % n) + n) % n;
    if (lo == 1 || lo == 3) return 0;
    flip = !flip;
    return -1 - i;
  }
  if (i >= n) {
    if (hi == 0) return i % n;
    if (hi == 1 || hi == 3) return n - 1;
    flip = !flip;
    return 2 * n - 1 - i;
  }
  return i;
}

template <class S> void fill_padded_s(const Conf& c, const S* U, std::vector<S>& P) {
  P.assign((size_t)c.nv * c.npad, S(0.0));
  for (int k = -c.g[2]; k < c.n[2] + c.g[2]; ++k)
    for (int j = -c.g[1]; j < c.n[1] + c.g[1]; ++j)
      for (int i = -c.g[0]; i < c.n[0] + c.g[0]; ++i) {
        int fl[3] = {0, 0, 0};
        const int ii = map_index(i, c.n[0], c.bclo[0], c.bchi[0], fl[0]);
        const int jj = map_index(j, c.n[1], c.bclo[1], c.bchi[1], fl[1]);
        const int kk = map_index(k, c.n[2], c.bclo[2], c.bchi[2], fl[2]);
        const long src = c.cidx(ii, jj, kk);
        const long dst = c.pidx(i, j, k);
        for (int v = 0; v < c.nv; ++v) {
          S x = U[(long)v * c.ncell + src];
          const int d = v - c.ns;
          if (d >= 0 && d < c.dim && fl[d]) x = -x;
          P[(size_t)v * c.npad + dst] = x;
        }
      }
}

// ---------------------------------------------------------------------------
// The face flux of Sec. 3.1.3 (Godunov steps 1-6), the limiters of Sec. 3.3,
// the regularization flux of Sec. 3.2.1 and the species diffusion flux.
// ---------------------------------------------------------------------------
struct FaceArgs {
  int d;         // sweep direction
  int t[2];      // tangential active directions (dim-1 of them)
  double lam;    // 2 D rk2 dt / dx_d  (pseudo-time factor of the flux limiter)
  double rk0, rk1;
  double Gamma;
};

template <class S>
void make_side_from_cell(const Conf& c, const Cellq<S>& q, const FaceArgs& fa, Side<S>& s) {
  s.rho = q.th.rho;
  s.un = q.th.vel[fa.d];
  for (int t = 0; t < c.dim - 1; ++t) s.ut[t] = q.th.vel[fa.t[t]];
  s.P = q.th.P;
  s.E = q.u[c.ns + c.dim];
  s.a = q.th.a;
  for (int k = 0; k < c.ns; ++k) s.rY[k] = q.u[k];
}

// rotated-frame flux -> flux in (x, y, z) layout
template <class S> void unrotate(const Conf& c, const FaceArgs& fa, const S* Fr, S* F) {
  for (int k = 0; k < c.ns; ++k) F[k] = Fr[k];
  F[c.ns + fa.d] = Fr[c.ns];
  for (int t = 0; t < c.dim - 1; ++t) F[c.ns + fa.t[t]] = Fr[c.ns + 1 + t];
  F[c.ns + c.dim] = Fr[c.ns + c.dim];
}

// Flux limiter pseudo-states (Sec. 3.3.2) of the two cells of a face: a for
// the left cell, b for the right one.  reading: the face flux enters with
// dt/dx and with the sign of an outflow (minus on the left cell, plus on the
// right cell), measured against the cell's own physical flux along the sweep
// (FcL, FcR).  The cell terms cancel between the two faces of a direction,
// so the mean over the 2D faces of a cell is still the RK stage update, and
// a uniform flow yields pseudo-states equal to the state.
template <class S>
void pseudo_pair(const Conf& c, const FaceArgs& fa, const S* UkL, const S* UnL, const S* FcL,
                 const S* UkR, const S* UnR, const S* FcR, const S* F, S* a, S* b) {
  for (int v = 0; v < c.nv; ++v) {
    a[v] = fa.rk0 * UnL[v] + fa.rk1 * UkL[v] - fa.lam * (F[v] - FcL[v]);
    b[v] = fa.rk0 * UnR[v] + fa.rk1 * UkR[v] + fa.lam * (F[v] - FcR[v]);
  }
}

template <class S>
bool pseudo_ok(const Conf& c, const FaceArgs& fa, const S* UkL, const S* UnL, const S* FcL,
               const S* UkR, const S* UnR, const S* FcR, const S* F) {
  S a[16], b[16];
  pseudo_pair(c, fa, UkL, UnL, FcL, UkR, UnR, FcR, F, a, b);
  return admissible(c, a) && admissible(c, b);
}

// Physical convective flux of a cell along the sweep, (x, y, z) layout.
template <class S> void cell_flux(const Conf& c, const FaceArgs& fa, const Cellq<S>& q, S* F) {
  Side<S> s;
  make_side_from_cell(c, q, fa, s);
  S Ur[16], Fr[16];
  side_UF(c, s, Ur, Fr);
  unrotate(c, fa, Fr, F);
}

// psi_B - psi_A of the first phase, as eps * ln of the ratio of the
// arguments of the two logarithms (same value, no cancellation).
template <class S> S dpsi(const Conf& c, const Cellq<S>& A, const Cellq<S>& B) {
  const S num = (psi_arg(c, B.phi[0], B.phi[1]) + c.delta) * (psi_arg(c, A.phi[1], A.phi[0]) + c.delta);
  const S den = (psi_arg(c, A.phi[0], A.phi[1]) + c.delta) * (psi_arg(c, B.phi[1], B.phi[0]) + c.delta);
  return c.eps * log(num / den);
}

template <class S>
void face_flux(const Conf& c, const FaceArgs& fa, const Cellq<S>* const* st /* i-2..i+3 */,
               const S* UnL, const S* UnR, const Cellq<S>* const (*tg)[2] /* [2*(dim-1)][2]:
               (t, -), (t, +) neighbours of cells i and i+1 */,
               S* Fout, uint16_t& mask) {
  const int ns = c.ns, nv = c.nv, nt = c.dim - 1;
  const Cellq<S>& CL = *st[2];
  const Cellq<S>& CR = *st[3];
  mask = 0;

  // --- Godunov step 1: face average of U (reading: arithmetic mean), its
  // equilibrium, and the eigenvector coefficients of App. A.
  S ubar[16];
  for (int v = 0; v < nv; ++v) ubar[v] = 0.5 * (CL.u[v] + CR.u[v]);
  Thermo<S> tf;
  equilibrium(c, ubar, tf);
  const S cT = tf.cT, z = tf.z;

  // --- characteristic variables S^-1 W on the six stencil cells
  // W = [T, Y_c, u_n, u_t.., P]; rows: T - cT P, Y_c, u_t, (z/2) u_n + P/2,
  // -(z/2) u_n + P/2.  All Y_c are kept (their rows of S^-1 are the identity).
  const int nw = ns + nt + 3;
  S w[6][24];
  for (int m = 0; m < 6; ++m) {
    const Thermo<S>& th = st[m]->th;
    const S un = th.vel[fa.d];
    int o = 0;
    w[m][o++] = th.T - cT * th.P;
    for (int k = 0; k < ns; ++k) w[m][o++] = th.Y[k];
    for (int t = 0; t < nt; ++t) w[m][o++] = th.vel[fa.t[t]];
    w[m][o++] = 0.5 * z * un + 0.5 * th.P;
    w[m][o++] = -0.5 * z * un + 0.5 * th.P;
  }
  // --- Godunov step 2: ENO-type interpolation, left (i-2..i+2) and right
  // (mirrored, i+3..i-1) states
  S wl[24], wr[24];
  for (int r = 0; r < nw && c.basis == 0; ++r) {
    // natural scale of the row for the round-off flatness test
    const double sc = (r >= 1 && r <= ns) ? 1.0 : ((r > ns && r <= ns + nt) ? re(tf.a) : 0.0);
    wl[r] = reconstruct(c, w[0][r], w[1][r], w[2][r], w[3][r], w[4][r], w[5][r], sc);
    wr[r] = reconstruct(c, w[5][r], w[4][r], w[3][r], w[2][r], w[1][r], w[0][r], sc);
  }
  S PL, PR, TL, TR, unL, unR, utL[2], utR[2], YL[8], YR[8];
  if (c.basis == 1) {
    // Negative control (Sec. 4.2.2, Table DropAdvectionNoIECResults): the
    // five-equation model's basis W = [rho Y_c, u, P], interpolated one
    // variable at a time without characteristic decomposition; the face
    // temperature is the one at which the interpolated partial densities
    // fill the volume at the interpolated pressure, sum_c rho Y_c v_c(P, T)
    // = 1 (linear in T for the NASG v_c = kappa_c(P) T + b_c), and
    // Y_c = rho Y_c / sum rho Y.
    S v6[6], rYL[8], rYR[8];
    auto recon_pair = [&](S& l, S& r) {
      l = reconstruct(c, v6[0], v6[1], v6[2], v6[3], v6[4], v6[5], 0.0);
      r = reconstruct(c, v6[5], v6[4], v6[3], v6[2], v6[1], v6[0], 0.0);
    };
    for (int k = 0; k < ns; ++k) {
      for (int m = 0; m < 6; ++m) v6[m] = st[m]->u[k];
      recon_pair(rYL[k], rYR[k]);
    }
    for (int m = 0; m < 6; ++m) v6[m] = st[m]->th.vel[fa.d];
    recon_pair(unL, unR);
    for (int t = 0; t < nt; ++t) {
      for (int m = 0; m < 6; ++m) v6[m] = st[m]->th.vel[fa.t[t]];
      recon_pair(utL[t], utR[t]);
    }
    for (int m = 0; m < 6; ++m) v6[m] = st[m]->th.P;
    recon_pair(PL, PR);
    auto face_T = [&](const S* rY, const S& P, S* Y, S& T) {
      S rho = 0.0, num = 1.0, den = 0.0;
      for (int k = 0; k < ns; ++k) {
        rho += rY[k];
        num -= rY[k] * c.b[k];
        den += rY[k] * kappa(c, k, P);
      }
      for (int k = 0; k < ns; ++k) Y[k] = rY[k] / rho;
      T = num / den;
    };
    face_T(rYL, PL, YL, TL);
    face_T(rYR, PR, YR, TR);
  } else {
    // --- Godunov step 3: back to physical space with S
    int o = 1 + ns + nt;
    PL = wl[o] + wl[o + 1];
    PR = wr[o] + wr[o + 1];
    unL = (wl[o] - wl[o + 1]) / z;
    unR = (wr[o] - wr[o + 1]) / z;
    TL = wl[0] + cT * PL;
    TR = wr[0] + cT * PR;
    for (int k = 0; k < ns; ++k) {
      YL[k] = wl[1 + k];
      YR[k] = wr[1 + k];
    }
    for (int t = 0; t < nt; ++t) {
      utL[t] = wl[1 + ns + t];
      utR[t] = wr[1 + ns + t];
    }
  }
  // --- interpolation limiters (Sec. 3.3.1)
  if (c.positivity) {
    ylimit(ns, YL, CL.th.Y);
    ylimit(ns, YR, CR.th.Y);
    // reading: T inadmissible if <= 0; P inadmissible if P + P_inf,c <= 0
    // for a component present (Y_c > 0) on that side.
    if (!(re(TL) > 0.0)) { TL = CL.th.T; mask |= ORACLE_M_TL; }
    if (!(re(TR) > 0.0)) { TR = CR.th.T; mask |= ORACLE_M_TR; }
    bool badL = false, badR = false;
    for (int k = 0; k < ns; ++k) {
      if (re(YL[k]) > 0.0 && !(re(S(PL + c.pinf[k])) > 0.0)) badL = true;
      if (re(YR[k]) > 0.0 && !(re(S(PR + c.pinf[k])) > 0.0)) badR = true;
    }
    if (badL) { PL = CL.th.P; mask |= ORACLE_M_PL; }
    if (badR) { PR = CR.th.P; mask |= ORACLE_M_PR; }
  }
  // --- Godunov steps 4-5: face states from the EOS
  Side<S> sL, sR;
  {
    S vel[3], uu[16], rho, a;
    vel[fa.d] = unL;
    for (int t = 0; t < nt; ++t) vel[fa.t[t]] = utL[t];
    state_from_PT(c, PL, TL, YL, vel, uu, rho, a);
    sL.rho = rho; sL.un = unL; sL.P = PL; sL.a = a; sL.E = uu[ns + c.dim];
    for (int t = 0; t < nt; ++t) sL.ut[t] = utL[t];
    for (int k = 0; k < ns; ++k) sL.rY[k] = uu[k];
    vel[fa.d] = unR;
    for (int t = 0; t < nt; ++t) vel[fa.t[t]] = utR[t];
    state_from_PT(c, PR, TR, YR, vel, uu, rho, a);
    sR.rho = rho; sR.un = unR; sR.P = PR; sR.a = a; sR.E = uu[ns + c.dim];
    for (int t = 0; t < nt; ++t) sR.ut[t] = utR[t];
    for (int k = 0; k < ns; ++k) sR.rY[k] = uu[k];
  }
  // --- Godunov step 6: HLLC
  S Fr[16], F[16];
  hllc(c, sL, sR, Fr);
  unrotate(c, fa, Fr, F);
  // --- advective flux limiter (Sec. 3.3.2)
  S FcL[16], FcR[16];
  if (c.positivity) {
    cell_flux(c, fa, CL, FcL);
    cell_flux(c, fa, CR, FcR);
    if (!pseudo_ok(c, fa, CL.u, UnL, FcL, CR.u, UnR, FcR, F)) {
      mask |= ORACLE_M_FALLBACK;
      Side<S> cl, cr;
      make_side_from_cell(c, CL, fa, cl);
      make_side_from_cell(c, CR, fa, cr);
      hllc(c, cl, cr, Fr);
      unrotate(c, fa, Fr, F);
      // reading: the first-order flux is used unconditionally; a failing
      // re-test is only counted.
      if (!pseudo_ok(c, fa, CL.u, UnL, FcL, CR.u, UnR, FcR, F)) mask |= ORACLE_M_UNRECOVERABLE;
    }
  }
  // --- interface regularization flux (Eqs. SkewSymmetricSplitting_Regularization)
  S Fdi[16];
  for (int v = 0; v < nv; ++v) Fdi[v] = 0.0;
  if (c.cdi && c.np == 2) {
    // reading: with two phases phi_2 = 1 - phi_1, so the regularization
    // velocity of the second phase is the negative of the first's; it is
    // evaluated once, for the first phase.
    const double dxn = c.dx[fa.d];
    const S gphi = (CR.phi[0] - CL.phi[0]) / dxn;
    const S psib = 0.5 * (CL.psi[0] + CR.psi[0]);
    // reading: face normal = discrete grad(psi)/|grad(psi)|, normal part a
    // two-point difference, tangential parts the mean of the two cells'
    // central differences, zero where the gradient vanishes.  Differences
    // of psi are evaluated as eps * ln of the ratio of the psi arguments.
    const S gn = dpsi(c, CL, CR) / dxn;
    S nrm2 = gn * gn;
    for (int t = 0; t < nt; ++t) {
      const S gt = (dpsi(c, *tg[2 * t][0], *tg[2 * t + 1][0]) +
                    dpsi(c, *tg[2 * t][1], *tg[2 * t + 1][1])) /
                   (4.0 * c.dx[fa.t[t]]);
      nrm2 += gt * gt;
    }
    S nhat = 0.0;
    if (re(nrm2) > 0.0) nhat = gn / sqrt(nrm2);
    const S th = tanh(psib / (2.0 * c.eps));
    const S a1 = fa.Gamma * (c.eps * gphi -
                             0.25 * (1.0 - th * th - 4.0 * c.phimin * (1.0 - c.phimin)) * nhat);
    S Rsum = 0.0, hR = 0.0;
    for (int p = 0; p < c.np; ++p) {
      const S ap = p == 0 ? a1 : S(-a1);
      for (int a = 0; a < c.pn[p]; ++a) {
        const int k = c.pc[p][a];
        const S Rk = -0.5 * (CL.yrho[k] + CR.yrho[k]) * ap;
        Fdi[k] = Rk;
        Rsum += Rk;
      }
      hR += -0.5 * (CL.hrho[p] + CR.hrho[p]) * ap;
    }
    S kb = 0.0;
    for (int dd = 0; dd < c.dim; ++dd) {
      const S ubd = 0.5 * (CL.th.vel[dd] + CR.th.vel[dd]);
      Fdi[ns + dd] = ubd * Rsum;
      kb += CL.th.vel[dd] * CR.th.vel[dd];
    }
    kb = 0.5 * kb;
    Fdi[ns + c.dim] = kb * Rsum + hR;
    if (c.positivity) {
      S Ft[16];
      for (int v = 0; v < nv; ++v) Ft[v] = F[v] + Fdi[v];
      if (!pseudo_ok(c, fa, CL.u, UnL, FcL, CR.u, UnR, FcR, Ft)) {
        // reading: the whole regularization flux of this face is dropped
        mask |= ORACLE_M_CDI_DROP;
        for (int v = 0; v < nv; ++v) Fdi[v] = 0.0;
      }
    }
  }
  // --- phase-confined species diffusion (Eq. SpeciesMassDiffusion, last
  // form) with the species enthalpy flux of q.  reading: face values are
  // arithmetic means, gradients two-point, K_c = D_c W_c/W_p averaged once.
  S Fdf[16];
  for (int v = 0; v < nv; ++v) Fdf[v] = 0.0;
  if (c.diffusion) {
    const double dxn = c.dx[fa.d];
    const S rhob = 0.5 * (CL.th.rho + CR.th.rho);
    S eflux = 0.0;
    for (int p = 0; p < c.np; ++p) {
      if (c.pn[p] < 2) continue;
      S Yb[8], Kb[8], G[8], Yp = 0.0, sKG = 0.0;
      for (int a = 0; a < c.pn[p]; ++a) {
        const int k = c.pc[p][a];
        Yb[a] = 0.5 * (CL.th.Y[k] + CR.th.Y[k]);
        Kb[a] = 0.5 * (CL.K[k] + CR.K[k]);
        G[a] = (CR.chi[k] - CL.chi[k]) / dxn;
        Yp += Yb[a];
        sKG += Kb[a] * G[a];
      }
      for (int a = 0; a < c.pn[p]; ++a) {
        const int k = c.pc[p][a];
        const S J = -rhob * (Kb[a] * Yp * G[a] - Yb[a] * sKG);
        Fdf[k] = J;
        eflux += J * (0.5 * (CL.h[k] + CR.h[k]));
      }
    }
    Fdf[ns + c.dim] = eflux;
  }
  // --- viscous stress and heat conduction (Eq. DiffusionTerms), second-order
  // central: face mu, lambda and velocity the means of the two cells; normal
  // derivatives two-point, tangential derivatives the mean of the two cells'
  // central differences.  reading: the energy entry is -sum_i u_i tau_di +
  // q_d (the printed entry has both signs flipped against its momentum
  // entries -tau_di and against the energy balance), q_d = -lambda dT/dx_d +
  // the species enthalpy flux above.
  S Fv[16];
  for (int v = 0; v < nv; ++v) Fv[v] = 0.0;
  if (c.viscous) {
    const int d = fa.d;
    const double dxn = c.dx[d];
    S g[3][3];  // g[i][j] = du_i/dx_j at the face
    for (int i = 0; i < c.dim; ++i) g[i][d] = (CR.th.vel[i] - CL.th.vel[i]) / dxn;
    for (int t = 0; t < nt; ++t) {
      const int j = fa.t[t];
      for (int i = 0; i < c.dim; ++i)
        g[i][j] = ((tg[2 * t + 1][0]->th.vel[i] - tg[2 * t][0]->th.vel[i]) +
                   (tg[2 * t + 1][1]->th.vel[i] - tg[2 * t][1]->th.vel[i])) /
                  (4.0 * c.dx[j]);
    }
    S div = 0.0;
    for (int i = 0; i < c.dim; ++i) div += g[i][i];
    const S muf = 0.5 * (CL.mu + CR.mu), lamf = 0.5 * (CL.lam + CR.lam);
    S work = 0.0;
    for (int i = 0; i < c.dim; ++i) {
      S tau = muf * (g[d][i] + g[i][d]);
      if (i == d) tau -= muf * (2.0 / 3.0) * div;
      Fv[ns + i] = -tau;
      work += 0.5 * (CL.th.vel[i] + CR.th.vel[i]) * tau;
    }
    Fv[ns + c.dim] = -work - lamf * (CR.th.T - CL.th.T) / dxn;
  }
  for (int v = 0; v < nv; ++v) Fout[v] = F[v] + Fdi[v] + Fdf[v] + Fv[v];
}

// ---------------------------------------------------------------------------
// Characteristic boundary flux (Sec. 3.5 cites the Navier-Stokes
// characteristic boundary conditions of Thompson and of Poinsot & Lele
// without formulas; reading).  At a boundary face of direction d on side s
// (outward normal +e_d for s = 1, -e_d for s = 0) the face state is built in
// the characteristic variables of the method (S^-1 W of App. A, linearized
// at the boundary cell: T - cT P, Y_c, u_t with speed u_n; P/2 + (z/2) u_n
// with speed u_n + a; P/2 - (z/2) u_n with speed u_n - a).  A variable whose
// wave leaves the domain (speed along the outward normal > 0) takes the
// cell's value; an entering one takes the cell's value moved by the factor
// sigma toward the target's (sigma = 0: no entering wave, non-reflecting;
// sigma = 1: the target imposed).  The flux is the physical convective flux
// of that state; no regularization, diffusion or viscous flux crosses the
// face.
// ---------------------------------------------------------------------------
template <class S>
void characteristic_flux(const Conf& c, const FaceArgs& fa, const Cellq<S>& q, int side, S* F) {
  const Conf::Target& tg = c.target[fa.d][side];
  const int ns = c.ns, nt = c.dim - 1;
  const double sgn = side == 1 ? 1.0 : -1.0;
  const S cT = q.th.cT, z = q.th.z, a = q.th.a;
  const S un = q.th.vel[fa.d];
  const double unt = tg.vel[fa.d];
  auto relax = [&](const S& cell, const S& target, const S& speed) -> S {
    if (re(S(sgn * speed)) > 0.0) return cell;   // leaves the domain
    return cell + tg.sigma * (target - cell);
  };
  // entropy-like and advected variables (speed u_n)
  const S w0 = relax(q.th.T - cT * q.th.P, S(tg.T) - cT * tg.P, un);
  S Y[8], ut[2];
  for (int k = 0; k < ns; ++k) Y[k] = relax(q.th.Y[k], S(tg.Y[k]), un);
  for (int t = 0; t < nt; ++t) ut[t] = relax(q.th.vel[fa.t[t]], S(tg.vel[fa.t[t]]), un);
  // acoustic variables (speeds u_n + a, u_n - a)
  const S wp = relax(0.5 * q.th.P + 0.5 * z * un, 0.5 * tg.P + 0.5 * z * unt, S(un + a));
  const S wm = relax(0.5 * q.th.P - 0.5 * z * un, 0.5 * tg.P - 0.5 * z * unt, S(un - a));
  // back to W, then the state and its flux
  const S P = wp + wm;
  const S unb = (wp - wm) / z;
  const S T = w0 + cT * P;
  S vel[3], uu[16], rho, ab;
  vel[fa.d] = unb;
  for (int t = 0; t < nt; ++t) vel[fa.t[t]] = ut[t];
  state_from_PT(c, P, T, Y, vel, uu, rho, ab);
  Side<S> sd;
  sd.rho = rho;
  sd.un = unb;
  sd.P = P;
  sd.a = ab;
  sd.E = uu[ns + c.dim];
  for (int t = 0; t < nt; ++t) sd.ut[t] = ut[t];
  for (int k = 0; k < ns; ++k) sd.rY[k] = uu[k];
  S Ur[16], Fr[16];
  side_UF(c, sd, Ur, Fr);
  unrotate(c, fa, Fr, F);
}

// ---------------------------------------------------------------------------
// The solver object
// ---------------------------------------------------------------------------
struct Oracle {
  Conf c;
};

inline void face_dirs(const Conf& c, int d, int* t) {
  int o = 0;
  for (int k = 0; k < c.dim; ++k)
    if (k != d) t[o++] = k;
}

long face_count(const Conf& c, int d) {
  long f = 1;
  for (int k = 0; k < 3; ++k) f *= (c.n[k] + (k == d ? 1 : 0));
  return f;
}

// dt and Gamma from the state (Sec. 3.4 and 3.2).
// reading: dt = CFL / max over cells and directions of (|u_d| + a)/dx_d and,
// with diffusion or viscous terms on, 4 mu/(rho dx_d^2), mu = sum_p phi_p mu_p;
// Gamma = gamma_scale * max |u_d|, both from U^n and held for the 3 stages.
template <class S>
void compute_dt_gamma(const Conf& c, const S* U, double& dt, double& gam) {
  double m = 0.0, g = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m, g)
  for (long i = 0; i < c.ncell; ++i) {
    S u[16];
    Cellq<S> q;
    for (int v = 0; v < c.nv; ++v) u[v] = U[(long)v * c.ncell + i];
    cell_quantities(c, u, q);
    for (int d = 0; d < c.dim; ++d) {
      const double au = std::fabs(re(q.th.vel[d]));
      m = std::max(m, (au + re(q.th.a)) / c.dx[d]);
      if (c.diffusion || c.viscous) m = std::max(m, 4.0 * re(q.mu) / (re(q.th.rho) * c.dx[d] * c.dx[d]));
      g = std::max(g, au);
    }
  }
  dt = c.cfl / m;
  gam = c.gscale * g;
}

// L(U_k) (Eq. DiscreteGoverningEquations).
// ps_lo, ps_hi (nullable, [dim][nv][cells]): the flux limiter's
// pseudo-states of every interior cell at its low and high face of each
// direction, formed with the face's final flux; Fall (nullable): the final
// face fluxes, directions in order, [nv][faces_d] each.
template <class S>
void rhs(const Conf& c, const S* Uk, const S* Un, double rk0, double rk1, double rk2, double dt,
         double Gamma, S* L, uint16_t* mask, uint64_t* cnt, S* ps_lo = nullptr, S* ps_hi = nullptr,
         S* Fall = nullptr) {
  std::vector<S> Pk, Pn;
  fill_padded_s(c, Uk, Pk);
  fill_padded_s(c, Un, Pn);
  std::vector<Cellq<S>> Q((size_t)c.npad);
  bucket<S>(0);
#pragma omp parallel for schedule(static)
  for (long p = 0; p < c.npad; ++p) {
    S u[16];
    for (int v = 0; v < c.nv; ++v) u[v] = Pk[(size_t)v * c.npad + p];
    cell_quantities(c, u, Q[p]);
  }
  std::vector<std::vector<S>> Fd(c.dim);
  long moff = 0;
  uint64_t cnt_loc[ORACLE_NCNT] = {0, 0, 0, 0, 0, 0, 0};
  // failure detection: interior cells of the stage input that are not
  // admissible (Eqs. PositivityReqs1-2, NaN included); a check, not counted
  // as work of the method
  bucket<S>(-1);
  for (long i = 0; i < c.ncell; ++i) {
    S u[16];
    for (int v = 0; v < c.nv; ++v) u[v] = Uk[(long)v * c.ncell + i];
    if (!admissible(c, u)) cnt_loc[ORACLE_CNT_BAD_CELLS]++;
  }
  for (int d = 0; d < c.dim; ++d) {
    const long nf = face_count(c, d);
    Fd[d].assign((size_t)c.nv * nf, S(0.0));
    FaceArgs fa;
    fa.d = d;
    face_dirs(c, d, fa.t);
    fa.lam = 2.0 * c.dim * rk2 * dt / c.dx[d];
    fa.rk0 = rk0;
    fa.rk1 = rk1;
    fa.Gamma = Gamma;
    int e[3] = {c.n[0], c.n[1], c.n[2]};
    e[d] += 1;
    const long sd = (d == 0 ? 1 : (d == 1 ? c.N[0] : (long)c.N[0] * c.N[1]));
    long st[3] = {1, c.N[0], (long)c.N[0] * c.N[1]};
    uint64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0;
    bucket<S>(1 + d);
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : c0, c1, c2, c3, c4)
    for (int k = 0; k < e[2]; ++k)
      for (int j = 0; j < e[1]; ++j)
        for (int i = 0; i < e[0]; ++i) {
          // face between the cell (i,j,k) - e_d and (i,j,k)
          int ic[3] = {i, j, k};
          ic[d] -= 1;
          const long pL = c.pidx(ic[0], ic[1], ic[2]);
          const Cellq<S>* stv[6];
          for (int m = 0; m < 6; ++m) stv[m] = &Q[pL + (m - 2) * sd];
          S UnL[16], UnR[16];
          for (int v = 0; v < c.nv; ++v) {
            UnL[v] = Pn[(size_t)v * c.npad + pL];
            UnR[v] = Pn[(size_t)v * c.npad + pL + sd];
          }
          const Cellq<S>* tgp[4][2];
          for (int t = 0; t < c.dim - 1; ++t) {
            const long s = st[fa.t[t]];
            tgp[2 * t][0] = &Q[pL - s];
            tgp[2 * t][1] = &Q[pL + sd - s];
            tgp[2 * t + 1][0] = &Q[pL + s];
            tgp[2 * t + 1][1] = &Q[pL + sd + s];
          }
          S F[16];
          uint16_t m16 = 0;
          face_flux(c, fa, stv, UnL, UnR, tgp, F, m16);
          // characteristic boundaries replace the boundary face's flux
          if (ic[d] + 1 == 0 && c.bclo[d] == 3) {
            characteristic_flux(c, fa, *stv[3], 0, F);
            m16 = 0;
          } else if (ic[d] + 1 == c.n[d] && c.bchi[d] == 3) {
            characteristic_flux(c, fa, *stv[2], 1, F);
            m16 = 0;
          }
          const long fidx = ((long)k * e[1] + j) * e[0] + i;
          if (ps_lo) {
            S FcL[16], FcR[16], a[16], b[16];
            cell_flux(c, fa, *stv[2], FcL);
            cell_flux(c, fa, *stv[3], FcR);
            pseudo_pair(c, fa, stv[2]->u, UnL, FcL, stv[3]->u, UnR, FcR, F, a, b);
            const long blk = (long)d * c.nv * c.ncell;
            if (ic[d] >= 0) {
              const long ci = c.cidx(ic[0], ic[1], ic[2]);
              for (int v = 0; v < c.nv; ++v) ps_hi[blk + (long)v * c.ncell + ci] = a[v];
            }
            if (ic[d] + 1 < c.n[d]) {
              int ir[3] = {ic[0], ic[1], ic[2]};
              ir[d] += 1;
              const long ci = c.cidx(ir[0], ir[1], ir[2]);
              for (int v = 0; v < c.nv; ++v) ps_lo[blk + (long)v * c.ncell + ci] = b[v];
            }
          }
          for (int v = 0; v < c.nv; ++v) Fd[d][(size_t)v * nf + fidx] = F[v];
          if (mask) mask[moff + fidx] = m16;
          if (m16 & (ORACLE_M_TL | ORACLE_M_TR)) c0++;
          if (m16 & (ORACLE_M_PL | ORACLE_M_PR)) c1++;
          if (m16 & ORACLE_M_FALLBACK) c2++;
          if (m16 & ORACLE_M_CDI_DROP) c3++;
          if (m16 & ORACLE_M_UNRECOVERABLE) c4++;
        }
    cnt_loc[0] += c0;
    cnt_loc[1] += c1;
    cnt_loc[2] += c2;
    cnt_loc[3] += c3;
    cnt_loc[4] += c4;
    cnt_loc[5] += nf;
    if (Fall)
      for (size_t q = 0; q < (size_t)c.nv * nf; ++q) Fall[(size_t)c.nv * moff + q] = Fd[d][q];
    moff += nf;
  }
  // L_i = -sum_d (F_{i+1/2} - F_{i-1/2}) / dx_d
  bucket<S>(4);
  for (int k = 0; k < c.n[2]; ++k)
    for (int j = 0; j < c.n[1]; ++j)
      for (int i = 0; i < c.n[0]; ++i) {
        const long ci = c.cidx(i, j, k);
        for (int v = 0; v < c.nv; ++v) {
          S acc = 0.0;
          for (int d = 0; d < c.dim; ++d) {
            int e[3] = {c.n[0], c.n[1], c.n[2]};
            e[d] += 1;
            int ih[3] = {i, j, k};
            ih[d] += 1;
            const long flo = ((long)k * e[1] + j) * e[0] + i;
            const long fhi = ((long)ih[2] * e[1] + ih[1]) * e[0] + ih[0];
            const long nf = face_count(c, d);
            acc += (Fd[d][(size_t)v * nf + fhi] - Fd[d][(size_t)v * nf + flo]) / c.dx[d];
          }
          L[(long)v * c.ncell + ci] = -acc;
        }
      }
  bucket<S>(-1);
  if (cnt)
    for (int q = 0; q < ORACLE_NCNT; ++q) cnt[q] += cnt_loc[q];
}

// SSP-RK3 (Eq. SSPRK3) with coefficients (rk0, rk1, rk2) per stage.
const double RK[3][3] = {{0.0, 1.0, 1.0}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};

template <class S>
void rk3(const Conf& c, S* U, double dt, double Gamma, uint16_t* masks, uint64_t* cnt) {
  const size_t n = (size_t)c.nv * c.ncell;
  std::vector<S> Un(U, U + n), Uk(U, U + n), L(n);
  long per_stage = 0;
  for (int d = 0; d < c.dim; ++d) per_stage += face_count(c, d);
  for (int s = 0; s < 3; ++s) {
    rhs(c, Uk.data(), Un.data(), RK[s][0], RK[s][1], RK[s][2], dt, Gamma, L.data(),
        masks ? masks + s * per_stage : nullptr, cnt);
    for (size_t i = 0; i < n; ++i) Uk[i] = RK[s][0] * Un[i] + RK[s][1] * Uk[i] + RK[s][2] * dt * L[i];
    // inflow cells are set back to their prescribed state after every stage
    const size_t nh = c.held.size();
    for (size_t k = 0; k < nh; ++k)
      for (int v = 0; v < c.nv; ++v) Uk[(size_t)v * c.ncell + c.held[k]] = S(c.held_U[v * nh + k]);
  }
  for (size_t i = 0; i < n; ++i) U[i] = Uk[i];
}

int setup(const oracle_grid* g, const oracle_eos* e, const oracle_opts* o, Conf& c) {
  if (!g || !e || !o) return -1;
  if (g->dim < 1 || g->dim > 3) return -1;
  c.dim = g->dim;
  for (int d = 0; d < 3; ++d) {
    c.n[d] = d < c.dim ? g->n[d] : 1;
    c.dx[d] = g->dx[d];
    c.bclo[d] = g->bc_lo[d];
    c.bchi[d] = g->bc_hi[d];
    if (d < c.dim && (c.n[d] < 1 || !(c.dx[d] > 0))) return -1;
    if (d < c.dim && (c.bclo[d] == 2 || c.bchi[d] == 2) && c.n[d] < 3) return -1;
    if (d < c.dim && (c.bclo[d] < 0 || c.bclo[d] > 3 || c.bchi[d] < 0 || c.bchi[d] > 3)) return -1;
    c.g[d] = d < c.dim ? 3 : 0;
    c.N[d] = c.n[d] + 2 * c.g[d];
  }
  c.ncell = (long)c.n[0] * c.n[1] * c.n[2];
  c.npad = (long)c.N[0] * c.N[1] * c.N[2];
  c.ns = e->n_species;
  if (c.ns < 1 || c.ns > 8) return -1;
  c.nv = c.ns + c.dim + 1;
  double pst = 0.0;
  int seen[2] = {0, 0};
  for (int k = 0; k < c.ns; ++k) {
    c.ph[k] = e->phase[k];
    c.cv[k] = e->cv[k];
    c.gam[k] = e->gamma[k];
    c.pinf[k] = e->pinf[k];
    c.b[k] = e->b[k];
    c.q[k] = e->q[k];
    c.W[k] = e->molar_mass[k];
    c.mu[k] = e->mu[k];
    c.Sc[k] = e->Sc[k];
    c.lamc[k] = e->lambda[k];
    if (c.ph[k] != 0 && c.ph[k] != 1) return -1;
    seen[c.ph[k]] = 1;
    if (c.pinf[k] != 0.0) {
      if (pst != 0.0 && pst != c.pinf[k]) c.multi = 1;  // the iterative solve
      pst = std::max(pst, c.pinf[k]);
    }
  }
  c.Pst = pst;
  c.np = 0;
  for (int p = 0; p < 2; ++p)
    if (seen[p]) {
      c.pid[c.np] = p;
      c.pn[c.np] = 0;
      for (int k = 0; k < c.ns; ++k)
        if (c.ph[k] == p) c.pc[c.np][c.pn[c.np]++] = k;
      c.np++;
    }
  c.cfl = o->cfl;
  c.cdi = o->cdi;
  c.eps = o->eps_cdi;
  c.phimin = o->phi_min;
  c.delta = o->delta;
  c.gscale = o->gamma_scale;
  c.diffusion = o->diffusion;
  c.positivity = o->positivity;
  c.weps = o->weno_eps;
  c.wp = o->weno_p;
  c.viscous = o->viscous;
  c.Pr = o->prandtl;
  if (c.viscous && !(c.Pr > 0)) return -1;
  if (o->weno < 0) return -1;
  if (o->weno > 3) return -5;
  c.weno = o->weno;
  if (o->basis < 0) return -1;
  if (o->basis > 1) return -5;
  c.basis = o->basis;
  if (c.cdi && !(c.eps > 0)) return -1;
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void* oracle_create(const oracle_grid* g, const oracle_eos* e, const oracle_opts* o, int* status) {
  Oracle* h = new Oracle;
  int s = setup(g, e, o, h->c);
  if (status) *status = s;
  if (s != 0) {
    delete h;
    return nullptr;
  }
  return h;
}

void oracle_destroy(void* h) { delete (Oracle*)h; }

int oracle_init_state(void* hh, const double* phi, const double* y, const double* P,
                      const double* T, const double* vel, double* U) {
  const Conf& c = ((Oracle*)hh)->c;
  for (long i = 0; i < c.ncell; ++i) {
    const double p = P[i], t = T[i];
    double rho = 0.0, rhoe = 0.0;
    double rY[8];
    for (int pp = 0; pp < c.np; ++pp) {
      const int pid = c.pid[pp];
      double vp = 0.0;
      for (int a = 0; a < c.pn[pp]; ++a) {
        const int k = c.pc[pp][a];
        vp += y[(long)k * c.ncell + i] * spec_vol(c, k, p, t);
      }
      const double rhop = 1.0 / vp;
      for (int a = 0; a < c.pn[pp]; ++a) {
        const int k = c.pc[pp][a];
        rY[k] = phi[(long)pid * c.ncell + i] * rhop * y[(long)k * c.ncell + i];
      }
    }
    for (int k = 0; k < c.ns; ++k) {
      U[(long)k * c.ncell + i] = rY[k];
      rho += rY[k];
      rhoe += rY[k] * spec_energy(c, k, p, t);
    }
    double ke = 0.0;
    for (int d = 0; d < c.dim; ++d) {
      const double vd = vel[(long)d * c.ncell + i];
      U[(long)(c.ns + d) * c.ncell + i] = rho * vd;
      ke += vd * vd;
    }
    U[(long)(c.ns + c.dim) * c.ncell + i] = rhoe + 0.5 * rho * ke;
  }
  return 0;
}

int oracle_compute_dt(void* hh, const double* U, double* dt, double* gamma) {
  const Conf& c = ((Oracle*)hh)->c;
  double a, b;
  compute_dt_gamma(c, U, a, b);
  if (dt) *dt = a;
  if (gamma) *gamma = b;
  return 0;
}

// ORACLE_EINADMISSIBLE when the counters of one call show an inadmissible
// stage input cell or an unrecoverable face.
static int status_of(const uint64_t* cnt) {
  return (cnt[ORACLE_CNT_UNRECOVERABLE] || cnt[ORACLE_CNT_BAD_CELLS]) ? ORACLE_EINADMISSIBLE : 0;
}

int oracle_rhs(void* hh, const double* Uk, const double* Un, double rk0, double rk1, double rk2,
               double dt, double gamma, double* L, uint16_t* mask, uint64_t* counters) {
  const Conf& c = ((Oracle*)hh)->c;
  uint64_t cnt[ORACLE_NCNT] = {0, 0, 0, 0, 0, 0, 0};
  rhs(c, Uk, Un, rk0, rk1, rk2, dt, gamma, L, mask, cnt);
  if (counters)
    for (int q = 0; q < ORACLE_NCNT; ++q) counters[q] += cnt[q];
  return status_of(cnt);
}

int oracle_pseudo_states(void* hh, const double* Uk, const double* Un, double rk0, double rk1,
                         double rk2, double dt, double gamma, double* L, double* lo, double* hi,
                         double* F) {
  const Conf& c = ((Oracle*)hh)->c;
  uint64_t cnt[ORACLE_NCNT] = {0, 0, 0, 0, 0, 0, 0};
  rhs(c, Uk, Un, rk0, rk1, rk2, dt, gamma, L, nullptr, cnt, lo, hi, F);
  return status_of(cnt);
}

int oracle_rk3_step(void* hh, double* U, const double* dt_in, const double* gamma_in,
                    double* dt_out, double* gamma_out, uint16_t* masks, uint64_t* counters) {
  const Conf& c = ((Oracle*)hh)->c;
  double dt, g;
  compute_dt_gamma(c, U, dt, g);
  if (dt_in) dt = *dt_in;
  if (gamma_in) g = *gamma_in;
  uint64_t cnt[ORACLE_NCNT] = {0, 0, 0, 0, 0, 0, 0};
  rk3(c, U, dt, g, masks, cnt);
  if (counters)
    for (int q = 0; q < ORACLE_NCNT; ++q) counters[q] += cnt[q];
  if (dt_out) *dt_out = dt;
  if (gamma_out) *gamma_out = g;
  return status_of(cnt);
}

// Inflow cells held at fixed conserved values through every RK stage (the
// water inlet of the Mach-100 water column, Sec. 4.2.4; the paper's NSCBC
// inflow is defined only in its references).  idx: count distinct cell
// indices; U: [nv][count].  count 0 clears.  Returns -1 on a bad index.
// Target state and relaxation factor of the characteristic boundary on side
// `side` (0 low, 1 high) of direction d: pressure P, temperature T, mass
// fractions Y[ns], velocity vel[dim], sigma in [0, 1].  Returns -1 on a bad
// argument (the side not characteristic, sigma outside [0, 1], T <= 0, a
// negative or non-normalized Y, P + P_inf <= 0 for a component present).
int oracle_set_boundary_target(void* hh, int d, int side, double P, double T, const double* Y,
                               const double* vel, double sigma) {
  Conf& c = ((Oracle*)hh)->c;
  if (d < 0 || d >= c.dim || (side != 0 && side != 1) || !Y || !vel) return -1;
  if ((side == 0 ? c.bclo[d] : c.bchi[d]) != 3) return -1;
  if (!(sigma >= 0.0 && sigma <= 1.0) || !(T > 0.0) || !std::isfinite(P)) return -1;
  double sy = 0.0;
  for (int k = 0; k < c.ns; ++k) {
    if (!(Y[k] >= 0.0)) return -1;
    if (Y[k] > 0.0 && !(P + c.pinf[k] > 0.0)) return -1;
    sy += Y[k];
  }
  if (std::fabs(sy - 1.0) > 1e-12) return -1;
  Conf::Target& t = c.target[d][side];
  t.P = P;
  t.T = T;
  for (int k = 0; k < c.ns; ++k) t.Y[k] = Y[k];
  for (int e = 0; e < 3; ++e) t.vel[e] = e < c.dim ? vel[e] : 0.0;
  t.sigma = sigma;
  return 0;
}

int oracle_set_held(void* hh, long count, const long* idx, const double* U) {
  Conf& c = ((Oracle*)hh)->c;
  if (count < 0 || (count > 0 && (!idx || !U))) return -1;
  std::vector<char> seen(c.ncell, 0);
  for (long k = 0; k < count; ++k) {
    if (idx[k] < 0 || idx[k] >= c.ncell || seen[idx[k]]) return -1;
    seen[idx[k]] = 1;
  }
  c.held.assign(idx, idx + count);
  c.held_U.assign(U, U + (size_t)c.nv * count);
  return 0;
}

int oracle_jvp_rk3_step(void* hh, const double* U, const double* dU, double dt, double gamma,
                        double* U_out, double* dU_out) {
  const Conf& c = ((Oracle*)hh)->c;
  const size_t n = (size_t)c.nv * c.ncell;
  const double h = 1e-30;
  std::vector<cplx> Uc(n);
  for (size_t i = 0; i < n; ++i) Uc[i] = cplx(U[i], h * dU[i]);
  rk3(c, Uc.data(), dt, gamma, nullptr, nullptr);
  for (size_t i = 0; i < n; ++i) {
    U_out[i] = Uc[i].real();
    dU_out[i] = Uc[i].imag() / h;
  }
  return 0;
}

int oracle_jvp_rhs(void* hh, const double* Uk, const double* dUk, const double* Un, double rk0,
                   double rk1, double rk2, double dt, double gamma, double* L, double* dL) {
  const Conf& c = ((Oracle*)hh)->c;
  const size_t n = (size_t)c.nv * c.ncell;
  const double h = 1e-30;
  std::vector<cplx> Ukc(n), Unc(n), Lc(n);
  for (size_t i = 0; i < n; ++i) {
    Ukc[i] = cplx(Uk[i], h * dUk[i]);
    Unc[i] = cplx(Un[i], 0.0);
  }
  rhs(c, Ukc.data(), Unc.data(), rk0, rk1, rk2, dt, gamma, Lc.data(), nullptr, nullptr);
  for (size_t i = 0; i < n; ++i) {
    L[i] = Lc[i].real();
    dL[i] = Lc[i].imag() / h;
  }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int oracle_count_ops(void* hh, const double* U, double dt, double gamma, long* out) {
  const Conf& c = ((Oracle*)hh)->c;
  const size_t n = (size_t)c.nv * c.ncell;
  std::vector<Cnt> Uc(U, U + n), L(n);
#ifdef _OPENMP
  const int nt = omp_get_max_threads();
  omp_set_num_threads(1);
#endif
  for (int b = 0; b < 8; ++b) g_bucket[b] = 0;
  rhs(c, Uc.data(), Uc.data(), 0.0, 1.0, 1.0, dt, gamma, L.data(), nullptr, nullptr);
#ifdef _OPENMP
  omp_set_num_threads(nt);
#endif
  for (int b = 0; b < 8; ++b) out[b] = g_bucket[b];
  out[5] = c.npad;
  return 0;
}

int oracle_cell_equilibrium(void* hh, const double* u, double* out) {
  const Conf& c = ((Oracle*)hh)->c;
  Thermo<double> t;
  equilibrium(c, u, t);
  out[0] = t.P; out[1] = t.T; out[2] = t.a; out[3] = t.rho; out[4] = t.beta;
  out[5] = t.alpha; out[6] = t.cT; out[7] = t.z; out[8] = t.e;
  return 0;
}

int oracle_state_from_PT(void* hh, double P, double T, const double* Y, const double* vel,
                         double* u_out, double* a_out) {
  const Conf& c = ((Oracle*)hh)->c;
  double rho, a;
  state_from_PT(c, P, T, Y, vel, u_out, rho, a);
  if (a_out) *a_out = a;
  return 0;
}

double oracle_weno5js(const double* f, double eps, int p) {
  return weno5js(f[0], f[1], f[2], f[3], f[4], eps, p);
}

double oracle_teno5(const double* f, double eps) { return teno5(f[0], f[1], f[2], f[3], f[4], eps); }
double oracle_teno6(const double* f, double eps, double* tau_out) {
  return teno6(f[0], f[1], f[2], f[3], f[4], f[5], eps, tau_out);
}

// Jiang-Shu indicator of the polynomial matching n cell averages f[0..n-1]
// on cells off..off+n-1 around the target cell [-1/2, 1/2]; *face receives
// its value at x = 1/2.
double oracle_js_indicator(const double* f, int off, int n, double* face) {
  if (n < 1 || n > 6) return -1.0;
  double a[6];
  poly_from_averages(f, off, n, a);
  if (face) *face = poly_at_face(a, n);
  return js_indicator(a, n);
}

double oracle_weno5z(const double* f, double eps, int p) {
  return weno5z(f[0], f[1], f[2], f[3], f[4], eps, p);
}

int oracle_ylimit(int ns, double* Ys, const double* Yc) { return ylimit(ns, Ys, Yc); }

int oracle_hllc(void* hh, const double* uL, const double* uR, double* F) {
  const Conf& c = ((Oracle*)hh)->c;
  FaceArgs fa;
  fa.d = 0;
  face_dirs(c, 0, fa.t);
  Cellq<double> qL, qR;
  cell_quantities(c, uL, qL);
  cell_quantities(c, uR, qR);
  Side<double> sL, sR;
  make_side_from_cell(c, qL, fa, sL);
  make_side_from_cell(c, qR, fa, sR);
  double Fr[16];
  hllc(c, sL, sR, Fr);
  unrotate(c, fa, Fr, F);
  return 0;
}

int oracle_euler_flux(void* hh, const double* u, double* F) {
  const Conf& c = ((Oracle*)hh)->c;
  FaceArgs fa;
  fa.d = 0;
  face_dirs(c, 0, fa.t);
  Cellq<double> q;
  cell_quantities(c, u, q);
  Side<double> s;
  make_side_from_cell(c, q, fa, s);
  double Ur[16], Fr[16];
  side_UF(c, s, Ur, Fr);
  unrotate(c, fa, Fr, F);
  return 0;
}

int oracle_admissible(void* hh, const double* u) {
  const Conf& c = ((Oracle*)hh)->c;
  return admissible(c, u) ? 1 : 0;
}

int oracle_cell_aux(void* hh, const double* u, double* out) {
  const Conf& c = ((Oracle*)hh)->c;
  Cellq<double> q;
  cell_quantities(c, u, q);
  for (int i = 0; i < 9; ++i) out[i] = 0.0;
  for (int p = 0; p < c.np; ++p) {
    const int pid = c.pid[p];
    out[0 + pid] = q.phi[p];
    out[2 + pid] = q.psi[p];
    out[4 + pid] = q.rhop[p];
    out[6 + pid] = q.hrho[p];
  }
  out[8] = q.mu;
  return 0;
}

double oracle_wilke(void* hh, int p, const double* y) {
  const Conf& c = ((Oracle*)hh)->c;
  for (int pp = 0; pp < c.np; ++pp)
    if (c.pid[pp] == p) return wilke(c, pp, y);
  return -1.0;
}

}  // extern "C"
