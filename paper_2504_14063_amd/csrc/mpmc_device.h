// mpmc_device.h -- device arithmetic of the four-equation MPMC hot path
// (Collis, Bezgin, Mirjalili & Mani, arXiv 2504.14063) for gfx950.
//
// Everything here is __device__ code templated on the number of components
// NS and of directions DIM (compile-time, so per-component loops unroll into
// registers) and, for the face pipeline, on the arithmetic type R (double for
// the FP64 form, float for the light parts of the mixed form).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define MPMC_HD __host__ __device__ __forceinline__

#include "mpmc_dual.h"

namespace mpmc {

using ::fabs;
using ::log;
using ::sqrt;
using ::tanh;

constexpr int MAXS = 8;  // components of the component table
// components up to which every form is built (FP64, mixed, fused layout,
// frozen-decision replay, adjoint); above it the FP64 forward only
constexpr int kFullNS = 3;

// Kernel parameters, passed by value (kernarg segment, scalar loads).
struct Params {
  int ns, dim, nv, np;
  int n[3];
  int bclo[3], bchi[3];
  long ncell;
  double dx[3], idx[3];
  int phase[MAXS];          // phase id per component (0 liquid, 1 gas)
  int pn[2];                // components in present phase p (p = 0 first)
  int pid[2];               // phase id of present phase p
  double inpn[2];           // 1 / pn
  double cv[MAXS], gam[MAXS], pinf[MAXS], b[MAXS], q[MAXS], W[MAXS], mu[MAXS], Sc[MAXS];
  double lamc[MAXS];        // heat conductivity of a liquid component
  double iPr;               // 1 / Prandtl number of the gas phase
  double gm1cv[MAXS];       // (gamma - 1) C_v
  double gcv[MAXS];         // gamma C_v = C_P
  double stiff[MAXS];       // 1 where P_inf != 0
  double inP[MAXS];         // 1 where the component belongs to present phase 0
  double Pst;               // the common non-zero P_inf (0 if none; the largest if several)
  int pgen;                 // several distinct non-zero P_inf: iterative pressure
  int stream;               // 1: the cell arrays far exceed the caches (the
                            // streamed loads and every store carry the
                            // non-temporal hint)
  double wilke[MAXS][MAXS]; // (W_i / W_j) Phi_ij
  int multi[2];             // phase p has >= 2 components
  double cfl, eps, phimin, delta, gscale, weps;
  double sharp_floor;       // 4 phi_min (1 - phi_min)
  int wp, cdi, diff, pos, visc;
  int scheme;               // 0 WENO5-Z, 1 WENO5-JS, 2 TENO5, 3 TENO6
  int basis;                // 0 characteristic [T, Y, u, P]; 1 [rho Y, u, P]
  // layout of the cell-quantity array Q[nq][ncell]
  int qT, qP, qY, qU, qRho, qA, qPhi0, qPhi1, qPsi, qYrho, qHrho, qChi, qK, qH, qMu, qLam, nq;
  // characteristic boundaries (type 3): per direction and side (0 low, 1
  // high) the target state and the relaxation factor sigma of the entering
  // characteristic variables
  double tgP[3][2], tgT[3][2], tgY[3][2][MAXS], tgV[3][2][3], tgSig[3][2];
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Element i of one row of a [rows][cells] FP64 array, addressed as the row's
// base plus a 32-bit byte offset: on the device a raw buffer load or store
// whose descriptor (built from the row's base, the same for the whole
// wavefront) sits in scalar registers, so no lane does 64-bit address
// arithmetic and the byte offsets of a stencil serve every row it reads.
// Needs i * 8 < 2^32: grids of at most 2^29 cells and faces per direction
// (checked at init).
#ifdef __HIP_DEVICE_COMPILE__
typedef unsigned BufU2 __attribute__((vector_size(8)));
// descriptor word 3 of the gfx9 family: 32-bit data format, no swizzle
constexpr int kBufWord3 = 0x00020000;
// cache-policy operand of the buffer builtins: the non-temporal (streaming) bit
constexpr int kBufNonTemporal = 2;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const double* row) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(row), 0, -1, kBufWord3);
}
#endif
MPMC_HD double ldrow(const double* __restrict__ row, int i) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row), (int)((unsigned)i * 8u), 0, 0));
#else
  return row[i];
#endif
}
// A load of data that the launch reads once, and a store: with `nt` (the
// cell arrays far exceed the caches) both carry the non-temporal hint, since
// what one launch writes is read back by a later one after more data than
// the caches hold has passed through them; below that size the hint would
// only evict lines that the next launch reads.
template <bool NT>
MPMC_HD double ldrow_t(const double* __restrict__ row, int i) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_bit_cast(
      double, __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row), (int)((unsigned)i * 8u), 0, NT ? kBufNonTemporal : 0));
#else
  return row[i];
#endif
}
template <bool NT>
MPMC_HD void strow_t(double* __restrict__ row, int i, double v) {
#ifdef __HIP_DEVICE_COMPILE__
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufU2, v), row_rsrc(row), (int)((unsigned)i * 8u), 0,
                                        NT ? kBufNonTemporal : 0);
#else
  row[i] = v;
#endif
}
// the same with the hint chosen at run time (a uniform branch per access;
// blocks of many accesses branch once and call the forms above)
MPMC_HD double ldrow_s(const double* __restrict__ row, int i, bool nt) {
  return nt ? ldrow_t<true>(row, i) : ldrow_t<false>(row, i);
}
MPMC_HD void strow(double* __restrict__ row, int i, double v, bool nt) {
  if (nt)
    strow_t<true>(row, i, v);
  else
    strow_t<false>(row, i, v);
}
// cell-quantity bytes above which the arrays count as streamed (the size of
// MI355X's last-level Infinity Cache)
constexpr long kStreamBytes = 256L << 20;
constexpr long kMaxCells = 1L << 29;

MPMC_HD int map_index(int i, int n, int lo, int hi, bool& flip) {
  if (i < 0) {
    if (lo == 0) {
      do i += n; while (i < 0);  // stencil offsets are at most 3
      return i;
    }
    if (lo == 1 || lo == 3) return 0;  // zero-gradient (characteristic: for the stencils)
    flip = !flip;
    return -1 - i;
  }
  if (i >= n) {
    if (hi == 0) {
      do i -= n; while (i >= n);
      return i;
    }
    if (hi == 1 || hi == 3) return n - 1;
    flip = !flip;
    return 2 * n - 1 - i;
  }
  return i;
}

template <class R> MPMC_HD R rmin(R a, R b) { return b < a ? b : a; }
template <class R> MPMC_HD R rmax(R a, R b) { return b > a ? b : a; }

// ---------------------------------------------------------------------------
// Component EOS, Eq. NASG_EOS:
//   v_c = kappa_c(P) T + b_c,  kappa_c = (gamma_c - 1) C_v,c / (P + P_inf,c)
//   e_c = eps_c(P) T + q_c,    eps_c   = C_v,c (P + gamma_c P_inf,c)/(P + P_inf,c)
//   h_c = C_P,c T + b_c P + q_c
// ---------------------------------------------------------------------------
template <class R>
MPMC_HD R kappa_c(const Params& p, int k, R P) {
  return (R)p.gm1cv[k] / (P + (R)p.pinf[k]);
}
template <class R>
MPMC_HD R epsT_c(const Params& p, int k, R P) {
  if (p.pinf[k] == 0.0) return (R)p.cv[k];
  return (R)p.cv[k] * (P + (R)(p.gam[k] * p.pinf[k])) / (P + (R)p.pinf[k]);
}

// Equilibrium sound speed, Eq. SpeedOfSound with the NASG beta and alpha;
// ipp[k] = 1/(P + P_inf,k).
template <int NS, class R>
MPMC_HD void sound(const Params& p, R rho, const R* Y, const R* ipp, R T, R& a,
                                      R& beta, R& alpha) {
  R sb = 0, sa = 0, Cp = 0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const R kp = (R)p.gm1cv[k] * ipp[k];
    sa += Y[k] * kp;
    sb += Y[k] * kp * ipp[k];
    Cp += Y[k] * (R)p.gcv[k];
  }
  sb *= T;
  beta = rho * sb;
  alpha = rho * sa;
  const R a2 = Cp / (rho * beta * Cp - alpha * alpha * T);
  a = sqrt(a2);
}

// ---------------------------------------------------------------------------
// Pressure-temperature equilibrium of a conserved state u[NV] (Sec. 2.3):
// closed form Eq. NASG_P (cancellation-free root), T from Eq. NASG_T1, then
// the sound speed and the eigenvector coefficients of App. A.  Always FP64.
// ---------------------------------------------------------------------------
template <int NS, int DIM, class S> struct ThermoT {
  S rho, Y[NS], vel[DIM], e, P, T, a, beta, alpha, cT, z;
};
template <int NS, int DIM> using Thermo = ThermoT<NS, DIM, double>;

// ---------------------------------------------------------------------------
// Pressure with several distinct P_inf (Sec. 2.3: the temperatures of Eqs.
// NASG_T1 and NASG_T2 equated, solved iteratively):
//   F(P) = (v - b) C_v - sum_c A_c / (P + P_inf,c) = 0,
//   A_c = Y_c (gamma_c - 1) C_v,c (e - q - (v - b) P_inf,c),
// the largest root above P_lo = max over present components of -P_inf,c.
// Above P_lo + 2 sum|A_c| / ((v - b) C_v) the sum is below half the constant,
// so F > 0 there and no root lies beyond.  Newton's method runs from that
// point on G(P) = (P - P_lo) F(P) (same roots; the pole at P_lo removed, so
// G is close to linear in a gas-liquid mixture) and is kept inside the
// bracket by bisection.  Every loop is bounded.  Duals get their tangent
// from one Newton step of F at the root.  NaN if the iteration ends away from
// a root (no admissible pressure).
// ---------------------------------------------------------------------------
template <int NS, class S>
MPMC_HD S pressure_general(const Params& p, const S* Y, S emq, S vmb) {
  S As[NS], Cv = 0.0;
  double A[NS], Plo = -1e300, sumA = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    Cv += Y[k] * p.cv[k];
    As[k] = Y[k] * p.gm1cv[k] * (emq - vmb * p.pinf[k]);
    A[k] = val(As[k]);
    sumA += fabs(A[k]);
    if (val(Y[k]) > 0.0) Plo = fmax(Plo, -p.pinf[k]);
  }
  const double C = val(S(vmb * Cv));
  auto F = [&](double P, double& dF) {
    double f = C;
    dF = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double w = 1.0 / (P + p.pinf[k]);
      f -= A[k] * w;
      dF += A[k] * w * w;
    }
    return f;
  };
  double lo = Plo, hi = Plo + fmax(2.0 * sumA / C, 1e-300), P = hi, dF;
  for (int it = 0; it < 200; ++it) {
    const double x = P - Plo;
    const double f = F(P, dF);
    if (f < 0.0)
      lo = P;
    else
      hi = P;
    const double G = x * f, dG = f + x * dF;
    double Pn = P - G / dG;
    if (!(Pn > lo && Pn < hi)) Pn = 0.5 * (lo + hi);
    const bool done = fabs(Pn - P) <= 4e-16 * fabs(Pn) || !(hi > lo);
    P = Pn;
    if (done) break;
  }
  // a root: G small against the size of its terms (else no sign change)
  const double fr = F(P, dF);
  if (!(fabs((P - Plo) * fr) <= 1e-10 * (C * fabs(P - Plo) + sumA))) return S(__builtin_nan(""));
  S Fs = vmb * Cv;
#pragma unroll
  for (int k = 0; k < NS; ++k) Fs -= As[k] / (P + p.pinf[k]);
  return S(P) - (Fs - val(Fs)) / dF;
}

template <int NS, int DIM, class S, bool GEN = false>
MPMC_HD void equilibrium_t(const Params& p, const S* u, ThermoT<NS, DIM, S>& t, bool coeffs) {
  S rho = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) rho += u[k];
  t.rho = rho;
#pragma unroll
  for (int k = 0; k < NS; ++k) t.Y[k] = u[k] / rho;
  S ke = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    t.vel[d] = u[NS + d] / rho;
    ke += 0.5 * u[NS + d] * t.vel[d];
  }
  t.e = (u[NS + DIM] - ke) / rho;
  const S v = 1.0 / rho;
  S qm = 0.0, bm = 0.0, Cv = 0.0, R1 = 0.0, Rg = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    qm += t.Y[k] * p.q[k];
    bm += t.Y[k] * p.b[k];
    Cv += t.Y[k] * p.cv[k];
    if (p.pinf[k] != 0.0)
      R1 += t.Y[k] * p.gm1cv[k];
    else
      Rg += t.Y[k] * p.gm1cv[k];
  }
  const double Pinf = p.Pst;
  const S Ep = (t.e - qm) / (v - bm);
  const S a1 = Cv;
  const S a2 = Ep * (R1 + Rg) - Pinf * (Cv + R1);
  const S a3 = Ep * Pinf * Rg;
  S P;
  if (GEN && p.pgen) {
    P = pressure_general<NS, S>(p, t.Y, S(t.e - qm), S(v - bm));
  } else if (val(Rg) == 0.0) {
    P = a2 / a1;
  } else {
    const S sD = sqrt(a2 * a2 + 4.0 * a1 * a3);
    P = val(a2) >= 0.0 ? S((a2 + sD) / (2.0 * a1)) : S(2.0 * a3 / (sD - a2));
  }
  t.P = P;
  S ipp[NS];
  S den = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    ipp[k] = 1.0 / (P + p.pinf[k]);
    // eps_c(P) = C_v (P + gamma P_inf) / (P + P_inf)
    den += t.Y[k] * (p.pinf[k] == 0.0 ? S(p.cv[k]) : S(p.cv[k] * (P + p.gam[k] * p.pinf[k]) * ipp[k]));
  }
  t.T = (t.e - qm) / den;
  sound<NS, S>(p, rho, t.Y, ipp, t.T, t.a, t.beta, t.alpha);
  if (coeffs) {
    const S a2s = t.a * t.a;
    t.cT = (rho * a2s * t.beta - 1.0) / (t.alpha * a2s * rho);
    t.z = t.a * rho;
  }
}

template <int NS, int DIM, bool GEN = false>
MPMC_HD void equilibrium(const Params& p, const double* u, Thermo<NS, DIM>& t, bool coeffs) {
  equilibrium_t<NS, DIM, double, GEN>(p, u, t, coeffs);
}

// ---------------------------------------------------------------------------
// WENO5-Z (Borges et al.): value at i+1/2 from f_{i-2..i+2}.
// ---------------------------------------------------------------------------
template <class R>
MPMC_HD R weno5z(R f0, R f1, R f2, R f3, R f4, R eps, int pw) {
  const R s6 = (R)(1.0 / 6.0);
  const R q0 = ((R)2 * f0 - (R)7 * f1 + (R)11 * f2) * s6;
  // the two inner candidates as 5 centre + (2 inner - outer): the mirrored
  // reconstruction's candidates 1 and 2 are this one's 2 and 1, formed once
  const R q1 = ((R)5 * f2 + ((R)2 * f3 - f1)) * s6;
  const R q2 = ((R)5 * f3 + ((R)2 * f2 - f4)) * s6;
  // the curvatures as (outer sum) - 2 centre: symmetric in the outer
  // values, so the mirrored reconstruction of the other face side shares two
  // of its three with this one
  const R t0 = (f0 + f2) - (R)2 * f1, s0 = f0 - (R)4 * f1 + (R)3 * f2;
  const R t1 = (f1 + f3) - (R)2 * f2, s1 = f1 - f3;
  const R t2 = (f2 + f4) - (R)2 * f3, s2 = (R)3 * f2 - (R)4 * f3 + f4;
  const R c13 = (R)(13.0 / 12.0);
  const R b0 = c13 * t0 * t0 + (R)0.25 * s0 * s0 + eps;
  const R b1 = c13 * t1 * t1 + (R)0.25 * s1 * s1 + eps;
  const R b2 = c13 * t2 * t2 + (R)0.25 * s2 * s2 + eps;
  const R tau = fabs(b0 - b2);
  R a0, a1, a2;
  if constexpr (!std::is_same<R, float>::value) {
    // alpha_k = d_k (1 + (tau/b_k)^p): scaled by prod_j b_j^p, one division
    if (pw == 2) {
      const R B0 = b0 * b0, B1 = b1 * b1, B2 = b2 * b2, T2 = tau * tau;
      a0 = (R)0.1 * (B0 + T2) * (B1 * B2);
      a1 = (R)0.6 * (B1 + T2) * (B0 * B2);
      a2 = (R)0.3 * (B2 + T2) * (B0 * B1);
    } else {
      a0 = (R)0.1 * (b0 + tau) * (b1 * b2);
      a1 = (R)0.6 * (b1 + tau) * (b0 * b2);
      a2 = (R)0.3 * (b2 + tau) * (b0 * b1);
    }
  } else {
    // FP32: hardware reciprocal for the weights (products would overflow)
#if defined(__HIP_DEVICE_COMPILE__)
    R r0 = tau * __builtin_amdgcn_rcpf(b0), r1 = tau * __builtin_amdgcn_rcpf(b1),
      r2 = tau * __builtin_amdgcn_rcpf(b2);
#else
    R r0 = tau / b0, r1 = tau / b1, r2 = tau / b2;
#endif
    if (pw == 2) {
      r0 *= r0;
      r1 *= r1;
      r2 *= r2;
    }
    a0 = (R)0.1 * ((R)1 + r0);
    a1 = (R)0.6 * ((R)1 + r1);
    a2 = (R)0.3 * ((R)1 + r2);
  }
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Mixed-precision WENO5-Z: the nonlinear weights in FP32 (smoothness
// indicators from FP64 undivided differences), the candidate values q_k and
// the combination in FP64, written relative to the candidate of largest
// weight m: q_m + sum_{k != m} w_k (q_k - q_m).  FP32 errors of the weights
// then multiply only the smaller weights, and constant data is reproduced
// exactly.  eps is raised to at least 1e-30 (FP32 range).
MPMC_HD float mixed_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
MPMC_HD double weno5z_mixed(double f0, double f1, double f2, double f3, double f4, float eps, int pw) {
  const double s6 = 1.0 / 6.0;
  const double q0 = (2.0 * f0 - 7.0 * f1 + 11.0 * f2) * s6;
  const double q1 = (-f1 + 5.0 * f2 + 2.0 * f3) * s6;
  const double q2 = (2.0 * f2 + 5.0 * f3 - f4) * s6;
  const float t0 = (float)(f0 - 2.0 * f1 + f2), s0 = (float)(f0 - 4.0 * f1 + 3.0 * f2);
  const float t1 = (float)(f1 - 2.0 * f2 + f3), s1 = (float)(f1 - f3);
  const float t2 = (float)(f2 - 2.0 * f3 + f4), s2 = (float)(3.0 * f2 - 4.0 * f3 + f4);
  const float c13 = 13.0f / 12.0f;
  const float b0 = c13 * t0 * t0 + 0.25f * s0 * s0 + eps;
  const float b1 = c13 * t1 * t1 + 0.25f * s1 * s1 + eps;
  const float b2 = c13 * t2 * t2 + 0.25f * s2 * s2 + eps;
  const float tau = fabsf(b0 - b2);
  float r0 = tau * mixed_rcp(b0), r1 = tau * mixed_rcp(b1), r2 = tau * mixed_rcp(b2);
  if (pw == 2) {
    r0 *= r0;
    r1 *= r1;
    r2 *= r2;
  }
  const float a0 = 0.1f * (1.0f + r0), a1 = 0.6f * (1.0f + r1), a2 = 0.3f * (1.0f + r2);
  const float inv = mixed_rcp(a0 + a1 + a2);
  const double w0 = (double)(a0 * inv), w1 = (double)(a1 * inv), w2 = (double)(a2 * inv);
  if (w0 >= w1 && w0 >= w2) return q0 + w1 * (q1 - q0) + w2 * (q2 - q0);
  if (w2 > w1) return q2 + w0 * (q0 - q2) + w1 * (q1 - q2);
  return q1 + w0 * (q0 - q1) + w2 * (q2 - q1);
}

// Scheme variants (cited in Sec. 4 beside the default WENO5-Z): WENO5-JS,
// alpha_k = d_k / (beta_k + eps)^p; TENO5, substencils whose share of
// (1 + tau5 / (beta_k + eps))^6 is below 1e-5 are cut off and the others keep
// their linear weights (shares scaled by the largest measure, no overflow).
MPMC_HD double weno5js(double f0, double f1, double f2, double f3, double f4, double eps, int pw) {
  const double s6 = 1.0 / 6.0;
  const double q0 = (2.0 * f0 - 7.0 * f1 + 11.0 * f2) * s6;
  const double q1 = (-f1 + 5.0 * f2 + 2.0 * f3) * s6;
  const double q2 = (2.0 * f2 + 5.0 * f3 - f4) * s6;
  const double t0 = f0 - 2.0 * f1 + f2, s0 = f0 - 4.0 * f1 + 3.0 * f2;
  const double t1 = f1 - 2.0 * f2 + f3, s1 = f1 - f3;
  const double t2 = f2 - 2.0 * f3 + f4, s2 = 3.0 * f2 - 4.0 * f3 + f4;
  const double c13 = 13.0 / 12.0;
  double g0 = c13 * t0 * t0 + 0.25 * s0 * s0 + eps;
  double g1 = c13 * t1 * t1 + 0.25 * s1 * s1 + eps;
  double g2 = c13 * t2 * t2 + 0.25 * s2 * s2 + eps;
  if (pw == 2) {
    g0 *= g0;
    g1 *= g1;
    g2 *= g2;
  }
  const double a0 = 0.1 / g0, a1 = 0.6 / g1, a2 = 0.3 / g2;
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

MPMC_HD double teno5(double f0, double f1, double f2, double f3, double f4, double eps) {
  const double s6 = 1.0 / 6.0;
  const double q0 = (2.0 * f0 - 7.0 * f1 + 11.0 * f2) * s6;
  const double q1 = (-f1 + 5.0 * f2 + 2.0 * f3) * s6;
  const double q2 = (2.0 * f2 + 5.0 * f3 - f4) * s6;
  const double t0 = f0 - 2.0 * f1 + f2, s0 = f0 - 4.0 * f1 + 3.0 * f2;
  const double t1 = f1 - 2.0 * f2 + f3, s1 = f1 - f3;
  const double t2 = f2 - 2.0 * f3 + f4, s2 = 3.0 * f2 - 4.0 * f3 + f4;
  const double c13 = 13.0 / 12.0;
  const double b0 = c13 * t0 * t0 + 0.25 * s0 * s0;
  const double b1 = c13 * t1 * t1 + 0.25 * s1 * s1;
  const double b2 = c13 * t2 * t2 + 0.25 * s2 * s2;
  const double tau = fabs(b0 - b2);
  const double a0 = 1.0 + tau / (b0 + eps), a1 = 1.0 + tau / (b1 + eps), a2 = 1.0 + tau / (b2 + eps);
  const double im = 1.0 / fmax(a0, fmax(a1, a2));
  auto p6 = [](double x) {
    const double x2 = x * x;
    return x2 * x2 * x2;
  };
  const double g0 = p6(a0 * im), g1 = p6(a1 * im), g2 = p6(a2 * im);
  const double sg = g0 + g1 + g2, ct = 1e-5;
  const double d0 = g0 / sg >= ct ? 0.1 : 0.0, d1 = g1 / sg >= ct ? 0.6 : 0.0, d2 = g2 / sg >= ct ? 0.3 : 0.0;
  return (d0 * q0 + d1 * q1 + d2 * q2) / (d0 + d1 + d2);
}

// Left and right face values of one characteristic variable from its six
// stencil values w[0..5] (cells i-2..i+3).  Kept out of line: the register
// pressure of the two evaluations then does not add to the caller's.
__host__ __device__ __noinline__ double2 weno5z_lr(double w0, double w1, double w2, double w3, double w4,
                                          double w5, double eps, int pw) {
  return make_double2(weno5z<double>(w0, w1, w2, w3, w4, eps, pw),
                      weno5z<double>(w5, w4, w3, w2, w1, eps, pw));
}

// TENO6 (Fu et al. 2016) at the face i+1/2 from f_{i-2..i+3}: candidate
// stencils central {i-1,i,i+1}, downwind {i,i+1,i+2}, upwind {i-2,i-1,i} and
// four-point {i..i+3} with linear weights 9/20, 3/10, 1/20, 1/5 (they
// recombine the six-point reconstruction); Jiang-Shu indicators over cell i;
// reference tau6 = |beta6 - (beta_u + beta_d + 4 beta_c)/6|, beta6 the
// indicator of the six-point quintic, written in the quintic's derivatives
// D1..D5 at the cell centre (unit cell width); measures (1 + tau6/(beta+eps))^6
// scaled by the largest, cut-off 1e-7.
__host__ __device__ __noinline__ double teno6(double f0, double f1, double f2, double f3, double f4, double f5,
                                              double eps) {
  const double s6 = 1.0 / 6.0;
  const double qc = (-f1 + 5.0 * f2 + 2.0 * f3) * s6;
  const double qd = (2.0 * f2 + 5.0 * f3 - f4) * s6;
  const double qu = (2.0 * f0 - 7.0 * f1 + 11.0 * f2) * s6;
  const double q4 = (3.0 * f2 + 13.0 * f3 - 5.0 * f4 + f5) * (1.0 / 12.0);
  const double c13 = 13.0 / 12.0;
  const double tc = f1 - 2.0 * f2 + f3, sc = f1 - f3;
  const double td = f2 - 2.0 * f3 + f4, sd = 3.0 * f2 - 4.0 * f3 + f4;
  const double tu = f0 - 2.0 * f1 + f2, su = f0 - 4.0 * f1 + 3.0 * f2;
  const double bc = c13 * tc * tc + 0.25 * sc * sc;
  const double bd = c13 * td * td + 0.25 * sd * sd;
  const double bu = c13 * tu * tu + 0.25 * su * su;
  const double r1 = -11.0 * f2 + 18.0 * f3 - 9.0 * f4 + 2.0 * f5;
  const double r2 = 2.0 * f2 - 5.0 * f3 + 4.0 * f4 - f5;
  const double r3 = -f2 + 3.0 * f3 - 3.0 * f4 + f5;
  const double b4 = (1.0 / 36.0) * r1 * r1 + c13 * r2 * r2 + (781.0 / 720.0) * r3 * r3;
  const double D1 = (341.0 * f0 - 2785.0 * f1 - 2590.0 * f2 + 6670.0 * f3 - 1895.0 * f4 + 259.0 * f5) * (1.0 / 5760.0);
  const double D2 = (-f0 + 12.0 * f1 - 22.0 * f2 + 12.0 * f3 - f4) * 0.125;
  const double D3 = (-5.0 * f0 - 11.0 * f1 + 70.0 * f2 - 94.0 * f3 + 47.0 * f4 - 7.0 * f5) * (1.0 / 24.0);
  const double D4 = f0 - 4.0 * f1 + 6.0 * f2 - 4.0 * f3 + f4;
  const double D5 = -f0 + 5.0 * f1 - 10.0 * f2 + 10.0 * f3 - 5.0 * f4 + f5;
  const double b6 = D1 * (D1 + D3 * (1.0 / 12.0) + D5 * (1.0 / 960.0)) + D2 * (c13 * D2 + D4 * (7.0 / 80.0)) +
                    D3 * ((1043.0 / 960.0) * D3 + D5 * (4709.0 / 53760.0)) + (87617.0 / 80640.0) * D4 * D4 +
                    (50467427.0 / 46448640.0) * D5 * D5;
  const double tau = fabs(b6 - (bu + bd + 4.0 * bc) * s6);
  const double ac = 1.0 + tau / (bc + eps), ad = 1.0 + tau / (bd + eps);
  const double au = 1.0 + tau / (bu + eps), a4 = 1.0 + tau / (b4 + eps);
  const double im = 1.0 / fmax(fmax(ac, ad), fmax(au, a4));
  auto p6 = [](double x) {
    const double x2 = x * x;
    return x2 * x2 * x2;
  };
  const double gc = p6(ac * im), gd = p6(ad * im), gu = p6(au * im), g4 = p6(a4 * im);
  const double sg = gc + gd + gu + g4, ct = 1e-7;
  const double dc = gc / sg >= ct ? 0.45 : 0.0, dd = gd / sg >= ct ? 0.3 : 0.0;
  const double du = gu / sg >= ct ? 0.05 : 0.0, d4 = g4 / sg >= ct ? 0.2 : 0.0;
  return (dc * qc + dd * qd + du * qu + d4 * q4) / (dc + dd + du + d4);
}

// weno5z_lr or, by scheme (1 WENO5-JS, 2 TENO5, 3 TENO6), a variant.
__host__ __device__ __noinline__ double2 weno_lr(double w0, double w1, double w2, double w3, double w4,
                                                 double w5, double eps, int pw, int scheme) {
  if (scheme == 1) return make_double2(weno5js(w0, w1, w2, w3, w4, eps, pw), weno5js(w5, w4, w3, w2, w1, eps, pw));
  if (scheme == 2) return make_double2(teno5(w0, w1, w2, w3, w4, eps), teno5(w5, w4, w3, w2, w1, eps));
  if (scheme == 3) return make_double2(teno6(w0, w1, w2, w3, w4, w5, eps), teno6(w5, w4, w3, w2, w1, w0, eps));
  return make_double2(weno5z<double>(w0, w1, w2, w3, w4, eps, pw), weno5z<double>(w5, w4, w3, w2, w1, eps, pw));
}

// Mass-fraction limiter of one face side (Sec. 3.3.1).
template <int NS, class R> MPMC_HD int ylimit(R* Ys, const R* Yc) {
  R sum = 0;
#pragma unroll
  for (int k = 0; k < NS; ++k) sum += Ys[k];
  R d[NS];
  int br;
  if (sum > (R)1) {
    br = 1;
#pragma unroll
    for (int k = 0; k < NS; ++k) d[k] = rmin(Ys[k], Yc[k]) - Ys[k];
  } else if (sum < (R)1) {
    br = 2;
#pragma unroll
    for (int k = 0; k < NS; ++k) d[k] = rmax(Ys[k], Yc[k]) - Ys[k];
  } else {
    return 0;
  }
  R sd = 0;
#pragma unroll
  for (int k = 0; k < NS; ++k) sd += d[k];
  if (::fabs((double)val(sd)) < 1e-300) return 0;
  const R f = ((R)1 - sum) / sd;
#pragma unroll
  for (int k = 0; k < NS; ++k) Ys[k] = Ys[k] + f * d[k];
  return br;
}

// One side of a face in the frame (n, t1, t2) of the sweep.
template <int NS, int DIM, class R> struct Side {
  R rho, un, ut[DIM > 1 ? DIM - 1 : 1], P, E, a, rY[NS];
};

// Conserved vector and physical flux of a side, frame layout
// [rhoY.., rho u_n, rho u_t.., E].
template <int NS, int DIM, class R>
MPMC_HD void side_UF(const Side<NS, DIM, R>& s, R* U, R* F) {
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    U[k] = s.rY[k];
    F[k] = s.rY[k] * s.un;
  }
  U[NS] = s.rho * s.un;
  F[NS] = s.rho * s.un * s.un + s.P;
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) {
    U[NS + 1 + t] = s.rho * s.ut[t];
    F[NS + 1 + t] = s.rho * s.un * s.ut[t];
  }
  U[NS + DIM] = s.E;
  F[NS + DIM] = s.un * (s.E + s.P);
}

// HLLC flux (App. B) in the face frame.
template <int NS, int DIM, class R>
MPMC_HD void hllc(const Side<NS, DIM, R>& L, const Side<NS, DIM, R>& Rs, R* F) {
  constexpr int NV = NS + DIM + 1;
  const R ub = (R)0.5 * (L.un + Rs.un), ab = (R)0.5 * (L.a + Rs.a);
  const R sL = rmin(ub - ab, L.un - L.a);
  const R sR = rmax(ub + ab, Rs.un + Rs.a);
  const R sm = rmin((R)0, sL), sp = rmax((R)0, sR);
  const R ss = (Rs.P - L.P + L.rho * L.un * (sL - L.un) - Rs.rho * Rs.un * (sR - Rs.un)) /
               (L.rho * (sL - L.un) - Rs.rho * (sR - Rs.un));
  R Ua[NV], Fa[NV], Fb[NV];
  // NaN in s* takes both halves (and yields NaN), as sign() would give 0
  if (!(ss < (R)0)) {
    side_UF<NS, DIM, R>(L, Ua, Fa);
    const R fac = (sL - L.un) / (sL - ss);
#pragma unroll
    for (int k = 0; k < NS; ++k) Fa[k] = Fa[k] + sm * (fac * L.rY[k] - Ua[k]);
    Fa[NS] = Fa[NS] + sm * (fac * (L.rho * ss) - Ua[NS]);
#pragma unroll
    for (int t = 0; t < DIM - 1; ++t)
      Fa[NS + 1 + t] = Fa[NS + 1 + t] + sm * (fac * (L.rho * L.ut[t]) - Ua[NS + 1 + t]);
    Fa[NS + DIM] = Fa[NS + DIM] +
                   sm * (fac * (L.E + (ss - L.un) * (L.rho * ss + L.P / (sL - L.un))) - Ua[NS + DIM]);
  }
  if (!(ss > (R)0)) {
    side_UF<NS, DIM, R>(Rs, Ua, Fb);
    const R fac = (sR - Rs.un) / (sR - ss);
#pragma unroll
    for (int k = 0; k < NS; ++k) Fb[k] = Fb[k] + sp * (fac * Rs.rY[k] - Ua[k]);
    Fb[NS] = Fb[NS] + sp * (fac * (Rs.rho * ss) - Ua[NS]);
#pragma unroll
    for (int t = 0; t < DIM - 1; ++t)
      Fb[NS + 1 + t] = Fb[NS + 1 + t] + sp * (fac * (Rs.rho * Rs.ut[t]) - Ua[NS + 1 + t]);
    Fb[NS + DIM] = Fb[NS + DIM] +
                   sp * (fac * (Rs.E + (ss - Rs.un) * (Rs.rho * ss + Rs.P / (sR - Rs.un))) - Ua[NS + DIM]);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (ss > (R)0)
      F[v] = Fa[v];
    else if (ss < (R)0)
      F[v] = Fb[v];
    else
      F[v] = (R)0.5 * Fa[v] + (R)0.5 * Fb[v];
  }
}

// Face state from (P, T, Y, u) by the EOS (Godunov steps 4-5).
template <int NS, int DIM, class R>
MPMC_HD void face_state(const Params& p, R P, R T, const R* Y, R un, const R* ut,
                                           Side<NS, DIM, R>& s) {
  R vm = 0, em = 0, ipp[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    ipp[k] = (R)1 / (P + (R)p.pinf[k]);
    vm += Y[k] * ((R)p.gm1cv[k] * ipp[k] * T + (R)p.b[k]);
    const R ek = p.pinf[k] == 0.0 ? (R)p.cv[k] : (R)p.cv[k] * (P + (R)(p.gam[k] * p.pinf[k])) * ipp[k];
    em += Y[k] * (ek * T + (R)p.q[k]);
  }
  const R rho = (R)1 / vm;
  s.rho = rho;
  s.un = un;
  R ke = un * un;
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) {
    s.ut[t] = ut[t];
    ke += ut[t] * ut[t];
  }
  s.P = P;
#pragma unroll
  for (int k = 0; k < NS; ++k) s.rY[k] = rho * Y[k];
  s.E = rho * em + (R)0.5 * rho * ke;
  R beta, alpha;
  sound<NS, R>(p, rho, Y, ipp, T, s.a, beta, alpha);
}

// ---------------------------------------------------------------------------
// Per-cell quantities: equilibrium plus the phase quantities of the
// regularization (Sec. 3.2) and of the species diffusion (Sec. 2.1-2.2).
// ---------------------------------------------------------------------------
template <int NS, int DIM, class S> struct CellQ {
  S T, P, Y[NS], vel[DIM], rho, a;
  S phi[2], psi, yrho[NS], hrho[2];
  S chi[NS], K[NS], h[NS];
  S mu, lam;  // mixture viscosity and heat conductivity, sum_p phi_p (.)_p
};

// psi of the first phase, eps ln((phi_1 + delta)/(phi_2 + delta)).
MPMC_HD double psi_of(const Params& p, double f0, double f1) {
  return p.eps * log((f0 + p.delta) / (f1 + p.delta));
}
// The transform is differentiated only in mixed cells, where both phases'
// volume fractions exceed the regularization floor phi_min (Sec. 3.2): in a
// pure region of either phase psi follows tails of the profile down to
// delta = 1e-100, its gradient is set by rounding, and the derivative of the
// normal grows without bound.
MPMC_HD bool psi_differentiable(const Params& p, double f0, double f1) {
  return f0 > p.phimin && f1 > p.phimin;
}
template <int N> MPMC_HD Dual<N> psi_of(const Params& p, const Dual<N>& f0, const Dual<N>& f1) {
  Dual<N> r(psi_of(p, f0.v, f1.v));
  const bool on = psi_differentiable(p, f0.v, f1.v);
  const double i0 = on ? p.eps / (f0.v + p.delta) : 0.0;
  const double i1 = on ? p.eps / (f1.v + p.delta) : 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) r.d[i] = f0.d[i] * i0 - f1.d[i] * i1;
  return r;
}

template <int NS, int DIM, class S, bool GEN = false>
MPMC_HD void cell_quantities_t(const Params& p, const S* u, CellQ<NS, DIM, S>& q, bool aux) {
  ThermoT<NS, DIM, S> t;
  equilibrium_t<NS, DIM, S, GEN>(p, u, t, false);
  q.T = t.T;
  q.P = t.P;
#pragma unroll
  for (int k = 0; k < NS; ++k) q.Y[k] = t.Y[k];
#pragma unroll
  for (int d = 0; d < DIM; ++d) q.vel[d] = t.vel[d];
  q.rho = t.rho;
  q.a = t.a;
  q.mu = 0.0;
  q.lam = 0.0;
  if (!aux) return;
  S vk[NS], hk[NS], y[NS], mup[2], lamp[2] = {S(0.0), S(0.0)};
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    vk[k] = (S(p.gm1cv[k]) / (t.P + p.pinf[k])) * t.T + p.b[k];
    hk[k] = p.gcv[k] * t.T + p.b[k] * t.P + p.q[k];
  }
  // (phase loops unrolled over the two possible phases: per-phase values stay
  // in registers)
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    if (pp >= p.np) break;
    const int ph = p.pid[pp];
    S rYp = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) rYp += u[k];
    // y_c = rhoY_c / rhoY_p, or 1/N_p where the phase is absent
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) y[k] = val(rYp) > 1e-300 ? S(u[k] / rYp) : S(p.inpn[pp]);
    S vp = 0.0, hp = 0.0, ph_ = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) {
        vp += y[k] * vk[k];
        hp += y[k] * hk[k];
        ph_ += u[k] * vk[k];
      }
    const S rhop = 1.0 / vp;
    q.hrho[pp] = rhop * hp;
    q.phi[pp] = ph_;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) q.yrho[k] = y[k] * rhop;
    // phase viscosity: Wilke for several components, else the constant
    if (p.multi[pp]) {
      S num = 0.0;
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        if (p.phase[a] != ph) continue;
        S den = 0.0;
#pragma unroll
        for (int b = 0; b < NS; ++b)
          if (p.phase[b] == ph) den += y[b] * p.wilke[a][b];
        num += y[a] * p.mu[a] / den;
      }
      mup[pp] = num;
      S winv = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) winv += y[k] / p.W[k];
      const S Wp = 1.0 / winv;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) {
          q.chi[k] = (y[k] / p.W[k]) * Wp;           // X_c / X_p
          const S Dk = mup[pp] / (rhop * p.Sc[k]);    // D_p^c = mu_p / (rho_p Sc)
          q.K[k] = Dk * p.W[k] / Wp;
        }
    } else {
      S m = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) {
          m = p.mu[k];
          q.chi[k] = 1.0;
          q.K[k] = 0.0;
        }
      mup[pp] = m;
    }
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) q.h[k] = hk[k];
    // heat conductivity of the phase (Sec. 2.2.1): the gas mu_g / Pr sum_c
    // y_c C_P,c, a liquid sum_c y_c lambda_c (its component's constant)
    if (p.visc) {
      S l = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) l += y[k] * (ph == 1 ? p.gcv[k] : p.lamc[k]);
      lamp[pp] = ph == 1 ? S(mup[pp] * p.iPr * l) : l;
    }
  }
  if (p.np == 2) {
    q.psi = psi_of(p, q.phi[0], q.phi[1]);
  } else {
    q.phi[1] = 0.0;
    q.psi = 0.0;
  }
  S mu = q.phi[0] * mup[0];
  if (p.np == 2) mu += q.phi[1] * mup[1];
  q.mu = mu;
  if (p.visc) {
    S lam = q.phi[0] * lamp[0];
    if (p.np == 2) lam += q.phi[1] * lamp[1];
    q.lam = lam;
  }
}

// Admissibility of a conserved state (Eqs. PositivityReqs1-2, pure-region
// reading): rhoY_c >= 0, rho > 0, rho(e - q) > 0, 1 - sum rhoY_c b_c > 0.
template <int NS, int DIM>
MPMC_HD bool admissible(const Params& p, const double* u) {
  double rho = 0.0, rq = 0.0, rb = 0.0;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    ok = ok && (u[k] >= 0.0);
    rho += u[k];
    rq += u[k] * p.q[k];
    rb += u[k] * p.b[k];
  }
  ok = ok && (rho > 0.0);
  double m2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) m2 += u[NS + d] * u[NS + d];
  const double rhoe = u[NS + DIM] - 0.5 * m2 / rho - rq;
  ok = ok && (rhoe > 0.0) && (1.0 - rb > 0.0);
  return ok;
}

}  // namespace mpmc
