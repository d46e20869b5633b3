// mpmc_adjoint.h -- discrete adjoint (vector-Jacobian products) of one SSP-RK3
// step of the four-equation MPMC hot path with frozen decisions.
//
// Frozen decisions: the limiter selections of Sec. 3.3 (T/P fallback,
// first-order flux, dropped regularization flux) are read from the masks the
// forward recompute of the same stage recorded; the arms of min/max/abs/sign
// (HLLC wave speeds and sign of s*, |beta_0 - beta_2| of WENO-Z, the Y-limiter
// branch) are those of the recomputed forward values.  The WENO-Z weights are
// differentiated.  Reverse-mode derivatives are written by hand for the face
// pipeline; the per-cell equilibrium and auxiliaries and the face-average
// equilibrium use forward-mode dual numbers over the conserved variables.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpmc_device.h"
#include "mpmc_dual.h"
#include "mpmc_kernels.h"

namespace mpmc {

// ---------------------------------------------------------------------------
// WENO5-Z: d out / d f_{0..4} applied to the cotangent ob (accumulated into fb)
// ---------------------------------------------------------------------------
MPMC_HD void weno5z_vjp(double f0, double f1, double f2, double f3, double f4, double eps, int pw,
                        double ob, double* fb, double scale = 0.0) {
  const double s6 = 1.0 / 6.0;
  const double t0 = f0 - 2 * f1 + f2, s0 = f0 - 4 * f1 + 3 * f2;
  const double t1 = f1 - 2 * f2 + f3, s1 = f1 - f3;
  const double t2 = f2 - 2 * f3 + f4, s2 = 3 * f2 - 4 * f3 + f4;
  // A substencil flat to round-off (its differences within 1e-7 of the
  // stencil's largest magnitude plus the variable's own scale: 1 for a mass
  // fraction, the face sound speed for a velocity) has a smoothness
  // indicator set by rounding noise, and the split of weight between two
  // such substencils is then noise too.  The derivative taken is the
  // exact-arithmetic one of a constant substencil: indicator eps, no
  // derivative.  (All three flat: the ideal weights.)
  const double m = fmax(fmax(fabs(f0), fabs(f1)), fmax(fmax(fabs(f2), fabs(f3)), fabs(f4)));
  const double tol = 1e-7 * (m + scale);
  const bool fl0 = fabs(t0) <= tol && fabs(s0) <= tol;
  const bool fl1 = fabs(t1) <= tol && fabs(s1) <= tol;
  const bool fl2 = fabs(t2) <= tol && fabs(s2) <= tol;
  const double q0 = (2 * f0 - 7 * f1 + 11 * f2) * s6;
  const double q1 = (-f1 + 5 * f2 + 2 * f3) * s6;
  const double q2 = (2 * f2 + 5 * f3 - f4) * s6;
  const double c13 = 13.0 / 12.0;
  const double b0 = fl0 ? eps : c13 * t0 * t0 + 0.25 * s0 * s0 + eps;
  const double b1 = fl1 ? eps : c13 * t1 * t1 + 0.25 * s1 * s1 + eps;
  const double b2 = fl2 ? eps : c13 * t2 * t2 + 0.25 * s2 * s2 + eps;
  const double sg = (b0 - b2) >= 0.0 ? 1.0 : -1.0;
  const double tau = sg * (b0 - b2);
  double a0, a1, a2;
  double B0 = b0, B1 = b1, B2 = b2, T2 = tau;
  if (pw == 2) {
    B0 = b0 * b0;
    B1 = b1 * b1;
    B2 = b2 * b2;
    T2 = tau * tau;
  }
  a0 = 0.1 * (B0 + T2) * (B1 * B2);
  a1 = 0.6 * (B1 + T2) * (B0 * B2);
  a2 = 0.3 * (B2 + T2) * (B0 * B1);
  const double D = a0 + a1 + a2;
  const double out = (a0 * q0 + a1 * q1 + a2 * q2) / D;
  const double Nb = ob / D, Db = -ob * out / D;
  const double ab0 = Nb * q0 + Db, ab1 = Nb * q1 + Db, ab2 = Nb * q2 + Db;
  const double qb0 = Nb * a0, qb1 = Nb * a1, qb2 = Nb * a2;
  // a_k in terms of B_k and T2
  double Bb0 = ab0 * 0.1 * (B1 * B2) + ab1 * 0.6 * (B1 + T2) * B2 + ab2 * 0.3 * (B2 + T2) * B1;
  double Bb1 = ab0 * 0.1 * (B0 + T2) * B2 + ab1 * 0.6 * (B0 * B2) + ab2 * 0.3 * (B2 + T2) * B0;
  double Bb2 = ab0 * 0.1 * (B0 + T2) * B1 + ab1 * 0.6 * (B1 + T2) * B0 + ab2 * 0.3 * (B0 * B1);
  double Tb = ab0 * 0.1 * (B1 * B2) + ab1 * 0.6 * (B0 * B2) + ab2 * 0.3 * (B0 * B1);
  double bb0 = Bb0, bb1 = Bb1, bb2 = Bb2, taub = Tb;
  if (pw == 2) {
    bb0 = 2 * b0 * Bb0;
    bb1 = 2 * b1 * Bb1;
    bb2 = 2 * b2 * Bb2;
    taub = 2 * tau * Tb;
  }
  bb0 += sg * taub;
  bb2 -= sg * taub;
  const double tb0 = fl0 ? 0.0 : 2 * c13 * t0 * bb0, sb0 = fl0 ? 0.0 : 0.5 * s0 * bb0;
  const double tb1 = fl1 ? 0.0 : 2 * c13 * t1 * bb1, sb1 = fl1 ? 0.0 : 0.5 * s1 * bb1;
  const double tb2 = fl2 ? 0.0 : 2 * c13 * t2 * bb2, sb2 = fl2 ? 0.0 : 0.5 * s2 * bb2;
  fb[0] += tb0 + sb0 + 2 * s6 * qb0;
  fb[1] += -2 * tb0 - 4 * sb0 + tb1 + sb1 - 7 * s6 * qb0 - s6 * qb1;
  fb[2] += tb0 + 3 * sb0 - 2 * tb1 + tb2 + 3 * sb2 + 11 * s6 * qb0 + 5 * s6 * qb1 + 2 * s6 * qb2;
  fb[3] += tb1 - sb1 - 2 * tb2 - 4 * sb2 + 2 * s6 * qb1 + 5 * s6 * qb2;
  fb[4] += tb2 + sb2 - s6 * qb2;
}

// ---------------------------------------------------------------------------
// Y-limiter of one side: Ys (before limiting), Yc (cell).  Yb_out is the
// cotangent of the limited values; accumulates into Ysb and Ycb.
// ---------------------------------------------------------------------------
template <int NS>
MPMC_HD void ylimit_vjp(const double* Ys, const double* Yc, const double* Yb_out, double* Ysb, double* Ycb) {
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    sum += Ys[k];
    Ysb[k] += Yb_out[k];
  }
  // a correction of round-off size is not differentiated
  if (::fabs(1.0 - sum) <= 1e-13) return;
  int br;
  bool useC[NS];
  double d[NS];
  // useC: the cell value is taken and differentiated (a difference of
  // round-off size, at most 1e-10, is a tie: no derivative through it)
  if (sum > 1.0) {
    br = 1;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      useC[k] = Yc[k] < Ys[k] - 1e-10;
      d[k] = rmin(Ys[k], Yc[k]) - Ys[k];
    }
  } else if (sum < 1.0) {
    br = 2;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      useC[k] = Yc[k] > Ys[k] + 1e-10;
      d[k] = rmax(Ys[k], Yc[k]) - Ys[k];
    }
  } else {
    return;
  }
  (void)br;
  double sd = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) sd += d[k];
  if (::fabs(sd) < 1e-300) return;
  const double f = (1.0 - sum) / sd;
  double fb = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) fb += Yb_out[k] * d[k];
  const double Sb = -fb / sd, sdb = -fb * f / sd;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double db = Yb_out[k] * f + sdb;
    if (useC[k]) {  // d_k = Yc_k - Ys_k; otherwise no derivative
      Ycb[k] += db;
      Ysb[k] -= db;
    }
    Ysb[k] += Sb;
  }
}

// ---------------------------------------------------------------------------
// face state (P, T, Y, u_n, u_t) -> side (rho, E, a, rhoY ...): VJP
// ---------------------------------------------------------------------------
template <int NS, int DIM>
MPMC_HD void face_state_vjp(const Params& p, double P, double T, const double* Y, double un,
                            const double* ut, const Side<NS, DIM, double>& sb, double& Pb, double& Tb,
                            double* Yb, double& unb, double* utb) {
  double ipp[NS], ek[NS], vm = 0.0, em = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    ipp[k] = 1.0 / (P + p.pinf[k]);
    vm += Y[k] * (p.gm1cv[k] * ipp[k] * T + p.b[k]);
    ek[k] = p.pinf[k] == 0.0 ? p.cv[k] : p.cv[k] * (P + p.gam[k] * p.pinf[k]) * ipp[k];
    em += Y[k] * (ek[k] * T + p.q[k]);
  }
  const double rho = 1.0 / vm;
  double ke = un * un;
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) ke += ut[t] * ut[t];
  double sa = 0.0, sbs = 0.0, Cp = 0.0, kp[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    kp[k] = p.gm1cv[k] * ipp[k];
    sa += Y[k] * kp[k];
    sbs += Y[k] * kp[k] * ipp[k];
    Cp += Y[k] * p.gcv[k];
  }
  const double sbv = sbs * T;
  const double beta = rho * sbv, alpha = rho * sa;
  const double Dn = rho * beta * Cp - alpha * alpha * T;
  const double a2 = Cp / Dn, a = ::sqrt(a2);
  // sound speed
  const double a2b = sb.a * 0.5 / a;
  double Cpb = a2b / Dn;
  const double Dnb = -a2b * a2 / Dn;
  double rhob = sb.rho + Dnb * beta * Cp;
  const double betab = Dnb * rho * Cp;
  Cpb += Dnb * rho * beta;
  const double alphab = -2.0 * alpha * T * Dnb;
  Tb += -alpha * alpha * Dnb;
  rhob += betab * sbv;
  const double sbvb = betab * rho;
  rhob += alphab * sa;
  const double sab = alphab * rho;
  const double sbsb = sbvb * T;
  Tb += sbvb * sbs;
  double ippb[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    Yb[k] += Cpb * p.gcv[k] + sab * kp[k] + sbsb * kp[k] * ipp[k];
    const double kpb = sab * Y[k] + sbsb * Y[k] * ipp[k];
    ippb[k] = sbsb * Y[k] * kp[k] + kpb * p.gm1cv[k];
  }
  // E = rho em + rho ke / 2
  rhob += sb.E * (em + 0.5 * ke);
  const double emb = sb.E * rho, keb = 0.5 * rho * sb.E;
  // rhoY = rho Y
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    rhob += sb.rY[k] * Y[k];
    Yb[k] += sb.rY[k] * rho;
  }
  unb += sb.un + 2.0 * un * keb;
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) utb[t] += sb.ut[t] + 2.0 * ut[t] * keb;
  // rho = 1/vm
  const double vmb = -rhob * rho * rho;
  double Pacc = sb.P;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    // em
    Yb[k] += emb * (ek[k] * T + p.q[k]);
    const double ekb = emb * Y[k] * T;
    Tb += emb * Y[k] * ek[k];
    if (p.pinf[k] != 0.0) {
      Pacc += ekb * p.cv[k] * ipp[k];
      ippb[k] += ekb * p.cv[k] * (P + p.gam[k] * p.pinf[k]);
    }
    // vm
    Yb[k] += vmb * (p.gm1cv[k] * ipp[k] * T + p.b[k]);
    ippb[k] += vmb * Y[k] * p.gm1cv[k] * T;
    Tb += vmb * Y[k] * p.gm1cv[k] * ipp[k];
    // ipp = 1/(P + P_inf)
    Pacc += -ippb[k] * ipp[k] * ipp[k];
  }
  Pb += Pacc;
}

// ---------------------------------------------------------------------------
// HLLC (App. B): VJP in the face frame.  Fb: cotangent of the frame flux.
// ---------------------------------------------------------------------------
template <int NS, int DIM>
MPMC_HD void hllc_branch_vjp(const Side<NS, DIM, double>& S, double sK, double ss, double sfac,
                             const double* g, Side<NS, DIM, double>& Sb, double& sKb, double& ssb,
                             double& sfacb) {
  constexpr int NV = NS + DIM + 1;
  const double un = S.un, rho = S.rho, P = S.P, E = S.E;
  double unb = 0.0;
  // physical flux F(U)
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    Sb.rY[k] += g[k] * un;
    unb += g[k] * S.rY[k];
  }
  Sb.rho += g[NS] * un * un;
  unb += g[NS] * 2.0 * rho * un;
  Sb.P += g[NS];
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) {
    Sb.rho += g[NS + 1 + t] * un * S.ut[t];
    unb += g[NS + 1 + t] * rho * S.ut[t];
    Sb.ut[t] += g[NS + 1 + t] * rho * un;
  }
  Sb.E += g[NV - 1] * un;
  Sb.P += g[NV - 1] * un;
  unb += g[NV - 1] * (E + P);
  // star-state term sfac (U* - U)
  const double A = sK - un, B = sK - ss, fac = A / B;
  const double Y1 = rho * ss + P / A;
  const double X = E + (ss - un) * Y1;
  double dsum = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) dsum += g[k] * (fac * S.rY[k] - S.rY[k]);
  dsum += g[NS] * (fac * rho * ss - rho * un);
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) dsum += g[NS + 1 + t] * (fac * rho * S.ut[t] - rho * S.ut[t]);
  dsum += g[NV - 1] * (fac * X - E);
  sfacb += dsum;
  double facb = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double us = sfac * g[k];
    facb += us * S.rY[k];
    Sb.rY[k] += us * fac - sfac * g[k];
  }
  {
    const double us = sfac * g[NS];
    facb += us * rho * ss;
    Sb.rho += us * fac * ss - sfac * g[NS] * un;
    ssb += us * fac * rho;
    unb += -sfac * g[NS] * rho;
  }
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) {
    const double us = sfac * g[NS + 1 + t];
    facb += us * rho * S.ut[t];
    Sb.rho += us * fac * S.ut[t] - sfac * g[NS + 1 + t] * S.ut[t];
    Sb.ut[t] += us * fac * rho - sfac * g[NS + 1 + t] * rho;
  }
  {
    const double us = sfac * g[NV - 1];
    facb += us * X;
    const double Xb = us * fac;
    Sb.E += Xb - sfac * g[NV - 1];
    ssb += Xb * Y1;
    unb -= Xb * Y1;
    const double Y1b = Xb * (ss - un);
    Sb.rho += Y1b * ss;
    ssb += Y1b * rho;
    Sb.P += Y1b / A;
    const double Ab = -Y1b * P / (A * A);
    sKb += Ab;
    unb -= Ab;
  }
  // fac = A / B
  const double Ab = facb / B, Bb = -facb * A / (B * B);
  sKb += Ab + Bb;
  unb -= Ab;
  ssb -= Bb;
  Sb.un += unb;
}

template <int NS, int DIM>
MPMC_HD void hllc_vjp(const Side<NS, DIM, double>& L, const Side<NS, DIM, double>& R, const double* Fb,
                      Side<NS, DIM, double>& Lb, Side<NS, DIM, double>& Rb) {
  constexpr int NV = NS + DIM + 1;
  const double ub = 0.5 * (L.un + R.un), ab = 0.5 * (L.a + R.a);
  // values as in the forward; derivative arms: a choice decided by rounding
  // (a near-tie within 1e-9 of the speed scale, s* within 1e-9 of zero) is
  // taken as in exact arithmetic at the tie: the averaged-state speed, and
  // the mean of the two star fluxes
  const double tS = 1e-9 * (ab + fabs(ub));
  const double sL = rmin(ub - ab, L.un - L.a);
  const double sR = rmax(ub + ab, R.un + R.a);
  const bool sLarm = (L.un - L.a) < (ub - ab) - tS;
  const bool sRarm = (R.un + R.a) > (ub + ab) + tS;
  const double sm = rmin(0.0, sL), sp = rmax(0.0, sR);
  const double num = R.P - L.P + L.rho * L.un * (sL - L.un) - R.rho * R.un * (sR - R.un);
  const double den = L.rho * (sL - L.un) - R.rho * (sR - R.un);
  const double ss = num / den;
  double gA[NV], gB[NV];
  const bool tie = fabs(ss) <= 1e-9 * fmax(fabs(sL), fabs(sR));
  const double wA = tie ? 0.5 : (ss > 0.0 ? 1.0 : 0.0);
  const double wB = tie ? 0.5 : (ss < 0.0 ? 1.0 : 0.0);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    gA[v] = wA * Fb[v];
    gB[v] = wB * Fb[v];
  }
  double sLb = 0.0, sRb = 0.0, ssb = 0.0, smb = 0.0, spb = 0.0;
  if (wA != 0.0) hllc_branch_vjp<NS, DIM>(L, sL, ss, sm, gA, Lb, sLb, ssb, smb);
  if (wB != 0.0) hllc_branch_vjp<NS, DIM>(R, sR, ss, sp, gB, Rb, sRb, ssb, spb);
  if (sL < 0.0) sLb += smb;  // sm = min(0, sL)
  if (sR > 0.0) sRb += spb;  // sp = max(0, sR)
  const double numb = ssb / den, denb = -ssb * ss / den;
  Rb.P += numb;
  Lb.P -= numb;
  Lb.rho += numb * L.un * (sL - L.un);
  Lb.un += numb * L.rho * (sL - 2.0 * L.un);
  sLb += numb * L.rho * L.un;
  Rb.rho -= numb * R.un * (sR - R.un);
  Rb.un -= numb * R.rho * (sR - 2.0 * R.un);
  sRb -= numb * R.rho * R.un;
  Lb.rho += denb * (sL - L.un);
  sLb += denb * L.rho;
  Lb.un -= denb * L.rho;
  Rb.rho -= denb * (sR - R.un);
  sRb -= denb * R.rho;
  Rb.un += denb * R.rho;
  double ubb = 0.0, abb = 0.0;
  if (sLarm) {
    Lb.un += sLb;
    Lb.a -= sLb;
  } else {
    ubb += sLb;
    abb -= sLb;
  }
  if (sRarm) {
    Rb.un += sRb;
    Rb.a += sRb;
  } else {
    ubb += sRb;
    abb += sRb;
  }
  Lb.un += 0.5 * ubb;
  Rb.un += 0.5 * ubb;
  Lb.a += 0.5 * abb;
  Rb.a += 0.5 * abb;
}

template <int NS, int DIM> MPMC_HD void side_zero(Side<NS, DIM, double>& s) {
  s.rho = s.un = s.P = s.E = s.a = 0.0;
#pragma unroll
  for (int t = 0; t < (DIM > 1 ? DIM - 1 : 1); ++t) s.ut[t] = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) s.rY[k] = 0.0;
}


// ---------------------------------------------------------------------------
// Scatter of cotangents: many faces touch one cell, so contributions to the
// per-cell cotangent arrays are added with hardware FP64 atomics.
// ---------------------------------------------------------------------------
MPMC_HD void aadd(double* a, double v) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (v != 0.0) unsafeAtomicAdd(a, v);
#else
  *a += v;  // host execution of the same code (test harness), sequential
#endif
}

// Six stencil cotangents returned by value (registers, no stack).
struct D6 {
  double v[6];
};

// Cotangents of the six stencil values w[0..5] of one characteristic
// variable from those of its left (cells 0..4) and right (cells 5..1)
// WENO5-Z face values.  Out of line for the same reason as weno5z_lr.
__host__ __device__ __noinline__ D6 weno5z_lr_vjp(double w0, double w1, double w2, double w3, double w4,
                                                  double w5, double eps, int pw, double obL, double obR,
                                                  double scale) {
  D6 r;
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  weno5z_vjp(w0, w1, w2, w3, w4, eps, pw, obL, g, scale);
  r.v[0] = g[0];
  r.v[1] = g[1];
  r.v[2] = g[2];
  r.v[3] = g[3];
  r.v[4] = g[4];
  r.v[5] = 0.0;
  double h[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  weno5z_vjp(w5, w4, w3, w2, w1, eps, pw, obR, h, scale);
  r.v[5] += h[0];
  r.v[4] += h[1];
  r.v[3] += h[2];
  r.v[2] += h[3];
  r.v[1] += h[4];
  return r;
}

// d/d phi of eps ln(phi + delta) for a cell with volume fractions (phi,
// other), taken only in mixed cells (the convention of psi_of for duals).
MPMC_HD double dlog_coef(const Params& p, double phi, double other) {
  return psi_differentiable(p, phi, other) ? p.eps / (phi + p.delta) : 0.0;
}

// Cotangent of a cell side (fallback flux) scattered to Q-bar and U-bar.
template <int NS, int DIM, int DIR>
MPMC_HD void scatter_cell_side(const Params& p, double* Qb, double* Ub, int l, bool flip,
                                                  const Side<NS, DIM, double>& sb) {
  const long n = p.ncell;
  aadd(Qb + p.qRho * n + l, sb.rho);
  aadd(Qb + p.qA * n + l, sb.a);
  aadd(Qb + (p.qU + DIR) * n + l, flip ? -sb.un : sb.un);
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) aadd(Qb + (p.qU + tdir<DIM, DIR>(t)) * n + l, sb.ut[t]);
  aadd(Qb + p.qP * n + l, sb.P);
  aadd(Ub + (NS + DIM) * n + l, sb.E);
#pragma unroll
  for (int k = 0; k < NS; ++k) aadd(Ub + k * n + l, sb.rY[k]);
}

// ---------------------------------------------------------------------------
// Regularization flux of one face (Sec. 3.2.1), reverse mode.  Fb: cotangent
// of the face flux in the global frame.
// ---------------------------------------------------------------------------
template <int NS, int DIM, int DIR>
__host__ __device__ void cdi_face_vjp(const Params& p, const double* __restrict__ Q, const int* c, const int* li,
                             bool fl2, bool fl3, double Gamma, const double* Fb, double* Qb) {
  constexpr int NT = DIM - 1;
  constexpr int NTa = NT > 0 ? NT : 1;
  const long n = p.ncell;
  const double dxn = p.dx[DIR];
  const int l2 = li[2], l3 = li[3];
  // ---- forward recompute
  const double f0L = Q[p.qPhi0 * n + l2], f1L = Q[p.qPhi1 * n + l2];
  const double f0R = Q[p.qPhi0 * n + l3], f1R = Q[p.qPhi1 * n + l3];
  const double psib = 0.5 * (Q[p.qPsi * n + l2] + Q[p.qPsi * n + l3]);
  const double gn = dpsi(p, f0L, f1L, f0R, f1R) / dxn;
  double nrm2 = gn * gn, gt[NTa];
  int lt[NTa][2][2];  // [t][side][sgn]
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int td = tdir<DIM, DIR>(t);
    const int stride_t = td == 0 ? 1 : (td == 1 ? p.n[0] : p.n[0] * p.n[1]);
    double g = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      double a0[2], a1v[2];
#pragma unroll
      for (int sgn = 0; sgn < 2; ++sgn) {
        bool flip = false;
        const int ct = c[td] + (sgn ? 1 : -1);
        const int mt = (ct < 0 || ct >= p.n[td]) ? map_index(ct, p.n[td], p.bclo[td], p.bchi[td], flip) : ct;
        lt[t][side][sgn] = li[2 + side] + (mt - c[td]) * stride_t;
        a0[sgn] = Q[p.qPhi0 * n + lt[t][side][sgn]];
        a1v[sgn] = Q[p.qPhi1 * n + lt[t][side][sgn]];
      }
      g += dpsi(p, a0[0], a1v[0], a0[1], a1v[1]);
    }
    gt[t] = g / (4.0 * p.dx[td]);
    nrm2 += gt[t] * gt[t];
  }
  const double s = nrm2 > 0.0 ? sqrt(nrm2) : 0.0;
  const double nhat = nrm2 > 0.0 ? gn / s : 0.0;
  const double th = tanh(psib / (2.0 * p.eps));
  const double shape = 1.0 - th * th - p.sharp_floor;
  const double a1 = Gamma * (p.eps * (f0R - f0L) / dxn - 0.25 * shape * nhat);
  double ap[2] = {a1, -a1};
  double Rk[NS], Rsum = 0.0, hR = 0.0;
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    const int ph = p.pid[pp];
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) {
        Rk[k] = -0.5 * (Q[(p.qYrho + k) * n + l2] + Q[(p.qYrho + k) * n + l3]) * ap[pp];
        Rsum += Rk[k];
      }
    hR += -0.5 * (Q[(p.qHrho + pp) * n + l2] + Q[(p.qHrho + pp) * n + l3]) * ap[pp];
  }
  double vL[DIM], vR[DIM], kb = 0.0;
#pragma unroll
  for (int dd = 0; dd < DIM; ++dd) {
    vL[dd] = Q[(p.qU + dd) * n + l2];
    vR[dd] = Q[(p.qU + dd) * n + l3];
    if (dd == DIR) {
      if (fl2) vL[dd] = -vL[dd];
      if (fl3) vR[dd] = -vR[dd];
    }
    kb += vL[dd] * vR[dd];
  }
  kb *= 0.5;
  (void)hR;
  // ---- reverse
  const double Eb = Fb[NS + DIM];
  double Rsumb = Eb * kb;
  const double kbb = Eb * Rsum;
#pragma unroll
  for (int dd = 0; dd < DIM; ++dd) {
    Rsumb += Fb[NS + dd] * 0.5 * (vL[dd] + vR[dd]);
    double vLb = Fb[NS + dd] * 0.5 * Rsum + 0.5 * kbb * vR[dd];
    double vRb = Fb[NS + dd] * 0.5 * Rsum + 0.5 * kbb * vL[dd];
    if (dd == DIR) {
      if (fl2) vLb = -vLb;
      if (fl3) vRb = -vRb;
    }
    aadd(Qb + (p.qU + dd) * n + l2, vLb);
    aadd(Qb + (p.qU + dd) * n + l3, vRb);
  }
  const double hRb = Eb;
  double a1b = 0.0;
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    const int ph = p.pid[pp];
    double apb = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) {
        const double Rkb = Fb[k] + Rsumb;
        apb += -0.5 * (Q[(p.qYrho + k) * n + l2] + Q[(p.qYrho + k) * n + l3]) * Rkb;
        const double yb = -0.5 * ap[pp] * Rkb;
        aadd(Qb + (p.qYrho + k) * n + l2, yb);
        aadd(Qb + (p.qYrho + k) * n + l3, yb);
      }
    apb += -0.5 * (Q[(p.qHrho + pp) * n + l2] + Q[(p.qHrho + pp) * n + l3]) * hRb;
    const double hb = -0.5 * ap[pp] * hRb;
    aadd(Qb + (p.qHrho + pp) * n + l2, hb);
    aadd(Qb + (p.qHrho + pp) * n + l3, hb);
    a1b += pp == 0 ? apb : -apb;
  }
  (void)Rk;
  // a1 = Gamma (eps gphi - shape nhat / 4)
  const double gphib = Gamma * p.eps * a1b;
  const double nhatb = -0.25 * Gamma * shape * a1b;
  const double thb = 0.5 * Gamma * th * nhat * a1b;
  const double psibb = thb * (1.0 - th * th) / (2.0 * p.eps);
  aadd(Qb + p.qPsi * n + l2, 0.5 * psibb);
  aadd(Qb + p.qPsi * n + l3, 0.5 * psibb);
  double f0Lb = -gphib / dxn, f0Rb = gphib / dxn, f1Lb = 0.0, f1Rb = 0.0;
  if (nrm2 > 0.0) {
    const double is3 = 1.0 / (s * nrm2);
    const double gnb = nhatb * (1.0 / s - gn * gn * is3);
    // gn = eps [ln(f0R+d) + ln(f1L+d) - ln(f0L+d) - ln(f1R+d)] / dx
    const double db = gnb / dxn;
    f0Rb += db * dlog_coef(p, f0R, f1R);
    f1Lb += db * dlog_coef(p, f1L, f0L);
    f0Lb -= db * dlog_coef(p, f0L, f1L);
    f1Rb -= db * dlog_coef(p, f1R, f0R);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int td = tdir<DIM, DIR>(t);
      const double gtb = -nhatb * gn * gt[t] * is3;
      const double dt_b = gtb / (4.0 * p.dx[td]);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        // dpsi(a0[0], a1[0], a0[1], a1[1]) with [0] the cell at -1, [1] at +1
        const int lm = lt[t][side][0], lp = lt[t][side][1];
        const double p0m = Q[p.qPhi0 * n + lm], p1m = Q[p.qPhi1 * n + lm];
        const double p0p = Q[p.qPhi0 * n + lp], p1p = Q[p.qPhi1 * n + lp];
        aadd(Qb + p.qPhi0 * n + lp, dt_b * dlog_coef(p, p0p, p1p));
        aadd(Qb + p.qPhi1 * n + lm, dt_b * dlog_coef(p, p1m, p0m));
        aadd(Qb + p.qPhi0 * n + lm, -dt_b * dlog_coef(p, p0m, p1m));
        aadd(Qb + p.qPhi1 * n + lp, -dt_b * dlog_coef(p, p1p, p0p));
      }
    }
  }
  aadd(Qb + p.qPhi0 * n + l2, f0Lb);
  aadd(Qb + p.qPhi0 * n + l3, f0Rb);
  aadd(Qb + p.qPhi1 * n + l2, f1Lb);
  aadd(Qb + p.qPhi1 * n + l3, f1Rb);
}

// ---------------------------------------------------------------------------
// Phase-confined species diffusion flux of one face, reverse mode.
// ---------------------------------------------------------------------------
template <int NS, int DIM, int DIR>
__host__ __device__ void diffusion_face_vjp(const Params& p, const double* __restrict__ Q, const int* li,
                                   const double* Fb, double* Qb) {
  const long n = p.ncell;
  const double dxn = p.dx[DIR];
  const int l2 = li[2], l3 = li[3];
  const double rhob = 0.5 * (Q[p.qRho * n + l2] + Q[p.qRho * n + l3]);
  double rhobb = 0.0;
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    if (pp >= p.np || !p.multi[pp]) continue;
    const int ph = p.pid[pp];
    double Yb[NS], Kb[NS], G[NS], Yp = 0.0, sKG = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) {
        Yb[k] = 0.5 * (Q[(p.qY + k) * n + l2] + Q[(p.qY + k) * n + l3]);
        Kb[k] = 0.5 * (Q[(p.qK + k) * n + l2] + Q[(p.qK + k) * n + l3]);
        G[k] = (Q[(p.qChi + k) * n + l3] - Q[(p.qChi + k) * n + l2]) / dxn;
        Yp += Yb[k];
        sKG += Kb[k] * G[k];
      }
    double Ypb = 0.0, sKGb = 0.0, Jb[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) {
        const double Hb = 0.5 * (Q[(p.qH + k) * n + l2] + Q[(p.qH + k) * n + l3]);
        const double inner = Kb[k] * Yp * G[k] - Yb[k] * sKG;
        const double J = -rhob * inner;
        Jb[k] = Fb[k] + Fb[NS + DIM] * Hb;
        const double Hbb = 0.5 * Fb[NS + DIM] * J;
        aadd(Qb + (p.qH + k) * n + l2, Hbb);
        aadd(Qb + (p.qH + k) * n + l3, Hbb);
        rhobb += -Jb[k] * inner;
        Ypb += -rhob * Jb[k] * Kb[k] * G[k];
        sKGb += rhob * Jb[k] * Yb[k];
      }
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) {
        const double Kbb = -rhob * Jb[k] * Yp * G[k] + sKGb * G[k];
        const double Gb = -rhob * Jb[k] * Kb[k] * Yp + sKGb * Kb[k];
        const double Ybb = rhob * Jb[k] * sKG + Ypb;
        aadd(Qb + (p.qK + k) * n + l2, 0.5 * Kbb);
        aadd(Qb + (p.qK + k) * n + l3, 0.5 * Kbb);
        aadd(Qb + (p.qChi + k) * n + l3, Gb / dxn);
        aadd(Qb + (p.qChi + k) * n + l2, -Gb / dxn);
        aadd(Qb + (p.qY + k) * n + l2, 0.5 * Ybb);
        aadd(Qb + (p.qY + k) * n + l3, 0.5 * Ybb);
      }
  }
  aadd(Qb + p.qRho * n + l2, 0.5 * rhobb);
  aadd(Qb + p.qRho * n + l3, 0.5 * rhobb);
}

// ---------------------------------------------------------------------------
// k_face_vjp: for every face of direction DIR, the cotangent of its flux
// F-bar = coef [dt] (lam_R - lam_L) / dx (from L_i = -(F_hi - F_lo)/dx) is
// pulled back through the face pipeline (recomputed forward, decisions from
// the stage mask) to the cell quantities (Q-bar) and to U^k (U-bar).
// ---------------------------------------------------------------------------
template <int NS, int DIM, int DIR>
__host__ __device__ void face_vjp(const Params& p, const int* c, const double* __restrict__ Uk,
                                  const double* __restrict__ Q, const uint16_t* __restrict__ mask,
                                  const double* __restrict__ dtg, double coef, bool use_dt,
                                  const double* __restrict__ lam, double* __restrict__ Qb,
                                  double* __restrict__ Ub) {
  constexpr int NV = NS + DIM + 1;
  constexpr int NT = DIM - 1;
  constexpr int NTa = NT > 0 ? NT : 1;
  const long n = p.ncell;
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1);
  const long f = ((long)c[2] * e1 + c[1]) * e0 + c[0];
  int li[6];
  const unsigned flips = face_stencil<DIR>(p, c, li);
  const bool fl2 = flips & 4u, fl3 = flips & 8u;
  // ---- cotangent of the face flux (global frame)
  const double sc = (use_dt ? coef * dtg[0] : coef) / p.dx[DIR];
  const bool inL = c[DIR] > 0, inR = c[DIR] < p.n[DIR];
  double Fb[NV];
  bool any = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double g = 0.0;
    if (inR) g += lam[v * n + li[3]];
    if (inL) g -= lam[v * n + li[2]];
    Fb[v] = sc * g;
    any = any || (g != 0.0);
  }
  if (!any) return;
  const uint16_t m16 = mask[f];
  // ---- diffusion and regularization fluxes
  if (p.diff) diffusion_face_vjp<NS, DIM, DIR>(p, Q, li, Fb, Qb);
  if (p.cdi && !(m16 & 32)) cdi_face_vjp<NS, DIM, DIR>(p, Q, c, li, fl2, fl3, dtg[1], Fb, Qb);
  // ---- advective flux: cotangent in the face frame
  double Frb[NV];
#pragma unroll
  for (int k = 0; k < NS; ++k) Frb[k] = Fb[k];
  Frb[NS] = Fb[NS + DIR];
#pragma unroll
  for (int t = 0; t < NT; ++t) Frb[NS + 1 + t] = Fb[NS + tdir<DIM, DIR>(t)];
  Frb[NS + DIM] = Fb[NS + DIM];
  if (m16 & 16) {
    // first-order fallback: HLLC of the two cell states
    Side<NS, DIM, double> cl, cr, clb, crb;
    cell_side_at<NS, DIM, DIR>(p, Q, Uk, li[2], fl2, cl);
    cell_side_at<NS, DIM, DIR>(p, Q, Uk, li[3], fl3, cr);
    side_zero<NS, DIM>(clb);
    side_zero<NS, DIM>(crb);
    hllc_vjp<NS, DIM>(cl, cr, Frb, clb, crb);
    scatter_cell_side<NS, DIM, DIR>(p, Qb, Ub, li[2], fl2, clb);
    scatter_cell_side<NS, DIM, DIR>(p, Qb, Ub, li[3], fl3, crb);
    return;
  }
  const double* __restrict__ QT = Q + p.qT * n;
  const double* __restrict__ QP = Q + p.qP * n;
  const double* __restrict__ QUn = Q + (p.qU + DIR) * n;
  // ---- forward recompute: face average, eigenvector coefficients
  double ub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double a = Uk[v * n + li[2]], b = Uk[v * n + li[3]];
    if (v == NS + DIR) {
      if (fl2) a = -a;
      if (fl3) b = -b;
    }
    ub[v] = 0.5 * (a + b);
  }
  double cT, z, af;
  {
    Thermo<NS, DIM> tf;
    equilibrium<NS, DIM>(p, ub, tf, true);
    cT = tf.cT;
    z = tf.z;
    af = tf.a;
  }
  // ---- forward recompute: reconstruction
  double w1L, w1R, w5L, w5R, w6L, w6R, YL[NS], YR[NS], utL[NTa], utR[NTa];
  {
    double w[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) w[m] = QT[li[m]] - cT * QP[li[m]];
    double2 o = weno5z_lr(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp);
    w1L = o.x;
    w1R = o.y;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double* __restrict__ QY = Q + (p.qY + k) * n;
      o = weno5z_lr(QY[li[0]], QY[li[1]], QY[li[2]], QY[li[3]], QY[li[4]], QY[li[5]], p.weps, p.wp);
      YL[k] = o.x;
      YR[k] = o.y;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double* __restrict__ QUt = Q + (p.qU + tdir<DIM, DIR>(t)) * n;
      o = weno5z_lr(QUt[li[0]], QUt[li[1]], QUt[li[2]], QUt[li[3]], QUt[li[4]], QUt[li[5]], p.weps, p.wp);
      utL[t] = o.x;
      utR[t] = o.y;
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double un = (flips >> m) & 1u ? -QUn[li[m]] : QUn[li[m]];
      w[m] = 0.5 * z * un + 0.5 * QP[li[m]];
    }
    o = weno5z_lr(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp);
    w5L = o.x;
    w5R = o.y;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double un = (flips >> m) & 1u ? -QUn[li[m]] : QUn[li[m]];
      w[m] = -0.5 * z * un + 0.5 * QP[li[m]];
    }
    o = weno5z_lr(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp);
    w6L = o.x;
    w6R = o.y;
  }
  const double PLr = w5L + w6L, PRr = w5R + w6R;
  const double unL = (w5L - w6L) / z, unR = (w5R - w6R) / z;
  const double TLr = w1L + cT * PLr, TRr = w1R + cT * PRr;
  double cYL[NS], cYR[NS], YLl[NS], YRl[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    cYL[k] = Q[(p.qY + k) * n + li[2]];
    cYR[k] = Q[(p.qY + k) * n + li[3]];
    YLl[k] = YL[k];
    YRl[k] = YR[k];
  }
  if (p.pos) {
    ylimit<NS, double>(YLl, cYL);
    ylimit<NS, double>(YRl, cYR);
  }
  const double TL = (m16 & 1) ? QT[li[2]] : TLr, TR = (m16 & 2) ? QT[li[3]] : TRr;
  const double PL = (m16 & 4) ? QP[li[2]] : PLr, PR = (m16 & 8) ? QP[li[3]] : PRr;
  // ---- reverse: HLLC and face EOS
  double PLb = 0.0, TLb = 0.0, unLb = 0.0, YLb[NS], utLb[NTa];
  double PRb = 0.0, TRb = 0.0, unRb = 0.0, YRb[NS], utRb[NTa];
#pragma unroll
  for (int k = 0; k < NS; ++k) YLb[k] = YRb[k] = 0.0;
#pragma unroll
  for (int t = 0; t < NTa; ++t) utLb[t] = utRb[t] = 0.0;
  {
    Side<NS, DIM, double> sL, sR, sLb, sRb;
    face_state<NS, DIM, double>(p, PL, TL, YLl, unL, utL, sL);
    face_state<NS, DIM, double>(p, PR, TR, YRl, unR, utR, sR);
    side_zero<NS, DIM>(sLb);
    side_zero<NS, DIM>(sRb);
    hllc_vjp<NS, DIM>(sL, sR, Frb, sLb, sRb);
    face_state_vjp<NS, DIM>(p, PL, TL, YLl, unL, utL, sLb, PLb, TLb, YLb, unLb, utLb);
    face_state_vjp<NS, DIM>(p, PR, TR, YRl, unR, utR, sRb, PRb, TRb, YRb, unRb, utRb);
  }
  // ---- reverse: interpolation limiters (decisions from the mask)
  double cTb = 0.0, zb = 0.0, w1Lb = 0.0, w1Rb = 0.0;
  if (m16 & 4) {
    aadd(Qb + p.qP * n + li[2], PLb);
    PLb = 0.0;
  }
  if (m16 & 8) {
    aadd(Qb + p.qP * n + li[3], PRb);
    PRb = 0.0;
  }
  if (m16 & 1) {
    aadd(Qb + p.qT * n + li[2], TLb);
  } else {
    w1Lb = TLb;
    cTb += TLb * PLr;
    PLb += cT * TLb;
  }
  if (m16 & 2) {
    aadd(Qb + p.qT * n + li[3], TRb);
  } else {
    w1Rb = TRb;
    cTb += TRb * PRr;
    PRb += cT * TRb;
  }
  double YLrb[NS], YRrb[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) YLrb[k] = YRrb[k] = 0.0;
  if (p.pos) {
    double cYLb[NS], cYRb[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) cYLb[k] = cYRb[k] = 0.0;
    ylimit_vjp<NS>(YL, cYL, YLb, YLrb, cYLb);
    ylimit_vjp<NS>(YR, cYR, YRb, YRrb, cYRb);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      aadd(Qb + (p.qY + k) * n + li[2], cYLb[k]);
      aadd(Qb + (p.qY + k) * n + li[3], cYRb[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      YLrb[k] = YLb[k];
      YRrb[k] = YRb[k];
    }
  }
  // P = w5 + w6, u_n = (w5 - w6) / z
  const double w5Lb = PLb + unLb / z, w6Lb = PLb - unLb / z;
  const double w5Rb = PRb + unRb / z, w6Rb = PRb - unRb / z;
  zb -= unLb * unL / z + unRb * unR / z;
  // ---- reverse: WENO5-Z of each characteristic variable, scattered to the stencil
  double Tb6[6], Pb6[6], Unb6[6];
  {
    double w[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) w[m] = QT[li[m]] - cT * QP[li[m]];
    const D6 g = weno5z_lr_vjp(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp, w1Lb, w1Rb, 0.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      Tb6[m] = g.v[m];
      Pb6[m] = -cT * g.v[m];
      cTb -= g.v[m] * QP[li[m]];
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double* __restrict__ QY = Q + (p.qY + k) * n;
    const D6 g = weno5z_lr_vjp(QY[li[0]], QY[li[1]], QY[li[2]], QY[li[3]], QY[li[4]], QY[li[5]], p.weps,
                               p.wp, YLrb[k], YRrb[k], 1.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) aadd(Qb + (p.qY + k) * n + li[m], g.v[m]);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int qf = p.qU + tdir<DIM, DIR>(t);
    const double* __restrict__ QUt = Q + qf * n;
    const D6 g = weno5z_lr_vjp(QUt[li[0]], QUt[li[1]], QUt[li[2]], QUt[li[3]], QUt[li[4]], QUt[li[5]], p.weps,
                               p.wp, utLb[t], utRb[t], af);
#pragma unroll
    for (int m = 0; m < 6; ++m) aadd(Qb + qf * n + li[m], g.v[m]);
  }
  {
    double un6[6], w[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      un6[m] = (flips >> m) & 1u ? -QUn[li[m]] : QUn[li[m]];
      w[m] = 0.5 * z * un6[m] + 0.5 * QP[li[m]];
    }
    const D6 g5 = weno5z_lr_vjp(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp, w5Lb, w5Rb, 0.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) w[m] = -0.5 * z * un6[m] + 0.5 * QP[li[m]];
    const D6 g6 = weno5z_lr_vjp(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp, w6Lb, w6Rb, 0.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      Pb6[m] += 0.5 * (g5.v[m] + g6.v[m]);
      const double unb = 0.5 * z * (g5.v[m] - g6.v[m]);
      Unb6[m] = (flips >> m) & 1u ? -unb : unb;
      zb += 0.5 * un6[m] * (g5.v[m] - g6.v[m]);
    }
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    aadd(Qb + p.qT * n + li[m], Tb6[m]);
    aadd(Qb + p.qP * n + li[m], Pb6[m]);
    aadd(Qb + (p.qU + DIR) * n + li[m], Unb6[m]);
  }
  // ---- reverse: face-average equilibrium (forward mode, one tangent per
  // conserved variable of the average)
  if (cTb != 0.0 || zb != 0.0) {
    for (int v = 0; v < NV; ++v) {
      Dual<1> ud[NV];
#pragma unroll
      for (int w = 0; w < NV; ++w) {
        ud[w] = Dual<1>(ub[w]);
        ud[w].d[0] = (w == v) ? 1.0 : 0.0;
      }
      ThermoT<NS, DIM, Dual<1>> td;
      equilibrium_t<NS, DIM, Dual<1>>(p, ud, td, true);
      const double gb = 0.5 * (cTb * td.cT.d[0] + zb * td.z.d[0]);
      const bool mom = (v == NS + DIR);
      aadd(Ub + v * n + li[2], (mom && fl2) ? -gb : gb);
      aadd(Ub + v * n + li[3], (mom && fl3) ? -gb : gb);
    }
  }
}

template <int NS, int DIM, int DIR>
__global__ __launch_bounds__(256) void k_face_vjp(const Params p, const double* __restrict__ Uk,
                                                  const double* __restrict__ Q,
                                                  const uint16_t* __restrict__ mask,
                                                  const double* __restrict__ dtg, double coef, bool use_dt,
                                                  const double* __restrict__ lam, double* __restrict__ Qb,
                                                  double* __restrict__ Ub) {
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1), e2 = p.n[2] + (DIR == 2);
  int c[3];
  if (!face_coords<DIR>(e0, e1, e2, c)) return;
  face_vjp<NS, DIM, DIR>(p, c, Uk, Q, mask, dtg, coef, use_dt, lam, Qb, Ub);
}

// ---------------------------------------------------------------------------
// k_cell_vjp: U-bar_i += (dQ_i / dU_i)^T Q-bar_i, forward mode through the
// per-cell equilibrium and auxiliaries (one tangent per conserved variable).
// ---------------------------------------------------------------------------
template <int NS, int DIM>
__host__ __device__ void cell_vjp(const Params& p, long i, const double* __restrict__ U,
                                  const double* __restrict__ Qb, double* __restrict__ Ub) {
  constexpr int NV = NS + DIM + 1;
  const long n = p.ncell;
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[v * n + i];
  const bool aux = p.cdi || p.diff;
  for (int v = 0; v < NV; ++v) {
    Dual<1> ud[NV];
#pragma unroll
    for (int w = 0; w < NV; ++w) {
      ud[w] = Dual<1>(u[w]);
      ud[w].d[0] = (w == v) ? 1.0 : 0.0;
    }
    CellQ<NS, DIM, Dual<1>> q;
    cell_quantities_t<NS, DIM, Dual<1>>(p, ud, q, aux);
    double acc = Qb[p.qT * n + i] * q.T.d[0] + Qb[p.qP * n + i] * q.P.d[0] +
                 Qb[p.qRho * n + i] * q.rho.d[0] + Qb[p.qA * n + i] * q.a.d[0];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc += Qb[(p.qY + k) * n + i] * q.Y[k].d[0];
#pragma unroll
    for (int d = 0; d < DIM; ++d) acc += Qb[(p.qU + d) * n + i] * q.vel[d].d[0];
    if (p.cdi) {
      acc += Qb[p.qPhi0 * n + i] * q.phi[0].d[0] + Qb[p.qPhi1 * n + i] * q.phi[1].d[0] +
             Qb[p.qPsi * n + i] * q.psi.d[0];
#pragma unroll
      for (int k = 0; k < NS; ++k) acc += Qb[(p.qYrho + k) * n + i] * q.yrho[k].d[0];
      acc += Qb[(p.qHrho + 0) * n + i] * q.hrho[0].d[0] + Qb[(p.qHrho + 1) * n + i] * q.hrho[1].d[0];
    }
    if (p.diff) {
#pragma unroll
      for (int k = 0; k < NS; ++k)
        acc += Qb[(p.qChi + k) * n + i] * q.chi[k].d[0] + Qb[(p.qK + k) * n + i] * q.K[k].d[0] +
               Qb[(p.qH + k) * n + i] * q.h[k].d[0];
    }
    Ub[v * n + i] += acc;
  }
}

template <int NS, int DIM>
__global__ __launch_bounds__(256) void k_cell_vjp(const Params p, const double* __restrict__ U,
                                                  const double* __restrict__ Qb, double* __restrict__ Ub) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.ncell) cell_vjp<NS, DIM>(p, i, U, Qb, Ub);
}

// out = a x + b y + c z over m values (y, z nullable)
__global__ __launch_bounds__(256) void k_lincomb(long m, double a, const double* __restrict__ x, double b,
                                                 const double* __restrict__ y, double c,
                                                 const double* __restrict__ zz, double* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double r = a * x[i];
  if (y) r += b * y[i];
  if (zz) r += c * zz[i];
  out[i] = r;
}

__global__ __launch_bounds__(256) void k_fill_zero(long m, double* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = 0.0;
}

}  // namespace mpmc
