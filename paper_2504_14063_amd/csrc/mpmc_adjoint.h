// mpmc_adjoint.h -- discrete adjoint (vector-Jacobian products) of one SSP-RK3
// step of the four-equation MPMC hot path with frozen decisions.
//
// Frozen decisions: the limiter selections of Sec. 3.3 (T/P fallback,
// first-order flux, dropped regularization flux) are read from the masks the
// forward recompute of the same stage recorded; the arms of min/max/abs/sign
// (HLLC wave speeds and sign of s*, |beta_0 - beta_2| of WENO-Z, the Y-limiter
// branch) are those of the recomputed forward values.  The WENO-Z weights are
// differentiated.  Reverse-mode derivatives are written by hand for the
// whole path: the face pipeline, the face-average and per-cell equilibria and
// the per-cell auxiliaries.  Faces write their cotangents into per-face
// records and each cell gathers them in a fixed order (no floating-point
// atomics), so results are bitwise reproducible.
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
  // the forward's operation order (curvatures and inner candidates shared
  // with the mirrored reconstruction of the face's other side)
  const double t0 = (f0 + f2) - 2 * f1, s0 = f0 - 4 * f1 + 3 * f2;
  const double t1 = (f1 + f3) - 2 * f2, s1 = f1 - f3;
  const double t2 = (f2 + f4) - 2 * f3, s2 = 3 * f2 - 4 * f3 + f4;
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
  const double q1 = (5 * f2 + (2 * f3 - f1)) * s6;
  const double q2 = (5 * f3 + (2 * f2 - f4)) * s6;
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
// Equilibrium of a conserved state (Sec. 2.3: closed-form pressure root, T,
// the sound speed), forward with its intermediates kept, and reverse from
// cotangents of a^2, beta, alpha, T, P, rho, Y_k and the velocity, with the
// branches the forward takes.
// ---------------------------------------------------------------------------
template <int NS, int DIM>
struct EqFwd {
  double rho, Y[NS], ke, e, v, qm, R1, Rg, vb, Ep, a1, a2, a3, sD, P, ipp[NS], ck[NS], den, T, sa, S2, Cp, sb,
      beta, alpha, W, a2s;
  bool lin;
};

template <int NS, int DIM>
MPMC_HD void eq_forward(const Params& p, const double* u, EqFwd<NS, DIM>& f) {
  double rho = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) rho += u[k];
  f.rho = rho;
#pragma unroll
  for (int k = 0; k < NS; ++k) f.Y[k] = u[k] / rho;
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) ke += 0.5 * u[NS + d] * (u[NS + d] / rho);
  f.ke = ke;
  f.e = (u[NS + DIM] - ke) / rho;
  f.v = 1.0 / rho;
  double qm = 0.0, bm = 0.0, Cv = 0.0, R1 = 0.0, Rg = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    qm += f.Y[k] * p.q[k];
    bm += f.Y[k] * p.b[k];
    Cv += f.Y[k] * p.cv[k];
    if (p.pinf[k] != 0.0)
      R1 += f.Y[k] * p.gm1cv[k];
    else
      Rg += f.Y[k] * p.gm1cv[k];
  }
  f.qm = qm;
  f.R1 = R1;
  f.Rg = Rg;
  f.vb = f.v - bm;
  f.Ep = (f.e - qm) / f.vb;
  f.a1 = Cv;
  f.a2 = f.Ep * (R1 + Rg) - p.Pst * (Cv + R1);
  f.a3 = f.Ep * p.Pst * Rg;
  f.lin = Rg == 0.0;
  f.sD = 0.0;
  if (f.lin) {
    f.P = f.a2 / f.a1;
  } else {
    f.sD = sqrt(f.a2 * f.a2 + 4.0 * f.a1 * f.a3);
    f.P = f.a2 >= 0.0 ? (f.a2 + f.sD) / (2.0 * f.a1) : 2.0 * f.a3 / (f.sD - f.a2);
  }
  double den = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    f.ipp[k] = 1.0 / (f.P + p.pinf[k]);
    f.ck[k] = p.pinf[k] == 0.0 ? p.cv[k] : p.cv[k] * (f.P + p.gam[k] * p.pinf[k]) * f.ipp[k];
    den += f.Y[k] * f.ck[k];
  }
  f.den = den;
  f.T = (f.e - qm) / den;
  double sa = 0.0, S2 = 0.0, Cp = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double kp = p.gm1cv[k] * f.ipp[k];
    sa += f.Y[k] * kp;
    S2 += f.Y[k] * kp * f.ipp[k];
    Cp += f.Y[k] * p.gcv[k];
  }
  f.sa = sa;
  f.S2 = S2;
  f.Cp = Cp;
  f.sb = S2 * f.T;
  f.beta = rho * f.sb;
  f.alpha = rho * sa;
  f.W = rho * f.beta * Cp - f.alpha * f.alpha * f.T;
  f.a2s = Cp / f.W;
}

// ub += (d(a^2, beta, alpha, T, P, rho, Y, vel) / d u)^T (cotangents); Yb0,
// velb0 nullable.
template <int NS, int DIM>
MPMC_HD void eq_reverse(const Params& p, const double* u, const EqFwd<NS, DIM>& f, double a2sb, double betab,
                        double alphab, double Tb, double Pb, double rhob, const double* Yb0, const double* velb0,
                        double* ub) {
  const double rho = f.rho, T = f.T, P = f.P;
  // a^2 = Cp / W, W = rho beta Cp - alpha^2 T
  double Cpb = a2sb / f.W;
  const double Wb = -a2sb * f.a2s / f.W;
  rhob += Wb * f.beta * f.Cp;
  betab += Wb * rho * f.Cp;
  Cpb += Wb * rho * f.beta;
  alphab -= Wb * 2.0 * f.alpha * T;
  Tb -= Wb * f.alpha * f.alpha;
  // beta = rho T S2, alpha = rho sa
  rhob += betab * f.sb + alphab * f.sa;
  const double sbb = betab * rho, sab = alphab * rho;
  Tb += sbb * f.S2;
  const double S2b = sbb * T;
  double Yb[NS], ippb[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double kp = p.gm1cv[k] * f.ipp[k];
    Yb[k] = (Yb0 ? Yb0[k] : 0.0) + sab * kp + S2b * kp * f.ipp[k] + Cpb * p.gcv[k];
    ippb[k] = sab * f.Y[k] * p.gm1cv[k] + S2b * f.Y[k] * 2.0 * p.gm1cv[k] * f.ipp[k];
  }
  // T = (e - qm) / den
  double eb = Tb / f.den, qmb = -Tb / f.den;
  const double denb = -Tb * T / f.den;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    Yb[k] += denb * f.ck[k];
    if (p.pinf[k] != 0.0) {
      Pb += denb * f.Y[k] * p.cv[k] * f.ipp[k];
      ippb[k] += denb * f.Y[k] * p.cv[k] * (P + p.gam[k] * p.pinf[k]);
    }
    Pb -= ippb[k] * f.ipp[k] * f.ipp[k];
  }
  // pressure root
  double a1b = 0.0, a2b = 0.0, a3b = 0.0;
  if (f.lin) {
    a2b += Pb / f.a1;
    a1b -= Pb * P / f.a1;
  } else {
    double sDb;
    if (f.a2 >= 0.0) {
      a2b += Pb / (2.0 * f.a1);
      sDb = Pb / (2.0 * f.a1);
      a1b -= Pb * P / f.a1;
    } else {
      a3b += Pb * 2.0 / (f.sD - f.a2);
      sDb = -Pb * P / (f.sD - f.a2);
      a2b += Pb * P / (f.sD - f.a2);
    }
    a2b += sDb * f.a2 / f.sD;
    a1b += sDb * 2.0 * f.a3 / f.sD;
    a3b += sDb * 2.0 * f.a1 / f.sD;
  }
  const double Pinf = p.Pst;
  const double Cvb = a1b - a2b * Pinf;
  const double Epb = a2b * (f.R1 + f.Rg) + a3b * Pinf * f.Rg;
  const double R1b = a2b * (f.Ep - Pinf);
  const double Rgb = a2b * f.Ep + a3b * f.Ep * Pinf;
  eb += Epb / f.vb;
  qmb -= Epb / f.vb;
  const double vbb = -Epb * f.Ep / f.vb;
  const double bmb = Epb * f.Ep / f.vb;
#pragma unroll
  for (int k = 0; k < NS; ++k)
    Yb[k] += qmb * p.q[k] + bmb * p.b[k] + Cvb * p.cv[k] + (p.pinf[k] != 0.0 ? R1b : Rgb) * p.gm1cv[k];
  rhob -= vbb * f.v * f.v;
  // e = (E - ke) / rho, ke = sum m_d^2 / (2 rho); vel_d = m_d / rho
  const double keb = -eb / rho;
  ub[NS + DIM] += eb / rho;
  rhob -= eb * f.e / rho + keb * f.ke / rho;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double vd = u[NS + d] / rho, vb_ = velb0 ? velb0[d] : 0.0;
    ub[NS + d] += keb * vd + vb_ / rho;
    rhob -= vb_ * vd / rho;
  }
  // Y_k = u_k / rho, rho = sum u_k
  double sY = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) sY += Yb[k] * f.Y[k];
  rhob -= sY / rho;
#pragma unroll
  for (int k = 0; k < NS; ++k) ub[k] += Yb[k] / rho + rhob;
}

// Eigenvector coefficients of the face-average state (App. A), reverse mode:
// ub += (d cT / d u)^T cTb + (d z / d u)^T zb.  One forward and one reverse
// sweep in place of one tangent pass per conserved variable.
template <int NS, int DIM>
MPMC_HD void equilibrium_cz_vjp(const Params& p, const double* u, double cTb, double zb, double* ub) {
  EqFwd<NS, DIM> f;
  eq_forward<NS, DIM>(p, u, f);
  const double rho = f.rho, a2s = f.a2s, a = sqrt(a2s);
  // cT = (rho a^2 beta - 1) / (alpha a^2 rho), z = a rho
  const double Nn = rho * a2s * f.beta - 1.0, Dd = f.alpha * a2s * rho, cT = Nn / Dd;
  double rhob = zb * a, a2sb = zb * rho / (2.0 * a);
  const double Nb = cTb / Dd, Db = -cTb * cT / Dd;
  rhob += Nb * a2s * f.beta + Db * f.alpha * a2s;
  a2sb += Nb * rho * f.beta + Db * f.alpha * rho;
  const double betab = Nb * rho * a2s, alphab = Db * a2s * rho;
  eq_reverse<NS, DIM>(p, u, f, a2sb, betab, alphab, 0.0, 0.0, rhob, nullptr, nullptr, ub);
}

// ---------------------------------------------------------------------------
// Cell quantities (the equilibrium and, with aux, the phase auxiliaries of
// Secs. 2.2 and 3.2: phase volume fractions, densities, the psi transform,
// Wilke viscosity and the diffusion coefficients), reverse mode: ub +=
// (dQ/du)^T qb for the cotangents of the quantities a face reads.
// ---------------------------------------------------------------------------
template <int NS, int DIM>
struct CellQb {
  double T, P, rho, a, phi0, phi1, psi, hrho[2];
  double Y[NS], vel[DIM], yrho[NS], chi[NS], K[NS], h[NS];
  MPMC_HD void zero() {
    T = P = rho = a = phi0 = phi1 = psi = hrho[0] = hrho[1] = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) Y[k] = yrho[k] = chi[k] = K[k] = h[k] = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) vel[d] = 0.0;
  }
};

template <int NS, int DIM>
MPMC_HD void cell_quantities_vjp(const Params& p, const double* u, const CellQb<NS, DIM>& qb, bool aux,
                                 double* ub) {
  EqFwd<NS, DIM> f;
  eq_forward<NS, DIM>(p, u, f);
  const double T = f.T, P = f.P;
  double Tb = qb.T, Pb = qb.P;
  if (aux) {
    // ---- forward of the phase auxiliaries
    double vk[NS], hk[NS], y[NS], rYp[2] = {0.0, 0.0}, rhop[2] = {0.0, 0.0}, hp[2] = {0.0, 0.0};
    double phi[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      vk[k] = (p.gm1cv[k] / (P + p.pinf[k])) * T + p.b[k];
      hk[k] = p.gcv[k] * T + p.b[k] * P + p.q[k];
    }
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      if (pp >= p.np) break;
      const int ph = p.pid[pp];
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) rYp[pp] += u[k];
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) y[k] = rYp[pp] > 1e-300 ? u[k] / rYp[pp] : p.inpn[pp];
      double vp = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) {
          vp += y[k] * vk[k];
          hp[pp] += y[k] * hk[k];
          phi[pp] += u[k] * vk[k];
        }
      rhop[pp] = 1.0 / vp;
    }
    // ---- reverse
    double phib[2] = {qb.phi0, qb.phi1};
    if (p.np == 2 && psi_differentiable(p, phi[0], phi[1])) {
      phib[0] += qb.psi * p.eps / (phi[0] + p.delta);
      phib[1] -= qb.psi * p.eps / (phi[1] + p.delta);
    }
    if (p.np < 2) phib[1] = 0.0;
    double vkb[NS], hkb[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      vkb[k] = 0.0;
      hkb[k] = p.diff ? qb.h[k] : 0.0;
    }
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      if (pp >= p.np) break;
      const int ph = p.pid[pp];
      double ykb[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) ykb[k] = 0.0;
      double rhopb = 0.0;
      if (p.diff && p.multi[pp]) {
        // mup = sum_a y_a mu_a / den_a, den_a = sum_b y_b wilke_ab; winv =
        // sum y_k / W_k, Wp = 1 / winv; chi_k = y_k Wp / W_k; K_k = mup W_k /
        // (rhop Sc_k Wp)
        double dena[NS], mup = 0.0, winv = 0.0;
#pragma unroll
        for (int a = 0; a < NS; ++a) {
          if (p.phase[a] != ph) continue;
          double d = 0.0;
#pragma unroll
          for (int b = 0; b < NS; ++b)
            if (p.phase[b] == ph) d += y[b] * p.wilke[a][b];
          dena[a] = d;
          mup += y[a] * p.mu[a] / d;
        }
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) winv += y[k] / p.W[k];
        const double Wp = 1.0 / winv;
        double mupb = 0.0, Wpb = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) {
            const double Kk = mup * p.W[k] / (rhop[pp] * p.Sc[k] * Wp);
            mupb += qb.K[k] * p.W[k] / (rhop[pp] * p.Sc[k] * Wp);
            rhopb -= qb.K[k] * Kk / rhop[pp];
            Wpb -= qb.K[k] * Kk / Wp;
            ykb[k] += qb.chi[k] * Wp / p.W[k];
            Wpb += qb.chi[k] * y[k] / p.W[k];
          }
        const double winvb = -Wpb * Wp * Wp;
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) ykb[k] += winvb / p.W[k];
#pragma unroll
        for (int a = 0; a < NS; ++a) {
          if (p.phase[a] != ph) continue;
          ykb[a] += mupb * p.mu[a] / dena[a];
          const double denb = -mupb * y[a] * p.mu[a] / (dena[a] * dena[a]);
#pragma unroll
          for (int b = 0; b < NS; ++b)
            if (p.phase[b] == ph) ykb[b] += denb * p.wilke[a][b];
        }
      }
      // yrho_k = y_k rhop, hrho = rhop hp, phi = sum u_k vk_k
      double hpb = 0.0;
      if (p.cdi) {
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) {
            ykb[k] += qb.yrho[k] * rhop[pp];
            rhopb += qb.yrho[k] * y[k];
          }
        rhopb += qb.hrho[pp] * hp[pp];
        hpb = qb.hrho[pp] * rhop[pp];
      }
      // rhop = 1 / vp, vp = sum y vk, hp = sum y hk
      const double vpb = -rhopb * rhop[pp] * rhop[pp];
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) {
          ub[k] += phib[pp] * vk[k];
          vkb[k] += phib[pp] * u[k] + vpb * y[k];
          hkb[k] += hpb * y[k];
          ykb[k] += vpb * vk[k] + hpb * hk[k];
        }
      // y_k = u_k / rYp (a constant where the phase is absent)
      if (rYp[pp] > 1e-300) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) s += ykb[k] * y[k];
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) ub[k] += (ykb[k] - s) / rYp[pp];
      }
    }
    // vk = gm1cv T / (P + pinf) + b, hk = gcv T + b P + q
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      Tb += vkb[k] * p.gm1cv[k] * f.ipp[k] + hkb[k] * p.gcv[k];
      Pb += -vkb[k] * p.gm1cv[k] * T * f.ipp[k] * f.ipp[k] + hkb[k] * p.b[k];
    }
  }
  // a = sqrt(a^2)
  const double a2sb = qb.a / (2.0 * sqrt(f.a2s));
  eq_reverse<NS, DIM>(p, u, f, a2sb, 0.0, 0.0, Tb, Pb, qb.rho, qb.Y, qb.vel, ub);
}

// ---------------------------------------------------------------------------
// Face records.  The pull-back of a face writes each cotangent it produces
// into a record of its own (every entry written by its face only); a per-cell
// pass then sums, for each cell, the entries of the faces that reference it,
// in a fixed order.  No address is written by two threads and no sum depends
// on scheduling, so the adjoint is bitwise reproducible.  Records are stored
// in tiles of 64 faces, [face / 64][slot][face % 64]: one wavefront's reads or
// writes of a slot are 512 contiguous bytes and its whole tile is contiguous.
//
//   far(m, j)   stencil position m = 0..5: cotangent of cell quantity j of
//               cell li[m] (T, P, u_n, Y_k, u_t; momentum flips of the
//               boundary maps applied); at m = 2, 3 (the face cells) it also
//               holds the direct terms (limiters, regularization, diffusion)
//   near(s, j)  face cell s (0: li[2], 1: li[3]): cotangents of rho, a,
//               phi_0, phi_1 and of the conserved E and rhoY_k
//   shared      one value for both face cells: yrho_k, hrho_0, hrho_1, psi,
//               h_k, K_k, chi_k (added to li[3], subtracted from li[2]) and the
//               face-average cotangent of U (normal momentum flipped per side)
//   tan(t)      cotangent of the tangential psi differences of the
//               regularization flux, multiplied in the gather by the target
//               cell's own d psi / d phi
//
// Entries that are zero by construction for a face are neither written nor
// read; both sides decide from the face's stage mask and the options:
//   near a, E, rhoY_k             only where the first-order fallback is on
//   shared face-average entries   only where it is off
//   near phi, yrho, hrho, psi, tan only where the regularization flux is on
//                                 and not dropped
//   h, K, chi                     only with diffusion
// (a face whose flux cotangent is zero writes every entry, as zero).
// ---------------------------------------------------------------------------
template <int NS, int DIM>
struct RecL {
  static constexpr int NT = DIM - 1, NV = NS + DIM + 1;
  static constexpr int NF = 3 + NS + NT;
  static constexpr int FT = 0, FP = 1, FUN = 2, FY = 3, FUT = 3 + NS;
  static constexpr int NRHO = 0, NA = 1, NPHI0 = 2, NPHI1 = 3, NE = 4, NRY = 5, NN = 5 + NS;
  static constexpr int NEAR = 6 * NF, SH = NEAR + 2 * NN;
  static constexpr int SYRHO = SH, SHRHO = SH + NS, SPSI = SHRHO + 2, SHH = SPSI + 1, SK = SHH + NS,
                       SCHI = SK + NS, SGB = SCHI + NS, TAN = SGB + NV, N = TAN + NT;
  static MPMC_HD constexpr int far(int m, int j) { return m * NF + j; }
  static MPMC_HD constexpr int near(int s, int j) { return NEAR + s * NN + j; }
  // position of entry (slot, face f) in a direction's record array
  static MPMC_HD long idx(int slot, long f) { return ((f >> 6) * N + slot) * 64 + (f & 63); }
};

// Record slots per face for ns species in dim dimensions (host sizing), and
// the doubles a direction with nf faces takes (whole tiles of 64 faces).
inline int rec_slots(int ns, int dim) {
  const int nt = dim - 1, nv = ns + dim + 1;
  return 6 * (3 + ns + nt) + 2 * (5 + ns) + (4 * ns + 3 + nv) + nt;
}
inline long rec_doubles(int ns, int dim, long nf) { return (long)rec_slots(ns, dim) * ((nf + 63) / 64) * 64; }

// Writer of one face's record.
template <int NS, int DIM>
struct RecW {
  double* __restrict__ r;
  long f;
  MPMC_HD void put(int slot, double v) const { r[RecL<NS, DIM>::idx(slot, f)] = v; }
  MPMC_HD void add(int slot, double v) const { r[RecL<NS, DIM>::idx(slot, f)] += v; }
};

// Hand-over between the two halves of a face's pull-back (slot-major, one
// entry per face): the cotangents of the reconstructed characteristic values
// of both sides, the partial cotangents of cT and z, and a flag (1: the
// reconstruction is to be pulled back; 0: the first half wrote the whole
// record).
template <int NS, int DIM>
struct MidL {
  static constexpr int NT = DIM - 1;
  static constexpr int W1L = 0, W1R = 1, W5L = 2, W5R = 3, W6L = 4, W6R = 5, YL = 6, YR = 6 + NS,
                       UTL = 6 + 2 * NS, UTR = UTL + NT, CTB = UTR + NT, ZB = CTB + 1, FLAG = ZB + 1,
                       N = FLAG + 1;
};
inline int mid_slots(int ns, int dim) { return 9 + 2 * ns + 2 * (dim - 1); }

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

// ---------------------------------------------------------------------------
// Regularization flux of one face (Sec. 3.2.1), reverse mode.  Fb: cotangent
// of the face flux in the global frame.  Writes the near u, phi entries, the
// shared yrho, hrho, psi entries and tan.
// ---------------------------------------------------------------------------
template <int NS, int DIM, int DIR>
__host__ __device__ void cdi_face_vjp(const Params& p, const double* __restrict__ Q, const int* c, const int* li,
                                      bool fl2, bool fl3, double Gamma, const double* Fb, const RecW<NS, DIM>& w) {
  using L = RecL<NS, DIM>;
  constexpr int NT = DIM - 1;
  constexpr int NTa = NT > 0 ? NT : 1;
  const long n = p.ncell;
  const double dxn = p.dx[DIR];
  const int l2 = li[2], l3 = li[3];
  // ---- forward recompute
  // (the same values as the forward kernel: psi differences of the stored psi)
  const double f0L = ldrow(Q + p.qPhi0 * n, l2), f1L = ldrow(Q + p.qPhi1 * n, l2);
  const double f0R = ldrow(Q + p.qPhi0 * n, l3), f1R = ldrow(Q + p.qPhi1 * n, l3);
  const double psiL = ldrow(Q + p.qPsi * n, l2), psiR = ldrow(Q + p.qPsi * n, l3);
  const double psib = 0.5 * (psiL + psiR);
  const double gn = (psiR - psiL) / dxn;
  double nrm2 = gn * gn, gt[NTa];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int td = tdir<DIM, DIR>(t);
    const int stride_t = td == 0 ? 1 : (td == 1 ? p.n[0] : p.n[0] * p.n[1]);
    double g = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      double ps[2];
#pragma unroll
      for (int sgn = 0; sgn < 2; ++sgn) {
        bool flip = false;
        const int ct = c[td] + (sgn ? 1 : -1);
        const int mt = (ct < 0 || ct >= p.n[td]) ? map_index(ct, p.n[td], p.bclo[td], p.bchi[td], flip) : ct;
        const int lt = li[2 + side] + (mt - c[td]) * stride_t;
        ps[sgn] = ldrow(Q + p.qPsi * n, lt);
      }
      g += ps[1] - ps[0];
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
  double Rsum = 0.0;
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    const int ph = p.pid[pp];
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) Rsum += -0.5 * (ldrow(Q + (p.qYrho + k) * n, l2) + ldrow(Q + (p.qYrho + k) * n, l3)) * ap[pp];
  }
  double vL[DIM], vR[DIM], kb = 0.0;
#pragma unroll
  for (int dd = 0; dd < DIM; ++dd) {
    vL[dd] = ldrow(Q + (p.qU + dd) * n, l2);
    vR[dd] = ldrow(Q + (p.qU + dd) * n, l3);
    if (dd == DIR) {
      if (fl2) vL[dd] = -vL[dd];
      if (fl3) vR[dd] = -vR[dd];
    }
    kb += vL[dd] * vR[dd];
  }
  kb *= 0.5;
  // ---- reverse
  const double Eb = Fb[NS + DIM];
  double Rsumb = Eb * kb;
  const double kbb = Eb * Rsum;
  double vLb[DIM], vRb[DIM];
#pragma unroll
  for (int dd = 0; dd < DIM; ++dd) {
    Rsumb += Fb[NS + dd] * 0.5 * (vL[dd] + vR[dd]);
    vLb[dd] = Fb[NS + dd] * 0.5 * Rsum + 0.5 * kbb * vR[dd];
    vRb[dd] = Fb[NS + dd] * 0.5 * Rsum + 0.5 * kbb * vL[dd];
  }
  w.put(L::far(2, L::FUN), fl2 ? -vLb[DIR] : vLb[DIR]);
  w.put(L::far(3, L::FUN), fl3 ? -vRb[DIR] : vRb[DIR]);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    w.put(L::far(2, L::FUT + t), vLb[tdir<DIM, DIR>(t)]);
    w.put(L::far(3, L::FUT + t), vRb[tdir<DIM, DIR>(t)]);
  }
  const double hRb = Eb;
  double a1b = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) w.put(L::SYRHO + k, 0.0);
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    const int ph = p.pid[pp];
    double apb = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) {
        const double Rkb = Fb[k] + Rsumb;
        apb += -0.5 * (ldrow(Q + (p.qYrho + k) * n, l2) + ldrow(Q + (p.qYrho + k) * n, l3)) * Rkb;
        w.put(L::SYRHO + k, -0.5 * ap[pp] * Rkb);
      }
    apb += -0.5 * (ldrow(Q + (p.qHrho + pp) * n, l2) + ldrow(Q + (p.qHrho + pp) * n, l3)) * hRb;
    w.put(L::SHRHO + pp, -0.5 * ap[pp] * hRb);
    a1b += pp == 0 ? apb : -apb;
  }
  // a1 = Gamma (eps gphi - shape nhat / 4)
  const double gphib = Gamma * p.eps * a1b;
  const double nhatb = -0.25 * Gamma * shape * a1b;
  const double thb = 0.5 * Gamma * th * nhat * a1b;
  const double psibb = thb * (1.0 - th * th) / (2.0 * p.eps);
  w.put(L::SPSI, 0.5 * psibb);
  double f0Lb = -gphib / dxn, f0Rb = gphib / dxn, f1Lb = 0.0, f1Rb = 0.0;
  double tanb[NTa];
#pragma unroll
  for (int t = 0; t < NTa; ++t) tanb[t] = 0.0;
  if (nrm2 > 0.0) {
    const double is3 = 1.0 / (s * nrm2);
    const double gnb = nhatb * (1.0 / s - gn * gn * is3);
    // gn = eps [ln(f0R+d) + ln(f1L+d) - ln(f0L+d) - ln(f1R+d)] / dx
    const double db = gnb / dxn;
    f0Rb += db * dlog_coef(p, f0R, f1R);
    f1Lb += db * dlog_coef(p, f1L, f0L);
    f0Lb -= db * dlog_coef(p, f0L, f1L);
    f1Rb -= db * dlog_coef(p, f1R, f0R);
    // gt[t] = sum over both face cells of dpsi(cell at -1, cell at +1) / (4 dx_t)
#pragma unroll
    for (int t = 0; t < NT; ++t) tanb[t] = -nhatb * gn * gt[t] * is3 / (4.0 * p.dx[tdir<DIM, DIR>(t)]);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) w.put(L::TAN + t, tanb[t]);
  w.put(L::near(0, L::NPHI0), f0Lb);
  w.put(L::near(1, L::NPHI0), f0Rb);
  w.put(L::near(0, L::NPHI1), f1Lb);
  w.put(L::near(1, L::NPHI1), f1Rb);
}

// Regularization off or dropped: the face cells' velocity entries start at
// zero (the regularization-only entries are not written).
template <int NS, int DIM>
MPMC_HD void cdi_face_zero(const RecW<NS, DIM>& w) {
  using L = RecL<NS, DIM>;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    w.put(L::far(2 + s, L::FUN), 0.0);
#pragma unroll
    for (int t = 0; t < DIM - 1; ++t) w.put(L::far(2 + s, L::FUT + t), 0.0);
  }
}

// ---------------------------------------------------------------------------
// Phase-confined species diffusion flux of one face, reverse mode.  Writes
// the shared h, K, chi entries, the face cells' Y entries and the near rho
// entries (zero when diffusion is off).
// ---------------------------------------------------------------------------
template <int NS, int DIM, int DIR>
__host__ __device__ void diffusion_face_vjp(const Params& p, const double* __restrict__ Q, const int* li,
                                            const double* Fb, const RecW<NS, DIM>& w) {
  using L = RecL<NS, DIM>;
  const long n = p.ncell;
  const double dxn = p.dx[DIR];
  const int l2 = li[2], l3 = li[3];
  double rhobb = 0.0, Hh[NS], Kh[NS], Gd[NS], Yh[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) Hh[k] = Kh[k] = Gd[k] = Yh[k] = 0.0;
  if (p.diff) {
    const double rhob = 0.5 * (ldrow(Q + p.qRho * n, l2) + ldrow(Q + p.qRho * n, l3));
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      if (pp >= p.np || !p.multi[pp]) continue;
      const int ph = p.pid[pp];
      double Yb[NS], Kb[NS], G[NS], Yp = 0.0, sKG = 0.0;
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) {
          Yb[k] = 0.5 * (ldrow(Q + (p.qY + k) * n, l2) + ldrow(Q + (p.qY + k) * n, l3));
          Kb[k] = 0.5 * (ldrow(Q + (p.qK + k) * n, l2) + ldrow(Q + (p.qK + k) * n, l3));
          G[k] = (ldrow(Q + (p.qChi + k) * n, l3) - ldrow(Q + (p.qChi + k) * n, l2)) / dxn;
          Yp += Yb[k];
          sKG += Kb[k] * G[k];
        }
      double Ypb = 0.0, sKGb = 0.0, Jb[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (p.phase[k] == ph) {
          const double Hb = 0.5 * (ldrow(Q + (p.qH + k) * n, l2) + ldrow(Q + (p.qH + k) * n, l3));
          const double inner = Kb[k] * Yp * G[k] - Yb[k] * sKG;
          const double J = -rhob * inner;
          Jb[k] = Fb[k] + Fb[NS + DIM] * Hb;
          Hh[k] = 0.5 * Fb[NS + DIM] * J;
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
          Kh[k] = 0.5 * Kbb;
          Gd[k] = Gb / dxn;
          Yh[k] = 0.5 * Ybb;
        }
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (p.diff) {
      w.put(L::SHH + k, Hh[k]);
      w.put(L::SK + k, Kh[k]);
      w.put(L::SCHI + k, Gd[k]);
    }
    w.put(L::far(2, L::FY + k), Yh[k]);
    w.put(L::far(3, L::FY + k), Yh[k]);
  }
  w.put(L::near(0, L::NRHO), 0.5 * rhobb);
  w.put(L::near(1, L::NRHO), 0.5 * rhobb);
}

// ---------------------------------------------------------------------------
// Pull-back of one face: the cotangent of the face flux, F-bar = coef [dt]
// (lam_R - lam_L) / dx (from L_i = -(F_hi - F_lo)/dx), through the face
// pipeline (recomputed forward, decisions from the stage mask) into the
// face's record in rec (the direction's record array).  Two halves, run as
// two kernels so that neither holds the whole pipeline's state:
//   face_vjp_a  regularization and diffusion fluxes, the first-order
//               fallback, and the reverse of HLLC, the face EOS and the
//               interpolation limiters down to the reconstructed values;
//   face_vjp_b  the WENO5-Z reconstructions and the face-average equilibrium.
// ---------------------------------------------------------------------------
template <int NS, int DIM, int DIR>
__host__ __device__ void face_vjp_a(const Params& p, const int* c, const double* __restrict__ Uk,
                                    const double* __restrict__ Q, const uint16_t* __restrict__ mask,
                                    const double* __restrict__ dtg, double coef, bool use_dt,
                                    const double* __restrict__ lam, double* __restrict__ rec,
                                    double* __restrict__ mid) {
  using L = RecL<NS, DIM>;
  using M = MidL<NS, DIM>;
  constexpr int NV = NS + DIM + 1;
  constexpr int NT = DIM - 1;
  constexpr int NTa = NT > 0 ? NT : 1;
  const long n = p.ncell;
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1), e2 = p.n[2] + (DIR == 2);
  const long f = ((long)c[2] * e1 + c[1]) * e0 + c[0];
  const long nfd = (long)e0 * e1 * e2;
  const RecW<NS, DIM> w{rec, f};
  auto mput = [&](int slot, double v) { strow_t<false>(mid + (long)slot * nfd, (int)f, v); };
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
    if (inR) g += ldrow(lam + v * n, li[3]);
    if (inL) g -= ldrow(lam + v * n, li[2]);
    Fb[v] = sc * g;
    any = any || (g != 0.0);
  }
  if (!any) {
    for (int s = 0; s < L::N; ++s) w.put(s, 0.0);
    mput(M::FLAG, 0.0);
    return;
  }
  const uint16_t m16 = mask[f];
  // ---- diffusion and regularization fluxes
  diffusion_face_vjp<NS, DIM, DIR>(p, Q, li, Fb, w);
  if (p.cdi && !(m16 & 32))
    cdi_face_vjp<NS, DIM, DIR>(p, Q, c, li, fl2, fl3, dtg[1], Fb, w);
  else
    cdi_face_zero<NS, DIM>(w);
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
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Side<NS, DIM, double>& sb = s ? crb : clb;
      const bool fl = s ? fl3 : fl2;
      w.add(L::near(s, L::NRHO), sb.rho);
      w.put(L::near(s, L::NA), sb.a);
      w.put(L::far(2 + s, L::FT), 0.0);
      w.put(L::far(2 + s, L::FP), sb.P);
      w.add(L::far(2 + s, L::FUN), fl ? -sb.un : sb.un);
#pragma unroll
      for (int t = 0; t < NT; ++t) w.add(L::far(2 + s, L::FUT + t), sb.ut[t]);
      w.put(L::near(s, L::NE), sb.E);
#pragma unroll
      for (int k = 0; k < NS; ++k) w.put(L::near(s, L::NRY + k), sb.rY[k]);
    }
    for (int m = 0; m < 6; ++m) {
      if (m == 2 || m == 3) continue;
#pragma unroll
      for (int j = 0; j < L::NF; ++j) w.put(L::far(m, j), 0.0);
    }
    mput(M::FLAG, 0.0);
    return;
  }
  const double* __restrict__ QT = Q + p.qT * n;
  const double* __restrict__ QP = Q + p.qP * n;
  const double* __restrict__ QUn = Q + (p.qU + DIR) * n;
  // ---- forward recompute: face average, eigenvector coefficients (the
  // average is formed again from fresh loads where its pull-back needs it)
  auto face_average = [&](double* ub) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double a = ldrow(Uk + v * n, li[2]), b = ldrow(Uk + v * n, li[3]);
      if (v == NS + DIR) {
        if (fl2) a = -a;
        if (fl3) b = -b;
      }
      ub[v] = 0.5 * (a + b);
    }
  };
  double cT, z, af;
  {
    double ub[NV];
    face_average(ub);
    Thermo<NS, DIM> tf;
    equilibrium<NS, DIM>(p, ub, tf, true);
    cT = tf.cT;
    z = tf.z;
    af = tf.a;
  }
  // ---- forward recompute: reconstruction
  double w1L, w1R, w5L, w5R, w6L, w6R, YL[NS], YR[NS], utL[NTa], utR[NTa];
  {
    double wv[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) wv[m] = ldrow(QT, li[m]) - cT * ldrow(QP, li[m]);
    double2 o = weno5z_lr(wv[0], wv[1], wv[2], wv[3], wv[4], wv[5], p.weps, p.wp);
    w1L = o.x;
    w1R = o.y;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double* __restrict__ QY = Q + (p.qY + k) * n;
      o = weno5z_lr(ldrow(QY, li[0]), ldrow(QY, li[1]), ldrow(QY, li[2]), ldrow(QY, li[3]), ldrow(QY, li[4]), ldrow(QY, li[5]), p.weps, p.wp);
      YL[k] = o.x;
      YR[k] = o.y;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double* __restrict__ QUt = Q + (p.qU + tdir<DIM, DIR>(t)) * n;
      o = weno5z_lr(ldrow(QUt, li[0]), ldrow(QUt, li[1]), ldrow(QUt, li[2]), ldrow(QUt, li[3]), ldrow(QUt, li[4]), ldrow(QUt, li[5]), p.weps, p.wp);
      utL[t] = o.x;
      utR[t] = o.y;
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double un = (flips >> m) & 1u ? -ldrow(QUn, li[m]) : ldrow(QUn, li[m]);
      wv[m] = 0.5 * z * un + 0.5 * ldrow(QP, li[m]);
    }
    o = weno5z_lr(wv[0], wv[1], wv[2], wv[3], wv[4], wv[5], p.weps, p.wp);
    w5L = o.x;
    w5R = o.y;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double un = (flips >> m) & 1u ? -ldrow(QUn, li[m]) : ldrow(QUn, li[m]);
      wv[m] = -0.5 * z * un + 0.5 * ldrow(QP, li[m]);
    }
    o = weno5z_lr(wv[0], wv[1], wv[2], wv[3], wv[4], wv[5], p.weps, p.wp);
    w6L = o.x;
    w6R = o.y;
  }
  const double PLr = w5L + w6L, PRr = w5R + w6R;
  const double unL = (w5L - w6L) / z, unR = (w5R - w6R) / z;
  const double TLr = w1L + cT * PLr, TRr = w1R + cT * PRr;
  double cYL[NS], cYR[NS], YLl[NS], YRl[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    cYL[k] = ldrow(Q + (p.qY + k) * n, li[2]);
    cYR[k] = ldrow(Q + (p.qY + k) * n, li[3]);
    YLl[k] = YL[k];
    YRl[k] = YR[k];
  }
  if (p.pos) {
    ylimit<NS, double>(YLl, cYL);
    ylimit<NS, double>(YRl, cYR);
  }
  const double TL = (m16 & 1) ? ldrow(QT, li[2]) : TLr, TR = (m16 & 2) ? ldrow(QT, li[3]) : TRr;
  const double PL = (m16 & 4) ? ldrow(QP, li[2]) : PLr, PR = (m16 & 8) ? ldrow(QP, li[3]) : PRr;
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
  // ---- reverse: interpolation limiters (decisions from the mask); the
  // cell values taken by the T/P fallback are direct (near) entries
  double cTb = 0.0, zb = 0.0, w1Lb = 0.0, w1Rb = 0.0;
  w.put(L::far(2, L::FP), (m16 & 4) ? PLb : 0.0);
  w.put(L::far(3, L::FP), (m16 & 8) ? PRb : 0.0);
  if (m16 & 4) PLb = 0.0;
  if (m16 & 8) PRb = 0.0;
  w.put(L::far(2, L::FT), (m16 & 1) ? TLb : 0.0);
  w.put(L::far(3, L::FT), (m16 & 2) ? TRb : 0.0);
  if (!(m16 & 1)) {
    w1Lb = TLb;
    cTb += TLb * PLr;
    PLb += cT * TLb;
  }
  if (!(m16 & 2)) {
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
      w.add(L::far(2, L::FY + k), cYLb[k]);
      w.add(L::far(3, L::FY + k), cYRb[k]);
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
  // ---- hand-over to the second half
  mput(M::W1L, w1Lb);
  mput(M::W1R, w1Rb);
  mput(M::W5L, w5Lb);
  mput(M::W5R, w5Rb);
  mput(M::W6L, w6Lb);
  mput(M::W6R, w6Rb);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    mput(M::YL + k, YLrb[k]);
    mput(M::YR + k, YRrb[k]);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    mput(M::UTL + t, utLb[t]);
    mput(M::UTR + t, utRb[t]);
  }
  mput(M::CTB, cTb);
  mput(M::ZB, zb);
  mput(M::FLAG, 1.0);
}

template <int NS, int DIM, int DIR>
__host__ __device__ void face_vjp_b(const Params& p, const int* c, const double* __restrict__ Uk,
                                    const double* __restrict__ Q, const double* __restrict__ mid,
                                    double* __restrict__ rec) {
  using L = RecL<NS, DIM>;
  using M = MidL<NS, DIM>;
  constexpr int NV = NS + DIM + 1;
  constexpr int NT = DIM - 1;
  constexpr int NTa = NT > 0 ? NT : 1;
  const long n = p.ncell;
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1), e2 = p.n[2] + (DIR == 2);
  const long f = ((long)c[2] * e1 + c[1]) * e0 + c[0];
  const long nfd = (long)e0 * e1 * e2;
  auto G = [&](int slot) { return ldrow(mid + (long)slot * nfd, (int)f); };
  if (G(M::FLAG) == 0.0) return;
  const RecW<NS, DIM> w{rec, f};
  int li[6];
  const unsigned flips = face_stencil<DIR>(p, c, li);
  const bool fl2 = flips & 4u, fl3 = flips & 8u;
  const double* __restrict__ QT = Q + p.qT * n;
  const double* __restrict__ QP = Q + p.qP * n;
  const double* __restrict__ QUn = Q + (p.qU + DIR) * n;
  auto face_average = [&](double* ub) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double a = ldrow(Uk + v * n, li[2]), b = ldrow(Uk + v * n, li[3]);
      if (v == NS + DIR) {
        if (fl2) a = -a;
        if (fl3) b = -b;
      }
      ub[v] = 0.5 * (a + b);
    }
  };
  double cT, z, af;
  {
    double ub[NV];
    face_average(ub);
    Thermo<NS, DIM> tf;
    equilibrium<NS, DIM>(p, ub, tf, true);
    cT = tf.cT;
    z = tf.z;
    af = tf.a;
  }
  double cTb = G(M::CTB), zb = G(M::ZB);
  const double w1Lb = G(M::W1L), w1Rb = G(M::W1R), w5Lb = G(M::W5L), w5Rb = G(M::W5R), w6Lb = G(M::W6L),
               w6Rb = G(M::W6R);
  double YLrb[NS], YRrb[NS], utLb[NTa], utRb[NTa];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    YLrb[k] = G(M::YL + k);
    YRrb[k] = G(M::YR + k);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    utLb[t] = G(M::UTL + t);
    utRb[t] = G(M::UTR + t);
  }
  // ---- reverse: WENO5-Z of each characteristic variable, into the far entries
  double Tb6[6], Pb6[6];
  {
    double wv[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) wv[m] = ldrow(QT, li[m]) - cT * ldrow(QP, li[m]);
    const D6 g = weno5z_lr_vjp(wv[0], wv[1], wv[2], wv[3], wv[4], wv[5], p.weps, p.wp, w1Lb, w1Rb, 0.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      Tb6[m] = g.v[m];
      Pb6[m] = -cT * g.v[m];
      cTb -= g.v[m] * ldrow(QP, li[m]);
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double* __restrict__ QY = Q + (p.qY + k) * n;
    const D6 g = weno5z_lr_vjp(ldrow(QY, li[0]), ldrow(QY, li[1]), ldrow(QY, li[2]), ldrow(QY, li[3]), ldrow(QY, li[4]), ldrow(QY, li[5]), p.weps,
                               p.wp, YLrb[k], YRrb[k], 1.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      if (m == 2 || m == 3)
        w.add(L::far(m, L::FY + k), g.v[m]);
      else
        w.put(L::far(m, L::FY + k), g.v[m]);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double* __restrict__ QUt = Q + (p.qU + tdir<DIM, DIR>(t)) * n;
    const D6 g = weno5z_lr_vjp(ldrow(QUt, li[0]), ldrow(QUt, li[1]), ldrow(QUt, li[2]), ldrow(QUt, li[3]), ldrow(QUt, li[4]), ldrow(QUt, li[5]), p.weps,
                               p.wp, utLb[t], utRb[t], af);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      if (m == 2 || m == 3)
        w.add(L::far(m, L::FUT + t), g.v[m]);
      else
        w.put(L::far(m, L::FUT + t), g.v[m]);
    }
  }
  {
    double un6[6], wv[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      un6[m] = (flips >> m) & 1u ? -ldrow(QUn, li[m]) : ldrow(QUn, li[m]);
      wv[m] = 0.5 * z * un6[m] + 0.5 * ldrow(QP, li[m]);
    }
    const D6 g5 = weno5z_lr_vjp(wv[0], wv[1], wv[2], wv[3], wv[4], wv[5], p.weps, p.wp, w5Lb, w5Rb, 0.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) wv[m] = -0.5 * z * un6[m] + 0.5 * ldrow(QP, li[m]);
    const D6 g6 = weno5z_lr_vjp(wv[0], wv[1], wv[2], wv[3], wv[4], wv[5], p.weps, p.wp, w6Lb, w6Rb, 0.0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double unb = 0.5 * z * (g5.v[m] - g6.v[m]);
      zb += 0.5 * un6[m] * (g5.v[m] - g6.v[m]);
      const double pb = Pb6[m] + 0.5 * (g5.v[m] + g6.v[m]), ub_ = (flips >> m) & 1u ? -unb : unb;
      if (m == 2 || m == 3) {
        w.add(L::far(m, L::FT), Tb6[m]);
        w.add(L::far(m, L::FP), pb);
        w.add(L::far(m, L::FUN), ub_);
      } else {
        w.put(L::far(m, L::FT), Tb6[m]);
        w.put(L::far(m, L::FP), pb);
        w.put(L::far(m, L::FUN), ub_);
      }
    }
  }
  // ---- reverse: face-average equilibrium (the average is half of each
  // face cell's state)
  double gub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) gub[v] = 0.0;
  if (cTb != 0.0 || zb != 0.0) {
    double ub[NV];
    face_average(ub);
    equilibrium_cz_vjp<NS, DIM>(p, ub, cTb, zb, gub);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) w.put(L::SGB + v, 0.5 * gub[v]);
}

// Two waves per SIMD where the first half fits 256 registers without spills
// (NS + DIM <= 4); the larger instances keep one wave and no scratch.
template <int NS, int DIM, int DIR>
__global__ __launch_bounds__(256, (NS + DIM <= 4) ? 2 : 1) void k_face_vjp_a(const Params p, const double* __restrict__ Uk,
                                                    const double* __restrict__ Q,
                                                    const uint16_t* __restrict__ mask,
                                                    const double* __restrict__ dtg, double coef, bool use_dt,
                                                    const double* __restrict__ lam, double* __restrict__ rec,
                                                    double* __restrict__ mid) {
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1), e2 = p.n[2] + (DIR == 2);
  int c[3];
  if (!face_coords<DIR>(e0, e1, e2, c)) return;
  face_vjp_a<NS, DIM, DIR>(p, c, Uk, Q, mask, dtg, coef, use_dt, lam, rec, mid);
}

template <int NS, int DIM, int DIR>
__global__ __launch_bounds__(256) void k_face_vjp_b(const Params p, const double* __restrict__ Uk,
                                                    const double* __restrict__ Q,
                                                    const double* __restrict__ mid, double* __restrict__ rec) {
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1), e2 = p.n[2] + (DIR == 2);
  int c[3];
  if (!face_coords<DIR>(e0, e1, e2, c)) return;
  face_vjp_b<NS, DIM, DIR>(p, c, Uk, Q, mid, rec);
}

// ---------------------------------------------------------------------------
// Gather: the cotangents of one cell's quantities, summed from the records
// of the faces that reference the cell.
// ---------------------------------------------------------------------------

// Faces of the DIR sweep that reference cell x (coordinates), in increasing
// face index: the six faces whose stencil holds x directly and, for a cell
// within three of a boundary, the boundary faces whose mapped ghost cells
// reach it.  qb, ub (conserved-variable cotangents) and stan (signed sum of
// the tangential regularization entries for x) are accumulated.
template <int NS, int DIM, int DIR>
MPMC_HD void gather_dir(const Params& p, const int* x, const double* __restrict__ rec,
                        const uint16_t* __restrict__ mask, CellQb<NS, DIM>& qb, double* ub, double& stan) {
  using L = RecL<NS, DIM>;
  constexpr int NT = DIM - 1;
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1), e2 = p.n[2] + (DIR == 2);
  (void)e2;
  const int nD = p.n[DIR], j = x[DIR];
  auto fidx = [&](int i, int td, int y) {
    int cf[3] = {x[0], x[1], x[2]};
    cf[DIR] = i;
    if (td >= 0) cf[td] = y;
    return ((long)cf[2] * e1 + cf[1]) * e0 + cf[0];
  };
  auto R = [&](long f, int slot) { return rec[L::idx(slot, f)]; };
  // entries of face i whose stencil position m holds x (flip: the map
  // mirrored it)
  auto take = [&](int i, int m, bool flip) {
    const long f = fidx(i, -1, 0);
    {
      const uint16_t m16 = mask[f];
      const bool fb = m16 & 16, cdi = p.cdi && !(m16 & 32);
      qb.T += R(f, L::far(m, L::FT));
      qb.P += R(f, L::far(m, L::FP));
      qb.vel[DIR] += R(f, L::far(m, L::FUN));
#pragma unroll
      for (int k = 0; k < NS; ++k) qb.Y[k] += R(f, L::far(m, L::FY + k));
#pragma unroll
      for (int t = 0; t < NT; ++t) qb.vel[tdir<DIM, DIR>(t)] += R(f, L::far(m, L::FUT + t));
      if (m == 2 || m == 3) {
        const int s = m - 2;
        qb.rho += R(f, L::near(s, L::NRHO));
        if (fb) {
          qb.a += R(f, L::near(s, L::NA));
          ub[NS + DIM] += R(f, L::near(s, L::NE));
#pragma unroll
          for (int k = 0; k < NS; ++k) ub[k] += R(f, L::near(s, L::NRY + k));
        } else {
#pragma unroll
          for (int v = 0; v < NS + DIM + 1; ++v) {
            const double g = R(f, L::SGB + v);
            ub[v] += (v == NS + DIR && flip) ? -g : g;
          }
        }
        if (cdi) {
          qb.phi0 += R(f, L::near(s, L::NPHI0));
          qb.phi1 += R(f, L::near(s, L::NPHI1));
#pragma unroll
          for (int k = 0; k < NS; ++k) qb.yrho[k] += R(f, L::SYRHO + k);
          qb.hrho[0] += R(f, L::SHRHO);
          qb.hrho[1] += R(f, L::SHRHO + 1);
          qb.psi += R(f, L::SPSI);
        }
        if (p.diff) {
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            qb.h[k] += R(f, L::SHH + k);
            qb.K[k] += R(f, L::SK + k);
            qb.chi[k] += s ? R(f, L::SCHI + k) : -R(f, L::SCHI + k);
          }
        }
      }
    }
  };
  auto visit = [&](int i) {
    for (int m = 0; m < 6; ++m) {
      int xm = i - 3 + m;
      bool flip = false;
      if (xm < 0 || xm >= nD) xm = map_index(xm, nD, p.bclo[DIR], p.bchi[DIR], flip);
      if (xm == j) take(i, m, flip);
    }
  };
  const int lo = j - 2 < 0 ? 0 : j - 2, hi = j + 3 > nD ? nD : j + 3;
  if (j > 2 && j < nD - 3) {
    // interior: face i = j + 3 - m holds x at position m, unmapped
    for (int m = 5; m >= 0; --m) take(j + 3 - m, m, false);
  } else {
    // boundary faces 0..2 and nD-2..nD as well (ghost references)
    for (int i = 0; i <= nD;) {
      visit(i);
      int nx = i + 1;
      if (nx > 2 && nx < lo) nx = lo;
      if (nx > hi && nx > 2 && nx < nD - 2) nx = nD - 2;
      i = nx;
    }
  }
  if (!p.cdi) return;
  // tangential psi differences: face cells whose neighbour along td (after
  // the boundary map) is x
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int td = tdir<DIM, DIR>(t);
    const int nt = p.n[td], xt = x[td];
    const int cand[4] = {xt - 1, xt + 1, 0, nt - 1};
    for (int a = 0; a < 4; ++a) {
      const int y = cand[a];
      if (y < 0 || y >= nt) continue;
      bool dup = false;
      for (int b = 0; b < a; ++b) dup = dup || cand[b] == y;
      if (dup) continue;
      for (int sgn = 0; sgn < 2; ++sgn) {
        const int ct = y + (sgn ? 1 : -1);
        bool fl = false;
        const int mt = (ct < 0 || ct >= nt) ? map_index(ct, nt, p.bclo[td], p.bchi[td], fl) : ct;
        if (mt != xt) continue;
        const double sg = sgn ? 1.0 : -1.0;
        auto tk = [&](int i) {
          const long f = fidx(i, td, y);
          if (!(mask[f] & 32)) stan += sg * R(f, L::TAN + t);
        };
        // side 1 (cell map(i)) : i = j, and i = nD where map(nD) = j
        tk(j);
        {
          bool f2 = false;
          if (map_index(nD, nD, p.bclo[DIR], p.bchi[DIR], f2) == j) tk(nD);
        }
        // side 0 (cell map(i - 1)) : i = j + 1, and i = 0 where map(-1) = j
        tk(j + 1);
        {
          bool f2 = false;
          if (map_index(-1, nD, p.bclo[DIR], p.bchi[DIR], f2) == j) tk(0);
        }
      }
    }
  }
}

// Ub = a x + b y + c z (each term optional) before a stage's pull-back adds
// to it.
struct LinComb {
  double a = 0.0, b = 0.0, c = 0.0;
  const double* x = nullptr;
  const double* y = nullptr;
  const double* z = nullptr;
};

// Gather of cell x from the records of every sweep (mask: the stage's face
// masks, directions in order), in registers: q receives its cell-quantity
// cotangents -- exactly the entries cell_vjp reads (T, P, rho, a, Y, u;
// with the regularization phi0, phi1 (the psi terms folded in), psi, Y rho,
// h rho; with diffusion chi, K, h), the rest zero -- and r the conserved
// cotangents lc + the direct terms.
template <int NS, int DIM>
MPMC_HD void gather_cell_q(const Params& p, const int* x, const double* __restrict__ Q,
                           const double* __restrict__ rec0, const double* __restrict__ rec1,
                           const double* __restrict__ rec2, const uint16_t* __restrict__ mask,
                           CellQb<NS, DIM>& q, double* r, const LinComb& lc) {
  constexpr int NV = NS + DIM + 1;
  const long n = p.ncell;
  const long i = lin3(p, x[0], x[1], x[2]);
  CellQb<NS, DIM> qb;
  qb.zero();
  double ubd[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) ubd[v] = 0.0;
  double stan = 0.0;
  const long nf0 = (long)(p.n[0] + 1) * p.n[1] * p.n[2];
  const long nf1 = (long)p.n[0] * (p.n[1] + 1) * p.n[2];
  gather_dir<NS, DIM, 0>(p, x, rec0, mask, qb, ubd, stan);
  if constexpr (DIM > 1) gather_dir<NS, DIM, 1>(p, x, rec1, mask + nf0, qb, ubd, stan);
  if constexpr (DIM > 2) gather_dir<NS, DIM, 2>(p, x, rec2, mask + nf0 + nf1, qb, ubd, stan);
  q.zero();
  q.T = qb.T;
  q.P = qb.P;
  q.rho = qb.rho;
  q.a = qb.a;
#pragma unroll
  for (int k = 0; k < NS; ++k) q.Y[k] = qb.Y[k];
#pragma unroll
  for (int d = 0; d < DIM; ++d) q.vel[d] = qb.vel[d];
  if (p.cdi) {
    const double p0 = ldrow(Q + p.qPhi0 * n, i), p1 = ldrow(Q + p.qPhi1 * n, i);
    q.phi0 = qb.phi0 + stan * dlog_coef(p, p0, p1);
    q.phi1 = qb.phi1 - stan * dlog_coef(p, p1, p0);
    q.psi = qb.psi;
#pragma unroll
    for (int k = 0; k < NS; ++k) q.yrho[k] = qb.yrho[k];
    q.hrho[0] = qb.hrho[0];
    q.hrho[1] = qb.hrho[1];
  }
  if (p.diff) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      q.chi[k] = qb.chi[k];
      q.K[k] = qb.K[k];
      q.h[k] = qb.h[k];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double rv = ubd[v];
    if (lc.x) rv += lc.a * ldrow(lc.x + v * n, i);
    if (lc.y) rv += lc.b * ldrow(lc.y + v * n, i);
    if (lc.z) rv += lc.c * ldrow(lc.z + v * n, i);
    r[v] = rv;
  }
}

// The cell-quantity cotangents q of cell i into Qb ([nq][cells]; the slots
// of switched-off terms are not written).
template <int NS, int DIM>
MPMC_HD void store_qb(const Params& p, long i, const CellQb<NS, DIM>& q, double* __restrict__ Qb) {
  const long n = p.ncell;
  strow(Qb + p.qT * n, i, q.T, p.stream);
  strow(Qb + p.qP * n, i, q.P, p.stream);
  strow(Qb + p.qRho * n, i, q.rho, p.stream);
  strow(Qb + p.qA * n, i, q.a, p.stream);
#pragma unroll
  for (int k = 0; k < NS; ++k) strow(Qb + (p.qY + k) * n, i, q.Y[k], p.stream);
#pragma unroll
  for (int d = 0; d < DIM; ++d) strow(Qb + (p.qU + d) * n, i, q.vel[d], p.stream);
  if (p.cdi) {
    strow(Qb + p.qPhi0 * n, i, q.phi0, p.stream);
    strow(Qb + p.qPhi1 * n, i, q.phi1, p.stream);
    strow(Qb + p.qPsi * n, i, q.psi, p.stream);
#pragma unroll
    for (int k = 0; k < NS; ++k) strow(Qb + (p.qYrho + k) * n, i, q.yrho[k], p.stream);
    strow(Qb + p.qHrho * n, i, q.hrho[0], p.stream);
    strow(Qb + (p.qHrho + 1) * n, i, q.hrho[1], p.stream);
  }
  if (p.diff) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      strow(Qb + (p.qChi + k) * n, i, q.chi[k], p.stream);
      strow(Qb + (p.qK + k) * n, i, q.K[k], p.stream);
      strow(Qb + (p.qH + k) * n, i, q.h[k], p.stream);
    }
  }
}

// Gather of cell x and the pull-back through its cell quantities in one
// pass: Ub = lc + direct terms + (dQ_i/dU_i)^T q, U the stage input (the
// cotangents never go through memory).
template <int NS, int DIM>
MPMC_HD void gather_cell_vjp(const Params& p, const int* x, const double* __restrict__ U,
                             const double* __restrict__ Q, const double* __restrict__ rec0,
                             const double* __restrict__ rec1, const double* __restrict__ rec2,
                             const uint16_t* __restrict__ mask, double* __restrict__ Ub, const LinComb& lc) {
  constexpr int NV = NS + DIM + 1;
  const long n = p.ncell;
  const long i = lin3(p, x[0], x[1], x[2]);
  CellQb<NS, DIM> q;
  double r[NV];
  gather_cell_q<NS, DIM>(p, x, Q, rec0, rec1, rec2, mask, q, r, lc);
  double u[NV], ub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    u[v] = ldrow(U + v * n, i);
    ub[v] = 0.0;
  }
  cell_quantities_vjp<NS, DIM>(p, u, q, p.cdi || p.diff, ub);
#pragma unroll
  for (int v = 0; v < NV; ++v) strow(Ub + v * n, i, r[v] + ub[v], p.stream);
}

template <int NS, int DIM>
__global__ __launch_bounds__(256) void k_gather_vjp(const Params p, const double* __restrict__ U,
                                                    const double* __restrict__ Q, const double* __restrict__ rec0,
                                                    const double* __restrict__ rec1,
                                                    const double* __restrict__ rec2, const uint16_t* __restrict__ mask,
                                                    double* __restrict__ Ub, LinComb lc) {
  const long i0 = (long)blockIdx.x * blockDim.x;
  if (i0 + (long)threadIdx.x >= p.ncell) return;
  int x[3];
  decompose(i0, p.n[0], p.n[1], x[0], x[1], x[2]);
  gather_cell_vjp<NS, DIM>(p, x, U, Q, rec0, rec1, rec2, mask, Ub, lc);
}

}  // namespace mpmc
