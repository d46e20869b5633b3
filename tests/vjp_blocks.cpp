// Host harness: the hand-written reverse-mode blocks of the discrete adjoint
// against forward-mode dual numbers pushed through the same templated
// forward code (WENO5-Z, Y-limiter, face EOS, HLLC, the cT and z of the
// equilibrium, the per-cell quantities).  For every block and a random cotangent ob it prints
// max_j |(J^T ob)_j - <ob, J e_j>| / scale.
#include <cmath>
#include <cstdio>
#include <random>

#include "../include/mpmc.h"
#include "../paper_2504_14063_amd/csrc/mpmc_adjoint.h"
#include "../paper_2504_14063_amd/csrc/mpmc_params.h"

using namespace mpmc;

static std::mt19937_64 rng(12345);
static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static Params params3() {
  Params p{};
  p.ns = 3;
  p.dim = 3;
  p.nv = 7;
  const double cv[3] = {718.0, 650.0, 1816.0}, gam[3] = {1.4, 1.3, 6.12}, pinf[3] = {0.0, 0.0, 3.43e8};
  const double b[3] = {0.0, 0.0, 6.2e-4}, q[3] = {0.0, 0.0, -1.177e6};
  for (int k = 0; k < 3; ++k) {
    p.cv[k] = cv[k];
    p.gam[k] = gam[k];
    p.pinf[k] = pinf[k];
    p.b[k] = b[k];
    p.q[k] = q[k];
    p.gm1cv[k] = (gam[k] - 1.0) * cv[k];
    p.gcv[k] = gam[k] * cv[k];
  }
  p.Pst = 3.43e8;
  return p;
}

static double report(const char* name, double err, double scale) {
  const double r = err / (scale > 0 ? scale : 1.0);
  std::printf("%s %.3e\n", name, r);
  return r;
}

// ---- WENO5-Z
static void test_weno(int pw, bool rough) {
  double worst = 0.0;
  for (int trial = 0; trial < 200; ++trial) {
    double f[5];
    for (int j = 0; j < 5; ++j) f[j] = rough ? U(-1.0, 1.0) : 1.0 + 0.1 * j + 0.01 * U(-1, 1) * j * j;
    const double eps = trial % 2 ? 1e-40 : 1e-6;
    Dual<5> fd[5];
    for (int j = 0; j < 5; ++j) fd[j] = Dual<5>::seed(f[j], j);
    const Dual<5> o = weno5z<Dual<5>>(fd[0], fd[1], fd[2], fd[3], fd[4], Dual<5>(eps), pw);
    const double ob = U(-2.0, 2.0);
    double fb[5] = {0, 0, 0, 0, 0};
    weno5z_vjp(f[0], f[1], f[2], f[3], f[4], eps, pw, ob, fb);
    double err = 0.0, sc = 0.0;
    for (int j = 0; j < 5; ++j) {
      err = std::fmax(err, std::fabs(fb[j] - ob * o.d[j]));
      sc = std::fmax(sc, std::fabs(ob * o.d[j]));
    }
    worst = std::fmax(worst, err / sc);
  }
  char name[64];
  std::snprintf(name, sizeof(name), "weno5z_p%d_%s", pw, rough ? "rough" : "smooth");
  report(name, worst, 1.0);
}

// ---- WENO5-Z on stencils flat to round-off: derivative of the ideal weights
static void test_weno_flat() {
  const double lin[5] = {1.0 / 30.0, -13.0 / 60.0, 47.0 / 60.0, 27.0 / 60.0, -1.0 / 20.0};
  double worst = 0.0;
  for (int trial = 0; trial < 100; ++trial) {
    const double c = trial % 3 == 0 ? 0.0 : U(-1e5, 1e5);
    double f[5];
    for (int j = 0; j < 5; ++j) f[j] = c * (1.0 + (trial % 2 ? 1e-9 : 1e-16) * U(-1, 1));
    const double ob = U(-2.0, 2.0);
    double fb[5] = {0, 0, 0, 0, 0};
    weno5z_vjp(f[0], f[1], f[2], f[3], f[4], 1e-40, 1 + trial % 2, ob, fb);
    for (int j = 0; j < 5; ++j) worst = std::fmax(worst, std::fabs(fb[j] - ob * lin[j]) / std::fabs(ob));
  }
  report("weno5z_flat", worst, 1.0);
}

// ---- Y-limiter
static void test_ylimit() {
  constexpr int NS = 3;
  double worst = 0.0;
  int branches[3] = {0, 0, 0};
  for (int trial = 0; trial < 300; ++trial) {
    double Yc[NS], Ys[NS], s = 0.0;
    for (int k = 0; k < NS; ++k) {
      Yc[k] = U(0.05, 1.0);
      s += Yc[k];
    }
    for (int k = 0; k < NS; ++k) {
      Yc[k] /= s;
      Ys[k] = Yc[k] + U(-0.08, 0.08);
    }
    Dual<2 * NS> Ysd[NS], Ycd[NS];
    for (int k = 0; k < NS; ++k) {
      Ysd[k] = Dual<2 * NS>::seed(Ys[k], k);
      Ycd[k] = Dual<2 * NS>::seed(Yc[k], NS + k);
    }
    const int br = ylimit<NS, Dual<2 * NS>>(Ysd, Ycd);
    branches[br]++;
    double ob[NS], Ysb[NS] = {0, 0, 0}, Ycb[NS] = {0, 0, 0};
    for (int k = 0; k < NS; ++k) ob[k] = U(-1, 1);
    ylimit_vjp<NS>(Ys, Yc, ob, Ysb, Ycb);
    double err = 0.0, sc = 1e-300;
    for (int j = 0; j < 2 * NS; ++j) {
      double ref = 0.0;
      for (int k = 0; k < NS; ++k) ref += ob[k] * Ysd[k].d[j];
      const double got = j < NS ? Ysb[j] : Ycb[j - NS];
      err = std::fmax(err, std::fabs(got - ref));
      sc = std::fmax(sc, std::fabs(ref));
    }
    worst = std::fmax(worst, err / sc);
  }
  report("ylimit", worst, 1.0);
  // a round-off-size correction is not differentiated: identity
  double wn = 0.0;
  for (int trial = 0; trial < 50; ++trial) {
    double Yc[NS] = {0.2, 0.3, 0.5}, Ys[NS], ob[NS], Ysb[NS] = {0, 0, 0}, Ycb[NS] = {0, 0, 0};
    for (int k = 0; k < NS; ++k) {
      Ys[k] = Yc[k] * (1.0 + 1e-16 * U(-1, 1));
      ob[k] = U(-1, 1);
    }
    ylimit_vjp<NS>(Ys, Yc, ob, Ysb, Ycb);
    for (int k = 0; k < NS; ++k) wn = std::fmax(wn, std::fabs(Ysb[k] - ob[k]) + std::fabs(Ycb[k]));
  }
  report("ylimit_noise", wn, 1.0);
  std::printf("ylimit_branches %d %d %d\n", branches[0], branches[1], branches[2]);
}

// ---- face EOS: (P, T, Y[3], u_n, u_t[2]) -> side
static void test_face_state() {
  constexpr int NS = 3, DIM = 3, NI = NS + 2 + DIM;
  const Params p = params3();
  double worst = 0.0;
  for (int trial = 0; trial < 200; ++trial) {
    double in[NI];
    in[0] = U(2e4, 5e6);   // P
    in[1] = U(250.0, 900.0);  // T
    double s = 0.0;
    for (int k = 0; k < NS; ++k) {
      in[2 + k] = U(0.0, 1.0);
      s += in[2 + k];
    }
    for (int k = 0; k < NS; ++k) in[2 + k] /= s;
    for (int d = 0; d < DIM; ++d) in[2 + NS + d] = U(-300.0, 300.0);
    Dual<NI> x[NI];
    for (int j = 0; j < NI; ++j) x[j] = Dual<NI>::seed(in[j], j);
    Side<NS, DIM, Dual<NI>> sd;
    face_state<NS, DIM, Dual<NI>>(p, x[0], x[1], x + 2, x[2 + NS], x + 3 + NS, sd);
    Side<NS, DIM, double> sv, sb;
    face_state<NS, DIM, double>(p, in[0], in[1], in + 2, in[2 + NS], in + 3 + NS, sv);
    // random cotangent scaled to each output's magnitude
    sb.rho = U(-1, 1) / sv.rho;
    sb.un = U(-1, 1) / 300.0;
    sb.ut[0] = U(-1, 1) / 300.0;
    sb.ut[1] = U(-1, 1) / 300.0;
    sb.P = U(-1, 1) / sv.P;
    sb.E = U(-1, 1) / sv.E;
    sb.a = U(-1, 1) / sv.a;
    for (int k = 0; k < NS; ++k) sb.rY[k] = U(-1, 1) / sv.rho;
    double gb[NI];
    for (int j = 0; j < NI; ++j) gb[j] = 0.0;
    face_state_vjp<NS, DIM>(p, in[0], in[1], in + 2, in[2 + NS], in + 3 + NS, sb, gb[0], gb[1], gb + 2,
                            gb[2 + NS], gb + 3 + NS);
    double err = 0.0;
    for (int j = 0; j < NI; ++j) {
      double ref = sb.rho * sd.rho.d[j] + sb.un * sd.un.d[j] + sb.P * sd.P.d[j] + sb.E * sd.E.d[j] +
                   sb.a * sd.a.d[j] + sb.ut[0] * sd.ut[0].d[j] + sb.ut[1] * sd.ut[1].d[j];
      double mag = std::fabs(sb.rho * sd.rho.d[j]) + std::fabs(sb.un * sd.un.d[j]) + std::fabs(sb.P * sd.P.d[j]) +
                   std::fabs(sb.E * sd.E.d[j]) + std::fabs(sb.a * sd.a.d[j]) + std::fabs(sb.ut[0] * sd.ut[0].d[j]) +
                   std::fabs(sb.ut[1] * sd.ut[1].d[j]);
      for (int k = 0; k < NS; ++k) {
        ref += sb.rY[k] * sd.rY[k].d[j];
        mag += std::fabs(sb.rY[k] * sd.rY[k].d[j]);
      }
      err = std::fmax(err, std::fabs(gb[j] - ref) / (mag > 0 ? mag : 1.0));
    }
    worst = std::fmax(worst, err);
  }
  report("face_state", worst, 1.0);
}

// ---- HLLC on two independent sides
static void test_hllc() {
  constexpr int NS = 3, DIM = 3, NF = 2 * NS + 2 * 6;  // per side: rho un ut0 ut1 P E a rY[3] = 10
  constexpr int NSD = 10, NIN = 2 * NSD;
  constexpr int NV = NS + DIM + 1;
  (void)NF;
  double worst = 0.0;
  int regimes[4] = {0, 0, 0, 0};
  for (int trial = 0; trial < 400; ++trial) {
    double in[NIN];
    const int regime = trial % 4;  // subsonic +/-, supersonic right-going, left-going
    for (int s = 0; s < 2; ++s) {
      double* v = in + s * NSD;
      v[0] = U(0.5, 1000.0);                                   // rho
      v[6] = U(300.0, 1500.0);                                 // a
      double un = U(-0.5, 0.5) * v[6];
      if (regime == 2) un = v[6] * U(1.2, 2.0);
      if (regime == 3) un = -v[6] * U(1.2, 2.0);
      v[1] = un;
      v[2] = U(-100, 100);
      v[3] = U(-100, 100);
      v[4] = U(1e5, 1e7);                                      // P
      v[5] = v[4] * U(2.0, 5.0) + 0.5 * v[0] * un * un;        // E
      double sum = 0.0;
      for (int k = 0; k < NS; ++k) {
        v[7 + k] = U(0.01, 1.0);
        sum += v[7 + k];
      }
      for (int k = 0; k < NS; ++k) v[7 + k] *= v[0] / sum;
    }
    Dual<NIN> x[NIN];
    for (int j = 0; j < NIN; ++j) x[j] = Dual<NIN>::seed(in[j], j);
    auto mk = [](auto* v, auto& s) {
      s.rho = v[0];
      s.un = v[1];
      s.ut[0] = v[2];
      s.ut[1] = v[3];
      s.P = v[4];
      s.E = v[5];
      s.a = v[6];
      for (int k = 0; k < NS; ++k) s.rY[k] = v[7 + k];
    };
    Side<NS, DIM, Dual<NIN>> Ld, Rd;
    mk(x, Ld);
    mk(x + NSD, Rd);
    Dual<NIN> Fd[NV];
    hllc<NS, DIM, Dual<NIN>>(Ld, Rd, Fd);
    Side<NS, DIM, double> L, R, Lb, Rb;
    mk(in, L);
    mk(in + NSD, R);
    side_zero<NS, DIM>(Lb);
    side_zero<NS, DIM>(Rb);
    double Fb[NV];
    for (int v = 0; v < NV; ++v) Fb[v] = U(-1, 1) / (1.0 + std::fabs(Fd[v].v));
    hllc_vjp<NS, DIM>(L, R, Fb, Lb, Rb);
    double got[NIN];
    auto unpack = [&](const Side<NS, DIM, double>& s, double* g) {
      g[0] = s.rho;
      g[1] = s.un;
      g[2] = s.ut[0];
      g[3] = s.ut[1];
      g[4] = s.P;
      g[5] = s.E;
      g[6] = s.a;
      for (int k = 0; k < NS; ++k) g[7 + k] = s.rY[k];
    };
    unpack(Lb, got);
    unpack(Rb, got + NSD);
    double err = 0.0;
    for (int j = 0; j < NIN; ++j) {
      double ref = 0.0, mag = 0.0;
      for (int v = 0; v < NV; ++v) {
        ref += Fb[v] * Fd[v].d[j];
        mag += std::fabs(Fb[v] * Fd[v].d[j]);
      }
      err = std::fmax(err, std::fabs(got[j] - ref) / (mag > 0 ? mag : 1e-300));
    }
    worst = std::fmax(worst, err);
    regimes[regime]++;
  }
  report("hllc", worst, 1.0);
}

// ---- eigenvector coefficients cT, z of the equilibrium of a conserved state
static void test_equilibrium_cz() {
  constexpr int NS = 3, DIM = 3, NV = NS + DIM + 1;
  const Params p = params3();
  double worst = 0.0;
  int branch[3] = {0, 0, 0};  // linear root, quadratic a2 >= 0, quadratic a2 < 0
  for (int trial = 0; trial < 300; ++trial) {
    const int kind = trial % 3;  // mixture, pure gas, pure liquid
    double Y[NS];
    if (kind == 0) {
      double sum = 0.0;
      for (int k = 0; k < NS; ++k) sum += (Y[k] = U(0.01, 1.0));
      for (int k = 0; k < NS; ++k) Y[k] /= sum;
    } else if (kind == 1) {
      Y[0] = U(0.1, 0.9);
      Y[1] = 1.0 - Y[0];
      Y[2] = 0.0;
    } else {
      Y[0] = Y[1] = 0.0;
      Y[2] = 1.0;
    }
    // a gas above ~Pst (every other pure-gas trial) takes the a2 >= 0 root
    const double P = (kind == 1 && trial % 2) ? U(5e8, 3e9) : U(2e4, 5e7), T = U(250.0, 900.0);
    const double vel[DIM] = {U(-300, 300), U(-300, 300), U(-300, 300)};
    Side<NS, DIM, double> sd;
    face_state<NS, DIM, double>(p, P, T, Y, vel[0], vel + 1, sd);
    double u[NV];
    for (int k = 0; k < NS; ++k) u[k] = sd.rY[k];
    for (int d = 0; d < DIM; ++d) u[NS + d] = sd.rho * vel[d];
    u[NS + DIM] = sd.E;
    Dual<NV> ud[NV];
    for (int j = 0; j < NV; ++j) ud[j] = Dual<NV>::seed(u[j], j);
    ThermoT<NS, DIM, Dual<NV>> td;
    equilibrium_t<NS, DIM, Dual<NV>>(p, ud, td, true);
    const double cTb = U(-1, 1) / std::fabs(td.cT.v), zb = U(-1, 1) / td.z.v;
    double gb[NV] = {0, 0, 0, 0, 0, 0, 0};
    equilibrium_cz_vjp<NS, DIM>(p, u, cTb, zb, gb);
    double err = 0.0;
    for (int j = 0; j < NV; ++j) {
      if (j < NS && u[j] == 0.0) continue;  // absent component: the state sits on its bound
      const double ref = cTb * td.cT.d[j] + zb * td.z.d[j];
      const double mag = std::fabs(cTb * td.cT.d[j]) + std::fabs(zb * td.z.d[j]);
      err = std::fmax(err, std::fabs(gb[j] - ref) / (mag > 0 ? mag : 1e-300));
    }
    worst = std::fmax(worst, err);
    // which root formula the state took
    double R1 = 0.0, Rg = 0.0;
    for (int k = 0; k < NS; ++k) (p.pinf[k] != 0.0 ? R1 : Rg) += Y[k] * p.gm1cv[k];
    if (Rg == 0.0) {
      branch[0]++;
    } else {
      double rho = 0.0, qm = 0.0, bm = 0.0, Cv = 0.0;
      for (int k = 0; k < NS; ++k) rho += u[k];
      double ke = 0.0;
      for (int d = 0; d < DIM; ++d) ke += 0.5 * u[NS + d] * u[NS + d] / rho;
      const double e = (u[NS + DIM] - ke) / rho;
      for (int k = 0; k < NS; ++k) {
        qm += Y[k] * p.q[k];
        bm += Y[k] * p.b[k];
        Cv += Y[k] * p.cv[k];
      }
      const double Ep = (e - qm) / (1.0 / rho - bm);
      const double a2 = Ep * (R1 + Rg) - p.Pst * (Cv + R1);
      branch[a2 >= 0.0 ? 1 : 2]++;
    }
  }
  report("equilibrium_cz", worst, 1.0);
  std::printf("equilibrium_cz_branches %d %d %d\n", branch[0], branch[1], branch[2]);
}

// ---- per-cell quantities (equilibrium and phase auxiliaries, with CDI and
// diffusion, a two-species gas phase and a liquid)
static void test_cell_quantities() {
  constexpr int NS = 3, DIM = 3, NV = NS + DIM + 1;
  mpmc_grid g{};
  g.dim = 3;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = 8;
    g.dx[d] = 1e-3;
  }
  mpmc_eos e{};
  e.n_species = 3;
  const int ph[3] = {1, 1, 0};
  const double cv[3] = {718.0, 3116.0, 1816.0}, gam[3] = {1.4, 1.667, 6.12}, pinf[3] = {0.0, 0.0, 3.43e8};
  const double W[3] = {0.029, 0.004, 0.018}, mu[3] = {1.81e-5, 1.96e-5, 8.9e-4}, Sc[3] = {1.0, 0.7, 1.0};
  for (int k = 0; k < 3; ++k) {
    e.phase[k] = ph[k];
    e.cv[k] = cv[k];
    e.gamma[k] = gam[k];
    e.pinf[k] = pinf[k];
    e.molar_mass[k] = W[k];
    e.mu[k] = mu[k];
    e.Sc[k] = Sc[k];
  }
  mpmc_opts o{};
  o.cfl = 0.5;
  o.cdi = 1;
  o.eps_cdi = 1.5e-3;
  o.phi_min = 1e-8;
  o.delta = 1e-100;
  o.gamma_scale = 1.0;
  o.diffusion = 1;
  o.positivity = 1;
  o.weno_eps = 1e-40;
  o.weno_p = 1;
  Params p;
  if (build_params(&g, &e, &o, p) != MPMC_OK) {
    std::printf("cell_quantities 1.0e+00\n");
    return;
  }
  double worst = 0.0;
  int kinds[3] = {0, 0, 0};
  for (int trial = 0; trial < 300; ++trial) {
    const int kind = trial % 3;  // mixed cell, pure gas (liquid absent), liquid-rich
    double phil = kind == 0 ? U(0.05, 0.95) : (kind == 1 ? 0.0 : U(0.999, 1.0 - 1e-9));
    const double P = U(5e4, 5e6), T = U(280.0, 600.0), yA = U(0.2, 0.8);
    // phase densities at (P, T) from the component volumes
    double vk[3];
    for (int k = 0; k < 3; ++k) vk[k] = p.gm1cv[k] / (P + p.pinf[k]) * T + p.b[k];
    const double rho_g = 1.0 / (yA * vk[0] + (1.0 - yA) * vk[1]), rho_l = 1.0 / vk[2];
    double u[NV];
    u[0] = (1.0 - phil) * rho_g * yA;
    u[1] = (1.0 - phil) * rho_g * (1.0 - yA);
    u[2] = phil * rho_l;
    const double rho = u[0] + u[1] + u[2];
    double ke = 0.0;
    for (int d = 0; d < DIM; ++d) {
      const double vel = U(-200, 200);
      u[NS + d] = rho * vel;
      ke += 0.5 * rho * vel * vel;
    }
    // energy consistent with (P, T): rho e = sum rhoY_k e_k(P, T)
    double re = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double ek = p.cv[k] * T * (P + p.gam[k] * p.pinf[k]) / (P + p.pinf[k]) + p.q[k];
      re += u[k] * ek;
    }
    u[NS + DIM] = re + ke;
    // forward duals
    Dual<NV> ud[NV];
    for (int j = 0; j < NV; ++j) ud[j] = Dual<NV>::seed(u[j], j);
    CellQ<NS, DIM, Dual<NV>> qd;
    cell_quantities_t<NS, DIM, Dual<NV>>(p, ud, qd, true);
    // random cotangent, each scaled to its quantity
    CellQb<NS, DIM> qb;
    qb.zero();
    auto r = [&](double scale) { return U(-1, 1) / (std::fabs(scale) + 1e-30); };
    qb.T = r(qd.T.v);
    qb.P = r(qd.P.v);
    qb.rho = r(qd.rho.v);
    qb.a = r(qd.a.v);
    qb.phi0 = r(1.0);
    qb.phi1 = r(1.0);
    qb.psi = r(p.eps * 10.0);
    qb.hrho[0] = r(qd.hrho[0].v);
    qb.hrho[1] = r(qd.hrho[1].v);
    for (int k = 0; k < NS; ++k) {
      qb.Y[k] = r(1.0);
      qb.yrho[k] = r(qd.yrho[k].v);
      qb.chi[k] = r(1.0);
      qb.K[k] = r(qd.K[k].v);
      qb.h[k] = r(qd.h[k].v);
    }
    for (int d = 0; d < DIM; ++d) qb.vel[d] = r(200.0);
    double got[NV] = {0, 0, 0, 0, 0, 0, 0};
    cell_quantities_vjp<NS, DIM>(p, u, qb, true, got);
    double err = 0.0;
    for (int j = 0; j < NV; ++j) {
      if (j < NS && u[j] == 0.0) continue;  // absent component: on its bound
      double ref = 0.0, mag = 0.0;
      auto acc = [&](double c, const Dual<NV>& q) {
        ref += c * q.d[j];
        mag += std::fabs(c * q.d[j]);
      };
      acc(qb.T, qd.T);
      acc(qb.P, qd.P);
      acc(qb.rho, qd.rho);
      acc(qb.a, qd.a);
      acc(qb.phi0, qd.phi[0]);
      acc(qb.phi1, qd.phi[1]);
      acc(qb.psi, qd.psi);
      acc(qb.hrho[0], qd.hrho[0]);
      acc(qb.hrho[1], qd.hrho[1]);
      for (int k = 0; k < NS; ++k) {
        acc(qb.Y[k], qd.Y[k]);
        acc(qb.yrho[k], qd.yrho[k]);
        acc(qb.chi[k], qd.chi[k]);
        acc(qb.K[k], qd.K[k]);
        acc(qb.h[k], qd.h[k]);
      }
      for (int d = 0; d < DIM; ++d) acc(qb.vel[d], qd.vel[d]);
      err = std::fmax(err, std::fabs(got[j] - ref) / (mag > 0 ? mag : 1e-300));
    }
    worst = std::fmax(worst, err);
    kinds[kind]++;
  }
  report("cell_quantities", worst, 1.0);
}

int main() {
  test_weno(1, false);
  test_weno(1, true);
  test_weno(2, false);
  test_weno(2, true);
  test_weno_flat();
  test_ylimit();
  test_face_state();
  test_hllc();
  test_equilibrium_cz();
  test_cell_quantities();
  return 0;
}
