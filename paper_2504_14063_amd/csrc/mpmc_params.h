// mpmc_params.h -- kernel parameter block from the C ABI descriptions
// (grid, component table, options): validation, derived EOS constants, the
// Wilke table and the layout of the cell-quantity array.  Host code.
#pragma once
#include <cmath>
#include <cstring>

#include "../../include/mpmc.h"
#include "mpmc_device.h"

namespace mpmc {

// Fills p from the descriptions; returns MPMC_OK or the ABI error code.
inline int build_params(const mpmc_grid* g, const mpmc_eos* e, const mpmc_opts* o, Params& p) {
  if (!g || !e || !o) return MPMC_EINVAL;
  if (g->dim < 1 || g->dim > 3) return MPMC_EINVAL;
  if (e->n_species < 1 || e->n_species > 8) return MPMC_EINVAL;
  if (e->n_species > MAXS) return MPMC_EUNSUPPORTED;
  if (o->weno < 0) return MPMC_EINVAL;
  if (o->weno > 3) return MPMC_EUNSUPPORTED;
  if (o->precision != 0 && o->precision != 1) return MPMC_EINVAL;
  if (o->step_layout < 0 || o->step_layout > 2) return MPMC_EINVAL;
  // above kFullNS components only the FP64 forward is built
  if (e->n_species > kFullNS && (o->precision != 0 || o->step_layout == 2)) return MPMC_EUNSUPPORTED;
  if (o->basis < 0) return MPMC_EINVAL;
  if (o->basis > 1) return MPMC_EUNSUPPORTED;
  // the scheme variants and the five-equation basis are built for the FP64
  // form only
  if ((o->weno != 0 || o->basis != 0) && o->precision != 0) return MPMC_EUNSUPPORTED;
  if (!(o->cfl > 0.0) || !(o->weno_eps >= 0.0) || (o->weno_p != 1 && o->weno_p != 2)) return MPMC_EINVAL;
  std::memset(&p, 0, sizeof(p));
  p.dim = g->dim;
  p.ns = e->n_species;
  p.nv = p.ns + p.dim + 1;
  long ncell = 1;
  for (int d = 0; d < 3; ++d) {
    p.n[d] = d < p.dim ? g->n[d] : 1;
    if (d >= p.dim && g->n[d] != 1 && g->n[d] != 0) return MPMC_EINVAL;
    if (p.n[d] < 1) return MPMC_EINVAL;
    p.dx[d] = g->dx[d];
    if (d < p.dim && !(p.dx[d] > 0.0)) return MPMC_EINVAL;
    p.idx[d] = d < p.dim ? 1.0 / p.dx[d] : 0.0;
    p.bclo[d] = g->bc_lo[d];
    p.bchi[d] = g->bc_hi[d];
    if (d < p.dim) {
      if (p.bclo[d] < 0 || p.bclo[d] > 3 || p.bchi[d] < 0 || p.bchi[d] > 3) return MPMC_EINVAL;
      if ((p.bclo[d] == 2 || p.bchi[d] == 2) && p.n[d] < 3) return MPMC_EINVAL;
    }
    ncell *= p.n[d];
  }
  if (ncell > kMaxCells) return MPMC_EINVAL;
  for (int d = 0; d < p.dim; ++d)
    if (ncell / p.n[d] * (p.n[d] + 1) > kMaxCells) return MPMC_EINVAL;
  p.ncell = ncell;
  double pst = 0.0;
  int seen[2] = {0, 0};
  for (int k = 0; k < p.ns; ++k) {
    if (e->phase[k] != 0 && e->phase[k] != 1) return MPMC_EINVAL;
    if (!(e->cv[k] > 0.0) || !(e->gamma[k] > 1.0) || !(e->molar_mass[k] > 0.0)) return MPMC_EINVAL;
    p.phase[k] = e->phase[k];
    seen[p.phase[k]] = 1;
    p.cv[k] = e->cv[k];
    p.gam[k] = e->gamma[k];
    p.pinf[k] = e->pinf[k];
    p.b[k] = e->b[k];
    p.q[k] = e->q[k];
    p.W[k] = e->molar_mass[k];
    p.mu[k] = e->mu[k];
    p.Sc[k] = e->Sc[k];
    p.lamc[k] = e->lambda[k];
    p.gm1cv[k] = (e->gamma[k] - 1.0) * e->cv[k];
    p.gcv[k] = e->gamma[k] * e->cv[k];
    p.stiff[k] = e->pinf[k] != 0.0 ? 1.0 : 0.0;
    if (e->pinf[k] != 0.0) {
      if (pst != 0.0 && pst != e->pinf[k]) p.pgen = 1;  // the iterative pressure
      pst = fmax(pst, e->pinf[k]);
    }
  }
  p.Pst = pst;
  // the iterative pressure is built for the FP64 form only
  if (p.pgen && o->precision != 0) return MPMC_EUNSUPPORTED;
  p.np = 0;
  for (int ph = 0; ph < 2; ++ph)
    if (seen[ph]) {
      p.pid[p.np] = ph;
      int cnt = 0;
      for (int k = 0; k < p.ns; ++k)
        if (p.phase[k] == ph) cnt++;
      p.pn[p.np] = cnt;
      p.inpn[p.np] = 1.0 / cnt;
      p.multi[p.np] = cnt >= 2;
      p.np++;
    }
  for (int k = 0; k < p.ns; ++k) p.inP[k] = (p.phase[k] == p.pid[0]) ? 1.0 : 0.0;
  for (int i = 0; i < p.ns; ++i)
    for (int j = 0; j < p.ns; ++j) {
      if (p.phase[i] != p.phase[j]) continue;
      const double r = p.W[i] / p.W[j];
      const double br = 1.0 + std::sqrt(p.mu[i] / p.mu[j]) * std::sqrt(std::sqrt(p.W[j] / p.W[i]));
      const double Phi = br * br / (std::sqrt(8.0) * std::sqrt(1.0 + r));
      p.wilke[i][j] = r * Phi;
    }
  p.cfl = o->cfl;
  p.cdi = (o->cdi && p.np == 2) ? 1 : 0;
  if (o->cdi && !(o->eps_cdi > 0.0)) return MPMC_EINVAL;
  p.eps = o->eps_cdi;
  p.phimin = o->phi_min;
  p.delta = o->delta;
  p.gscale = o->gamma_scale;
  p.sharp_floor = 4.0 * o->phi_min * (1.0 - o->phi_min);
  p.diff = o->diffusion ? 1 : 0;
  p.visc = o->viscous ? 1 : 0;
  if (p.visc && !(o->prandtl > 0.0)) return MPMC_EINVAL;
  p.iPr = p.visc ? 1.0 / o->prandtl : 0.0;
  p.pos = o->positivity ? 1 : 0;
  p.weps = o->weno_eps;
  p.wp = o->weno_p;
  p.scheme = o->weno;
  p.basis = o->basis;
  // cell-quantity layout
  int q = 0;
  p.qT = q++;
  p.qP = q++;
  p.qY = q;
  q += p.ns;
  p.qU = q;
  q += p.dim;
  p.qRho = q++;
  p.qA = q++;
  if (p.cdi) {
    p.qPhi0 = q++;
    p.qPhi1 = q++;
    p.qPsi = q++;
    p.qYrho = q;
    q += p.ns;
    p.qHrho = q;
    q += 2;
  }
  if (p.diff) {
    p.qChi = q;
    q += p.ns;
    p.qK = q;
    q += p.ns;
    p.qH = q;
    q += p.ns;
  }
  if (p.visc) {
    p.qMu = q++;
    p.qLam = q++;
  }
  p.nq = q;
  p.stream = (long)q * ncell * 8 > kStreamBytes ? 1 : 0;

  return MPMC_OK;
}

}  // namespace mpmc
