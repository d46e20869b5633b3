// Host harness: the library's equilibrium with the iterative pressure
// (several distinct P_inf) compiled for the host.  Reads the component table
// "ns cv.. gamma.. pinf.. b.. q.." and then conserved 1D states
// "rhoY_1..rhoY_ns rho u E" from stdin; prints P and T of each state.
#include <cstdio>

#include "../include/mpmc.h"
#include "../paper_2504_14063_amd/csrc/mpmc_device.h"

using namespace mpmc;

int main() {
  Params p{};
  int ns;
  if (std::scanf("%d", &ns) != 1 || ns != 3) return 1;
  p.ns = 3;
  p.dim = 1;
  p.nv = 5;
  p.pgen = 1;
  double* fields[5] = {p.cv, p.gam, p.pinf, p.b, p.q};
  for (auto* f : fields)
    for (int k = 0; k < 3; ++k)
      if (std::scanf("%lf", &f[k]) != 1) return 1;
  for (int k = 0; k < 3; ++k) {
    p.gm1cv[k] = (p.gam[k] - 1.0) * p.cv[k];
    p.gcv[k] = p.gam[k] * p.cv[k];
  }
  double u[5];
  while (std::scanf("%lf %lf %lf %lf %lf", &u[0], &u[1], &u[2], &u[3], &u[4]) == 5) {
    ThermoT<3, 1, double> t;
    equilibrium_t<3, 1, double, true>(p, u, t, false);
    std::printf("%.17g %.17g\n", t.P, t.T);
  }
  return 0;
}
