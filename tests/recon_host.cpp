// Host harness: the library's face reconstruction (weno_lr, every scheme)
// compiled for the host by hipcc.  Reads lines "scheme eps p w0 .. w5" from
// stdin and prints the left and right face values of each.
#include <cstdio>

#include "../include/mpmc.h"
#include "../paper_2504_14063_amd/csrc/mpmc_device.h"

int main() {
  int scheme, pw;
  double eps, w[6];
  while (std::scanf("%d %lf %d %lf %lf %lf %lf %lf %lf", &scheme, &eps, &pw, &w[0], &w[1], &w[2], &w[3], &w[4],
                    &w[5]) == 9) {
    const double2 o = mpmc::weno_lr(w[0], w[1], w[2], w[3], w[4], w[5], eps, pw, scheme);
    std::printf("%.17g %.17g\n", o.x, o.y);
  }
  return 0;
}
