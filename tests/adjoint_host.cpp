// Test harness: the adjoint's per-face and per-cell reverse code executed
// sequentially on the host (the same __host__ __device__ functions the GPU
// kernels run), for checking one stage pull-back against the oracle's
// complex-step stage derivative.  Not part of the library.
#include <cmath>
#include <cstdint>
#include <vector>

#include "../include/mpmc.h"
#include "../paper_2504_14063_amd/csrc/mpmc_adjoint.h"
#include "../paper_2504_14063_amd/csrc/mpmc_params.h"

using namespace mpmc;

template <int NS, int DIM>
static void stage(const Params& p, const double* Uk, const uint16_t* mask, const double* dtg, double coef,
                  const double* lam, double* out, double* qb_out) {
  const long n = p.ncell;
  std::vector<double> Q((size_t)p.nq * n);
  for (long i = 0; i < n; ++i) {
    CellQ<NS, DIM, double> q;
    store_cell_quantities<NS, DIM>(p, i, Uk, Q.data(), q, p.cdi || p.diff);
  }
  // face records, NaN-filled: an entry a face does not write (or adds to
  // before writing) poisons the result
  std::vector<double> rec[3];
  long off = 0;
  auto sweep = [&](auto dirc) {
    constexpr int DIR = decltype(dirc)::value;
    const int e[3] = {p.n[0] + (DIR == 0), p.n[1] + (DIR == 1), p.n[2] + (DIR == 2)};
    const long nfd = (long)e[0] * e[1] * e[2];
    rec[DIR].assign((size_t)rec_doubles(NS, DIM, nfd), std::nan(""));
    std::vector<double> mid((size_t)mid_slots(NS, DIM) * nfd, std::nan(""));
    for (int c2 = 0; c2 < e[2]; ++c2)
      for (int c1 = 0; c1 < e[1]; ++c1)
        for (int c0 = 0; c0 < e[0]; ++c0) {
          const int c[3] = {c0, c1, c2};
          face_vjp_a<NS, DIM, DIR>(p, c, Uk, Q.data(), mask + off, dtg, coef, true, lam, rec[DIR].data(),
                                   mid.data());
        }
    for (int c2 = 0; c2 < e[2]; ++c2)
      for (int c1 = 0; c1 < e[1]; ++c1)
        for (int c0 = 0; c0 < e[0]; ++c0) {
          const int c[3] = {c0, c1, c2};
          face_vjp_b<NS, DIM, DIR>(p, c, Uk, Q.data(), mid.data(), rec[DIR].data());
        }
    off += nfd;
  };
  sweep(std::integral_constant<int, 0>());
  if constexpr (DIM > 1) sweep(std::integral_constant<int, 1>());
  if constexpr (DIM > 2) sweep(std::integral_constant<int, 2>());
  // the cell-quantity cotangents first (for qb_out), then the one-pass
  // gather and pull-back the device runs: out = out + direct terms + the
  // cell pull-back
  std::vector<double> Qb((size_t)p.nq * n, std::nan(""));
  for (int x2 = 0; x2 < p.n[2]; ++x2)
    for (int x1 = 0; x1 < p.n[1]; ++x1)
      for (int x0 = 0; x0 < p.n[0]; ++x0) {
        const int x[3] = {x0, x1, x2};
        CellQb<NS, DIM> q;
        double r[NS + DIM + 1];
        gather_cell_q<NS, DIM>(p, x, Q.data(), rec[0].data(), rec[1].data(), rec[2].data(), mask, q, r,
                               LinComb());
        store_qb<NS, DIM>(p, lin3(p, x0, x1, x2), q, Qb.data());
      }
  for (int x2 = 0; x2 < p.n[2]; ++x2)
    for (int x1 = 0; x1 < p.n[1]; ++x1)
      for (int x0 = 0; x0 < p.n[0]; ++x0) {
        const int x[3] = {x0, x1, x2};
        LinComb lc;
        lc.a = 1.0;
        lc.x = out;
        gather_cell_vjp<NS, DIM>(p, x, Uk, Q.data(), rec[0].data(), rec[1].data(), rec[2].data(), mask, out, lc);
      }
  if (qb_out)
    for (size_t i = 0; i < Qb.size(); ++i) qb_out[i] = Qb[i];
}

// out += (dL(U_k)/dU_k)^T (coef dt lam), decisions from mask (one uint16
// per face, directions in order); qb_out (nullable, [nq][cells]) receives the
// cell-quantity cotangents.
extern "C" int emu_stage_vjp(const mpmc_grid* g, const mpmc_eos* e, const mpmc_opts* o, const double* Uk,
                             const uint16_t* mask, double dt, double gamma, double coef, const double* lam,
                             double* out, double* qb_out) {
  Params p;
  const int st = build_params(g, e, o, p);
  if (st != MPMC_OK) return st;
  const double dtg[2] = {dt, gamma};
  const int k = p.ns * 10 + p.dim;
  switch (k) {
    case 11: stage<1, 1>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 12: stage<1, 2>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 13: stage<1, 3>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 21: stage<2, 1>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 22: stage<2, 2>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 23: stage<2, 3>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 31: stage<3, 1>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 32: stage<3, 2>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    case 33: stage<3, 3>(p, Uk, mask, dtg, coef, lam, out, qb_out); break;
    default: return MPMC_EUNSUPPORTED;
  }
  return MPMC_OK;
}
