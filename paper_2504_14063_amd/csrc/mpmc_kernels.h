// mpmc_kernels.h -- kernels of the four-equation MPMC hot path for gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mpmc_device.h"

namespace mpmc {

// compiler barrier: memory operations are not moved across it, and the
// machine scheduler does not interleave instructions across it (bounds the
// registers live at once in the long face pipeline)
#define KBARRIER()                    \
  do {                                \
    asm volatile("" ::: "memory");    \
    __builtin_amdgcn_sched_barrier(0); \
  } while (0)

MPMC_HD long lin3(const Params& p, int c0, int c1, int c2) {
  return ((long)c2 * p.n[1] + c1) * p.n[0] + c0;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map the hardware workgroup id to a logical block so that each XCD
// walks one contiguous range of logical blocks (a bijection on [0, nb)).
__device__ __forceinline__ unsigned xcd_block(unsigned w, unsigned nb) {
  const unsigned q = nb >> 3, r = nb & 7, k = w & 7, j = w >> 3;
  return k * q + (k < r ? k : r) + j;
}

// Cell coordinates of linear index i0 + threadIdx.x in an (e0, e1, e2) box:
// the block start is decomposed once (uniform), lanes carry forward.
__device__ __forceinline__ void decompose(long i0, int e0, int e1, int& c0, int& c1, int& c2) {
  const long r0 = i0 / e0;
  int x = (int)(i0 - r0 * e0) + (int)threadIdx.x;
  int y = (int)(r0 % e1), z = (int)(r0 / e1);
  while (x >= e0) {
    x -= e0;
    if (++y == e1) {
      y = 0;
      ++z;
    }
  }
  c0 = x;
  c1 = y;
  c2 = z;
}

// tangential direction t (0..DIM-2) of a sweep along DIR, increasing order
template <int DIM, int DIR> MPMC_HD constexpr int tdir(int t) {
  return (DIR == 0) ? t + 1 : ((DIR == 1) ? (t == 0 ? 0 : 2) : t);
}

// Wavefront (64 lanes) + block max of a non-negative double, one atomicMax of
// its bit pattern per block (non-negative doubles order like their bits).
// The step reductions (max rate, max |u|) go to kRateSlots slots per
// quantity, 256 bytes apart, chosen by block index: one atomic per block
// on a single address serializes every block of the grid at one L2 channel.
// k_dt_finish takes the max over the slots (order-independent: the same
// bits as one slot).
constexpr int kRateSlots = 64, kRateStride = 32;
constexpr int kRateWords = 2 * kRateSlots * kRateStride;  // u64 words of the rates buffer

__device__ __forceinline__ void block_max_atomic(double v, unsigned long long* dst) {
  __shared__ double sm[16];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sm[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sm[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, sm[i]);
    atomicMax(dst + (blockIdx.x & (kRateSlots - 1)) * kRateStride, (unsigned long long)__double_as_longlong(m));
  }
  __syncthreads();
}

// Limiter and failure counters: kCntN per slot, kCntSlots slots 128 bytes
// apart, the slot chosen by block index (one address per counter would
// serialize every block's atomics at one L2 channel); mpmc_stats adds the
// slots.  Indices below.
constexpr int kCntSlots = 64, kCntStride = 16, kCntN = 8;
constexpr int kCntWords = kCntSlots * kCntStride;
enum { kCntT = 0, kCntP = 1, kCntFallback = 2, kCntDrop = 3, kCntUnrec = 4, kCntFaces = 5, kCntBadCells = 6 };

__device__ __forceinline__ unsigned long long* cnt_slot(unsigned long long* cnt) {
  return cnt + (blockIdx.x & (kCntSlots - 1)) * kCntStride;
}

// Failure flag: a word of host-visible memory set by a plain vector store
// (any block may set it; the value is always 1) and read by the host at the
// next entry point without synchronizing.
__device__ __forceinline__ void raise_flag(unsigned* flag) {
  if (flag) *(volatile unsigned*)flag = 1u;
}

__global__ void k_zero_rates(unsigned long long* r) {
  if (threadIdx.x < kRateSlots) {
    r[threadIdx.x * kRateStride] = 0ull;
    r[(kRateSlots + threadIdx.x) * kRateStride] = 0ull;
  }
}

// dt = cfl / max rate, Gamma = gscale * max |u| (or the frozen inputs).
__global__ void k_dt_finish(double cfl, double gscale, const unsigned long long* rates, double* dtg,
                            const double* dt_in, const double* g_in, double* dt_out, double* g_out) {
  double dt = 0.0, g = 0.0;
  if (rates) {
    unsigned long long r0 = 0ull, r1 = 0ull;
    for (int k = 0; k < kRateSlots; ++k) {
      r0 = max(r0, rates[k * kRateStride]);
      r1 = max(r1, rates[(kRateSlots + k) * kRateStride]);
    }
    dt = cfl / __longlong_as_double((long long)r0);
    g = gscale * __longlong_as_double((long long)r1);
  }
  if (dt_in) dt = *dt_in;
  if (g_in) g = *g_in;
  dtg[0] = dt;
  dtg[1] = g;
  if (dt_out) *dt_out = dt;
  if (g_out) *g_out = g;
}

__global__ void k_set_dtg(double* dtg, const double* dt, const double* g) {
  dtg[0] = *dt;
  dtg[1] = *g;
}

// Face coordinates c of this thread for a sweep along DIR over an
// (e0, e1, e2) face box; returns false for padding threads.
template <int DIR>
__device__ __forceinline__ bool face_coords(int e0, int e1, int e2, int* c) {
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
  if constexpr (DIR == 0) {
    // x sweep: faces enumerated linearly (x fastest, rows packed)
    decompose((long)lb * blockDim.x, e0, e1, c[0], c[1], c[2]);
    return c[2] < e2;
  } else {
    // y / z sweeps: blocks of blockDim.x consecutive x, ordered x chunk
    // first, then the sweep coordinate: the contiguous range of blocks an
    // XCD walks covers successive rows along the sweep, which share five of
    // their six stencil rows in its L2 (the sweep coordinate first measures
    // the same)
    const int nbx = (e0 + (int)blockDim.x - 1) / (int)blockDim.x;
    const int eD = DIR == 1 ? e1 : e2, eO = DIR == 1 ? e2 : e1;
    const unsigned bx = lb % nbx, rest = lb / nbx;
    c[0] = bx * blockDim.x + threadIdx.x;
    c[DIR] = (int)(rest % eD);
    c[DIR == 1 ? 2 : 1] = (int)(rest / eD);
    return c[0] < e0 && (int)(rest / eD) < eO;
  }
}

// Stencil cells i-2..i+3 along DIR of the face at c (the face lies between
// m = 2 and m = 3): linear cell indices li[6] after the boundary index maps;
// bit m of the result is set where the map mirrors (normal momentum flips).
template <int DIR>
MPMC_HD unsigned face_stencil(const Params& p, const int* c, int* li) {
  unsigned flips = 0;
  const int nD = p.n[DIR];
  const int strideD = DIR == 0 ? 1 : (DIR == 1 ? p.n[0] : p.n[0] * p.n[1]);
  int ccb[3] = {c[0], c[1], c[2]};
  ccb[DIR] = 0;
  const int base = (int)lin3(p, ccb[0], ccb[1], ccb[2]);
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    int xm = c[DIR] - 3 + m;
    if (xm < 0 || xm >= nD) {
      bool flip = false;
      xm = map_index(xm, nD, p.bclo[DIR], p.bchi[DIR], flip);
      if (flip) flips |= 1u << m;
    }
    li[m] = base + xm * strideD;
  }
  return flips;
}

// The stores of cell i's quantities into the SoA array Q, with or without
// the non-temporal hint.
template <bool NT, int NS, int DIM>
MPMC_HD void put_cell_quantities(const Params& p, long i, double* __restrict__ Q, const CellQ<NS, DIM, double>& q) {
  const long n = p.ncell;
  strow_t<NT>(Q + p.qT * n, i, q.T);
  strow_t<NT>(Q + p.qP * n, i, q.P);
#pragma unroll
  for (int k = 0; k < NS; ++k) strow_t<NT>(Q + (p.qY + k) * n, i, q.Y[k]);
#pragma unroll
  for (int d = 0; d < DIM; ++d) strow_t<NT>(Q + (p.qU + d) * n, i, q.vel[d]);
  strow_t<NT>(Q + p.qRho * n, i, q.rho);
  strow_t<NT>(Q + p.qA * n, i, q.a);
  if (p.cdi) {
    strow_t<NT>(Q + p.qPhi0 * n, i, q.phi[0]);
    strow_t<NT>(Q + p.qPhi1 * n, i, q.phi[1]);
    strow_t<NT>(Q + p.qPsi * n, i, q.psi);
#pragma unroll
    for (int k = 0; k < NS; ++k) strow_t<NT>(Q + (p.qYrho + k) * n, i, q.yrho[k]);
    strow_t<NT>(Q + (p.qHrho + 0) * n, i, q.hrho[0]);
    strow_t<NT>(Q + (p.qHrho + 1) * n, i, q.hrho[1]);
  }
  if (p.diff) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      strow_t<NT>(Q + (p.qChi + k) * n, i, q.chi[k]);
      strow_t<NT>(Q + (p.qK + k) * n, i, q.K[k]);
      strow_t<NT>(Q + (p.qH + k) * n, i, q.h[k]);
    }
  }
  if (p.visc) {
    strow_t<NT>(Q + p.qMu * n, i, q.mu);
    strow_t<NT>(Q + p.qLam * n, i, q.lam);
  }
}

// Cell quantities of cell i of U (equilibrium and, with aux, the phase and
// diffusion auxiliaries) stored into the SoA array Q; q receives them.
// Returns, with check, the admissibility of the cell's state (Eqs.
// PositivityReqs1-2; NaN fails), else true.  The loads and stores branch
// once on the cache hint.
template <int NS, int DIM, bool GEN = false>
MPMC_HD bool store_cell_quantities(const Params& p, long i, const double* __restrict__ U,
                                   double* __restrict__ Q, CellQ<NS, DIM, double>& q, bool aux,
                                   bool check = false) {
  constexpr int NV = NS + DIM + 1;
  const long n = p.ncell;
  double u[NV];
  if (p.stream) {
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = ldrow_t<true>(U + v * n, i);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = ldrow_t<false>(U + v * n, i);
  }
  const bool ok = check ? admissible<NS, DIM>(p, u) : true;
  cell_quantities_t<NS, DIM, double, GEN>(p, u, q, aux);
  if (p.stream)
    put_cell_quantities<true>(p, i, Q, q);
  else
    put_cell_quantities<false>(p, i, Q, q);
  return ok;
}

// ---------------------------------------------------------------------------
// k_cell: per-cell equilibrium and auxiliaries -> Q (GEN: the iterative
// pressure of several distinct P_inf)
// ---------------------------------------------------------------------------
// cnt (nullable): count the cells whose state is not admissible (failure
// detection) and raise flag if there are any.
template <int NS, int DIM, bool GEN = false>
__global__ __launch_bounds__(256) void k_cell(const Params p, const double* __restrict__ U,
                                              double* __restrict__ Q,
                                              unsigned long long* __restrict__ rates,
                                              unsigned long long* __restrict__ cnt, unsigned* flag) {
  const long n = p.ncell;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double rate = 0.0, umax = 0.0;
  bool ok = true;
  if (i < n) {
    CellQ<NS, DIM, double> q;
    ok = store_cell_quantities<NS, DIM, GEN>(p, i, U, Q, q, p.cdi || p.diff || p.visc || rates, cnt != nullptr);
    if (rates) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double au = fabs(q.vel[d]);
        rate = fmax(rate, (au + q.a) / p.dx[d]);
        if (p.diff || p.visc) rate = fmax(rate, 4.0 * q.mu / (q.rho * p.dx[d] * p.dx[d]));
        umax = fmax(umax, au);
      }
    }
  }
  if (rates) {
    block_max_atomic(rate, rates);
    block_max_atomic(umax, rates + kRateSlots * kRateStride);
  }
  if (cnt) {
    const int nbad = __syncthreads_count(!ok);
    if (threadIdx.x == 0 && nbad) {
      atomicAdd(cnt_slot(cnt) + kCntBadCells, (unsigned long long)nbad);
      raise_flag(flag);
    }
  }
}

// ---------------------------------------------------------------------------
// k_face: flux through the faces of direction DIR (x fastest)
// ---------------------------------------------------------------------------
template <int NS, int DIM, int DIR>
MPMC_HD void unrotate(const double* Fr, double* F) {
#pragma unroll
  for (int k = 0; k < NS; ++k) F[k] = Fr[k];
  F[NS + DIR] = Fr[NS];
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) F[NS + tdir<DIM, DIR>(t)] = Fr[NS + 1 + t];
  F[NS + DIM] = Fr[NS + DIM];
}

// Cell state of cell l as one side of a face of direction DIR (the
// first-order fallback of the flux limiter), from Q and U^k; flip mirrors the
// normal velocity.
template <int NS, int DIM, int DIR>
MPMC_HD void cell_side_at(const Params& p, const double* __restrict__ Q,
                                             const double* __restrict__ Uk, int l, bool flip,
                                             Side<NS, DIM, double>& cs) {
  const long n = p.ncell;
  cs.rho = ldrow(Q + p.qRho * n, l);
  cs.a = ldrow(Q + p.qA * n, l);
  const double un = ldrow(Q + (p.qU + DIR) * n, l);
  cs.un = flip ? -un : un;
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) cs.ut[t] = ldrow(Q + (p.qU + tdir<DIM, DIR>(t)) * n, l);
  cs.P = ldrow(Q + p.qP * n, l);
  cs.E = ldrow(Uk + (NS + DIM) * n, l);
#pragma unroll
  for (int k = 0; k < NS; ++k) cs.rY[k] = ldrow(Uk + k * n, l);
}

// Fused sweeps (divergence and RK combination in the face kernel): tiles of
// faces that overlap by one face along the sweep, so that every cell's two
// faces of the direction are computed in one workgroup and exchanged through
// LDS.  x sweep: 256 consecutive faces (rows packed) per workgroup, 255 apart.
// y / z sweeps: kFuseTX consecutive x times kFuseTY faces along the sweep,
// kFuseTY - 1 apart; tiles ordered with the sweep coordinate fastest, then x.
constexpr int kFuseTX = 8, kFuseTY = 32;
static_assert(kFuseTX * kFuseTY == 256, "fused tiles are 256 threads");

// Face coordinates c of this thread in a fused sweep along DIR over an
// (e0, e1, e2) face box; *up receives the LDS slot of the face above it along
// the sweep (its cell's high face) or -1 where the thread updates no cell;
// *own is false for the overlap face that the next tile also computes (it
// is counted and its decision stored there).  Returns false for padding.
template <int DIR>
__device__ __forceinline__ bool fused_coords(int e0, int e1, int e2, int t, int* c, int* up, bool* own) {
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
  const long nf = (long)e0 * e1 * e2;
  if constexpr (DIR == 0) {
    const long f0 = (long)lb * 255;
    const long fl = f0 + t;
    const long r = fl / e0;
    c[0] = (int)(fl - r * e0);
    c[1] = (int)(r % e1);
    c[2] = (int)(r / e1);
    const bool valid = fl < nf;
    *own = t < 255 || fl == nf - 1;
    *up = (valid && t < 255 && c[0] < e0 - 1) ? t + 1 : -1;
    return valid;
  } else {
    const int eD = DIR == 1 ? e1 : e2, eO = DIR == 1 ? e2 : e1;
    const int nbj = (eD - 1 + kFuseTY - 2) / (kFuseTY - 1);
    const int nbx = (e0 + kFuseTX - 1) / kFuseTX;
    const int tx = t % kFuseTX, ty = t / kFuseTX;
    const unsigned bj = lb % nbj, rest = lb / nbj;
    const unsigned bx = rest % nbx, o = rest / nbx;
    c[0] = (int)bx * kFuseTX + tx;
    c[DIR] = (int)bj * (kFuseTY - 1) + ty;
    c[DIR == 1 ? 2 : 1] = (int)o;
    const bool valid = c[0] < e0 && c[DIR] < eD && (int)o < eO;
    *own = ty < kFuseTY - 1 || c[DIR] == eD - 1;
    *up = (valid && ty < kFuseTY - 1 && c[DIR] < eD - 1) ? t + kFuseTX : -1;
    return valid;
  }
}

// Characteristic boundary flux (a reading of the Navier-Stokes characteristic
// boundary conditions that Sec. 3.5 cites without formulas).  The face state
// of a boundary face on side `side` (0 low, 1 high) is built in the
// characteristic variables of App. A linearized at the boundary cell l:
// T - cT P, Y_c and u_t (speed u_n), P/2 + (z/2) u_n (speed u_n + a),
// P/2 - (z/2) u_n (speed u_n - a).  Where a wave leaves the domain (speed
// along the outward normal > 0) the variable keeps the cell's value; where
// it enters, the cell's value moves by the factor sigma toward the target's.
// The flux is the convective flux of that state (no regularization,
// diffusion or viscous flux through the face).
template <int NS, int DIM, int DIR, bool GEN>
MPMC_HD void characteristic_flux(const Params& p, const double* __restrict__ Uk, int l, int side,
                                 double* F) {
  constexpr int NV = NS + DIM + 1;
  constexpr int NTa = DIM > 1 ? DIM - 1 : 1;
  const long n = p.ncell;
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = ldrow(Uk + v * n, l);
  Thermo<NS, DIM> tf;
  equilibrium<NS, DIM, GEN>(p, u, tf, true);
  const double sg = side ? 1.0 : -1.0, sig = p.tgSig[DIR][side];
  const double cT = tf.cT, z = tf.z, un = tf.vel[DIR];
  auto relax = [&](double cell, double target, double speed) {
    return sg * speed > 0.0 ? cell : cell + sig * (target - cell);
  };
  const double tP = p.tgP[DIR][side], tT = p.tgT[DIR][side], tun = p.tgV[DIR][side][DIR];
  const double w0 = relax(tf.T - cT * tf.P, tT - cT * tP, un);
  double Y[NS], ut[NTa];
#pragma unroll
  for (int k = 0; k < NS; ++k) Y[k] = relax(tf.Y[k], p.tgY[DIR][side][k], un);
#pragma unroll
  for (int t = 0; t < DIM - 1; ++t) {
    const int td = tdir<DIM, DIR>(t);
    ut[t] = relax(tf.vel[td], p.tgV[DIR][side][td], un);
  }
  const double wp = relax(0.5 * tf.P + 0.5 * z * un, 0.5 * tP + 0.5 * z * tun, un + tf.a);
  const double wm = relax(0.5 * tf.P - 0.5 * z * un, 0.5 * tP - 0.5 * z * tun, un - tf.a);
  const double P = wp + wm;
  const double unb = (wp - wm) / z;
  const double T = w0 + cT * P;
  Side<NS, DIM, double> sd;
  face_state<NS, DIM, double>(p, P, T, Y, unb, ut, sd);
  double Ur[NV], Fr[NV];
  side_UF<NS, DIM, double>(sd, Ur, Fr);
  unrotate<NS, DIM, DIR>(Fr, F);
}

// REPLAY: the limiter decisions (T/P fallback, first-order flux, dropped
// regularization flux) are read from mrep instead of tested -- the
// frozen-decision forward map, for finite-difference checks of the adjoint.
// VAR: the FP64 form with a scheme variant (WENO5-JS, TENO5, TENO6, chosen by
// p.scheme) in place of WENO5-Z, with the five-equation basis (p.basis), or
// with several distinct P_inf (p.pgen, the iterative pressure).
// A separate instantiation: the variants'
// reconstruction call clobbers more registers than WENO5-Z's, which would
// cost the default kernel an occupancy level.
// FUSE: the fused sweep.  Fo is then the stage's accumulator [nv][ncell]
// (the stage output buffer): fmode 0 writes acc = 0 + dF/dx_d (first
// direction), 1 adds dF/dx_d, 2 finishes the last direction -- L = -(acc +
// dF/dx_d) and Fo = rk0 U^n + rk1 U^k + rk2 dt L in place -- and 3 is the
// first direction and the last (1D).  The order of the operations is that of
// k_update, so both paths give the same bits.  Without FUSE, Fo is the face
// flux array of the direction [nv][faces].
// Every instantiation up to kFullNS components is held to 3 waves per SIMD
// (<= 168 VGPRs): left alone, the FP32 x sweep and the fused x sweep take
// 172-173 and drop to 2 (the FP32 x sweep then runs 25 % slower); a few
// bytes of spill cost less.  More components take the registers they need.
template <int NS, int DIM, int DIR, class R, bool REPLAY = false, bool VAR = false, bool FUSE = false>
__global__ __launch_bounds__(256, NS <= kFullNS ? 3 : 1) void k_face(const Params p, const double* __restrict__ Uk,
                                              const double* __restrict__ Un,
                                              const double* __restrict__ Q, double* __restrict__ Fo,
                                              uint16_t* __restrict__ mask,
                                              const double* __restrict__ dtg, double rk0, double rk1,
                                              double rk2, unsigned long long* __restrict__ cnt,
                                              const uint16_t* __restrict__ mrep, unsigned* flag, int fmode) {
  constexpr int NV = NS + DIM + 1;
  constexpr int NT = DIM - 1;
  constexpr int NTa = NT > 0 ? NT : 1;
  constexpr bool MIXED = std::is_same<R, float>::value;
  const long n = p.ncell;
  const int e0 = p.n[0] + (DIR == 0), e1 = p.n[1] + (DIR == 1), e2 = p.n[2] + (DIR == 2);
  const long nf = (long)e0 * e1 * e2;
  int c[3];
  bool valid;
  if constexpr (FUSE) {
    int up0;
    bool own0;
    valid = fused_coords<DIR>(e0, e1, e2, (int)threadIdx.x, c, &up0, &own0);
  } else {
    valid = face_coords<DIR>(e0, e1, e2, c);
  }
  const long f = ((long)c[2] * e1 + c[1]) * e0 + c[0];
  uint16_t m16 = 0;
  double Fsum[NV];
  // a face on a characteristic boundary (type 3) takes the characteristic flux
  const int bside = (p.bclo[DIR] == 3 && c[DIR] == 0) ? 0 : ((p.bchi[DIR] == 3 && c[DIR] == p.n[DIR]) ? 1 : -1);
  if (valid && bside >= 0) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[DIR] = bside ? p.n[DIR] - 1 : 0;
    characteristic_flux<NS, DIM, DIR, VAR>(p, Uk, (int)lin3(p, cc[0], cc[1], cc[2]), bside, Fsum);
  } else if (valid) {
    // ---- stencil cells i-2..i+3 along DIR (face between m = 2 and m = 3)
    int li[6];
    const unsigned flips = face_stencil<DIR>(p, c, li);
    const bool fl2 = flips & 4u, fl3 = flips & 8u;
    const double* __restrict__ QT = Q + p.qT * n;
    const double* __restrict__ QP = Q + p.qP * n;
    const double* __restrict__ QUn = Q + (p.qU + DIR) * n;
    // ---- Godunov step 1: face average of the two face cells' conserved
    // states, its equilibrium, eigenvector coefficients
    double cT, z;
    {
      double ub[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double a = ldrow(Uk + v * n, li[2]), b = ldrow(Uk + v * n, li[3]);
        if (v == NS + DIR) {
          if (fl2) a = -a;
          if (fl3) b = -b;
        }
        ub[v] = 0.5 * (a + b);
      }
      Thermo<NS, DIM> tf;
      equilibrium<NS, DIM, VAR>(p, ub, tf, true);
      cT = tf.cT;
      z = tf.z;
    }
    // ---- Godunov steps 1c-3: characteristic WENO5-Z, one variable at a
    // time (its six stencil values are loaded just before use; the compiler
    // barriers keep the loads from being hoisted, which bounds live registers)
    double TL, TR, PL, PR, unL, unR, utL[NTa], utR[NTa], YL[NS], YR[NS];
    {
      const float weps = fmaxf((float)p.weps, 1e-30f);
      auto recon = [&](const double* w, double& l, double& rr) {
        if constexpr (MIXED) {
          // FP32 weights, FP64 candidates and combination
          l = weno5z_mixed(w[0], w[1], w[2], w[3], w[4], weps, p.wp);
          __builtin_amdgcn_sched_barrier(0);
          rr = weno5z_mixed(w[5], w[4], w[3], w[2], w[1], weps, p.wp);
        } else {
          double2 o2;
          if constexpr (VAR)
            o2 = weno_lr(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp, p.scheme);
          else
            o2 = weno5z_lr(w[0], w[1], w[2], w[3], w[4], w[5], p.weps, p.wp);
          l = o2.x;
          rr = o2.y;
        }
        __builtin_amdgcn_sched_barrier(0);
      };
      double w[6], w1L, w1R, w5L, w5R, w6L, w6R;
      if (VAR && p.basis == 1) {
        // Negative control (Sec. 4.2.2, Table DropAdvectionNoIECResults):
        // the five-equation model's basis [rho Y_c, u, P], one variable at a
        // time; the face T fills the volume with the interpolated partial
        // densities at the interpolated P (sum_c rho Y_c v_c(P, T) = 1,
        // linear in T), Y_c = rho Y_c / sum rho Y.
        double rYL[NS], rYR[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          KBARRIER();
#pragma unroll
          for (int m = 0; m < 6; ++m) w[m] = ldrow(Uk + k * n, li[m]);
          recon(w, rYL[k], rYR[k]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          KBARRIER();
          const double* __restrict__ QUt = Q + (p.qU + tdir<DIM, DIR>(t)) * n;
#pragma unroll
          for (int m = 0; m < 6; ++m) w[m] = ldrow(QUt, li[m]);
          recon(w, utL[t], utR[t]);
        }
        KBARRIER();
#pragma unroll
        for (int m = 0; m < 6; ++m) w[m] = (flips >> m) & 1u ? -ldrow(QUn, li[m]) : ldrow(QUn, li[m]);
        recon(w, unL, unR);
        KBARRIER();
#pragma unroll
        for (int m = 0; m < 6; ++m) w[m] = ldrow(QP, li[m]);
        recon(w, PL, PR);
        auto face_T = [&](const double* rY, double P, double* Y, double& T) {
          double rho = 0.0, num = 1.0, den = 0.0;
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            rho += rY[k];
            num -= rY[k] * p.b[k];
            den += rY[k] * kappa_c<double>(p, k, P);
          }
          const double ir = 1.0 / rho;
#pragma unroll
          for (int k = 0; k < NS; ++k) Y[k] = rY[k] * ir;
          T = num / den;
        };
        face_T(rYL, PL, YL, TL);
        face_T(rYR, PR, YR, TR);
      } else {
       if constexpr (VAR) {
        // the variants' reconstruction call (scheme by option), one
        // characteristic variable at a time
        KBARRIER();
#pragma unroll
        for (int m = 0; m < 6; ++m) w[m] = ldrow(QT, li[m]) - cT * ldrow(QP, li[m]);
        recon(w, w1L, w1R);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          KBARRIER();
          const double* __restrict__ QY = Q + (p.qY + k) * n;
#pragma unroll
          for (int m = 0; m < 6; ++m) w[m] = ldrow(QY, li[m]);
          recon(w, YL[k], YR[k]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          KBARRIER();
          const double* __restrict__ QUt = Q + (p.qU + tdir<DIM, DIR>(t)) * n;
#pragma unroll
          for (int m = 0; m < 6; ++m) w[m] = ldrow(QUt, li[m]);
          recon(w, utL[t], utR[t]);
        }
        KBARRIER();
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          const double un = (flips >> m) & 1u ? -ldrow(QUn, li[m]) : ldrow(QUn, li[m]);
          w[m] = 0.5 * z * un + 0.5 * ldrow(QP, li[m]);
        }
        recon(w, w5L, w5R);
        KBARRIER();
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          const double un = (flips >> m) & 1u ? -ldrow(QUn, li[m]) : ldrow(QUn, li[m]);
          w[m] = -0.5 * z * un + 0.5 * ldrow(QP, li[m]);
        }
        recon(w, w6L, w6R);
        KBARRIER();
       } else {
        // Characteristic variables of S^-1 W, one per iteration of a loop
        // that is not unrolled (one copy of the reconstruction, no call):
        // variable v is w = fma(a, A, b B) over the six stencil cells, A and
        // B rows of Q -- v = 0: -cT P + T; then Y_k; then the tangential
        // velocities; then (z/2) u_n + P/2 and -(z/2) u_n + P/2 with u_n
        // negated where a mirror maps the cell.  The stencil of variable v + 1
        // is loaded while variable v is reconstructed.
        constexpr int NW = NS + NT + 3;
        auto rows = [&](int v, int& qa, int& qb, double& a, double& b) {
          qb = -1;
          b = 0.0;
          a = 1.0;
          if (v == 0) {
            qa = p.qP;
            qb = p.qT;
            a = -cT;
            b = 1.0;
          } else if (v <= NS) {
            qa = p.qY + v - 1;
          } else if (v <= NS + NT) {
            qa = p.qU + tdir<DIM, DIR>(v - 1 - NS == 0 ? 0 : 1);
          } else {
            qa = p.qU + DIR;
            qb = p.qP;
            a = v == NW - 2 ? 0.5 * z : -0.5 * z;
            b = 0.5;
          }
        };
        double nA[6], nB[6];
        double qL[NW], qR[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) qL[k] = qR[k] = 0.0;
        auto fetch = [&](int qa, int qb) {
          const double* __restrict__ A = Q + qa * n;
#pragma unroll
          for (int m = 0; m < 6; ++m) nA[m] = ldrow(A, li[m]);
          if (qb >= 0) {
            const double* __restrict__ B = Q + qb * n;
#pragma unroll
            for (int m = 0; m < 6; ++m) nB[m] = ldrow(B, li[m]);
          }
        };
        int qa, qb;
        double ca, cb;
        rows(0, qa, qb, ca, cb);
        fetch(qa, qb);
#pragma unroll 1
        for (int v = 0; v < NW; ++v) {
          // combine the fetched rows (u_n mirrored where the map flips)
          const bool un_row = v >= NW - 2;
#pragma unroll
          for (int m = 0; m < 6; ++m) {
            const double av = (un_row && ((flips >> m) & 1u)) ? -nA[m] : nA[m];
            w[m] = qb >= 0 ? fma(ca, av, cb * nB[m]) : av;
          }
          if (v + 1 < NW) {
            rows(v + 1, qa, qb, ca, cb);
            fetch(qa, qb);
          }
          double l, r;
          if constexpr (MIXED) {
            l = weno5z_mixed(w[0], w[1], w[2], w[3], w[4], weps, p.wp);
            __builtin_amdgcn_sched_barrier(0);
            r = weno5z_mixed(w[5], w[4], w[3], w[2], w[1], weps, p.wp);
          } else {
            l = weno5z<double>(w[0], w[1], w[2], w[3], w[4], p.weps, p.wp);
            r = weno5z<double>(w[5], w[4], w[3], w[2], w[1], p.weps, p.wp);
          }
          // shift the results down one slot and append this variable's:
          // after the last iteration slot k holds variable k (register
          // moves, no selects on the loop index)
#pragma unroll
          for (int k = 0; k + 1 < NW; ++k) {
            qL[k] = qL[k + 1];
            qR[k] = qR[k + 1];
          }
          qL[NW - 1] = l;
          qR[NW - 1] = r;
        }
        KBARRIER();
        w1L = qL[0];
        w1R = qR[0];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          YL[k] = qL[1 + k];
          YR[k] = qR[1 + k];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          utL[t] = qL[1 + NS + t];
          utR[t] = qR[1 + NS + t];
        }
        w5L = qL[NW - 2];
        w5R = qR[NW - 2];
        w6L = qL[NW - 1];
        w6R = qR[NW - 1];
       }
        PL = w5L + w6L;
        PR = w5R + w6R;
        unL = (w5L - w6L) / z;
        unR = (w5R - w6R) / z;
        TL = w1L + cT * PL;
        TR = w1R + cT * PR;
      }
    }
    // cell values of the two face cells
    double cYL[NS], cYR[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      cYL[k] = ldrow(Q + (p.qY + k) * n, li[2]);
      cYR[k] = ldrow(Q + (p.qY + k) * n, li[3]);
    }
    const double cTL = ldrow(QT, li[2]), cTR = ldrow(QT, li[3]), cPL = ldrow(QP, li[2]), cPR = ldrow(QP, li[3]);
    const double cUnL = fl2 ? -ldrow(QUn, li[2]) : ldrow(QUn, li[2]), cUnR = fl3 ? -ldrow(QUn, li[3]) : ldrow(QUn, li[3]);
    // ---- interpolation limiters (Sec. 3.3.1)
    if (p.pos) {
      ylimit<NS, double>(YL, cYL);
      ylimit<NS, double>(YR, cYR);
      if constexpr (REPLAY) {
        const uint16_t r = mrep[f];
        if (r & 1) TL = cTL;
        if (r & 2) TR = cTR;
        if (r & 4) PL = cPL;
        if (r & 8) PR = cPR;
        m16 |= r & 15;
      } else {
        if (!(TL > 0.0)) { TL = cTL; m16 |= 1; }
        if (!(TR > 0.0)) { TR = cTR; m16 |= 2; }
        bool badL = false, badR = false;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          if (YL[k] > 0.0 && !(PL + p.pinf[k] > 0.0)) badL = true;
          if (YR[k] > 0.0 && !(PR + p.pinf[k] > 0.0)) badR = true;
        }
        if (badL) { PL = cPL; m16 |= 4; }
        if (badR) { PR = cPR; m16 |= 8; }
      }
    }
    // ---- Godunov steps 4-6: face EOS and HLLC (FP64)
    double F[NV];
    {
      Side<NS, DIM, double> sL, sR;
      face_state<NS, DIM, double>(p, PL, TL, YL, unL, utL, sL);
      face_state<NS, DIM, double>(p, PR, TR, YR, unR, utR, sR);
      double Fr[NV];
      hllc<NS, DIM, double>(sL, sR, Fr);
      unrotate<NS, DIM, DIR>(Fr, F);
    }
    KBARRIER();
    const double dt = dtg[0], Gamma = dtg[1];
    // ---- advective flux limiter (Sec. 3.3.2).  The pseudo-states are
    // rk0 U^n + rk1 U^k -+ lam (F - F_cell); their F-independent parts are
    // formed once (baseL, baseR).
    const double lam = 2.0 * DIM * rk2 * dt / p.dx[DIR];
    // cell side of one face cell, from Q and U^k
    auto cell_side = [&](int l, bool flip, Side<NS, DIM, double>& cs) {
      cell_side_at<NS, DIM, DIR>(p, Q, Uk, l, flip, cs);
    };
    // F-independent part of the pseudo-state of cell l, rk0 U^n + rk1 U^k +
    // sgn lam F_cell, from fresh loads of U^n, U^k and Q (so no cell state
    // stays live across the reconstruction for it)
    auto make_base = [&](int l, bool flip, double sgn, double* base) {
      Side<NS, DIM, double> cs;
      double Ua[NV], Fr[NV], Fc[NV];
      cell_side(l, flip, cs);
      side_UF<NS, DIM, double>(cs, Ua, Fr);
      unrotate<NS, DIM, DIR>(Fr, Fc);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double un_ = ldrow(Un + v * n, l), uk_ = ldrow(Uk + v * n, l);
        if (v == NS + DIR && flip) {
          un_ = -un_;
          uk_ = -uk_;
        }
        base[v] = rk0 * un_ + rk1 * uk_ + sgn * lam * Fc[v];
      }
    };
    double baseL[NV], baseR[NV];
    auto pseudo_test = [&](const double* G) {
      double a[NV], b[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        a[v] = baseL[v] - lam * G[v];
        b[v] = baseR[v] + lam * G[v];
      }
      return admissible<NS, DIM>(p, a) && admissible<NS, DIM>(p, b);
    };
    if (REPLAY && p.pos) {
      if (mrep[f] & 16) {
        m16 |= mrep[f] & (16 | 64);
        Side<NS, DIM, double> cl, cr;
        double Fr[NV];
        cell_side(li[2], fl2, cl);
        cell_side(li[3], fl3, cr);
        hllc<NS, DIM, double>(cl, cr, Fr);
        unrotate<NS, DIM, DIR>(Fr, F);
      }
    } else if (p.pos) {
      make_base(li[2], fl2, 1.0, baseL);
      make_base(li[3], fl3, -1.0, baseR);
      if (!pseudo_test(F)) {
        m16 |= 16;
        Side<NS, DIM, double> cl, cr;
        double Fr[NV];
        cell_side(li[2], fl2, cl);
        cell_side(li[3], fl3, cr);
        hllc<NS, DIM, double>(cl, cr, Fr);
        unrotate<NS, DIM, DIR>(Fr, F);
        if (!pseudo_test(F)) m16 |= 64;
      }
    }
    KBARRIER();
    double Fdi[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fdi[v] = 0.0;
    // ---- interface regularization flux (Sec. 3.2.1), first phase, a_2 = -a_1
    if (p.cdi) {
      const double dxn = p.dx[DIR];
      const double f0L = ldrow(Q + p.qPhi0 * n, li[2]), f0R = ldrow(Q + p.qPhi0 * n, li[3]);
      const double gphi = (f0R - f0L) / dxn;
      const double psiL = ldrow(Q + p.qPsi * n, li[2]), psiR = ldrow(Q + p.qPsi * n, li[3]);
      const double psib = 0.5 * (psiL + psiR);
      const double gn = (psiR - psiL) / dxn;
      double nrm2 = gn * gn;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        constexpr int dummy = 0;
        (void)dummy;
        const int td = tdir<DIM, DIR>(t);
        double gt = 0.0;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          double ps[2];
#pragma unroll
          for (int sgn = 0; sgn < 2; ++sgn) {
            // cell li[2 + side] moved by -1 / +1 along the tangential direction
            bool flip = false;
            const int ct = c[td] + (sgn ? 1 : -1);
            const int stride_t = td == 0 ? 1 : (td == 1 ? p.n[0] : p.n[0] * p.n[1]);
            const int mt = (ct < 0 || ct >= p.n[td]) ? map_index(ct, p.n[td], p.bclo[td], p.bchi[td], flip) : ct;
            const int lt = li[2 + side] + (mt - c[td]) * stride_t;
            ps[sgn] = ldrow(Q + p.qPsi * n, lt);
          }
          gt += ps[1] - ps[0];
        }
        gt = gt / (4.0 * p.dx[td]);
        nrm2 += gt * gt;
      }
      double nhat, th;
      if constexpr (MIXED) {
        // FP32 normal and profile; a_1 and the fluxes built from it in FP64
        const float n2f = (float)nrm2;
        nhat = n2f > 0.0f ? (double)((float)gn * __frsqrt_rn(n2f)) : 0.0;
        th = (double)tanhf((float)(psib / (2.0 * p.eps)));
      } else {
        nhat = nrm2 > 0.0 ? gn / sqrt(nrm2) : 0.0;
        th = tanh(psib / (2.0 * p.eps));
      }
      const double a1 = Gamma * (p.eps * gphi - 0.25 * (1.0 - th * th - p.sharp_floor) * nhat);
      double Rsum = 0.0, hR = 0.0;
#pragma unroll
      for (int pp = 0; pp < 2; ++pp) {
        const double ap = pp == 0 ? a1 : -a1;
        const int ph = p.pid[pp];
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) {
            const double Rk = -0.5 * (ldrow(Q + (p.qYrho + k) * n, li[2]) + ldrow(Q + (p.qYrho + k) * n, li[3])) * ap;
            Fdi[k] = Rk;
            Rsum += Rk;
          }
        hR += -0.5 * (ldrow(Q + (p.qHrho + pp) * n, li[2]) + ldrow(Q + (p.qHrho + pp) * n, li[3])) * ap;
      }
      double kb = 0.0;
#pragma unroll
      for (int dd = 0; dd < DIM; ++dd) {
        double vL = ldrow(Q + (p.qU + dd) * n, li[2]), vR = ldrow(Q + (p.qU + dd) * n, li[3]);
        if (dd == DIR) {
          vL = cUnL;
          vR = cUnR;
        }
        Fdi[NS + dd] = 0.5 * (vL + vR) * Rsum;
        kb += vL * vR;
      }
      kb = 0.5 * kb;
      Fdi[NS + DIM] = kb * Rsum + hR;
      if (REPLAY && p.pos) {
        if (mrep[f] & 32) {
          m16 |= 32;
#pragma unroll
          for (int v = 0; v < NV; ++v) Fdi[v] = 0.0;
        }
      } else if (p.pos) {
        double Ft[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Ft[v] = F[v] + Fdi[v];
        if (!pseudo_test(Ft)) {
          m16 |= 32;
#pragma unroll
          for (int v = 0; v < NV; ++v) Fdi[v] = 0.0;
        }
      }
    }
    // ---- phase-confined species diffusion and its enthalpy flux
    double Fdf[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fdf[v] = 0.0;
    if (p.diff) {
      const double dxn = p.dx[DIR];
      const double rhob = 0.5 * (ldrow(Q + p.qRho * n, li[2]) + ldrow(Q + p.qRho * n, li[3]));
      double eflux = 0.0;
      for (int pp = 0; pp < p.np; ++pp) {
        if (!p.multi[pp]) continue;
        const int ph = p.pid[pp];
        double Yb[NS], Kb[NS], G[NS], Yp = 0.0, sKG = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) {
            Yb[k] = 0.5 * (cYL[k] + cYR[k]);
            Kb[k] = 0.5 * (ldrow(Q + (p.qK + k) * n, li[2]) + ldrow(Q + (p.qK + k) * n, li[3]));
            G[k] = (ldrow(Q + (p.qChi + k) * n, li[3]) - ldrow(Q + (p.qChi + k) * n, li[2])) / dxn;
            Yp += Yb[k];
            sKG += Kb[k] * G[k];
          }
#pragma unroll
        for (int k = 0; k < NS; ++k)
          if (p.phase[k] == ph) {
            const double J = -rhob * (Kb[k] * Yp * G[k] - Yb[k] * sKG);
            Fdf[k] = J;
            eflux += J * (0.5 * (ldrow(Q + (p.qH + k) * n, li[2]) + ldrow(Q + (p.qH + k) * n, li[3])));
          }
      }
      Fdf[NS + DIM] = eflux;
    }
    // ---- viscous stress and heat conduction (Eq. DiffusionTerms), second-
    // order central: face mu, lambda and velocity the means of the two face
    // cells, normal derivatives two-point, tangential derivatives the mean of
    // the two cells' central differences; the energy entry is -u.tau + q
    if (p.visc) {
      const double dxn = p.dx[DIR];
      // velocity component i of cell l, with the mirror flips of its maps
      auto vel_at = [&](int l, int i, bool flipn, bool flipt, int td) {
        double v = ldrow(Q + (p.qU + i) * n, l);
        if ((i == DIR && flipn) != (i == td && flipt)) v = -v;
        return v;
      };
      double g[DIM][DIM];  // g[i][j] = du_i / dx_j at the face
      double work_u[DIM];
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        const double a = vel_at(li[2], i, fl2, false, -1), b = vel_at(li[3], i, fl3, false, -1);
        g[i][DIR] = (b - a) / dxn;
        work_u[i] = 0.5 * (a + b);
      }
#pragma unroll
      for (int t = 0; t < DIM - 1; ++t) {
        const int td = tdir<DIM, DIR>(t);
        const int stride_t = td == 0 ? 1 : (td == 1 ? p.n[0] : p.n[0] * p.n[1]);
        double acc[DIM];
#pragma unroll
        for (int i = 0; i < DIM; ++i) acc[i] = 0.0;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const bool fn_ = side ? fl3 : fl2;
#pragma unroll
          for (int sgn = 0; sgn < 2; ++sgn) {
            bool ft = false;
            const int ct = c[td] + (sgn ? 1 : -1);
            const int mt = (ct < 0 || ct >= p.n[td]) ? map_index(ct, p.n[td], p.bclo[td], p.bchi[td], ft) : ct;
            const int lt = li[2 + side] + (mt - c[td]) * stride_t;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              const double v = vel_at(lt, i, fn_, ft, td);
              acc[i] += sgn ? v : -v;
            }
          }
        }
#pragma unroll
        for (int i = 0; i < DIM; ++i) g[i][td] = acc[i] / (4.0 * p.dx[td]);
      }
      double div = 0.0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) div += g[i][i];
      const double muf = 0.5 * (ldrow(Q + p.qMu * n, li[2]) + ldrow(Q + p.qMu * n, li[3]));
      const double lamf = 0.5 * (ldrow(Q + p.qLam * n, li[2]) + ldrow(Q + p.qLam * n, li[3]));
      double work = 0.0;
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        double tau = muf * (g[DIR][i] + g[i][DIR]);
        if (i == DIR) tau -= muf * (2.0 / 3.0) * div;
        Fdf[NS + i] -= tau;
        work += work_u[i] * tau;
      }
      Fdf[NS + DIM] += -work - lamf * (ldrow(Q + p.qT * n, li[3]) - ldrow(Q + p.qT * n, li[2])) / dxn;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Fsum[v] = F[v] + Fdi[v] + Fdf[v];
  }
  int up = -1;
  bool own = true;
  if constexpr (!FUSE) {
    if (valid) {
      if (p.stream) {
#pragma unroll
        for (int v = 0; v < NV; ++v) strow_t<true>(Fo + v * nf, (int)f, Fsum[v]);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) strow_t<false>(Fo + v * nf, (int)f, Fsum[v]);
      }
      if (mask) mask[f] = m16;
    }
  } else {
    // the tile coordinates again, from a thread index the compiler cannot
    // carry over from the start (keeps them out of the face computation's
    // registers)
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    int cu[3];
    fused_coords<DIR>(e0, e1, e2, tid, cu, &up, &own);
    if (valid && mask && own) mask[((long)cu[2] * e1 + cu[1]) * e0 + cu[0]] = m16;
    // exchange the face fluxes through LDS; the thread of a cell's low face
    // updates the cell with the flux of its high face (slot up)
    __shared__ double sF[NV][256];
    if (valid) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[v][threadIdx.x] = Fsum[v];
    }
    __syncthreads();
    if (up >= 0) {
      const long i = lin3(p, cu[0], cu[1], cu[2]);
      const double dt = dtg[0];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double d = (sF[v][up] - sF[v][threadIdx.x]) / p.dx[DIR];
        if (fmode == 0) {
          strow(Fo + v * n, i, 0.0 + d, p.stream);
        } else if (fmode == 1) {
          strow(Fo + v * n, i, ldrow(Fo + v * n, i) + d, p.stream);
        } else {
          const double acc = (fmode == 3 ? 0.0 : ldrow(Fo + v * n, i)) + d;
          const double L = -acc;
          strow(Fo + v * n, i, rk0 * ldrow(Un + v * n, i) + rk1 * ldrow(Uk + v * n, i) + rk2 * dt * L, p.stream);
        }
      }
    }
  }
  if (cnt) {
    // per wavefront (ballots, no block barrier: a wave retires as soon as it
    // is done), one set of atomics per wave
    const bool vo = valid && own;
    const int nT = __popcll(__ballot(vo && (m16 & 3)));
    const int nP = __popcll(__ballot(vo && (m16 & 12)));
    const int nF = __popcll(__ballot(vo && (m16 & 16)));
    const int nD = __popcll(__ballot(vo && (m16 & 32)));
    const int nU = __popcll(__ballot(vo && (m16 & 64)));
    const int nV = __popcll(__ballot(vo));
    if ((threadIdx.x & 63) == 0) {
      unsigned long long* cs = cnt_slot(cnt);
      if (nT) atomicAdd(cs + kCntT, (unsigned long long)nT);
      if (nP) atomicAdd(cs + kCntP, (unsigned long long)nP);
      if (nF) atomicAdd(cs + kCntFallback, (unsigned long long)nF);
      if (nD) atomicAdd(cs + kCntDrop, (unsigned long long)nD);
      if (nU) {
        atomicAdd(cs + kCntUnrec, (unsigned long long)nU);
        raise_flag(flag);
      }
      atomicAdd(cs + kCntFaces, (unsigned long long)nV);
    }
  }
}

// ---------------------------------------------------------------------------
// k_update: L = -sum_d (F_hi - F_lo)/dx_d and the RK stage combination
// ---------------------------------------------------------------------------
// One cell's L and stage combination (k_update), with or without the
// non-temporal hint on its streamed loads and stores.
template <bool NT, int NV, int DIM>
__device__ __forceinline__ void update_cell(const Params& p, long i, const double* __restrict__ Un,
                                            const double* __restrict__ Uk, const double* const* Fd,
                                            const long* nfd, const long* lo, const long* hi, double dt,
                                            double rk0, double rk1, double rk2, double* __restrict__ Uout,
                                            double* __restrict__ Lout) {
  const long n = p.ncell;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      acc += (ldrow(Fd[d] + v * nfd[d], (int)hi[d]) - ldrow(Fd[d] + v * nfd[d], (int)lo[d])) / p.dx[d];
    const double L = -acc;
    if (Lout) strow_t<NT>(Lout + v * n, i, L);
    if (Uout)
      strow_t<NT>(Uout + v * n, i, rk0 * ldrow_t<NT>(Un + v * n, i) + rk1 * ldrow_t<NT>(Uk + v * n, i) + rk2 * dt * L);
  }
}

template <int NS, int DIM>
__global__ __launch_bounds__(256) void k_update(const Params p, const double* __restrict__ Un,
                                                const double* __restrict__ Uk,
                                                const double* __restrict__ F0,
                                                const double* __restrict__ F1,
                                                const double* __restrict__ F2,
                                                const double* __restrict__ dtg, double rk0,
                                                double rk1, double rk2, double* __restrict__ Uout,
                                                double* __restrict__ Lout) {
  constexpr int NV = NS + DIM + 1;
  const long n = p.ncell;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int c0, c1, c2;
  decompose((long)blockIdx.x * blockDim.x, p.n[0], p.n[1], c0, c1, c2);
  if (i >= n) return;
  const double* Fd[3] = {F0, F1, F2};
  long lo[3], hi[3], nfd[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int e0 = p.n[0] + (d == 0), e1 = p.n[1] + (d == 1), e2 = p.n[2] + (d == 2);
    nfd[d] = (long)e0 * e1 * e2;
    lo[d] = ((long)c2 * e1 + c1) * e0 + c0;
    hi[d] = lo[d] + (d == 0 ? 1 : (d == 1 ? (long)e0 : (long)e0 * e1));
  }
  const double dt = dtg[0];
  if (p.stream)
    update_cell<true, NV, DIM>(p, i, Un, Uk, Fd, nfd, lo, hi, dt, rk0, rk1, rk2, Uout, Lout);
  else
    update_cell<false, NV, DIM>(p, i, Un, Uk, Fd, nfd, lo, hi, dt, rk0, rk1, rk2, Uout, Lout);
}

// ---------------------------------------------------------------------------
// initial state from primitive fields (mixing rules of Sec. 2.2)
// ---------------------------------------------------------------------------
template <int NS, int DIM>
__global__ void k_init_state(const Params p, const double* __restrict__ phi,
                             const double* __restrict__ y, const double* __restrict__ P,
                             const double* __restrict__ T, const double* __restrict__ vel,
                             double* __restrict__ U) {
  const long n = p.ncell;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double Pc = P[i], Tc = T[i];
  double rY[NS];
  for (int pp = 0; pp < p.np; ++pp) {
    const int ph = p.pid[pp];
    double vp = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) vp += y[k * n + i] * (kappa_c<double>(p, k, Pc) * Tc + p.b[k]);
    const double rhop = 1.0 / vp;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (p.phase[k] == ph) rY[k] = phi[ph * n + i] * rhop * y[k * n + i];
  }
  double rho = 0.0, rhoe = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    strow(U + k * n, i, rY[k], p.stream);
    rho += rY[k];
    rhoe += rY[k] * (epsT_c<double>(p, k, Pc) * Tc + p.q[k]);
  }
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double vd = vel[d * n + i];
    strow(U + (NS + d) * n, i, rho * vd, p.stream);
    ke += vd * vd;
  }
  strow(U + (NS + DIM) * n, i, rhoe + 0.5 * rho * ke, p.stream);
}

// ---------------------------------------------------------------------------
// deterministic conservation sums: per-block partials, then one block per
// variable adds the partials in index order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sum_partial(const double* __restrict__ U, long n,
                                                     double* __restrict__ part) {
  __shared__ double sm[256];
  const int v = blockIdx.y;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc += ldrow(U + v * n, i);
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[v * gridDim.x + blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ part, int nb,
                                                   double* __restrict__ out) {
  __shared__ double sm[256];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[v * nb + i];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sm[0];
}

}  // namespace mpmc
