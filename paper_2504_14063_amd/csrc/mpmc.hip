// mpmc.hip -- MI355X (gfx950) kernels and C ABI of the four-equation MPMC hot
// path (Collis, Bezgin, Mirjalili & Mani, arXiv 2504.14063): finite-volume
// right-hand side (Eq. DiscreteGoverningEquations) advanced by SSP-RK3
// (Eq. SSPRK3).  The ABI is declared in include/mpmc.h.
//
// Per RK stage:
//   k_cell    one thread per cell: equilibrium (Sec. 2.3), sound speed, phase
//             and diffusion auxiliaries -> cell-quantity array Q (SoA), and
//             optionally the dt / Gamma maxima (wavefront + block reduction,
//             one 64-bit atomicMax per block).
//   k_face<d> one thread per face of direction d, threads along x in every
//             direction (coalesced): face average and its eigenvector
//             coefficients, characteristic WENO5-Z, limiters, face EOS, HLLC,
//             flux limiter, regularization and diffusion fluxes -> F_d.
//   k_update  one thread per cell: L = -sum_d dF/dx_d and the RK combination.
// Boundary conditions are index maps applied when a stencil is loaded; no
// ghost storage.  No atomics touch floating-point data: results are
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mpmc.h"
#include "mpmc_device.h"
#include "mpmc_kernels.h"
#include "mpmc_adjoint.h"
#include "mpmc_params.h"

using namespace mpmc;

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct mpmc_ctx {
  Params p;
  int ns = 0, dim = 0, nv = 0, precision = 0, split = 0;
  double* Q = nullptr;
  double* F[3] = {nullptr, nullptr, nullptr};
  double* S1 = nullptr;
  double* S2 = nullptr;
  double* dtg = nullptr;                 // [dt, Gamma]
  unsigned long long* rates = nullptr;   // max rate, max |u| as ordered bits, kRateSlots slots each
  unsigned long long* cnt = nullptr;     // limiter and failure counters, kCntSlots slots
  // failure flag (host-visible word, set by kernels that meet an
  // inadmissible cell or an unrecoverable face; read by the next call)
  unsigned* hflag = nullptr;  // host address
  unsigned* dflag = nullptr;  // device address of the same word
  double* partial = nullptr;             // conservation partial sums
  long nf[3] = {0, 0, 0};
  long masksize = 0;
  int nblk_sum = 0;
  int device = 0;   // device current at mpmc_init
  hipStream_t last = nullptr;
  // inflow cells held at fixed conserved values (mpmc_set_held_cells):
  // indices [nheld] and values [nv][nheld]
  long nheld = 0;
  long* held_idx = nullptr;
  double* held_U = nullptr;
  // adjoint scratch, allocated by the first mpmc_adjoint_step:
  // frec: the face records of the pull-back, rec_doubles of each direction
  // (directions in order); lam2 / lam1 [nv][cells] stage cotangents; amask
  // [3][masksize] face decisions of the recomputed stages
  double* frec = nullptr;
  double* fmid = nullptr;  // hand-over between the face pull-back's halves
  // the y sweep's pull-back runs beside the x (and z) sweep's on a second
  // stream of default priority, with its own hand-over buffer
  double* fmid2 = nullptr;
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* lam2 = nullptr;
  double* lam1 = nullptr;
  uint16_t* amask = nullptr;
  // kernel timing (mpmc_profile)
  struct Rec {
    hipEvent_t a, b;
    int cls;
  };
  bool prof = false;
  std::vector<Rec> recs;
  size_t nrec = 0;
  double prof_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long prof_n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

// Accumulate the recorded event pairs into the per-class totals.
static int prof_flush(mpmc_ctx* c) {
  if (c->nrec == 0) return MPMC_OK;
  if (hipStreamSynchronize(c->last) != hipSuccess) return MPMC_EHIP;
  for (size_t i = 0; i < c->nrec; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->recs[i].a, c->recs[i].b) != hipSuccess) return MPMC_EHIP;
    c->prof_ms[c->recs[i].cls] += ms;
    c->prof_n[c->recs[i].cls] += 1;
  }
  c->nrec = 0;
  return MPMC_OK;
}

static int prof_begin(mpmc_ctx* c, hipStream_t s) {
  if (!c->prof) return -1;
  if (c->nrec >= 4096) prof_flush(c);
  if (c->nrec == c->recs.size()) {
    mpmc_ctx::Rec r;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    c->recs.push_back(r);
  }
  (void)hipEventRecord(c->recs[c->nrec].a, s);
  return (int)c->nrec++;
}

static void prof_end(mpmc_ctx* c, int id, int cls, hipStream_t s) {
  if (id < 0) return;
  c->recs[id].cls = cls;
  (void)hipEventRecord(c->recs[id].b, s);
}

#define TIMED(c, cls, s, launch)          \
  do {                                    \
    const int _id = prof_begin(c, s);     \
    launch;                               \
    prof_end(c, _id, cls, s);             \
  } while (0)

static const char* kErr[] = {"ok", "invalid argument", "out of device memory", "HIP runtime error",
                             "inadmissible state after all fallbacks", "unsupported configuration"};

extern "C" const char* mpmc_strerror(int code) {
  if (code > 0 || code < -5) return "unknown error";
  return kErr[-code];
}

#define HIPCHK(x)                                  \
  do {                                             \
    if ((x) != hipSuccess) return MPMC_EHIP;       \
  } while (0)

static inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Return value of an entry point that enqueued its work: MPMC_EINADMISSIBLE
// once after kernels of earlier calls (already completed) met an
// inadmissible cell or an unrecoverable face, else MPMC_OK.  The host reads
// the flag without synchronizing and clears it (it is reported once; the
// counters of mpmc_stats keep the totals).
static int enqueue_status(mpmc_ctx* c) {
  HIPCHK(hipGetLastError());
  if (__atomic_exchange_n(c->hflag, 0u, __ATOMIC_ACQ_REL) != 0u) return MPMC_EINADMISSIBLE;
  return MPMC_OK;
}

// ---------------------------------------------------------------------------
// Dispatch over (NS, DIM): every form up to kFullNS components
// ---------------------------------------------------------------------------
#define DISPATCH(ctx, ...)                                               \
  do {                                                                   \
    const int _k = (ctx)->ns * 10 + (ctx)->dim;                          \
    switch (_k) {                                                        \
      case 11: { constexpr int NS = 1, DIM = 1; __VA_ARGS__; } break;           \
      case 12: { constexpr int NS = 1, DIM = 2; __VA_ARGS__; } break;           \
      case 13: { constexpr int NS = 1, DIM = 3; __VA_ARGS__; } break;           \
      case 21: { constexpr int NS = 2, DIM = 1; __VA_ARGS__; } break;           \
      case 22: { constexpr int NS = 2, DIM = 2; __VA_ARGS__; } break;           \
      case 23: { constexpr int NS = 2, DIM = 3; __VA_ARGS__; } break;           \
      case 31: { constexpr int NS = 3, DIM = 1; __VA_ARGS__; } break;           \
      case 32: { constexpr int NS = 3, DIM = 2; __VA_ARGS__; } break;           \
      case 33: { constexpr int NS = 3, DIM = 3; __VA_ARGS__; } break;           \
      default: return MPMC_EUNSUPPORTED;                                 \
    }                                                                    \
  } while (0)

// The FP64 forward entry points: also 4 to MAXS components.
#define WIDE_CASES(NSV, ...)                                                   \
  case NSV * 10 + 1: { constexpr int NS = NSV, DIM = 1; __VA_ARGS__; } break; \
  case NSV * 10 + 2: { constexpr int NS = NSV, DIM = 2; __VA_ARGS__; } break; \
  case NSV * 10 + 3: { constexpr int NS = NSV, DIM = 3; __VA_ARGS__; } break;
#define DISPATCH_WIDE(ctx, ...)                                          \
  do {                                                                   \
    const int _k = (ctx)->ns * 10 + (ctx)->dim;                          \
    switch (_k) {                                                        \
      WIDE_CASES(1, __VA_ARGS__)                                         \
      WIDE_CASES(2, __VA_ARGS__)                                         \
      WIDE_CASES(3, __VA_ARGS__)                                         \
      WIDE_CASES(4, __VA_ARGS__)                                         \
      WIDE_CASES(5, __VA_ARGS__)                                         \
      WIDE_CASES(6, __VA_ARGS__)                                         \
      WIDE_CASES(7, __VA_ARGS__)                                         \
      WIDE_CASES(8, __VA_ARGS__)                                         \
      default: return MPMC_EUNSUPPORTED;                                 \
    }                                                                    \
  } while (0)

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
// check: count the inadmissible cells of U (the stage inputs of the forward
// entry points; failure detection).
template <int NS, int DIM>
static void launch_cell(mpmc_ctx* c, const double* U, bool rates, hipStream_t s, bool check = false) {
  const int bs = 256;
  unsigned long long* cnt = check ? c->cnt : nullptr;
  if (rates) TIMED(c, 5, s, hipLaunchKernelGGL(k_zero_rates, dim3(1), dim3(64), 0, s, c->rates));
  if (c->p.pgen)
    TIMED(c, 0, s,
          hipLaunchKernelGGL((k_cell<NS, DIM, true>), dim3(nblocks(c->p.ncell, bs)), dim3(bs), 0, s, c->p, U,
                             c->Q, rates ? c->rates : nullptr, cnt, c->dflag));
  else
    TIMED(c, 0, s,
          hipLaunchKernelGGL((k_cell<NS, DIM>), dim3(nblocks(c->p.ncell, bs)), dim3(bs), 0, s, c->p, U,
                             c->Q, rates ? c->rates : nullptr, cnt, c->dflag));
}

template <int NS, int DIM>
static void launch_faces(mpmc_ctx* c, const double* Uk, const double* Un, double rk0, double rk1,
                         double rk2, uint16_t* mask, hipStream_t s, bool count = true,
                         const uint16_t* mrep = nullptr) {
  unsigned long long* cnt = count ? c->cnt : nullptr;
  // one wavefront per workgroup: the face kernel has no block barrier in
  // this layout, so waves are retired and replaced one at a time (the
  // 256^3 step 1.7 % faster than with 256-thread workgroups)
  const int bs = 64;
  long off = 0;
  for (int d = 0; d < DIM; ++d) {
    uint16_t* m = mask ? mask + off : nullptr;
    const uint16_t* mr = mrep ? mrep + off : nullptr;
    // x: linear over faces; y, z: (x chunks) x (faces along d) x (other rows)
    const unsigned nb = d == 0 ? nblocks(c->nf[d], bs)
                               : (unsigned)(nblocks(c->p.n[0], bs) * (c->nf[d] / c->p.n[0]));
    constexpr int D1 = DIM > 1 ? 1 : 0, D2 = DIM > 2 ? 2 : 0;
    const int _id = prof_begin(c, s);
#define FACE_LAUNCH(DIRV, R, RP, VAR)                                                                     \
  hipLaunchKernelGGL((k_face<NS, DIM, DIRV, R, RP, VAR>), dim3(nb), dim3(bs), 0, s, c->p, Uk, Un, c->Q, c->F[d], \
                     m, c->dtg, rk0, rk1, rk2, cnt, mr, c->dflag, 0)
    if (mr) {  // frozen-decision forward (FP64 WENO5-Z only)
      if constexpr (NS <= kFullNS) {
        if (d == 0) FACE_LAUNCH(0, double, true, false);
        if (DIM > 1 && d == 1) FACE_LAUNCH(D1, double, true, false);
        if (DIM > 2 && d == 2) FACE_LAUNCH(D2, double, true, false);
      }
    } else if (c->precision == 0 && (c->p.scheme != 0 || c->p.basis != 0 || c->p.pgen)) {
      if (d == 0) FACE_LAUNCH(0, double, false, true);
      if (DIM > 1 && d == 1) FACE_LAUNCH(D1, double, false, true);
      if (DIM > 2 && d == 2) FACE_LAUNCH(D2, double, false, true);
    } else if (c->precision == 0) {
      if (d == 0) FACE_LAUNCH(0, double, false, false);
      if (DIM > 1 && d == 1) FACE_LAUNCH(D1, double, false, false);
      if (DIM > 2 && d == 2) FACE_LAUNCH(D2, double, false, false);
    } else {
      if constexpr (NS <= kFullNS) {
        if (d == 0) FACE_LAUNCH(0, float, false, false);
        if (DIM > 1 && d == 1) FACE_LAUNCH(D1, float, false, false);
        if (DIM > 2 && d == 2) FACE_LAUNCH(D2, float, false, false);
      }
    }
#undef FACE_LAUNCH
    prof_end(c, _id, 1 + d, s);
    off += c->nf[d];
  }
}

// The fused sweeps of one stage: every direction's face kernel also takes
// the divergence of its fluxes into the accumulator acc (the stage output
// buffer), the last one finishing the RK combination in place (FUSE of
// k_face).  Same bits as launch_faces followed by launch_update.
template <int NS, int DIM>
static void launch_faces_fused(mpmc_ctx* c, const double* Uk, const double* Un, double rk0, double rk1,
                               double rk2, double* acc, uint16_t* mask, hipStream_t s,
                               const uint16_t* mrep = nullptr) {
  unsigned long long* cnt = c->cnt;
  const int bs = 256;
  long off = 0;
  for (int d = 0; d < DIM; ++d) {
    uint16_t* m = mask ? mask + off : nullptr;
    const uint16_t* mr = mrep ? mrep + off : nullptr;
    unsigned nb;
    if (d == 0) {
      nb = (unsigned)((c->nf[0] - 1 + 254) / 255);
    } else {
      const int eD = c->p.n[d] + 1, eO = d == 1 ? c->p.n[2] : c->p.n[1];
      const long nbj = (eD - 1 + kFuseTY - 2) / (kFuseTY - 1);
      const long nbx = (c->p.n[0] + kFuseTX - 1) / kFuseTX;
      nb = (unsigned)(nbj * nbx * eO);
    }
    const bool first = d == 0, last = d == DIM - 1;
    const int fmode = first ? (last ? 3 : 0) : (last ? 2 : 1);
    constexpr int D1 = DIM > 1 ? 1 : 0, D2 = DIM > 2 ? 2 : 0;
    const int _id = prof_begin(c, s);
#define FUSED_LAUNCH(DIRV, R, RP, VAR)                                                                     \
  hipLaunchKernelGGL((k_face<NS, DIM, DIRV, R, RP, VAR, true>), dim3(nb), dim3(bs), 0, s, c->p, Uk, Un, c->Q, \
                     acc, m, c->dtg, rk0, rk1, rk2, cnt, mr, c->dflag, fmode)
    if (mr) {  // frozen-decision forward (FP64 WENO5-Z only)
      if (d == 0) FUSED_LAUNCH(0, double, true, false);
      if (DIM > 1 && d == 1) FUSED_LAUNCH(D1, double, true, false);
      if (DIM > 2 && d == 2) FUSED_LAUNCH(D2, double, true, false);
    } else if (c->precision == 0 && (c->p.scheme != 0 || c->p.basis != 0 || c->p.pgen)) {
      if (d == 0) FUSED_LAUNCH(0, double, false, true);
      if (DIM > 1 && d == 1) FUSED_LAUNCH(D1, double, false, true);
      if (DIM > 2 && d == 2) FUSED_LAUNCH(D2, double, false, true);
    } else if (c->precision == 0) {
      if (d == 0) FUSED_LAUNCH(0, double, false, false);
      if (DIM > 1 && d == 1) FUSED_LAUNCH(D1, double, false, false);
      if (DIM > 2 && d == 2) FUSED_LAUNCH(D2, double, false, false);
    } else {
      if (d == 0) FUSED_LAUNCH(0, float, false, false);
      if (DIM > 1 && d == 1) FUSED_LAUNCH(D1, float, false, false);
      if (DIM > 2 && d == 2) FUSED_LAUNCH(D2, float, false, false);
    }
#undef FUSED_LAUNCH
    prof_end(c, _id, 1 + d, s);
    off += c->nf[d];
  }
}

// dst = src over n doubles (the last stage's result into the state).
__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ src, double* __restrict__ dst, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <int NS, int DIM>
static void launch_update(mpmc_ctx* c, const double* Un, const double* Uk, double rk0, double rk1,
                          double rk2, double* Uout, double* Lout, hipStream_t s) {
  const int bs = 256;
  TIMED(c, 4, s,
        hipLaunchKernelGGL((k_update<NS, DIM>), dim3(nblocks(c->p.ncell, bs)), dim3(bs), 0, s, c->p, Un,
                           Uk, c->F[0], c->F[1], c->F[2], c->dtg, rk0, rk1, rk2, Uout, Lout));
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free conservation sum (mpmc_conserve_sum_static):
// the per-block partial sums, kSumBlocks blocks x at most kSumMaxVars
// variables, in a file-scope device array.  Every device the library runs on
// holds its own copy until the process ends; host code never uses the
// array's name, only its device address, fetched once per device (with that
// device current) by mpmc_init.
// ---------------------------------------------------------------------------
constexpr int kSumBlocks = 1024, kSumMaxVars = 8, kMaxDevices = 64;
static __device__ __align__(256) double scratch[kSumBlocks * kSumMaxVars];
static double* g_scratch[kMaxDevices] = {nullptr};
static std::mutex g_scratch_mu;

// Device address of this device's scratch array (looked up on first use on
// the device; dev must be current).  nullptr on failure.
static double* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[dev] = (double*)ptr;
  }
  return g_scratch[dev];
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int mpmc_init(const mpmc_grid* g, const mpmc_eos* e, const mpmc_opts* o, mpmc_ctx** out) {
  if (!g || !e || !o || !out) return MPMC_EINVAL;
  *out = nullptr;
  Params p;
  const int st = build_params(g, e, o, p);
  if (st != MPMC_OK) return st;
  mpmc_ctx* c = new (std::nothrow) mpmc_ctx;
  if (!c) return MPMC_ENOMEM;
  c->p = p;
  c->ns = p.ns;
  c->dim = p.dim;
  c->nv = p.nv;
  c->precision = o->precision;
  c->split = o->step_layout != 2;
  long ms = 0;
  for (int d = 0; d < p.dim; ++d) {
    long f = 1;
    for (int k = 0; k < 3; ++k) f *= p.n[k] + (k == d ? 1 : 0);
    c->nf[d] = f;
    ms += f;
  }
  c->masksize = ms;
  c->nblk_sum = kSumBlocks;
  if (hipGetDevice(&c->device) != hipSuccess || !scratch_of(c->device)) {
    delete c;
    return MPMC_EHIP;
  }
  bool ok = true;
  ok = ok && hipMalloc(&c->Q, sizeof(double) * p.nq * p.ncell) == hipSuccess;
  for (int d = 0; d < p.dim; ++d) ok = ok && hipMalloc(&c->F[d], sizeof(double) * p.nv * c->nf[d]) == hipSuccess;
  ok = ok && hipMalloc(&c->S1, sizeof(double) * p.nv * p.ncell) == hipSuccess;
  ok = ok && hipMalloc(&c->S2, sizeof(double) * p.nv * p.ncell) == hipSuccess;
  ok = ok && hipMalloc(&c->dtg, sizeof(double) * 2) == hipSuccess;
  ok = ok && hipMalloc(&c->rates, sizeof(unsigned long long) * kRateWords) == hipSuccess;
  ok = ok && hipMalloc(&c->cnt, sizeof(unsigned long long) * kCntWords) == hipSuccess;
  ok = ok && hipMalloc(&c->partial, sizeof(double) * p.nv * c->nblk_sum) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->hflag, sizeof(unsigned), hipHostMallocMapped) == hipSuccess;
  if (ok) ok = hipHostGetDevicePointer((void**)&c->dflag, c->hflag, 0) == hipSuccess;
  if (ok) *(volatile unsigned*)c->hflag = 0u;
  if (ok) ok = hipMemset(c->cnt, 0, sizeof(unsigned long long) * kCntWords) == hipSuccess;
  if (ok) ok = hipMemset(c->dtg, 0, sizeof(double) * 2) == hipSuccess;
  if (ok) ok = hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    mpmc_free(c);
    return MPMC_ENOMEM;
  }
  // make the kernel variants of this configuration resident
  *out = c;
  return MPMC_OK;
}

extern "C" int mpmc_free(mpmc_ctx* c) {
  if (!c) return MPMC_EINVAL;
  (void)hipDeviceSynchronize();
  (void)hipFree(c->Q);
  for (int d = 0; d < 3; ++d) (void)hipFree(c->F[d]);
  (void)hipFree(c->S1);
  (void)hipFree(c->S2);
  (void)hipFree(c->dtg);
  (void)hipFree(c->rates);
  (void)hipFree(c->cnt);
  (void)hipFree(c->partial);
  (void)hipFree(c->frec);
  (void)hipFree(c->fmid);
  (void)hipFree(c->fmid2);
  if (c->s2) (void)hipStreamDestroy(c->s2);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  (void)hipFree(c->lam2);
  (void)hipFree(c->lam1);
  (void)hipFree(c->amask);
  (void)hipFree(c->held_idx);
  (void)hipFree(c->held_U);
  if (c->hflag) (void)hipHostFree(c->hflag);
  for (auto& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  delete c;
  return MPMC_OK;
}

extern "C" long mpmc_mask_size(const mpmc_ctx* c) { return c ? c->masksize : -1; }

extern "C" int mpmc_init_state(mpmc_ctx* c, const double* phi, const double* y, const double* P,
                               const double* T, const double* vel, double* U, void* stream) {
  if (!c || !phi || !y || !P || !T || !vel || !U) return MPMC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH_WIDE(c, hipLaunchKernelGGL((k_init_state<NS, DIM>), dim3(nblocks(c->p.ncell, 256)), dim3(256), 0, s,
                                 c->p, phi, y, P, T, vel, U));
  return enqueue_status(c);
}

template <int NS, int DIM>
static void compute_dt_impl(mpmc_ctx* c, const double* U, double* dt_out, double* g_out,
                            hipStream_t s) {
  launch_cell<NS, DIM>(c, U, true, s);
  hipLaunchKernelGGL(k_dt_finish, dim3(1), dim3(1), 0, s, c->p.cfl, c->p.gscale, c->rates, c->dtg,
                     (const double*)nullptr, (const double*)nullptr, dt_out, g_out);
}

extern "C" int mpmc_compute_dt(mpmc_ctx* c, const double* U, double* dt_dev, double* gamma_dev,
                               void* stream) {
  if (!c || !U) return MPMC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH_WIDE(c, compute_dt_impl<NS, DIM>(c, U, dt_dev, gamma_dev, s));
  return enqueue_status(c);
}

extern "C" int mpmc_rhs(mpmc_ctx* c, const double* Uk, const double* Un, double rk0, double rk1,
                        double rk2, const double* dt_dev, const double* gamma_dev, double* L,
                        uint16_t* mask, void* stream) {
  if (!c || !Uk || !Un || !dt_dev || !gamma_dev || !L) return MPMC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  hipLaunchKernelGGL(k_set_dtg, dim3(1), dim3(1), 0, s, c->dtg, dt_dev, gamma_dev);
  DISPATCH_WIDE(c, {
    launch_cell<NS, DIM>(c, Uk, false, s, true);
    launch_faces<NS, DIM>(c, Uk, Un, rk0, rk1, rk2, mask, s);
    launch_update<NS, DIM>(c, Un, Uk, rk0, rk1, rk2, nullptr, L, s);
  });
  return enqueue_status(c);
}

// Set the held inflow cells of U back to their values (one thread per held
// cell; the indices were checked against the grid when they were set).
__global__ void k_hold(double* __restrict__ U, long ncell, int nv, long nheld, const long* __restrict__ idx,
                       const double* __restrict__ vals) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= nheld) return;
  const long i = idx[k];
  for (int v = 0; v < nv; ++v) U[v * ncell + i] = vals[v * nheld + k];
}

static void launch_hold(mpmc_ctx* c, double* U, hipStream_t s) {
  if (c->nheld == 0) return;
  TIMED(c, 5, s,
        hipLaunchKernelGGL(k_hold, dim3(nblocks(c->nheld, 256)), dim3(256), 0, s, U, c->p.ncell, c->nv, c->nheld,
                           c->held_idx, c->held_U));
}

static const double kRK[3][3] = {{0.0, 1.0, 1.0}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};

template <int NS, int DIM>
static void rk3_impl(mpmc_ctx* c, double* U, const double* dt_in, const double* g_in, double* dt_out,
                     double* g_out, uint16_t* masks, hipStream_t s, const uint16_t* mrep = nullptr,
                     double* s1_out = nullptr, double* s2_out = nullptr) {
  // stage 1 (U^k = U^n = U): equilibrium of U^n also yields dt and Gamma
  const bool need_rates = !(dt_in && g_in);
  launch_cell<NS, DIM>(c, U, need_rates, s, true);
  TIMED(c, 5, s,
        hipLaunchKernelGGL(k_dt_finish, dim3(1), dim3(1), 0, s, c->p.cfl, c->p.gscale,
                           need_rates ? c->rates : nullptr, c->dtg, dt_in, g_in, dt_out, g_out));
  const double* Uk = U;
  double* outs[3] = {s1_out ? s1_out : c->S1, s2_out ? s2_out : c->S2, U};
  for (int st = 0; st < 3; ++st) {
    if (st > 0) launch_cell<NS, DIM>(c, Uk, false, s, true);
    // split layout: face flux arrays, then the combination pass (the only
    // layout built above kFullNS components; mpmc_init keeps such contexts
    // there)
    if (c->split || NS > kFullNS) {
      launch_faces<NS, DIM>(c, Uk, U, kRK[st][0], kRK[st][1], kRK[st][2],
                            masks ? masks + st * c->masksize : nullptr, s, true,
                            mrep ? mrep + st * c->masksize : nullptr);
      launch_update<NS, DIM>(c, U, Uk, kRK[st][0], kRK[st][1], kRK[st][2], outs[st], nullptr, s);
    } else if constexpr (NS <= kFullNS) {
      // fused sweeps; the last stage combines into the free stage buffer S1
      // (U is still U^n for the other cells' limiter tests) and is copied
      double* acc = st < 2 ? outs[st] : c->S1;
      launch_faces_fused<NS, DIM>(c, Uk, U, kRK[st][0], kRK[st][1], kRK[st][2], acc,
                                  masks ? masks + st * c->masksize : nullptr, s,
                                  mrep ? mrep + st * c->masksize : nullptr);
      if (st == 2) {
        const long nd = (long)c->nv * c->p.ncell;
        TIMED(c, 4, s, hipLaunchKernelGGL(k_copy, dim3(nblocks(nd, 256) < 65536 ? nblocks(nd, 256) : 65536),
                                          dim3(256), 0, s, (const double*)c->S1, U, nd));
      }
    }
    launch_hold(c, outs[st], s);
    Uk = outs[st];
  }
}

extern "C" int mpmc_rk3_step(mpmc_ctx* c, double* U, const double* dt_in, const double* g_in,
                             double* dt_out, double* g_out, uint16_t* masks, void* stream) {
  if (!c || !U) return MPMC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH_WIDE(c, rk3_impl<NS, DIM>(c, U, dt_in, g_in, dt_out, g_out, masks, s));
  return enqueue_status(c);
}

extern "C" int mpmc_rk3_step_replay(mpmc_ctx* c, double* U, const double* dt_dev, const double* gamma_dev,
                                    const uint16_t* masks_in, void* stream) {
  if (!c || !U || !dt_dev || !gamma_dev || !masks_in) return MPMC_EINVAL;
  if (c->precision != 0 || c->p.scheme != 0 || c->p.basis != 0 || c->p.pgen) return MPMC_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH(c, rk3_impl<NS, DIM>(c, U, dt_dev, gamma_dev, nullptr, nullptr, nullptr, s, masks_in));
  return enqueue_status(c);
}

extern "C" int mpmc_rk3_step_stages(mpmc_ctx* c, double* U, const double* dt_dev, const double* gamma_dev,
                                    double* stage1_out, double* stage2_out, uint16_t* masks_out,
                                    void* stream) {
  if (!c || !U || !dt_dev || !gamma_dev || !stage1_out || !stage2_out || !masks_out) return MPMC_EINVAL;
  if (stage1_out == U || stage2_out == U || stage1_out == stage2_out) return MPMC_EINVAL;
  if (c->precision != 0) return MPMC_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH(c, rk3_impl<NS, DIM>(c, U, dt_dev, gamma_dev, nullptr, nullptr, masks_out, s, nullptr, stage1_out,
                                stage2_out));
  return enqueue_status(c);
}

// Any characteristic boundary (type 3) in the context.
static bool has_characteristic(const mpmc_ctx* c) {
  for (int d = 0; d < c->p.dim; ++d)
    if (c->p.bclo[d] == 3 || c->p.bchi[d] == 3) return true;
  return false;
}

extern "C" int mpmc_set_boundary_target(mpmc_ctx* c, int d, int side, double P, double T, const double* Y,
                                        const double* vel, double sigma) {
  if (!c || !Y || !vel || d < 0 || d >= c->p.dim || (side != 0 && side != 1)) return MPMC_EINVAL;
  if ((side == 0 ? c->p.bclo[d] : c->p.bchi[d]) != 3) return MPMC_EINVAL;
  if (!(sigma >= 0.0 && sigma <= 1.0) || !(T > 0.0) || !std::isfinite(P) || !std::isfinite(T)) return MPMC_EINVAL;
  double sy = 0.0;
  for (int k = 0; k < c->ns; ++k) {
    if (!(Y[k] >= 0.0)) return MPMC_EINVAL;
    if (Y[k] > 0.0 && !(P + c->p.pinf[k] > 0.0)) return MPMC_EINVAL;
    sy += Y[k];
  }
  if (std::fabs(sy - 1.0) > 1e-12) return MPMC_EINVAL;
  for (int e = 0; e < c->p.dim; ++e)
    if (!std::isfinite(vel[e])) return MPMC_EINVAL;
  // kernels take the parameter block by value at launch: later launches
  // see the new target
  c->p.tgP[d][side] = P;
  c->p.tgT[d][side] = T;
  for (int k = 0; k < MAXS; ++k) c->p.tgY[d][side][k] = k < c->ns ? Y[k] : 0.0;
  for (int e = 0; e < 3; ++e) c->p.tgV[d][side][e] = e < c->p.dim ? vel[e] : 0.0;
  c->p.tgSig[d][side] = sigma;
  return MPMC_OK;
}

extern "C" int mpmc_set_held_cells(mpmc_ctx* c, long count, const long* idx, const double* values) {
  if (!c || count < 0 || (count > 0 && (!idx || !values))) return MPMC_EINVAL;
  const long n = c->p.ncell;
  std::vector<char> seen(count > 0 ? n : 0, 0);
  for (long k = 0; k < count; ++k) {
    if (idx[k] < 0 || idx[k] >= n || seen[idx[k]]) return MPMC_EINVAL;
    seen[idx[k]] = 1;
  }
  for (long k = 0; k < count; ++k)
    for (int v = 0; v < c->nv; ++v) {
      const double x = values[v * count + k];
      if (!std::isfinite(x) || (v < c->ns && x < 0.0)) return MPMC_EINVAL;
    }
  HIPCHK(hipDeviceSynchronize());
  (void)hipFree(c->held_idx);
  (void)hipFree(c->held_U);
  c->held_idx = nullptr;
  c->held_U = nullptr;
  c->nheld = 0;
  if (count == 0) return MPMC_OK;
  if (hipMalloc(&c->held_idx, sizeof(long) * count) != hipSuccess ||
      hipMalloc(&c->held_U, sizeof(double) * c->nv * count) != hipSuccess) {
    (void)hipFree(c->held_idx);
    c->held_idx = nullptr;
    c->held_U = nullptr;
    return MPMC_ENOMEM;
  }
  HIPCHK(hipMemcpy(c->held_idx, idx, sizeof(long) * count, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->held_U, values, sizeof(double) * c->nv * count, hipMemcpyHostToDevice));
  HIPCHK(hipDeviceSynchronize());
  c->nheld = count;
  return MPMC_OK;
}

extern "C" int mpmc_conserve_sum(mpmc_ctx* c, const double* U, double* sums, void* stream) {
  if (!c || !U || !sums) return MPMC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  hipLaunchKernelGGL(k_sum_partial, dim3(c->nblk_sum, c->nv), dim3(256), 0, s, U, c->p.ncell, c->partial);
  hipLaunchKernelGGL(k_sum_final, dim3(c->nv), dim3(256), 0, s, c->partial, c->nblk_sum, sums);
  return enqueue_status(c);
}

extern "C" int mpmc_conserve_sum_static(mpmc_ctx* c, const double* U, double* sums, void* stream) {
  if (!c || !U || !sums) return MPMC_EINVAL;
  if (c->nv > kSumMaxVars) return MPMC_EINVAL;
  double* part = g_scratch[c->device];  // looked up by mpmc_init on this device
  if (!part) return MPMC_EHIP;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  hipLaunchKernelGGL(k_sum_partial, dim3(kSumBlocks, c->nv), dim3(256), 0, s, U, c->p.ncell, part);
  hipLaunchKernelGGL(k_sum_final, dim3(c->nv), dim3(256), 0, s, (const double*)part, kSumBlocks, sums);
  return enqueue_status(c);
}

extern "C" int mpmc_stats(mpmc_ctx* c, mpmc_stats_t* out, int reset) {
  if (!c || !out) return MPMC_EINVAL;
  HIPCHK(hipStreamSynchronize(c->last));
  std::vector<unsigned long long> slots(kCntWords);
  HIPCHK(hipMemcpy(slots.data(), c->cnt, sizeof(unsigned long long) * kCntWords, hipMemcpyDeviceToHost));
  unsigned long long h[kCntN] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int sl = 0; sl < kCntSlots; ++sl)
    for (int q = 0; q < kCntN; ++q) h[q] += slots[sl * kCntStride + q];
  out->faces_T = h[kCntT];
  out->faces_P = h[kCntP];
  out->fallback = h[kCntFallback];
  out->cdi_drop = h[kCntDrop];
  out->unrecoverable = h[kCntUnrec];
  out->faces = h[kCntFaces];
  out->inadmissible_cells = h[kCntBadCells];
  if (reset) {
    HIPCHK(hipMemset(c->cnt, 0, sizeof(unsigned long long) * kCntWords));
    HIPCHK(hipDeviceSynchronize());
    __atomic_store_n(c->hflag, 0u, __ATOMIC_RELEASE);
  }
  return (h[kCntUnrec] || h[kCntBadCells]) ? MPMC_EINADMISSIBLE : MPMC_OK;
}

// Pull-back of one stage: out = lc + (dL(U^k)/dU^k)^T (coef dt lam).  Q
// must hold the cell quantities of U^k; M is the stage's face-decision mask.
// Every face writes its record, then every cell gathers from the records of
// the faces that reference it (no atomics: the result is reproducible).
template <int NS, int DIM>
static void stage_vjp(mpmc_ctx* c, const double* Uk, const uint16_t* M, const double* lam, double coef,
                      double* out, const LinComb& lc, hipStream_t s, bool use_dt = true) {
  const int bs = 256;
  double* rec[3] = {c->frec, c->frec, c->frec};
  for (int d = 1; d < DIM; ++d) rec[d] = rec[d - 1] + rec_doubles(NS, DIM, c->nf[d - 1]);
  // with DIM > 1 and kernel timing off, the y sweep's pull-back runs on the
  // second stream beside the x and z sweeps' (the records and hand-over
  // buffers are disjoint; the gather waits for both)
  const bool split = DIM > 1 && !c->prof && c->s2;
  if (split) {
    (void)hipEventRecord(c->ev_fork, s);
    (void)hipStreamWaitEvent(c->s2, c->ev_fork, 0);
  }
  long off = 0;
  for (int d = 0; d < DIM; ++d) {
    const unsigned nb = d == 0 ? nblocks(c->nf[d], bs)
                               : (unsigned)(nblocks(c->p.n[0], bs) * (c->nf[d] / c->p.n[0]));
    hipStream_t sd = (split && d == 1) ? c->s2 : s;
    double* mid = (split && d == 1) ? c->fmid2 : c->fmid;
    const int _id = prof_begin(c, sd);
    if (d == 0) {
      hipLaunchKernelGGL((k_face_vjp_a<NS, DIM, 0>), dim3(nb), dim3(bs), 0, sd, c->p, Uk, c->Q, M + off, c->dtg,
                         coef, use_dt, lam, rec[0], mid);
      hipLaunchKernelGGL((k_face_vjp_b<NS, DIM, 0>), dim3(nb), dim3(bs), 0, sd, c->p, Uk, c->Q, mid, rec[0]);
    }
    if (DIM > 1 && d == 1) {
      hipLaunchKernelGGL((k_face_vjp_a<NS, DIM, (DIM > 1 ? 1 : 0)>), dim3(nb), dim3(bs), 0, sd, c->p, Uk, c->Q,
                         M + off, c->dtg, coef, use_dt, lam, rec[1], mid);
      hipLaunchKernelGGL((k_face_vjp_b<NS, DIM, (DIM > 1 ? 1 : 0)>), dim3(nb), dim3(bs), 0, sd, c->p, Uk, c->Q,
                         mid, rec[1]);
    }
    if (DIM > 2 && d == 2) {
      hipLaunchKernelGGL((k_face_vjp_a<NS, DIM, (DIM > 2 ? 2 : 0)>), dim3(nb), dim3(bs), 0, sd, c->p, Uk, c->Q,
                         M + off, c->dtg, coef, use_dt, lam, rec[2], mid);
      hipLaunchKernelGGL((k_face_vjp_b<NS, DIM, (DIM > 2 ? 2 : 0)>), dim3(nb), dim3(bs), 0, sd, c->p, Uk, c->Q,
                         mid, rec[2]);
    }
    prof_end(c, _id, 6, sd);
    off += c->nf[d];
  }
  if (split) {
    (void)hipEventRecord(c->ev_join, c->s2);
    (void)hipStreamWaitEvent(s, c->ev_join, 0);
  }
  TIMED(c, 6, s,
        hipLaunchKernelGGL((k_gather_vjp<NS, DIM>), dim3(nblocks(c->p.ncell, bs)), dim3(bs), 0, s, c->p, Uk,
                           c->Q, rec[0], rec[1], rec[2], M, out, lc));
}

// Discrete adjoint of SSP-RK3 (Eq. SSPRK3) with frozen dt and Gamma:
//   U1 = U + dt L(U),  U2 = 3/4 U + 1/4 (U1 + dt L(U1)),  U3 = 1/3 U + 2/3 (U2 + dt L(U2))
//   lam2 = 2/3 lam3 + J(U2)^T (2/3 dt lam3)
//   lam1 = 1/4 lam2 + J(U1)^T (1/4 dt lam2)
//   lam0 = 1/3 lam3 + 3/4 lam2 + lam1 + J(U)^T (dt lam1)
// Reverse sweep over the stages U^n, U1 = S1, U2 = S2 with stage masks M
// [3][masksize]; dtg must hold dt and Gamma.  q_ready: Q already holds the
// cell quantities of U2.
template <int NS, int DIM>
static void adjoint_reverse(mpmc_ctx* c, const double* Un, const double* S1, const double* S2,
                            const uint16_t* M, const double* lam3, double* lam0, hipStream_t s, bool q_ready) {
  if (!q_ready) launch_cell<NS, DIM>(c, S2, false, s);
  LinComb l2;
  l2.a = kRK[2][1];
  l2.x = lam3;
  stage_vjp<NS, DIM>(c, S2, M + 2 * c->masksize, lam3, kRK[2][2], c->lam2, l2, s);
  launch_cell<NS, DIM>(c, S1, false, s);
  LinComb l1;
  l1.a = kRK[1][1];
  l1.x = c->lam2;
  stage_vjp<NS, DIM>(c, S1, M + c->masksize, c->lam2, kRK[1][2], c->lam1, l1, s);
  launch_cell<NS, DIM>(c, Un, false, s);
  LinComb l0;
  l0.a = kRK[2][0];
  l0.x = lam3;
  l0.b = kRK[1][0];
  l0.y = c->lam2;
  l0.c = 1.0;
  l0.z = c->lam1;
  stage_vjp<NS, DIM>(c, Un, M, c->lam1, kRK[0][2], lam0, l0, s);
}

template <int NS, int DIM>
static void adjoint_impl(mpmc_ctx* c, const double* Un, const double* dt, const double* g, const double* lam3,
                         double* lam0, hipStream_t s) {
  TIMED(c, 5, s, hipLaunchKernelGGL(k_set_dtg, dim3(1), dim3(1), 0, s, c->dtg, dt, g));
  // forward recompute of the stages, recording their face decisions
  const double* Uk = Un;
  double* outs[2] = {c->S1, c->S2};
  for (int st = 0; st < 3; ++st) {
    launch_cell<NS, DIM>(c, Uk, false, s);
    launch_faces<NS, DIM>(c, Uk, Un, kRK[st][0], kRK[st][1], kRK[st][2], c->amask + st * c->masksize, s,
                          false);
    if (st < 2) {
      launch_update<NS, DIM>(c, Un, Uk, kRK[st][0], kRK[st][1], kRK[st][2], outs[st], nullptr, s);
      Uk = outs[st];
    }
  }
  // Q holds the quantities of U2 here
  adjoint_reverse<NS, DIM>(c, Un, c->S1, c->S2, c->amask, lam3, lam0, s, true);
}

template <int NS, int DIM>
static void adjoint_stages_impl(mpmc_ctx* c, const double* Un, const double* S1, const double* S2,
                                const uint16_t* M, const double* dt, const double* g, const double* lam3,
                                double* lam0, hipStream_t s) {
  TIMED(c, 5, s, hipLaunchKernelGGL(k_set_dtg, dim3(1), dim3(1), 0, s, c->dtg, dt, g));
  adjoint_reverse<NS, DIM>(c, Un, S1, S2, M, lam3, lam0, s, false);
}

// Adjoint scratch, allocated on first use (freed by mpmc_free).
static int ensure_adjoint_scratch(mpmc_ctx* c) {
  if (c->frec) return MPMC_OK;
  const long nc = c->p.ncell;
  long nrec = 0;
  for (int d = 0; d < c->p.dim; ++d) nrec += rec_doubles(c->p.ns, c->p.dim, c->nf[d]);
  long nfmax = 0;
  for (int d = 0; d < c->p.dim; ++d) nfmax = c->nf[d] > nfmax ? c->nf[d] : nfmax;
  bool ok = hipMalloc(&c->frec, sizeof(double) * nrec) == hipSuccess;
  ok = ok && hipMalloc(&c->fmid, sizeof(double) * mid_slots(c->p.ns, c->p.dim) * nfmax) == hipSuccess;
  if (c->p.dim > 1) {
    ok = ok && hipMalloc(&c->fmid2, sizeof(double) * mid_slots(c->p.ns, c->p.dim) * c->nf[1]) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipMalloc(&c->lam2, sizeof(double) * c->nv * nc) == hipSuccess;
  ok = ok && hipMalloc(&c->lam1, sizeof(double) * c->nv * nc) == hipSuccess;
  ok = ok && hipMalloc(&c->amask, sizeof(uint16_t) * 3 * c->masksize) == hipSuccess;
  if (!ok) {
    (void)hipFree(c->frec);
    (void)hipFree(c->fmid);
    (void)hipFree(c->fmid2);
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    c->s2 = nullptr;
    c->ev_fork = c->ev_join = nullptr;
    c->fmid2 = nullptr;
    (void)hipFree(c->lam2);
    (void)hipFree(c->lam1);
    (void)hipFree(c->amask);
    c->frec = c->fmid = c->lam2 = c->lam1 = nullptr;
    c->amask = nullptr;
    return MPMC_ENOMEM;
  }
  return MPMC_OK;
}

extern "C" int mpmc_adjoint_step(mpmc_ctx* c, const double* U_n, const double* dt_dev,
                                 const double* gamma_dev, const double* lam_np1, double* lam_n,
                                 void* stream) {
  if (!c || !U_n || !dt_dev || !gamma_dev || !lam_np1 || !lam_n) return MPMC_EINVAL;
  if (lam_n == lam_np1 || lam_n == U_n) return MPMC_EINVAL;
  if (c->ns > kFullNS || c->precision != 0 || c->p.visc || c->p.scheme != 0 || c->p.basis != 0 || c->p.pgen ||
      c->nheld || has_characteristic(c))
    return MPMC_EUNSUPPORTED;
  const int r = ensure_adjoint_scratch(c);
  if (r != MPMC_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH(c, adjoint_impl<NS, DIM>(c, U_n, dt_dev, gamma_dev, lam_np1, lam_n, s));
  return enqueue_status(c);
}

extern "C" int mpmc_adjoint_step_stages(mpmc_ctx* c, const double* U_n, const double* stage1,
                                        const double* stage2, const uint16_t* masks, const double* dt_dev,
                                        const double* gamma_dev, const double* lam_np1, double* lam_n,
                                        void* stream) {
  if (!c || !U_n || !stage1 || !stage2 || !masks || !dt_dev || !gamma_dev || !lam_np1 || !lam_n)
    return MPMC_EINVAL;
  if (lam_n == lam_np1 || lam_n == U_n || lam_n == stage1 || lam_n == stage2) return MPMC_EINVAL;
  if (c->ns > kFullNS || c->precision != 0 || c->p.visc || c->p.scheme != 0 || c->p.basis != 0 || c->p.pgen ||
      c->nheld || has_characteristic(c))
    return MPMC_EUNSUPPORTED;
  const int r = ensure_adjoint_scratch(c);
  if (r != MPMC_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH(c, adjoint_stages_impl<NS, DIM>(c, U_n, stage1, stage2, masks, dt_dev, gamma_dev, lam_np1, lam_n, s));
  return enqueue_status(c);
}

template <int NS, int DIM>
static void rhs_vjp_impl(mpmc_ctx* c, const double* Uk, const uint16_t* mask, const double* dt,
                         const double* g, const double* Lbar, double* Ubar, hipStream_t s) {
  TIMED(c, 5, s, hipLaunchKernelGGL(k_set_dtg, dim3(1), dim3(1), 0, s, c->dtg, dt, g));
  launch_cell<NS, DIM>(c, Uk, false, s);
  stage_vjp<NS, DIM>(c, Uk, mask, Lbar, 1.0, Ubar, LinComb(), s, false);
}

extern "C" int mpmc_rhs_vjp(mpmc_ctx* c, const double* Uk, const uint16_t* mask, const double* dt_dev,
                            const double* gamma_dev, const double* Lbar, double* Ubar, void* stream) {
  if (!c || !Uk || !mask || !dt_dev || !gamma_dev || !Lbar || !Ubar) return MPMC_EINVAL;
  if (Ubar == Lbar || Ubar == Uk) return MPMC_EINVAL;
  if (c->ns > kFullNS || c->precision != 0 || c->p.visc || c->p.scheme != 0 || c->p.basis != 0 || c->p.pgen ||
      c->nheld || has_characteristic(c))
    return MPMC_EUNSUPPORTED;
  const int r = ensure_adjoint_scratch(c);
  if (r != MPMC_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  c->last = s;
  DISPATCH(c, rhs_vjp_impl<NS, DIM>(c, Uk, mask, dt_dev, gamma_dev, Lbar, Ubar, s));
  return enqueue_status(c);
}

extern "C" int mpmc_profile(mpmc_ctx* c, int enable) {
  if (!c) return MPMC_EINVAL;
  if (!enable) {
    const int r = prof_flush(c);
    c->prof = false;
    return r;
  }
  c->prof = true;
  return MPMC_OK;
}

extern "C" int mpmc_profile_read(mpmc_ctx* c, double* ms, long* launches, int reset) {
  if (!c || !ms || !launches) return MPMC_EINVAL;
  const int r = prof_flush(c);
  if (r != MPMC_OK) return r;
  for (int i = 0; i < 8; ++i) {
    ms[i] = c->prof_ms[i];
    launches[i] = c->prof_n[i];
    if (reset) {
      c->prof_ms[i] = 0.0;
      c->prof_n[i] = 0;
    }
  }
  return MPMC_OK;
}
