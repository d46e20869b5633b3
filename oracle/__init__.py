"""ctypes shim of the CPU oracle (test infrastructure only).

The oracle is a plain FP64 C++ implementation of the finite-volume step of the
four-equation multi-phase multi-component method (arXiv 2504.14063).  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may use
it; the GPU library neither imports nor links it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.cpp")

NCNT = 7
(ORACLE_CNT_T, ORACLE_CNT_P, ORACLE_CNT_FALLBACK, ORACLE_CNT_CDI_DROP, ORACLE_CNT_UNRECOVERABLE,
 ORACLE_CNT_FACES, ORACLE_CNT_BAD_CELLS) = range(7)
EINADMISSIBLE = -4
M_TL, M_TR, M_PL, M_PR, M_FALLBACK, M_CDI_DROP, M_UNRECOVERABLE = 1, 2, 4, 8, 16, 32, 64


def build(verbose=False):
    """Compile liboracle.so with g++ (FP64, no FMA contraction, OpenMP)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", LIB_PATH + ".tmp", SRC]
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    if verbose:
        print("built", LIB_PATH)


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3),
                ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3)]


class Eos(C.Structure):
    _fields_ = [("n_species", C.c_int), ("phase", C.c_int * 8), ("cv", C.c_double * 8),
                ("gamma", C.c_double * 8), ("pinf", C.c_double * 8), ("b", C.c_double * 8),
                ("q", C.c_double * 8), ("molar_mass", C.c_double * 8), ("mu", C.c_double * 8),
                ("Sc", C.c_double * 8), ("lambda", C.c_double * 8)]


class Opts(C.Structure):
    _fields_ = [("cfl", C.c_double), ("cdi", C.c_int), ("eps_cdi", C.c_double),
                ("phi_min", C.c_double), ("delta", C.c_double), ("gamma_scale", C.c_double),
                ("diffusion", C.c_int), ("positivity", C.c_int), ("precision", C.c_int),
                ("weno", C.c_int), ("weno_eps", C.c_double), ("weno_p", C.c_int),
                ("viscous", C.c_int), ("prandtl", C.c_double), ("basis", C.c_int)]


def _fill(struct, d):
    s = struct()
    for name, typ in struct._fields_:
        if name not in d:
            continue
        v = d[name]
        if hasattr(typ, "_length_"):
            arr = getattr(s, name)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(s, name, v)
    return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        D = C.POINTER(C.c_double)
        L.oracle_create.restype = C.c_void_p
        L.oracle_create.argtypes = [C.POINTER(Grid), C.POINTER(Eos), C.POINTER(Opts), C.POINTER(C.c_int)]
        L.oracle_destroy.argtypes = [P]
        L.oracle_init_state.argtypes = [P, D, D, D, D, D, D]
        L.oracle_compute_dt.argtypes = [P, D, D, D]
        L.oracle_rhs.argtypes = [P, D, D, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_double, D, C.POINTER(C.c_uint16), C.POINTER(C.c_uint64)]
        L.oracle_pseudo_states.argtypes = [P, D, D, C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_double, D, D, D, D]
        L.oracle_rk3_step.argtypes = [P, D, D, D, D, D, C.POINTER(C.c_uint16), C.POINTER(C.c_uint64)]
        L.oracle_jvp_rk3_step.argtypes = [P, D, D, C.c_double, C.c_double, D, D]
        L.oracle_set_held.argtypes = [P, C.c_long, C.POINTER(C.c_long), D]
        L.oracle_set_boundary_target.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_double, D, D, C.c_double]
        L.oracle_jvp_rhs.argtypes = [P, D, D, D, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, D, D]
        L.oracle_cell_equilibrium.argtypes = [P, D, D]
        L.oracle_state_from_PT.argtypes = [P, C.c_double, C.c_double, D, D, D, D]
        L.oracle_weno5z.restype = C.c_double
        L.oracle_weno5z.argtypes = [D, C.c_double, C.c_int]
        L.oracle_weno5js.restype = C.c_double
        L.oracle_weno5js.argtypes = [D, C.c_double, C.c_int]
        L.oracle_teno5.restype = C.c_double
        L.oracle_teno5.argtypes = [D, C.c_double]
        L.oracle_teno6.restype = C.c_double
        L.oracle_teno6.argtypes = [D, C.c_double, D]
        L.oracle_js_indicator.restype = C.c_double
        L.oracle_js_indicator.argtypes = [D, C.c_int, C.c_int, D]
        L.oracle_ylimit.argtypes = [C.c_int, D, D]
        L.oracle_hllc.argtypes = [P, D, D, D]
        L.oracle_euler_flux.argtypes = [P, D, D]
        L.oracle_admissible.argtypes = [P, D]
        L.oracle_cell_aux.argtypes = [P, D, D]
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        L.oracle_count_ops.argtypes = [P, D, C.c_double, C.c_double, C.POINTER(C.c_long)]
        L.oracle_wilke.restype = C.c_double
        L.oracle_wilke.argtypes = [P, C.c_int, D]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """One solver instance over a grid, a material table and options."""

    def __init__(self, grid: dict, eos: dict, opts: dict):
        self.grid, self.eos, self.opts = grid, eos, opts
        st = C.c_int(0)
        self._g, self._e, self._o = _fill(Grid, grid), _fill(Eos, eos), _fill(Opts, opts)
        self.h = lib().oracle_create(C.byref(self._g), C.byref(self._e), C.byref(self._o), C.byref(st))
        if not self.h:
            raise ValueError(f"oracle_create failed with status {st.value}")
        self.dim = grid["dim"]
        self.n = [grid["n"][d] if d < self.dim else 1 for d in range(3)]
        self.ns = eos["n_species"]
        self.nv = self.ns + self.dim + 1
        self.ncell = int(np.prod(self.n))
        self.status = 0

    @classmethod
    def from_case(cls, case):
        """An oracle for the case, with the targets of its characteristic
        boundaries (case.extra['boundary_targets']) set."""
        o = cls(case.grid_dict(), case.eos_dict(), case.opts)
        for t in case.extra.get("boundary_targets", ()):
            o.set_boundary_target(*t)
        return o

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None and callable(getattr(_lib, "oracle_destroy", None)):
            try:
                _lib.oracle_destroy(h)
            except Exception:
                pass
            self.h = None

    # --- state helpers
    def face_counts(self):
        out = []
        for d in range(self.dim):
            f = 1
            for k in range(3):
                f *= self.n[k] + (1 if k == d else 0)
            out.append(f)
        return out

    def init_state(self, case):
        phi, y, P, T, vel = case.prim_arrays()
        U = np.zeros(self.nv * self.ncell)
        lib().oracle_init_state(self.h, _dp(phi), _dp(y), _dp(P), _dp(T), _dp(vel), _dp(U))
        return U

    def compute_dt(self, U):
        dt, g = C.c_double(), C.c_double()
        lib().oracle_compute_dt(self.h, _dp(U), C.byref(dt), C.byref(g))
        return dt.value, g.value

    def rhs(self, Uk, Un, rk=(0.0, 1.0, 1.0), dt=0.0, gamma=0.0, with_mask=False):
        L = np.zeros_like(Uk)
        cnt = np.zeros(NCNT, dtype=np.uint64)
        mask = np.zeros(sum(self.face_counts()), dtype=np.uint16) if with_mask else None
        self.status = lib().oracle_rhs(self.h, _dp(Uk), _dp(Un), rk[0], rk[1], rk[2], dt, gamma, _dp(L),
                                       mask.ctypes.data_as(C.POINTER(C.c_uint16)) if mask is not None else None,
                                       cnt.ctypes.data_as(C.POINTER(C.c_uint64)))
        return (L, cnt, mask) if with_mask else L

    def pseudo_states(self, Uk, Un, rk=(0.0, 1.0, 1.0), dt=0.0, gamma=0.0, with_flux=False):
        """(L, lo, hi[, F]): the stage right-hand side and the flux limiter's
        pseudo-states of every interior cell at its low and high face of each
        direction ([dim][nv][cells]), formed with the faces' final fluxes;
        with_flux: also those fluxes, a list over directions of [nv][faces]."""
        L = np.zeros_like(Uk)
        lo = np.zeros(self.dim * self.nv * self.ncell)
        hi = np.zeros_like(lo)
        fc = self.face_counts()
        F = np.zeros(self.nv * sum(fc))
        self.status = lib().oracle_pseudo_states(self.h, _dp(Uk), _dp(Un), rk[0], rk[1], rk[2], dt, gamma,
                                                 _dp(L), _dp(lo), _dp(hi), _dp(F))
        sh = (self.dim, self.nv, self.ncell)
        if not with_flux:
            return L, lo.reshape(sh), hi.reshape(sh)
        out, off = [], 0
        for nf in fc:
            out.append(F[off:off + self.nv * nf].reshape(self.nv, nf))
            off += self.nv * nf
        return L, lo.reshape(sh), hi.reshape(sh), out

    def step(self, U, dt=None, gamma=None, with_mask=False, counters=None):
        """One SSP-RK3 step in place; returns (dt, gamma[, masks]).  The
        call's status (0, or EINADMISSIBLE after an inadmissible stage input
        cell or an unrecoverable face) is left in self.status."""
        dti = C.c_double(dt) if dt is not None else None
        gi = C.c_double(gamma) if gamma is not None else None
        dto, go = C.c_double(), C.c_double()
        cnt = counters if counters is not None else np.zeros(NCNT, dtype=np.uint64)
        masks = np.zeros(3 * sum(self.face_counts()), dtype=np.uint16) if with_mask else None
        self.status = lib().oracle_rk3_step(
            self.h, _dp(U), C.byref(dti) if dti is not None else None,
            C.byref(gi) if gi is not None else None, C.byref(dto), C.byref(go),
            masks.ctypes.data_as(C.POINTER(C.c_uint16)) if masks is not None else None,
            cnt.ctypes.data_as(C.POINTER(C.c_uint64)))
        if with_mask:
            return dto.value, go.value, masks
        return dto.value, go.value

    def set_held(self, idx, U):
        """Hold the cells idx at the conserved values U[v::ncell][idx] of the
        state U through every RK stage of step (the inflow cells of the Mach-100
        water column, Sec. 4.2.4).  An empty idx clears."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= self.ncell):
            raise ValueError("held cells: index out of range")
        vals = np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(self.nv, self.ncell)[:, idx])
        r = lib().oracle_set_held(self.h, len(idx), idx.ctypes.data_as(C.POINTER(C.c_long)), _dp(vals))
        if r != 0:
            raise ValueError("held cells: index out of range or repeated")

    def set_boundary_target(self, d, side, P, T, Y, vel, sigma):
        """Target state (P, T, Y, vel) and relaxation factor sigma of the
        characteristic boundary on side (0 low, 1 high) of direction d."""
        Yv = np.ascontiguousarray(Y, dtype=np.float64)
        vv = np.ascontiguousarray(list(vel) + [0.0] * (3 - len(vel)), dtype=np.float64)
        if lib().oracle_set_boundary_target(self.h, d, side, P, T, _dp(Yv), _dp(vv), sigma) != 0:
            raise ValueError("characteristic boundary target rejected")

    def jvp_step(self, U, dU, dt, gamma):
        Uo = np.zeros_like(U)
        dUo = np.zeros_like(U)
        lib().oracle_jvp_rk3_step(self.h, _dp(U), _dp(dU), dt, gamma, _dp(Uo), _dp(dUo))
        return Uo, dUo

    def jvp_rhs(self, Uk, dUk, Un, rk, dt, gamma):
        """(L(U_k), dL/dU_k [dU_k]) of one stage by complex step."""
        L = np.zeros_like(Uk)
        dL = np.zeros_like(Uk)
        lib().oracle_jvp_rhs(self.h, _dp(Uk), _dp(dUk), _dp(Un), rk[0], rk[1], rk[2], dt, gamma, _dp(L), _dp(dL))
        return L, dL

    # --- pieces
    def equilibrium(self, u):
        out = np.zeros(9)
        lib().oracle_cell_equilibrium(self.h, _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(out))
        return dict(zip(["P", "T", "a", "rho", "beta", "alpha", "cT", "z", "e"], out))

    def state_from_PT(self, P, T, Y, vel):
        u = np.zeros(self.nv)
        a = C.c_double()
        lib().oracle_state_from_PT(self.h, P, T, _dp(np.asarray(Y, dtype=np.float64)),
                                   _dp(np.asarray(list(vel) + [0.0] * 3, dtype=np.float64)),
                                   _dp(u), C.byref(a))
        return u, a.value

    def hllc(self, uL, uR):
        F = np.zeros(self.nv)
        lib().oracle_hllc(self.h, _dp(np.ascontiguousarray(uL, dtype=np.float64)),
                          _dp(np.ascontiguousarray(uR, dtype=np.float64)), _dp(F))
        return F

    def euler_flux(self, u):
        F = np.zeros(self.nv)
        lib().oracle_euler_flux(self.h, _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(F))
        return F

    def admissible(self, u):
        return bool(lib().oracle_admissible(self.h, _dp(np.ascontiguousarray(u, dtype=np.float64))))

    def cell_aux(self, u):
        out = np.zeros(9)
        lib().oracle_cell_aux(self.h, _dp(np.ascontiguousarray(u, dtype=np.float64)), _dp(out))
        return dict(phi=out[0:2], psi=out[2:4], rhop=out[4:6], hrho=out[6:8], mu=out[8])

    def count_ops(self, U, dt, gamma):
        out = (C.c_long * 8)()
        lib().oracle_count_ops(self.h, _dp(U), dt, gamma, out)
        return dict(cell=out[0], face_x=out[1], face_y=out[2], face_z=out[3], divergence=out[4],
                    padded_cells=out[5])

    def wilke(self, phase, y):
        return lib().oracle_wilke(self.h, phase, _dp(np.asarray(y, dtype=np.float64)))


def num_threads():
    return int(lib().oracle_num_threads())


def set_num_threads(n):
    lib().oracle_set_num_threads(int(n))


def weno5z(f, eps=1e-40, p=1):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().oracle_weno5z(_dp(f), eps, p)


def weno5js(f, eps=1e-6, p=2):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().oracle_weno5js(_dp(f), eps, p)


def teno5(f, eps=1e-40):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return lib().oracle_teno5(_dp(f), eps)


def teno6(f, eps=1e-40, with_tau=False):
    """TENO6 face value at i+1/2 from f_{i-2..i+3} (and its reference
    indicator tau6 with with_tau)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert f.size == 6
    tau = np.zeros(1)
    v = lib().oracle_teno6(_dp(f), eps, _dp(tau))
    return (v, float(tau[0])) if with_tau else v


def js_indicator(f, off):
    """(indicator, face value) of the polynomial matching the averages f on
    cells off..off+len(f)-1 around the target cell."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    face = np.zeros(1)
    b = lib().oracle_js_indicator(_dp(f), off, f.size, _dp(face))
    return b, float(face[0])


def ylimit(Ys, Ycell):
    Ys = np.array(Ys, dtype=np.float64)
    Yc = np.ascontiguousarray(Ycell, dtype=np.float64)
    br = lib().oracle_ylimit(len(Ys), _dp(Ys), _dp(Yc))
    return Ys, br
