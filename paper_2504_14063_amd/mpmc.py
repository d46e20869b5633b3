"""Python binding of libmpmc.so (include/mpmc.h): argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts torch
device tensors and streams to raw pointers and back.  There is no CPU path: if
the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpmc.so")

MPMC_OK, MPMC_EINVAL, MPMC_ENOMEM, MPMC_EHIP, MPMC_EINADMISSIBLE, MPMC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
M_TL, M_TR, M_PL, M_PR, M_FALLBACK, M_CDI_DROP, M_UNRECOVERABLE = 1, 2, 4, 8, 16, 32, 64


class mpmc_grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3),
                ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3)]


class mpmc_eos(C.Structure):
    _fields_ = [("n_species", C.c_int), ("phase", C.c_int * 8), ("cv", C.c_double * 8),
                ("gamma", C.c_double * 8), ("pinf", C.c_double * 8), ("b", C.c_double * 8),
                ("q", C.c_double * 8), ("molar_mass", C.c_double * 8), ("mu", C.c_double * 8),
                ("Sc", C.c_double * 8), ("lambda", C.c_double * 8)]


class mpmc_opts(C.Structure):
    _fields_ = [("cfl", C.c_double), ("cdi", C.c_int), ("eps_cdi", C.c_double),
                ("phi_min", C.c_double), ("delta", C.c_double), ("gamma_scale", C.c_double),
                ("diffusion", C.c_int), ("positivity", C.c_int), ("precision", C.c_int),
                ("weno", C.c_int), ("weno_eps", C.c_double), ("weno_p", C.c_int),
                ("viscous", C.c_int), ("prandtl", C.c_double), ("basis", C.c_int),
                ("step_layout", C.c_int)]


class mpmc_stats_t(C.Structure):
    _fields_ = [("faces_T", C.c_uint64), ("faces_P", C.c_uint64), ("fallback", C.c_uint64),
                ("cdi_drop", C.c_uint64), ("unrecoverable", C.c_uint64), ("faces", C.c_uint64),
                ("inadmissible_cells", C.c_uint64)]


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
    """Load libmpmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2504_14063_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, D, V = C.c_void_p, C.c_void_p, C.c_void_p
        L.mpmc_init.argtypes = [C.POINTER(mpmc_grid), C.POINTER(mpmc_eos), C.POINTER(mpmc_opts),
                                C.POINTER(C.c_void_p)]
        L.mpmc_free.argtypes = [P]
        L.mpmc_mask_size.restype = C.c_long
        L.mpmc_mask_size.argtypes = [P]
        L.mpmc_init_state.argtypes = [P, D, D, D, D, D, D, V]
        L.mpmc_compute_dt.argtypes = [P, D, D, D, V]
        L.mpmc_rhs.argtypes = [P, D, D, C.c_double, C.c_double, C.c_double, D, D, D, V, V]
        L.mpmc_rk3_step.argtypes = [P, D, D, D, D, D, V, V]
        L.mpmc_adjoint_step.argtypes = [P, D, D, D, D, D, V]
        L.mpmc_rhs_vjp.argtypes = [P, D, V, D, D, D, D, V]
        L.mpmc_rk3_step_replay.argtypes = [P, D, D, D, V, V]
        L.mpmc_rk3_step_stages.argtypes = [P, D, D, D, D, D, V, V]
        L.mpmc_adjoint_step_stages.argtypes = [P, D, D, D, V, D, D, D, D, V]
        L.mpmc_conserve_sum.argtypes = [P, D, D, V]
        L.mpmc_conserve_sum_static.argtypes = [P, D, D, V]
        L.mpmc_set_held_cells.argtypes = [P, C.c_long, C.POINTER(C.c_long), C.POINTER(C.c_double)]
        L.mpmc_set_boundary_target.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_double, C.POINTER(C.c_double),
                                               C.POINTER(C.c_double), C.c_double]
        L.mpmc_stats.argtypes = [P, C.POINTER(mpmc_stats_t), C.c_int]
        L.mpmc_profile.argtypes = [P, C.c_int]
        L.mpmc_profile_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_long), C.c_int]
        L.mpmc_strerror.restype = C.c_char_p
        L.mpmc_strerror.argtypes = [C.c_int]
        _lib = L
    return _lib


class MpmcError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {lib().mpmc_strerror(code).decode()} ({code})")
        self.code = code


class Inadmissible(MpmcError):
    """MPMC_EINADMISSIBLE from a call that enqueued work: kernels of earlier
    calls met an inadmissible cell or an unrecoverable face (the call's own
    work was enqueued)."""


def _chk(code, where):
    if code == MPMC_EINADMISSIBLE:
        raise Inadmissible(code, where)
    if code != MPMC_OK:
        raise MpmcError(code, where)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """An mpmc_ctx: one grid, component table and option set."""

    def __init__(self, grid: dict, eos: dict, opts: dict, raise_inadmissible=True):
        """raise_inadmissible: raise Inadmissible when a call reports an
        inadmissible cell or unrecoverable face met by earlier kernels; when
        False such reports are counted in self.inadmissible_reports (runs that
        tolerate them; mpmc_stats has the totals)."""
        self.raise_inadmissible = raise_inadmissible
        self.inadmissible_reports = 0
        self.grid, self.eos, self.opts = grid, eos, dict(opts)
        self._g, self._e, self._o = _fill(mpmc_grid, grid), _fill(mpmc_eos, eos), _fill(mpmc_opts, opts)
        h = C.c_void_p()
        _chk(lib().mpmc_init(C.byref(self._g), C.byref(self._e), C.byref(self._o), C.byref(h)), "mpmc_init")
        self.h = h
        self.dim = grid["dim"]
        self.n = [grid["n"][d] if d < self.dim else 1 for d in range(3)]
        self.ns = eos["n_species"]
        self.nv = self.ns + self.dim + 1
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        self.mask_size = lib().mpmc_mask_size(self.h)
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self._setters = []  # (method name, args) of the calls that configure it
        self._twin = None

    @classmethod
    def from_case(cls, case, raise_inadmissible=True, **opt_overrides):
        """A context for the case; the targets of its characteristic
        boundaries (case.extra['boundary_targets']) are set."""
        o = dict(case.opts)
        o.update(opt_overrides)
        c = cls(case.grid_dict(), case.eos_dict(), o, raise_inadmissible=raise_inadmissible)
        for t in case.extra.get("boundary_targets", ()):
            c.mpmc_set_boundary_target(*t)
        return c

    def _chk(self, code, where):
        if code == MPMC_EINADMISSIBLE and not self.raise_inadmissible:
            self.inadmissible_reports += 1
            return
        _chk(code, where)

    def close(self):
        if getattr(self, "_twin", None) is not None:
            self._twin.close()
            self._twin = None
        if getattr(self, "h", None):
            lib().mpmc_free(self.h)
            self.h = None

    def twin(self):
        """A second context with the same grid, components, options, boundary
        targets and held cells (its own scratch), created on first use and
        closed with this one: work that runs beside this context's on
        another stream (the rollout recomputes the next segment with it
        while the adjoint sweeps the current one)."""
        if self._twin is None:
            t = Context(self.grid, self.eos, self.opts, raise_inadmissible=self.raise_inadmissible)
            for name, args in self._setters:
                getattr(t, name)(*args)
            self._twin = t
        return self._twin

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tensors ---------------------------------------------------------
    def empty_state(self):
        return torch.empty(self.nv * self.ncell, dtype=torch.float64, device=self.dev)

    def scalar(self, value=None):
        t = torch.zeros(1, dtype=torch.float64, device=self.dev)
        if value is not None:
            t.fill_(float(value))
        return t

    # -- ABI calls ---------------------------------------------------------
    def mpmc_init_state(self, phi, y, P, T, vel, U=None, stream=None):
        U = self.empty_state() if U is None else U
        self._chk(lib().mpmc_init_state(self.h, _ptr(phi), _ptr(y), _ptr(P), _ptr(T), _ptr(vel), _ptr(U),
                                   _stream(stream)), "mpmc_init_state")
        return U

    def init_state_from_case(self, case, stream=None):
        dev = self.dev
        t = lambda a: torch.from_numpy(a).to(dev)
        phi, y, P, T, vel = case.prim_arrays()
        return self.mpmc_init_state(t(phi), t(y), t(P), t(T), t(vel), stream=stream)

    def mpmc_compute_dt(self, U, stream=None):
        dt, g = self.scalar(), self.scalar()
        self._chk(lib().mpmc_compute_dt(self.h, _ptr(U), _ptr(dt), _ptr(g), _stream(stream)), "mpmc_compute_dt")
        return dt, g

    def mpmc_rhs(self, Uk, Un, rk, dt, gamma, L=None, mask=None, stream=None):
        L = torch.empty_like(Uk) if L is None else L
        self._chk(lib().mpmc_rhs(self.h, _ptr(Uk), _ptr(Un), float(rk[0]), float(rk[1]), float(rk[2]),
                            _ptr(dt), _ptr(gamma), _ptr(L), _ptr(mask), _stream(stream)), "mpmc_rhs")
        return L

    def mpmc_rk3_step(self, U, dt_in=None, gamma_in=None, dt_out=None, gamma_out=None, masks=None,
                      stream=None):
        self._chk(lib().mpmc_rk3_step(self.h, _ptr(U), _ptr(dt_in), _ptr(gamma_in), _ptr(dt_out),
                                 _ptr(gamma_out), _ptr(masks), _stream(stream)), "mpmc_rk3_step")
        return U

    def mpmc_rk3_step_replay(self, U, dt, gamma, masks_in, stream=None):
        self._chk(lib().mpmc_rk3_step_replay(self.h, _ptr(U), _ptr(dt), _ptr(gamma), _ptr(masks_in), _stream(stream)),
             "mpmc_rk3_step_replay")
        return U

    def mpmc_rk3_step_stages(self, U, dt, gamma, stage1, stage2, masks, stream=None):
        self._chk(lib().mpmc_rk3_step_stages(self.h, _ptr(U), _ptr(dt), _ptr(gamma), _ptr(stage1), _ptr(stage2),
                                        _ptr(masks), _stream(stream)), "mpmc_rk3_step_stages")
        return U

    def mpmc_adjoint_step_stages(self, U_n, stage1, stage2, masks, dt, gamma, lam_np1, lam_n=None,
                                 stream=None):
        lam_n = torch.empty_like(lam_np1) if lam_n is None else lam_n
        self._chk(lib().mpmc_adjoint_step_stages(self.h, _ptr(U_n), _ptr(stage1), _ptr(stage2), _ptr(masks),
                                            _ptr(dt), _ptr(gamma), _ptr(lam_np1), _ptr(lam_n),
                                            _stream(stream)), "mpmc_adjoint_step_stages")
        return lam_n

    def mpmc_adjoint_step(self, U_n, dt, gamma, lam_np1, lam_n=None, stream=None):
        lam_n = torch.empty_like(lam_np1) if lam_n is None else lam_n
        self._chk(lib().mpmc_adjoint_step(self.h, _ptr(U_n), _ptr(dt), _ptr(gamma), _ptr(lam_np1),
                                     _ptr(lam_n), _stream(stream)), "mpmc_adjoint_step")
        return lam_n

    def mpmc_rhs_vjp(self, Uk, mask, dt, gamma, Lbar, Ubar=None, stream=None):
        Ubar = torch.empty_like(Lbar) if Ubar is None else Ubar
        self._chk(lib().mpmc_rhs_vjp(self.h, _ptr(Uk), _ptr(mask), _ptr(dt), _ptr(gamma), _ptr(Lbar), _ptr(Ubar),
                                _stream(stream)), "mpmc_rhs_vjp")
        return Ubar

    def mpmc_set_boundary_target(self, d, side, P, T, Y, vel, sigma):
        """Target state (P, T, Y[ns], vel[dim]) and relaxation factor sigma of
        the characteristic boundary on side (0 low, 1 high) of direction d."""
        self._setters.append(("mpmc_set_boundary_target", (d, side, P, T, Y, vel, sigma)))
        Yv = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(-1))
        vv = np.ascontiguousarray(np.asarray(list(vel) + [0.0] * (3 - len(vel)), dtype=np.float64))
        self._chk(lib().mpmc_set_boundary_target(self.h, int(d), int(side), float(P), float(T),
                                                 Yv.ctypes.data_as(C.POINTER(C.c_double)),
                                                 vv.ctypes.data_as(C.POINTER(C.c_double)), float(sigma)),
                  "mpmc_set_boundary_target")

    def mpmc_set_held_cells(self, idx, values):
        """Hold the cells idx (host int64 [count]) at the conserved values
        (host float64 [nv][count]) through every RK stage; empty idx clears."""
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1))
        vals = np.ascontiguousarray(np.asarray(values, dtype=np.float64).reshape(self.nv, len(idx)))
        self._setters.append(("mpmc_set_held_cells", (idx.copy(), vals.copy())))
        self._chk(lib().mpmc_set_held_cells(self.h, len(idx), idx.ctypes.data_as(C.POINTER(C.c_long)),
                                       vals.ctypes.data_as(C.POINTER(C.c_double))), "mpmc_set_held_cells")

    def mpmc_conserve_sum(self, U, stream=None):
        out = torch.zeros(self.nv, dtype=torch.float64, device=self.dev)
        self._chk(lib().mpmc_conserve_sum(self.h, _ptr(U), _ptr(out), _stream(stream)), "mpmc_conserve_sum")
        return out

    def mpmc_conserve_sum_static(self, U, out=None, stream=None):
        """mpmc_conserve_sum without allocation in the library: the partial
        sums live in the library's fixed per-device scratch; out (optional)
        is a caller-provided device tensor of nv doubles."""
        out = torch.zeros(self.nv, dtype=torch.float64, device=self.dev) if out is None else out
        self._chk(lib().mpmc_conserve_sum_static(self.h, _ptr(U), _ptr(out), _stream(stream)),
                  "mpmc_conserve_sum_static")
        return out

    def mpmc_stats(self, reset=False):
        s = mpmc_stats_t()
        code = lib().mpmc_stats(self.h, C.byref(s), 1 if reset else 0)
        if code not in (MPMC_OK, MPMC_EINADMISSIBLE):
            _chk(code, "mpmc_stats")
        return dict(faces_T=s.faces_T, faces_P=s.faces_P, fallback=s.fallback, cdi_drop=s.cdi_drop,
                    unrecoverable=s.unrecoverable, faces=s.faces,
                    inadmissible_cells=s.inadmissible_cells, code=code)

    def mpmc_profile(self, enable=True):
        self._chk(lib().mpmc_profile(self.h, 1 if enable else 0), "mpmc_profile")

    KERNEL_CLASSES = ("cell", "face_x", "face_y", "face_z", "update", "small", "adjoint", "spare")

    def mpmc_profile_read(self, reset=False):
        ms = (C.c_double * 8)()
        n = (C.c_long * 8)()
        self._chk(lib().mpmc_profile_read(self.h, ms, n, 1 if reset else 0), "mpmc_profile_read")
        return {k: (ms[i], n[i]) for i, k in enumerate(self.KERNEL_CLASSES)}

    def new_masks(self):
        return torch.zeros(3 * self.mask_size, dtype=torch.int16, device=self.dev)
