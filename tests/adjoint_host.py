"""Loader of the host execution of the adjoint's reverse code (test harness)
and the SSP-RK3 pull-back composed from it, with the stage states and the
decision masks supplied by the oracle."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
RK = [(0.0, 1.0, 1.0), (0.75, 0.25, 0.25), (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0)]


def build(outdir):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    so = os.path.join(outdir, "libadj_host.so")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
                           "-o", so, os.path.join(HERE, "adjoint_host.cpp")])
    return so


class HostAdjoint:
    def __init__(self, so, case):
        from paper_2504_14063_amd.mpmc import _fill, mpmc_eos, mpmc_grid, mpmc_opts
        self.lib = C.CDLL(so)
        D = C.POINTER(C.c_double)
        self.lib.emu_stage_vjp.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, D, C.c_void_p, C.c_double,
                                           C.c_double, C.c_double, D, D, C.c_void_p]
        self.g = _fill(mpmc_grid, case.grid_dict())
        self.e = _fill(mpmc_eos, case.eos_dict())
        self.o = _fill(mpmc_opts, dict(case.opts))

    def stage_vjp(self, Uk, mask, dt, g, coef, lam, out, qb=None):
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        mask = np.ascontiguousarray(mask, dtype=np.uint16)
        r = self.lib.emu_stage_vjp(C.byref(self.g), C.byref(self.e), C.byref(self.o), dp(Uk),
                                   mask.ctypes.data_as(C.c_void_p), dt, g, coef, dp(lam), dp(out),
                                   None if qb is None else qb.ctypes.data_as(C.c_void_p))
        assert r == 0, r
        return out

    def step_vjp(self, o, U, dt, g, lam3):
        """(dU^{n+1}/dU^n)^T lam3 with stages and masks from the oracle o."""
        states, masks = [U], []
        Uk = U
        for st in range(3):
            L, _, m = o.rhs(Uk, U, RK[st], dt, g, with_mask=True)
            masks.append(m)
            if st < 2:
                Uk = RK[st][0] * U + RK[st][1] * Uk + RK[st][2] * dt * L
                states.append(Uk)
        lam2 = RK[2][1] * lam3
        self.stage_vjp(states[2], masks[2], dt, g, RK[2][2], lam3, lam2)
        lam1 = RK[1][1] * lam2
        self.stage_vjp(states[1], masks[1], dt, g, RK[1][2], lam2, lam1)
        lam0 = RK[2][0] * lam3 + RK[1][0] * lam2 + lam1
        self.stage_vjp(states[0], masks[0], dt, g, RK[0][2], lam1, lam0)
        return lam0
