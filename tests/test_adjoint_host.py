"""The adjoint's reverse code executed on the host (the same functions the
GPU kernels run, see adjoint_host.cpp) against the oracle's complex-step
derivatives: every Jacobian column of one step on tiny grids, dot products of
one step on smooth states, and stage pull-backs on shock and interface
states.  Stage states and decision masks come from the oracle."""
import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs
from tests import adjoint_host
from tests.test_adjoint import DOT, STAGE, TINY, cotangent, direction

RK = adjoint_host.RK


@pytest.fixture(scope="module")
def so(tmp_path_factory):
    return adjoint_host.build(str(tmp_path_factory.mktemp("adjhost")))


@pytest.mark.parametrize("name", sorted(TINY))
def test_host_adjoint_every_column(so, name):
    case = TINY[name]()
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    dt, g = o.compute_dt(U)
    h = adjoint_host.HostAdjoint(so, case)
    lam3 = cotangent(U, o.ns, o.dim, np.random.default_rng(7))
    lam0 = h.step_vjp(o, U, dt, g, lam3)
    nv, n = o.nv, o.ncell
    Ur = U.reshape(nv, n)
    for j in range(nv * n):
        v, i = divmod(j, n)
        if v < o.ns and Ur[v, i] == 0.0:
            continue
        e = np.zeros(nv * n)
        e[j] = 1.0
        ref = lam3 @ o.jvp_step(U, e, dt, g)[1]
        sc = np.abs(lam0.reshape(nv, n)[v]).max()
        assert abs(lam0[j] - ref) <= 1e-10 * sc, (j, lam0[j], ref)


@pytest.mark.parametrize("name", sorted(DOT) + sorted(STAGE))
def test_host_adjoint_dot_products(so, name):
    case = (DOT.get(name) or STAGE[name])()
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    dt, g = o.compute_dt(U)
    rng = np.random.default_rng(3)
    h = adjoint_host.HostAdjoint(so, case)
    lam3 = cotangent(U, o.ns, o.dim, rng)
    lam0 = h.step_vjp(o, U, dt, g, lam3)
    for _ in range(3):
        dU = direction(U, o.ns, o.dim, rng)
        lhs = lam3 @ o.jvp_step(U, dU, dt, g)[1]
        assert abs(lhs - lam0 @ dU) <= 1e-9 * np.abs(lam0 * dU).sum()


@pytest.mark.parametrize("name", sorted(STAGE))
def test_host_stage_pullbacks(so, name):
    case = STAGE[name]()
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    dt, g = o.compute_dt(U)
    rng = np.random.default_rng(11)
    h = adjoint_host.HostAdjoint(so, case)
    Uk = U
    for st in range(3):
        L, _, m = o.rhs(Uk, U, RK[st], dt, g, with_mask=True)
        Lbar = cotangent(U, o.ns, o.dim, rng)
        out = np.zeros_like(U)
        h.stage_vjp(Uk, m, dt, g, 1.0, Lbar, out)  # dt J^T Lbar
        for _ in range(2):
            dU = direction(Uk, o.ns, o.dim, rng)
            lhs = dt * (Lbar @ o.jvp_rhs(Uk, dU, U, RK[st], dt, g)[1])
            assert abs(lhs - out @ dU) <= 1e-9 * np.abs(out * dU).sum(), st
        Uk = RK[st][0] * U + RK[st][1] * Uk + RK[st][2] * dt * L
