"""Pins of the oracle's general pressure solve (several distinct P_inf: the
equality of Eqs. NASG_T1 and NASG_T2 solved iteratively, Sec. 2.3)."""
import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs


def make(case):
    return oracle.Oracle.from_case(case)


@pytest.mark.parametrize("seed", range(4))
def test_round_trip_recovers_pressure_and_temperature(seed):
    """The conserved state of (P, T, Y, u) (Eq. NASG_EOS, built directly)
    must return the same P and T from the equilibrium: two liquids of
    different P_inf (one with the NASG co-volume and reference energy of
    water) and a gas, all present, over four decades of pressure."""
    o = make(inputs.random_smooth_state_case(dim=1, n=(8, 1, 1), multi_pinf=True))
    rng = np.random.default_rng(seed)
    for _ in range(50):
        P = 10 ** rng.uniform(4, 8)
        T = rng.uniform(250.0, 600.0)
        Y = rng.dirichlet(np.ones(3))
        Y = np.maximum(Y, 1e-12)
        Y /= Y.sum()
        u, _ = o.state_from_PT(P, T, Y, [rng.uniform(-50, 50)])
        e = o.equilibrium(u)
        assert abs(e["P"] / P - 1) <= 1e-9, (P, e["P"])
        assert abs(e["T"] / T - 1) <= 1e-9, (T, e["T"])


def test_general_solve_meets_the_closed_form():
    """Two liquids whose P_inf differ by one part in 1e12 take the iterative
    path; on the same conserved states it must agree with the closed form of
    Eq. NASG_P for equal P_inf."""
    base = inputs.random_smooth_state_case(dim=1, n=(8, 1, 1), multi_pinf=True)
    same = inputs.random_smooth_state_case(dim=1, n=(8, 1, 1), multi_pinf=True)
    for case, pinf in ((base, 3.43e8 * (1 + 1e-12)), (same, 3.43e8)):
        case.materials[1].pinf = pinf
        case.materials[1].b = 0.0
        case.materials[1].q = 0.0
    og, oc = make(base), make(same)
    rng = np.random.default_rng(5)
    for _ in range(30):
        Y = rng.dirichlet(np.ones(3))
        u, _ = oc.state_from_PT(10 ** rng.uniform(4, 8), rng.uniform(250, 600), Y, [0.0])
        pg, pc = og.equilibrium(u)["P"], oc.equilibrium(u)["P"]
        assert abs(pg / pc - 1) <= 1e-8, (pg, pc)


def test_pressure_is_the_largest_root():
    """Every root of T1 = T2 above P_lo, found independently by dense sampling
    of F on a log grid, lies at or below the oracle's pressure."""
    o = make(inputs.random_smooth_state_case(dim=1, n=(8, 1, 1), multi_pinf=True))
    case = inputs.random_smooth_state_case(dim=1, n=(8, 1, 1), multi_pinf=True)
    m = case.materials
    rng = np.random.default_rng(9)
    for _ in range(20):
        Y = rng.dirichlet(np.ones(3))
        u, _ = o.state_from_PT(10 ** rng.uniform(4, 8), rng.uniform(250, 600), Y, [0.0])
        rho = u[:3].sum()
        Yc = u[:3] / rho
        e = u[-1] / rho - 0.5 * (u[3] / rho) ** 2
        q = sum(Yc[k] * m[k].q for k in range(3))
        b = sum(Yc[k] * m[k].b for k in range(3))
        Cv = sum(Yc[k] * m[k].cv for k in range(3))
        A = [Yc[k] * (m[k].gamma - 1) * m[k].cv * (e - q - (1 / rho - b) * m[k].pinf) for k in range(3)]
        F = lambda P: (1 / rho - b) * Cv - sum(A[k] / (P + m[k].pinf) for k in range(3))
        Ps = np.logspace(-3, 12, 200001)  # P_lo = 0: the gas is present
        Fv = np.array([F(p) for p in Ps[::50]])
        roots = Ps[::50][1:][np.sign(Fv[1:]) != np.sign(Fv[:-1])]
        P = o.equilibrium(u)["P"]
        assert len(roots) >= 1 and roots.max() <= P * 1.01, (roots, P)
