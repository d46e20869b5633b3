"""Pins of the oracle's characteristic boundary (a reading of the
Navier-Stokes characteristic boundary conditions cited in Sec. 3.5): the
boundary face state is built in the characteristic variables of App. A; a
variable whose wave leaves keeps the boundary cell's value, an entering one
moves by sigma toward the target's.

What fixes each check:
 - all characteristics leave (supersonic outflow): the face flux is the
   physical flux of the cell state, whatever the target;
 - all enter (supersonic inflow, sigma = 1): it is the physical flux of the
   target state;
 - a uniform flow whose target is its own state stays uniform;
 - linear acoustics: a right-running pulse leaves through a non-reflecting
   boundary without a reflected wave (measured against a reflective wall,
   which returns the whole pulse);
 - sigma relaxes the incoming acoustic variable toward the target pressure.
"""
import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs
from tests import util

R_AIR = inputs.R_UNIVERSAL / 0.029


def air_case(n, bc, P, T, u, dx=None):
    air = inputs.ideal_gas("air", 1.4, 0.029)
    dx = 1.0 / n if dx is None else dx
    sh = (1, 1, n)
    return inputs.Case("line", 1, (n, 1, 1), (dx,) * 3, (bc, 0, 0), (bc, 0, 0), [air], inputs.default_opts(),
                       np.stack([np.zeros(n), np.ones(n)]).reshape((2,) + sh), np.ones((1,) + sh),
                       np.broadcast_to(P, (n,)).reshape(sh).copy(), np.broadcast_to(T, (n,)).reshape(sh).copy(),
                       np.broadcast_to(u, (n,)).reshape((1,) + sh).copy())


def boundary_fluxes(o, U):
    dt, g = o.compute_dt(U)
    _, _, _, F = o.pseudo_states(U, U, (0.0, 1.0, 1.0), dt, g, with_flux=True)
    return F[0][:, 0], F[0][:, -1]


def test_supersonic_outflow_takes_the_cell_state():
    """u > a at both ends (flow to the right): at the right end every wave
    leaves, so the face flux is the physical flux of the last cell for any
    target and sigma."""
    a = np.sqrt(1.4 * R_AIR * 300.0)
    x = (np.arange(16) + 0.5) / 16
    case = air_case(16, 3, 1e5 * (1 + 0.1 * np.sin(2 * np.pi * x)), 300.0, 2.0 * a)
    o = oracle.Oracle.from_case(case)
    o.set_boundary_target(0, 1, 3e5, 500.0, [1.0], [-10.0], 1.0)
    U = o.init_state(case)
    _, Fhi = boundary_fluxes(o, U)
    ref = o.euler_flux(U.reshape(o.nv, -1)[:, -1])
    assert np.all(np.abs(Fhi - ref) <= 1e-14 * np.abs(ref).max())


def test_supersonic_inflow_imposes_the_target():
    """u > a entering at the left end with sigma = 1: the face flux is the
    physical flux of the target state (every wave enters)."""
    a = np.sqrt(1.4 * R_AIR * 300.0)
    case = air_case(16, 3, 1e5, 300.0, 1.5 * a)
    o = oracle.Oracle.from_case(case)
    Pt, Tt, ut = 2.5e5, 420.0, 2.2 * a
    o.set_boundary_target(0, 0, Pt, Tt, [1.0], [ut], 1.0)
    U = o.init_state(case)
    Flo, _ = boundary_fluxes(o, U)
    ut_state, _ = o.state_from_PT(Pt, Tt, [1.0], [ut])
    ref = o.euler_flux(ut_state)
    assert np.all(np.abs(Flo - ref) <= 1e-13 * np.abs(ref).max())
    # with sigma = 0 nothing enters: the flux of the first cell instead
    o.set_boundary_target(0, 0, Pt, Tt, [1.0], [ut], 0.0)
    Flo0, _ = boundary_fluxes(o, U)
    ref0 = o.euler_flux(U.reshape(o.nv, -1)[:, 0])
    assert np.all(np.abs(Flo0 - ref0) <= 1e-14 * np.abs(ref0).max())


@pytest.mark.parametrize("sigma", [0.0, 0.3, 1.0])
def test_uniform_flow_stays_uniform(sigma):
    """A subsonic uniform flow of the multi-phase mixture (stiffened liquid
    and two gases) through characteristic ends whose targets are the flow's
    own state: 20 steps leave it uniform to rounding."""
    mats = [util.stiff_liquid(), inputs.ideal_gas("A", 1.4, 0.029), inputs.ideal_gas("B", 1.667, 0.004)]
    case = util.uniform_case(mats, (0.3, 0.7), (1.0, 0.6, 0.4), 2e5, 320.0, [40.0], n=24, dim=1, bc=3)
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    u = U0.reshape(o.nv, -1)[:, 0]
    Y = u[:3] / u[:3].sum()
    for side in (0, 1):
        o.set_boundary_target(0, side, 2e5, 320.0, Y, [40.0], sigma)
    U = U0.copy()
    for _ in range(20):
        o.step(U)
    dev = np.abs(U - U0).reshape(o.nv, -1).max(1) / np.abs(U0.reshape(o.nv, -1)).max(1)
    assert np.all(dev <= 1e-13), dev


def acoustic_pulse(n, bc, amp=1e-3, x0=0.6, w=0.05):
    """A right-running isentropic pulse in air at rest (p0 = 1e5 Pa,
    T0 = 300 K) on [0, 1]: p' = amp p0 exp(-((x - x0)/w)^2), u' = p'/(rho0 a0)."""
    p0, T0 = 1e5, 300.0
    rho0 = p0 / (R_AIR * T0)
    a0 = np.sqrt(1.4 * p0 / rho0)
    x = (np.arange(n) + 0.5) / n
    pp = amp * p0 * np.exp(-((x - x0) / w) ** 2)
    P = p0 + pp
    case = air_case(n, bc, P, T0 * (P / p0) ** (0.4 / 1.4), pp / (rho0 * a0))
    return case, p0, T0, a0, amp * p0


def remaining_pulse(bc, sigma=0.0, n=200):
    """Largest pressure deviation left in the domain once the pulse has had
    time to leave through the right end (t = 0.75 / a0), over its amplitude."""
    case, p0, T0, a0, A = acoustic_pulse(n, bc)
    o = oracle.Oracle.from_case(case)
    if bc == 3:
        for side in (0, 1):
            o.set_boundary_target(0, side, p0, T0, [1.0], [0.0], sigma)
    U = o.init_state(case)
    t, tend = 0.0, 0.75 / a0
    while t < tend:
        dt, g = o.compute_dt(U)
        dt = min(dt, tend - t)
        o.step(U, dt=dt, gamma=g)
        t += dt
    P = np.array([o.equilibrium(U[i::n])["P"] for i in range(n)])
    return np.abs(P - p0).max() / A


def test_acoustic_pulse_leaves_without_reflection():
    """The pulse leaves through a non-reflecting characteristic boundary
    (sigma = 0) leaving less than 1e-5 of its amplitude behind (measured
    4.6e-6); relaxing the entering wave fully toward the rest state
    (sigma = 1) leaves less than 1e-3 (2.0e-4); a reflective wall sends the
    whole pulse back (> 0.99)."""
    wall = remaining_pulse(2)
    r0 = remaining_pulse(3, 0.0)
    r1 = remaining_pulse(3, 1.0)
    print("wall", wall, "characteristic sigma 0", r0, "sigma 1", r1)
    assert wall > 0.99
    assert r0 < 1e-5 and r1 < 1e-3


def test_sigma_relaxes_the_pressure_toward_the_target():
    """A flow at rest between two characteristic ends whose target pressure is
    2 % above its own: with sigma = 0 nothing enters and the state stays
    put; with sigma = 0.05 pressure waves enter and the mean pressure rises
    toward the target."""
    p0, T0 = 1e5, 300.0
    case = air_case(50, 3, p0, T0, 0.0)
    res = {}
    for sigma in (0.0, 0.05):
        o = oracle.Oracle.from_case(case)
        for side in (0, 1):
            o.set_boundary_target(0, side, 1.02 * p0, T0, [1.0], [0.0], sigma)
        U = o.init_state(case)
        means = []
        for k in range(400):
            o.step(U)
            if k % 100 == 99:
                means.append(np.mean([o.equilibrium(U[i::50])["P"] for i in range(50)]) / p0 - 1.0)
        res[sigma] = means
    print(res)
    assert max(abs(m) for m in res[0.0]) <= 1e-13
    m = res[0.05]
    assert all(b > a for a, b in zip(m, m[1:])) and 0.004 < m[-1] < 0.0201


def test_target_rejections():
    case = air_case(8, 3, 1e5, 300.0, 0.0)
    o = oracle.Oracle.from_case(case)
    for args in ((0, 0, 1e5, 300.0, [1.0], [0.0], 1.5), (0, 0, 1e5, -1.0, [1.0], [0.0], 0.5),
                 (0, 2, 1e5, 300.0, [1.0], [0.0], 0.5), (1, 0, 1e5, 300.0, [1.0], [0.0], 0.5),
                 (0, 0, -2e5, 300.0, [1.0], [0.0], 0.5), (0, 0, 1e5, 300.0, [0.9], [0.0], 0.5)):
        with pytest.raises(ValueError):
            o.set_boundary_target(*args)
    o1 = oracle.Oracle.from_case(air_case(8, 1, 1e5, 300.0, 0.0))
    with pytest.raises(ValueError):
        o1.set_boundary_target(0, 0, 1e5, 300.0, [1.0], [0.0], 0.5)
