"""Pins of the oracle's viscous stress and heat conduction (Eq. DiffusionTerms,
viscous fluxes by second-order central differences).

Each check is a closed form: a sine or cosine mode is an eigenvector of the
discrete operators, so the right-hand side is the mode times its discrete
eigenvalue.  Where the convective terms do not vanish on their own, the
viscous part is the difference of two right-hand sides, with the viscous
terms on and off (the other terms and the limiter decisions are the same)."""
import math

import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs

GAS_MU = 2e-3          # [Pa s], large enough to dominate rounding of P-scale fluxes
AIR = inputs.ideal_gas("air", 1.4, 0.029, mu=GAS_MU)
WATER = inputs.Material("water", inputs.LIQUID, 1816.0, 6.12, pinf=3.43e8, molar_mass=0.018, mu=1e-2,
                        lam=0.6)


def case_of(mat, n, dx, vel, T, bc=(0, 0, 0), viscous=1, P=1e5):
    dim = len([m for m in n if m > 1]) if len(n) == 3 else len(n)
    n3 = tuple(n) + (1,) * (3 - len(n))
    sh = (n3[2], n3[1], n3[0])
    liquid = mat.phase == inputs.LIQUID
    phi = np.stack([np.full(sh, 1.0 if liquid else 0.0), np.full(sh, 0.0 if liquid else 1.0)])
    vel3 = np.stack([np.broadcast_to(v, sh).astype(float) for v in vel])
    return inputs.Case("visc", dim, n3, tuple(dx) + (dx[0],) * (3 - len(dx)), bc, bc, [mat],
                       inputs.default_opts(viscous=viscous, positivity=1, prandtl=0.71),
                       phi, np.ones((1,) + sh), np.full(sh, P), np.broadcast_to(T, sh).astype(float), vel3)


def rhs_of(case):
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    return o.rhs(U, U, (0.0, 1.0, 1.0), 1e-9, 0.0).reshape(case.nv, -1), o


def viscous_part(case):
    L1, o = rhs_of(case)
    case.opts = dict(case.opts, viscous=0)
    L0, _ = rhs_of(case)
    case.opts = dict(case.opts, viscous=1)
    return L1 - L0


def close(a, b, tol=1e-9):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() <= tol * scale, (np.abs(a - b).max(), scale)


def test_shear_wave_momentum_and_viscous_work():
    """u = U0 sin(k y), v = 0 at uniform P, T (2D periodic): every other term
    cancels, L(rho u) = mu D2y u and L(E) = mu D2y(u^2)/2, both closed forms."""
    ny, dy, U0 = 32, 1e-3, 3.0
    k = 2 * math.pi / (ny * dy)
    y = (np.arange(ny) + 0.5) * dy
    u = U0 * np.sin(k * y)[:, None] * np.ones((ny, 8))
    case = case_of(AIR, (8, ny), (dy, dy), [u, np.zeros_like(u)], 300.0)
    L, _ = rhs_of(case)
    lam2 = (2.0 - 2.0 * math.cos(k * dy)) / dy ** 2
    exp_mom = -GAS_MU * lam2 * u.reshape(-1)
    ok, info = close(L[1], exp_mom)
    assert ok, info
    assert np.abs(L[2]).max() <= 1e-9 * np.abs(exp_mom).max()
    assert np.abs(L[0]).max() <= 1e-12 * np.abs(exp_mom).max()
    # D2 of u^2 = U0^2 (1 - cos 2ky)/2
    exp_E = GAS_MU * U0 ** 2 * np.cos(2 * k * y)[:, None] * (1 - math.cos(2 * k * dy)) / (2 * dy ** 2)
    ok, info = close(L[3], (exp_E * np.ones((ny, 8))).reshape(-1))
    assert ok, info


@pytest.mark.parametrize("mat", ["gas", "liquid"])
def test_heat_conduction_mode(mat):
    """T = T0 + T1 sin(k x) at uniform P, u = 0 (1D periodic, a contact at
    rest): L(E) = lambda D2x T with lambda = mu C_P / Pr for the gas and the
    component's constant for the liquid; mass and momentum stay put."""
    nx, dx = 40, 1e-3
    k = 2 * math.pi / (nx * dx)
    x = (np.arange(nx) + 0.5) * dx
    T = 300.0 + 20.0 * np.sin(k * x)
    m = AIR if mat == "gas" else WATER
    case = case_of(m, (nx,), (dx,), [np.zeros(nx)], T)
    L, _ = rhs_of(case)
    lam = GAS_MU * m.gamma * m.cv / 0.71 if mat == "gas" else m.lam
    exp_E = -lam * (2.0 - 2.0 * math.cos(k * dx)) / dx ** 2 * (T - 300.0)
    ok, info = close(L[2], exp_E, tol=1e-8)
    assert ok, info
    assert np.abs(L[0]).max() <= 1e-9 * np.abs(exp_E).max() / 300.0
    assert np.abs(L[1]).max() <= 1e-9 * np.abs(exp_E).max()


def test_cross_terms_and_bulk_part():
    """u = U0 sin(kx) sin(ky), v = 0 (2D periodic): the viscous parts are
    L(rho u) = mu [4/3 D2x u + D2y u] and L(rho v) = mu/3 U0 cos(kx) cos(ky)
    sin(k dx)/dx sin(k dy)/dy (cross derivatives from the means of the two
    cells' central differences; 1 - 2/3 from the bulk term)."""
    n, h, U0 = 24, 1e-3, 2.0
    k = 2 * math.pi / (n * h)
    c = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c)  # [y, x]
    u = U0 * np.sin(k * X) * np.sin(k * Y)
    case = case_of(AIR, (n, n), (h, h), [u, np.zeros_like(u)], 300.0)
    Lv = viscous_part(case)
    lam2 = (2.0 - 2.0 * math.cos(k * h)) / h ** 2
    ok, info = close(Lv[1], (-GAS_MU * (4.0 / 3.0 + 1.0) * lam2 * u).reshape(-1), tol=1e-7)
    assert ok, info
    s = math.sin(k * h) / h
    ok, info = close(Lv[2], (GAS_MU / 3.0 * U0 * np.cos(k * X) * np.cos(k * Y) * s * s).reshape(-1), tol=1e-7)
    assert ok, info


def test_reflective_walls():
    """Reflective x-walls (1D): the tangential velocity is mirrored evenly,
    the normal one oddly, so v = V0 cos(k x) and u = U0 sin(k x) with k L = pi
    m stay eigenvectors: L(rho v) = -mu lam2 v, L(rho u) = -4/3 mu lam2 u."""
    nx, dx, m = 30, 1e-3, 2
    k = m * math.pi / (nx * dx)
    x = (np.arange(nx) + 0.5) * dx
    lam2 = (2.0 - 2.0 * math.cos(k * dx)) / dx ** 2
    v = 2.0 * np.cos(k * x)
    case = case_of(AIR, (nx, 4), (dx, dx), [np.zeros((4, nx)), v[None, :] * np.ones((4, nx))], 300.0,
                   bc=(2, 0, 0))
    L, _ = rhs_of(case)
    ok, info = close(L[2], (-GAS_MU * lam2 * v[None, :] * np.ones((4, nx))).reshape(-1))
    assert ok, info
    u = 1.5 * np.sin(k * x)
    case = case_of(AIR, (nx,), (dx,), [u], 300.0, bc=(2, 0, 0))
    Lv = viscous_part(case)
    ok, info = close(Lv[1], -4.0 / 3.0 * GAS_MU * lam2 * u, tol=1e-7)
    assert ok, info


def test_viscous_time_step_limit():
    """dt = CFL / max((|u| + a)/dx, 4 mu / (rho dx^2)) (Sec. 3.4) with the
    viscous terms on; a large viscosity makes the second bound."""
    mat = inputs.ideal_gas("thick", 1.4, 0.029, mu=50.0)
    nx, dx = 16, 1e-3
    case = case_of(mat, (nx,), (dx,), [np.zeros(nx)], 300.0)
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    dt, _ = o.compute_dt(U)
    R = 8.314462618 / 0.029
    rho = 1e5 / (R * 300.0)
    a = math.sqrt(1.4 * R * 300.0)
    expect = 0.5 / max(a / dx, 4.0 * 50.0 / (rho * dx * dx))
    assert abs(dt - expect) <= 1e-12 * expect, (dt, expect)
