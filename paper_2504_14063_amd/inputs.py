"""Seeded synthetic inputs for the four-equation MPMC solver.

This module is shared by the GPU path and by the CPU oracle.  It holds none of
the method's arithmetic: it only lays out *primitive* initial fields -- phase
volume fractions phi_p, intraphase mass fractions y_c, pressure P,
temperature T and velocity -- plus the material table and solver options.
Each side turns those into a conserved state with its own equation of state.

The workloads follow the setups the paper runs (droplet advection of
Sec. 4.2.2, shock-bubble of Sec. 4.1.1, shock-droplet of Sec. 4.2.3) at the
sizes of the benchmark configurations.  Interfaces use the equilibrium
profile phi = (1 + tanh(d / (2 eps))) / 2 of the regularization with
eps = 1.5 dx, d the signed distance into the phase.  Shock states come from
the normal-shock (Rankine-Hugoniot) relations of an ideal gas.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

R_UNIVERSAL = 8.314462618  # J/(mol K)

# phase ids used by both sides
LIQUID = 0
GAS = 1


@dataclass
class Material:
    name: str
    phase: int
    cv: float
    gamma: float
    pinf: float = 0.0
    b: float = 0.0
    q: float = 0.0
    molar_mass: float = 0.029
    mu: float = 0.0
    Sc: float = 1.0
    lam: float = 0.0     # heat conductivity of a liquid component [W/(m K)]


@dataclass
class Case:
    """Everything a solver needs for one workload."""
    name: str
    dim: int
    n: tuple
    dx: tuple
    bc_lo: tuple
    bc_hi: tuple
    materials: list
    opts: dict
    phi: np.ndarray      # [2, nz, ny, nx]   phase volume fractions (liquid, gas)
    y: np.ndarray        # [ns, nz, ny, nx]  intraphase mass fractions
    P: np.ndarray        # [nz, ny, nx]
    T: np.ndarray        # [nz, ny, nx]
    vel: np.ndarray      # [dim, nz, ny, nx]
    steps: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def ns(self):
        return len(self.materials)

    @property
    def nv(self):
        return self.ns + self.dim + 1

    @property
    def ncell(self):
        return int(np.prod(self.n))

    def grid_dict(self):
        return dict(dim=self.dim, n=list(self.n), dx=list(self.dx),
                    bc_lo=list(self.bc_lo), bc_hi=list(self.bc_hi))

    def eos_dict(self):
        m = self.materials
        return dict(n_species=len(m), phase=[x.phase for x in m], cv=[x.cv for x in m],
                    gamma=[x.gamma for x in m], pinf=[x.pinf for x in m], b=[x.b for x in m],
                    q=[x.q for x in m], molar_mass=[x.molar_mass for x in m],
                    mu=[x.mu for x in m], Sc=[x.Sc for x in m], **{"lambda": [x.lam for x in m]})

    def prim_arrays(self):
        """Flattened float64 arrays (phi[2,N], y[ns,N], P[N], T[N], vel[dim,N])."""
        N = self.ncell
        f = lambda a, k: np.ascontiguousarray(a.reshape(k, N), dtype=np.float64)
        return (f(self.phi, 2), f(self.y, self.ns), np.ascontiguousarray(self.P.reshape(N)),
                np.ascontiguousarray(self.T.reshape(N)), f(self.vel, self.dim))


def default_opts(**kw):
    o = dict(cfl=0.5, cdi=0, eps_cdi=0.0, phi_min=1e-8, delta=1e-100, gamma_scale=1.0,
             diffusion=0, positivity=1, precision=0, weno=0, weno_eps=1e-40, weno_p=1, viscous=0,
             prandtl=0.71, basis=0)
    o.update(kw)
    return o


def ideal_gas(name, gamma, molar_mass, mu=0.0, Sc=1.0, cv=None):
    if cv is None:
        cv = R_UNIVERSAL / (molar_mass * (gamma - 1.0))
    return Material(name, GAS, cv, gamma, 0.0, 0.0, 0.0, molar_mass, mu, Sc)


def normal_shock(gamma, R, M, p1, T1):
    """Post-shock (p2, T2, u2) behind a shock of Mach M moving into gas at rest."""
    p2 = p1 * (1.0 + 2.0 * gamma * (M * M - 1.0) / (gamma + 1.0))
    r21 = (gamma + 1.0) * M * M / ((gamma - 1.0) * M * M + 2.0)
    a1 = math.sqrt(gamma * R * T1)
    u2 = M * a1 * (1.0 - 1.0 / r21)
    T2 = T1 * (p2 / p1) / r21
    return p2, T2, u2, M * a1


def _tanh_profile(d, eps):
    """1/2 (1 + tanh(d / 2 eps)), written as the logistic function 1/(1 + e^(-d/eps))
    so that the complementary profile _tanh_profile(-d, eps) carries no
    cancellation (1 - profile rounds to 0 or 1e-16 deep inside)."""
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-d / eps))


def _centers(n, dx):
    return (np.arange(n, dtype=np.float64) + 0.5) * dx


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def interface_advection_1d(n=400, steps=200, u0=100.0, cdi=1, length=1.0):
    """1D two-phase interface advection: ideal gas A | stiffened gas B slab."""
    dx = length / n
    eps = 1.5 * dx
    A = Material("A", GAS, 718.0, 1.4, molar_mass=R_UNIVERSAL / (0.4 * 718.0))
    B = Material("B", LIQUID, 1816.0, 6.12, pinf=3.43e8, molar_mass=0.018)
    x = _centers(n, dx)
    phiB = _tanh_profile(x - 0.3 * length, eps) - _tanh_profile(x - 0.7 * length, eps)
    phiA = _tanh_profile(0.3 * length - x, eps) + _tanh_profile(x - 0.7 * length, eps)
    sh = (1, 1, n)
    phi = np.stack([phiB, phiA]).reshape((2,) + sh)
    y = np.ones((2,) + sh)
    P = np.full(sh, 1e5)
    T = np.full(sh, 300.0)
    vel = np.full((1,) + sh, u0)
    return Case("interface_advection_1d", 1, (n, 1, 1), (dx, dx, dx), (0, 0, 0), (0, 0, 0),
                [A, B], default_opts(cdi=cdi, eps_cdi=eps), phi, y, P, T, vel, steps)


def shock_bubble_2d(nx=1024, ny=256, steps=2000, dx=1e-3, radius=25.0, center=(320.0, 128.0),
                    shock_x=280.0, mach=1.22):
    """2D shock-bubble: Mach 1.22 shock in gas A hits a bubble of gas B (one gas phase)."""
    A = ideal_gas("A", 1.4, 0.029, mu=1.81e-5, Sc=1.0)
    B = ideal_gas("B", 1.667, 0.004, mu=1.96e-5, Sc=0.70)
    eps = 1.5 * dx
    x = _centers(nx, dx)[None, :]
    yy = _centers(ny, dx)[:, None]
    r = np.sqrt((x - center[0] * dx) ** 2 + (yy - center[1] * dx) ** 2)
    yB = _tanh_profile(radius * dx - r, eps)
    yA = _tanh_profile(r - radius * dx, eps)
    p1, T1 = 1e5, 300.0
    p2, T2, u2, ws = normal_shock(1.4, R_UNIVERSAL / 0.029, mach, p1, T1)
    post = np.broadcast_to(x < shock_x * dx, (ny, nx))
    P = np.where(post, p2, p1)
    T = np.where(post, T2, T1)
    u = np.where(post, u2, 0.0)
    sh = (1, ny, nx)
    phi = np.stack([np.zeros((ny, nx)), np.ones((ny, nx))]).reshape((2,) + sh)
    y = np.stack([yA, yB]).reshape((2,) + sh)
    vel = np.stack([u, np.zeros((ny, nx))]).reshape((2,) + sh)
    return Case("shock_bubble_2d", 2, (nx, ny, 1), (dx, dx, dx), (1, 2, 0), (1, 2, 0), [A, B],
                default_opts(diffusion=1), phi, y, P.reshape(sh), T.reshape(sh), vel, steps,
                extra=dict(shock_speed=ws, p2=p2, T2=T2, u2=u2, shock_x=shock_x * dx))


def _smooth_noise(rng, shape_xyz, L, modes=4):
    nx, ny, nz = shape_xyz
    k = rng.integers(1, 5, size=(modes, 3))
    th = rng.uniform(0.0, 2 * math.pi, size=modes)
    a = rng.uniform(0.5, 1.0, size=modes)
    return k, th, a


def droplet_crossflow_3d(n=256, steps=100, dx=None, radius=None, seed=0, u0=50.0, floor=True):
    """3D liquid droplet (stiffened gas) in a crossflow of a two-species ideal-gas
    mixture; volume fractions floored at phi_min (floor=True, see floor_phi)."""
    if dx is None:
        dx = 0.256 / n
    if radius is None:
        radius = 32.0 * n / 256.0
    L = n * dx
    eps = 1.5 * dx
    liq = Material("liquid", LIQUID, 1816.0, 6.12, pinf=3.43e8, molar_mass=0.018, mu=8.9e-4, lam=0.6)
    A = ideal_gas("A", 1.4, 0.029, mu=1.81e-5, Sc=1.0)
    B = ideal_gas("B", 1.667, 0.004, mu=1.96e-5, Sc=0.70)
    rng = np.random.default_rng(seed)
    c0 = n / 2.0 + rng.uniform(-2.0, 2.0, size=3)
    k, th, a = _smooth_noise(rng, (n, n, n), L)
    x = _centers(n, dx)
    X = x[None, None, :]
    Y = x[None, :, None]
    Z = x[:, None, None]
    r = np.sqrt((X - c0[0] * dx) ** 2 + (Y - c0[1] * dx) ** 2 + (Z - c0[2] * dx) ** 2)
    phil = _tanh_profile(radius * dx - r, eps)
    phig = _tanh_profile(r - radius * dx, eps)
    s = np.zeros((n, n, n))
    for m in range(len(a)):
        s = s + a[m] * np.sin(2 * math.pi * (k[m, 0] * X + k[m, 1] * Y + k[m, 2] * Z) / L + th[m])
    s = s / a.sum()
    yA = 0.7 * (1.0 + 0.01 * s)
    yB = 1.0 - yA
    sh = (n, n, n)
    phi = np.stack([phil, phig])
    y = np.stack([np.ones(sh), yA, yB])
    P = np.full(sh, 1e5)
    T = np.full(sh, 300.0)
    vel = np.stack([u0 * phig, np.zeros(sh), np.zeros(sh)])
    case = Case("droplet_crossflow_3d", 3, (n, n, n), (dx, dx, dx), (0, 0, 0), (0, 0, 0),
                [liq, A, B], default_opts(cdi=1, eps_cdi=eps, diffusion=1), phi, y, P, T, vel,
                steps, extra=dict(center=c0, radius=radius))
    return floor_phi(case) if floor else case


def shock_droplet_2d(n=512, steps=200, dx=1e-3, radius=40.0, center=None, shock_x=200.0,
                     mach=1.5, floor=False):
    """2D shock-droplet: Mach 1.5 shock in an ideal gas hits a stiffened-gas
    droplet.  floor: volume fractions floored at phi_min (see floor_phi; the
    radius derivative dphil_dR is then zero where the floor holds)."""
    if center is None:
        center = (n / 2.0, n / 2.0)
    gas = Material("gas", GAS, 718.0, 1.4, molar_mass=R_UNIVERSAL / (0.4 * 718.0), mu=1.81e-5)
    liq = Material("liquid", LIQUID, 1816.0, 6.12, pinf=3.43e8, molar_mass=0.018, mu=8.9e-4)
    eps = 1.5 * dx
    x = _centers(n, dx)[None, :]
    yy = _centers(n, dx)[:, None]
    r = np.sqrt((x - center[0] * dx) ** 2 + (yy - center[1] * dx) ** 2)
    phil = _tanh_profile(radius * dx - r, eps)
    phig = _tanh_profile(r - radius * dx, eps)
    p1, T1 = 1e5, 300.0
    p2, T2, u2, ws = normal_shock(1.4, 0.4 * 718.0, mach, p1, T1)
    post = np.broadcast_to(x < shock_x * dx, (n, n))
    P = np.where(post, p2, p1)
    T = np.where(post, T2, T1)
    u = np.where(post, u2, 0.0)
    sh = (1, n, n)
    phi = np.stack([phil, phig]).reshape((2,) + sh)
    y = np.ones((2,) + sh)
    vel = np.stack([u, np.zeros((n, n))]).reshape((2,) + sh)
    dphil_dR = phil * phig / eps * dx  # d/dR of the logistic profile, R in cells
    case = Case("shock_droplet_2d", 2, (n, n, 1), (dx, dx, dx), (1, 2, 0), (1, 2, 0),
                [gas, liq], default_opts(cdi=1, eps_cdi=eps), phi, y, P.reshape(sh),
                T.reshape(sh), vel, steps,
                extra=dict(dphil_dR=dphil_dR.reshape(sh), shock_speed=ws, radius=radius))
    if floor:
        pm = case.opts["phi_min"]
        inside = (phil > pm) & (phil < 1.0 - pm)
        case.extra["dphil_dR"] = np.where(inside, dphil_dR, 0.0).reshape(sh)
        floor_phi(case)
    return case


def floor_phi(case):
    """Hold the volume fractions within [phi_min, 1 - phi_min], the floor the
    interface regularization relaxes towards (Sec. 3.2: phi_min = 1e-8 in all
    the paper's cases), instead of logistic tails that fall to zero."""
    pm = case.opts["phi_min"]
    ph = np.clip(case.phi, pm, 1.0 - pm)
    case.phi = ph / ph.sum(0, keepdims=True)
    return case


def shock_droplet_air_water_2d(n=1024, floor=True):
    """Shock-droplet interaction, air-water (Sec. 4.2.3, Table
    ShockDroplet-AirWaterSetup): a Mach 1.47 shock in air (post-shock
    2.14 kg/m^3, 228.007 m/s, 238500 Pa) onto a water droplet at rest at
    101325 Pa, water and air with the NASG constants of Table
    NASGMaterialParamters.  The schematic is not available: the droplet
    geometry of shock_droplet_2d (radius n/12.8 cells, centre of the box,
    shock at 200/512 of the width, outflow x, reflective y, 1 mm cells), one
    temperature per side from the table's densities, volume fractions floored
    at phi_min (floor=True)."""
    case = shock_droplet_2d(n=n, radius=n / 12.8, shock_x=n * 200.0 / 512.0)
    water = Material("water", LIQUID, 4185.0 / 1.0123, 1.0123, pinf=1.835e8, b=9.203e-4, q=-1.143e6,
                     molar_mass=0.018, mu=8.9e-4)
    cp, g = 1011.0, 1.4
    air = Material("air", GAS, cp / g, g, molar_mass=R_UNIVERSAL / (cp - cp / g), mu=1.81e-5)
    case.materials = [air, water]
    R = cp - cp / g
    x = _centers(n, 1.0)
    post = np.broadcast_to(x[None, :] < n * 200.0 / 512.0, (n, n)).reshape(1, n, n)
    case.P = np.where(post, 238500.0, 101325.0)
    case.T = np.where(post, 238500.0 / (2.14 * R), 101325.0 / (1.18 * R))
    case.vel = np.stack([np.where(post[0], 228.007, 0.0), np.zeros((n, n))]).reshape(2, 1, n, n)
    case.name = "shock_droplet_air_water_2d"
    return floor_phi(case) if floor else case


def _nasg_water_air():
    """Water and air with the NASG constants of Table NASGMaterialParamters."""
    water = Material("water", LIQUID, 4185.0 / 1.0123, 1.0123, pinf=1.835e8, b=9.203e-4, q=-1.143e6,
                     molar_mass=0.018, mu=0.0)
    cp, g = 1011.0, 1.4
    air = Material("air", GAS, cp / g, g, molar_mass=R_UNIVERSAL / (cp - cp / g), mu=0.0)
    return water, air


def held_values(case, U):
    """Conserved values [nv][count] of the case's held inflow cells in U."""
    nv = case.ns + case.dim + 1
    return np.asarray(U).reshape(nv, case.ncell)[:, case.extra["held"]]


def mach100_water_column_2d(nx=2048, ny=1025, floor=True, dx=1.0 / 512.0):
    """Mach-100 water column in air (Sec. 4.2.4, Table
    Mach100WaterColumnSetup): water at 997 kg/m^3, 150 km/s, 101325 Pa enters
    at x = 0 over |y| < 0.5 into air at rest (1.18 kg/m^3, 101325 Pa),
    inviscid, NASG water and air, 2048 x 1025 cells, constant dt 7.5e-4 us.
    The table gives no domain size: 1/512 m cells (x in [0, 4] m, y centred on
    0), so that the 1 m wide column spans half the height.  The inlet is the
    first column of cells with |y| < 0.5, held at the water state (their
    indices in extra['held']); every side is zero-gradient (the paper's
    non-reflecting NSCBC is defined only in its references).  Temperatures
    from each material's EOS at the table's density and pressure; volume
    fractions floored at phi_min (floor=True).  A coarser dx with nx = 4 m /
    dx keeps the geometry (parity cases)."""
    water, air = _nasg_water_air()
    x = _centers(nx, dx)
    yc = (np.arange(ny) - (ny - 1) / 2.0) * dx
    sh = (1, ny, nx)
    inlet = np.zeros((ny, nx), dtype=bool)
    inlet[:, 0] = np.abs(yc) < 0.5
    P0 = 101325.0
    Tw = (P0 + water.pinf) * (1.0 / 997.0 - water.b) / ((water.gamma - 1.0) * water.cv)
    Ta = P0 / (1.18 * (air.gamma - 1.0) * air.cv)
    phil = np.where(inlet, 1.0, 0.0)
    phi = np.stack([phil, 1.0 - phil]).reshape((2,) + sh)
    T = np.where(inlet, Tw, Ta).reshape(sh)
    vel = np.stack([np.where(inlet, 150000.0, 0.0), np.zeros((ny, nx))]).reshape((2,) + sh)
    case = Case("mach100_water_column_2d", 2, (nx, ny, 1), (dx, dx, dx), (1, 1, 0), (1, 1, 0), [water, air],
                default_opts(cdi=1, eps_cdi=1.5 * dx), phi, np.ones((2,) + sh), np.full(sh, P0), T, vel, 0,
                extra=dict(held=np.flatnonzero(inlet.ravel()), dt=7.5e-10, x=x, y=yc))
    return floor_phi(case) if floor else case


def water_inflow_1d(n=200, u_in=150000.0, length=1.0, floor=True):
    """One-dimensional Mach-100 inflow: a column of water entering air at rest
    (the centre line of Sec. 4.2.4's water column), water a stiffened gas
    (gamma 4.4, P_inf 6e8 Pa, 1000 kg/m^3), air an ideal gas, both at
    101325 Pa and 300 K.  Cell 0 is the held inlet behind a zero-gradient
    boundary; at this speed every wave of the water-air Riemann problem runs
    downstream, so on x > dx the solution is that problem's exact one with
    the jump at x = dx (extra: left, right states for the exact solver).
    CFL 0.1: with u >> a the regularization's explicit diffusion number
    Gamma eps dt / dx^2 = (eps / dx) CFL u / (u + a) exceeds the stability
    limit of the RK3 step at CFL 0.5 (the paper runs its water column at a
    constant dt, an advective CFL of about 0.06 on 1/512 m cells)."""
    rw, P0, T0, gw, pinfw = 1000.0, 101325.0, 300.0, 4.4, 6e8
    water = Material("water", LIQUID, (P0 + pinfw) / ((gw - 1.0) * rw * T0), gw, pinf=pinfw,
                     molar_mass=0.018, mu=0.0)
    cp, g = 1011.0, 1.4
    air = Material("air", GAS, cp / g, g, molar_mass=R_UNIVERSAL / (cp - cp / g), mu=0.0)
    ra = P0 / ((g - 1.0) * air.cv * T0)
    dx = length / n
    x = _centers(n, dx)
    sh = (1, 1, n)
    phil = np.zeros(n)
    phil[0] = 1.0
    phi = np.stack([phil, 1.0 - phil]).reshape((2,) + sh)
    vel = np.where(phil > 0.5, u_in, 0.0).reshape((1,) + sh)
    case = Case("water_inflow_1d", 1, (n, 1, 1), (dx, dx, dx), (1, 0, 0), (1, 0, 0), [water, air],
                default_opts(cdi=1, eps_cdi=1.5 * dx, cfl=0.1), phi, np.ones((2,) + sh), np.full(sh, P0),
                np.full(sh, T0), vel, 0,
                extra=dict(held=np.array([0]), left=(rw, u_in, P0, gw, pinfw), right=(ra, 0.0, P0, g, 0.0),
                           x=x, x0=dx))
    return floor_phi(case) if floor else case


# ---------------------------------------------------------------------------
# Small verification problems
# ---------------------------------------------------------------------------
def sod_1d(n=400, x0=0.5):
    """Sod shock tube, single ideal gas, gamma 1.4, c_v 2.5 (so R = 1, T = P/rho)."""
    gas = Material("sod", GAS, 2.5, 1.4, molar_mass=R_UNIVERSAL, mu=0.0)
    dx = 1.0 / n
    x = _centers(n, dx)
    left = x < x0
    rho = np.where(left, 1.0, 0.125)
    P = np.where(left, 1.0, 0.1)
    T = P / rho
    sh = (1, 1, n)
    phi = np.stack([np.zeros(n), np.ones(n)]).reshape((2,) + sh)
    y = np.ones((1,) + sh)
    vel = np.zeros((1,) + sh)
    return Case("sod_1d", 1, (n, 1, 1), (dx, dx, dx), (1, 0, 0), (1, 0, 0), [gas],
                default_opts(), phi, y, P.reshape(sh), T.reshape(sh), vel, 0)


def gas_liquid_riemann_1d(n=200, eps_cells=1.5, cdi=1):
    """Gas-liquid Riemann problem (Sec. 4.2.1, Table GasLiqSetup): compressed
    air | water on [-1, 1], non-dimensional, outflow ends, the interface
    regularization on (eps = eps_cells dx).  The table gives rho, u, P; the
    material constants are those of the cited setup: air an ideal gas with
    gamma 1.4 and R = 1 (c_v 2.5), water a stiffened gas with gamma 5.5 and
    P_inf 1.505, its c_v chosen so that both sides start at the same
    temperature (the four-equation model's single T in mixed cells)."""
    rhoL, uL, PL = 1.241, 1.0, 2.753
    rhoR, uR, PR = 0.991, 0.0, 3.059e-4
    gw, pinfw = 5.5, 1.505
    T0 = PL / rhoL
    air = Material("air", GAS, 2.5, 1.4, molar_mass=R_UNIVERSAL, mu=0.0)
    water = Material("water", LIQUID, (PR + pinfw) / ((gw - 1.0) * rhoR * T0), gw, pinf=pinfw,
                     molar_mass=R_UNIVERSAL, mu=0.0)
    dx = 2.0 / n
    x = -1.0 + _centers(n, dx)
    eps = eps_cells * dx
    sh = (1, 1, n)
    phil = _tanh_profile(x, eps)
    phi = np.stack([phil, _tanh_profile(-x, eps)]).reshape((2,) + sh)
    left = x < 0.0
    P = np.where(left, PL, PR)
    vel = np.where(left, uL, uR)
    case = Case("gas_liquid_riemann_1d", 1, (n, 1, 1), (dx, dx, dx), (1, 0, 0), (1, 0, 0), [water, air],
                default_opts(cdi=cdi, eps_cdi=eps), phi, np.ones((2,) + sh), P.reshape(sh),
                np.full(sh, T0), vel.reshape((1,) + sh), 0)
    case.extra = dict(t_end=0.2, left=(rhoL, uL, PL, 1.4, 0.0), right=(rhoR, uR, PR, gw, pinfw), x=x)
    return case


def mpmc_shu_osher_1d(n=400, cdi=1, eps_cells=1.0):
    """Multi-phase multi-component Shu-Osher problem (Sec. 4.3.1, Table
    MPMC_ShuOsherSetp) on [0, 20], to t = 4: ideal gases with gamma 1.4 (the
    first phase), 1.3 and 1.885 (the second phase, their mixture giving
    1/(gamma - 1) = 1.33 + 0.2 sin(5 (x - 5))), a Mach 3 shock at x = 1 and
    the immiscible interface there.  Equal molar masses (mole fractions =
    mass fractions) and R = 1; characteristic ends (Sec. 3.5): the left one
    a supersonic inflow imposing the post-shock state of the first phase
    (sigma = 1), the right one non-reflecting (sigma = 0); the
    regularization on with cdi = 1 (eps = eps_cells dx; the paper's eps ~ dx:
    with 1.5 dx the regularized interface is wider at t = 4 than the
    unregularized one)."""
    g = (1.4, 1.3, 1.885)
    mats = [Material(f"gamma{k + 1}", LIQUID if k == 0 else GAS, 1.0 / (g[k] - 1.0), g[k],
                     molar_mass=R_UNIVERSAL, mu=0.0) for k in range(3)]
    L = 20.0
    dx = L / n
    x = _centers(n, dx)
    eps = eps_cells * dx
    sh = (1, 1, n)
    left = x < 1.0
    sn = np.sin(5.0 * (x - 5.0))
    rho = np.where(left, 3.857143, 1.0 + 0.2 * sn)
    P = np.where(left, 10.3333, 1.0)
    vel = np.where(left, 2.629369, 0.0)
    inv_gm1 = 1.33 + 0.2 * sn
    X2 = (inv_gm1 - 1.0 / (g[2] - 1.0)) / (1.0 / (g[1] - 1.0) - 1.0 / (g[2] - 1.0))
    phi1 = _tanh_profile(1.0 - x, eps)
    phi = np.stack([phi1, _tanh_profile(x - 1.0, eps)]).reshape((2,) + sh)
    y = np.stack([np.ones(n), X2, 1.0 - X2]).reshape((3,) + sh)
    case = Case("mpmc_shu_osher_1d", 1, (n, 1, 1), (dx, dx, dx), (3, 0, 0), (3, 0, 0), mats,
                default_opts(cdi=cdi, eps_cdi=eps if cdi else 0.0), phi, y, P.reshape(sh),
                (P / rho).reshape(sh), vel.reshape((1,) + sh), 0)
    targets = [(0, 0, 10.3333, 10.3333 / 3.857143, [1.0, 0.0, 0.0], [2.629369], 1.0),
               (0, 1, 1.0, 1.0 / rho[-1], [0.0, X2[-1], 1.0 - X2[-1]], [0.0], 0.0)]
    case.extra = dict(t_end=4.0, x=x, boundary_targets=targets)
    return case


def phase_constrained_mixing_2d(n=400, L=0.4, bubble=0.3, pocket=0.05, eps_cells=1.5, floor=True):
    """Phase-constrained multi-component mixing (Sec. 4.3.2, Table
    PhaseConstrainedDiffustionSetup): a helium bubble holding five air pockets,
    immiscible with the surrounding SF6, all at rest at 101325 Pa, viscosities
    10^4 times physical (the table's values) so that diffusion sets dt.  The
    paper's schematic is not available: the bubble (diameter bubble * L) sits
    at the centre of a periodic L x L box and the pockets (diameter
    pocket * L) on a circle of half the bubble radius.  Molar masses follow the
    table's densities at one temperature (293.6 K); gamma 1.1, 1.4, 5/3;
    volume fractions floored at phi_min (floor=True, see floor_phi)."""
    P0, T0 = 101325.0, 293.6
    W = {k: rho * R_UNIVERSAL * T0 / P0 for k, rho in (("sf6", 6.06), ("air", 1.18), ("he", 0.166))}
    sf6 = ideal_gas("SF6", 1.1, W["sf6"], mu=1.5e-1, Sc=1.0)
    sf6.phase = LIQUID
    air = ideal_gas("air", 1.4, W["air"], mu=1.81e-1, Sc=1.0)
    he = ideal_gas("He", 5.0 / 3.0, W["he"], mu=1.96e-1, Sc=0.7)
    dx = L / n
    eps = eps_cells * dx
    x = _centers(n, dx)
    X = x[None, None, :]
    Y = x[None, :, None]
    c = 0.5 * L
    r = np.sqrt((X - c) ** 2 + (Y - c) ** 2)
    R = 0.5 * bubble * L
    phi_in = _tanh_profile(R - r, eps)
    phi_out = _tanh_profile(r - R, eps)
    ya = np.zeros((1, n, n))
    for k in range(5):
        a = 2.0 * math.pi * k / 5.0
        px, py = c + 0.5 * R * math.cos(a), c + 0.5 * R * math.sin(a)
        rp = np.sqrt((X - px) ** 2 + (Y - py) ** 2)
        ya = np.maximum(ya, _tanh_profile(0.5 * pocket * L - rp, eps))
    sh = (1, n, n)
    phi = np.stack([phi_out, phi_in]).reshape((2,) + sh)
    y = np.stack([np.ones(sh), ya.reshape(sh), 1.0 - ya.reshape(sh)])
    case = Case("phase_constrained_mixing_2d", 2, (n, n, 1), (dx, dx, dx), (0, 0, 0), (0, 0, 0),
                [sf6, air, he], default_opts(cdi=1, eps_cdi=eps, diffusion=1, viscous=1), phi, y,
                np.full(sh, P0), np.full(sh, T0), np.zeros((2,) + sh), 0,
                extra=dict(radius=R, center=(c, c)))
    return floor_phi(case) if floor else case


def shu_osher_1d(n=200):
    """Shu-Osher shock tube (App. "Shu-Osher shock tube", Table ShuOsherSetp):
    one ideal gas (gamma 1.4, R = 1) on [0, 10], a Mach 3 shock at x = 1 into
    rho = 1 + 0.2 sin(5 (x - 5)); outflow ends; run with the constant
    dt = 4e-3 (200 cells, scaled with the cell size) to t = 1.8."""
    gas = Material("gas", GAS, 2.5, 1.4, molar_mass=R_UNIVERSAL, mu=0.0)
    dx = 10.0 / n
    x = _centers(n, dx)
    left = x < 1.0
    rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * (x - 5.0)))
    P = np.where(left, 10.3333, 1.0)
    vel = np.where(left, 2.629369, 0.0)
    sh = (1, 1, n)
    case = Case("shu_osher_1d", 1, (n, 1, 1), (dx, dx, dx), (1, 0, 0), (1, 0, 0), [gas], default_opts(),
                np.stack([np.zeros(n), np.ones(n)]).reshape((2,) + sh), np.ones((1,) + sh), P.reshape(sh),
                (P / rho).reshape(sh), vel.reshape((1,) + sh), 0)
    case.extra = dict(t_end=1.8, dt=4e-3 * 200.0 / n, x=x)
    return case


def isentropic_vortex_2d(n=64, L=10.0, beta=5.0, uinf=(1.0, 1.0), t_end=2.0):
    """Two-dimensional vortex advection (App. "Two-dimensional vortex
    advection"; the cited setup is not in the paper): the isentropic vortex of
    strength beta in an ideal gas (gamma 1.4, R = 1) on a periodic L x L box,
    carried by the free stream uinf.  Point values at cell centres; the exact
    solution at time t is the initial field translated by uinf t."""
    gas = Material("gas", GAS, 2.5, 1.4, molar_mass=R_UNIVERSAL, mu=0.0)
    dx = L / n
    x = _centers(n, dx)
    case = Case("isentropic_vortex_2d", 2, (n, n, 1), (dx, dx, dx), (0, 0, 0), (0, 0, 0), [gas],
                default_opts(), None, None, None, None, None, 0)
    rho, u, v, P = _vortex_fields(x, x, 0.0, L, beta, uinf)
    sh = (1, n, n)
    case.phi = np.stack([np.zeros(sh), np.ones(sh)])
    case.y = np.ones((1,) + sh)
    case.P = P.reshape(sh)
    case.T = (P / rho).reshape(sh)
    case.vel = np.stack([u.reshape(sh), v.reshape(sh)])
    case.extra = dict(t_end=t_end, exact=lambda t: _vortex_fields(x, x, t, L, beta, uinf))
    return case


def _vortex_fields(xc, yc, t, L, beta, uinf, gamma=1.4):
    """(rho, u, v, P) of the isentropic vortex centred at L/2 + uinf t
    (periodic images summed over the nearest copies)."""
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    cx = (0.5 * L + uinf[0] * t) % L
    cy = (0.5 * L + uinf[1] * t) % L
    dxv = (X - cx + 0.5 * L) % L - 0.5 * L
    dyv = (Y - cy + 0.5 * L) % L - 0.5 * L
    r2 = dxv ** 2 + dyv ** 2
    f = np.exp(0.5 * (1.0 - r2))
    dT = -(gamma - 1.0) * beta ** 2 / (8.0 * gamma * math.pi ** 2) * f * f
    rho = (1.0 + dT) ** (1.0 / (gamma - 1.0))
    u = uinf[0] - beta / (2.0 * math.pi) * f * dyv
    v = uinf[1] + beta / (2.0 * math.pi) * f * dxv
    P = rho ** gamma
    return rho, u, v, P


def density_wave_1d(n=64, amp=0.2):
    """Smooth density wave of one ideal gas (R = 1): rho = 1 + amp sin(2 pi x), u = 1, p = 1.
    The cell-average initial data are set by the test; this returns point values."""
    gas = Material("g", GAS, 2.5, 1.4, molar_mass=R_UNIVERSAL, mu=0.0)
    dx = 1.0 / n
    x = _centers(n, dx)
    rho = 1.0 + amp * np.sin(2 * math.pi * x)
    P = np.ones(n)
    sh = (1, 1, n)
    phi = np.stack([np.zeros(n), np.ones(n)]).reshape((2,) + sh)
    return Case("density_wave_1d", 1, (n, 1, 1), (dx, dx, dx), (0, 0, 0), (0, 0, 0), [gas],
                default_opts(), phi, np.ones((1,) + sh), P.reshape(sh), (P / rho).reshape(sh),
                np.ones((1,) + sh), 0)


def many_component_case(dim=2, n=(16, 12, 1), seed=0, n_liquid=2, n_gas=3, bc=(0, 0, 0), distinct_pinf=False,
                        cdi=1, diffusion=1, amp=0.05, floor=True):
    """A droplet of n_liquid stiffened-gas components in n_gas ideal gases (up
    to 8 components together), smooth random fields: parity cases for more
    components than the paper's workloads use.  The liquids share
    P_inf = 3.43e8 Pa (distinct values 3.43e8 / (1 + k) with distinct_pinf)
    and differ in C_v, gamma, molar mass and viscosity; the gases in gamma,
    molar mass, viscosity and Schmidt number; each phase's mass fractions
    are positive smooth fields summing to one.  Volume fractions floored at
    phi_min (floor=True): with more than one component in a phase, a phase
    present only in traces diffuses with its own diffusivity, which the
    time-step bound (mixture viscosity) does not cover."""
    assert 1 <= n_liquid and 1 <= n_gas and n_liquid + n_gas <= 8
    rng = np.random.default_rng(seed)
    dx = 1e-3
    mats = []
    for k in range(n_liquid):
        mats.append(Material(f"liquid{k}", LIQUID, 1816.0 * (1.0 + 0.15 * k), 6.12 - 0.6 * k,
                             pinf=3.43e8 / (1.0 + k) if distinct_pinf else 3.43e8,
                             molar_mass=0.018 * (1.0 + 0.5 * k), mu=8.9e-4 * (1.0 + 0.2 * k), Sc=1.0 + 0.3 * k))
    gas_gamma = [1.4, 1.667, 1.3, 1.33, 1.4, 1.667, 1.29]
    gas_w = [0.029, 0.004, 0.044, 0.016, 0.028, 0.040, 0.032]
    for k in range(n_gas):
        mats.append(ideal_gas(f"gas{k}", gas_gamma[k], gas_w[k], mu=(1.8 + 0.1 * k) * 1e-5, Sc=0.7 + 0.1 * k))
    nn = tuple(n[d] if d < dim else 1 for d in range(3))
    shape = (nn[2], nn[1], nn[0])
    Z, Yg, X = np.meshgrid(*[(np.arange(nn[d]) + 0.5) / nn[d] for d in (2, 1, 0)], indexing="ij")

    def field_(scale):
        out = np.zeros(shape)
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            out += np.sin(2 * math.pi * (k[0] * X + k[1] * Yg * (dim > 1) + k[2] * Z * (dim > 2)) + ph)
        return scale * out / 3.0

    eps = 1.5 * dx
    c0 = (0.5 + 0.0317, 0.5 - 0.0211, 0.5 + 0.0123)
    dist = (0.3 - np.sqrt((X - c0[0]) ** 2 + ((Yg - c0[1]) ** 2 if dim > 1 else 0)
                          + ((Z - c0[2]) ** 2 if dim > 2 else 0))) * nn[0] * dx
    phi = np.stack([_tanh_profile(dist, eps), _tanh_profile(-dist, eps)])

    def fractions(m):
        w = np.stack([1.0 + field_(0.3) for _ in range(m)])
        return w / w.sum(0)

    y = np.concatenate([fractions(n_liquid), fractions(n_gas)])
    P = 1e5 * (1.0 + field_(amp))
    T = 300.0 * (1.0 + field_(amp))
    vel = np.stack([30.0 * field_(1.0) + 20.0 for _ in range(dim)])
    case = Case("many_component", dim, nn, (dx, dx, dx), bc, bc, mats,
                default_opts(cdi=cdi, eps_cdi=eps, diffusion=diffusion), phi, y, P, T, vel, 0)
    return floor_phi(case) if floor else case


def smooth_field(nx, ny, seed):
    """Seeded smooth field on the unit square sampled at nx x ny cell centres
    (flattened, x fastest), |s| <= 1: four plane waves
    sin(2 pi (kx x + ky y) + theta) with integer wave numbers 1..4 and
    weights in [0.5, 1] (directions of derivative checks)."""
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid((np.arange(nx) + 0.5) / nx, (np.arange(ny) + 0.5) / ny)
    s, am = np.zeros_like(X), 0.0
    for _ in range(4):
        kx, ky = rng.integers(1, 5, size=2)
        th, a = rng.uniform(0, 2 * np.pi), rng.uniform(0.5, 1.0)
        s += a * np.sin(2 * np.pi * (kx * X + ky * Y) + th)
        am += a
    return (s / am).reshape(-1)


def random_smooth_state_case(dim=2, n=(12, 10, 1), seed=0, two_phase=True, cdi=1, diffusion=1,
                             bc=(0, 0, 0), amp=0.05, multi_pinf=False):
    """Small generic multi-phase multi-component case with smooth random fields
    (used for parity and derivative checks on tiny grids).  multi_pinf: the
    liquid phase holds two components of different P_inf (the stiffened
    liquid and water with the NASG constants of Table NASGMaterialParamters),
    the gas phase one ideal gas."""
    rng = np.random.default_rng(seed)
    dx = 1e-3
    liq = Material("liquid", LIQUID, 1816.0, 6.12, pinf=3.43e8, molar_mass=0.018, mu=8.9e-4)
    A = ideal_gas("A", 1.4, 0.029, mu=1.81e-5, Sc=1.0)
    B = ideal_gas("B", 1.667, 0.004, mu=1.96e-5, Sc=0.70)
    mats = [liq, A, B] if two_phase else [A, B]
    if multi_pinf:
        water = Material("water", LIQUID, 4185.0 / 1.0123, 1.0123, pinf=1.835e8, b=9.203e-4, q=-1.143e6,
                         molar_mass=0.018, mu=8.9e-4, Sc=1.0)
        mats = [liq, water, A]
    nn = tuple(n[d] if d < dim else 1 for d in range(3))
    shape = (nn[2], nn[1], nn[0])
    grids = np.meshgrid(*[(np.arange(nn[d]) + 0.5) / nn[d] for d in (2, 1, 0)], indexing="ij")
    Z, Yg, X = grids

    def field_(scale):
        out = np.zeros(shape)
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            out += np.sin(2 * math.pi * (k[0] * X + k[1] * Yg * (dim > 1) + k[2] * Z * (dim > 2)) + ph)
        return scale * out / 3.0

    eps = 1.5 * dx
    if two_phase:
        # off-centre droplet: no face sits on an exact extremum of phi
        c0 = (0.5 + 0.0317, 0.5 - 0.0211, 0.5 + 0.0123)
        dist = (0.3 - np.sqrt((X - c0[0]) ** 2 + ((Yg - c0[1]) ** 2 if dim > 1 else 0)
                              + ((Z - c0[2]) ** 2 if dim > 2 else 0))) * nn[0] * dx
        phil = _tanh_profile(dist, eps)
        phi = np.stack([phil, _tanh_profile(-dist, eps)])
        yA = 0.6 + field_(0.2)
        y = np.stack([np.ones(shape), yA, 1.0 - yA])
        if multi_pinf:
            y = np.stack([yA, 1.0 - yA, np.ones(shape)])
    else:
        phi = np.stack([np.zeros(shape), np.ones(shape)])
        yA = 0.5 + field_(0.3)
        y = np.stack([yA, 1.0 - yA])
    P = 1e5 * (1.0 + field_(amp))
    T = 300.0 * (1.0 + field_(amp))
    vel = np.stack([30.0 * field_(1.0) + 20.0 for _ in range(dim)])
    return Case("random_smooth", dim, nn, (dx, dx, dx), bc, bc, mats,
                default_opts(cdi=cdi if two_phase else 0, eps_cdi=eps, diffusion=diffusion),
                phi, y, P, T, vel, 1)
