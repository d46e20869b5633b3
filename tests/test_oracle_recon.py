"""Pins of the oracle's reconstruction and Riemann pieces: WENO5-Z (exactness,
order, non-oscillation), the mass-fraction limiter of Sec. 3.3.1, and HLLC
(App. B) -- consistency, contact preservation, upwinding -- plus the Sod
shock tube against the textbook exact Riemann solution."""
import math

import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs
from tests import util


def cell_avg_poly(coef, a, b):
    """Exact average of sum coef[k] x^k over [a, b]."""
    P = np.polynomial.polynomial.Polynomial(coef).integ()
    return (P(b) - P(a)) / (b - a)


def test_weno_exact_for_quadratics():
    rng = np.random.default_rng(0)
    for _ in range(200):
        coef = rng.normal(size=3) * [1, 10, 100]
        h = 10 ** rng.uniform(-3, 0)
        f = [cell_avg_poly(coef, (k - 0.5) * h, (k + 0.5) * h) for k in range(-2, 3)]
        x = 0.5 * h
        exact = coef[0] + coef[1] * x + coef[2] * x * x
        assert abs(oracle.weno5z(f) - exact) <= 1e-12 * (abs(exact) + abs(coef).sum())


def test_weno_constant_and_linear_invariance():
    for c in [0.0, 1.0, -3.5, 1e5, 4.1e8]:
        assert oracle.weno5z([c] * 5) == pytest.approx(c, rel=1e-15, abs=0)
    f = np.array([0.1, 0.7, 0.2, 0.9, 0.4])
    v = oracle.weno5z(f)
    assert oracle.weno5z(-f) == pytest.approx(-v, rel=1e-14)
    assert oracle.weno5z(f + 10.0) == pytest.approx(v + 10.0, rel=1e-14)
    assert oracle.weno5z(3.0 * f) == pytest.approx(3.0 * v, rel=1e-14)


def test_weno_fifth_order_smooth():
    """Face value from cell averages of sin: error ~ h^5 at a generic point."""
    errs = []
    hs = [0.1, 0.05, 0.025, 0.0125]
    x0 = 0.3
    for h in hs:
        f = [(math.cos(x0 + (k - 0.5) * h) - math.cos(x0 + (k + 0.5) * h)) / h for k in range(-2, 3)]
        errs.append(abs(oracle.weno5z(f) - math.sin(x0 + 0.5 * h)))
    orders = [math.log(errs[i] / errs[i + 1], 2) for i in range(len(errs) - 1)]
    assert min(orders) > 4.5, orders


def test_weno_step_no_new_extrema():
    for f in ([0, 0, 0, 1, 1], [1, 1, 1, 0, 0], [0, 0, 1, 1, 1], [0, 1, 1, 1, 1]):
        v = oracle.weno5z(np.array(f, dtype=float))
        assert -1e-12 <= v <= 1 + 1e-12
    # upwind of a step the smooth stencil dominates
    assert abs(oracle.weno5z(np.array([0, 0, 0, 1, 1.0]))) < 1e-2


def test_ylimit_properties():
    rng = np.random.default_rng(1)
    for _ in range(500):
        ns = rng.integers(2, 6)
        Yc = rng.dirichlet(np.ones(ns))
        Ys = Yc + rng.normal(scale=0.05, size=ns)
        inert = rng.random(ns) < 0.3
        Ys[inert] = Yc[inert]
        Y0 = Ys.copy()
        out, br = oracle.ylimit(Ys, Yc)
        s0 = Y0.sum()
        if s0 == 1.0:
            assert br == 0
            continue
        lo = np.minimum(Y0, Yc)
        hi = np.maximum(Y0, Yc)
        if br != 0:
            assert abs(out.sum() - 1.0) < 1e-14
            assert np.all(out >= lo - 1e-15) and np.all(out <= hi + 1e-15)
        assert np.all(out[inert] == Y0[inert])
        assert br == (1 if s0 > 1 else 2) or br == 0


def make_gas_oracle(dim=1, mats=None):
    if mats is None:
        mats = [util.stiff_liquid(), inputs.ideal_gas("A", 1.4, 0.029), inputs.ideal_gas("B", 1.667, 0.004)]
    return oracle.Oracle(util.grid_dict(dim=dim), util.eos_dict(mats), inputs.default_opts()), mats


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_hllc_consistency(dim):
    o, mats = make_gas_oracle(dim)
    rng = np.random.default_rng(dim)
    for _ in range(30):
        yg = rng.uniform(0, 1)
        Y = [1 - yg, 0.5 * yg, 0.5 * yg]
        u, _ = o.state_from_PT(rng.uniform(5e4, 5e5), rng.uniform(250, 500), Y,
                               list(rng.uniform(-200, 200, size=dim)))
        F = o.hllc(u, u)
        Fp = o.euler_flux(u)
        assert np.allclose(F, Fp, rtol=1e-13, atol=1e-13 * np.abs(Fp).max())


def test_hllc_contact_and_supersonic():
    o, mats = make_gas_oracle(1)
    # contact: equal P and u, different composition/temperature
    uL, _ = o.state_from_PT(1e5, 300.0, [1.0, 0.0, 0.0], [50.0])
    uR, _ = o.state_from_PT(1e5, 400.0, [0.0, 0.3, 0.7], [50.0])
    F = o.hllc(uL, uR)
    Fp = o.euler_flux(uL)  # u > 0: upwind (left) physical flux
    assert np.allclose(F, Fp, rtol=1e-11, atol=1e-9)
    # supersonic to the right: F = F(U_L)
    uL, aL = o.state_from_PT(1e5, 300.0, [0.0, 1.0, 0.0], [900.0])
    uR, _ = o.state_from_PT(2e5, 350.0, [0.0, 1.0, 0.0], [950.0])
    assert 900.0 - aL > 0
    assert np.allclose(o.hllc(uL, uR), o.euler_flux(uL), rtol=1e-13)
    # mirror symmetry: swapping sides and reversing velocity flips the flux
    uL, _ = o.state_from_PT(1.3e5, 320.0, [0.2, 0.5, 0.3], [30.0])
    uR, _ = o.state_from_PT(0.8e5, 280.0, [0.0, 0.1, 0.9], [-20.0])
    F = o.hllc(uL, uR)
    mL = uL.copy(); mL[3] = -mL[3]
    mR = uR.copy(); mR[3] = -mR[3]
    G = o.hllc(mR, mL)
    expect = -F
    expect[3] = F[3]
    assert np.allclose(G, expect, rtol=1e-12, atol=1e-12 * np.abs(F).max())


# ----------------------------------------------------------------------------
# Sod shock tube against the exact solution (textbook two-shock/rarefaction
# pressure function, Newton for p*).
# ----------------------------------------------------------------------------
def exact_riemann_ideal(rl, ul, pl, rr, ur, pr, g, xi):
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def fk(p, rk, pk, ak):
        if p > pk:
            A, B = 2 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            q = math.sqrt(A / (p + B))
            return (p - pk) * q, q * (1 - (p - pk) / (2 * (B + p)))
        pr_ = (p / pk) ** ((g - 1) / (2 * g))
        return 2 * ak / (g - 1) * (pr_ - 1), 1 / (rk * ak) * (p / pk) ** (-(g + 1) / (2 * g))

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = fk(p, rl, pl, al)
        f2, d2 = fk(p, rr, pr, ar)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    f1, _ = fk(p, rl, pl, al)
    f2, _ = fk(p, rr, pr, ar)
    us = 0.5 * (ul + ur) + 0.5 * (f2 - f1)
    out = np.zeros((len(xi), 3))
    for i, s in enumerate(xi):
        if s < us:  # left of contact
            if p > pl:
                sl = ul - al * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
                if s < sl:
                    out[i] = rl, ul, pl
                else:
                    r = rl * ((p / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pl + 1))
                    out[i] = r, us, p
            else:
                shl = ul - al
                asl = al * (p / pl) ** ((g - 1) / (2 * g))
                stl = us - asl
                if s < shl:
                    out[i] = rl, ul, pl
                elif s > stl:
                    out[i] = rl * (p / pl) ** (1 / g), us, p
                else:
                    c = 2 / (g + 1) + (g - 1) / ((g + 1) * al) * (ul - s)
                    out[i] = rl * c ** (2 / (g - 1)), 2 / (g + 1) * (al + (g - 1) / 2 * ul + s), pl * c ** (2 * g / (g - 1))
        else:
            if p > pr:
                sr = ur + ar * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
                if s > sr:
                    out[i] = rr, ur, pr
                else:
                    r = rr * ((p / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pr + 1))
                    out[i] = r, us, p
            else:
                shr = ur + ar
                asr = ar * (p / pr) ** ((g - 1) / (2 * g))
                str_ = us + asr
                if s > shr:
                    out[i] = rr, ur, pr
                elif s < str_:
                    out[i] = rr * (p / pr) ** (1 / g), us, p
                else:
                    c = 2 / (g + 1) - (g - 1) / ((g + 1) * ar) * (ur - s)
                    out[i] = rr * c ** (2 / (g - 1)), 2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s), pr * c ** (2 * g / (g - 1))
    return out


def run_sod(n, tend=0.2):
    case = inputs.sod_1d(n)
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    t = 0.0
    while t < tend - 1e-15:
        dt, _ = o.compute_dt(U)
        dt = min(dt, tend - t)
        o.step(U, dt=dt)
        t += dt
    x = (np.arange(n) + 0.5) / n
    ex = exact_riemann_ideal(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4, (x - 0.5) / tend)
    return U[:n], ex[:, 0]


def test_sod_exact_solution():
    errs = {}
    for n in (100, 200, 400, 800):
        rho, ex = run_sod(n)
        errs[n] = np.abs(rho - ex).mean()
    assert errs[400] <= 5e-3, errs
    orders = [math.log(errs[a] / errs[b], 2) for a, b in ((100, 200), (200, 400), (400, 800))]
    assert min(orders) >= 0.8, (errs, orders)
