"""Pins of the oracle's scheme variants (WENO5-JS, TENO5; cited in Sec. 4 as
alternatives to the default WENO5-Z) against properties fixed by their
definitions and against the paper's droplet-advection table."""
import numpy as np
import pytest

import oracle
from tests import util
from tests.test_oracle_scheme import drop_advection_case, prims

SCHEMES = {"weno5z": lambda f: oracle.weno5z(f), "weno5js": lambda f: oracle.weno5js(f, 1e-6, 2),
           "teno5": lambda f: oracle.teno5(f)}


def cell_averages(coef, h=0.1, x0=0.3):
    """Cell averages over cells i-2..i+2 of sum_k coef[k] x^k, and the value
    of that polynomial at the face i+1/2."""
    P = np.polynomial.polynomial.Polynomial(coef)
    I = P.integ()
    lo = x0 + (np.arange(5) - 2.5) * h
    return np.array([(I(a + h) - I(a)) / h for a in lo]), P(x0 + 0.5 * h)


@pytest.mark.parametrize("scheme", sorted(SCHEMES))
def test_exact_on_quadratics(scheme):
    """Each substencil reproduces quadratics, so every convex combination does."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        f, exact = cell_averages(rng.uniform(-1, 1, 3))
        assert abs(SCHEMES[scheme](f) - exact) <= 1e-13, scheme


def test_teno5_recovers_the_linear_scheme_on_quartics():
    """Smooth data: no substencil is cut, the weights are the linear ones and
    the five-point reconstruction is exact up to degree 4 (WENO5-JS, whose
    weights only approach the linear ones, is not)."""
    rng = np.random.default_rng(2)
    worst_js = 0.0
    for _ in range(20):
        f, exact = cell_averages(rng.uniform(-1, 1, 5))
        assert abs(oracle.teno5(f) - exact) <= 1e-12
        worst_js = max(worst_js, abs(oracle.weno5js(f, 1e-6, 2) - exact))
    assert worst_js > 1e-9


def test_teno5_cuts_substencils_across_a_jump():
    """A jump inside the stencil cuts the substencils that cross it off
    entirely: the face value is that of the smooth substencil."""
    assert oracle.teno5([0.0, 0.0, 0.0, 1.0, 1.0]) == 0.0
    assert oracle.teno5([0.0, 0.0, 1.0, 1.0, 1.0]) == 1.0
    assert abs(oracle.teno5([2.0, 2.0, 2.0, 5.0, 5.0]) - 2.0) <= 1e-15
    # WENO5-JS only makes the crossing weights small
    assert 0.0 < abs(oracle.weno5js([0.0, 0.0, 0.0, 1.0, 1.0], 1e-6, 2)) < 1e-10


@pytest.mark.slow
@pytest.mark.parametrize("scheme,over", [("weno5js", dict(weno=1, weno_eps=1e-6, weno_p=2)),
                                         ("teno5", dict(weno=2, weno_eps=1e-40))])
def test_iec_paper_droplet_advection_variants(scheme, over):
    """The paper's droplet advection (Table DropAdvectionIECResults) with the
    variant schemes: max relative P, T, u errors of the order the paper
    prints for the same schemes, and no limiter firing."""
    ref = util.golden()[f"iec_drop_advection_{scheme}"]
    g = util.golden()["iec_drop_advection_setup"]
    case = drop_advection_case(g["cells"])
    case.opts = dict(case.opts, **over)
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    t, tend = 0.0, 1.0 / g["u"]
    cnt = np.zeros(oracle.NCNT, dtype=np.uint64)
    while t < tend:
        dt, _ = o.compute_dt(U)
        dt = min(dt, tend - t)
        o.step(U, dt=dt, counters=cnt)
        t += dt
    P, T, u = prims(o, U)
    eP = np.abs(P / g["P"] - 1).max()
    eT = np.abs(T / g["T"] - 1).max()
    eu = np.abs(u / g["u"] - 1).max()
    assert eP <= 5 * ref["max_rel_P"] and eT <= 5 * ref["max_rel_T"] and eu <= 5 * ref["max_rel_u"], (eP, eT, eu)
    assert cnt[:5].sum() == 0
