"""Scheme variants on the GPU (WENO5-JS, TENO5, TENO6, cited beside WENO5-Z in
Sec. 4 and Table DropAdvectionIECResults) and the five-equation basis (the
negative control of Table DropAdvectionNoIECResults): parity of the HIP
library with the oracle, and the paper's droplet advection run to the end on
the GPU."""
import numpy as np
import pytest

import oracle
from tests import util
from tests.test_gpu_parity import (SMALL_CASES, ctx_of, field_scales, grouped_rel_l1, mask_u16,
                                   to_dev)
from tests.test_oracle_scheme import drop_advection_case

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SCHEMES = {"weno5js": dict(weno=1, weno_eps=1e-6, weno_p=2), "teno5": dict(weno=2, weno_eps=1e-40),
           "teno6": dict(weno=3, weno_eps=1e-40)}

VARIANT_CASES = ["1d_two_phase_cdi_periodic", "1d_gas_mix_outflow", "2d_all_reflect", "3d_all_mixed_bc",
                 "sod", "shock_droplet_small", "droplet3d_small"]


def with_scheme(case, scheme):
    case.opts = dict(case.opts, **SCHEMES[scheme])
    return case


@pytest.mark.parametrize("scheme", sorted(SCHEMES))
@pytest.mark.parametrize("name", VARIANT_CASES)
def test_rhs_parity_scheme_variant(name, scheme):
    """One stage against the oracle: same face decisions, every field within
    1e-12 of its scale; the variant's result differs from WENO5-Z's far above
    that bound (the option reaches the kernel), except on Sod's
    piecewise-constant data, where every scheme takes the substencils clear of
    the jump and the results agree to a few 1e-11."""
    case = with_scheme(SMALL_CASES[name](), scheme)
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    dt, g = o.compute_dt(U0)
    rk = (0.0, 1.0, 1.0)
    Lo, _, mo = o.rhs(U0, U0, rk, dt, g, with_mask=True)
    c = ctx_of(case)
    mask = torch.zeros(c.mask_size, dtype=torch.int16, device="cuda")
    Lg = c.mpmc_rhs(to_dev(U0), to_dev(U0), rk, c.scalar(dt), c.scalar(g), mask=mask).cpu().numpy()
    c.close()
    scale = field_scales(U0, o.ns, o.dim)
    nmis = int((mask_u16(mask) != mo).sum())
    assert nmis == 0, f"{nmis} face decisions differ"
    err = (dt * np.abs(Lg - Lo)).reshape(o.nv, -1).max(1) / scale
    assert np.all(err <= 1e-12), err.tolist()
    if name == "sod":
        return
    cz = ctx_of(case, weno=0, weno_eps=1e-40, weno_p=1)
    Lz = cz.mpmc_rhs(to_dev(U0), to_dev(U0), rk, cz.scalar(dt), cz.scalar(g)).cpu().numpy()
    cz.close()
    dz = float(((dt * np.abs(Lz - Lg)).reshape(o.nv, -1).max(1) / scale).max())
    assert dz > 1e-9, dz


@pytest.mark.parametrize("scheme", sorted(SCHEMES))
@pytest.mark.parametrize("name,steps", [("shock_bubble_small", 20), ("1d_two_phase_cdi_periodic", 30),
                                        ("3d_all_mixed_bc", 4)])
def test_multistep_parity_scheme_variant(name, steps, scheme):
    """Several steps against the oracle, within 1e-11 relative L1.  The cases
    are ones where the oracle itself carries a 1e-15 relative perturbation of
    the initial state through the same steps below 1e-12.  The small
    shock-droplet is not one under WENO5-JS: there the oracle amplifies such a
    perturbation about fifty-fold per step (1e-3 after 20 steps), so only its
    single-stage parity is a meaningful check."""
    case = with_scheme(SMALL_CASES[name](), scheme)
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    Uo = U0.copy()
    for _ in range(steps):
        o.step(Uo)
    c = ctx_of(case)
    Ug = to_dev(U0)
    for _ in range(steps):
        c.mpmc_rk3_step(Ug)
    c.close()
    rel = grouped_rel_l1(Ug.cpu().numpy(), Uo, o.ns, o.dim)
    assert np.all(rel <= 1e-11), rel.tolist()


@pytest.mark.parametrize("scheme", sorted(SCHEMES))
def test_droplet_advection_flow_through(scheme):
    """The paper's 1D water droplet in air (100 cells, CDI on) for one
    flow-through on the GPU: the first 2000 steps within 1e-11 relative L1 of
    the oracle, then the max relative P, T, u errors at the end of the order
    the paper prints for the same scheme, with no limiter firing."""
    ref = util.golden()[f"iec_drop_advection_{scheme}"]
    gs = util.golden()["iec_drop_advection_setup"]
    case = with_scheme(drop_advection_case(gs["cells"]), scheme)
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    c = ctx_of(case)
    Ug = to_dev(U0)
    Uo = U0.copy()
    nchk = 2000
    for _ in range(nchk):
        o.step(Uo)
        c.mpmc_rk3_step(Ug)
    rel = grouped_rel_l1(Ug.cpu().numpy(), Uo, o.ns, o.dim)
    assert np.all(rel <= 1e-11), rel.tolist()
    c.mpmc_stats(reset=True)
    Ug = to_dev(U0)
    t, tend = 0.0, 1.0 / gs["u"]
    dt_in = c.scalar()
    while t < tend:
        dt, g = c.mpmc_compute_dt(Ug)
        h = min(float(dt), tend - t)
        dt_in.fill_(h)
        c.mpmc_rk3_step(Ug, dt_in=dt_in, gamma_in=g)
        t += h
    st = c.mpmc_stats()
    c.close()
    U = Ug.cpu().numpy()
    n = o.ncell
    P = np.array([o.equilibrium(U[i::n])["P"] for i in range(n)])
    T = np.array([o.equilibrium(U[i::n])["T"] for i in range(n)])
    u = U[o.ns * n:(o.ns + 1) * n] / U[:o.ns * n].reshape(o.ns, n).sum(0)
    eP = np.abs(P / gs["P"] - 1).max()
    eT = np.abs(T / gs["T"] - 1).max()
    eu = np.abs(u / gs["u"] - 1).max()
    assert eP <= 5 * ref["max_rel_P"] and eT <= 5 * ref["max_rel_T"] and eu <= 5 * ref["max_rel_u"], (eP, eT, eu)
    assert st["faces_T"] + st["faces_P"] + st["fallback"] + st["cdi_drop"] + st["unrecoverable"] == 0, st


def test_variants_rejected_by_mixed_form_and_adjoint():
    from paper_2504_14063_amd import mpmc
    case = with_scheme(SMALL_CASES["2d_all_periodic"](), "teno5")
    with pytest.raises(mpmc.MpmcError):
        ctx_of(case, precision=1)
    c = ctx_of(case)
    U = c.init_state_from_case(case)
    dt, g = c.mpmc_compute_dt(U)
    with pytest.raises(mpmc.MpmcError):
        c.mpmc_adjoint_step(U, dt, g, torch.ones_like(U))
    c.close()


BASIS5 = {"weno5z_eps1e-6": dict(basis=1, weno=0, weno_eps=1e-6, weno_p=2),
          "weno5js": dict(basis=1, weno=1, weno_eps=1e-6, weno_p=2),
          "teno5": dict(basis=1, weno=2, weno_eps=1e-40)}


@pytest.mark.parametrize("scheme", sorted(BASIS5))
@pytest.mark.parametrize("name", ["1d_two_phase_cdi_periodic", "2d_all_reflect", "3d_all_mixed_bc",
                                  "shock_droplet_small", "droplet3d_small"])
def test_rhs_parity_five_equation_basis(name, scheme):
    """The five-equation basis [rho Y, u, P] (the negative control of Sec.
    4.2.2): one stage against the oracle, same decisions, within 1e-12."""
    case = SMALL_CASES[name]()
    case.opts = dict(case.opts, **BASIS5[scheme])
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    dt, g = o.compute_dt(U0)
    rk = (0.0, 1.0, 1.0)
    Lo, _, mo = o.rhs(U0, U0, rk, dt, g, with_mask=True)
    c = ctx_of(case)
    mask = torch.zeros(c.mask_size, dtype=torch.int16, device="cuda")
    Lg = c.mpmc_rhs(to_dev(U0), to_dev(U0), rk, c.scalar(dt), c.scalar(g), mask=mask).cpu().numpy()
    c.close()
    nmis = int((mask_u16(mask) != mo).sum())
    assert nmis == 0, f"{nmis} face decisions differ"
    scale = field_scales(U0, o.ns, o.dim)
    err = (dt * np.abs(Lg - Lo)).reshape(o.nv, -1).max(1) / scale
    assert np.all(err <= 1e-12), err.tolist()


@pytest.mark.parametrize("name,steps", [("shock_bubble_small", 20), ("1d_two_phase_cdi_periodic", 30),
                                        ("3d_all_mixed_bc", 4)])
def test_multistep_parity_five_equation_basis(name, steps):
    case = SMALL_CASES[name]()
    case.opts = dict(case.opts, **BASIS5["weno5z_eps1e-6"])
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    Uo = U0.copy()
    for _ in range(steps):
        o.step(Uo)
    c = ctx_of(case)
    Ug = to_dev(U0)
    for _ in range(steps):
        c.mpmc_rk3_step(Ug)
    c.close()
    rel = grouped_rel_l1(Ug.cpu().numpy(), Uo, o.ns, o.dim)
    assert np.all(rel <= 1e-11), rel.tolist()


def test_five_equation_basis_droplet_advection_on_gpu():
    """The negative control run to one flow-through on the GPU (WENO5-Z,
    eps = 1e-6, p = 2): P, T, u errors of the order of the paper's WENO5Z row
    of Table DropAdvectionNoIECResults (within 5x), orders of magnitude above
    the proposed basis.  Not compared with the oracle state by state: the
    oracle itself carries a 1e-15 perturbation of the initial state to 1e-6
    within 200 steps of this run (the IEC error grows from round-off)."""
    ref = util.golden()["iec_drop_advection_5eq_weno5z"]
    gs = util.golden()["iec_drop_advection_setup"]
    case = drop_advection_case(gs["cells"])
    case.opts = dict(case.opts, **BASIS5["weno5z_eps1e-6"])
    o = oracle.Oracle.from_case(case)
    c = ctx_of(case)
    Ug = to_dev(o.init_state(case))
    t, tend = 0.0, 1.0 / gs["u"]
    dt_in = c.scalar()
    c.mpmc_stats(reset=True)
    while t < tend:
        dt, g = c.mpmc_compute_dt(Ug)
        h = min(float(dt), tend - t)
        dt_in.fill_(h)
        c.mpmc_rk3_step(Ug, dt_in=dt_in, gamma_in=g)
        t += h
    st = c.mpmc_stats()
    c.close()
    U = Ug.cpu().numpy()
    n = o.ncell
    P = np.array([o.equilibrium(U[i::n])["P"] for i in range(n)])
    T = np.array([o.equilibrium(U[i::n])["T"] for i in range(n)])
    u = U[o.ns * n:(o.ns + 1) * n] / U[:o.ns * n].reshape(o.ns, n).sum(0)
    e = (np.abs(P / gs["P"] - 1).max(), np.abs(T / gs["T"] - 1).max(), np.abs(u / gs["u"] - 1).max())
    r = (ref["max_rel_P"], ref["max_rel_T"], ref["max_rel_u"])
    assert all(x / 5 <= y <= 5 * x for x, y in zip(r, e)), e
    assert st["faces_T"] + st["faces_P"] + st["fallback"] + st["unrecoverable"] == 0, st


def test_five_equation_basis_rejected_by_mixed_form_and_adjoint():
    from paper_2504_14063_amd import mpmc
    case = SMALL_CASES["2d_all_periodic"]()
    case.opts = dict(case.opts, basis=1)
    with pytest.raises(mpmc.MpmcError):
        ctx_of(case, precision=1)
    c = ctx_of(case)
    U = c.init_state_from_case(case)
    dt, g = c.mpmc_compute_dt(U)
    with pytest.raises(mpmc.MpmcError):
        c.mpmc_adjoint_step(U, dt, g, torch.ones_like(U))
    c.close()
