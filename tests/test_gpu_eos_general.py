"""Several distinct P_inf on the GPU (the iterative pressure of Sec. 2.3):
parity of the HIP library with the oracle on states whose liquid phase mixes
a stiffened liquid and NASG water."""
import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs
from tests.test_gpu_parity import (ctx_of, field_scales, grouped_rel_l1, mask_u16, to_dev)

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CASES = {
    "1d_periodic": lambda: inputs.random_smooth_state_case(dim=1, n=(40, 1, 1), seed=11, multi_pinf=True),
    "2d_reflect": lambda: inputs.random_smooth_state_case(dim=2, n=(19, 13, 1), seed=12, bc=(2, 2, 2),
                                                          multi_pinf=True),
    "3d_mixed_bc": lambda: inputs.random_smooth_state_case(dim=3, n=(8, 7, 6), seed=13, bc=(1, 2, 0),
                                                           multi_pinf=True),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_init_state_and_dt_general_eos(name):
    case = CASES[name]()
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    c = ctx_of(case)
    Ug = c.init_state_from_case(case).cpu().numpy()
    rel = grouped_rel_l1(Ug, U0, o.ns, o.dim)
    assert np.all(rel <= 1e-14), rel.tolist()
    dt, g = o.compute_dt(U0)
    dtg, gg = c.mpmc_compute_dt(to_dev(U0))
    assert abs(float(dtg) / dt - 1) <= 1e-12 and abs(float(gg) / g - 1) <= 1e-12
    c.close()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("stage", [0, 2])
def test_rhs_parity_general_eos(name, stage):
    """One stage against the oracle: same face decisions, every field within
    1e-12 of its scale."""
    case = CASES[name]()
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    dt, g = o.compute_dt(U0)
    rk = [(0.0, 1.0, 1.0), (0.75, 0.25, 0.25), (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0)][stage]
    Uk = U0 + 0.5 * dt * o.rhs(U0, U0, (0.0, 1.0, 1.0), dt, g) if stage else U0.copy()
    Lo, _, mo = o.rhs(Uk, U0, rk, dt, g, with_mask=True)
    c = ctx_of(case)
    mask = torch.zeros(c.mask_size, dtype=torch.int16, device="cuda")
    Lg = c.mpmc_rhs(to_dev(Uk), to_dev(U0), rk, c.scalar(dt), c.scalar(g), mask=mask).cpu().numpy()
    c.close()
    nmis = int((mask_u16(mask) != mo).sum())
    assert nmis == 0, f"{nmis} face decisions differ"
    scale = field_scales(Uk, o.ns, o.dim)
    err = (dt * np.abs(Lg - Lo)).reshape(o.nv, -1).max(1) / scale
    assert np.all(err <= 1e-12), err.tolist()


@pytest.mark.parametrize("name,steps", [("1d_periodic", 30), ("2d_reflect", 10), ("3d_mixed_bc", 4)])
def test_multistep_parity_general_eos(name, steps):
    case = CASES[name]()
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    Uo = U0.copy()
    for _ in range(steps):
        o.step(Uo)
    c = ctx_of(case, raise_inadmissible=False)   # parity of a free run, decisions included
    Ug = to_dev(U0)
    for _ in range(steps):
        c.mpmc_rk3_step(Ug)
    c.close()
    rel = grouped_rel_l1(Ug.cpu().numpy(), Uo, o.ns, o.dim)
    assert np.all(rel <= 1e-11), rel.tolist()


def test_general_eos_rejected_by_mixed_form_adjoint_and_replay():
    from paper_2504_14063_amd import mpmc
    case = CASES["2d_reflect"]()
    with pytest.raises(mpmc.MpmcError):
        ctx_of(case, precision=1)
    c = ctx_of(case)
    U = c.init_state_from_case(case)
    dt, g = c.mpmc_compute_dt(U)
    with pytest.raises(mpmc.MpmcError):
        c.mpmc_adjoint_step(U, dt, g, torch.ones_like(U))
    with pytest.raises(mpmc.MpmcError):
        c.mpmc_rk3_step_replay(U, dt, g, c.new_masks())
    c.close()
