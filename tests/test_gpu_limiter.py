"""GPU parity of the limiter decisions of Sec. 3.3 on states that force
them (tests/golden/forced_limiter_states.json: a temperature fallback, a
pressure fallback, the first-order flux, the dropped regularization flux),
and failure detection through the C ABI (an inadmissible cell is counted by
mpmc_stats and reported by the next call's return)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs
from tests.forced_cases import BITS, N, build_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
RK = [(0.0, 1.0, 1.0), (0.75, 0.25, 0.25), (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0)]


def forced(kind):
    with open(os.path.join(HERE, "golden", "forced_limiter_states.json")) as fh:
        return json.load(fh)[kind]


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ctx_of(case):
    from paper_2504_14063_amd import mpmc
    return mpmc.Context.from_case(case)


@pytest.mark.parametrize("kind", ["T", "P", "FB", "DROP"])
@pytest.mark.parametrize("stage", [0, 2])
def test_forced_decisions_parity(kind, stage):
    """The same face decisions as the oracle on every face (the forced one
    included) and the same right-hand side within 1e-12 of the state."""
    f = forced(kind)
    case = build_case(f)
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    dt, g = o.compute_dt(U0)
    Uk = U0 + 0.5 * dt * o.rhs(U0, U0, RK[0], dt, g) if stage else U0.copy()
    Lo, cnt, mo = o.rhs(Uk, U0, RK[stage], dt, g, with_mask=True)
    if stage == 0:
        assert np.any(mo & BITS[kind])
    c = ctx_of(case)
    mask = torch.zeros(c.mask_size, dtype=torch.int16, device="cuda")
    Lg = c.mpmc_rhs(to_dev(Uk), to_dev(U0), RK[stage], c.scalar(dt), c.scalar(g), mask=mask).cpu().numpy()
    mg = mask.cpu().numpy().view(np.uint16)
    print(kind, "stage", stage, "oracle", mo.tolist(), "gpu", mg.tolist())
    assert np.array_equal(mg, mo)
    sc = np.abs(Uk.reshape(o.nv, N)).max(1)
    err = (dt * np.abs(Lg - Lo)).reshape(o.nv, N).max(1) / np.maximum(sc, 1e-300)
    assert np.all(err <= 1e-12), err
    c.close()


@pytest.mark.parametrize("kind", ["T", "P", "FB", "DROP"])
def test_forced_decisions_step_parity(kind):
    """One SSP-RK3 step from the forced states: the three stage masks equal
    the oracle's and the states agree within 1e-12 per variable."""
    f = forced(kind)
    case = build_case(f)
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    Uo = U0.copy()
    dt, g, mo = o.step(Uo, with_mask=True)
    c = ctx_of(case)
    Ug = to_dev(U0)
    masks = c.new_masks()
    c.mpmc_rk3_step(Ug, dt_in=c.scalar(dt), gamma_in=c.scalar(g), masks=masks)
    mg = masks.cpu().numpy().view(np.uint16)
    assert np.array_equal(mg, mo)
    sc = np.maximum(np.abs(Uo.reshape(o.nv, N)).max(1), np.abs(Uo.reshape(o.nv, N)[:3]).sum(0).max() * 1e-300)
    d = np.abs(Ug.cpu().numpy() - Uo).reshape(o.nv, N).max(1)
    assert np.all(d <= 1e-12 * np.where(sc > 0, sc, 1.0)), (d, sc)
    c.close()


@pytest.mark.parametrize("where,value", [("partial_density", -1e-3), ("energy", float("nan"))])
def test_failure_detection(where, value):
    """A stage input cell with a negative partial density or a NaN: counted
    by mpmc_stats (inadmissible_cells, status EINADMISSIBLE) and reported by
    the return of the next call that enqueues work, once; mpmc_stats with
    reset clears it.  An admissible run reports nothing."""
    from paper_2504_14063_amd import mpmc
    case = inputs.random_smooth_state_case(dim=2, n=(12, 9, 1), seed=4)
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    c = ctx_of(case)
    Ug = to_dev(U)
    c.mpmc_stats(reset=True)
    c.mpmc_rk3_step(Ug)
    torch.cuda.synchronize()
    c.mpmc_compute_dt(Ug)
    st = c.mpmc_stats(reset=True)
    assert st["code"] == 0 and st["inadmissible_cells"] == 0
    V = U.copy()
    V[5 if where == "partial_density" else (o.nv - 1) * o.ncell + 17] = value
    cnt = np.zeros(oracle.NCNT, dtype=np.uint64)
    o.step(V.copy(), counters=cnt)
    assert o.status == oracle.EINADMISSIBLE
    Vg = to_dev(V)
    dt, gm = c.scalar(1e-9), c.scalar(1.0)
    # reported by the launching call itself when a kernel that met it has
    # completed when the call returns, else by the next call; once reported
    # the flag is clear until a kernel meets trouble again
    c.raise_inadmissible = False
    c.mpmc_rk3_step(Vg, dt_in=dt, gamma_in=gm)
    torch.cuda.synchronize()
    c.mpmc_compute_dt(Ug)
    n1 = c.inadmissible_reports
    c.mpmc_compute_dt(Ug)
    assert n1 >= 1 and c.inadmissible_reports == n1
    c.raise_inadmissible = True
    with pytest.raises(mpmc.Inadmissible):
        c.mpmc_rk3_step(Vg, dt_in=dt, gamma_in=gm)
        torch.cuda.synchronize()
        c.mpmc_compute_dt(Ug)
    st = c.mpmc_stats()
    assert st["code"] == mpmc.MPMC_EINADMISSIBLE and st["inadmissible_cells"] >= 1
    c.mpmc_stats(reset=True)
    c.mpmc_rk3_step(Ug)
    torch.cuda.synchronize()
    c.mpmc_compute_dt(Ug)
    assert c.mpmc_stats()["code"] == 0
    c.close()
