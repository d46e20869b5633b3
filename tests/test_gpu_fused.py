"""The fused RK step (each direction's face sweep also takes the divergence
of its fluxes, the last one the RK combination of Eq. SSPRK3) against the
split layout (face flux arrays, then a separate combination pass): the same
bits for the states, the face decisions and the limiter counters, on grids
whose extents leave ragged tiles in every direction, every boundary type,
both precisions, the scheme variants, held inflow cells, the frozen-decision
replay and the recorded stages."""
import pytest

from paper_2504_14063_amd import inputs
from tests.test_gpu_nscbc import with_targets
from tests.test_gpu_parity import ctx_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rs(**kw):
    return lambda: inputs.random_smooth_state_case(**kw)


def mach100_small():
    return inputs.mach100_water_column_2d(nx=256, ny=129, dx=4.0 / 256)


CASES = {
    "1d_600": (rs(dim=1, n=(600, 1, 1), seed=1, bc=(1, 1, 1)), {}, 8),
    "2d_periodic_wall": (rs(dim=2, n=(37, 70, 1), seed=2, bc=(0, 2, 0)), {}, 6),
    "3d_mixed_bc": (rs(dim=3, n=(21, 33, 64), seed=3, bc=(2, 0, 1)), {}, 4),
    "3d_mixed_precision": (rs(dim=3, n=(19, 40, 35), seed=4, bc=(0, 1, 2)), dict(precision=1), 4),
    "2d_teno5_viscous": (rs(dim=2, n=(45, 66, 1), seed=5, bc=(1, 2, 0)), dict(weno=2, viscous=1), 5),
    "2d_five_eq_basis": (rs(dim=2, n=(33, 40, 1), seed=6, bc=(0, 0, 0)), dict(basis=1), 5),
    "3d_multi_pinf": (rs(dim=3, n=(17, 22, 40), seed=7, bc=(1, 1, 1), multi_pinf=True), {}, 4),
    "2d_characteristic": (lambda: with_targets(inputs.random_smooth_state_case(
        dim=2, n=(40, 50, 1), seed=8, bc=(3, 3, 0)), 0.4), {}, 6),
    "water_inflow_1d": (lambda: inputs.water_inflow_1d(300), {}, 60),
    "mach100_256x129": (mach100_small, {}, 30),
    "droplet_3d_40": (lambda: inputs.droplet_crossflow_3d(n=40, steps=1), {}, 3),
}


def run(case, opts, steps, layout):
    c = ctx_of(case, raise_inadmissible=False, step_layout=layout, **opts)
    U = c.init_state_from_case(case)
    held = case.extra.get("held")
    if held is not None:
        c.mpmc_set_held_cells(held, inputs.held_values(case, U.cpu().numpy()))
    dt_in = c.scalar(case.extra["dt"]) if "dt" in case.extra else None
    g_in = None
    if dt_in is not None:
        _, g_in = c.mpmc_compute_dt(U)
    masks = []
    for _ in range(steps):
        m = torch.zeros(3 * c.mask_size, dtype=torch.int16, device="cuda")
        c.mpmc_rk3_step(U, dt_in=dt_in, gamma_in=g_in, masks=m)
        masks.append(m)
    torch.cuda.synchronize()
    st = c.mpmc_stats()
    c.close()
    return U, torch.stack(masks), st


@pytest.mark.parametrize("name", sorted(CASES))
def test_fused_matches_split(name):
    make, opts, steps = CASES[name]
    case = make()
    Ua, ma, sa = run(case, opts, steps, 1)
    Ub, mb, sb = run(case, opts, steps, 2)
    print(name, sa)
    assert torch.equal(ma, mb)
    assert torch.equal(Ua.view(torch.int64), Ub.view(torch.int64))
    assert sa == sb


def test_fused_replay_and_stages_match_split():
    """Frozen-decision replay and the recorded step (stage states handed
    back) in both layouts."""
    case = inputs.random_smooth_state_case(dim=3, n=(23, 36, 33), seed=9, bc=(1, 2, 0))
    res = []
    for layout in (1, 2):
        c = ctx_of(case, step_layout=layout)
        U0 = c.init_state_from_case(case)
        dt, g = c.mpmc_compute_dt(U0)
        masks = torch.zeros(3 * c.mask_size, dtype=torch.int16, device="cuda")
        U = U0.clone()
        c.mpmc_rk3_step(U, dt_in=dt, gamma_in=g, masks=masks)
        Ur = U0.clone()
        c.mpmc_rk3_step_replay(Ur, dt, g, masks)
        Us = U0.clone()
        s1, s2 = torch.empty_like(U0), torch.empty_like(U0)
        ms = torch.zeros_like(masks)
        c.mpmc_rk3_step_stages(Us, dt, g, s1, s2, ms)
        torch.cuda.synchronize()
        c.close()
        assert torch.equal(Ur, U) and torch.equal(Us, U) and torch.equal(ms, masks)
        res.append((U, s1, s2, masks))
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_rejects_bad_step_layout():
    from paper_2504_14063_amd import mpmc
    case = inputs.random_smooth_state_case(dim=1, n=(20, 1, 1), seed=1, bc=(1, 1, 1))
    with pytest.raises(mpmc.MpmcError):
        ctx_of(case, step_layout=3)
