"""Held inflow cells on the GPU (mpmc_set_held_cells) and the Mach-100 water
column of Sec. 4.2.4: parity with the oracle with its decisions replayed,
the one-dimensional inflow against the exact solution, and the paper-size
run (2048 x 1025, constant dt 7.5e-4 us, to 6 us) completing without
failure, as the paper reports for its positivity-preserving procedure."""
import numpy as np
import pytest

import oracle
from oracle import riemann
from paper_2504_14063_amd import inputs
from paper_2504_14063_amd.mpmc import MpmcError
from tests.test_gpu_parity import ctx_of, grouped_rel_l1, to_dev
from tests.test_oracle_inflow import air_shock_speed, inflow_errors

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def held_ctx(case, U0):
    c = ctx_of(case, raise_inadmissible=False)   # unrecoverable faces are counted and checked
    c.mpmc_set_held_cells(case.extra["held"], inputs.held_values(case, U0))
    return c


def replay_run(case, steps=None, t_end=None, dt_fixed=None):
    """The oracle steps the case (held cells set) and the GPU replays its dt,
    Gamma and decisions; also a free-running GPU copy at the same dt, Gamma.
    Returns (U0, oracle U, replayed GPU U, free GPU U, GPU counters)."""
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    o.set_held(case.extra["held"], U0)
    c = held_ctx(case, U0)
    Uo, Ur, Uf = U0.copy(), to_dev(U0), to_dev(U0)
    c.mpmc_stats(reset=True)
    t, k = 0.0, 0
    while (steps is not None and k < steps) or (t_end is not None and t < t_end):
        dt, g = o.compute_dt(Uo)
        if dt_fixed is not None:
            dt = dt_fixed
        if t_end is not None:
            dt = min(dt, t_end - t)
        _, _, mo = o.step(Uo, dt=dt, gamma=g, with_mask=True)
        c.mpmc_rk3_step_replay(Ur, c.scalar(dt), c.scalar(g), torch.from_numpy(mo.view(np.int16)).cuda())
        c.mpmc_rk3_step(Uf, dt_in=c.scalar(dt), gamma_in=c.scalar(g))
        t += dt
        k += 1
    st = c.mpmc_stats()
    c.close()
    return U0, Uo, Ur.cpu().numpy(), Uf.cpu().numpy(), st


def test_water_inflow_1d_replay_parity_and_exact_solution():
    """The 1D Mach-100 inflow (200 cells): over the first 300 steps, with the
    oracle's decisions replayed, the GPU state is within 1e-11 relative L1 of
    the oracle's and the held cell keeps its values bit for bit.  Longer
    replays are not well conditioned: the air left at the floor behind the
    inlet weighs 1e-8 kg/m^3 against 1e3 of water, so a 1e-11 difference
    of the total density is as large as the trace itself, and a replayed
    decision can then meet an inadmissible trace state (the replay reaches
    one at step 1878; the free-running GPU run does not).  Free-running until
    the air shock has crossed 70 % of the domain, the GPU's P and u approach
    the exact solution under refinement as the oracle's do."""
    case = inputs.water_inflow_1d(200)
    L, R = riemann.Side(*case.extra["left"]), riemann.Side(*case.extra["right"])
    tend = 0.7 / air_shock_speed(L, R)
    U0, Uo, Ur, Uf, st = replay_run(case, steps=300)
    n = case.ncell
    rel = grouped_rel_l1(Ur, Uo, case.ns, case.dim)
    print("replayed", rel.tolist(), "free", grouped_rel_l1(Uf, Uo, case.ns, case.dim).tolist())
    assert np.all(rel <= 1e-11), rel.tolist()
    assert np.array_equal(Ur[0::n], U0[0::n]) and np.array_equal(Uf[0::n], U0[0::n])
    assert st["unrecoverable"] == 0 and np.isfinite(Uf).all()
    errs = []
    for nn in (200, 400):
        cs = inputs.water_inflow_1d(nn)
        o = oracle.Oracle.from_case(cs)
        U0 = o.init_state(cs)
        c = held_ctx(cs, U0)
        U = to_dev(U0)
        t = 0.0
        dt_in = c.scalar()
        while t < tend:
            dt, g = c.mpmc_compute_dt(U)
            h = min(float(dt), tend - t)
            dt_in.fill_(h)
            c.mpmc_rk3_step(U, dt_in=dt_in, gamma_in=g)
            t += h
        assert c.mpmc_stats()["unrecoverable"] == 0
        c.close()
        Uh = U.cpu().numpy()
        assert np.isfinite(Uh).all()
        errs.append(inflow_errors(cs, o, Uh, tend))
    print("GPU errors vs exact", errs)
    assert errs[1][0] < 0.85 * errs[0][0] and errs[1][1] < 0.85 * errs[0][1], errs


def test_mach100_column_coarse_parity():
    """The water column's geometry on 1/16 m cells (64 x 33), 40 steps at the
    paper's dt scaled with the cell size: replayed decisions within 1e-11."""
    case = inputs.mach100_water_column_2d(64, 33, dx=1.0 / 16.0)
    U0, Uo, Ur, Uf, st = replay_run(case, steps=40, dt_fixed=case.extra["dt"] * 32.0)
    rel = grouped_rel_l1(Ur, Uo, case.ns, case.dim)
    print("replayed", rel.tolist(), "free", grouped_rel_l1(Uf, Uo, case.ns, case.dim).tolist())
    assert np.all(rel <= 1e-11), rel.tolist()
    assert st["unrecoverable"] == 0


def test_mach100_water_column_paper_size():
    """2048 x 1025 cells, dt 7.5e-4 us, 8000 steps (6 us) run to the end:
    the state finite, the held inlet unchanged, every stage state admissible
    (no inadmissible cell), the water mass gained within 2 % of the water the
    inlet faces admit (rho Y u per held row, every wave downstream; measured
    +1.4 %: the held edge cells also refill the water that the
    regularization diffuses into their air neighbours across the column's
    edges), and the column's head (furthest cell with water mass fraction
    above 1/2) between 0.6 and 1.1 times the inflow speed times t (measured
    0.927 m against 0.9 m).

    Unrecoverable faces (the first-order fallback's pseudo-state still
    inadmissible): 55-130 of 1.6e10 face evaluations (the count and places
    move with bit-level changes of the kernels' rounding), mostly on the
    column's edge rows 56-59 cells behind the inlet from step ~1060, some
    inside the column and near its head later.  Cause, reproduced with the
    oracle on the GPU's pre-step state around such faces: water compressed
    to within 2e-4 of its co-volume at ~10 GPa, where HLLC's star state
    compresses past v = b and the pseudo-state fails only the co-volume
    condition 1 - sum rhoY_c b_c > 0 (the cells themselves stay admissible;
    test_oracle_limiter.py pins the mechanism).  Checked here for every such
    face: its cells' co-volume margin before the step is below 5e-3, and no
    cell is ever inadmissible; the count is capped at a few hundred."""
    case = inputs.mach100_water_column_2d()
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    c = held_ctx(case, U0)
    U = to_dev(U0)
    dt, steps = case.extra["dt"], 8000
    dt_d = c.scalar(dt)
    nx, ny = case.n[0], case.n[1]
    nfx = (nx + 1) * ny
    masks = c.new_masks()
    where, margins = [], []
    w = [k for k, m in enumerate(case.materials) if m.phase == inputs.LIQUID][0]
    bw = case.materials[w].b
    Uprev = torch.empty_like(U)
    c.mpmc_stats(reset=True)
    for k in range(steps):
        Uprev.copy_(U)
        _, g = c.mpmc_compute_dt(U)
        c.mpmc_rk3_step(U, dt_in=dt_d, gamma_in=g, masks=masks)
        m = masks.view(3, -1)
        bad = torch.nonzero((m & 64) != 0)
        if bad.shape[0]:
            rYw = Uprev.view(case.nv, ny, nx)[w]
            for s, fi in bad.cpu().numpy().tolist():
                d, (i, j) = (0, (fi % (nx + 1), fi // (nx + 1))) if fi < nfx else (1, ((fi - nfx) % nx, (fi - nfx) // nx))
                where.append((k, d, i, j))
                # the two cells of the face (clamped at the zero-gradient ends)
                cells = [(j, min(max(i - 1, 0), nx - 1)), (j, min(i, nx - 1))] if d == 0 else \
                    [(min(max(j - 1, 0), ny - 1), i), (min(j, ny - 1), i)]
                margins.append(min(1.0 - float(rYw[a, b]) * bw for a, b in cells))
    st = c.mpmc_stats()
    reports = c.inadmissible_reports
    c.close()
    print("unrecoverable faces (step, dir, i, j):", where[:10], "... total", len(where), "reports", reports)
    assert reports >= 1
    assert st["inadmissible_cells"] == 0
    assert len(where) == st["unrecoverable"] and 0 < st["unrecoverable"] <= 400
    print("co-volume margin 1 - rhoY_w b of the faces' cells before the step: max %.3g" % max(margins))
    assert max(margins) < 5e-3, margins
    Uh = U.cpu().numpy()
    n, (nx, ny) = case.ncell, case.n[:2]
    held = case.extra["held"]
    faces = st["faces"]
    print("limiter activity per face evaluation: P fallback %.3g T %.3g first-order %.3g cdi drop %.3g" % (
        st["faces_P"] / faces, st["faces_T"] / faces, st["fallback"] / faces, st["cdi_drop"] / faces))
    print("unrecoverable", st["unrecoverable"], "of", faces)
    assert np.isfinite(Uh).all()
    assert np.array_equal(Uh.reshape(case.nv, n)[:, held], U0.reshape(case.nv, n)[:, held])
    assert np.all(Uh[:case.ns * n] >= 0.0)
    t = steps * dt
    w = [k for k, m in enumerate(case.materials) if m.phase == inputs.LIQUID][0]
    dx, dy = case.dx[0], case.dx[1]
    mw = lambda V: V[w * n:(w + 1) * n].sum() * dx * dy
    mom = U0[case.ns * n:(case.ns + 1) * n][held]
    rYw = U0[w * n:(w + 1) * n][held]
    rho0 = U0[:case.ns * n].reshape(case.ns, n).sum(0)[held]
    admitted = (rYw * mom / rho0).sum() * dy * t
    ratio = (mw(Uh) - mw(U0)) / admitted
    Y = (Uh[w * n:(w + 1) * n] / Uh[:case.ns * n].reshape(case.ns, n).sum(0)).reshape(ny, nx)
    head = (np.nonzero((Y > 0.5).any(0))[0].max() + 0.5) * dx
    print("water gained / admitted", ratio, "head", head, "u t", 150000.0 * t)
    assert abs(ratio - 1.0) < 2e-2
    assert 0.6 * 150000.0 * t <= head <= 1.1 * 150000.0 * t


def test_held_cells_rejections():
    case = inputs.water_inflow_1d(20)
    o = oracle.Oracle.from_case(case)
    U0 = o.init_state(case)
    c = ctx_of(case)
    vals = inputs.held_values(case, U0)
    for idx in ([20], [-1]):
        with pytest.raises(MpmcError):
            c.mpmc_set_held_cells(idx, vals)
    with pytest.raises(MpmcError):
        c.mpmc_set_held_cells([0, 0], np.concatenate([vals, vals], axis=1))
    bad = vals.copy()
    bad[0, 0] = -1.0
    with pytest.raises(MpmcError):
        c.mpmc_set_held_cells([0], bad)
    c.mpmc_set_held_cells([0], vals)
    lam = to_dev(np.ones_like(U0))
    with pytest.raises(MpmcError):
        c.mpmc_adjoint_step(to_dev(U0), c.scalar(1e-9), c.scalar(1.0), lam)
    c.mpmc_set_held_cells([], np.zeros((case.nv, 0)))
    c.close()
