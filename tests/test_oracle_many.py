"""Pins of the oracle with more components than the paper's workloads use
(up to 8; the GPU's forward entry points are checked against it in
test_gpu_many.py).

What fixes each check:
 - the interface-equilibrium property of the method (Sec. 3.1.2): a droplet
   of three liquids in five gases at uniform P, T and u keeps them uniform to
   round-off, while the components move;
 - splitting a component into two identical copies whose mass fractions sum
   to the original's changes nothing: the copies' partial densities add up to
   the original one and every other variable is unchanged (a dropped or
   misindexed term of any per-component loop breaks this);
 - discrete conservation of every partial density on a periodic box.
"""
import copy

import numpy as np

import oracle
from paper_2504_14063_amd import inputs


def cell_prims(o, U):
    n = U.size // o.nv
    e = [o.equilibrium(U[i::n]) for i in range(n)]
    P = np.array([x["P"] for x in e])
    T = np.array([x["T"] for x in e])
    Ur = U.reshape(o.nv, n)
    u = Ur[o.ns] / Ur[:o.ns].sum(0)
    return P, T, u


def test_eight_components_keep_interface_equilibrium():
    """Measured after 20 steps: P 1.6e-11, T 4.8e-15, u 1.4e-13 relative."""
    case = inputs.many_component_case(dim=1, n=(64, 1, 1), seed=7, n_liquid=3, n_gas=5, diffusion=0, floor=False)
    case.P[:] = 1e5
    case.T[:] = 300.0
    case.vel[:] = 20.0
    o = oracle.Oracle.from_case(case)
    U = o.init_state(case)
    U0 = U.copy()
    for _ in range(20):
        o.step(U)
    assert o.status == 0
    P, T, u = cell_prims(o, U)
    dP, dT, du = np.abs(P / 1e5 - 1).max(), np.abs(T / 300 - 1).max(), np.abs(u / 20 - 1).max()
    print("8 components, 20 steps: P", dP, "T", dT, "u", du)
    assert dP <= 1e-9 and dT <= 1e-12 and du <= 1e-11
    # the components did move: the liquid fractions changed by more than round-off
    assert np.abs(U - U0)[: o.ns * 64].max() > 1e-3 * np.abs(U0[: o.ns * 64]).max()
    # periodic box: every partial density is conserved
    s0 = U0.reshape(o.nv, -1).sum(1)
    s1 = U.reshape(o.nv, -1).sum(1)
    assert np.all(np.abs(s1 - s0)[: o.ns] <= 1e-13 * np.abs(U0.reshape(o.nv, -1)[: o.ns]).sum(1))


def split_copy(case, k, frac=0.5):
    """The case with component k replaced by two identical copies holding
    frac and 1 - frac of its mass fraction."""
    c2 = copy.deepcopy(case)
    m = case.materials[k]
    c2.materials = case.materials[: k + 1] + [copy.deepcopy(m)] + case.materials[k + 1:]
    y = case.y
    c2.y = np.concatenate([y[:k], frac * y[k:k + 1], (1.0 - frac) * y[k:k + 1], y[k + 1:]])
    return c2


def test_split_component_changes_nothing():
    """Two liquids and three gases; the second gas split into two copies
    (6 components), and the first liquid split as well (7), over 8 steps in
    2D with diffusion and the regularization on: the sums of the copies and
    every other variable agree with the unsplit run."""
    base = inputs.many_component_case(dim=2, n=(14, 12, 1), seed=11, n_liquid=2, n_gas=3, bc=(0, 2, 0))
    for ks in ((3,), (3, 0)):
        case = base
        for k in ks:
            case = split_copy(case, k, 0.3)
        oa = oracle.Oracle.from_case(base)
        ob = oracle.Oracle.from_case(case)
        Ua = oa.init_state(base)
        Ub = ob.init_state(case)
        for _ in range(8):
            oa.step(Ua)
            ob.step(Ub)
        assert oa.status == 0 and ob.status == 0
        n = base.ncell
        A = Ua.reshape(oa.nv, n)
        B = Ub.reshape(ob.nv, n)
        # fold the copies back: each split at k adds row k + 1 (indices of
        # the later split are those of the case it was applied to)
        for k in reversed(ks):
            B = np.concatenate([B[:k], B[k:k + 1] + B[k + 1:k + 2], B[k + 2:]])
        rho = A[: oa.ns].sum(0).max()
        scale = np.array([rho] * oa.ns + [np.abs(A[oa.ns:-1]).max()] * base.dim + [np.abs(A[-1]).max()])
        err = np.abs(B - A).max(1) / scale
        print("split", ks, err)
        assert np.all(err <= 1e-12), err
