"""Shared helpers of the test-suite (no method arithmetic)."""
import json
import os

import numpy as np

from paper_2504_14063_amd import inputs
from paper_2504_14063_amd.inputs import GAS, LIQUID, Material

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name="paper_values.json"):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def paper_water():
    w = golden()["nasg_materials"]["water"]
    return Material("water", LIQUID, w["Cp"] / w["gamma"], w["gamma"], pinf=w["pinf"], b=w["b"],
                    q=w["q"], molar_mass=0.018, mu=8.9e-4)


def paper_gas(name):
    g = golden()["nasg_materials"][name]
    cv = g["Cp"] / g["gamma"]
    W = inputs.R_UNIVERSAL / (g["Cp"] - cv)
    return Material(name, GAS, cv, g["gamma"], molar_mass=W, mu=1.8e-5)


def stiff_liquid():
    return Material("liquid", LIQUID, 1816.0, 6.12, pinf=3.43e8, molar_mass=0.018, mu=8.9e-4)


def eos_dict(mats):
    return dict(n_species=len(mats), phase=[m.phase for m in mats], cv=[m.cv for m in mats],
                gamma=[m.gamma for m in mats], pinf=[m.pinf for m in mats], b=[m.b for m in mats],
                q=[m.q for m in mats], molar_mass=[m.molar_mass for m in mats],
                mu=[m.mu for m in mats], Sc=[m.Sc for m in mats])


def grid_dict(dim=1, n=(8, 1, 1), dx=1e-3, bc=0):
    n = tuple(n[d] if d < dim else 1 for d in range(3))
    return dict(dim=dim, n=list(n), dx=[dx] * 3, bc_lo=[bc] * 3, bc_hi=[bc] * 3)


def uniform_case(mats, phi, y, P, T, vel, n=8, dim=1, dx=1e-3, bc=0, **opts):
    """Case with uniform primitive fields."""
    nn = tuple(n if d < dim else 1 for d in range(3))
    shape = (nn[2], nn[1], nn[0])
    c = inputs.Case("uniform", dim, nn, (dx, dx, dx), (bc,) * 3, (bc,) * 3, mats,
                    inputs.default_opts(**opts),
                    np.stack([np.full(shape, phi[0]), np.full(shape, phi[1])]),
                    np.stack([np.full(shape, yy) for yy in y]), np.full(shape, P),
                    np.full(shape, T), np.stack([np.full(shape, v) for v in vel[:dim]]))
    return c


def rel_l1(a, b, nv, ncell):
    a = a.reshape(nv, ncell)
    b = b.reshape(nv, ncell)
    return np.abs(a - b).sum(1) / np.maximum(np.abs(b).sum(1), 1e-300)
