"""Builders of the small forced-decision states of
tests/golden/forced_limiter_states.json (no method arithmetic)."""
import numpy as np

from paper_2504_14063_amd import inputs
from paper_2504_14063_amd.inputs import GAS, Material
from tests.util import stiff_liquid

N = 8
BITS = {"T": 3, "P": 12, "FB": 16, "DROP": 32, "UNREC": 64}


def materials():
    return [stiff_liquid(), Material("A", GAS, 716.76, 1.4, molar_mass=0.029, mu=1.81e-5),
            Material("B", GAS, 3116.4, 1.667, molar_mass=0.004, mu=1.96e-5)]


def build_case(f, cdi=None, positivity=1):
    """8 cells on a periodic line of 1 mm cells; f: primitive fields phil
    (liquid volume fraction), yA (first gas' share of the gas), P, T, u, and
    cdi (regularization on)."""
    if f is None:
        f = dict(phil=[0.0] * N, yA=[0.5] * N, P=[1e5] * N, T=[300.0] * N, u=[0.0] * N)
    cdi = f.get("cdi", False) if cdi is None else cdi
    opts = inputs.default_opts(cdi=int(cdi), eps_cdi=1.5e-3, positivity=positivity)
    phil, yA = np.asarray(f["phil"]), np.asarray(f["yA"])
    phi = np.stack([phil, 1.0 - phil]).reshape(2, 1, 1, N)
    y = np.stack([np.ones(N), yA, 1.0 - yA]).reshape(3, 1, 1, N)
    return inputs.Case("forced", 1, (N, 1, 1), (1e-3,) * 3, (0,) * 3, (0,) * 3, materials(), opts, phi, y,
                       np.asarray(f["P"], dtype=float).reshape(1, 1, N),
                       np.asarray(f["T"], dtype=float).reshape(1, 1, N),
                       np.asarray(f["u"], dtype=float).reshape(1, 1, 1, N))
