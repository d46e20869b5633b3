"""The library's iterative pressure (several distinct P_inf, Sec. 2.3),
compiled for the host, against the oracle on (P, T) round-trip states: two
liquids of different P_inf (one NASG water) and a gas over four decades of
pressure, including states with vanishing fractions of one component."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("eos") / "eos_host")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Wno-unused-result", "-o", exe, os.path.join(HERE, "eos_host.cpp")])
    return exe


def test_general_pressure_matches_oracle(harness):
    case = inputs.random_smooth_state_case(dim=1, n=(8, 1, 1), multi_pinf=True)
    o = oracle.Oracle.from_case(case)
    m = case.materials
    head = "3 " + " ".join(" ".join(repr(float(getattr(x, f))) for x in m)
                           for f in ("cv", "gamma", "pinf", "b", "q")) + "\n"
    rng = np.random.default_rng(21)
    states, ref = [], []
    for i in range(3000):
        P, T = 10 ** rng.uniform(4, 8), rng.uniform(250.0, 600.0)
        Y = rng.dirichlet(np.ones(3))
        if i % 3 == 0:
            Y[rng.integers(0, 3)] = 10.0 ** rng.uniform(-14, -6)
            Y /= Y.sum()
        u, _ = o.state_from_PT(P, T, Y, [rng.uniform(-100, 100)])
        states.append(u)
        ref.append((P, T))
    inp = head + "".join(" ".join(repr(float(x)) for x in u) + "\n" for u in states)
    out = subprocess.run([harness], input=inp, capture_output=True, text=True, check=True).stdout.split()
    got = np.array(out, dtype=np.float64).reshape(-1, 2)
    ref = np.array(ref)
    orc = np.array([[o.equilibrium(u)["P"], o.equilibrium(u)["T"]] for u in states[:300]])
    assert np.all(np.isfinite(got))
    assert np.abs(got[:, 0] / ref[:, 0] - 1).max() <= 1e-9
    assert np.abs(got[:, 1] / ref[:, 1] - 1).max() <= 1e-9
    # the pressure of a liquid mixture is conditioned by P + P_inf, not by P:
    # compare it on that scale
    pmax = max(x.pinf for x in m)
    assert np.abs(got[:300, 0] - orc[:, 0]).max() <= 1e-14 * (np.abs(orc[:, 0]) + pmax).max()
    assert np.abs(got[:300, 1] / orc[:, 1] - 1).max() <= 1e-12
