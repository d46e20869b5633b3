"""Host check of the hand-written reverse-mode blocks of the adjoint (WENO5-Z,
Y-limiter, face EOS, HLLC, equilibrium coefficients, per-cell quantities): each against
forward-mode dual numbers pushed through the same templated forward code,
compiled for the host by hipcc."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("vjp") / "vjp_blocks")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Wno-unused-result", "-o", exe, os.path.join(HERE, "vjp_blocks.cpp")])
    out = subprocess.check_output([exe], text=True)
    res = {}
    for line in out.splitlines():
        k, *v = line.split()
        res[k] = [float(x) for x in v]
    return res


@pytest.mark.parametrize("block", ["weno5z_p1_smooth", "weno5z_p1_rough", "weno5z_p2_smooth",
                                   "weno5z_p2_rough", "weno5z_flat", "ylimit", "ylimit_noise",
                                   "face_state", "hllc"])
def test_vjp_block_matches_forward_duals(harness, block):
    assert harness[block][0] <= 1e-11, harness[block]


def test_equilibrium_coefficients_vjp(harness):
    # the momentum derivatives are ~1e-8 of the density derivatives here and
    # carry the rounding of the dual chain at ~1e-10 of their own size
    assert harness["equilibrium_cz"][0] <= 1e-9, harness["equilibrium_cz"]
    lin, quad_pos, quad_neg = harness["equilibrium_cz_branches"]
    assert lin > 50 and quad_pos > 20 and quad_neg > 50


def test_cell_quantities_vjp(harness):
    # equilibrium and phase auxiliaries (CDI, diffusion with a Wilke gas
    # phase) over mixed, pure-gas and liquid-rich cells
    assert harness["cell_quantities"][0] <= 1e-11, harness["cell_quantities"]


def test_ylimit_both_branches_exercised(harness):
    _, above, below = harness["ylimit_branches"]
    assert above > 50 and below > 50
