"""The library's face reconstruction of every scheme (WENO5-Z, WENO5-JS,
TENO5, TENO6), compiled for the host, against the oracle's on seeded
stencils: smooth, rough, with jumps and with flat parts."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

SCHEMES = {0: ("weno5z", 1e-40, 1), 1: ("weno5js", 1e-6, 2), 2: ("teno5", 1e-40, 1), 3: ("teno6", 1e-40, 1)}


def stencils(seed=7, n=400):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        kind = i % 4
        if kind == 0:    # smooth: samples of a low-frequency sine
            x = np.arange(6) * rng.uniform(0.01, 0.5)
            w = np.sin(x + rng.uniform(0, 6)) * rng.uniform(0.1, 1e3)
        elif kind == 1:  # rough
            w = rng.normal(size=6) * 10 ** rng.uniform(-3, 3)
        elif kind == 2:  # a jump at a random position
            w = np.where(np.arange(6) < rng.integers(1, 6), 0.0, 1.0) * rng.uniform(0.5, 2) + rng.uniform(-1, 1)
        else:            # flat with one perturbed value
            w = np.full(6, rng.uniform(-1, 1))
            w[rng.integers(0, 6)] += rng.uniform(-1e-3, 1e-3)
        out.append(w)
    return np.array(out)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("recon") / "recon_host")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Wno-unused-result", "-o", exe, os.path.join(HERE, "recon_host.cpp")])
    return exe


@pytest.mark.parametrize("scheme", sorted(SCHEMES))
def test_reconstruction_matches_oracle(harness, scheme):
    name, eps, pw = SCHEMES[scheme]
    W = stencils()
    inp = "".join(f"{scheme} {eps!r} {pw} " + " ".join(repr(float(v)) for v in w) + "\n" for w in W)
    out = subprocess.run([harness], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([[float(v) for v in line.split()] for line in out.splitlines()])
    assert got.shape == (len(W), 2)
    fn = {"weno5z": lambda f: oracle.weno5z(f[:5], eps, pw), "weno5js": lambda f: oracle.weno5js(f[:5], eps, pw),
          "teno5": lambda f: oracle.teno5(f[:5], eps), "teno6": lambda f: oracle.teno6(f, eps)}[name]
    worst = 0.0
    for w, (l, r) in zip(W, got):
        scale = np.abs(w).max() + 1e-300
        worst = max(worst, abs(l - fn(w)) / scale, abs(r - fn(w[::-1])) / scale)
    assert worst <= 1e-13, (name, worst)
