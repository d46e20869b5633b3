"""The allocation-free entry point mpmc_conserve_sum_static against
mpmc_conserve_sum (fixed-order sums, so the two agree bit for bit): two
calls in a row on one device, the second on a smaller input (another
context), and again after the first context's own sums."""
import numpy as np
import pytest

import oracle
from paper_2504_14063_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def state(case):
    from paper_2504_14063_amd import mpmc
    o = oracle.Oracle.from_case(case)
    U = torch.from_numpy(o.init_state(case)).cuda()
    return mpmc.Context.from_case(case), U


def test_conserve_sum_static_matches_allocating_sum():
    big = inputs.droplet_crossflow_3d(n=40, radius=6.0, dx=1e-3)
    small = inputs.interface_advection_1d(n=50)
    cb, Ub = state(big)
    cs, Us = state(small)
    cb.mpmc_rk3_step(Ub)
    first = cb.mpmc_conserve_sum_static(Ub)
    ref_b = cb.mpmc_conserve_sum(Ub)
    second = cs.mpmc_conserve_sum_static(Us)
    ref_s = cs.mpmc_conserve_sum(Us)
    again = cb.mpmc_conserve_sum_static(Ub)
    torch.cuda.synchronize()
    assert torch.equal(first, ref_b) and torch.equal(again, ref_b)
    assert torch.equal(second, ref_s)
    assert second.numel() == cs.nv < cb.nv == first.numel()
    # the sums themselves, against a plain host sum of the same state
    for got, U, c in ((first, Ub, cb), (second, Us, cs)):
        V = U.cpu().numpy().reshape(c.nv, -1)
        host, size = V.sum(1), np.abs(V).sum(1)
        assert np.all(np.abs(got.cpu().numpy() - host) <= 1e-13 * size)
    cb.close()
    cs.close()
