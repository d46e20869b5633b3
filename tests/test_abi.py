"""The C-ABI library loads and exports every entry point its header declares
(no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpmc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mpmc_init", "mpmc_free", "mpmc_rhs", "mpmc_rk3_step", "mpmc_adjoint_step",
                     "mpmc_compute_dt", "mpmc_stats"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2504_14063_amd import mpmc
    if not os.path.exists(mpmc.LIB_PATH):
        pytest.skip("libmpmc.so not built")
    lib = ctypes.CDLL(mpmc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_oracle_is_not_linked_by_the_library():
    from paper_2504_14063_amd import mpmc
    if not os.path.exists(mpmc.LIB_PATH):
        pytest.skip("libmpmc.so not built")
    lib = ctypes.CDLL(mpmc.LIB_PATH)
    assert not hasattr(lib, "oracle_rk3_step")
    for f in os.listdir(os.path.join(ROOT, "paper_2504_14063_amd", "csrc")):
        txt = open(os.path.join(ROOT, "paper_2504_14063_amd", "csrc", f)).read()
        assert "oracle" not in txt.lower(), f


def _init_code(grid, eos, opts):
    """mpmc_init's return code for the configuration (validation happens
    before any device call, so rejected configurations touch no GPU)."""
    from paper_2504_14063_amd import mpmc
    h = ctypes.c_void_p()
    g, e, o = mpmc._fill(mpmc.mpmc_grid, grid), mpmc._fill(mpmc.mpmc_eos, eos), mpmc._fill(mpmc.mpmc_opts, opts)
    code = mpmc.lib().mpmc_init(ctypes.byref(g), ctypes.byref(e), ctypes.byref(o), ctypes.byref(h))
    assert h.value is None, "a rejected configuration must not return a context"
    return code


def _base():
    from paper_2504_14063_amd import inputs
    case = inputs.droplet_crossflow_3d(n=16)
    return case.grid_dict(), case.eos_dict(), dict(case.opts)


def _with(d, **kw):
    out = {k: (list(v) if isinstance(v, list) else v) for k, v in d.items()}
    out.update(kw)
    return out


@pytest.mark.parametrize("what", [
    "empty_grid", "negative_cells", "dim_0", "dim_4", "inactive_direction_not_1", "dx_zero",
    "bc_code", "reflect_n2", "too_many_cells", "cells_above_2_29", "faces_above_2_29", "no_species", "nine_species", "phase_code", "gamma_le_1", "cv_zero",
    "precision_2", "cfl_zero", "weno_p_3", "negative_weno_eps", "viscous_without_prandtl",
    "negative_weno_scheme", "negative_basis"])
def test_init_rejects_invalid_configurations(what):
    from paper_2504_14063_amd import mpmc
    if not os.path.exists(mpmc.LIB_PATH):
        pytest.skip("libmpmc.so not built")
    g, e, o = _base()
    if what == "empty_grid":
        g = _with(g, n=[0, 16, 16])
    elif what == "negative_cells":
        g = _with(g, n=[16, -4, 16])
    elif what == "dim_0":
        g = _with(g, dim=0)
    elif what == "dim_4":
        g = _with(g, dim=4)
    elif what == "inactive_direction_not_1":
        g = _with(g, dim=2, n=[16, 16, 5])
    elif what == "dx_zero":
        g = _with(g, dx=[1e-3, 0.0, 1e-3])
    elif what == "bc_code":
        g = _with(g, bc_lo=[0, 4, 0])
    elif what == "reflect_n2":
        g = _with(g, n=[16, 2, 16], bc_lo=[0, 2, 0], bc_hi=[0, 2, 0])
    elif what == "too_many_cells":
        g = _with(g, n=[2048, 2048, 1024])
    elif what == "cells_above_2_29":
        # rows are addressed with 32-bit byte offsets: at most 2^29 cells
        g = _with(g, n=[1024, 1024, 513])
    elif what == "faces_above_2_29":
        # 2^29 cells, but 1025 * 1024 * 512 faces normal to x
        g = _with(g, n=[1024, 1024, 512])
    elif what == "no_species":
        e = _with(e, n_species=0)
    elif what == "nine_species":
        e = _with(e, n_species=9)
    elif what == "phase_code":
        e = _with(e, phase=[0, 2, 1])
    elif what == "gamma_le_1":
        e = _with(e, gamma=[6.12, 1.0, 1.667])
    elif what == "cv_zero":
        e = _with(e, cv=[1816.0, 0.0, 3116.0])
    elif what == "precision_2":
        o = _with(o, precision=2)
    elif what == "cfl_zero":
        o = _with(o, cfl=0.0)
    elif what == "weno_p_3":
        o = _with(o, weno_p=3)
    elif what == "negative_weno_eps":
        o = _with(o, weno_eps=-1.0)
    elif what == "viscous_without_prandtl":
        o = _with(o, viscous=1, prandtl=0.0)
    elif what == "negative_weno_scheme":
        o = _with(o, weno=-1)
    elif what == "negative_basis":
        o = _with(o, basis=-1)
    assert _init_code(g, e, o) == mpmc.MPMC_EINVAL


@pytest.mark.parametrize("what", ["four_species_mixed", "four_species_fused", "two_distinct_pinf_mixed",
                                  "unknown_weno_scheme", "weno_variant_mixed", "unknown_basis",
                                  "five_equation_basis_mixed"])
def test_init_reports_unsupported_configurations(what):
    from paper_2504_14063_amd import mpmc
    if not os.path.exists(mpmc.LIB_PATH):
        pytest.skip("libmpmc.so not built")
    g, e, o = _base()
    if what.startswith("four_species"):
        # more than 3 components: the FP64 forward only
        e = {k: (v + [v[-1]] if isinstance(v, list) else v) for k, v in e.items()}
        e["n_species"] = 4
        o = _with(o, precision=1) if what == "four_species_mixed" else _with(o, step_layout=2)
    elif what == "two_distinct_pinf_mixed":
        e = _with(e, phase=[0, 0, 1], pinf=[3.43e8, 6.0e8, 0.0])
        o = _with(o, precision=1)
    elif what == "unknown_weno_scheme":
        o = _with(o, weno=4)
    elif what == "weno_variant_mixed":
        o = _with(o, weno=2, precision=1)
    elif what == "unknown_basis":
        o = _with(o, basis=2)
    elif what == "five_equation_basis_mixed":
        o = _with(o, basis=1, precision=1)
    assert _init_code(g, e, o) == mpmc.MPMC_EUNSUPPORTED
