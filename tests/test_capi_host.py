"""Host-side checks of the C ABI library: it loads, exports every symbol
include/sbp.h declares, and its reference operators (host setup logic) agree
with the oracle's independently built ones (no GPU needed)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "sbp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(sbp_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2305_07181_amd import sbp
    lib = sbp._lib
    syms = header_symbols()
    assert "sbp_setup_mesh" in syms and "sbp_residual" in syms and "sbp_rrk_step" in syms
    for name in syms:
        assert hasattr(lib, name), name
    assert set(syms) == set(sbp.SYMBOLS)


def test_unsupported_degree_is_an_error():
    from paper_2305_07181_amd import sbp
    with pytest.raises(sbp.SbpError) as ei:
        sbp.reference_operator(3, 4)
    assert ei.value.code == sbp.SBP_ENOTSUP


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_reference_operator_matches_oracle(dim, p):
    from paper_2305_07181_amd import sbp
    from oracle.operators import reference_operator
    a = sbp.reference_operator(dim, p)
    b = reference_operator(dim, p)
    assert a["n_p"] == b["n_p"] and a["n_f"] == b["n_f"]
    assert np.abs(a["nodes"] - b["nodes"]).max() < 1e-14
    assert np.abs(a["h"] - b["h"]).max() < 1e-15
    assert np.abs(a["E"] - b["E"]).max() < 1e-15
    assert (a["facet_nodes"] == b["facet_nodes"]).all()
    assert np.abs(a["facet_w"] - b["facet_w"]).max() < 1e-15
    scale = np.abs(b["Q"]).max()
    assert np.abs(a["Q"] - b["Q"]).max() < 1e-13 * scale


def test_null_handles_and_invalid_setups_are_errors():
    """Every call that takes a handle refuses a null one with SBP_EINVAL (and
    a message), before touching a device; sbp_setup_mesh refuses invalid
    descriptions during its host-side checks: a bad dimension, and a
    quadratic tetrahedral map at degree 1 (Assumption 1)."""
    import ctypes as C
    from paper_2305_07181_amd import sbp, workloads as wl
    lib = sbp._lib
    null = None
    buf = (C.c_double * 8)()
    calls = {
        "sbp_mesh_info": lambda: lib.sbp_mesh_info(null, None),
        "sbp_residual": lambda: lib.sbp_residual(null, buf, buf, None, None),
        "sbp_residual_vjp": lambda: lib.sbp_residual_vjp(null, buf, buf, buf, None),
        "sbp_rrk_step": lambda: lib.sbp_rrk_step(null, buf, C.c_double(0.1), C.c_double(0.1), None, None),
        "sbp_diagnostics": lambda: lib.sbp_diagnostics(null, buf, buf, None),
        "sbp_check_device": lambda: lib.sbp_check_device(null, None),
        "sbp_set_time": lambda: lib.sbp_set_time(null, C.c_double(1.0)),
        "sbp_use_graphs": lambda: lib.sbp_use_graphs(null, 1),
        "sbp_autotune": lambda: lib.sbp_autotune(null, buf, None, None, None),
        "sbp_get_launch_shape": lambda: lib.sbp_get_launch_shape(null, 0, 1, None, None),
        "sbp_set_launch_shape": lambda: lib.sbp_set_launch_shape(null, 0, 1, 0, 1),
        "sbp_set_volume_form": lambda: lib.sbp_set_volume_form(null, None),
        "sbp_set_source": lambda: lib.sbp_set_source(null, 1, None),
        "sbp_source_state": lambda: lib.sbp_source_state(null, C.c_double(0.0), buf, None),
        "sbp_source_error": lambda: lib.sbp_source_error(null, buf, C.c_double(0.0), 1, buf, None),
    }
    for name, call in calls.items():
        assert call() == sbp.SBP_EINVAL, name
        assert lib.sbp_last_error(), name
    assert lib.sbp_destroy_mesh(null) == sbp.SBP_OK
    # invalid descriptions, refused by the host checks
    out = C.c_void_p()
    ph = sbp.Physics(1.4, 2.5, 0, 0, 0, 1, 0.0, 0.71, 1.0, 0)
    assert lib.sbp_setup_mesh(None, C.byref(ph), None, C.byref(out)) == sbp.SBP_EINVAL
    desc = wl.curved_tet_mesh(2, 1.0, 0.03)
    vert = np.ascontiguousarray(desc["vert_xyz"], dtype=np.float64)
    elem = np.ascontiguousarray(desc["elem_vert"], dtype=np.int32)
    period = np.ascontiguousarray(desc["period"], dtype=np.float64)
    geom = np.ascontiguousarray(desc["geom_nodes"], dtype=np.float64)
    deg = np.ones(len(elem), dtype=np.int32)
    d = sbp.MeshDesc()
    d.dim, d.n_vert, d.n_elem = 3, len(vert), len(elem)
    d.vert_xyz, d.elem_vert, d.period, d.elem_degree = sbp._dp(vert), sbp._ip(elem), sbp._dp(period), sbp._ip(deg)
    d.p_geom, d.geom_nodes, d.n_problems = 2, sbp._dp(geom), 1
    assert lib.sbp_setup_mesh(C.byref(d), C.byref(ph), None, C.byref(out)) == sbp.SBP_EINVAL
    assert b"Assumption 1" in lib.sbp_last_error()
    d.dim = 4
    assert lib.sbp_setup_mesh(C.byref(d), C.byref(ph), None, C.byref(out)) == sbp.SBP_EINVAL
    assert not out.value
