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
