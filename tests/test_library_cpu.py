"""CPU-side checks of the C-ABI library: it loads, exports exactly what
include/dg.h declares, and its host-built reference element (an independent
Bernstein-basis construction) matches the oracle's."""
import os
import re as regex

import numpy as np
import pytest

from oracle import reference_element as ore
from paper_2512_17101_amd import dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "dg.h")).read()
    src = regex.sub(r"/\*.*?\*/", "", src, flags=regex.S)
    return set(regex.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src))


def test_library_exports_every_declared_symbol():
    L = dg.lib()
    declared = _declared_functions()
    assert declared == set(dg.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_library_reference_element_matches_oracle(p):
    lib_ops = dg.reference_operators(p)
    o = ore.operators(p)
    np.testing.assert_allclose(lib_ops["rst"], o["rst"], atol=1e-14)
    assert np.array_equal(lib_ops["Fmask"], o["Fmask"])
    for k in ("Dr", "Ds", "Dt"):
        np.testing.assert_allclose(lib_ops[k], o[k], atol=1e-12 * np.abs(o[k]).max())
    np.testing.assert_allclose(lib_ops["LIFT"], o["LIFT"], atol=1e-12 * np.abs(o["LIFT"]).max())


def test_reference_operators_rejects_bad_order():
    with pytest.raises(dg.DGError) as ei:
        dg.reference_operators(5)
    assert ei.value.status == 1
