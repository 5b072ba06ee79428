"""CPU-side checks of the C-ABI library: it loads, exports exactly what
include/dg.h declares, and its host-built reference element (an independent
Bernstein-basis construction) matches the oracle's."""
import os
import re as regex

import numpy as np
import pytest

from oracle import reference_element as ore
from paper_2512_17101_amd import dg, hexdg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    out = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = regex.sub(r"/\*.*?\*/", "", src, flags=regex.S)
            out |= set(regex.findall(r"\b(dg_[a-z0-9_]+)\s*\(", src))
    return out


def test_library_exports_every_declared_symbol():
    L = hexdg.lib()
    declared = _declared_functions()
    assert declared == set(dg.EXPORTS) | set(hexdg.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_library_hex_tables_match_oracle(p):
    """Binary128 tables rounded once against the oracle's rational ones: the
    same correctly rounded values (zero entries may carry a residue below
    1e-30)."""
    from oracle import hex as oh
    L, o = hexdg.reference_operators(p), oh.operators_1d(p)
    u = 2.0 ** -53
    for k in ("x", "D", "lift"):
        assert np.all(np.abs(L[k] - o[k]) <= u * np.abs(o[k]) + 1e-30), k


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_library_reference_element_matches_oracle(p):
    """The library forms nodes and operators in binary128 and rounds once;
    the oracle uses decimal nodes and exact rational operators.  Both are
    the correctly rounded values, so they agree to the last bit, apart from
    entries whose exact value is zero (the binary128 residue, below 1e-30)."""
    lib_ops = dg.reference_operators(p)
    o = ore.operators(p)
    u = 2.0 ** -53
    np.testing.assert_allclose(lib_ops["rst"], o["rst"], rtol=0, atol=1e-30)
    assert np.array_equal(lib_ops["Fmask"], o["Fmask"])
    for k in ("Dr", "Ds", "Dt", "LIFT"):
        assert np.all(np.abs(lib_ops[k] - o[k]) <= u * np.abs(o[k]) + 1e-30), k


def test_reference_operators_rejects_bad_order():
    with pytest.raises(dg.DGError) as ei:
        dg.reference_operators(5)
    assert ei.value.status == 1


def test_host_side_argument_checks_need_no_device():
    """Entry points reject null handles and bad arguments before touching a
    device, with a status code and a message (no exception crosses the ABI)."""
    import ctypes
    L = dg.lib()
    cfg = dg.LaunchConfig(4, 1)
    assert L.dg_mesh_set_launch(None, 0, ctypes.byref(cfg)) == 1
    assert b"null" in L.dg_last_error()
    assert L.dg_mesh_get_launch(None, 0, ctypes.byref(cfg)) == 1
    prm = dg._params(1.4)
    assert L.dg_autotune(None, ctypes.byref(prm), 0, None, 3, None, None, None) == 1
    assert L.dg_rhs(None, ctypes.byref(prm), 0, None, None, None) == 1
    assert L.dg_rk_step(None, ctypes.byref(prm), 0, None, None, 0.0, 1e-3, None) == 1
    out = ctypes.c_void_p()
    assert L.dg_batch_create(None, 0, 1, ctypes.byref(out)) == 1 and not out.value
    assert L.dg_batch_rk_step(None, ctypes.byref(prm), 1, None) == 1
    bc = dg.BatchConfig(4, 2, 0, 0, 1)
    assert L.dg_batch_set_config(None, ctypes.byref(bc)) == 1
    assert L.dg_lsrk_update(-1, 0.0, 1.0, 1e-3, None, None, None, None) == 1
    assert L.dg_lsrk_update(0, 0.0, 1.0, 1e-3, None, None, None, None) == 0  # nothing to do
    # destroying null handles is a no-op
    assert L.dg_batch_destroy(None) == 0


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_library_hex_oi_tables_match_oracle(p):
    """Gauss points and weights correctly rounded on both sides, and the
    overintegration tables exact at them and rounded once: the same values,
    except that an entry whose exact value is a rounding tie (a product such
    as 1.5 x an FP64 weight needs 54 bits) may round either way under the
    binary128 route's last-bit error: one unit in the last place allowed."""
    from oracle import hex as oh
    L, o = hexdg.oi_operators(p), oh.oi_operators(p)
    assert L["nq"] == o["nq"]
    u = 2.0 ** -53
    for k in ("xq", "wq", "B", "lift"):
        assert np.all(np.abs(L[k] - o[k]) <= u * np.abs(o[k]) + 1e-30), k
    for k in ("S", "P"):
        assert np.all(np.abs(L[k] - o[k]) <= 2 * u * np.abs(o[k]) + 1e-30), k
