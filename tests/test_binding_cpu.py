"""CPU tests of the Python binding's argument checks and of the C ABI's
host-side validation for the reacting model, the reordered thermochemistry
calls and the status call (no GPU needed: every case is rejected before a
kernel could be launched)."""
import ctypes
import types

import numpy as np
import pytest

from paper_2512_17101_amd import dg

torch = pytest.importorskip("torch")


def _fake_mesh(E=10, Np=20, device=0):
    return types.SimpleNamespace(E=E, Np=Np, device=device, handle=ctypes.c_void_p())


def test_rhs_rejects_wrongly_sized_state():
    m = _fake_mesh()
    good = torch.zeros(5 * 10 * 20, dtype=torch.float64)
    bad = torch.zeros(5 * 10 * 20 - 1, dtype=torch.float64)
    with pytest.raises(ValueError, match="q must hold"):
        dg.rhs(m, bad, good)
    with pytest.raises(ValueError, match="out must hold"):
        dg.rhs(m, good, bad)
    # a 12-field state is not an Euler state
    with pytest.raises(ValueError):
        dg.rhs(m, torch.zeros(12 * 200, dtype=torch.float64), good)


def test_rk_step_rejects_short_work_and_wrong_state():
    m = _fake_mesh()
    q = torch.zeros(5, 10, 20, dtype=torch.float64)
    with pytest.raises(ValueError, match="two state arrays"):
        dg.rk_step(m, q, torch.zeros(1000 * 2 - 1, dtype=torch.float64), 0.0, 1e-3)
    with pytest.raises(ValueError, match="q must hold"):
        dg.rk_step(_fake_mesh(E=11), q, torch.zeros(4000, dtype=torch.float64), 0.0, 1e-3)


def test_host_tensors_are_refused():
    m = _fake_mesh()
    q = torch.zeros(5, 10, 20, dtype=torch.float64)
    with pytest.raises(TypeError, match="HIP torch tensor"):
        dg.rhs(m, q, torch.zeros_like(q))


def test_reacting_entry_points_check_sizes():
    m = _fake_mesh()
    q = torch.zeros(12, 10, 20, dtype=torch.float64)
    with pytest.raises(ValueError, match="35 E Np"):
        dg.reacting_rhs(m, None, q, torch.zeros_like(q), torch.zeros(34 * 200, dtype=torch.float64))
    with pytest.raises(ValueError, match="59 E Np"):
        dg.reacting_rk_step(m, None, q, torch.zeros(58 * 200, dtype=torch.float64), 1e-9)


def test_c_abi_model_and_precision_checks():
    L = dg.lib()
    prm = dg._params(1.4)
    prm.model = 2
    assert L.dg_rhs(None, ctypes.byref(prm), 0, None, None, None) == 1  # null mesh first
    # model 1 with a reduced-precision contraction is a valid request the library does not implement
    assert L.dg_rk_step(None, None, 0, None, None, 0.0, 1e-3, None) == 1


def test_thermo_calls_reject_null_handles():
    L = dg.lib()
    assert L.dg_temperature(4, None, None, None, None, None, 1e-10, 50, None, None) == 1
    assert b"null thermo" in L.dg_last_error()
    assert L.dg_sources(4, None, None, None, None, None) == 1
    assert b"null mechanism" in L.dg_last_error()


def test_synchronize_rejects_bad_device():
    L = dg.lib()
    assert L.dg_synchronize(-1, None) == 1
    assert L.dg_synchronize(1 << 20, None) == 1
