"""The library's FP64 Euler RHS and LSRK step on the stored oracle fixture
(tests/golden/euler_p1_3cubed.txt, written from the oracle by
tests/golden/make_golden.py), through the C ABI: within 1e-12 of each
field's largest value (the momentum components share one scale)."""
import importlib.util
import os

import numpy as np
import pytest

from paper_2512_17101_amd import dg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
mg = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(mg)


def _err(got, ref):
    scale = np.abs(ref).max(axis=(1, 2))
    scale[1:4] = scale[1:4].max()
    return np.abs(got - ref).max(axis=(1, 2)) / scale


def test_rhs_and_step_match_golden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    g = mg.read(os.path.join(HERE, "golden", "euler_p1_3cubed.txt"))
    ne = g["rhs"].shape[1]
    xyz, vid, _, _, _, q = mg.case()
    mesh = dg.Mesh(mg.P, xyz, vid, 0)
    qt = torch.from_numpy(q).to(dev)
    out = torch.empty_like(qt)
    dg.rhs(mesh, qt, out)
    dg.synchronize()
    er = _err(out.cpu().numpy()[:, :ne], g["rhs"])
    work = torch.empty((2,) + tuple(qt.shape), dtype=torch.float64, device=dev)
    dg.rk_step(mesh, qt, work, 0.0, mg.DT)
    dg.synchronize()
    eq = _err(qt.cpu().numpy()[:, :ne], g["q1"])
    print(f"golden p=1 3^3: rhs error per field {np.array2string(er, precision=2)}, "
          f"step {np.array2string(eq, precision=2)}", flush=True)
    assert np.all(er <= 1e-12) and np.all(eq <= 1e-12)
