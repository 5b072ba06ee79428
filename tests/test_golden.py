"""The stored oracle fixtures of tests/golden (written by
tests/golden/make_golden.py from the oracle alone): the oracle recomputes
them, so a change to its arithmetic shows up here.  The paper prints no
worked numerical example of these operators; the fixtures pin the oracle
against itself over time, not against the paper."""
import importlib.util
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
mg = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(mg)

from oracle import euler as oe, lsrk as olsrk  # noqa: E402


def _close(got, ref, rel):
    return np.abs(got - ref).max() <= rel * np.abs(ref).max()


def test_reference_element_p1_matches_fixture():
    g = mg.read(os.path.join(HERE, "golden", "ref_p1.txt"))
    _, _, ops, _, _, _ = mg.case()
    for k in ("rst", "Dr", "Ds", "Dt", "LIFT"):
        assert np.array_equal(np.asarray(ops[k]), g[k]), k  # the operators are correctly rounded: exact
    assert np.array_equal(np.asarray(ops["Fmask"], dtype=np.float64).reshape(g["Fmask"].shape), g["Fmask"])


def test_euler_rhs_and_step_match_fixture():
    g = mg.read(os.path.join(HERE, "golden", "euler_p1_3cubed.txt"))
    _, _, ops, geo, conn, q = mg.case()
    r = oe.rhs(ops, geo, conn, q)
    q1, _ = olsrk.lsrk_step(lambda qq, tt: oe.rhs(ops, geo, conn, qq), q, 0.0, mg.DT)
    ne = g["rhs"].shape[1]
    # summation order inside the BLAS calls may differ between machines
    for f in range(5):
        assert _close(r[f, :ne], g["rhs"][f], 1e-13), f
        assert _close(q1[f, :ne], g["q1"][f], 1e-14), f
