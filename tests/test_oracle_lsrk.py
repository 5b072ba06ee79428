"""Pins of the low-storage RK(5,4) coefficients: the expanded Butcher tableau
satisfies the eight fourth-order conditions, the published c_s are its row
sums, and the empirical order on y' = lambda y is four (classic RK4 too)."""
import numpy as np

from oracle import lsrk


def _order_conditions(A, b, c):
    return {
        "b": (b.sum(), 1.0),
        "bc": (b @ c, 1 / 2),
        "bc2": (b @ c ** 2, 1 / 3),
        "bAc": (b @ A @ c, 1 / 6),
        "bc3": (b @ c ** 3, 1 / 4),
        "bcAc": (b @ (c * (A @ c)), 1 / 8),
        "bAc2": (b @ A @ c ** 2, 1 / 12),
        "bAAc": (b @ A @ A @ c, 1 / 24),
    }


def test_lsrk_order_conditions():
    A, b, c = lsrk.butcher_tableau()
    for name, (val, exact) in _order_conditions(A, b, c).items():
        assert abs(val - exact) < 1e-14, name
    np.testing.assert_allclose(c, np.array(lsrk.C), atol=1e-14)


def test_classic_rk4_order_conditions():
    A = np.array([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1, 0]])
    b = np.array([1, 2, 2, 1]) / 6
    c = A.sum(1)
    for name, (val, exact) in _order_conditions(A, b, c).items():
        assert abs(val - exact) < 1e-15, name


def _empirical_order(step):
    lam = -1.0 + 0.5j
    f = lambda y, t: lam * y
    errs = []
    for n in (20, 40):
        dt = 1.0 / n
        y = np.array([1.0 + 0j])
        for s in range(n):
            out = step(f, y, s * dt, dt)
            y = out[0] if isinstance(out, tuple) else out
        errs.append(abs(y[0] - np.exp(lam)))
    return np.log2(errs[0] / errs[1])


def test_empirical_order_four():
    assert 3.8 < _empirical_order(lsrk.lsrk_step) < 4.3
    assert 3.8 < _empirical_order(lsrk.rk4_step) < 4.3
