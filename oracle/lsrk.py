"""Low-storage explicit Runge-Kutta time stepping (oracle, FP64).
Test infrastructure only (see the package docstring).

The paper advances its Euler/vortex runs with explicit fourth-order
Runge-Kutta (Sec. 5.2).  The low-storage reading is Carpenter & Kennedy's
five-stage, fourth-order, 2N-storage scheme (NASA TM-109112, 1994; the same
coefficients are printed in Hesthaven & Warburton's nodal DG text):

  res <- 0
  for stage s = 1..5:  res <- a_s res + dt * f(q, t + c_s dt);  q <- q + b_s res

Classic four-stage RK4 is provided as an alternative reading.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

# Carpenter & Kennedy (1994) 2N-storage RK(5,4) coefficients, as published
# (ratios of integers).
LSRK_A = (
    Fraction(0),
    Fraction(-567301805773, 1357537059087),
    Fraction(-2404267990393, 2016746695238),
    Fraction(-3550918686646, 2091501179385),
    Fraction(-1275806237668, 842570457699),
)
LSRK_B = (
    Fraction(1432997174477, 9575080441755),
    Fraction(5161836677717, 13612068292357),
    Fraction(1720146321549, 2090206949498),
    Fraction(3134564353537, 4481467310338),
    Fraction(2277821191437, 14882151754819),
)
LSRK_C = (
    Fraction(0),
    Fraction(1432997174477, 9575080441755),
    Fraction(2526269341429, 6820363962896),
    Fraction(2006345519317, 3224310063776),
    Fraction(2802321613138, 2924317926251),
)

A = tuple(float(x) for x in LSRK_A)
B = tuple(float(x) for x in LSRK_B)
C = tuple(float(x) for x in LSRK_C)


def butcher_tableau():
    """Expand the 2N-storage scheme into its (6-stage-point) Butcher form.

    Returns (Amat [5x5], b [5], c [5]) as float64, where stage s evaluates f
    at q + dt * sum_i Amat[s, i] k_i.
    """
    a = [float(x) for x in LSRK_A]
    b = [float(x) for x in LSRK_B]
    S = 5
    # res_j = sum_{i<=j} (prod_{l=i+1..j} a_l) dt k_i ;  q_{s} = q_0 + sum_{j<s} b_j res_j
    R = np.zeros((S, S))
    for j in range(S):
        for i in range(j + 1):
            prod = 1.0
            for l in range(i + 1, j + 1):
                prod *= a[l]
            R[j, i] = prod
    Amat = np.zeros((S, S))
    for s in range(S):
        for j in range(s):
            Amat[s] += b[j] * R[j]
    bvec = np.zeros(S)
    for j in range(S):
        bvec += b[j] * R[j]
    return Amat, bvec, Amat.sum(axis=1)


def lsrk_step(f, q: np.ndarray, t: float, dt: float, stage_filter=None):
    """One LSRK(5,4) step of dq/dt = f(q, t); returns (q_new, res).
    stage_filter (optional) maps every stage state to the one the next stage
    uses (a limiter); the residual is left as it is."""
    q = q.copy()
    res = np.zeros_like(q)
    for s in range(5):
        res = A[s] * res + dt * f(q, t + C[s] * dt)
        q = q + B[s] * res
        if stage_filter is not None:
            q = stage_filter(q)
    return q, res


def rk4_step(f, q: np.ndarray, t: float, dt: float):
    """Classic four-stage RK4 step (alternative reading)."""
    k1 = f(q, t)
    k2 = f(q + 0.5 * dt * k1, t + 0.5 * dt)
    k3 = f(q + 0.5 * dt * k2, t + 0.5 * dt)
    k4 = f(q + dt * k3, t + dt)
    return q + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
