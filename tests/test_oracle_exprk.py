"""Pins of the exponential Runge-Kutta oracle (Section 5, Table RK) and of
Problem 3's manufactured source.

* The source: with the Dirichlet FD Laplacian (exact on quadratics), the
  exact solution satisfies the semi-discrete equation to rounding:
  d/dt u_ex = -A u_ex + 1/(1 + u_ex^2) + f at every node.
* Orders 1, 2, 3 of exponential Euler, RK2 (c2 = 1/2) and RK3 (c2 = 1/3) at
  T = 1 against the exact solution (no space error with this source).
* Linear problems (g = g(t) only): Euler is exact for constant g.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import exprk as R
from oracle import phi_exact as X
from paper_2211_00696_amd import inputs as I


def lap2d(n):
    return [I.fd_laplacian(n), I.fd_laplacian(n)]


def test_manufactured_source_is_exact_for_the_fd_system():
    n = 9
    mats = lap2d(n)
    A = X.kron_sum(mats)
    for t in (0.0, 0.3, 1.0):
        ue = R.exact(n, t)
        rhs = -A @ ue + R.g_ho(n)(t, ue)
        assert np.max(np.abs(rhs - ue)) < 1e-12 * np.max(np.abs(ue)) * 100


@pytest.mark.parametrize("method,c2,order", [(1, 0.5, 1), (2, 0.5, 2), (3, 1.0 / 3.0, 3)])
def test_orders(method, c2, order):
    n = 7
    mats = lap2d(n)
    u0 = R.exact(n, 0.0)
    ue = R.exact(n, 1.0)
    errs = []
    for steps in (4, 8, 16):
        u = R.solve(mats, method, 1.0, steps, u0, R.g_ho(n), c2)
        errs.append(np.max(np.abs(u - ue)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(method, errs, rates)
    assert all(order - 0.35 < r < order + 0.6 for r in rates), rates


def test_euler_exact_for_constant_source():
    n = 5
    mats = lap2d(n)
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal(n * n)
    c = rng.standard_normal(n * n)
    tau = 0.1
    u = R.step(mats, 1, tau, 0.0, u0, lambda t, v: c, 0.5)
    M = -tau * X.kron_sum(mats)
    ref = scipy.linalg.expm(M) @ u0 + np.linalg.solve(M, scipy.linalg.expm(M) - np.eye(n * n)) @ (tau * c)
    assert np.max(np.abs(u - ref)) < 1e-12
