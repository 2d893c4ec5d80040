"""Pins of the ETD-RK4 oracle (Cox-Matthews) against closed forms and order.

* F = 0: one step is the exact e^{-hA} u.
* F = constant c: the scheme integrates exactly, u(h) = e^{-hA} u + h phi_1(-hA) c
  (f1 + 4 f2 + f3 = phi_1; a wrong sign or coefficient in f1..f3 breaks it).
* Scalar u' = -lam u + u - u^3 (a Bernoulli equation with a closed form):
  the global error at T = 1 falls by ~2^4 per halving of h.
* A small 2D Allen-Cahn problem against scipy's implicit Radau solution at
  tight tolerance: fourth order again.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import etdrk4 as E
from oracle import phi_exact as X
from paper_2211_00696_amd import inputs as I

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def dense(mats):
    return X.kron_sum(mats)


def test_zero_forcing_is_exact():
    rng = np.random.default_rng(0)
    mats = [I.fd_laplacian(6), I.adv_diff_1d(5, 0.7, 3.0)]
    u = rng.standard_normal(30)
    h = 0.03
    got = E.etdrk4_step(mats, h, u, lambda x: np.zeros_like(x))
    ref = scipy.linalg.expm(-h * dense(mats)) @ u
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_constant_forcing_is_exact():
    rng = np.random.default_rng(1)
    mats = [I.fd_laplacian(5), I.fd_laplacian(4), I.adv_diff_1d(3, 2.0, 1.0)]
    N = 60
    u = rng.standard_normal(N)
    c = rng.standard_normal(N)
    h = 0.05
    got = E.etdrk4_step(mats, h, u, lambda x: c)
    M = -h * dense(mats)
    phi1 = np.linalg.solve(M, scipy.linalg.expm(M) - np.eye(N))
    ref = scipy.linalg.expm(M) @ u + h * (phi1 @ c)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def bernoulli(u0, a, t):
    # u' = a u - u^3
    e = math.exp(2 * a * t)
    return u0 * math.exp(a * t) / math.sqrt(1.0 + u0 * u0 * (e - 1.0) / a)


@pytest.mark.parametrize("lam", [2.0, 5.0])
def test_scalar_fourth_order(lam):
    mats = [np.array([[lam]])]
    u0 = np.array([0.8])
    T = 1.0
    errs = []
    for steps in (10, 20, 40):
        u = E.etdrk4(mats, T / steps, u0, steps, F=lambda x: E.cubic(x, 1.0, -1.0))
        errs.append(abs(u[0] - bernoulli(0.8, 1.0 - lam, T)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(lam, errs, rates)
    assert all(3.6 < r < 4.6 for r in rates), rates


def test_allen_cahn_2d_fourth_order():
    n = 6
    mats = [0.05 * I.fd_laplacian(n), 0.05 * I.fd_laplacian(n)]
    A = dense(mats)
    rng = np.random.default_rng(0)
    u0 = rng.uniform(-1.0, 1.0, n * n)
    T = 0.5
    sol = scipy.integrate.solve_ivp(lambda t, u: -A @ u + u - u ** 3, (0, T), u0, method="Radau",
                                    rtol=1e-13, atol=1e-13, jac=lambda t, u: -A + np.diag(1 - 3 * u * u))
    ref = sol.y[:, -1]
    errs = []
    for steps in (4, 8, 16):
        errs.append(np.max(np.abs(E.etdrk4(mats, T / steps, u0, steps) - ref)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(errs, rates)
    assert all(3.5 < r < 4.7 for r in rates), rates
