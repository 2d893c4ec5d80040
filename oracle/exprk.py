"""Exponential Runge-Kutta methods of Section 5 (Table RK), oracle.

Test infrastructure only.  For u' = -A u + g(t, u) (the paper's form with
A the positive operator) and step tau, every method reads

  u+ = u + tau sum_i b_i(-tau A) (g(t + c_i tau, U_i) - A u),
  U_i = u + tau sum_j a_ij(-tau A) (g(t + c_j tau, U_j) - A u),

with the coefficients of Table RK, phi_{i,j} = phi_i(-c_j tau A):
  exponential Euler: b_1 = phi_1;
  RK2 (c_2):         a_21 = c_2 phi_{1,2}; b_1 = (1 - 1/(2 c_2)) phi_1,
                     b_2 = phi_1 / (2 c_2);
  RK3 (c_2, c_3 = 2/3): a_21 = c_2 phi_{1,2};
                     a_31 = (2/3) phi_{1,3} - 4/(9 c_2) phi_{2,3},
                     a_32 = 4/(9 c_2) phi_{2,3};
                     b_1 = phi_1 - (3/2) phi_2, b_2 = 0, b_3 = (3/2) phi_2.
The products with A are formed explicitly (dense), the phi actions by
`phi` (default: the augmented-matrix exponential, small grids).

Problem 3 (Hochbruck-Ostermann): on (0,1)^2 with Dirichlet conditions,
u_t - Lap u = 1/(1 + u^2) + f(x, y, t), f chosen so that
u = x(1-x) y(1-y) e^t solves it:
  f = u_ex + 2 e^t (x(1-x) + y(1-y)) - 1/(1 + u_ex^2).
"""
from __future__ import annotations

import math

import numpy as np

from .phi_exact import kron_sum, phi_dense_aug


def grid(n):
    return np.arange(1, n + 1) / (n + 1)


def exact(n, t):
    x = grid(n)
    q = x * (1 - x)
    return (np.multiply.outer(q, q) * math.exp(t)).reshape(-1)


def source(n, t):
    x = grid(n)
    q = x * (1 - x)
    ue = np.multiply.outer(q, q) * math.exp(t)
    lap = 2 * math.exp(t) * (np.add.outer(q, q))  # -Lap u_ex
    return (ue + lap - 1.0 / (1.0 + ue * ue)).reshape(-1)


def g_ho(n):
    def g(t, u):
        return 1.0 / (1.0 + u * u) + source(n, t)
    return g


def step(mats, method, tau, t, u, g, c2, phi=phi_dense_aug):
    A = kron_sum(mats)
    Au = A @ u

    def ph(c, v, k):  # phi_k(-c tau A) v
        return phi(mats, c * tau, v, k)[k]

    g1 = g(t, u)
    if method == 1:
        return u + tau * ph(1.0, g1 - Au, 1)
    if method == 2:
        U2 = u + tau * c2 * ph(c2, g1 - Au, 1)
        g2 = g(t + c2 * tau, U2)
        b1 = 1.0 - 1.0 / (2 * c2)
        b2 = 1.0 / (2 * c2)
        return u + tau * (b1 * ph(1.0, g1 - Au, 1) + b2 * ph(1.0, g2 - Au, 1))
    c3 = 2.0 / 3.0
    U2 = u + tau * c2 * ph(c2, g1 - Au, 1)
    g2 = g(t + c2 * tau, U2)
    U3 = u + tau * ((2.0 / 3.0) * ph(c3, g1 - Au, 1) - 4.0 / (9 * c2) * ph(c3, g1 - Au, 2)
                    + 4.0 / (9 * c2) * ph(c3, g2 - Au, 2))
    g3 = g(t + c3 * tau, U3)
    return u + tau * (ph(1.0, g1 - Au, 1) - 1.5 * ph(1.0, g1 - Au, 2) + 1.5 * ph(1.0, g3 - Au, 2))


def solve(mats, method, T, steps, u0, g, c2, phi=phi_dense_aug):
    tau = T / steps
    u = np.array(u0, dtype=np.float64, copy=True)
    for k in range(steps):
        u = step(mats, method, tau, k * tau, u, g, c2, phi)
    return u
