"""Quadrature rules on [0, 1] (oracle; test infrastructure only).

The phi integral (Section 3.1) is taken over theta in [0, 1]; the rules are
built on s in [-1, 1] and mapped by theta = (1 + s)/2, w = omega/2, the same
change of variables as in the proof of Thm 3.2.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_legendre(m):
    """m-point Gauss-Legendre rule on [0, 1]: (theta, w), theta ascending."""
    s, omega = np.polynomial.legendre.leggauss(m)
    return (1.0 + s) / 2.0, omega / 2.0


def clenshaw_curtis(n):
    """(n+1)-point Clenshaw-Curtis rule on [0, 1], n >= 1.

    Nodes s_j = cos(j pi / n), j = 0..n (so theta runs from 1 down to 0).
    Weights integrate the degree-n interpolant at these points exactly:
    with the Chebyshev expansion of the interpolant and int T_k = 2/(1-k^2)
    for even k (0 for odd k) one gets
        omega_j = (c_j/n) * (1 - sum_{k=1}^{floor(n/2)} b_k cos(2 k j pi/n)/(4k^2 - 1)),
    c_j = 1 at j in {0, n} else 2, b_k = 1 if 2k = n else 2.
    Nested: the nodes with even j of the (2n+1)-point rule are the nodes of
    the (n+1)-point rule, in the same order (Algorithm 2).
    """
    j = np.arange(n + 1)
    s = np.cos(j * math.pi / n)
    omega = np.empty(n + 1)
    for jj in range(n + 1):
        acc = 1.0
        for k in range(1, n // 2 + 1):
            b = 1.0 if 2 * k == n else 2.0
            acc -= b * math.cos(2.0 * k * jj * math.pi / n) / (4.0 * k * k - 1.0)
        c = 1.0 if jj in (0, n) else 2.0
        omega[jj] = c * acc / n
    return (1.0 + s) / 2.0, omega / 2.0
