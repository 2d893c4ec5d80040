"""CPU pins of the input generators that are not plain uniform differences:
the non-uniform three-point operator is exact on quadratics and the upwind
difference on linear functions; the Shishkin mesh has its two uniform parts;
the consistent-mass FE operator has the known discrete eigenpairs."""
import math

import numpy as np

from paper_2211_00696_amd import inputs as I


def test_shishkin_mesh_pieces():
    n, eps = 63, 1e-3
    x = I.shishkin_mesh(n, eps)
    tau = min(0.5, 2 * eps * math.log(n + 1))
    xs = np.concatenate([[0.0], x, [1.0]])
    h = np.diff(xs)
    assert x.size == n and np.all(h > 0)
    assert np.allclose(h[:32], (1 - tau) / 32) and np.allclose(h[32:], tau / 32)


def test_nonuniform_operator_exact_on_quadratics():
    eps, beta = 0.01, 3.0
    x = I.shishkin_mesh(31, eps, beta)
    A = I.fd_adv_diff_nonuniform(x, eps, beta)
    u = x * x
    r = A @ u
    # interior rows away from the boundary: -eps * 2 + beta * (upwind of x^2)
    xs = np.concatenate([[0.0], x, [1.0]])
    hl = np.diff(xs)[:-1]
    up = (x * x - (x - hl) ** 2) / hl
    ref = -2 * eps + beta * up
    assert np.max(np.abs(r[1:-1] - ref[1:-1])) < 1e-9 * np.max(np.abs(ref))
    # the upwind difference is exact on linear functions
    A0 = I.fd_adv_diff_nonuniform(x, 0.0, 1.0)
    assert np.max(np.abs((A0 @ x)[1:] - 1.0)) < 1e-12


def test_fem_consistent_mass_eigenpairs():
    n = 24
    A = I.fem_p1_consistent(n)
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    for k in (1, 5, 17):
        v = np.sin(k * math.pi * j * h)
        c = math.cos(k * math.pi * h)
        lam = 6.0 / h ** 2 * (1 - c) / (2 + c)
        assert np.max(np.abs(A @ v - lam * v)) < 1e-9 * lam
    assert np.count_nonzero(np.abs(A) > 1e-12) > n * n // 2  # dense
