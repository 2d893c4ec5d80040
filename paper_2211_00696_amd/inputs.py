"""Seeded synthetic inputs for the phi-action workloads.

This module only builds inputs: 1D finite-difference operators, coefficient
draws and random vectors.  It holds none of the method's arithmetic and
imports nothing from the rest of the package, so both the oracle-based tests
and the HIP path can take their inputs from it.

Operators (1D, Dirichlet, n interior points, h = 1/(n+1)):
  * diffusion  T_n = tridiag(-1, 2, -1) / h^2   (FE-P1 with lumped mass gives
    the same matrix, Section 4, Problem 1)
  * advection  U_n = tridiag(-1, 1, 0) / h      (first-order upwind, backward
    difference for a non-negative velocity)
  * A^d = a_d T_n + b_d U_n
  * on a Shishkin mesh: -eps u'' + beta u' with non-uniform differences
  * FE-P1 with the consistent mass matrix: the dense M^{-1} K

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order:
a_1..a_d (log-uniform in [0.1, 10]), then b_1..b_d (uniform in [0, 50]),
then v ~ N(0, 1) of length N, stored row-major with axis 0 slowest.
"""
from __future__ import annotations

import math

import numpy as np


def fd_laplacian(n: int) -> np.ndarray:
    """Dirichlet second-difference matrix tridiag(-1, 2, -1)/h^2, h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    a = np.zeros((n, n))
    idx = np.arange(n)
    a[idx, idx] = 2.0
    a[idx[1:], idx[:-1]] = -1.0
    a[idx[:-1], idx[1:]] = -1.0
    return a / (h * h)


def fd_upwind(n: int) -> np.ndarray:
    """First-order upwind (backward difference) matrix tridiag(-1, 1, 0)/h."""
    h = 1.0 / (n + 1)
    a = np.zeros((n, n))
    idx = np.arange(n)
    a[idx, idx] = 1.0
    a[idx[1:], idx[:-1]] = -1.0
    return a / h


def adv_diff_1d(n: int, a: float, b: float) -> np.ndarray:
    """a * diffusion + b * upwind advection, both on n interior points."""
    return a * fd_laplacian(n) + b * fd_upwind(n)


def shishkin_mesh(n: int, eps: float, beta: float = 1.0, sigma: float = 2.0) -> np.ndarray:
    """The n interior nodes of a piecewise-uniform Shishkin mesh on (0, 1) for
    a boundary layer at x = 1 (advection to the right): (n+1)/2 equal cells on
    [0, 1 - tau] and (n+1)/2 on [1 - tau, 1], tau = min(1/2, sigma eps ln(n+1) / beta).
    n must be odd."""
    if n % 2 == 0:
        raise ValueError("n must be odd")
    cells = n + 1
    tau = min(0.5, sigma * eps * math.log(cells) / beta)
    left = np.linspace(0.0, 1.0 - tau, cells // 2 + 1)
    right = np.linspace(1.0 - tau, 1.0, cells // 2 + 1)
    x = np.concatenate([left, right[1:]])
    return x[1:-1]


def fd_adv_diff_nonuniform(x: np.ndarray, eps: float, beta: float) -> np.ndarray:
    """-eps u'' + beta u' on the interior nodes x of (0, 1), Dirichlet: the
    three-point second difference 2/(h_l + h_r) ((u_r - u)/h_r - (u - u_l)/h_l)
    (exact on quadratics) and the upwind difference (u - u_l)/h_l."""
    n = x.size
    xs = np.concatenate([[0.0], x, [1.0]])
    a = np.zeros((n, n))
    for i in range(n):
        hl = xs[i + 1] - xs[i]
        hr = xs[i + 2] - xs[i + 1]
        c = 2.0 / (hl + hr)
        a[i, i] = eps * c * (1.0 / hl + 1.0 / hr) + beta / hl
        if i > 0:
            a[i, i - 1] = -eps * c / hl - beta / hl
        if i < n - 1:
            a[i, i + 1] = -eps * c / hr
    return a


def fem_p1_consistent(n: int) -> np.ndarray:
    """Dense M^{-1} K of linear finite elements on n interior nodes of (0, 1)
    (uniform, Dirichlet): K = tridiag(-1, 2, -1)/h, consistent mass
    M = h tridiag(1/6, 2/3, 1/6); the product is a dense 1D operator."""
    h = 1.0 / (n + 1)
    idx = np.arange(n)
    K = np.zeros((n, n))
    K[idx, idx] = 2.0
    K[idx[1:], idx[:-1]] = -1.0
    K[idx[:-1], idx[1:]] = -1.0
    K /= h
    M = np.zeros((n, n))
    M[idx, idx] = 2.0 / 3.0
    M[idx[1:], idx[:-1]] = 1.0 / 6.0
    M[idx[:-1], idx[1:]] = 1.0 / 6.0
    M *= h
    return np.linalg.solve(M, K)


def draw_coefficients(rng: np.random.Generator, dim: int):
    """Per-axis (a_d, b_d): a_d log-uniform in [0.1, 10], b_d uniform in [0, 50]."""
    a = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=dim))
    b = rng.uniform(0.0, 50.0, size=dim)
    return a, b


def random_vector(rng: np.random.Generator, N: int) -> np.ndarray:
    return rng.standard_normal(N)


def problem(name: str, seed: int = 0, n: int | None = None, dim: int | None = None,
            t: float | None = None, p: int | None = None, tol: float | None = None):
    """Build one named synthetic workload.

    Returns a dict with keys: name, mats (list of n_d x n_d float64 arrays,
    axis 0 first), t, p, tol, v (float64, length N), coef (list of (a, b)).

    Names:
      * ``laplace2d`` -- 2D, A^x = A^y = T_32, t = 0.01, p = 3, tol 1e-8
      * ``advdiff3d`` -- 3D adv-diff, n = 128 by default, t = 1e-3, p = 3,
        tol 1e-8, coefficients drawn from the seed
      * ``advdiff``   -- same draw in any dim / n (small parity cases)
      * ``heat3d_eig``-- 3D Laplacian, n = 2^r - 1, t = 1/8, p = 20,
        tol 1e-14, v = sin(pi x) sin(pi y) sin(pi z) at the nodes
    """
    rng = np.random.default_rng(seed)
    if name == "laplace2d":
        n = 32 if n is None else n
        dim = 2 if dim is None else dim
        mats = [fd_laplacian(n) for _ in range(dim)]
        coef = [(1.0, 0.0)] * dim
        v = random_vector(rng, n ** dim)
        t = 0.01 if t is None else t
        p = 3 if p is None else p
        tol = 1e-8 if tol is None else tol
    elif name in ("advdiff3d", "advdiff"):
        n = 128 if n is None else n
        dim = 3 if dim is None else dim
        a, b = draw_coefficients(rng, dim)
        mats = [adv_diff_1d(n, float(a[d]), float(b[d])) for d in range(dim)]
        coef = [(float(a[d]), float(b[d])) for d in range(dim)]
        v = random_vector(rng, n ** dim)
        t = 1e-3 if t is None else t
        p = 3 if p is None else p
        tol = 1e-8 if tol is None else tol
    elif name == "heat3d_eig":
        n = 15 if n is None else n
        dim = 3 if dim is None else dim
        mats = [fd_laplacian(n) for _ in range(dim)]
        coef = [(1.0, 0.0)] * dim
        x = np.arange(1, n + 1) / (n + 1)
        s = np.sin(np.pi * x)
        v = s
        for _ in range(dim - 1):
            v = np.multiply.outer(v, s)
        v = np.ascontiguousarray(v).reshape(-1)
        t = 0.125 if t is None else t
        p = 20 if p is None else p
        tol = 1e-14 if tol is None else tol
    else:
        raise ValueError(f"unknown workload {name!r}")
    return dict(name=name, mats=mats, t=float(t), p=int(p), tol=float(tol), v=v,
                coef=coef, n=n, dim=dim, seed=seed)


def batch_mix(seed: int = 0, count: int = 512, n_min: int = 16, n_max: int = 192, p_max: int = 4,
              t_range=(1e-4, 1e-1), dims=(2, 3)):
    """A batch of independent problems of mixed shape.

    Per problem, drawn in this order from one ``default_rng(seed)``: the
    dimension (uniform over ``dims``), n (uniform integer in [n_min, n_max],
    the same on every axis), p (uniform in 1..p_max), t (log-uniform in
    t_range), the coefficients (a_d, b_d) as for ``advdiff``, then v ~ N(0, 1).
    Tolerance 1e-8.  Returns a list of problem dicts (see ``problem``).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dim = int(dims[rng.integers(0, len(dims))])
        n = int(rng.integers(n_min, n_max + 1))
        p = int(rng.integers(1, p_max + 1))
        t = float(math.exp(rng.uniform(math.log(t_range[0]), math.log(t_range[1]))))
        a, b = draw_coefficients(rng, dim)
        mats = [adv_diff_1d(n, float(a[d]), float(b[d])) for d in range(dim)]
        v = random_vector(rng, n ** dim)
        out.append(dict(name="batch_mix", mats=mats, t=t, p=p, tol=1e-8, v=v,
                        coef=[(float(a[d]), float(b[d])) for d in range(dim)], n=n, dim=dim, seed=seed, index=i))
    return out
