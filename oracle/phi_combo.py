"""Linear combinations sum_{j=0}^{p} phi_j(-tA) b_j (oracle).

Test infrastructure only.

* `combo_exact` is the definition: every term phi_j(-tA) b_j from the dense
  augmented-matrix exponential, summed.
* `combo_quad` follows the remark on linear combinations after Algorithm 2:
  sum_{j>=1} phi_j(Z) b_j = int_0^1 e^{(1-theta) Z} g(theta) dtheta with the
  forcing g(theta) = sum_j theta^{j-1}/(j-1)! b_j, Z = -tA.  The paper gives
  the one-pass quadrature without scaling; the scaling and squaring used here
  is this library's reading, written in the unnormalised form:
    x(s) = sum_j s^j phi_j(sZ) b_j solves x' = Z x + g(s), x(0) = 0;
    X_i(s) = sum_{k=1}^{p-i} s^k phi_k(sZ) b_{k+i}   (forcing shifted i places)
    X_i(2s) = e^{sZ} X_i(s) + sum_{r=0}^{p-1-i} s^r / r! X_{i+r}(s)
  (the second half of [0, 2s] is the same problem with g(r + s), whose
  Taylor expansion about r mixes the shifted forcings), and at the base
  s = 2^{-l} the Gauss rule gives
    X_i(s) = s sum_q w_q e^{(1 - theta_q) s Z} sum_k (s theta_q)^{k-1}/(k-1)! b_{k+i}.
  The result is e^{Z} b_0 + X_0(1).
The 1D exponentials are applied by mode products (eq. Expkron).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import quadrature
from .phi_exact import apply_kron, phi_dense_aug


def combo_exact(mats, t, bs):
    """sum_j phi_j(-tA) bs[j] (bs[j] may be None) from the augmented matrix."""
    p = len(bs) - 1
    out = None
    for j, b in enumerate(bs):
        if b is None:
            continue
        term = phi_dense_aug(mats, t, np.asarray(b, dtype=np.float64), max(j, 0))[j]
        out = term if out is None else out + term
    return out


def combo_quad(mats, t, bs, l, m):
    """The same sum by m-point Gauss quadrature at s = 2^{-l} and l doublings."""
    sizes = [a.shape[0] for a in mats]
    p = len(bs) - 1
    N = int(np.prod(sizes))
    b = [np.zeros(N) if x is None else np.asarray(x, dtype=np.float64).reshape(-1) for x in bs]
    Z1d = [-float(t) * np.asarray(a, dtype=np.float64) for a in mats]
    out = apply_kron([scipy.linalg.expm(z) for z in Z1d], b[0], sizes)
    if p == 0:
        return out
    s = 2.0 ** (-l)
    theta, w = quadrature.gauss_legendre(m)
    X = []
    for i in range(p):
        acc = np.zeros(N)
        for th, wq in zip(theta, w):
            g = np.zeros(N)
            for k in range(1, p - i + 1):
                g += (s * th) ** (k - 1) / math.factorial(k - 1) * b[k + i]
            acc += wq * apply_kron([scipy.linalg.expm((1.0 - th) * s * z) for z in Z1d], g, sizes)
        X.append(s * acc)
    for _ in range(l):
        E = [scipy.linalg.expm(s * z) for z in Z1d]
        new = []
        for i in range(p):
            nxt = apply_kron(E, X[i], sizes)
            for r in range(0, p - i):
                nxt = nxt + s ** r / math.factorial(r) * X[i + r]
            new.append(nxt)
        X = new
        s *= 2.0
    return out + X[0]
