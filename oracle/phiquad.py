"""The paper's algorithm, written out plainly in FP64 numpy (oracle).

Test infrastructure only.  Steps follow Section 3 in the paper's order:
  * Algorithm 1 (fixed-point quadrature): v_i = e^{(1-x_i) A} b at every
    node, then y_j = sum_i w_i x_i^{j-1}/(j-1)! v_i for j = 1..p, the sum
    taken over all n+1 nodes.
  * Algorithm 2 (adaptive Clenshaw-Curtis): start with the 7-point rule
    (n = 3), double n while max_j ||y_j - y~_j||_inf/||y_j||_inf > eps,
    reusing the node vectors of the previous rule.
  * Algorithm phiquadmv (scaling and modified squaring): choose (l, n) by
    setup_quadrature, run the quadrature on 2^{-l} A, then for k = 0..l-1
    y_i <- 2^{-i} (e^{2^{k-l} A} y_i + sum_{j=1}^{i} y_j/(i-j)!)
    (eq. squaring), squaring the 1D exponentials between steps.
  * e^{A} b is applied through the 1D exponentials (eq. Expkron, KronAb).
All phi are of the matrix -t A.  phi_0 = e^{-tA} b is added from the
separable exponential, since the method's output starts at phi_1.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import bounds, quadrature
from .phi_exact import apply_kron


def _expm_1d(mats, scale):
    return [scipy.linalg.expm(scale * m) for m in mats]


def phiquadmv(mats, t, b, p, eps=1e-14, l=None, n=None, rule="gauss", alpha=None,
              beta=None, c1=0.0, c2=1.0, max_doublings=12, return_info=False):
    """phi_k(-t A) b for k = 0..p as an array (p+1, N).

    mats : list of n_d x n_d arrays A^d (axis 0 first, row-major tensor).
    beta : the vector-norm factor of the bound; default ||b||_inf as in the
           paper (pass 1.0 to read eps relative to ||b||_inf).
    l, n : override the selection (n is the paper's n; n+1 Gauss nodes).
    """
    sizes = [m.shape[0] for m in mats]
    M1d = [-float(t) * np.asarray(m, dtype=np.float64) for m in mats]
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    out = np.empty((p + 1, b.size))
    out[0] = apply_kron(_expm_1d(M1d, 1.0), b, sizes)
    info = dict(l=0, m=0, doublings=0)
    if p == 0:
        return (out, info) if return_info else out
    if alpha is None:
        alpha = bounds.infnorm_upper_bound(M1d)
    if beta is None:
        beta = float(np.max(np.abs(b)))
        if beta == 0.0:
            beta = 1.0
    if l is None:
        l_sel, n_sel, _ = bounds.setup_quadrature(eps, p, alpha, beta, rule, c1, c2, len(mats))
        l = l_sel
        if n is None:
            n = n_sel
    scaled = [2.0 ** (-l) * m for m in M1d]

    def node_vector(x):
        return apply_kron(_expm_1d(scaled, 1.0 - x), b, sizes)

    def weighted_sums(xs, ws, vs):
        ys = []
        for j in range(1, p + 1):
            y = np.zeros(b.size)
            for x, w, vv in zip(xs, ws, vs):
                y += w * x ** (j - 1) / math.factorial(j - 1) * vv
            ys.append(y)
        return ys

    if rule == "gauss":
        if n is None:
            raise ValueError("n required with a fixed l for the Gauss rule")
        xs, ws = quadrature.gauss_legendre(n + 1)
        vs = [node_vector(x) for x in xs]
        ys = weighted_sums(xs, ws, vs)
        info["m"] = n + 1
    else:
        nn = 3
        xs, ws = quadrature.clenshaw_curtis(2 * nn)
        vs = [node_vector(x) for x in xs]
        ys = weighted_sums(xs, ws, vs)
        err = math.inf
        doublings = 0
        while err > eps:
            if doublings >= max_doublings:
                raise RuntimeError("adaptive Clenshaw-Curtis did not converge")
            nn *= 2
            doublings += 1
            y_old = ys
            xs, ws = quadrature.clenshaw_curtis(2 * nn)
            new_vs = []
            for i in range(2 * nn + 1):
                if i % 2 == 0:
                    new_vs.append(vs[i // 2])
                else:
                    new_vs.append(node_vector(xs[i]))
            vs = new_vs
            ys = weighted_sums(xs, ws, vs)
            err = 0.0
            for y, yo in zip(ys, y_old):
                num = float(np.max(np.abs(y - yo)))
                den = float(np.max(np.abs(y)))
                err = max(err, num / den if den > 0 else num)
        info["m"] = 2 * nn + 1
        info["doublings"] = doublings
    info["l"] = l

    E = _expm_1d(scaled, 1.0)
    for k in range(l):
        new = []
        for i in range(1, p + 1):
            acc = apply_kron(E, ys[i - 1], sizes)
            for j in range(1, i + 1):
                acc = acc + ys[j - 1] / math.factorial(i - j)
            new.append(2.0 ** (-i) * acc)
        ys = new
        if k < l - 1:
            E = [e @ e for e in E]
    for j in range(1, p + 1):
        out[j] = ys[j - 1]
    return (out, info) if return_info else out
