"""A priori quadrature error bound and parameter selection (oracle).

Test infrastructure only.  Follows Section 3.2-3.3:
  * Thm 3.1 (Trefethen, Thm 19.3): Gauss error <= 144/35 M rho^{-2n}/(rho^2-1),
    Clenshaw-Curtis error <= 144/35 M rho^{1-n}/(rho^2-1), for (n+1) nodes.
  * Thm 3.2: M(rho) = g^p/(2^{p+1} p!) e^{g alpha/2} beta, g = (rho+1)^2/(2 rho),
    and the minimising rho solves rho^4 + a3 rho^3 + a2 rho^2 + a1 rho + 1 = 0
    with the coefficients of eq. polycoeffs.
  * Algorithm quaderr (max over q = 1..p, coefficients with p = q-1),
    Algorithm quadnodes (doubling, then a scalar root on [n/2, n], ceil),
    Algorithm setup_quadrature (l from ceil(log2 alpha) down to 0, stop when
    the cost C(n, l, p) = c1 d n + c2 (n + l p) stops decreasing).
  * The remark after Algorithm quadnodes: bounds are handled as logarithms.
  * eq. infnorm_upper_bnd: ||A||_inf <= sum_d ||A^d||_inf.
Corollary 3.3's closed forms are here too; they serve as pins.

Readings (where the text is silent):
  * rule "gauss" or "cc"; n is the paper's n (the rule has n+1 nodes).
  * roots: every real root > 1 of the quartic (imaginary part below
    1e-9 |rho|) is tried and the one with the smallest bound taken.
  * quadnodes: if the starting n already meets the tolerance it is returned
    unchanged (the bracket [n/2, n] would leave the theorem's range).
  * alpha <= 1e-12 (t = 0 or A = 0): the integrand is a polynomial of degree
    p-1, so l = 0 and ceil(p/2) Gauss nodes are exact.
  * ceil(log2 alpha) < 0 is clamped to 0.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.optimize

ALPHA_ZERO = 1e-12


def infnorm_upper_bound(mats, t=1.0):
    """alpha = sum_d ||t A^d||_inf  (eq. infnorm_upper_bnd)."""
    return sum(abs(float(t)) * float(np.max(np.sum(np.abs(m), axis=1))) for m in mats)


def polycoeffs(n, p, alpha, rule):
    """(a3, a2, a1) of eq. polycoeffs for the bound on phi_{p+1}."""
    if rule == "cc":
        a3 = -4.0 / alpha * (n + 1 - p)
        a1 = 4.0 / alpha * (n - 1 + p)
    else:
        a3 = -4.0 / alpha * (2 * (n + 1) - p)
        a1 = 4.0 / alpha * (2 * n + p)
    a2 = -(2.0 + 8.0 * p / alpha)
    return a3, a2, a1


def log_bound(rho, n, p, alpha, beta, rule):
    """log of the Thm 3.2 bound on ||phi_{p+1}(A) b - quadrature||_inf at rho."""
    g = (rho + 1.0) ** 2 / (2.0 * rho)
    logM = p * math.log(g) - (p + 1) * math.log(2.0) - math.lgamma(p + 1) + 0.5 * g * alpha + math.log(beta)
    if rule == "cc":
        lr = (1.0 - n) * math.log(rho)
    else:
        lr = -2.0 * n * math.log(rho)
    return math.log(144.0 / 35.0) + logM + lr - math.log(rho * rho - 1.0)


def best_rho(n, p, alpha, beta, rule):
    """Real root > 1 of the quartic minimising the bound: (rho, log bound)."""
    a3, a2, a1 = polycoeffs(n, p, alpha, rule)
    roots = np.roots([1.0, a3, a2, a1, 1.0])
    best = (None, math.inf)
    for r in roots:
        if abs(r.imag) <= 1e-9 * abs(r) and r.real > 1.0:
            lb = log_bound(float(r.real), n, p, alpha, beta, rule)
            if lb < best[1]:
                best = (float(r.real), lb)
    if best[0] is None:
        raise ArithmeticError("no real root > 1 (the proof of Thm 3.2 guarantees one)")
    return best


def log_quaderr(n, p, alpha, beta, rule):
    """Algorithm quaderr in log form: max over q = 1..p of the Thm 3.2 bound."""
    E = -math.inf
    for q in range(1, p + 1):
        _, lb = best_rho(n, q - 1, alpha, beta, rule)
        E = max(E, lb)
    return E


def quaderr(n, p, alpha, beta, rule):
    return math.exp(log_quaderr(n, p, alpha, beta, rule))


def quadnodes(eps, p, alpha, beta, rule):
    """Algorithm quadnodes: the paper's n (the rule then has n+1 nodes)."""
    n = 2 if rule == "gauss" else 4
    leps = math.log(eps)
    E = log_quaderr(n, p, alpha, beta, rule)
    if E <= leps:
        return n
    while E > leps:
        n *= 2
        E = log_quaderr(n, p, alpha, beta, rule)
    h = lambda x: log_quaderr(x, p, alpha, beta, rule) - leps
    root = scipy.optimize.brentq(h, n / 2.0, float(n), xtol=1e-12, rtol=1e-14, maxiter=200)
    return int(math.ceil(root))


def setup_quadrature(eps, p, alpha, beta, rule, c1=0.0, c2=1.0, d=3):
    """Algorithm setup_quadrature: returns (l, n, C) with the rule of n+1 nodes."""
    if p == 0:
        return 0, -1, 0.0
    if alpha <= ALPHA_ZERO:
        m = max(1, (p + 1) // 2)
        return 0, m - 1, c1 * d * (m - 1) + c2 * (m - 1)
    lmax = max(0, int(math.ceil(math.log2(alpha))))
    best = (None, None, math.inf)
    for l in range(lmax, -1, -1):
        al = alpha * 2.0 ** (-l)
        n = quadnodes(eps, p, al, beta, rule)
        C = c1 * d * n + c2 * (n + l * p)
        if C < best[2]:
            best = (l, n, C)
        else:
            break
    return best


def corollary_log_bound(n, p, alpha, beta, rule):
    """log of Corollary 3.3's closed-form bound on phi_{p+1} (valid range applies)."""
    if rule == "cc":
        nn = n if n % 2 == 0 else n - 1
        k = nn - p
    else:
        k = 2 * n - p
    return (math.log(beta) - (p + 1) * math.log(2.0) - math.lgamma(p + 1)
            - k * (math.log(k) - math.log(math.e / 2.0 * alpha)))
