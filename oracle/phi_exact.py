"""Exact phi-function actions by definition (oracle; test infrastructure only).

Definitions followed (Section 2.1, eq. Varphi and eq. recurrence):
    phi_0(M) = e^M,
    phi_k(M) = int_0^1 e^{(1-theta) M} theta^{k-1}/(k-1)! dtheta,   k >= 1,
    phi_{k-1}(M) = M phi_k(M) + I/(k-1)!.
Kronecker sum (Section 2.2, eq. KronA):
    A = A^0 (x) I (x) I + I (x) A^1 (x) I + I (x) I (x) A^2,
with axis 0 the slowest-varying index of the row-major tensor, i.e. the
order of numpy.kron.  Every phi is taken of M = -t A (the experiments of
Section 4 use phi_p(-tau A)).
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
import scipy.linalg


# ----------------------------------------------------------------------------
# Kronecker sum, dense (eq. KronA)
# ----------------------------------------------------------------------------
def kron_sum(mats):
    """Dense A = sum_d I (x) .. (x) A^d (x) .. (x) I, axis 0 slowest."""
    sizes = [m.shape[0] for m in mats]
    N = int(np.prod(sizes))
    A = np.zeros((N, N))
    for d, Ad in enumerate(mats):
        term = np.ones((1, 1))
        for e, ne in enumerate(sizes):
            term = np.kron(term, Ad if e == d else np.eye(ne))
        A += term
    return A


# ----------------------------------------------------------------------------
# O1: augmented-matrix exponential (exact up to the expm's own rounding)
# ----------------------------------------------------------------------------
def phi_dense_aug(mats, t, v, p):
    """Return an array (p+1, N) with row k = phi_k(-t A) v, A = kron_sum(mats).

    Construction: with J the p x p shift (ones on the superdiagonal) and
    e_1 the first unit vector, exp([[M, v e_1^T], [0, J]]) has in its column
    N+j-1 (j = 1..p) the vector phi_j(M) v.  Reason: z' = J z, z(0) = e_j
    gives z_1(theta) = theta^{j-1}/(j-1)!, and x' = M x + v z_1, x(0) = 0
    gives x(1) = int_0^1 e^{(1-theta) M} v theta^{j-1}/(j-1)! dtheta, which
    is eq. Varphi applied to v.  Feasible only for tiny N.
    """
    M = -float(t) * kron_sum(mats)
    N = M.shape[0]
    v = np.asarray(v, dtype=np.float64).reshape(N)
    out = np.empty((p + 1, N))
    out[0] = scipy.linalg.expm(M) @ v
    if p == 0:
        return out
    big = np.zeros((N + p, N + p))
    big[:N, :N] = M
    big[:N, N] = v
    for j in range(p - 1):
        big[N + j, N + j + 1] = 1.0
    X = scipy.linalg.expm(big)
    for j in range(1, p + 1):
        out[j] = X[:N, N + j - 1]
    return out


# ----------------------------------------------------------------------------
# scalar phi_k
# ----------------------------------------------------------------------------
def phi_scalar_mp(k, z, dps=50):
    """phi_k(z) for a real scalar z, in mpmath at `dps` digits.

    |z| <= 1: the power series sum_i z^i/(i+k)! (eq. Varphi integrated term
    by term); otherwise phi_0 = e^z and phi_j = (phi_{j-1} - 1/(j-1)!)/z
    (eq. recurrence), carried with k+25 guard digits, which covers the
    worst cancellation (a factor of at most j per step when |z| >= 1).
    """
    with mpmath.workdps(dps + k + 25):
        z = mpmath.mpf(z)
        if abs(z) <= 1:
            s = mpmath.mpf(0)
            term = 1 / mpmath.factorial(k)
            i = 0
            while abs(term) > mpmath.mpf(10) ** (-(dps + k + 20)) / mpmath.factorial(k):
                s += term
                i += 1
                term = term * z / (i + k)
            return +s
        ph = mpmath.e ** z
        for j in range(1, k + 1):
            ph = (ph - 1 / mpmath.factorial(j - 1)) / z
        return +ph


def phi_scalar(k, z):
    """phi_k(z) in float64 for an array of real z <= 0 (vectorised).

    |z| <= max(1, k+1): power series sum_i z^i/(i+k)!  (terms shrink from
    the first one, so little cancellation);
    otherwise: phi_0 = e^z then phi_j = (phi_{j-1} - 1/(j-1)!)/z, the scalar
    form of eq. recurrence, which is stable there because each step divides
    the error by |z| > j.
    """
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) <= max(1.0, k + 1.0)
    if np.any(small):
        zs = z[small]
        s = np.zeros_like(zs)
        term = np.full_like(zs, 1.0 / math.factorial(k))
        for i in range(1, 200):
            s += term
            term = term * zs / (i + k)
        out[small] = s
    big = ~small
    if np.any(big):
        zb = z[big]
        ph = np.exp(zb)
        for j in range(1, k + 1):
            ph = (ph - 1.0 / math.factorial(j - 1)) / zb
        out[big] = ph
    return out


# ----------------------------------------------------------------------------
# helpers: mode products on a row-major tensor (oracle's own)
# ----------------------------------------------------------------------------
def apply_kron(factors, v, sizes):
    """(F^0 (x) F^1 (x) ...) v for a row-major tensor of shape `sizes`.

    Mode d contracts axis d with F^d: out[.., i', ..] = sum_i F^d[i', i] x[.., i, ..]
    (eq. KronAb in row-major form).
    """
    X = np.asarray(v, dtype=np.float64).reshape(sizes)
    for d, F in enumerate(factors):
        X = np.moveaxis(np.tensordot(F, X, axes=([1], [d])), 0, d)
    return np.ascontiguousarray(X).reshape(-1)


def phi0_separable(mats, t, v):
    """phi_0(-tA) v = (e^{-tA^0} (x) e^{-tA^1} (x) ...) v  (eq. Expkron)."""
    sizes = [m.shape[0] for m in mats]
    return apply_kron([scipy.linalg.expm(-float(t) * m) for m in mats], v, sizes)


# ----------------------------------------------------------------------------
# O3: eigendecomposition closed form for A^d = a_d tridiag(-1,2,-1)/h^2
# ----------------------------------------------------------------------------
def laplacian_eig(n):
    """Eigenpairs of tridiag(-1,2,-1)/h^2, h = 1/(n+1), Dirichlet.

    lambda_k = (4/h^2) sin^2(k pi h / 2);  S[j,k] = sqrt(2/(n+1)) sin(j k pi h),
    j, k = 1..n.  S is symmetric and orthogonal.
    """
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    lam = (4.0 / h ** 2) * np.sin(k * np.pi * h / 2.0) ** 2
    S = math.sqrt(2.0 / (n + 1)) * np.sin(np.outer(k, k) * np.pi * h)
    return lam, S


def phi_eig_laplacian(sizes, diff_coefs, t, v, p):
    """phi_k(-t A) v, k = 0..p, for A = (+)_d a_d T_{n_d}, by diagonalisation.

    A = S (sum_d a_d Lambda_d) S with S = S_0 (x) S_1 (x) ... orthogonal, so
    phi_k(-tA) v = S [phi_k(-t lambda) .* (S v)] elementwise in the
    eigenbasis.  Valid only for symmetric (pure diffusion) operators.
    """
    lams, Ss = [], []
    for n, a in zip(sizes, diff_coefs):
        lam, S = laplacian_eig(n)
        lams.append(a * lam)
        Ss.append(S)
    lam_sum = np.zeros(())
    for lam in lams:
        lam_sum = np.add.outer(lam_sum, lam)
    lam_sum = lam_sum.reshape(-1)
    w = apply_kron(Ss, v, sizes)
    out = np.empty((p + 1, w.size))
    for k in range(p + 1):
        out[k] = apply_kron(Ss, phi_scalar(k, -float(t) * lam_sum) * w, sizes)
    return out


def laplacian_min_eig_3d_scalar(n):
    """(4/h^2) sin^2(pi h/2): the smallest eigenvalue of tridiag(-1,2,-1)/h^2."""
    h = 1.0 / (n + 1)
    return (4.0 / h ** 2) * math.sin(math.pi * h / 2.0) ** 2


# ----------------------------------------------------------------------------
# O4 helpers: Kronecker-sum matvec and recurrence residual (eq. recurrence)
# ----------------------------------------------------------------------------
def kron_sum_matvec(mats, x):
    """A x with A = (+)_d A^d, without forming A (sum of single-mode products)."""
    sizes = [m.shape[0] for m in mats]
    X = np.asarray(x, dtype=np.float64).reshape(sizes)
    out = np.zeros_like(X)
    for d, Ad in enumerate(mats):
        out += np.moveaxis(np.tensordot(Ad, X, axes=([1], [d])), 0, d)
    return out.reshape(-1)


def recurrence_residual(mats, t, v, phis):
    """max_k || M phi_k + v/(k-1)! - phi_{k-1} ||_inf / ||phi_{k-1}||_inf, M = -tA."""
    res = []
    for k in range(1, len(phis)):
        r = -float(t) * kron_sum_matvec(mats, phis[k]) + v / math.factorial(k - 1) - phis[k - 1]
        res.append(np.max(np.abs(r)) / np.max(np.abs(phis[k - 1])))
    return res
