"""Pins of the CPU oracle against facts the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, brute force on tiny inputs, values printed in the paper, identities
evaluated in high precision, and invariants.  CPU only.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import bounds, phi_exact as X, phiquad as Q, quadrature as R
from paper_2211_00696_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# --------------------------------------------------------------------------
# scalar phi_k: eq. Varphi integrated numerically in mpmath
# --------------------------------------------------------------------------
def phi_by_integral(k, z):
    with mpmath.workdps(40):
        z = mpmath.mpf(z)
        if k == 0:
            return mpmath.e ** z
        f = lambda th: mpmath.e ** ((1 - th) * z) * th ** (k - 1) / mpmath.factorial(k - 1)
        return mpmath.quad(f, [0, 0.25, 0.5, 0.75, 1])


@pytest.mark.parametrize("k", [0, 1, 2, 3, 5, 8])
@pytest.mark.parametrize("z", [0.0, -1e-6, -0.3, -1.0, -2.5, -7.0, -40.0, -900.0])
def test_scalar_phi_matches_integral_definition(k, z):
    ref = phi_by_integral(k, z)
    mp = phi_scalar_mp = X.phi_scalar_mp(k, z)
    assert abs(mp - ref) <= 1e-28 * abs(ref)
    f = X.phi_scalar(k, np.array([z]))[0]
    assert abs(f - float(ref)) <= 2e-14 * abs(float(ref))


@pytest.mark.parametrize("k", [0, 1, 4, 10, 20])
def test_scalar_phi_float64_against_mp_grid(k):
    zs = -np.concatenate([np.linspace(0, 3, 31), np.geomspace(3, 2e4, 40)])
    f = X.phi_scalar(k, zs)
    for z, fz in zip(zs, f):
        ref = float(X.phi_scalar_mp(k, float(z)))
        assert abs(fz - ref) <= 5e-14 * abs(ref), (k, z, fz, ref)


def test_phi_at_zero_is_inverse_factorial():
    for k in range(0, 21):
        assert X.phi_scalar(k, np.array([0.0]))[0] == pytest.approx(1.0 / math.factorial(k), rel=1e-15)


# --------------------------------------------------------------------------
# Kronecker sum and mode products: brute force on tiny tensors (eq. KronA, KronAb)
# --------------------------------------------------------------------------
def test_kron_sum_matches_bruteforce_2d_and_3d():
    rng = np.random.default_rng(1)
    A0, A1, A2 = rng.standard_normal((2, 2)), rng.standard_normal((3, 3)), rng.standard_normal((4, 4))
    x = rng.standard_normal((2, 3, 4))
    ref = np.zeros_like(x)
    for i in range(2):
        for j in range(3):
            for k in range(4):
                s = 0.0
                for a in range(2):
                    s += A0[i, a] * x[a, j, k]
                for b in range(3):
                    s += A1[j, b] * x[i, b, k]
                for c in range(4):
                    s += A2[k, c] * x[i, j, c]
                ref[i, j, k] = s
    assert np.allclose(X.kron_sum([A0, A1, A2]) @ x.reshape(-1), ref.reshape(-1), rtol=0, atol=1e-13)
    assert np.allclose(X.kron_sum_matvec([A0, A1, A2], x.reshape(-1)), ref.reshape(-1), rtol=0, atol=1e-13)
    y = rng.standard_normal((2, 3))
    ref2 = A0 @ y + y @ A1.T
    assert np.allclose(X.kron_sum([A0, A1]) @ y.reshape(-1), ref2.reshape(-1), atol=1e-13)


def test_apply_kron_matches_bruteforce():
    rng = np.random.default_rng(2)
    F = [rng.standard_normal((2, 2)), rng.standard_normal((3, 3)), rng.standard_normal((4, 4))]
    x = rng.standard_normal((2, 3, 4))
    ref = np.einsum("ai,bj,ck,ijk->abc", F[0], F[1], F[2], x)
    assert np.allclose(X.apply_kron(F, x.reshape(-1), [2, 3, 4]), ref.reshape(-1), atol=1e-13)


# --------------------------------------------------------------------------
# O1 (augmented matrix) against closed forms
# --------------------------------------------------------------------------
def test_dense_aug_at_t0_gives_v_over_factorial():
    pr = I.problem("advdiff", seed=4, n=4, dim=2)
    out = X.phi_dense_aug(pr["mats"], 0.0, pr["v"], 5)
    for k in range(6):
        assert np.allclose(out[k], pr["v"] / math.factorial(k), rtol=1e-15, atol=0)


def test_dense_aug_scalar_case_matches_mpmath():
    # 1x1 axes: A = a0 + a1 + a2 is a scalar
    mats = [np.array([[2.5]]), np.array([[0.75]]), np.array([[4.0]])]
    t, v = 0.9, np.array([1.7])
    out = X.phi_dense_aug(mats, t, v, 6)
    z = -t * (2.5 + 0.75 + 4.0)
    for k in range(7):
        assert out[k][0] == pytest.approx(float(X.phi_scalar_mp(k, z)) * 1.7, rel=1e-13)


@pytest.mark.parametrize("sizes,coefs", [([9, 9], [1.0, 1.0]), ([6, 5, 7], [0.3, 2.0, 1.1]), ([13, 11], [0.5, 3.0])])
def test_dense_aug_matches_laplacian_eigen_closed_form(sizes, coefs):
    mats = [a * I.fd_laplacian(n) for n, a in zip(sizes, coefs)]
    rng = np.random.default_rng(5)
    v = rng.standard_normal(int(np.prod(sizes)))
    t = 3e-3
    o1 = X.phi_dense_aug(mats, t, v, 4)
    o3 = X.phi_eig_laplacian(sizes, coefs, t, v, 4)
    for k in range(5):
        assert rel(o1[k], o3[k]) < 1e-12


def test_dense_aug_satisfies_recurrence_nonsymmetric():
    pr = I.problem("advdiff", seed=7, n=6, dim=3, t=2e-2)
    o1 = X.phi_dense_aug(pr["mats"], pr["t"], pr["v"], 4)
    for r in X.recurrence_residual(pr["mats"], pr["t"], pr["v"], o1):
        assert r < 1e-12


def test_phi0_kronecker_of_1d_exponentials():
    pr = I.problem("advdiff", seed=8, n=5, dim=3, t=1e-2)
    o1 = X.phi_dense_aug(pr["mats"], pr["t"], pr["v"], 0)
    assert rel(X.phi0_separable(pr["mats"], pr["t"], pr["v"]), o1[0]) < 1e-13


def test_heat_eigenvector_closed_form_small():
    # Problem 1 (Section 4): b = sin(pi x) sin(pi y) sin(pi z) is the (1,1,1)
    # eigenvector, so phi_p(-tau A) b = phi_p(-tau lambda_111) b.
    pr = I.problem("heat3d_eig", n=7)
    lam = 3 * X.laplacian_min_eig_3d_scalar(7)
    o1 = X.phi_dense_aug(pr["mats"], pr["t"], pr["v"], 6)
    for k in range(7):
        ref = float(X.phi_scalar_mp(k, -pr["t"] * lam)) * pr["v"]
        assert rel(o1[k], ref) < 1e-12


# --------------------------------------------------------------------------
# quadrature rules
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [1, 2, 3, 5, 9, 16, 37])
def test_gauss_legendre_exact_to_degree_2m_minus_1(m):
    x, w = R.gauss_legendre(m)
    for deg in range(2 * m):
        assert np.dot(w, x ** deg) == pytest.approx(1.0 / (deg + 1), rel=1e-13, abs=1e-15)
    if m <= 5:  # and not exact one degree higher (the error is visible for small m)
        assert abs(np.dot(w, x ** (2 * m)) - 1.0 / (2 * m + 1)) > 1e-12


@pytest.mark.parametrize("n", [2, 4, 6, 12, 24, 48, 96])
def test_clenshaw_curtis_exact_to_degree_n(n):
    x, w = R.clenshaw_curtis(n)
    for deg in range(n + 1):
        assert np.dot(w, x ** deg) == pytest.approx(1.0 / (deg + 1), rel=1e-12, abs=1e-14)


def test_clenshaw_curtis_small_cases_and_nesting():
    x, w = R.clenshaw_curtis(2)  # Simpson's rule on [0, 1]
    assert np.allclose(x, [1.0, 0.5, 0.0]) and np.allclose(w, [1 / 6, 4 / 6, 1 / 6], atol=1e-15)
    for n in (3, 6, 12, 24):
        xo, _ = R.clenshaw_curtis(n)
        xn, _ = R.clenshaw_curtis(2 * n)
        assert np.allclose(xn[0::2], xo, atol=1e-15)


# --------------------------------------------------------------------------
# bounds and parameter selection
# --------------------------------------------------------------------------
def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("fname", ["points_laplace.json", "points_advdiff.json"])
def test_setup_quadrature_reproduces_paper_tables(fname):
    g = _golden(fname)
    p, eps = g["p"], g["eps"]
    for row in g["rows"]:
        _, alpha, gm, gc, gl, _cm, cc_cost, cl = row
        l, n, C = bounds.setup_quadrature(eps, p, alpha, 1.0, "gauss")
        assert (l, n + 1, n + 1 + l * p) == (gl, gm, gc)
        l2, _, _ = bounds.setup_quadrature(eps, p, alpha, 1.0, "cc")
        assert l2 == cl
        # the printed CC cost is consistent with its node count and scaling
        assert cc_cost == _cm + cl * p


def test_maximal_scaling_example_21_nodes():
    # Section 3.3: with l = log2(e/2 ||A||) the scaled norm is 2/e, and 21
    # nodes (n = 20) bring the bound below 1e-20 ||b|| for p <= 20.  For
    # Gauss this holds with a wide margin.  For Clenshaw-Curtis the same
    # closed form peaks at 1.6e-20 (p = 11), so the claim is read as an
    # order of magnitude there, and it needs n > p + 1.
    alpha = 2.0 / math.e
    for p in range(0, 21):
        assert bounds.corollary_log_bound(20, p, alpha, 1.0, "gauss") < math.log(1e-20)
    worst = max(bounds.corollary_log_bound(20, p, alpha, 1.0, "cc") for p in range(0, 19))
    assert math.log(1e-20) < worst < math.log(2e-20)
    # exact values of the closed forms at two points
    assert bounds.corollary_log_bound(20, 10, alpha, 1.0, "cc") == pytest.approx(
        math.log(10.0 ** -10 / (2 ** 11 * math.factorial(10))), rel=1e-13)
    assert bounds.corollary_log_bound(20, 3, alpha, 1.0, "gauss") == pytest.approx(
        math.log(37.0 ** -37 / (2 ** 4 * math.factorial(3))), rel=1e-13)


def test_theorem_bound_not_above_corollary_bound():
    for alpha in (0.5, 3.0, 10.0):
        for p in (0, 2, 5):
            for rule in ("gauss", "cc"):
                if rule == "gauss":
                    n0 = max(2, math.ceil((1 + math.sqrt(2)) / 4 * alpha + p / 2))
                else:
                    n0 = max(4, math.ceil((1 + math.sqrt(2)) / 2 * alpha + p))
                    n0 += n0 % 2
                for n in (n0, n0 + 2, n0 + 10):
                    _, lb = bounds.best_rho(n, p, alpha, 1.0, rule)
                    assert lb <= bounds.corollary_log_bound(n, p, alpha, 1.0, rule) + 1e-12


def test_quartic_root_is_the_minimiser_of_the_bound():
    for alpha, n, p, rule in [(5.0, 6, 0, "gauss"), (40.0, 20, 3, "gauss"), (12.0, 16, 2, "cc")]:
        rho, lb = bounds.best_rho(n, p, alpha, 1.0, rule)
        grid = np.linspace(1.0001, 30.0, 200000)
        vals = [bounds.log_bound(r, n, p, alpha, 1.0, rule) for r in grid[::50]]
        assert lb <= min(vals) + 1e-9


@pytest.mark.parametrize("rule", ["gauss", "cc"])
def test_bound_dominates_measured_quadrature_error(rule):
    # l = 0, fixed n: the Thm 3.2 bound (beta = ||b||_inf) must exceed the
    # actual error of the quadrature against the exact augmented-matrix action.
    pr = I.problem("advdiff", seed=11, n=5, dim=2, t=2e-3)
    exact = X.phi_dense_aug(pr["mats"], pr["t"], pr["v"], 3)
    alpha = bounds.infnorm_upper_bound(pr["mats"], pr["t"])
    beta = float(np.max(np.abs(pr["v"])))
    nmin = 2 if rule == "gauss" else 4
    for n in range(nmin, nmin + 12, 2):
        if rule == "cc":
            xs, ws = R.clenshaw_curtis(n)
        else:
            xs, ws = R.gauss_legendre(n + 1)
        # direct Algorithm 1 with the exact node exponentials
        import scipy.linalg
        M = -pr["t"] * X.kron_sum(pr["mats"])
        vs = [scipy.linalg.expm((1 - x) * M) @ pr["v"] for x in xs]
        for j in range(1, 4):
            y = sum(w * x ** (j - 1) / math.factorial(j - 1) * vv for x, w, vv in zip(xs, ws, vs))
            err = float(np.max(np.abs(y - exact[j])))
            _, lb = bounds.best_rho(n, j - 1, alpha, beta, rule)
            assert err <= math.exp(lb) * (1 + 1e-9) + 1e-15


def test_quadnodes_result_is_minimal_and_sufficient():
    for alpha, p, eps, rule in [(6.0, 3, 1e-8, "gauss"), (48.0, 20, 1e-14, "gauss"), (12.0, 4, 1e-10, "cc")]:
        n = bounds.quadnodes(eps, p, alpha, 1.0, rule)
        assert bounds.log_quaderr(n, p, alpha, 1.0, rule) <= math.log(eps)
        assert bounds.log_quaderr(n - 1, p, alpha, 1.0, rule) > math.log(eps)


def test_zero_norm_uses_exact_polynomial_rule():
    l, n, _ = bounds.setup_quadrature(1e-8, 5, 0.0, 1.0, "gauss")
    assert l == 0 and n + 1 == 3


# --------------------------------------------------------------------------
# O2 (the paper's algorithm in numpy) against the exact definitions
# --------------------------------------------------------------------------
@pytest.mark.parametrize("rule", ["gauss", "cc"])
def test_phiquadmv_matches_dense_2d_laplace(rule):
    pr = I.problem("laplace2d")
    o1 = X.phi_dense_aug(pr["mats"], pr["t"], pr["v"], 3)
    o2 = Q.phiquadmv(pr["mats"], pr["t"], pr["v"], 3, eps=1e-8, rule=rule, beta=1.0)
    for k in range(4):
        assert rel(o2[k], o1[k]) < 1e-8


@pytest.mark.parametrize("rule", ["gauss", "cc"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_phiquadmv_matches_dense_3d_nonsymmetric(rule, seed):
    pr = I.problem("advdiff", seed=seed, n=7, dim=3, t=1e-2)
    o1 = X.phi_dense_aug(pr["mats"], pr["t"], pr["v"], 4)
    o2 = Q.phiquadmv(pr["mats"], pr["t"], pr["v"], 4, eps=1e-8, rule=rule, beta=1.0)
    for k in range(5):
        assert rel(o2[k], o1[k]) < 1e-8


def test_phiquadmv_unequal_axes():
    rng = np.random.default_rng(3)
    mats = [I.adv_diff_1d(5, 0.7, 3.0), I.adv_diff_1d(8, 2.0, 10.0), I.adv_diff_1d(3, 0.2, 1.0)]
    v = rng.standard_normal(5 * 8 * 3)
    o1 = X.phi_dense_aug(mats, 5e-3, v, 3)
    o2 = Q.phiquadmv(mats, 5e-3, v, 3, eps=1e-10, beta=1.0)
    for k in range(4):
        assert rel(o2[k], o1[k]) < 1e-10


def test_phiquadmv_squaring_pinned_on_scalars():
    # 1x1 axes make every quantity a scalar; force several squaring steps
    # and compare with mpmath phi_k (eq. squaring must reproduce them).
    mats = [np.array([[3.0]]), np.array([[5.5]])]
    t, v = 2.0, np.array([1.0])
    z = -t * 8.5
    for l in (1, 3, 6):
        out = Q.phiquadmv(mats, t, v, 5, l=l, n=30, rule="gauss")
        for k in range(6):
            assert out[k][0] == pytest.approx(float(X.phi_scalar_mp(k, z)), rel=1e-12)


def test_phiquadmv_problem1_eigenvector_r5():
    # Problem 1 at r = 5 (N = 29791), p = 20, eps = 1e-14: errors below 1e-12
    # are what the paper reports (Section 4, Problem 1).
    pr = I.problem("heat3d_eig", n=31)
    lam = 3 * X.laplacian_min_eig_3d_scalar(31)
    out, info = Q.phiquadmv(pr["mats"], pr["t"], pr["v"], 20, eps=1e-14, return_info=True)
    assert (info["l"], info["m"]) == (5, 37)
    for k in range(21):
        ref = float(X.phi_scalar_mp(k, -pr["t"] * lam)) * pr["v"]
        assert rel(out[k], ref) < 1e-12
