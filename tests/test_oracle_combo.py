"""Pins of the linear-combination oracle (the remark on linear combinations
after Algorithm 2, with scaling and squaring by the shifted-forcing recursion).

* The quadrature-and-squaring form against the definition (every term from
  the dense augmented-matrix exponential) on non-symmetric 2D and 3D
  operators, p = 1..4 and l = 0, 1, 3: a wrong factor s^r/r!, shift index or
  sign in the doubling fails at p >= 3 with l >= 1.
* A single vector in slot j reduces to the paper's algorithm for phi_j.
* Scalar closed form: 1 x 1 "matrices" give sum_j phi_j(z) b_j with phi_j
  evaluated in 50-digit arithmetic.
* The definition itself against the eigendecomposition closed form
  (symmetric diffusion).
"""
import numpy as np
import pytest

from oracle import phi_combo as C
from oracle import phi_exact as X
from oracle import phiquad as Q
from paper_2211_00696_amd import inputs as I


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def ops(dim):
    rng = np.random.default_rng(7)
    sizes = [5, 6] if dim == 2 else [3, 4, 5]
    mats = []
    for n in sizes:
        a = float(np.exp(rng.uniform(np.log(0.1), np.log(10))))
        b = float(rng.uniform(0, 50))
        mats.append(I.adv_diff_1d(n, a, b))
    return mats, sizes


def vectors(rng, p, N):
    return [rng.standard_normal(N) for _ in range(p + 1)]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("l", [0, 1, 3])
def test_quadrature_with_squaring_matches_definition(dim, p, l):
    mats, sizes = ops(dim)
    N = int(np.prod(sizes))
    alpha = sum(np.max(np.sum(np.abs(a), axis=1)) for a in mats)
    t = 6.0 / alpha  # ||tA||_inf = 6
    rng = np.random.default_rng(p * 10 + l)
    bs = vectors(rng, p, N)
    ref = C.combo_exact(mats, t, bs)
    got = C.combo_quad(mats, t, bs, l=l, m=16)
    assert rel(got, ref) < 1e-12


@pytest.mark.parametrize("j,p", [(1, 1), (2, 3), (3, 3), (4, 4)])
def test_single_vector_reduces_to_the_papers_algorithm(j, p):
    mats, sizes = ops(3)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(j)
    v = rng.standard_normal(N)
    t = 0.05
    l, m = 3, 10
    bs = [None] * (p + 1)
    bs[j] = v
    got = C.combo_quad(mats, t, bs, l=l, m=m)
    ref = Q.phiquadmv(mats, t, v, j, l=l, n=m - 1)[j]
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("z", [-0.5, -3.0, -30.0])
@pytest.mark.parametrize("l", [0, 2, 5])
def test_scalar_closed_form(z, l):
    p = 4
    coef = [0.7, -1.3, 2.1, 0.4, -0.9]
    ref = sum(c * float(X.phi_scalar_mp(j, z)) for j, c in enumerate(coef))
    bs = [np.array([c]) for c in coef]
    got = C.combo_quad([np.array([[1.0]])], -z, bs, l=l, m=20)
    assert abs(got[0] - ref) <= 1e-13 * max(1.0, abs(ref))


def test_none_entries_are_zero_vectors():
    mats, sizes = ops(2)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(3)
    bs = vectors(rng, 3, N)
    bs_none = [bs[0], None, bs[2], None]
    bs_zero = [bs[0], np.zeros(N), bs[2], np.zeros(N)]
    a = C.combo_quad(mats, 0.02, bs_none, l=2, m=10)
    b = C.combo_quad(mats, 0.02, bs_zero, l=2, m=10)
    assert np.array_equal(a, b)
    assert rel(C.combo_exact(mats, 0.02, bs_none), C.combo_exact(mats, 0.02, bs_zero)) < 1e-15


def test_definition_against_eigendecomposition():
    sizes, coefs = [6, 7], [0.8, 2.5]
    mats = [a * I.fd_laplacian(n) for n, a in zip(sizes, coefs)]
    N = int(np.prod(sizes))
    rng = np.random.default_rng(11)
    bs = vectors(rng, 3, N)
    t = 0.004
    ref = sum(X.phi_eig_laplacian(sizes, coefs, t, b, 3)[j] for j, b in enumerate(bs))
    assert rel(C.combo_exact(mats, t, bs), ref) < 1e-13
