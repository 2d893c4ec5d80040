"""Pins of the selector network's oracle: the hand-written backward pass
against central finite differences of the loss (FP64), and the parameter
count of the layout."""
import numpy as np

from oracle import mlp as M
from paper_2211_00696_amd import selector as S


def test_layout():
    assert M.NPARAM == 4866 == S.NPARAM


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    w = rng.standard_normal(M.NPARAM) * 0.3
    X = rng.standard_normal((37, 8))
    T = rng.standard_normal((37, 2))
    g = M.grad(w, X, T)
    idx = rng.choice(M.NPARAM, size=120, replace=False)
    idx = np.concatenate([idx, [0, 511, 512, 575, 576, 4671, 4672, 4799, 4800, 4863, 4864, 4865]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss(w + e, X, T) - M.loss(w - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_matches_sample_loop():
    rng = np.random.default_rng(1)
    w = rng.standard_normal(M.NPARAM) * 0.2
    X = rng.standard_normal((5, 8))
    W1, b1, W2, b2, W3, b3 = M.unpack(w)
    _, _, y = M.forward(w, X)
    for b in range(5):
        h1 = [np.tanh(sum(W1[i, k] * X[b, k] for k in range(8)) + b1[i]) for i in range(64)]
        h2 = [np.tanh(sum(W2[i, j] * h1[j] for j in range(64)) + b2[i]) for i in range(64)]
        for o in range(2):
            yo = sum(W3[o, i] * h2[i] for i in range(64)) + b3[o]
            assert abs(yo - y[b, o]) < 1e-12
