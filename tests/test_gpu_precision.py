"""Lower-precision mode products (FP32 MFMA, split-bf16 x3) against the oracle.

Error model (per mode product of length K, FP32 accumulation):
  * FP32: operands rounded to 2^-24, accumulation error ~ K 2^-24 in the
    worst case, ~ sqrt(K) 2^-24 typically -> ~1e-6 relative after three
    modes and the recurrence.
  * split bf16: x = hi + lo keeps 16 significant bits (representation error
    <= 2^-17 |x|); the dropped lo*lo term is <= 2^-16 |a b|; so each product
    carries ~2^-15 relative error -> ~1e-5..1e-4 after three modes.
The thresholds below sit above these estimates with a margin; the measured
values are printed.  The 1D exponentials, node sums and squaring
recurrence stay FP64, so the errors do not grow with the number of squaring
steps beyond the error of each product.
"""
import numpy as np
import pytest

from oracle import phi_exact as X, phiquad as Q
from paper_2211_00696_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_KRON = {"fp32": 2e-6, "bf16x3": 2e-4}
TOL_PHI = {"fp32": 2e-5, "bf16x3": 1e-3}


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_00696_amd import phiq

    hd = phiq.Handle(0)
    yield hd
    hd.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(x):
    torch.cuda.synchronize()
    return x.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("sizes", [(16, 16), (33, 20, 17), (64, 64, 64), (128, 128), (130, 7, 65)])
def test_kron_apply_low_precision(h, prec, sizes):
    rng = np.random.default_rng(len(sizes) * 100 + sizes[0])
    # factors like the 1D exponentials: well-scaled, mostly positive
    F = [np.abs(rng.standard_normal((n, n))) / n + np.eye(n) for n in sizes]
    N = int(np.prod(sizes))
    x = rng.standard_normal((2, N))
    y = host(h.kron_apply([dev(f) for f in F], dev(x), precision=prec))
    errs = [rel(y[r], X.apply_kron(F, x[r], list(sizes))) for r in range(2)]
    print(prec, sizes, errs, flush=True)
    assert max(errs) < TOL_KRON[prec], errs


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("rule", ["gauss", "cc"])
def test_phi_action_low_precision_small(h, prec, rule):
    pr = I.problem("advdiff", seed=2, n=9, dim=3, t=1e-2)
    out, rep = h.action(pr["mats"], pr["t"], 3, dev(pr["v"]), tol=1e-8, rule=rule, precision=prec)
    ref = X.phi_dense_aug(pr["mats"], pr["t"], pr["v"], 3)
    o = host(out)
    errs = [rel(o[k], ref[k]) for k in range(4)]
    print(prec, rule, rep["l"], rep["m"], errs, flush=True)
    assert max(errs) < TOL_PHI[prec], errs


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_phi_action_low_precision_n64_vs_fp64_path(h, prec):
    pr = I.problem("advdiff3d", seed=1, n=64)
    v = dev(pr["v"])
    ref, _ = h.action(pr["mats"], pr["t"], 3, v, tol=1e-10)
    out, rep = h.action(pr["mats"], pr["t"], 3, v, tol=1e-10, precision=prec)
    r, o = host(ref), host(out)
    errs = [rel(o[k], r[k]) for k in range(4)]
    print(prec, "n=64", rep["l"], rep["m"], errs, flush=True)
    assert max(errs) < TOL_PHI[prec], errs
    # the FP64 path itself against the oracle's quadrature
    o2 = Q.phiquadmv(pr["mats"], pr["t"], pr["v"], 3, eps=1e-14, beta=1.0)
    assert max(rel(r[k], o2[k]) for k in range(4)) < 1e-10
