"""Section 5's exponential Runge-Kutta methods on Problem 3 (phiq_exprk)
against the oracle's Table RK schemes, and their convergence orders.

Bars: relative max-norm difference to the oracle below 1e-10 (plans at tol
1e-12); at n = 127 (2^7 elements per axis) the error at T = 1 against the
exact solution x(1-x) y(1-y) e^t falls at rates 1, 2, 3 (windows of
+-0.35..0.6).  The FD system carries no space error for this source, so the
rates are those of the time integrators alone.
"""
import math

import numpy as np
import pytest

from oracle import exprk as R
from paper_2211_00696_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_00696_amd import phiq

    hd = phiq.Handle(0)
    yield hd
    hd.close()


def lap2d(n):
    return [I.fd_laplacian(n), I.fd_laplacian(n)]


@pytest.mark.parametrize("method", [1, 2, 3])
@pytest.mark.parametrize("rule,form", [("gauss", "separate"), ("gauss", "combo"), ("cc", "separate"), ("cc", "combo")])
def test_exprk_vs_oracle(h, method, rule, form):
    n = 7
    mats = lap2d(n)
    c2 = 0.5 if method == 2 else 1.0 / 3.0
    u0 = R.exact(n, 0.0)
    print("method", method, rule, form, flush=True)
    u = torch.from_numpy(u0.copy()).cuda()
    h.exprk(mats, method, 4, u, T=1.0, c2=c2, tol=1e-12, rule=rule, form=form)
    ref = R.solve(mats, method, 1.0, 4, u0, R.g_ho(n), c2)
    e = float(np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    print(e, flush=True)
    assert e < 1e-10, e


@pytest.mark.parametrize("method,order", [(1, 1), (2, 2), (3, 3)])
def test_exprk_orders_n127(h, method, order):
    n = 127
    mats = lap2d(n)
    ue = R.exact(n, 1.0)
    errs = []
    for steps in (4, 8, 16, 32):
        u = torch.from_numpy(R.exact(n, 0.0)).cuda()
        h.exprk(mats, method, steps, u, T=1.0, tol=1e-12)
        errs.append(float(np.max(np.abs(u.cpu().numpy() - ue))))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    print(method, errs, rates, flush=True)
    assert all(order - 0.35 < r < order + 0.6 for r in rates), rates
