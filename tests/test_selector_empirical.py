"""Host logic of the empirical mode of the learned (l, m) selector.

A sweep record lists forced pairs (l, m) of one problem with the measured
relative error e and the log10 a priori bound (Thm 3.2).  Checked without a
GPU, on hand-made records whose errors are built from the bound itself:

  * `norm_ratio` recovers the norm ratio rho a record was built with (the
    smallest rho whose bound at rho ||tA|| covers twice every error above
    1e-10), returns the lowest ratio when nothing is above the floor, and
    None when even the full norm does not cover an error;
  * the samples' targets are l / 8 of the cheapest modelled pair with m from
    Algorithm quadnodes at rho ||tA||, and log10 rho;
  * the host copy of the planner's empirical choice: l from the first
    output, m = Algorithm quadnodes at 10^y1 ||tA|| / 2^l (y1 clamped to
    [-1, 0]), Algorithm setup_quadrature's pair below tol 1e-10 (used 0) or
    when the network's pair costs over 1.5x its chain count (used 3);
  * a predicted pair is looked up in a record: a pair past the end of its
    l's sweep takes the sweep's last error there, a pair inside a gap the
    error at the largest swept m below it, a pair at an unswept l is
    unknown;
  * the packaged empirical network on stored held-out sweeps
    (tests/data/selector_holdout_sweeps.json, measured on the GPU by
    `selector sweep-errors`): every chosen pair's measured error is within
    tol.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2211_00696_amd import phiq
from paper_2211_00696_amd import selector as S

LN10 = math.log(10.0)


def bound10(m, p, alpha, l):
    return phiq.log_quaderr(m - 1, p, math.ldexp(alpha, -l)) / LN10


def record(p, alpha, rho, ls, ms, scale=0.5):
    """Errors = scale x the bound at rho alpha (the bound covers them exactly at scale 0.5)."""
    pts = []
    for l in ls:
        for m in ms:
            e = scale * 10.0 ** bound10(m, p, alpha * rho, l)
            pts.append([l, m, e, bound10(m, p, alpha, l)])
    return dict(n=64, dim=3, p=p, t=1e-3, alpha=alpha, norms=[alpha / 3] * 3, points=pts)


@pytest.mark.parametrize("p,alpha,rho", [(1, 40.0, 0.5), (3, 300.0, 0.62), (4, 2000.0, 0.4)])
def test_norm_ratio_recovers_the_ratio(p, alpha, rho):
    rec = record(p, alpha, rho, ls=range(max(0, int(math.log2(alpha)) - 6), int(math.log2(alpha)) + 1),
                 ms=range(2, 12))
    # keep only errors above the floor so that they bind
    lr = S.norm_ratio(rec)
    assert lr == pytest.approx(math.log10(rho), abs=1e-6)
    # an error twice as large needs a larger norm
    rec2 = record(p, alpha, rho, ls=[int(math.log2(alpha)) - 2], ms=range(2, 12), scale=1.0)
    assert S.norm_ratio(rec2) > lr


def test_norm_ratio_edges():
    # nothing above the floor: the lowest ratio
    rec = dict(n=32, dim=3, p=2, t=1e-3, alpha=50.0, norms=[1, 1, 1], points=[[3, 9, 1e-12, -9.0], [2, 12, 3e-11, -8.0]])
    assert S.norm_ratio(rec) == -1.0
    # an error the full norm's bound does not cover
    bad = record(2, 50.0, 1.0, ls=[2], ms=[4], scale=5.0)
    assert S.norm_ratio(bad) is None


def test_dataset_targets():
    rho = 0.5
    recs = [record(2, 120.0, rho, ls=range(1, 8), ms=range(2, 14)), record(3, 900.0, 0.7, ls=range(3, 11), ms=range(2, 16))]
    costs = {"64": dict(a=1.0, b=1.5, c=0.2, d=0.0), "128": dict(a=1.0, b=1.5, c=0.2, d=0.0)}
    T = S.cost_fn(costs)
    X, Y, meta = S.empirical_dataset(recs, costs, tols_per_problem=6, seed=2)
    assert X.shape == (12, S.NFEAT) and Y.shape == (12, 2)
    for y, mt, rec in zip(Y, meta, [recs[0]] * 6 + [recs[1]] * 6):
        lr = S.norm_ratio(rec)
        assert y[1] == pytest.approx(lr)
        l, m = S.label(T, rec["n"], rec["p"], rec["alpha"] * 10.0 ** lr, mt["tol"])
        assert (mt["l"], mt["m"]) == (l, m)
        assert y[0] == pytest.approx(l / S.L_SCALE)
        assert 1e-10 <= mt["tol"] <= 1e-6


def net(l, lr):
    """A network whose outputs are the constants (l / 8, lr)."""
    w = np.zeros(S.NPARAM, dtype=np.float32)
    w[-2:] = [l / S.L_SCALE, lr]
    return w


def test_empirical_pair_host_copy():
    rec = dict(n=128, dim=3, p=3, t=1e-3, alpha=500.0, norms=[200.0, 200.0, 100.0], points=[])
    l5, n5, _ = phiq.setup_quadrature(1e-8, 3, 500.0)
    for l, lr in ((l5, -0.3), (l5 - 1, -0.25), (l5 - 2, -0.4)):
        got = S.empirical_pair(net(l, lr), rec, 1e-8)
        assert got == (l, phiq.quadnodes(1e-8, 3, math.ldexp(500.0 * 10 ** lr, -l)) + 1, 4)
    # y1 is clamped to [-1, 0]
    assert S.empirical_pair(net(l5, 0.7), rec, 1e-8)[:2] == (l5, phiq.quadnodes(1e-8, 3, math.ldexp(500.0, -l5)) + 1)
    assert S.empirical_pair(net(l5, -3.0), rec, 1e-8)[:2] == (l5, phiq.quadnodes(1e-8, 3, math.ldexp(50.0, -l5)) + 1)
    # below the mode's range: Algorithm setup_quadrature's pair
    l9, n9, _ = phiq.setup_quadrature(1e-11, 3, 500.0)
    assert S.empirical_pair(net(l5, -0.3), rec, 1e-11) == (l9, n9 + 1, 0)
    # l = 0 at this norm costs far more than the paper's chain count: rejected
    assert S.empirical_pair(net(0, -0.3), rec, 1e-8) == (l5, n5 + 1, 3)


def test_lookup_of_a_predicted_pair():
    rec = dict(points=[[5, 2, 1e-3, -1.0], [5, 3, 1e-6, -4.0], [5, 4, 1e-9, -7.0], [5, 5, 1e-13, -10.0],
                       [4, 4, 1e-8, -5.0], [3, 2, 1e-1, 2.0], [3, 5, 1e-9, -3.0], [3, 8, 1e-14, -9.0]])
    assert S.swept_error(rec, 4, 4) == pytest.approx(1e-8)
    # past the end of l = 5's sweep: the last error measured there
    assert S.swept_error(rec, 5, 9) == pytest.approx(1e-13)
    # inside l = 3's gap: the largest swept m below (errors fall as m grows)
    assert S.swept_error(rec, 3, 4) == pytest.approx(1e-1)
    # l outside the swept range, or nothing at or below m
    assert S.swept_error(rec, 7, 4) is None
    assert S.swept_error(rec, 4, 3) is None


HOLDOUT = os.path.join(os.path.dirname(__file__), "data", "selector_holdout_sweeps.json")


@pytest.mark.skipif(not os.path.exists(S.WEIGHTS_EMPIRICAL), reason="no empirical selector weights in the package")
def test_committed_network_meets_tol_on_held_out_sweeps():
    """The packaged empirical network on the held-out sweeps (60 3D and 30 2D problems, seeds 2024 and
    2025, not used in training): at tol 1e-10..1e-6 every chosen pair lies in the sweep and its measured
    error is at most tol; the modelled time against Algorithm setup_quadrature's pair is printed."""
    recs = json.load(open(HOLDOUT))["records"]
    w = S.load_empirical()
    rows, summ = S.holdout(recs, w, S.load_costs())
    print(json.dumps(summ))
    assert summ["cases"] == 5 * len(recs) == 450
    assert summ["known"] == summ["cases"]
    assert summ["met"] == summ["cases"], [r for r in rows if r["err"] is not None and r["err"] > r["tol"]][:3]
    assert all(r["used"] == 4 for r in rows)
    assert summ["median_modelled_speedup"] > 1.05
