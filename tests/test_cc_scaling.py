"""Scaling of adaptive Clenshaw-Curtis by the cost of the nodes Algorithm 2 runs (phiq_cc_scaling).

Algorithm 2 runs nested rules of 7, 13, 25, ... points and stops at the first
level whose change from the previous one is below eps, so it pays for one
level past the first accurate rule.  The planner's default predicts that
level from the Clenshaw-Curtis bound of Thm 3.2 at a quarter of the norm and
takes the l in [l_paper - 1, l_paper + 3] with the least chain count n + l p
(n + 1 = the nodes run).  Checked on the host:

  * the rule, restated here, on a grid of tolerances, orders and norms;
  * limits: alpha = 0 and p = 0 keep the paper's l, argument errors;
  * against measured run times (tests/data/cc_scaling_n128.json, 16 draws of
    the 3D n = 128 problem at the paper's l and three above it): on every
    draw the rule's l runs within 7% of the fastest measured l, and over the
    16 draws it takes 0.85x the time of Algorithm setup_quadrature's l (bar 0.86).
"""
import json
import math
import os

import pytest

from paper_2211_00696_amd import phiq

DATA = os.path.join(os.path.dirname(__file__), "data", "cc_scaling_n128.json")


def rule(eps, p, alpha, cap=6):
    l0, _, _ = phiq.setup_quadrature(eps, p, alpha, rule="cc")
    best = (math.inf, l0)
    for l in range(max(0, l0 - 1), l0 + 4):
        acc = next((j for j in range(cap) if phiq.log_quaderr(6 * 2 ** j, p, math.ldexp(alpha / 4, -l), 1.0, "cc")
                    <= math.log(eps)), None)
        if acc is None:
            continue
        n = 6 * 2 ** max(1, acc + 1)
        if n + l * p < best[0]:
            best = (n + l * p, l)
    return best[1]


@pytest.mark.parametrize("eps", [1e-6, 1e-8, 1e-10, 1e-12])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_rule(eps, p):
    for k in range(-4, 17):
        alpha = 10.0 ** (k / 4.0)
        assert phiq.cc_scaling(eps, p, alpha) == rule(eps, p, alpha), (eps, p, alpha)


def test_limits_and_errors():
    assert phiq.cc_scaling(1e-8, 3, 0.0) == phiq.setup_quadrature(1e-8, 3, 0.0, rule="cc")[0]
    assert phiq.cc_scaling(1e-8, 0, 500.0) == 0
    for args in ((0.0, 3, 10.0), (1e-8, -1, 10.0), (1e-8, 3, -1.0)):
        with pytest.raises(phiq.PhiqError, match="INVALID_ARG"):
            phiq.cc_scaling(*args)
    with pytest.raises(phiq.PhiqError, match="NONFINITE"):
        phiq.cc_scaling(1e-8, 3, float("nan"))
    with pytest.raises(phiq.PhiqError, match="INVALID_ARG"):
        phiq.cc_scaling(1e-8, 3, 10.0, max_doublings=0)


def test_against_measured_times():
    draws = json.load(open(DATA))["draws"]
    assert len(draws) == 16
    t_rule = t_paper = 0.0
    for d in draws:
        times = {int(l): v[1] for l, v in d["cc"].items()}
        l0 = phiq.setup_quadrature(1e-8, 3, d["alpha"], rule="cc")[0]
        lr = phiq.cc_scaling(1e-8, 3, d["alpha"])
        assert l0 in times and lr in times, (d["seed"], l0, lr, sorted(times))
        fastest = min(times.values())
        print(d["seed"], "paper l", l0, times[l0], "rule l", lr, times[lr], "fastest", fastest)
        assert times[lr] <= 1.07 * fastest, d["seed"]
        t_rule += times[lr]
        t_paper += times[l0]
    print("total: rule %.2f ms, paper %.2f ms, ratio %.3f" % (t_rule, t_paper, t_rule / t_paper))
    assert t_rule <= 0.86 * t_paper
