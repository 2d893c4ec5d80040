"""3D advection-diffusion at n = 256 per axis (N = 16,777,216), phi_0..phi_3:
every precision form against the oracle, element by element.

The reference is the oracle's quadrature (Algorithm phiquadmv written out in
numpy, its own selection at eps = 1e-14, beta = 1), itself pinned against
the augmented-matrix definition in the CPU tests.  The error measure is the
relative inf-norm error per phi_k (Section 4).

  * FP64 mode products at tol 1e-8: every phi_k within 1e-8, with the
    Gauss rule and with adaptive Clenshaw-Curtis (Algorithm 2) at its
    default scaling (phiq_cc_scaling).
  * FP32 and split-bf16 products at tol 1e-6 and 1e-10: both tolerances lie
    below or near the forms' rounding floors, so the floor is accepted
    explicitly and asserted instead (PHIQ_FLOOR_FP32 = 2e-6,
    PHIQ_FLOOR_BF16X3 = 3e-5); the report must say whether tol was met.

Seed 0 is the benchmark's coefficient draw (alpha ~ 665); seeds 1 and 4
draw larger norms (more squaring steps).
"""
import numpy as np
import pytest

from oracle import phiquad as Q
from paper_2211_00696_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FLOOR = {"fp32": 2e-6, "bf16x3": 3e-5}


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_00696_amd import phiq

    hd = phiq.Handle(0)
    yield hd
    hd.close()


def rel_per_k(o, ref):
    return [float(np.max(np.abs(o[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in range(ref.shape[0])]


@pytest.mark.parametrize("seed", [0, 1, 4])
def test_c3_every_form_vs_oracle(h, seed):
    pr = I.problem("advdiff3d", seed=seed, n=256)
    print(f"C3 n=256 seed {seed}: oracle", flush=True)
    ref = Q.phiquadmv(pr["mats"], pr["t"], pr["v"], 3, eps=1e-14, beta=1.0)
    v = torch.from_numpy(pr["v"]).cuda()
    out = torch.empty((4, v.numel()), dtype=torch.float64, device="cuda")
    cases = [("fp64", 1e-8, "gauss"), ("fp64", 1e-8, "cc"), ("fp32", 1e-6, "gauss"), ("fp32", 1e-10, "gauss"),
             ("bf16x3", 1e-6, "gauss"), ("bf16x3", 1e-10, "gauss")]
    rows, bad = [], []
    for prec, tol, rule in cases:
        print(f"C3 seed {seed} {prec} {rule} tol {tol:g}", flush=True)
        kw = dict(rule=rule) if prec == "fp64" else dict(accept_floor=True)
        _, rep = h.action(pr["mats"], pr["t"], 3, v, tol=tol, precision=prec, out=out, **kw)
        torch.cuda.synchronize()
        errs = rel_per_k(out.cpu().numpy(), ref)
        bar = tol if prec == "fp64" else FLOOR[prec]
        rows.append((prec, rule, tol, rep["l"], rep["m"], errs, rep["tol_met"]))
        print(f"  l={rep['l']} m={rep['m']} alpha={rep['alpha']:.1f} tol_met={rep['tol_met']} "
              "rel err phi_0..3 = " + " ".join(f"{e:.2e}" for e in errs), flush=True)
        if max(errs) >= bar:
            bad.append((prec, rule, tol, errs, bar))
        assert rep["tol_met"] == (1 if tol >= (FLOOR.get(prec, 0.0)) else 0)
    assert not bad, bad
