"""phiq_plan_execute_noalloc: the plan execution that allocates nothing (its
intermediates in the library's fixed device array) against phiq_plan_execute
on the same plan and vector, through the C ABI.  Two calls in a row, the
second with a smaller problem; the array keeps the first call's contents, so
the second also checks that nothing stale is read.  Same kernels, same
launch sequence: the results must agree bit for bit."""
import numpy as np
import pytest

from paper_2211_00696_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SCRATCH = 64 << 20  # PHIQ_NOALLOC_SCRATCH_BYTES


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_00696_amd import phiq

    hd = phiq.Handle(0)
    yield hd
    hd.close()


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_noalloc_matches_plan_execute(h, precision):
    kw = dict(precision=precision, accept_floor=precision != "fp64")
    for pr in (I.problem("advdiff", seed=31, n=64, dim=3, t=1e-3), I.problem("advdiff", seed=32, n=40, dim=3, t=2e-3)):
        print("noalloc", precision, "n", pr["n"], flush=True)
        plan = h.plan(pr["mats"], pr["t"], 3, tol=1e-8, **kw)
        v = torch.from_numpy(pr["v"]).cuda()
        ref, _ = plan.execute(v)
        out = torch.full((4, v.numel()), float("nan"), dtype=torch.float64, device="cuda")
        need = plan.execute_noalloc(v, out)
        torch.cuda.synchronize()
        assert 0 < need <= SCRATCH
        assert torch.equal(out, ref.view(4, -1)), float((out - ref.view(4, -1)).abs().max())
        plan.close()


def test_noalloc_limits(h):
    from paper_2211_00696_amd import phiq

    # 3D n = 128: the intermediates exceed the fixed array
    pr = I.problem("advdiff3d", seed=0, n=128)
    plan = h.plan(pr["mats"], pr["t"], 3, tol=1e-8)
    v = torch.from_numpy(pr["v"]).cuda()
    out = torch.empty((4, v.numel()), dtype=torch.float64, device="cuda")
    with pytest.raises(phiq.PhiqError, match="OOM"):
        plan.execute_noalloc(v, out)
    plan.close()
    # the adaptive rule is refused
    pr = I.problem("advdiff", seed=33, n=16, dim=2, t=1e-2)
    plan = h.plan(pr["mats"], pr["t"], 2, tol=1e-8, rule="cc")
    v = torch.from_numpy(pr["v"]).cuda()
    out = torch.empty((3, v.numel()), dtype=torch.float64, device="cuda")
    with pytest.raises(phiq.PhiqError, match="UNSUPPORTED"):
        plan.execute_noalloc(v, out)
    plan.close()
