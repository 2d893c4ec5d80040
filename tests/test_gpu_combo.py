"""phiq_plan_execute_combo: sum_j phi_j(-tA) b_j (the remark on linear
combinations after Algorithm 2, with scaling and squaring) against the
oracle, through the C ABI.

Bars:
* against the definition (dense augmented exponential, tiny grids) with plans
  at tol 1e-12: relative max-norm error below 1e-10;
* against the oracle's quadrature-and-squaring form with the same (l, m) on
  grids spanning several tiles with ragged tails: below 1e-12 (the same
  approximation, summed in another order);
* at the 3D n = 128 size (p = 3): against the sum of phi_j(-tA) b_j from
  separate plan executions (themselves parity-tested against the oracle at
  that size), below 1e-12;
* the exponential Runge-Kutta stages as combinations agree with the
  per-vector form to 1e-12 and with the oracle's Table RK schemes to 1e-10;
* with the adaptive Clenshaw-Curtis rule (Algorithm 2's doubling test on
  the base sums y_1..y_pe): against the definition (tiny grids, plan tol
  1e-12, also with scaling exponent l = 0 and with empty slots) below 1e-10,
  against the oracle's Gauss form with 24 nodes on grids spanning several
  tiles below 1e-9 (plan tol 1e-10), and a single vector in slot j against
  the plain adaptive execution to 1e-10;
* FP32 and split-bf16 plans (mode products in that form, node sums and
  squaring in FP64): against the FP64 combination with the same (l, m)
  below 3e-6 and 3e-5, the forms' error floors (8e-7 and 9e-6 per
  phi-action, measured) with room for the p terms; FP32 also at 3D n = 128
  with the resident-factor kernels forced on the plain and the squaring
  products (the last squaring step with an order offset and an accumulating
  store), below 3e-6.
"""
import numpy as np
import pytest

from oracle import exprk as R
from oracle import phi_combo as C
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


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def ops(sizes, seed=7):
    rng = np.random.default_rng(seed)
    mats = []
    for n in sizes:
        a = float(np.exp(rng.uniform(np.log(0.1), np.log(10))))
        b = float(rng.uniform(0, 50))
        mats.append(I.adv_diff_1d(n, a, b))
    return mats


def draw(rng, p, N, none=()):
    return [None if j in none else rng.standard_normal(N) for j in range(p + 1)]


def run(h, mats, t, bs, tol=1e-12, **opts):
    plan = h.plan(mats, t, len(bs) - 1, tol=tol, **opts)
    dev = [None if b is None else torch.from_numpy(b).cuda() for b in bs]
    out = plan.execute_combo(dev)
    torch.cuda.synchronize()
    rep = plan.report
    plan.close()
    return out.cpu().numpy(), rep


@pytest.mark.parametrize("sizes", [[9, 11], [5, 6, 7]])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("l", [None, 0, 1, 3])
def test_combo_vs_definition(h, sizes, p, l):
    mats = ops(sizes)
    N = int(np.prod(sizes))
    t = 0.02 if l is None else 4e-3
    rng = np.random.default_rng(100 * p + (l or 0))
    bs = draw(rng, p, N)
    print("combo vs definition", sizes, p, l, flush=True)
    kw = {} if l is None else dict(l=l, m=18)
    got, rep = run(h, mats, t, bs, **kw)
    ref = C.combo_exact(mats, t, bs)
    e = rel(got, ref)
    print(rep["l"], rep["m"], e, flush=True)
    assert e < 1e-10, e


@pytest.mark.parametrize("sizes,p,l,m", [([37, 50, 29], 3, 4, 10), ([130, 67], 4, 5, 11), ([70, 65, 33], 2, 2, 9),
                                         ([200, 150], 3, 6, 12)])
def test_combo_vs_oracle_quadrature(h, sizes, p, l, m):
    mats = ops(sizes, seed=3)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(5)
    bs = draw(rng, p, N)
    t = 1e-3
    print("combo vs oracle quadrature", sizes, p, l, m, flush=True)
    got, rep = run(h, mats, t, bs, l=l, m=m)
    assert (rep["l"], rep["m"]) == (l, m)
    ref = C.combo_quad(mats, t, bs, l=l, m=m)
    e = rel(got, ref)
    print(e, flush=True)
    assert e < 1e-12, e


@pytest.mark.parametrize("none", [(0,), (1,), (3,), (1, 2), (0, 1, 2), (1, 2, 3), (0, 2)])
def test_combo_zero_entries(h, none):
    sizes = [12, 17, 9]
    mats = ops(sizes, seed=9)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(len(none))
    bs = draw(rng, 3, N, none=none)
    print("combo with None at", none, flush=True)
    got, rep = run(h, mats, 0.01, bs)
    ref = C.combo_exact(mats, 0.01, bs)
    e = rel(got, ref)
    print(rep["l"], rep["m"], e, flush=True)
    assert e < 1e-10, e


def test_combo_single_vector_equals_execute(h):
    sizes = [33, 40, 21]
    mats = ops(sizes, seed=4)
    N = int(np.prod(sizes))
    v = torch.from_numpy(np.random.default_rng(8).standard_normal(N)).cuda()
    plan = h.plan(mats, 0.003, 3, tol=1e-10)
    full, _ = plan.execute(v)
    for j in range(4):
        bs = [None] * 4
        bs[j] = v
        got = plan.execute_combo(bs)
        e = float((got - full[0, j]).abs().max() / full[0, j].abs().max())
        print("slot", j, e, flush=True)
        assert e < 1e-13, (j, e)
    plan.close()


def test_combo_errors(h):
    from paper_2211_00696_amd import phiq

    sizes = [8, 8]
    mats = ops(sizes)
    N = 64
    b = torch.randn(N, dtype=torch.float64, device="cuda")
    plan = h.plan(mats, 0.01, 2)
    with pytest.raises(phiq.PhiqError, match="INVALID_ARG"):
        plan.execute_combo([None, None, None], out=torch.empty_like(b))
    with pytest.raises(phiq.PhiqError, match="INVALID_ARG"):
        plan.execute_combo([b, b, None], out=b)
    plan.close()
    b32 = torch.randn(32 * 32, dtype=torch.float64, device="cuda")
    plan = h.plan(ops([32, 32]), 0.01, 2, precision="int8")
    with pytest.raises(phiq.PhiqError, match="UNSUPPORTED"):
        plan.execute_combo([b32, b32, b32])
    plan.close()
    # the adaptive rule's doubling cap reached before the tolerance (at the paper's scaling: the
    # default picks an l whose 7-point rule converges within the cap)
    plan = h.plan(mats, 0.01, 2, tol=1e-14, rule="cc", cc_max_doublings=1, cc_scaling="paper")
    with pytest.raises(phiq.PhiqError, match="NOT_CONVERGED"):
        plan.execute_combo([b, b, b])
    plan.close()


def test_combo_full_size_n128(h):
    """3D n = 128, p = 3 at the advection-diffusion workload's plan."""
    pr = I.problem("advdiff3d", seed=0, n=128)
    mats, t = pr["mats"], pr["t"]
    N = 128 ** 3
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    bs = [torch.randn(N, dtype=torch.float64, device="cuda", generator=g) for _ in range(4)]
    plan = h.plan(mats, t, 3, tol=1e-8)
    print("full size combo, plan", plan.report["l"], plan.report["m"], flush=True)
    got = plan.execute_combo(bs)
    ref = torch.zeros(N, dtype=torch.float64, device="cuda")
    for j, b in enumerate(bs):
        out, _ = plan.execute(b)
        ref += out[0, j]
    torch.cuda.synchronize()
    e = float((got - ref).abs().max() / ref.abs().max())
    print(e, flush=True)
    plan.close()
    assert e < 1e-12, e


@pytest.mark.parametrize("method", [1, 2, 3])
def test_exprk_forms_agree(h, method):
    n = 127
    mats = [I.fd_laplacian(n), I.fd_laplacian(n)]
    u0 = torch.from_numpy(R.exact(n, 0.0)).cuda()
    ua = u0.clone()
    ub = u0.clone()
    print("exprk forms", method, flush=True)
    h.exprk(mats, method, 8, ua, tol=1e-12, form="separate")
    h.exprk(mats, method, 8, ub, tol=1e-12, form="combo")
    e = float((ua - ub).abs().max() / ua.abs().max())
    print(e, flush=True)
    assert e < 1e-12, e


@pytest.mark.parametrize("sizes", [[9, 11], [5, 6, 7]])
@pytest.mark.parametrize("p,t,none", [(1, 0.02, ()), (3, 0.02, ()), (4, 4e-3, (2,)), (3, 1e-5, ()), (2, 1e-5, (0,))])
def test_combo_cc_vs_definition(h, sizes, p, t, none):
    mats = ops(sizes, seed=11)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(7 * p)
    bs = draw(rng, p, N, none=none)
    print("cc combo vs definition", sizes, p, t, none, flush=True)
    got, rep = run(h, mats, t, bs, rule="cc")
    ref = C.combo_exact(mats, t, bs)
    e = rel(got, ref)
    print(rep["l"], e, flush=True)
    assert e < 1e-10, e
    if t == 1e-5:
        assert rep["l"] == 0


@pytest.mark.parametrize("sizes,p", [([37, 50, 29], 3), ([130, 67], 2), ([70, 65, 33], 4)])
def test_combo_cc_vs_oracle_gauss(h, sizes, p):
    mats = ops(sizes, seed=12)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(13)
    bs = draw(rng, p, N)
    t = 1e-3
    print("cc combo vs oracle Gauss form", sizes, p, flush=True)
    got, rep = run(h, mats, t, bs, tol=1e-10, rule="cc")
    ref = C.combo_quad(mats, t, bs, l=rep["l"], m=24)
    e = rel(got, ref)
    print(rep["l"], e, flush=True)
    assert e < 1e-9, e


def test_combo_cc_single_vector_equals_execute(h):
    sizes = [33, 40, 21]
    mats = ops(sizes, seed=14)
    N = int(np.prod(sizes))
    v = torch.from_numpy(np.random.default_rng(15).standard_normal(N)).cuda()
    plan = h.plan(mats, 0.003, 3, tol=1e-12, rule="cc")
    full, _ = plan.execute(v)
    for j in range(4):
        bs = [None] * 4
        bs[j] = v
        got = plan.execute_combo(bs)
        e = float((got - full[0, j]).abs().max() / full[0, j].abs().max())
        print("cc slot", j, e, flush=True)
        assert e < 1e-10, (j, e)
    plan.close()


@pytest.mark.parametrize("method", [1, 3])
def test_exprk_forms_agree_clenshaw_curtis(h, method):
    n = 63
    mats = [I.fd_laplacian(n), I.fd_laplacian(n)]
    u0 = torch.from_numpy(R.exact(n, 0.0)).cuda()
    ua = u0.clone()
    ub = u0.clone()
    print("exprk forms, cc", method, flush=True)
    h.exprk(mats, method, 4, ua, tol=1e-12, form="separate", rule="cc")
    h.exprk(mats, method, 4, ub, tol=1e-12, form="combo", rule="cc")
    e = float((ua - ub).abs().max() / ua.abs().max())
    print(e, flush=True)
    assert e < 1e-10, e


@pytest.mark.parametrize("precision,bar", [("fp32", 3e-6), ("bf16x3", 3e-5)])
@pytest.mark.parametrize("rule", ["gauss", "cc"])
def test_combo_lower_precision_vs_fp64(h, precision, bar, rule):
    sizes = [37, 50, 29]
    mats = ops(sizes, seed=16)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(17)
    bs = draw(rng, 3, N)
    print("combo", precision, rule, flush=True)
    ref, rep = run(h, mats, 1e-3, bs, tol=1e-8, rule=rule)
    kw = dict(l=rep["l"], m=rep["m"]) if rule == "gauss" else {}
    # tol 1e-8 lies below the form's rounding floor: accepted explicitly, the
    # bar is the floor
    got, _ = run(h, mats, 1e-3, bs, tol=1e-8, rule=rule, precision=precision, accept_floor=True, **kw)
    e = rel(got, ref)
    print(rep["l"], rep["m"], e, flush=True)
    assert e < bar, e


@pytest.mark.parametrize("sizes,p,b0,t", [([24, 40, 56], 3, True, 2e-3), ([64, 48], 1, True, 5e-3),
                                          ([33, 20, 17], 4, False, 2e-3), ([16, 24, 20], 2, True, 1e-7)])
def test_combo_fused_matches_separate_launches(h, sizes, p, b0, t):
    """With every b_1..b_p set (FP64, p <= 4) the node chains of all b_j and phi_0's chain of b_0 share one
    launch per mode product and one node sum (the combined coefficient table).  Same sums as the launches
    per vector (rhs_per_launch = 1) in another rounding order; fewer launches."""
    mats = ops(sizes, seed=11)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(p)
    bs = draw(rng, p, N, none=() if b0 else (0,))
    dev = [None if b is None else torch.from_numpy(b).cuda() for b in bs]
    print("combo fused vs separate", sizes, p, b0, t, flush=True)
    outs, counts = [], []
    for grp in (0, 1):
        plan = h.plan(mats, t, p, tol=1e-10, rhs_per_launch=grp)
        plan.execute_combo(dev)
        torch.cuda.synchronize()
        h.profile_start()
        o = plan.execute_combo(dev)
        st = h.profile_stop()
        outs.append(o.cpu().numpy())
        counts.append(sum(s["launches"] for k, s in st.items() if k.startswith("ttm")))
        plan.close()
    e = rel(outs[0], outs[1])
    print("rel diff", e, "mode-product launches fused / separate", counts, flush=True)
    assert e < 1e-13, e
    assert counts[0] < counts[1], counts


@pytest.fixture(scope="module")
def combo128(h):
    pr = I.problem("advdiff3d", seed=0, n=128)
    N = 128 ** 3
    rng = np.random.default_rng(23)
    bs = [rng.standard_normal(N) for _ in range(4)]
    ref, rep = run(h, pr["mats"], pr["t"], bs, tol=1e-8)
    return pr, bs, ref, rep


@pytest.mark.parametrize("store_cfg,square_cfg", [(1, 1), (3, 2), (0, 1), (0, 0), (-1, -1)])
def test_combo_fp32_n128_resident_vs_fp64(h, combo128, store_cfg, square_cfg):
    """FP32 linear combination at 3D n = 128 (p = 3, every b_j set) with the
    FP32 resident-factor kernels forced (kind 3: plain products, kind 4: the
    squaring steps, including the last one with an order offset and the
    accumulating store) or the general kernel (cfg 0), against the FP64
    combination with the same (l, m), below the FP32 bar 3e-6."""
    pr, bs, ref, rep = combo128
    h.tile_config(3, store_cfg)
    h.tile_config(4, square_cfg)
    try:
        got, _ = run(h, pr["mats"], pr["t"], bs, tol=1e-8, precision="fp32", accept_floor=True, l=rep["l"],
                     m=rep["m"])
    finally:
        h.tile_config(3, -1)
        h.tile_config(4, -1)
    e = rel(got, ref)
    print("fp32 combo n=128", store_cfg, square_cfg, rep["l"], rep["m"], e, flush=True)
    assert rep["l"] >= 1
    assert e < 3e-6, e
