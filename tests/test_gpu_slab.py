"""Products along axes 2 and 1 in one pass per 128 x 128 slab (three-axis
tensors with n_1 = n_2 = 128, FP64), followed by the axis-0 product on the
natural layout.  The slab form computes the same sums as one axis per pass
(eq. Expkron), with the k-loops associated differently, so:

* against the one-axis-per-pass path on the same plan (itself parity-tested
  against the oracle): relative max-norm difference per phi_k below 1e-12;
* against the oracle's quadrature-and-squaring form (n_0 = 9): below the
  requested tolerance 1e-10;
* with slab_products = 2 the node chains (any node count), the squaring
  steps, phi_0 alone, the adaptive Clenshaw-Curtis rule and linear
  combinations all take the slab path; n_0 = 1 and n_0 not a multiple of
  anything exercise the block split;
* slab_products = 1 takes it for single-vector chains only; the default is
  0 (one axis per pass everywhere).
"""
import numpy as np
import pytest

from oracle import phiquad as Q
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


def ops(sizes, seed):
    rng = np.random.default_rng(seed)
    a, b = I.draw_coefficients(rng, len(sizes))
    return [I.adv_diff_1d(n, float(a[d]), float(b[d])) for d, n in enumerate(sizes)]


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def both(h, mats, t, p, v, **kw):
    """The slab path and the one-axis-per-pass path on the same inputs."""
    s, rs = h.action(mats, t, p, v, slab_products=2, **kw)
    r, rr = h.action(mats, t, p, v, slab_products=0, **kw)
    torch.cuda.synchronize()
    assert (rs["l"], rs["m"]) == (rr["l"], rr["m"])
    return s, r, rs


@pytest.mark.parametrize("n0,p,seed", [(128, 3, 0), (40, 2, 1), (1, 3, 2), (3, 4, 3), (129, 1, 4)])
def test_slab_matches_one_axis_path(h, n0, p, seed):
    sizes = [n0, 128, 128]
    mats = ops(sizes, seed)
    N = int(np.prod(sizes))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    v = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    print("slab vs one axis per pass", sizes, p, flush=True)
    s, r, rep = both(h, mats, 1e-3, p, v, tol=1e-8)
    errs = [rel(s[k], r[k]) for k in range(p + 1)]
    print(rep["l"], rep["m"], errs, flush=True)
    assert max(errs) < 1e-12, errs


@pytest.mark.parametrize("m", [1, 3, 17])
def test_slab_node_counts(h, m):
    """Forced node counts: slab counts 40 m, not multiples of the 128 block pairs."""
    sizes = [40, 128, 128]
    mats = ops(sizes, 10 + m)
    N = int(np.prod(sizes))
    v = torch.from_numpy(np.random.default_rng(m).standard_normal(N)).cuda()
    print("slab, forced m", m, flush=True)
    s, r, rep = both(h, mats, 1e-3, 3, v, tol=1e-8, l=2, m=m)
    errs = [rel(s[k], r[k]) for k in range(4)]
    print(rep["l"], rep["m"], errs, flush=True)
    assert max(errs) < 1e-12, errs


def test_slab_phi0_only(h):
    sizes = [64, 128, 128]
    mats = ops(sizes, 20)
    N = int(np.prod(sizes))
    v = torch.from_numpy(np.random.default_rng(20).standard_normal(N)).cuda()
    s, r, _ = both(h, mats, 2e-3, 0, v, tol=1e-10)
    e = rel(s[0], r[0])
    print("phi_0 only", e, flush=True)
    assert e < 1e-12, e


def test_slab_clenshaw_curtis(h):
    sizes = [24, 128, 128]
    mats = ops(sizes, 21)
    N = int(np.prod(sizes))
    v = torch.from_numpy(np.random.default_rng(21).standard_normal(N)).cuda()
    s, r, rep = both(h, mats, 1e-3, 3, v, tol=1e-8, rule="cc")
    errs = [rel(s[k], r[k]) for k in range(4)]
    print("cc", rep["l"], rep["m"], errs, flush=True)
    assert max(errs) < 1e-12, errs


def test_slab_combination(h):
    sizes = [32, 128, 128]
    mats = ops(sizes, 22)
    N = int(np.prod(sizes))
    rng = np.random.default_rng(22)
    bs = [torch.from_numpy(rng.standard_normal(N)).cuda() for _ in range(4)]
    got = []
    for slab in (2, 0):
        plan = h.plan(mats, 1e-3, 3, tol=1e-10, slab_products=slab)
        got.append(plan.execute_combo(bs))
        plan.close()
    torch.cuda.synchronize()
    e = rel(got[0], got[1])
    print("combination", e, flush=True)
    assert e < 1e-12, e


def test_slab_vs_oracle_quadrature(h):
    sizes = [9, 128, 128]
    mats = ops(sizes, 23)
    N = int(np.prod(sizes))
    v = np.random.default_rng(23).standard_normal(N)
    print("slab vs oracle quadrature", sizes, flush=True)
    out, rep = h.action(mats, 1e-3, 2, torch.from_numpy(v).cuda(), tol=1e-10, slab_products=2)
    ref = Q.phiquadmv(mats, 1e-3, v, 2, eps=1e-14, beta=1.0)
    o = out.cpu().numpy()
    errs = [float(np.max(np.abs(o[k] - ref[k])) / np.max(np.abs(ref[k]))) for k in range(3)]
    print(rep["l"], rep["m"], errs, flush=True)
    assert max(errs) < 1e-10, errs


def test_slab_repeat_bitwise(h):
    """Same inputs twice: the same bits (no order-dependent reduction)."""
    sizes = [128, 128, 128]
    mats = ops(sizes, 24)
    v = torch.from_numpy(np.random.default_rng(24).standard_normal(128 ** 3)).cuda()
    a, _ = h.action(mats, 1e-3, 3, v, tol=1e-8, slab_products=2)
    b, _ = h.action(mats, 1e-3, 3, v, tol=1e-8, slab_products=2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_slab_modes(h):
    """slab_products = 1: the phi_0 chain takes the slab path, the batched
    chains do not, so phi_1.. agree bitwise with 0 and phi_0 with 2 up to the
    order of the k sums (the per-axis products of the node batch, which
    carries phi_0 as slot m, take the resident-factor kernel at n = 128 with
    eight or more vectors, whose k order differs from the slab kernel's);
    the default is 0."""
    sizes = [128, 128, 128]
    mats = ops(sizes, 25)
    v = torch.from_numpy(np.random.default_rng(25).standard_normal(128 ** 3)).cuda()
    one, _ = h.action(mats, 1e-3, 3, v, tol=1e-8, slab_products=1)
    zero, _ = h.action(mats, 1e-3, 3, v, tol=1e-8, slab_products=0)
    two, _ = h.action(mats, 1e-3, 3, v, tol=1e-8, slab_products=2)
    dflt, _ = h.action(mats, 1e-3, 3, v, tol=1e-8)
    torch.cuda.synchronize()
    assert torch.equal(one[1:], zero[1:])
    e0 = float((one[0] - two[0]).abs().max() / two[0].abs().max())
    assert e0 < 1e-13, e0
    assert torch.equal(dflt, zero)
