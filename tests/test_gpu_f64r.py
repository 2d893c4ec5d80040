"""FP64 mode products with the 1D factor resident in LDS (kernels_f64r.hip).

The plain product (phiq_tile_config kind 5) and the product fused with the
modified squaring of eq. squaring (kind 6) for n_d in {64, 128, 256},
forced on every launch (cfg 1: four waves with all row blocks, 2: eight
waves in two row groups, 3: eight waves in one row group, 4 (plain):
sixteen, 5 (plain) / 4 (squaring): eight waves on 64-row blocks, 6 (plain):
sixteen waves on 64-row blocks; the default takes cfg 4 / 3 for n = 256
launches with at least one unit per CU and cfg 6 for n = 128 node batches
of eight or more), through the C ABI:

  * Kronecker products (F^0 (x) F^1 (x) F^2) x against the oracle's
    apply_kron (numpy, FP64) and against the tile kernels (cfg 0): the same
    sums in another k order, so within a few units of rounding;
  * ragged column counts (L not a multiple of the 64-column unit), batches
    of vectors, one factor per batch entry (node chains);
  * phi-actions (3D advection-diffusion) with both kinds forced, against the
    oracle's quadrature (Algorithm phiquadmv), and linear combinations
    (whose last squaring step reads an order offset and accumulates) against
    the definition.
"""
import numpy as np
import pytest

from oracle import phi_combo as C, phi_exact as X, phiquad as Q
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(x):
    torch.cuda.synchronize()
    return x.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


class forced:
    """Force the resident kernels' shape (kinds 5, 6 and 7) for a block of launches."""

    def __init__(self, h, store, square, accum=-1):
        self.h, self.cfg = h, {5: store, 6: square, 7: accum}

    def __enter__(self):
        for k, c in self.cfg.items():
            self.h.tile_config(k, c)

    def __exit__(self, *exc):
        for k in self.cfg:
            self.h.tile_config(k, -1)


SIZES = [(128, 128, 128), (64, 64, 64), (256, 64, 30), (128, 37, 6), (64, 256), (256, 256, 4), (6, 128, 64)]


@pytest.mark.parametrize("sizes", SIZES)
@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5, 6])
def test_f64r_kron_apply_vs_oracle_and_tiles(h, sizes, cfg):
    rng = np.random.default_rng(sum(sizes) + cfg)
    F = [rng.standard_normal((n, n)) / np.sqrt(n) for n in sizes]
    N = int(np.prod(sizes))
    x = rng.standard_normal((3, N))
    print("f64r kron_apply", sizes, "cfg", cfg, flush=True)
    Fd, xd = [dev(f) for f in F], dev(x)
    with forced(h, cfg, 0):
        y = host(h.kron_apply(Fd, xd))
    with forced(h, 0, 0):
        yt = host(h.kron_apply(Fd, xd))
    errs = [rel(y[r], X.apply_kron(F, x[r], list(sizes))) for r in range(3)]
    et = rel(y, yt)
    print(errs, et, flush=True)
    assert max(errs) < 1e-13, errs
    assert et < 1e-13, et


@pytest.fixture(scope="module")
def adv128():
    pr = I.problem("advdiff3d", seed=0, n=128)
    ref = Q.phiquadmv(pr["mats"], pr["t"], pr["v"], 3, eps=1e-14, beta=1.0)
    return pr, ref


@pytest.mark.parametrize("store,square,accum", [(1, 1, 1), (2, 1, 0), (2, 2, 1), (3, 3, 1), (4, 3, 1), (5, 4, 0), (6, 0, 0), (1, 0, 0),
                                                (0, 2, 0), (0, 0, 1), (-1, -1, -1)])
def test_f64r_phi_action_n128_vs_oracle(h, adv128, store, square, accum):
    """3D n = 128 phi_0..phi_3 (seed 0, tol 1e-8) with the resident kernels
    forced on the plain, squaring and/or node-sum products (0: the tile
    kernels; -1: the default choice)."""
    pr, ref = adv128
    with forced(h, store, square, accum):
        out, rep = h.action(pr["mats"], pr["t"], 3, dev(pr["v"]), tol=1e-8)
        o = host(out)
    errs = [rel(o[k], ref[k]) for k in range(4)]
    print("f64r phi-action", store, square, rep["l"], rep["m"], errs, flush=True)
    assert max(errs) < 1e-8, errs


@pytest.mark.parametrize("cfg,grp", [(1, 0), (2, 0), (3, 0), (1, 1), (3, 1)])
@pytest.mark.parametrize("sizes,p", [([64, 8], 3), ([128, 6], 1), ([64, 4, 5], 2), ([128, 9], 4)])
def test_f64r_combination_vs_definition(h, sizes, p, cfg, grp):
    """sum_j phi_j(-tA) b_j with the kinds forced: the last squaring step
    forms y_p alone (order offset p - 1) and adds it to phi_0 b_0; with
    rhs_per_launch = 1 every b_j has its own node sum (scaled weights, added
    into the running y), on the resident node-sum kernel."""
    rng = np.random.default_rng(p)
    mats = []
    for n in sizes:
        a, b = rng.uniform(0.5, 2.0), rng.uniform(0.0, 20.0)
        mats.append(I.adv_diff_1d(n, a, b))
    N = int(np.prod(sizes))
    bs = [rng.standard_normal(N) for _ in range(p + 1)]
    t = 0.01
    print("f64r combination", sizes, p, cfg, grp, flush=True)
    with forced(h, cfg, cfg, 1):
        plan = h.plan(mats, t, p, tol=1e-12, rhs_per_launch=grp)
        got = host(plan.execute_combo([dev(b) for b in bs]))
        rep = plan.report
        plan.close()
    ref = C.combo_exact(mats, t, bs)
    e = rel(got, ref)
    print(rep["l"], rep["m"], e, flush=True)
    assert rep["l"] > 0
    assert e < 1e-10, e
