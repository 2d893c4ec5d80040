"""Learned choice of (l, m) for the Gauss-rule phi-action.

The paper picks the scaling exponent l and the node count m with
Algorithm setup_quadrature: the cheapest pair, under the cost model
C = c1 d n + c2 (n + l p), whose a priori bound (Thm 3.2) meets the
tolerance.  On the MI355X the two kinds of work do not cost the same: the m
node chains run as batched mode products, while each of the l squaring
steps runs p chains and a GEMM one after another.  This module

  1. measures that cost (`measure`, GPU): phi-action time over forced
     (l, m) for 3D grids n = 32..256 and p = 1..4, and fits, per n,
        T(l, m) = a m + (b p + c) l + d                       (milliseconds);
  2. labels generated problems (`dataset`, host): for every l, the smallest
     m that meets the bound (Algorithm quadnodes), and the (l, m) with the
     least fitted T;
  3. trains the 8 -> 64 -> 64 -> 2 network on those labels (`train`, GPU,
     through the library's own forward / backward / Adam kernels);
and the planner uses the network with the bound as the judge (Algorithm
setup_quadrature is the fallback): phiq_options.selector = PHIQ_SEL_MLP.

Two modes:
  * certified (`train`, PHIQ_SEL_MLP): the labels are pairs the a priori
    bound accepts, so the network can only reorder (l, m) by cost, never use
    fewer nodes or squarings than the bound asks for; the bound judges its
    choice;
  * empirical (`sweep-errors`, `train-empirical`, PHIQ_SEL_MLP_EMPIRICAL):
    `sweep_errors` runs the method itself over forced (l, m) on generated
    problems and measures each error against the method's own result at tol
    1e-14.  Per problem, `norm_ratio` finds the smallest rho for which the
    bound at the norm rho ||tA|| covers twice every measured error above
    1e-10 (for these advection-diffusion operators rho is 0.39..0.75: the
    infinity norm overstates the reach of the spectrum).  The network learns
    log10 rho and the scaling l with the least modelled time; the planner
    takes m from Algorithm quadnodes at rho ||tA|| / 2^l, so a wrong l costs
    time, not accuracy, and a margin (the largest shortfall of the predicted
    log10 rho on the training samples) is added to the output's bias.

Features (8): log10 of t ||A^d||_inf for axes 0..2 (-3 for an absent axis),
n / 256, dim, p, log10 t, log10 tol.  Outputs (2): l / 8 and m / 16
(certified) or l / 8 and log10 rho (empirical).
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

from . import inputs as I
from . import phiq

PKG = os.path.dirname(os.path.abspath(__file__))
COSTS = os.path.join(PKG, "selector_costs.json")
WEIGHTS = os.path.join(PKG, "selector_weights.json")
ERRORS = os.path.join(PKG, "selector_errors.json")
WEIGHTS_EMPIRICAL = os.path.join(PKG, "selector_weights_empirical.json")
NFEAT, NHID, NOUT = 8, 64, 2
NPARAM = NHID * NFEAT + NHID + NHID * NHID + NHID + NOUT * NHID + NOUT
L_SCALE, M_SCALE = 8.0, 16.0


def features(norms, n, dim, p, t, tol):
    """norms: t ||A^d||_inf per axis (already multiplied by t)."""
    f = [math.log10(max(float(x), 1e-300)) for x in list(norms)[:3]]
    f += [-3.0] * (3 - len(f))
    return np.array(f + [n / 256.0, float(dim), float(p), math.log10(t), math.log10(tol)], dtype=np.float64)


def infnorm(a):
    return float(np.max(np.sum(np.abs(a), axis=1)))


def feasible_m(tol, p, alpha, l):
    """Gauss nodes the bound needs at scaling l (Algorithm quadnodes, n + 1 nodes)."""
    return phiq.quadnodes(tol, p, math.ldexp(alpha, -l)) + 1


# ---------------------------------------------------------------------------
# 1. cost measurement on the GPU
# ---------------------------------------------------------------------------
def measure(sizes=(32, 48, 64, 96, 128, 160, 192, 256), ps=(1, 2, 3, 4), reps=5, seed=0, log=print):
    import torch

    h = phiq.Handle(0)
    rng = np.random.default_rng(seed)
    recs = []
    for n in sizes:
        for p in ps:
            for t in (1e-3, 1e-2):
                a, b = I.draw_coefficients(rng, 3)
                mats = [I.adv_diff_1d(n, float(a[d]), float(b[d])) for d in range(3)]
                alpha = t * sum(infnorm(m) for m in mats)
                v = torch.from_numpy(rng.standard_normal(n ** 3)).cuda()
                _, rep = h.action(mats, t, p, v, tol=1e-8)
                l0 = rep["l"]
                for l in range(max(0, l0 - 3), l0 + 3):
                    m = feasible_m(1e-8, p, alpha, l)
                    if m > 48:
                        continue
                    for extra in (0, 3):
                        kw = dict(l=l, m=m + extra)
                        # two warm-up calls: one-call plans alternate between two
                        # buffers, each may grow once for a new size
                        h.action(mats, t, p, v, tol=1e-8, **kw)
                        h.action(mats, t, p, v, tol=1e-8, **kw)
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        for _ in range(reps):
                            h.action(mats, t, p, v, tol=1e-8, **kw)
                        torch.cuda.synchronize()
                        ms = (time.perf_counter() - t0) * 1e3 / reps
                        recs.append(dict(n=n, p=p, l=l, m=m + extra, t=t, ms=ms))
                log("n=%d p=%d t=%g done (%d records)" % (n, p, t, len(recs)))
    h.close()
    return recs


def fit(recs):
    """Per n: least squares T = a m + b p l + c l + d, then once more without the
    points whose residual exceeds five times the median absolute residual
    (one-off stalls such as a buffer growing inside a timed call)."""
    out = {}
    for n in sorted(set(r["n"] for r in recs)):
        rs = [r for r in recs if r["n"] == n]
        A = np.array([[r["m"], r["p"] * r["l"], r["l"], 1.0] for r in rs])
        y = np.array([r["ms"] for r in rs])
        coef, *_ = np.linalg.lstsq(A, y, rcond=None)
        res = np.abs(A @ coef - y)
        keep = res <= 5.0 * max(np.median(res), 1e-6)
        coef, *_ = np.linalg.lstsq(A[keep], y[keep], rcond=None)
        resid = float(np.sqrt(np.mean((A[keep] @ coef - y[keep]) ** 2)))
        out[int(n)] = dict(a=float(coef[0]), b=float(coef[1]), c=float(coef[2]), d=float(coef[3]),
                           rms_ms=resid, points=int(keep.sum()), dropped=int((~keep).sum()))
    return out


def cost_fn(costs):
    ns = np.array(sorted(int(k) for k in costs))
    tab = {k: np.array([costs[str(n)][k] if str(n) in costs else costs[n][k] for n in ns]) for k in "abcd"}
    ln = np.log(ns)

    def interp(key, n):
        return float(np.interp(math.log(n), ln, tab[key]))

    def T(n, p, l, m):
        return interp("a", n) * m + (interp("b", n) * p + interp("c", n)) * l + interp("d", n)

    return T


# ---------------------------------------------------------------------------
# 2. labels
# ---------------------------------------------------------------------------
def label(T, n, p, alpha, tol):
    """(l, m) with the least modelled time among the pairs the bound accepts."""
    if alpha <= 1e-12:
        return 0, max(1, (p + 1) // 2)
    lmax = max(0, math.ceil(math.log2(alpha))) + 2
    best = None
    for l in range(0, lmax + 1):
        try:
            m = feasible_m(tol, p, alpha, l)
        except phiq.PhiqError:
            continue
        c = T(n, p, l, m)
        if best is None or c < best[0]:
            best = (c, l, m)
    return best[1], best[2]


def draw_problem(rng, n_range=(16, 256), dims=(2, 3)):
    dim = int(dims[rng.integers(0, len(dims))])
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    p = int(rng.integers(1, 5))
    t = float(math.exp(rng.uniform(math.log(1e-4), math.log(1e-1))))
    tol = float(math.exp(rng.uniform(math.log(1e-10), math.log(1e-6))))
    a, b = I.draw_coefficients(rng, dim)
    norms = [t * (4 * a[d] * (n + 1) ** 2 + 2 * b[d] * (n + 1)) for d in range(dim)]
    return dict(dim=dim, n=n, p=p, t=t, tol=tol, a=a.tolist(), b=b.tolist(), norms=norms)


def dataset(count, seed, costs):
    T = cost_fn(costs)
    rng = np.random.default_rng(seed)
    X = np.zeros((count, NFEAT))
    Y = np.zeros((count, NOUT))
    meta = []
    for i in range(count):
        pr = draw_problem(rng)
        alpha = sum(pr["norms"])
        l, m = label(T, pr["n"], pr["p"], alpha, pr["tol"])
        X[i] = features(pr["norms"], pr["n"], pr["dim"], pr["p"], pr["t"], pr["tol"])
        Y[i] = (l / L_SCALE, m / M_SCALE)
        meta.append(dict(pr, l=l, m=m))
    return X, Y, meta


# ---------------------------------------------------------------------------
# 3. the network (host copy of the forward pass, for checks)
# ---------------------------------------------------------------------------
def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    parts = []
    for shape in ((NHID, NFEAT), (NHID,), (NHID, NHID), (NHID,), (NOUT, NHID), (NOUT,)):
        k = int(np.prod(shape))
        parts.append(w[o:o + k].reshape(shape))
        o += k
    return parts


def init_weights(seed):
    """Glorot-uniform weights, zero biases (the random draw is made here and passed to the kernels)."""
    rng = np.random.default_rng(seed)
    out = []
    for fan_in, fan_out in ((NFEAT, NHID), (NHID, NHID), (NHID, NOUT)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        out.append(rng.uniform(-lim, lim, fan_out * fan_in))
        out.append(np.zeros(fan_out))
    return np.concatenate(out).astype(np.float32)


def load_costs(path=COSTS):
    d = json.load(open(path))
    return d["fit"]


def train(h, count=20000, seed=1, steps=3000, lr=3e-3, costs=None, log=print):
    """Generate `count` labelled problems and fit the network on the GPU."""
    costs = load_costs() if costs is None else costs
    X, Y, meta = dataset(count, seed, costs)
    w0 = init_weights(seed + 1000)
    w, hist = h.mlp_train(X, Y, w0, steps, lr)
    pred = predict(w, X)
    l_err = np.abs(np.rint(pred[:, 0] * L_SCALE) - np.rint(Y[:, 0] * L_SCALE))
    m_err = np.abs(np.rint(pred[:, 1] * M_SCALE) - np.rint(Y[:, 1] * M_SCALE))
    stats = dict(count=count, seed=seed, steps=steps, lr=lr, loss_first=float(hist[0]), loss_last=float(hist[-1]),
                 l_exact=float(np.mean(l_err == 0)), m_within_1=float(np.mean(m_err <= 1)))
    log(json.dumps(stats))
    return w, hist, stats


def predict(w, X):
    """Host FP64 forward pass (the same network), for statistics."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    h1 = np.tanh(np.asarray(X) @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3.T + b3


def save_weights(w, stats, path=WEIGHTS):
    json.dump({"weights": [float(x) for x in np.asarray(w, dtype=np.float32)], "stats": stats}, open(path, "w"))


def load_weights(path=WEIGHTS):
    return np.array(json.load(open(path))["weights"], dtype=np.float32)


def save_weights_bin(w, path):
    """The weight vector as raw little-endian float32, the file phiq_selector_load reads."""
    np.asarray(w, dtype="<f4").tofile(path)


# ---------------------------------------------------------------------------
# 4. empirical labels: the method's measured error over forced (l, m)
# ---------------------------------------------------------------------------
def draw_sweep_problem(rng, sizes=(32, 48, 64, 96, 128, 192, 256), dims=(3,)):
    dim = int(dims[rng.integers(0, len(dims))])
    n = int(sizes[rng.integers(0, len(sizes))])
    p = int(rng.integers(1, 5))
    t = float(math.exp(rng.uniform(math.log(1e-4), math.log(1e-1))))
    a, b = I.draw_coefficients(rng, dim)
    return dict(dim=dim, n=n, p=p, t=t, a=[float(x) for x in a], b=[float(x) for x in b])


def sweep_errors(h, count=240, seed=11, emin=1e-12, mmax=20, dims=(3,), log=print):
    """For `count` generated problems: the relative error (max over phi_k of the inf-norm error over
    the inf-norm of the reference) of the FP64 phi-action at forced (l, m), against the method's own
    result at tol 1e-14.  For each l from the paper's choice at tol 1e-10 down to six below it, m
    rises from 2 until the error is below emin (or m = mmax)."""
    import torch

    rng = np.random.default_rng(seed)
    recs = []
    for i in range(count):
        pr = draw_sweep_problem(rng, dims=dims)
        n, dim, p, t = pr["n"], pr["dim"], pr["p"], pr["t"]
        mats = [I.adv_diff_1d(n, pr["a"][d], pr["b"][d]) for d in range(dim)]
        v = torch.from_numpy(rng.standard_normal(n ** dim)).cuda()
        ref, rr = h.action(mats, t, p, v, tol=1e-14)
        den = ref.abs().amax(dim=1)
        _, r10 = h.action(mats, t, p, v, tol=1e-10)
        out = torch.empty((p + 1, v.numel()), dtype=torch.float64, device="cuda")
        pts = []
        for l in range(r10["l"], max(-1, r10["l"] - 7), -1):
            for m in range(2, mmax + 1):
                _, rep = h.action(mats, t, p, v, tol=1e-10, l=l, m=m, out=out)
                e = float(((out - ref).abs().amax(dim=1) / den).max())
                pts.append([l, m, e, rep["log10_bound"]])
                if e < emin:
                    break
        recs.append(dict(pr, alpha=rr["alpha"], norms=[t * infnorm(mm) for mm in mats], points=pts))
        log("problem %d: dim=%d n=%d p=%d alpha=%.3g, %d points" % (i, dim, n, p, rr["alpha"], len(pts)))
    return recs


EMPIRICAL_TOL_MIN = 1e-10  # the planner's empirical mode declines below this tolerance


def _covered(rec, lr, floor, safety):
    a = rec["alpha"] * 10.0 ** lr
    for l, m, e, _ in rec["points"]:
        if e <= safety * floor or m < 2:
            continue
        if phiq.log_quaderr(m - 1, rec["p"], math.ldexp(a, -l)) / math.log(10.0) < math.log10(e / safety):
            return False
    return True


def norm_ratio(rec, floor=EMPIRICAL_TOL_MIN, safety=0.5, iters=30):
    """log10 rho of a sweep record: the smallest rho in [0.1, 1] for which the a priori bound (Thm 3.2)
    at the norm rho ||tA|| covers twice (1 / safety) every measured error above safety * floor; then
    Algorithm quadnodes at rho ||tA|| picks, for any tol >= floor, only pairs whose measured error is
    at most safety * tol.  None if even rho = 1 does not cover them."""
    lo, hi = -1.0, 0.0
    if not _covered(rec, hi, floor, safety):
        return None
    if _covered(rec, lo, floor, safety):
        return lo
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if _covered(rec, mid, floor, safety):
            hi = mid
        else:
            lo = mid
    return hi


def swept_error(rec, l, m):
    """Measured error of the pair (l, m) in a sweep record: the pair itself, else the error at the
    largest swept m below m at that l (the error falls as m grows, and a sweep of one l stops once
    it is below the floor); None if that l was not swept or nothing at or below m was."""
    best = None
    for pl, pm, e, _ in rec["points"]:
        if pl == l and pm <= m and (best is None or pm > best[0]):
            best = (pm, e)
    return None if best is None else best[1]


def empirical_dataset(recs, costs, tols_per_problem=8, seed=5):
    """Samples (features, (l / 8, log10 rho)): rho the record's norm ratio, l the scaling with the least
    modelled time when m is Algorithm quadnodes at rho ||tA|| (tols log-uniform in [1e-10, 1e-6])."""
    T = cost_fn(costs)
    rng = np.random.default_rng(seed)
    X, Y, meta = [], [], []
    for rec in recs:
        lr = norm_ratio(rec)
        if lr is None:
            continue
        for _ in range(tols_per_problem):
            tol = float(math.exp(rng.uniform(math.log(EMPIRICAL_TOL_MIN), math.log(1e-6))))
            l, m = label(T, rec["n"], rec["p"], rec["alpha"] * 10.0 ** lr, tol)
            X.append(features(rec["norms"], rec["n"], rec["dim"], rec["p"], rec["t"], tol))
            Y.append((l / L_SCALE, lr))
            meta.append(dict(n=rec["n"], dim=rec["dim"], p=rec["p"], alpha=rec["alpha"], tol=tol, l=l, m=m, log10_rho=lr))
    return np.array(X), np.array(Y), meta


def train_empirical(h, recs, seed=3, steps=6000, lr=3e-3, costs=None, log=print):
    """Fit the network on the empirical samples (GPU), then add to the bias of the log10 rho output
    the largest amount by which it fell short of a training target (rounded up to 0.005 decades), so
    that on every training sample the planner uses a norm at least the one that covered the errors."""
    costs = load_costs() if costs is None else costs
    X, Y, meta = empirical_dataset(recs, costs)
    w0 = init_weights(seed + 1000)
    w, hist = h.mlp_train(X, Y, w0, steps, lr)
    pred = predict(w, X)
    short = float(np.max(Y[:, 1] - pred[:, 1]))
    margin = math.ceil(max(0.0, short) / 0.005) * 0.005
    w = np.asarray(w, dtype=np.float32).copy()
    w[-1] += np.float32(margin)
    l_err = np.abs(np.rint(pred[:, 0] * L_SCALE) - np.rint(Y[:, 0] * L_SCALE))
    stats = dict(mode="empirical", samples=len(meta), problems=len(recs),
                 problems_used=len({(m["n"], m["p"], m["alpha"]) for m in meta}), steps=steps, lr=lr,
                 loss_first=float(hist[0]), loss_last=float(hist[-1]), l_exact=float(np.mean(l_err == 0)),
                 rho_rms=float(np.sqrt(np.mean((pred[:, 1] - Y[:, 1]) ** 2))), margin=margin,
                 log10_rho_range=[float(Y[:, 1].min()), float(Y[:, 1].max())])
    log(json.dumps(stats))
    return w, hist, stats


def empirical_pair(w, rec, tol):
    """Host copy of the planner's empirical mode (phiq_options.selector = PHIQ_SEL_MLP_EMPIRICAL):
    (l, m, used), used 4 = the network's pair, 3 = rejected, 0 = tol below the mode's range (both
    then Algorithm setup_quadrature's pair)."""
    p, alpha = rec["p"], rec["alpha"]
    l5, n5, _ = phiq.setup_quadrature(tol, p, alpha)
    if tol < EMPIRICAL_TOL_MIN:
        return l5, n5 + 1, 0
    y = predict(w, features(rec["norms"], rec["n"], rec["dim"], p, rec["t"], tol)[None])[0]
    lp = min(60, max(0, int(math.floor(y[0] * L_SCALE + 0.5))))
    ratio = 10.0 ** min(0.0, max(-1.0, float(y[1])))
    nq = phiq.quadnodes(tol, p, math.ldexp(alpha * ratio, -lp))
    if nq + 1 + lp * p > 1.5 * ((n5 + 1) + l5 * p):
        return l5, n5 + 1, 3
    return lp, nq + 1, 4


def holdout(recs, w, costs, tols=(1e-10, 1e-9, 1e-8, 1e-7, 1e-6)):
    """For held-out sweep records: the empirical pair at each tol, its measured error (looked up in
    the record) and Algorithm setup_quadrature's, and the modelled time ratio of the two."""
    T = cost_fn(costs)
    rows = []
    for rec in recs:
        for tol in tols:
            l, m, used = empirical_pair(w, rec, tol)
            l5, n5, _ = phiq.setup_quadrature(tol, rec["p"], rec["alpha"])
            rows.append(dict(dim=rec["dim"], n=rec["n"], p=rec["p"], alpha=rec["alpha"], tol=tol, l=l, m=m,
                             used=used, err=swept_error(rec, l, m), l5=l5, m5=n5 + 1,
                             err5=swept_error(rec, l5, n5 + 1),
                             speedup=T(rec["n"], rec["p"], l5, n5 + 1) / T(rec["n"], rec["p"], l, m)))
    known = [r for r in rows if r["err"] is not None]
    summ = dict(cases=len(rows), known=len(known), met=sum(r["err"] <= r["tol"] for r in known),
                worst_over_tol=max([r["err"] / r["tol"] for r in known] or [0.0]),
                median_modelled_speedup=float(np.median([r["speedup"] for r in rows])))
    return rows, summ


def load_empirical(path=WEIGHTS_EMPIRICAL):
    """Weights of the empirical-mode network (its margin already in the last bias)."""
    return np.array(json.load(open(path))["weights"], dtype=np.float32)


def _device_handle():
    """torch's device first (its lazy initialisation fails once another library has set HIP up in
    the process), then the library's handle."""
    import torch

    torch.zeros(1, device="cuda")
    return phiq.Handle(0)


def main(argv):
    if len(argv) >= 1 and argv[0] == "train":
        out = argv[1] if len(argv) > 1 else WEIGHTS
        costs = load_costs(argv[2]) if len(argv) > 2 else None
        h = phiq.Handle(0)
        w, hist, stats = train(h, costs=costs, log=lambda s: print(s, flush=True))
        h.close()
        save_weights(w, stats, out)
        return 0
    if len(argv) >= 1 and argv[0] == "sweep-errors":
        out = argv[1] if len(argv) > 1 else ERRORS
        count = int(argv[2]) if len(argv) > 2 else 240
        seed = int(argv[3]) if len(argv) > 3 else 11
        dims = tuple(int(x) for x in argv[4].split(",")) if len(argv) > 4 else (3,)
        h = _device_handle()
        recs = sweep_errors(h, count=count, seed=seed, dims=dims, log=lambda s: print(s, flush=True))
        h.close()
        json.dump({"records": recs}, open(out, "w"))
        return 0
    if len(argv) >= 1 and argv[0] == "train-empirical":
        srcs = (argv[1] if len(argv) > 1 else ERRORS).split(",")
        out = argv[2] if len(argv) > 2 else WEIGHTS_EMPIRICAL
        recs = [r for src in srcs for r in json.load(open(src))["records"]]
        costs = load_costs(argv[3]) if len(argv) > 3 else None
        h = _device_handle()
        w, hist, stats = train_empirical(h, recs, costs=costs, log=lambda s: print(s, flush=True))
        h.close()
        save_weights(w, stats, out)
        return 0
    if len(argv) >= 1 and argv[0] == "refit":
        d = json.load(open(COSTS))
        d["fit"] = fit(d["records"])
        json.dump(d, open(COSTS, "w"), indent=1)
        print(json.dumps(d["fit"], indent=1))
        return 0
    if len(argv) >= 1 and argv[0] == "measure":
        out = argv[1] if len(argv) > 1 else COSTS
        recs = measure(log=lambda s: print(s, flush=True))
        costs = fit(recs)
        json.dump({"records": recs, "fit": costs}, open(out, "w"), indent=1)
        print(json.dumps(costs, indent=1))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
