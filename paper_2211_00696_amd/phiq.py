"""Thin Python binding of libphiq.so: argument marshalling only.

Device buffers are torch CUDA tensors (float64, contiguous); the 1D
matrices A^d are host numpy arrays.  Every step of the phi-action runs in
the library's HIP kernels; nothing here computes.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_size_t, c_void_p

import numpy as np

from . import _lib as L


class PhiqError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.name = L.STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.name}")


def _check(st: int, where: str):
    if st != 0:
        raise PhiqError(st, where)


def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _dev_ptr(x, name):
    import torch

    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    return c_void_p(x.data_ptr())


def _f32_ptr(x, name):
    import torch

    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 tensor")
    return c_void_p(x.data_ptr())


class _Op:
    """Keeps the host copies of A^d alive while the KronOp points at them."""

    def __init__(self, mats):
        if len(mats) < 1 or len(mats) > L.MAX_DIM:
            raise ValueError("between 1 and %d matrices" % L.MAX_DIM)
        self.mats = [np.ascontiguousarray(np.asarray(m, dtype=np.float64)) for m in mats]
        self.op = L.KronOp()
        self.op.dim = len(self.mats)
        for d, m in enumerate(self.mats):
            if m.ndim != 2 or m.shape[0] != m.shape[1]:
                raise ValueError("A^d must be square")
            self.op.n[d] = m.shape[0]
            self.op.A[d] = m.ctypes.data_as(POINTER(c_double))
        self.sizes = [m.shape[0] for m in self.mats]
        self.N = int(np.prod(self.sizes))


def options(rule="gauss", precision="fp64", l=None, m=None, alpha=None, c1=None, c2=None,
            cc_max_doublings=None, workspace_cap=None, use_graphs=None, selector=None, slab_products=None,
            accept_floor=None, selector_slack=None, batch_persistent=None, rhs_per_launch=None, cc_scaling=None):
    lib = L.load()
    o = L.Options()
    _check(lib.phiq_options_default(byref(o)), "phiq_options_default")
    o.rule = L.RULE[rule]
    o.precision = L.PRECISION[precision]
    if l is not None:
        o.l = int(l)
    if m is not None:
        o.m = int(m)
    if alpha is not None:
        o.alpha = float(alpha)
    if c1 is not None:
        o.c1 = float(c1)
    if c2 is not None:
        o.c2 = float(c2)
    if cc_max_doublings is not None:
        o.cc_max_doublings = int(cc_max_doublings)
    if workspace_cap is not None:
        o.workspace_cap = int(workspace_cap)
    if use_graphs is not None:
        o.use_graphs = int(bool(use_graphs))
    if selector is not None:
        o.selector = L.SELECTOR[selector]
    if slab_products is not None:
        o.slab_products = int(slab_products)
    if accept_floor is not None:
        o.accept_floor = int(bool(accept_floor))
    if cc_scaling is not None:
        o.cc_scaling = L.CC_SCALING[cc_scaling]
    if selector_slack is not None:
        o.selector_slack = float(selector_slack)
    if batch_persistent is not None:
        o.batch_persistent = int(bool(batch_persistent))
    if rhs_per_launch is not None:
        o.rhs_per_launch = int(rhs_per_launch)
    return o


# ---------------------------------------------------------------------------
# host-only planning
# ---------------------------------------------------------------------------
def norm_bound(mats, t):
    lib = L.load()
    op = _Op(mats)
    a = c_double()
    _check(lib.phiq_norm_bound(byref(op.op), float(t), byref(a)), "phiq_norm_bound")
    return a.value


def setup_quadrature(eps, p, alpha, beta=1.0, rule="gauss", c1=0.0, c2=1.0, d=3):
    """(l, n, cost) of the parameter selection; the rule has n+1 nodes."""
    lib = L.load()
    l, n, c = c_int(), c_int(), c_double()
    _check(lib.phiq_setup_quadrature(float(eps), int(p), float(alpha), float(beta), L.RULE[rule], float(c1),
                                     float(c2), int(d), byref(l), byref(n), byref(c)), "phiq_setup_quadrature")
    return l.value, n.value, c.value


def cc_scaling(eps, p, alpha, c1=0.0, c2=1.0, d=3, max_doublings=6):
    """Scaling l of adaptive Clenshaw-Curtis by the predicted cost of the nodes Algorithm 2 runs
    (phiq_cc_scaling; the plans' default)."""
    lib = L.load()
    l = c_int()
    _check(lib.phiq_cc_scaling(float(eps), int(p), float(alpha), float(c1), float(c2), int(d), int(max_doublings),
                               byref(l)), "phiq_cc_scaling")
    return l.value


def log_quaderr(n, p, alpha, beta=1.0, rule="gauss"):
    lib = L.load()
    e = c_double()
    _check(lib.phiq_log_quaderr(float(n), int(p), float(alpha), float(beta), L.RULE[rule], byref(e)),
           "phiq_log_quaderr")
    return e.value


def quadnodes(eps, p, alpha, beta=1.0, rule="gauss"):
    """Algorithm quadnodes: smallest n (n+1 nodes) meeting eps at norm alpha."""
    lib = L.load()
    n = c_int()
    _check(lib.phiq_quadnodes(float(eps), int(p), float(alpha), float(beta), L.RULE[rule], byref(n)), "phiq_quadnodes")
    return n.value


def quadrature_rule(rule, m):
    lib = L.load()
    th = np.zeros(m)
    w = np.zeros(m)
    _check(lib.phiq_quadrature_rule(L.RULE[rule], int(m), th.ctypes.data_as(POINTER(c_double)),
                                    w.ctypes.data_as(POINTER(c_double))), "phiq_quadrature_rule")
    return th, w


def status_string(st):
    return L.load().phiq_status_string(int(st)).decode()


# ---------------------------------------------------------------------------
# device
# ---------------------------------------------------------------------------
def batch_info(problems, **opts):
    """Host-only dry run of Handle.action_batched (no GPU): the schedule's size
    and a check of its addresses and ordering.  problems: dicts with mats, t,
    p, tol and the integer addresses v_ptr / out_ptr and nrhs (default 1)."""
    lib = L.load()
    arr = (L.Problem * max(1, len(problems)))()
    keep = []
    for i, pr in enumerate(problems):
        op = _Op(pr["mats"])
        keep.append(op)
        arr[i].op = op.op
        arr[i].t = float(pr["t"])
        arr[i].p = int(pr["p"])
        arr[i].tol = float(pr.get("tol", 1e-8))
        arr[i].nrhs = int(pr.get("nrhs", 1))
        arr[i].v = int(pr["v_ptr"])
        arr[i].out = int(pr["out_ptr"])
    st = L.BatchStats()
    _check(lib.phiq_batch_info(len(problems), arr, byref(options(**opts)), byref(st)), "phiq_batch_info")
    return st.as_dict()


class Plan:
    def __init__(self, handle, ptr, p, N, report):
        self._h = handle
        self._ptr = ptr
        self.p = p
        self.N = N
        self.report = report

    def execute(self, v, out=None, stream=None):
        import torch

        lib = L.load()
        nrhs = v.numel() // self.N
        if v.numel() != nrhs * self.N or nrhs < 1:
            raise ValueError("v must hold nrhs x N values")
        if out is None:
            out = torch.empty((nrhs, self.p + 1, self.N), dtype=torch.float64, device=v.device)
        rep = L.Report()
        _check(lib.phiq_plan_execute(self._ptr, _dev_ptr(v, "v"), nrhs, _dev_ptr(out, "out"), byref(rep),
                                     _stream_ptr(stream)), "phiq_plan_execute")
        return out, rep.as_dict()

    def execute_noalloc(self, v, out, stream=None):
        """One vector through phiq_plan_execute_noalloc: the plan's intermediates in the library's
        fixed device array (nothing allocated).  out (p+1, N) float64 CUDA tensor, caller-owned.
        Returns the bytes of the array the plan needs."""
        lib = L.load()
        if v.numel() != self.N or out.numel() != (self.p + 1) * self.N:
            raise ValueError("v must hold N values and out (p+1) x N")
        need = c_size_t()
        _check(lib.phiq_plan_execute_noalloc(self._ptr, _dev_ptr(v, "v"), _dev_ptr(out, "out"), byref(need),
                                             _stream_ptr(stream)), "phiq_plan_execute_noalloc")
        return need.value

    def execute_combo(self, bs, out=None, stream=None):
        """out = sum_j phi_j(-tA) bs[j], j = 0..p; bs holds p+1 entries, each a
        float64 CUDA tensor of N values or None (a zero vector)."""
        import torch

        lib = L.load()
        if len(bs) != self.p + 1:
            raise ValueError("bs must hold p+1 entries")
        arr = (c_void_p * (self.p + 1))()
        dev = None
        for j, b in enumerate(bs):
            if b is None:
                arr[j] = None
                continue
            if b.numel() != self.N:
                raise ValueError("every b_j must hold N values")
            arr[j] = _dev_ptr(b, "b[%d]" % j).value
            dev = b.device
        if out is None:
            if dev is None:
                raise ValueError("at least one b_j is needed")
            out = torch.empty(self.N, dtype=torch.float64, device=dev)
        _check(lib.phiq_plan_execute_combo(self._ptr, arr, _dev_ptr(out, "out"), _stream_ptr(stream)),
               "phiq_plan_execute_combo")
        return out

    def close(self):
        if self._ptr:
            L.load().phiq_plan_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Handle:
    """A library handle on one HIP device (owns the reusable workspace)."""

    def __init__(self, device=0):
        lib = L.load()
        h = c_void_p()
        _check(lib.phiq_create(byref(h), int(device)), "phiq_create")
        self._h = h
        self.device = device

    def close(self):
        if self._h:
            L.load().phiq_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_start(self, classes=None):
        """Bracket later kernel launches of the given classes (all if None) with HIP events."""
        mask = 0
        for c in classes or []:
            mask |= 1 << L.PROFILE_CLASSES.index(c)
        _check(L.load().phiq_profile_start(self._h, mask), "phiq_profile_start")

    def profile_enable(self, on=True):
        """Pause (False) or resume (True) the bracketing, keeping what was recorded."""
        _check(L.load().phiq_profile_enable(self._h, int(bool(on))), "phiq_profile_enable")

    def profile_stop(self):
        """Synchronise and return {kernel class: dict(launches, ms, flops, bytes)}."""
        arr = (L.KernelStat * 16)()
        n = c_int()
        _check(L.load().phiq_profile_stop(self._h, arr, 16, byref(n)), "phiq_profile_stop")
        return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops,
                                           bytes=arr[i].bytes) for i in range(n.value)}

    def autotune(self, sizes, p, m, stream=None):
        """Time the FP64 mode-product tile shapes for these sizes; returns ms [shape][tile]."""
        times = np.full(64 * 16, -1.0)
        n = (c_int * len(sizes))(*sizes)
        _check(L.load().phiq_autotune(self._h, len(sizes), n, int(p), int(m),
                                      times.ctypes.data_as(POINTER(c_double)), _stream_ptr(stream)),
               "phiq_autotune")
        t = times.reshape(64, 16)
        rows = [r for r in range(64) if (t[r] >= 0).any()]
        return t[rows]

    def action(self, mats, t, p, v, tol=1e-8, out=None, stream=None, **opts):
        """out[k] = phi_k(-t A) v, k = 0..p; returns (out (p+1, N), report dict)."""
        import torch

        lib = L.load()
        op = _Op(mats)
        if v.numel() != op.N:
            raise ValueError("v has %d entries, the operator needs %d" % (v.numel(), op.N))
        if out is None:
            out = torch.empty((p + 1, op.N), dtype=torch.float64, device=v.device)
        o = options(**opts)
        rep = L.Report()
        _check(lib.phiq_action(self._h, byref(op.op), float(t), int(p), _dev_ptr(v, "v"), float(tol), byref(o),
                               _dev_ptr(out, "out"), byref(rep), _stream_ptr(stream)), "phiq_action")
        return out, rep.as_dict()

    def action_batched(self, problems, stream=None, **opts):
        """Many phi-actions launched together (phiq_action_batched).

        problems: list of dicts with keys mats, t, p, v (device tensor with N
        or nrhs x N entries), tol (default 1e-8) and optionally out
        (nrhs x (p+1) x N).  Returns (outs, reports), outs[i] shaped
        (nrhs, p+1, N).  Asynchronous on the stream (synchronise before
        reading the outputs on the host)."""
        import torch

        lib = L.load()
        nprob = len(problems)
        arr = (L.Problem * max(1, nprob))()
        keep, outs, reps = [], [], []
        for i, pr in enumerate(problems):
            op = _Op(pr["mats"])
            v = pr["v"]
            if v.numel() % op.N:
                raise ValueError("problem %d: v has %d entries, not a multiple of N = %d" % (i, v.numel(), op.N))
            nrhs = v.numel() // op.N
            p = int(pr["p"])
            out = pr.get("out")
            if out is None:
                out = torch.empty((nrhs, p + 1, op.N), dtype=torch.float64, device=v.device)
            if out.numel() != nrhs * (p + 1) * op.N:
                raise ValueError("problem %d: out must hold nrhs x (p+1) x N values" % i)
            rep = L.Report()
            arr[i].op = op.op
            arr[i].t = float(pr["t"])
            arr[i].p = p
            arr[i].tol = float(pr.get("tol", 1e-8))
            arr[i].nrhs = nrhs
            arr[i].v = _dev_ptr(v, "v").value
            arr[i].out = _dev_ptr(out, "out").value
            arr[i].rep = ctypes.pointer(rep)
            keep.append(op)
            outs.append(out.view(nrhs, p + 1, op.N))
            reps.append(rep)
        o = options(**opts)
        _check(lib.phiq_action_batched(self._h, nprob, arr, byref(o), _stream_ptr(stream)), "phiq_action_batched")
        return outs, [r.as_dict() for r in reps]

    def etdrk4(self, mats, tau, nsteps, u, c1=1.0, c3=-1.0, tol=1e-8, graph=True, form="combo", stream=None):
        """ETD-RK4 steps of u' = -A u + c1 u + c3 u^3 in place on the device tensor u (phiq_etdrk4).
        form: "combo" (one linear combination per stage) or "separate".  Returns the report dict."""
        lib = L.load()
        if form not in ("separate", "combo"):
            raise ValueError("form must be 'separate' or 'combo'")
        op = _Op(mats)
        if u.numel() != op.N:
            raise ValueError("u has %d entries, the operator needs %d" % (u.numel(), op.N))
        rep = L.EtdReport()
        _check(lib.phiq_etdrk4(self._h, byref(op.op), float(tau), int(nsteps), float(c1), float(c3), float(tol),
                               int(bool(graph)), 1 if form == "combo" else 0, _dev_ptr(u, "u"), byref(rep),
                               _stream_ptr(stream)), "phiq_etdrk4")
        return rep.as_dict()

    def exprk(self, mats, method, nsteps, u, T=1.0, c2=None, tol=1e-8, form="auto", stream=None, **opts):
        """Section 5's exponential Euler (1), RK2 (2) or RK3 (3) on Problem 3, in place on u; report dict.

        form: "separate" (phi_0..p of every stage vector), "combo" (one linear
        combination per stage) or "auto" (combo for every precision but the int8 digits, which have
        no combination form)."""
        lib = L.load()
        if form == "auto":
            form = "separate" if opts.get("precision", "fp64") == "int8" else "combo"
        if form not in ("separate", "combo"):
            raise ValueError("form must be 'separate', 'combo' or 'auto'")
        op = _Op(mats)
        if u.numel() != op.N:
            raise ValueError("u has %d entries, the operator needs %d" % (u.numel(), op.N))
        if c2 is None:
            c2 = 0.5 if method == 2 else 1.0 / 3.0
        rep = L.Report()
        _check(lib.phiq_exprk(self._h, byref(op.op), int(method), float(c2), int(nsteps), float(T), float(tol),
                              byref(options(**opts)), 1 if form == "combo" else 0, _dev_ptr(u, "u"), byref(rep),
                              _stream_ptr(stream)), "phiq_exprk")
        return rep.as_dict()

    # ---- the learned selector's network (FP32) ----
    def mlp_forward(self, X, w, stream=None):
        """Y = net(X) on the device: X (B, 8) float32, w (NPARAM,) float32 device tensors."""
        import torch

        lib = L.load()
        B = X.shape[0]
        Y = torch.empty((B, 2), dtype=torch.float32, device=X.device)
        _check(lib.phiq_mlp_forward(self._h, int(B), _f32_ptr(X, "X"), _f32_ptr(w, "w"), _f32_ptr(Y, "Y"),
                                    _stream_ptr(stream)), "phiq_mlp_forward")
        return Y

    def mlp_grad(self, X, T, w, stream=None):
        """(gradient (NPARAM,) float32 device tensor, loss) of the mean squared error."""
        import torch

        lib = L.load()
        g = torch.empty_like(w)
        loss = c_double()
        _check(lib.phiq_mlp_grad(self._h, int(X.shape[0]), _f32_ptr(X, "X"), _f32_ptr(T, "T"), _f32_ptr(w, "w"),
                                 _f32_ptr(g, "grad"), byref(loss), _stream_ptr(stream)), "phiq_mlp_grad")
        return g, loss.value

    def mlp_train(self, X, T, w, steps, lr=1e-3):
        """Full-batch Adam on the GPU from host arrays; returns (weights, loss history)."""
        lib = L.load()
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        w = np.array(w, dtype=np.float32, copy=True)
        hist = np.zeros(max(1, steps), dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(lib.phiq_mlp_train(self._h, int(X.shape[0]), X.ctypes.data_as(fp), T.ctypes.data_as(fp),
                                  w.ctypes.data_as(fp), int(steps), float(lr), hist.ctypes.data_as(fp)),
               "phiq_mlp_train")
        return w, hist[:steps]

    def tile_config(self, kind, cfg=-1):
        """Force tile shape cfg for every launch of a kind: FP64 0 (store), 1 (node sum), 2 (squaring);
        split bf16 and FP32 3 (store) and 4 (squaring), where 0 is the general tile kernel and 1.. keep
        the 1D factor resident in LDS (FP32: n_d in {128, 256}, store 1..3, squaring 1..2); FP64 with the factor resident in LDS 5 (store), 6 (squaring),
        7 (node sum), where 0 declines to the tile kernels.  -1 restores the tuned/default choice.
        Returns the number of shapes of the kind."""
        lib = L.load()
        n = c_int()
        _check(lib.phiq_tile_config(self._h, int(kind), int(cfg), byref(n)), "phiq_tile_config")
        return n.value

    def selector_set(self, w):
        """Install the selector network (host float32 array) or clear it (None)."""
        lib = L.load()
        if w is None:
            _check(lib.phiq_selector_set(self._h, None), "phiq_selector_set")
            return
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib.phiq_selector_set(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "phiq_selector_set")

    def selector_load(self, path):
        """Install the selector network from a file of PHIQ_MLP_NPARAM float32 values
        (phiq_selector_load; `selector.save_weights_bin` writes one)."""
        _check(L.load().phiq_selector_load(self._h, os.fsencode(path)), "phiq_selector_load")

    def plan(self, mats, t, p, tol=1e-8, stream=None, **opts):
        lib = L.load()
        op = _Op(mats)
        o = options(**opts)
        ptr = c_void_p()
        rep = L.Report()
        _check(lib.phiq_plan_create(self._h, byref(op.op), float(t), int(p), float(tol), byref(o), byref(ptr),
                                    byref(rep), _stream_ptr(stream)), "phiq_plan_create")
        return Plan(self, ptr, p, op.N, rep.as_dict())

    def kron_apply(self, factors, x, out=None, precision="fp64", stream=None):
        """y = (F^0 (x) F^1 (x) ...) x for x of shape (nvec, N) (device tensors)."""
        import torch

        lib = L.load()
        dim = len(factors)
        n = (c_int * dim)(*[f.shape[0] for f in factors])
        F = (c_void_p * dim)(*[_dev_ptr(f, "F").value for f in factors])
        N = int(np.prod([f.shape[0] for f in factors]))
        nvec = x.numel() // N
        if out is None:
            out = torch.empty_like(x)
        _check(lib.phiq_kron_apply(self._h, dim, n, F, _dev_ptr(x, "x"), _dev_ptr(out, "out"), nvec,
                                   L.PRECISION[precision], _stream_ptr(stream)), "phiq_kron_apply")
        return out

    def expm(self, X, xnorm, out=None, stream=None):
        """E[b] = exp(X[b]) for X of shape (nmat, n, n) on the device; xnorm: host bounds."""
        import torch

        lib = L.load()
        nmat, n, _ = X.shape
        xn = np.ascontiguousarray(np.asarray(xnorm, dtype=np.float64).reshape(nmat))
        if out is None:
            out = torch.empty_like(X)
        _check(lib.phiq_expm(self._h, int(n), int(nmat), _dev_ptr(X, "X"), xn.ctypes.data_as(POINTER(c_double)),
                             _dev_ptr(out, "E"), _stream_ptr(stream)), "phiq_expm")
        return out
