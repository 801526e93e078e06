"""Learned warm start for the batched dual ascent (GPU pipeline).

The ascent of Section 3.3 starts from lambda = mu = 0.  Here a network
(dcopf_mlp.h) maps an instance's load vector to initial multipliers:

1. scenarios: per-bus load multipliers exp(N(0, sigma^2)) on one network
   (``synth.make_scenarios``);
2. targets: the multipliers the method itself reaches from a cold start
   (batched GPU solves, ``dcopf_batch``);
3. training: standardised inputs and targets, mean squared error, Adam, on
   the GPU with the library's own forward/backward kernels;
4. use: predicted multipliers, mu projected onto mu >= 0, set as the start of
   a batched solve.  Fallback (``run_with_fallback``): a cold start runs
   beside it, and after ``fallback_at`` iterations each instance keeps, on
   the device, whichever trajectory has the larger exact bound.  Every bound
   reported is an exact dual value.

Every numerical step runs in the HIP library; this module moves arrays.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import _abi, synth


@dataclasses.dataclass
class Standardizer:
    """Per-column mean and spread of a device matrix (torch tensors on the
    GPU), computed and applied by the library (dcopf_mlp_column_stats /
    dcopf_mlp_standardize)."""
    mean: "object"
    std: "object"

    @staticmethod
    def fit(model: "_abi.MLP", A) -> "Standardizer":
        import torch
        rows, cols = A.shape
        mean = torch.empty(cols, dtype=torch.float32, device=A.device)
        std = torch.empty(cols, dtype=torch.float32, device=A.device)
        model.column_stats(A.data_ptr(), rows, cols, mean.data_ptr(), std.data_ptr())
        return Standardizer(mean, std)

    def apply(self, model: "_abi.MLP", A, inverse=False):
        import torch
        out = torch.empty_like(A)
        model.standardize(A.data_ptr(), A.shape[0], A.shape[1], self.mean.data_ptr(),
                          self.std.data_ptr(), out.data_ptr(), inverse)
        return out


def fold_standardizers(model: "_abi.MLP", sx: Standardizer, st: Standardizer):
    """The model's parameters become those of the same network acting on raw
    loads and returning raw multipliers (dcopf_mlp_fold_standardizers)."""
    model.fold_standardizers(sx.mean.data_ptr(), sx.std.data_ptr(), st.mean.data_ptr(),
                             st.std.data_ptr())


def he_init(rng, dims):
    """Initial parameters of the network with layer widths ``dims``: weights
    [fan_out, fan_in] drawn N(0, 2 / fan_in) (He initialisation), layer by
    layer from ``rng``, biases zero.  FP64; the caller casts."""
    out = []
    for fan_in, fan_out in zip(dims[:-1], dims[1:]):
        out.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(fan_out, fan_in)))
        out.append(np.zeros(fan_out))
    return out


def cold_solve(base, D, iters, alpha, rho, stream=None, chunk=8192, trend_window=1000):
    """Multipliers after ``iters`` cold-start GDM iterations for every load
    scenario D [B, n_bus] (batched GPU solves, chunks of ``chunk``).
    Returns (targets [B, 2 n_line + 1] = [mu+, mu-, lambda], exact bounds at
    ``iters``, exact bounds ``trend_window`` iterations earlier)."""
    out, bounds, earlier = [], [], []
    C = np.tile(base.c, (D.shape[0], 1))
    w = min(trend_window, iters)
    for s in range(0, D.shape[0], chunk):
        Dc = D[s:s + chunk]
        net = _abi.BatchNetwork(base, Dc, C[s:s + chunk], None, alpha=alpha, rho=rho)
        with _abi.BatchSolver([net], stream=stream, graph_iters=50, gamma_cap=1) as b:
            b.step(iters - w)
            earlier.append(b.bound())
            b.step(w)
            bounds.append(b.bound())
            lam, mp, mm = b.get_multipliers(0)
        out.append(np.concatenate([mp, mm, lam[:, None]], axis=1))
    return np.concatenate(out), np.concatenate(bounds), np.concatenate(earlier)


def settled(bound, earlier, cost_ub, rel=1e-3):
    """Scenarios whose cold-start ascent has settled: finite targets, a bound
    below the largest possible cost, and a bound that rose by at most ``rel``
    (relative) over the trend window.  An infeasible scenario has an
    unbounded dual, so its bound keeps rising; it fails this test."""
    ok = np.isfinite(bound) & np.isfinite(earlier) & (bound <= cost_ub)
    with np.errstate(invalid="ignore", divide="ignore"):
        rise = (bound - earlier) / np.abs(bound)
    return ok & (rise <= rel)


def train(model: "_abi.MLP", X, T, epochs, batch, lr, seed=0, lr_decay=0.9, log=None):
    """Mini-batch training on device tensors X [N, n_in], T [N, n_out] (FP32,
    already standardised).  Returns the per-epoch mean batch loss."""
    import torch
    N = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(X.device)
        tot, nb = 0.0, 0
        for s in range(0, N - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            want = (s // batch) % 20 == 0
            l = model.train_step(xb.data_ptr(), tb.data_ptr(), batch, lr, want_loss=want)
            if want:
                tot += l
                nb += 1
        losses.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e} lr {lr:.2e}")
        lr *= lr_decay
    return losses


def predict(model: "_abi.MLP", X, sx: Standardizer, st: Standardizer, batch=256):
    """Warm-start rows [N, 2 n_line + 1] = [mu+, mu-, lambda] on the device
    for raw load vectors X [N, n_bus] (host), from a model trained on
    standardised data: inputs standardised and outputs mapped back by the
    library (mu is projected onto mu >= 0 where the rows become a start)."""
    import torch
    N = X.shape[0]
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Xn = sx.apply(model, Xd)
    Y = torch.empty((N, model.dims[-1]), dtype=torch.float32, device="cuda")
    for s in range(0, N, batch):
        n = min(batch, N - s)
        model.forward(Xn[s:s + n].data_ptr(), n, Y[s:s + n].data_ptr())
    return st.apply(model, Y, inverse=True)


def predict_dev(model: "_abi.MLP", X, batch=256):
    """Raw warm-start rows [N, 2 n_line + 1] = [mu+, mu-, lambda] on the
    device (a torch tensor) for raw load vectors X [N, n_bus] (host), from a
    model whose parameters carry the folded standardisations."""
    import torch
    N = X.shape[0]
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Y = torch.empty((N, model.dims[-1]), dtype=torch.float32, device="cuda")
    for s in range(0, N, batch):
        n = min(batch, N - s)
        model.forward(Xd[s:s + n].data_ptr(), n, Y[s:s + n].data_ptr())
    torch.cuda.synchronize()
    return Y


def run_to_gap(base, D, opt, alpha, rho, start=None, max_iters=5000, check_every=10,
               probe_at=100, stream=None, stats=None):
    """Batched solve of the scenarios D (cold; from start = (lam, mu+, mu-)
    on the host; or from a device tensor start of rows [mu+, mu-, lambda]).
    Returns (iteration of the first exact bound within 0.1 % of opt per
    instance, -1 if none; exact bound at iteration probe_at).  If ``stats``
    is a dict it receives the iterations run, their wall time (the start
    hand-off included) and the wall time at each checked iteration."""
    C = np.tile(base.c, (D.shape[0], 1))
    net = _abi.BatchNetwork(base, D, C, None, alpha=alpha, rho=rho)
    with _abi.BatchSolver([net], stream=stream, graph_iters=10, gamma_cap=1) as b:
        t0 = time.perf_counter()
        if isinstance(start, tuple):
            b.set_multipliers(0, *start)
        elif start is not None:
            b.set_start_dev(0, start.data_ptr(), start.shape[1])
        hit = np.full(D.shape[0], -1, np.int64)
        probe = None
        it = 0
        vals = b.bound()
        hit[(opt - vals) <= 1e-3 * np.abs(opt)] = 0
        seconds_at = {0: time.perf_counter() - t0}
        while it < max_iters and np.any(hit < 0):
            b.step(check_every)
            it += check_every
            vals = b.bound()
            newly = (hit < 0) & ((opt - vals) <= 1e-3 * np.abs(opt))
            hit[newly] = it
            seconds_at[it] = time.perf_counter() - t0
            if it == probe_at:
                probe = vals.copy()
        if probe is None:
            probe = vals.copy()
        if stats is not None:
            stats["iterations"] = it
            stats["seconds"] = time.perf_counter() - t0
            stats["seconds_at"] = seconds_at
    return hit, probe


def run_with_fallback(base, D, opt, alpha, rho, start, fallback_at=100, max_iters=5000,
                      check_every=10, stream=None):
    """The warm start with its fallback, in one pipeline on the device: the
    scenarios D run from ``start`` (a device tensor of rows [mu+, mu-,
    lambda]) and, beside them, from the cold start of Algorithm 1 for
    ``fallback_at`` iterations; then, per instance, the trajectory with the
    larger exact bound is kept on the device (dcopf_batch_adopt_better) and
    the cold shadow is destroyed; the kept trajectories continue alone.

    Returns a dict: ``hit`` (iteration of the first exact bound within 0.1 %
    of opt per instance, -1 if none; before the fallback either trajectory
    counts), ``kept_cold`` (instances that continued from the cold start),
    ``bound_after`` (exact bound of the kept trajectory at ``fallback_at``),
    ``seconds_at`` (wall time from the hand-off of the start to each checked
    iteration, the shadow's iterations included), ``iterations`` and
    ``instance_iterations`` (the shadow's included)."""
    C = np.tile(base.c, (D.shape[0], 1))
    net_w = _abi.BatchNetwork(base, D, C, None, alpha=alpha, rho=rho)
    net_c = _abi.BatchNetwork(base, D, C, None, alpha=alpha, rho=rho)
    n = D.shape[0]
    hit = np.full(n, -1, np.int64)
    seconds_at = {}
    inst_iters = 0

    def record(it, vals):
        hit[(hit < 0) & ((opt - vals) <= 1e-3 * np.abs(opt))] = it

    with _abi.BatchSolver([net_w], stream=stream, graph_iters=10, gamma_cap=1) as w:
        cold = _abi.BatchSolver([net_c], stream=stream, graph_iters=10, gamma_cap=1)
        try:
            t0 = time.perf_counter()
            w.set_start_dev(0, start.data_ptr(), start.shape[1])
            it = 0
            for b in (w, cold):
                record(0, b.bound())
            seconds_at[0] = time.perf_counter() - t0
            while it < fallback_at:
                k = min(check_every, fallback_at - it)
                it += k
                for b in (w, cold):
                    b.step(k)
                    record(it, b.bound())
                inst_iters += 2 * n * k
                seconds_at[it] = time.perf_counter() - t0
            kept_cold = w.adopt_better(0, cold, 0).astype(bool)
        finally:
            cold.close()
        bound_after = w.bound()
        seconds_at[it] = time.perf_counter() - t0
        while it < max_iters and np.any(hit < 0):
            w.step(check_every)
            it += check_every
            inst_iters += n * check_every
            record(it, w.bound())
            seconds_at[it] = time.perf_counter() - t0
    return dict(hit=hit, kept_cold=kept_cold, bound_after=bound_after, seconds_at=seconds_at,
                iterations=it, instance_iterations=inst_iters)


def median_seconds(hit, seconds_at, cap_seconds):
    """Median over instances of the wall time at which each was certified
    (unreached instances count at ``cap_seconds``)."""
    t = np.array([seconds_at[h] if h >= 0 else cap_seconds for h in hit])
    return float(np.median(t))


def combine_with_fallback(hit_cold, probe_cold, hit_warm, probe_warm, probe_at):
    """Warm start with a cold shadow: both trajectories run until probe_at;
    an instance certified by either of them by then stops at the first
    certification; otherwise the trajectory with the larger exact bound at
    probe_at continues alone.  Returns (iterations to the gap, -1 if never;
    which instances kept the warm trajectory)."""
    use_warm = probe_warm >= probe_cold
    big = np.iinfo(np.int64).max
    ew = np.where((hit_warm >= 0) & (hit_warm <= probe_at), hit_warm, big)
    ec = np.where((hit_cold >= 0) & (hit_cold <= probe_at), hit_cold, big)
    early = np.minimum(ew, ec)
    later = np.where(use_warm, hit_warm, hit_cold)
    return np.where(early < big, early, later), use_warm


def median_iters(hit, cap):
    """Median with unreached instances counted at the cap."""
    return float(np.median(np.where(hit >= 0, hit, cap)))


def timed(fn, *a, **k):
    t = time.perf_counter()
    r = fn(*a, **k)
    return r, time.perf_counter() - t
