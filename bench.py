"""Benchmark of the projected dual ascent (instance-iterations/s and time to a
bound within 0.1 % of the FP64 optimum) on one MI355X.

Default workload: the mixed batch, 512 load/cost scenarios of a 4600-bus
network, 128 of a 2000-bus network and 32 of a 10,000-bus network with
quadratic costs, advanced together (split-BF16 MFMA products, FP32 line
state, FP64 lambda and exact bound).  A step is one ascent iteration of
every instance (reduced costs, inner minimiser, residuals, step +
projection).  Inputs are resident in HBM before the timed region; the
iteration loop is replayed as captured HIP graphs.  Other workloads
(--workload): a single instance (bus2000, bus4600, bus10000), the learned
warm start, the PTDF build, step rules, the iterated-s QP dual, and the
device-copy calibration of the traffic counters.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "instance-iterations/s of dual ascent; time to bound within 0.1% of FP64 optimum"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.md")
SINGLE_SRC = ("paper_2406_13191_amd/csrc/common.h", "paper_2406_13191_amd/csrc/single.hip")
BATCH_SRC = ("paper_2406_13191_amd/csrc/common.h", "paper_2406_13191_amd/csrc/batch.hip")


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key, files):
    """HBM bytes per launch of kernel `key` from the rocprofv3 counter runs
    recorded in profiles/hbm_traffic.md: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), each scaled by what the counter reads for a plain 1 GiB copy.
    None when not recorded or when the kernel's sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            m = re.search(r"```json\n(.*?)\n```", f.read(), re.S)
        table = json.loads(m.group(1))
        e = table["kernels"][key]
        cal = table["copy_calibration"]
    except (OSError, AttributeError, KeyError, ValueError):
        return None
    if e.get("source_sha256") != source_sha(files):
        return None
    return int(round(e["fetch_kib"] * 1024 * cal["fetch_scale"]
                     + e["write_kib"] * 1024 * cal["write_scale"]))


def copy_calibration():
    """A plain 1 GiB device copy, three times: the kernel whose counter
    readings calibrate FETCH_SIZE and WRITE_SIZE."""
    import torch
    a = torch.empty(2 ** 28, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": 2 ** 30,
                      "bytes_written": 2 ** 30, "repeats": 3}), flush=True)


def panel_bytes(n_line, n_cols, n_gen, scheme="two_pass"):
    """Algorithmic HBM bytes of one launch of each pass (FP32 panel, every
    vector read or written once).  Two-pass: both passes read the panel.
    Read-once: only the line pass reads it; the per-workgroup partials of
    P^T v it writes and the unit pass reads are workspace, reported apart
    (partial_bytes)."""
    panel = 4.0 * n_line * n_cols
    units = n_gen * (4 * 8 + 4) + 4 * (n_cols + 1)
    if scheme == "read_once":
        # unit pass: unit data and boundaries read, x written
        col = units + 4 * n_cols
        # line pass: x, f_d, f_max, mu+-, velocity+- read; mu+-, velocity+- written
        line = panel + 4 * n_cols + n_line * (6 * 8 + 4 * 8)
        return col, line
    col = panel + 4 * n_line + 4 * n_cols + units
    # line pass: x, f_d, f_max, mu+-, velocity+- read; mu+-, velocity+-, v written
    line = panel + 4 * n_cols + n_line * (6 * 8 + 4 * 8 + 4)
    return col, line


def cpu_baseline(p, alpha, rho, budget_s=15.0):
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import dual as D
    K = D.canonical(p)
    t = time.perf_counter()
    D.ascent(K, 20, alpha=alpha, rho=rho)
    per = (time.perf_counter() - t) / 20
    n = int(max(50, min(20000, budget_s / per)))
    t = time.perf_counter()
    D.ascent(K, n, alpha=alpha, rho=rho)
    dt = time.perf_counter() - t
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    # the same oracle with one BLAS thread, a shorter sample
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        n1 = max(20, n // 10)
        t = time.perf_counter()
        D.ascent(K, n1, alpha=alpha, rho=rho)
        dt1 = time.perf_counter() - t
    return dict(value=n / dt, unit="instance-iterations/s", cores=int(threads),
                kind="oracle",
                sample=f"{n} FP64 GDM iterations of the same {p.n_bus}-bus instance "
                       f"(numpy, {threads} BLAS threads), {dt:.1f} s",
                value_one_thread=n1 / dt1, sample_one_thread=f"{n1} iterations, {dt1:.1f} s")


MIXED = [("bus4600", 4600, 512, 46_000_000), ("bus2000", 2000, 128, 20_000_000),
         ("bus10000", 10000, 32, 100_000_000)]
BF16_PEAK_TFLOPS = 2500.0
TTB_CHECK = 100


def _make_net(spec):
    from paper_2406_13191_amd import synth
    name, seed = spec
    t = time.perf_counter()
    net, prob = synth.make_network(name, seed)
    return net, prob, time.perf_counter() - t


def _pool(n):
    import multiprocessing as mp
    return mp.get_context("spawn").Pool(n)


def _finish(pool):
    """Let the workers exit by themselves (no SIGTERM from terminate())."""
    pool.close()
    pool.join()


def prep_mixed(log):
    """Host-side inputs of the mixed batch, before any GPU call: the three
    networks (generated in parallel), every instance's load and cost
    scenario, and the HiGHS optimum of every LP instance (reference leg of
    the time to bound).  The QP network's instances get their target from a
    certified upper bound later."""
    import numpy as np

    from paper_2406_13191_amd import synth
    t0 = time.perf_counter()
    with _pool(len(MIXED)) as pool:
        made = pool.map(_make_net, [(n, s) for n, s, _, _ in MIXED])
        _finish(pool)
    for (name, *_), (_, _, dt) in zip(MIXED, made):
        log(f"network {name}: {dt:.1f} s")
    nets = []
    jobs, owner = [], []
    for k, ((name, seed, B, seed0), (topo, base, _)) in enumerate(zip(MIXED, made)):
        Dm, Cc, Q = synth.make_scenarios(base, seed0, B, 0.1, 0.1)
        nets.append(dict(name=name, topo=topo, base=base, D=Dm, C=Cc, Q=Q, B=B,
                         n_cols=int(len(np.unique(base.gen_bus)))))
        if not base.is_qp:
            light = base.replace(H=None)
            for i in range(B):
                jobs.append((topo, light.replace(d=Dm[i], c=Cc[i])))
                owner.append((k, i))
    log(f"HiGHS optima for {len(jobs)} LP instances")
    opts = _cached_optima("mixed", jobs)
    for n in nets:
        n["opt"] = np.full(n["B"], np.nan)
    for (k, i), o in zip(owner, opts):
        nets[k]["opt"][i] = o
    log(f"host inputs ready in {time.perf_counter() - t0:.1f} s")
    return nets


def _batch_networks(nets):
    from paper_2406_13191_amd import _abi, synth
    out = []
    for n in nets:
        r = synth.STEP_RULES[n["name"]]
        out.append(_abi.BatchNetwork(n["base"], n["D"], n["C"],
                                     n["Q"] if n["base"].is_qp else None,
                                     alpha=r["alpha"], rho=r["rho"]))
    return out


def _solver(stream, bnets, tiles):
    from paper_2406_13191_amd import _abi
    b = _abi.BatchSolver(bnets, stream=stream.cuda_stream, autotune=False, graph_iters=20,
                         gamma_cap=64)
    for k, t in enumerate(tiles):
        b.set_tiles(k, t["w_tile"], t["w_split"], t["f_tile"])
    return b


def bench_mixed(args, stream, nets, log):
    """The mixed batch: 512 scenarios of the 4600-bus network, 128 of the
    2000-bus and 32 of the 10000-bus (QP) network in one batched launch per
    phase, split-BF16 products, autotuned tiles, HIP-graph replay."""
    import numpy as np
    import torch

    from paper_2406_13191_amd import _abi, synth
    bnets = _batch_networks(nets)
    shapes = [(n["name"], n["base"].n_line, n["n_cols"], n["base"].n_gen, n["B"]) for n in nets]
    pinned = json.loads(args.tiles) if args.tiles else None
    t0 = time.perf_counter()
    b = _abi.BatchSolver(bnets, stream=stream.cuda_stream, autotune=pinned is None,
                         graph_iters=20, gamma_cap=64)
    t_create = time.perf_counter() - t0
    if pinned:
        for k, t in enumerate(pinned):
            b.set_tiles(k, t["w_tile"], t["w_split"], t["f_tile"])
    n_total = b.n_total
    b.step(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    log(f"{args.steps} iterations of {n_total} instances in {ms:.3f} ms")
    # per-phase durations: median of three samples of 20 iterations each,
    # events attached to each dispatch on the batch's stream
    ms_w, ms_u, ms_f = (float(v) for v in
                        np.median(np.array([b.time_phases(20) for _ in range(3)]), axis=0))
    tiles = [b.info(k) for k in range(len(bnets))]
    b.close()
    bw, bu, bf = batch_phase_bytes(shapes, [t["w_split"] for t in tiles])
    # the same instances one at a time on the single-instance path (FP32
    # products): seconds for one iteration of all of them, against the batch
    single = {}
    for n in nets:
        r = synth.STEP_RULES[n["name"]]
        with _abi.DualSolver(n["base"], stream=stream.cuda_stream, rule="gdm",
                             alpha=r["alpha"], rho=r["rho"], precision="fp32",
                             graph_iters=100) as s1:
            s1.step(200)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1.step(2000)
            torch.cuda.synchronize()
            single[n["name"]] = 2000 / (time.perf_counter() - t0)
    t_single = sum(n["B"] / single[n["name"]] for n in nets)
    t_batch = ms / args.steps / 1e3
    phases = {"w": ("W product (W^T = V^T P, split-BF16 MFMA; lambda step of the previous "
                    "iteration)", ms_w, bw),
              "units": ("unit pass (reduced costs, inner minimiser)", ms_u, bu),
              "f": ("F product (F^T = X^T P^T, split-BF16 MFMA, mu step)", ms_f, bf)}
    key = max(phases, key=lambda k: phases[k][1])
    kname, kms, kbytes = phases[key]
    achieved = kbytes / (kms * 1e-3) / 1e9
    useful = sum(2.0 * nl * nc * B for _, nl, nc, ng, B in shapes)  # one product
    issued = 3 * useful  # three split-BF16 terms
    mfma_issued = 2 * issued / ((ms_w + ms_f) * 1e-3) / 1e12
    mfma_useful = 2 * useful / ((ms_w + ms_f) * 1e-3) / 1e12
    iter_bytes = bw + bu + bf
    cert = batch_certified(stream, bnets, nets, tiles, log)
    ttb = batch_time_to_bound(args, stream, bnets, nets, tiles, cert["upper_bounds"], log)
    return dict(
        value=n_total * args.steps / (ms / 1e3), ms=ms, n_total=n_total, time_to_bound=ttb,
        certified={k: v for k, v in cert.items() if k != "upper_bounds"},
        create_seconds=round(t_create, 3),
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                      unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                      traffic=measured_traffic("mixed:" + key, BATCH_SRC), kernel=kname,
                      kernel_ms=round(kms, 5), bytes_per_launch=int(kbytes),
                      phase_ms={k: round(v[1], 5) for k, v in phases.items()},
                      phase_bytes={k: int(v[2]) for k, v in phases.items()},
                      phase_gbs={k: round(v[2] / (v[1] * 1e-3) / 1e9, 1)
                                 for k, v in phases.items()},
                      phase_traffic={k: measured_traffic("mixed:" + k, BATCH_SRC)
                                     for k in phases},
                      iteration=dict(bytes=int(iter_bytes), us=round(t_batch * 1e6, 2),
                                     gbs=round(iter_bytes / t_batch / 1e9, 1),
                                     frac=round(iter_bytes / t_batch / 1e9 / HBM_PEAK_GBS, 4)),
                      mfma=dict(issued_flops_per_product=issued, useful_flops_per_product=useful,
                                issued_tflops=round(mfma_issued, 2),
                                useful_tflops=round(mfma_useful, 2),
                                peak_tflops=BF16_PEAK_TFLOPS,
                                issued_frac=round(mfma_issued / BF16_PEAK_TFLOPS, 4),
                                useful_frac=round(mfma_useful / BF16_PEAK_TFLOPS, 4))),
        shapes=shapes, tiles=tiles,
        single_path=dict(rates={k: round(v, 1) for k, v in single.items()},
                         unit="instance-iterations/s",
                         seconds_per_batch_iteration=t_single,
                         batched_seconds_per_iteration=t_batch,
                         speedup=round(t_single / t_batch, 1)))


def batch_certified(stream, bnets, nets, tiles, log, n_iters=10000):
    """Certified gaps of every instance with no external solver: n_iters
    iterations with each instance's exact bound checked every 100 and its
    inner minimisers averaged over the second half, then every network's
    averages repaired into feasible dispatches (a scenario with no feasible
    dispatch stays unrepaired); gap = (repaired cost - best bound) / cost.
    The repaired costs are upper bounds on each instance's optimum."""
    import numpy as np
    import torch

    b = _solver(stream, bnets, tiles)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(0, n_iters, 100):
        if it == n_iters // 2:
            b.average(True)
        b.step(100)
        b.bound()
    best, _ = b.best()
    t_iter = time.perf_counter() - t0
    t0 = time.perf_counter()
    reps = [b.repair(k, max_rounds=64) for k in range(len(bnets))]
    t_rep = time.perf_counter() - t0
    b.close()
    offs = np.cumsum([0] + [n["B"] for n in nets])
    per, ub = {}, []
    for k, n in enumerate(nets):
        r = reps[k]
        ok = r["feasible"]
        ub.append(np.where(ok, r["cost"], np.nan))
        gap = (r["cost"] - best[offs[k]:offs[k + 1]]) / np.abs(r["cost"])
        g = gap[ok]
        per[n["name"]] = dict(instances=int(n["B"]), repaired=int(ok.sum()),
                              median_gap=float(np.median(g)) if g.size else None,
                              max_gap=float(g.max()) if g.size else None,
                              within_1e_3=int((g <= 1e-3).sum()),
                              within_1e_4=int((g <= 1e-4).sum()),
                              max_rounds=int(r["rounds"][ok].max()) if g.size else None,
                              max_lines_held=int(r["n_active"][ok].max()) if g.size else None)
        log(f"certified {n['name']}: {int(ok.sum())}/{n['B']} repaired, median gap "
            f"{per[n['name']]['median_gap']:.2e}")
    return dict(iterations=n_iters, average_from=n_iters // 2, check_every=100,
                seconds_iterations=round(t_iter, 3), seconds_repair=round(t_rep, 3),
                per_network=per, upper_bounds=ub)


def batch_time_to_bound(args, stream, bnets, nets, tiles, ub, log):
    """Iterations and wall time until every instance's exact bound is within
    0.1 % of its target, checked every TTB_CHECK iterations, with an
    iteration cap of its own (--ttb-cap).  Targets: the HiGHS optimum of an
    LP instance (the FP64 optimum); for a QP instance (no QP solver here)
    the certified upper bound of its repaired average, which is at least the
    optimum, so reaching it certifies a 0.1 % gap.  Instances with neither
    (no feasible dispatch) have no target."""
    import numpy as np
    import torch

    offs = np.cumsum([0] + [n["B"] for n in nets])
    target = np.full(int(offs[-1]), np.nan)
    kind = []
    for k, n in enumerate(nets):
        target[offs[k]:offs[k + 1]] = ub[k] if n["base"].is_qp else n["opt"]
        kind.append("certified upper bound" if n["base"].is_qp else "HiGHS optimum")
    has = np.isfinite(target)
    b = _solver(stream, bnets, tiles)
    hit = np.full(target.size, -1, np.int64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, t_all = 0, None
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    dev_ms = 0.0
    while it < args.ttb_cap:
        e0.record(stream)
        b.step(TTB_CHECK)
        e1.record(stream)
        it += TTB_CHECK
        vals = b.bound()
        dev_ms += e0.elapsed_time(e1)
        newly = has & (hit < 0) & (target - vals <= 1e-3 * np.abs(target))
        hit[newly] = it
        if np.all(hit[has] >= 0):
            t_all = time.perf_counter() - t0
            break
    b.close()
    per = {}
    for k, n in enumerate(nets):
        h = hit[offs[k]:offs[k + 1]][has[offs[k]:offs[k + 1]]]
        if h.size:
            per[n["name"]] = dict(target=kind[k], instances=int(h.size),
                                  median_iterations=float(np.median(
                                      np.where(h >= 0, h, args.ttb_cap))),
                                  max_iterations=int(h.max()) if np.all(h >= 0) else None,
                                  reached=float((h >= 0).mean()))
    log(f"time to bound: {'all reached at %d iterations' % it if t_all else 'not all reached'}")
    return dict(reached=t_all is not None, instances_with_target=int(has.sum()),
                instances=int(target.size), check_every=TTB_CHECK, iteration_cap=args.ttb_cap,
                iterations=it if t_all is not None else None,
                seconds=None if t_all is None else round(t_all, 4),
                device_seconds_iterations=round(dev_ms / 1e3, 4), per_network=per,
                note="wall time of the whole batch (every instance advancing together) "
                     "including the exact-bound checks and their read-back")


def cpu_baseline_batch(nets, budget_s=15.0):
    """The FP64 oracle run as batched GEMMs over the same instances (every
    instance of every network, oracle.batch.ascent_batch), timed on a
    bounded number of iterations that fills about budget_s seconds; then the
    same with one BLAS thread on a shorter sample."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import batch as OB
    from paper_2406_13191_amd import synth
    KBs = []
    for n in nets:
        r = synth.STEP_RULES[n["name"]]
        KBs.append((OB.canonical_batch(n["base"], n["D"], n["C"],
                                       n["Q"] if n["base"].is_qp else None),
                    r["alpha"], r["rho"]))
    n_inst = sum(n["B"] for n in nets)

    def run(iters):
        t = time.perf_counter()
        for KB, a, rho in KBs:
            OB.ascent_batch(KB, iters, alpha=a, rho=rho)
        return time.perf_counter() - t

    per = run(2) / 2
    n = int(max(3, min(2000, budget_s / per)))
    dt = run(n)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        n1 = max(2, n // 8)
        dt1 = run(n1)
    return dict(value=n_inst * n / dt, unit="instance-iterations/s", cores=int(threads),
                kind="oracle",
                sample=f"{n} FP64 GDM iterations of all {n_inst} instances of the mixed batch "
                       f"(oracle.batch: numpy FP64 GEMMs over each network's instances, "
                       f"{threads} BLAS threads), {dt:.1f} s",
                seconds_per_iteration=dt / n,
                value_one_thread=n_inst * n1 / dt1,
                sample_one_thread=f"{n1} iterations, {dt1:.1f} s")


def batch_phase_bytes(shapes, splits):
    """Algorithmic HBM bytes of one launch of each batched phase, summed over
    the networks (GDM state; split-BF16 operands are 4 bytes per element)."""
    w = u = f = 0
    for (_, nl, nc, ng, B), S in zip(shapes, splits):
        ntl = (nl + 31) // 32
        # W: P^T hi/lo, V hi/lo read; FP32 split-K partials written; the
        # fold of the previous iteration reads its line terms
        w += 4 * nl * nc + 4 * B * nl + 4 * S * B * nc + 8 * B * ntl
        # units: partials, costs, generator bounds and columns read; X hi/lo
        # written
        u += 4 * S * B * nc + 16 * B * ng + 20 * ng + 4 * B * nc
        # F: P hi/lo, X hi/lo, f_max read; f_d, mu+-, velocity+- read,
        # mu+-, velocity+-, V hi/lo written (40 bytes per line and instance)
        f += 4 * nl * nc + 4 * B * nc + 4 * nl + 40 * B * nl + 8 * B * ntl
    return w, u, f


def _lp_optimum(net, prob):
    """Reference optimum of an LP instance (the time-to-bound target): HiGHS
    on the DCOPF in bus-angle form.  Variables: generator outputs p within
    their bounds, bus angles theta (slack angle fixed at 0).  Each bus
    balances generation minus load against the flows leaving it, and each
    line's flow b_l (theta_from - theta_to) stays within +-f_max.  Returns
    NaN when HiGHS finds no optimum."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.optimize import linprog
    nb, ng, nl = net.n_bus, prob.n_gen, net.n_line
    lines = np.arange(nl)
    # flow of line l as a function of theta: b_l theta_from - b_l theta_to
    flow = sp.coo_matrix((np.r_[net.b, -net.b], (np.r_[lines, lines], np.r_[net.fbus, net.tbus])),
                         shape=(nl, nb)).tocsr()
    # net outflow at bus k: flows of lines leaving k minus flows of lines entering k
    out_of = sp.coo_matrix((np.r_[np.ones(nl), -np.ones(nl)],
                            (np.r_[net.fbus, net.tbus], np.r_[lines, lines])),
                           shape=(nb, nl)).tocsr()
    gen_at = sp.coo_matrix((np.ones(ng), (prob.gen_bus, np.arange(ng))), shape=(nb, ng)).tocsr()
    A_eq = sp.hstack([gen_at, -(out_of @ flow)]).tocsr()      # C_g p - outflow(theta) = d
    A_ub = sp.vstack([sp.hstack([sp.csr_matrix((nl, ng)), flow]),
                      sp.hstack([sp.csr_matrix((nl, ng)), -flow])]).tocsr()
    b_ub = np.r_[prob.f_max, prob.f_max]
    bounds = [(lo, hi) for lo, hi in zip(prob.p_min, prob.p_max)] + [(None, None)] * nb
    bounds[ng + net.slack] = (0.0, 0.0)
    res = linprog(np.r_[prob.c, np.zeros(nb)], A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=prob.d,
                  bounds=bounds, method="highs")
    return float(res.fun) if res.status == 0 else float("nan")


def _highs_opt(args):
    net, prob = args
    return _lp_optimum(net, prob)


def _cached_optima(tag, jobs):
    """HiGHS optima of the jobs (a pool of 16 processes).  When
    DCOPF_SYNTH_CACHE names a cache directory (as for the synthetic
    networks), they are kept there, keyed by the instances' data and by the
    sources of the generator and of this reference, so that later runs (a
    profiled one, say) reuse them instead of starting the pool."""
    import numpy as np
    root = os.environ.get("DCOPF_SYNTH_CACHE")
    path = None
    if root:
        h = hashlib.sha256()
        for f in ("paper_2406_13191_amd/synth.py", "bench.py"):
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        for net, prob in jobs:
            for a in (net.fbus, net.tbus, net.b, prob.gen_bus, prob.c, prob.q, prob.p_min,
                      prob.p_max, prob.d, prob.f_max):
                h.update(b"-" if a is None else np.ascontiguousarray(a, np.float64).tobytes())
        path = os.path.join(root, f"highs_{tag}_{h.hexdigest()[:16]}.npy")
        if os.path.exists(path):
            return list(np.load(path, allow_pickle=False))
    with _pool(16) as pool:
        opts = pool.map(_highs_opt, jobs, chunksize=8)
        _finish(pool)
    if path:
        os.makedirs(root, exist_ok=True)
        np.save(path, np.asarray(opts, dtype=np.float64), allow_pickle=False)
    return opts


SCREENING = [("bus2000", 2000), ("bus2000_raw", 2000), ("bus4600", 4600), ("bus4600_raw", 4600)]


def prep_screening(log, n_inst=32):
    """Host-side inputs of the screening comparison: the 2000- and 4600-bus
    networks with their default limits and with the unscreened recipe (any
    heavily loaded line may be tightened, no limit price capped), n_inst
    load and cost scenarios of each, and every instance's HiGHS optimum."""
    from paper_2406_13191_amd import synth
    with _pool(len(SCREENING)) as pool:
        made = pool.map(_make_net, SCREENING)
        _finish(pool)
    nets, jobs, owner = [], [], []
    for k, ((name, _), (topo, base, dt)) in enumerate(zip(SCREENING, made)):
        log(f"network {name}: {dt:.1f} s")
        Dm, Cc, Q = synth.make_scenarios(base, 7_000_000, n_inst, 0.1, 0.1)
        nets.append(dict(name=name, topo=topo, base=base, D=Dm, C=Cc, B=n_inst))
        light = base.replace(H=None)
        for i in range(n_inst):
            jobs.append((topo, light.replace(d=Dm[i], c=Cc[i])))
            owner.append((k, i))
    log(f"HiGHS optima for {len(jobs)} LP instances")
    opts = _cached_optima("screening", jobs)
    import numpy as np
    for n in nets:
        n["opt"] = np.full(n["B"], np.nan)
    for (k, i), o in zip(owner, opts):
        nets[k]["opt"][i] = o
    return nets


def bench_screening(args, stream, nets, log):
    """Iterations to an exact bound within 0.1 % of the HiGHS optimum, per
    instance, for each network of prep_screening run alone as a batch (GDM
    with the network's frozen rule, bound checked every TTB_CHECK
    iterations, capped at --ttb-cap)."""
    import numpy as np

    from paper_2406_13191_amd import _abi, synth
    out = {}
    for n in nets:
        r = synth.STEP_RULES[n["name"]]
        net = _abi.BatchNetwork(n["base"], n["D"], n["C"], None, alpha=r["alpha"], rho=r["rho"])
        has = np.isfinite(n["opt"])
        hit = np.full(n["B"], -1)
        with _abi.BatchSolver([net], stream=stream.cuda_stream, graph_iters=20,
                              gamma_cap=64) as b:
            it = 0
            while it < args.ttb_cap and np.any(hit[has] < 0):
                b.step(TTB_CHECK)
                it += TTB_CHECK
                v = b.bound()
                hit[has & (hit < 0) & (n["opt"] - v <= 1e-3 * np.abs(n["opt"]))] = it
        h = hit[has]
        out[n["name"]] = dict(instances=int(has.sum()),
                              median_iterations=float(np.median(np.where(h >= 0, h, args.ttb_cap))),
                              max_iterations=int(h.max()) if np.all(h >= 0) else None,
                              reached=round(float((h >= 0).mean()), 3))
        log(f"{n['name']}: median {out[n['name']]['median_iterations']:.0f} iterations")
    return out


def prep_warmstart(args, log):
    """Host-side inputs of the warm-start workload, before any GPU call: the
    2000-bus network, training and held-out load scenarios, and the HiGHS
    optimum of every held-out scenario (reference leg)."""
    import numpy as np

    from paper_2406_13191_amd import synth
    net, base = synth.make_network("bus2000", 2000)
    Dtr, _, _ = synth.make_scenarios(base, 5_000_000, args.train, 0.15, 0.0)
    Dev, _, _ = synth.make_scenarios(base, 6_000_000, args.eval, 0.15, 0.0)
    light = base.replace(H=None)
    opt = []
    with _pool(16) as pool:
        for o in pool.imap(_highs_opt, [(net, light.replace(d=Dev[i]))
                                        for i in range(Dev.shape[0])], chunksize=16):
            opt.append(o)
            if len(opt) % 512 == 0:
                log(f"HiGHS optima: {len(opt)} of {Dev.shape[0]}")
        _finish(pool)
    return net, base, Dtr, Dev, np.array(opt)


def bench_warmstart(args, stream, prep):
    """Learned warm start on the 2000-bus network: training scenarios with
    per-bus load multipliers exp(N(0, 0.15^2)), targets from cold batched
    solves, training with the library's kernels, evaluation on held-out
    scenarios against HiGHS optima (reference leg) with the cold fallback."""
    import numpy as np
    import torch

    from paper_2406_13191_amd import _abi, synth
    from paper_2406_13191_amd import warmstart as W
    log = lambda m: print("[warm]", m, file=sys.stderr, flush=True)  # noqa: E731
    net, base, Dtr, Dev, opt = prep
    r = synth.STEP_RULES["bus2000"]
    log(f"targets: {args.train} cold solves of {args.target_iters} iterations")
    (T, tb, te), t_data = W.timed(W.cold_solve, base, Dtr, args.target_iters, r["alpha"],
                                  r["rho"], stream.cuda_stream)
    cost_ub = float(np.sum(np.maximum(base.c * base.p_min, base.c * base.p_max)))
    ok = W.settled(tb, te, cost_ub) & np.all(np.isfinite(T), axis=1)
    if not ok.any():
        sys.exit("no training scenario passed the settled test: --target-iters must exceed "
                 "the 1000-iteration trend window by enough for the bounds to settle")
    log(f"targets: {ok.sum()} of {ok.size} scenarios kept, {t_data:.1f} s")
    Dtr, T = Dtr[ok], T[ok]
    dims = (base.n_bus, 1024, 1024, 2 * base.n_line + 1)
    model = _abi.MLP(*dims, max_batch=256, stream=stream.cuda_stream)
    # standardised inputs and targets, by the library on the device
    Xraw = torch.tensor(Dtr, dtype=torch.float32, device="cuda")
    Traw = torch.tensor(T, dtype=torch.float32, device="cuda")
    sx, st = W.Standardizer.fit(model, Xraw), W.Standardizer.fit(model, Traw)
    X, Y = sx.apply(model, Xraw), st.apply(model, Traw)
    model.set_params([p.astype(np.float32) for p in
                      W.he_init(np.random.default_rng(0), dims)])
    ms_step = model.time_train(X[:256].data_ptr(), Y[:256].data_ptr(), 256, 20)
    losses, t_train = W.timed(W.train, model, X, Y, args.epochs, 256, 1e-3, 0, 0.9, log)
    # inference for the held-out scenarios: the standardisations folded into
    # the first and last layers, raw loads in, raw multipliers out, handed to
    # the batch on the device
    W.fold_standardizers(model, sx, st)
    keep = np.isfinite(opt)
    Dev, opt = Dev[keep], opt[keep]
    torch.cuda.synchronize()
    start, t_pred = W.timed(W.predict_dev, model, Dev)
    model.close()
    log(f"{int(keep.sum())} held-out scenarios with an optimum; cold solves")
    sc_, sw_ = {}, {}
    (hc, pc), t_cold = W.timed(W.run_to_gap, base, Dev, opt, r["alpha"], r["rho"], None,
                               args.max_iters, 10, 100, stream.cuda_stream, sc_)
    log(f"cold: {t_cold:.1f} s; warm solves")
    (hw, pw), t_warm = W.timed(W.run_to_gap, base, Dev, opt, r["alpha"], r["rho"], start,
                               args.max_iters, 10, 100, stream.cuda_stream, sw_)
    log(f"warm: {t_warm:.1f} s; warm start with its cold shadow in one pipeline")
    # the deployed form: warm and cold shadow side by side for 100
    # iterations, the better trajectory kept per instance on the device
    pipe, t_pipe = W.timed(W.run_with_fallback, base, Dev, opt, r["alpha"], r["rho"], start,
                           100, args.max_iters, 10, stream.cuda_stream)
    hf, used_cold = pipe["hit"], pipe["kept_cold"]
    log(f"warm + fallback: {t_pipe:.1f} s")
    # wall time per iteration of the batched solve (bound checks every 10
    # iterations included), and the time at which the median instance is
    # certified (the shadow's iterations included); the warm start adds one
    # inference pass
    spi_c = sc_["seconds"] / max(sc_["iterations"], 1)
    spi_w = sw_["seconds"] / max(sw_["iterations"], 1)
    cap_c = sc_["seconds_at"][max(sc_["seconds_at"])]
    cap_f = pipe["seconds_at"][max(pipe["seconds_at"])]
    flops = 6.0 * 256 * sum(a * b for a, b in zip(dims[:-1], dims[1:]))
    return dict(
        n_train=int(ok.sum()), n_eval=int(keep.sum()), n_eval_drawn=int(keep.size),
        n_eval_infeasible=int(keep.size - keep.sum()), data_seconds=t_data,
        train_seconds=t_train, epochs=args.epochs, final_loss=losses[-1], first_loss=losses[0],
        train_step_ms=ms_step, train_tflops=flops / (ms_step * 1e-3) / 1e12,
        median_iters_cold=W.median_iters(hc, args.max_iters),
        median_iters_warm=W.median_iters(hw, args.max_iters),
        median_iters_warm_fallback=W.median_iters(hf, args.max_iters),
        reached_cold=float((hc >= 0).mean()), reached_warm_fallback=float((hf >= 0).mean()),
        warm_kept=float(1.0 - used_cold.mean()), solve_seconds_cold=t_cold,
        solve_seconds_warm=t_warm, solve_seconds_warm_fallback=t_pipe,
        instance_iterations_warm_fallback=pipe["instance_iterations"],
        batch_ms_per_iteration_cold=spi_c * 1e3, batch_ms_per_iteration_warm=spi_w * 1e3,
        median_seconds_to_gap_cold=W.median_seconds(hc, sc_["seconds_at"], cap_c),
        median_seconds_to_gap_warm_fallback=W.median_seconds(hf, pipe["seconds_at"], cap_f)
        + t_pred, inference_seconds=t_pred,
        timing_note="median wall time from the hand-off of the start to the check at which "
                    "the median instance is certified; warm + fallback includes the cold "
                    "shadow's 100 iterations, the per-instance choice on the device and one "
                    "inference pass")


def ptdf_tiles(n):
    """64 x 64 x 64 tile products the PTDF build issues for n reduced buses:
    Cholesky panels and trailing updates, the forward substitution on the
    identity, and the lower block triangle of W^T W."""
    T = -(-n // 64)
    chol = sum((T - k - 1) + (T - k - 1) * (T - k) // 2 for k in range(T))
    trsm = sum((i + 1) + (T - i - 1) * (i + 1) for i in range(T))
    xprod = sum((a + 1) * (T - a) for a in range(T))
    return chol + trsm + xprod


def bench_ptdf(args, stream):
    """PTDF construction of the 2000- and 10,000-bus networks: the library's
    dense FP64 path (wall time of the synchronous call, workspace allocation
    included) against the host build of the inputs (SciPy's sparse LU)."""
    import numpy as np
    import torch

    from paper_2406_13191_amd import _abi, synth
    rows = []
    for name, seed, reps in [("bus2000", 2000, 10), ("bus10000", 10000, 3)]:
        net = synth.make_topology(name, seed)
        H = torch.empty((net.n_line, net.n_bus), dtype=torch.float64, device="cuda")

        def call():
            _abi.ptdf(net.n_bus, net.fbus, net.tbus, net.b, net.slack, H.data_ptr(),
                      stream=stream.cuda_stream)
        call()
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            call()
            times.append(time.perf_counter() - t0)
        t_gpu = float(np.median(times))
        flops = ptdf_tiles(net.n_bus - 1) * 2 * 64 ** 3
        print(f"[bench] ptdf {name}: {t_gpu * 1e3:.2f} ms, {flops / t_gpu / 1e12:.2f} TFLOP/s "
              f"issued", file=sys.stderr, flush=True)
        row = dict(network=name, n_bus=net.n_bus, n_line=net.n_line, seconds=round(t_gpu, 5),
                   issued_flops=flops, tflops=round(flops / t_gpu / 1e12, 2))
        if not args.no_cpu:
            t0 = time.perf_counter()
            synth.ptdf(net)
            row["scipy_sparse_lu_seconds"] = round(time.perf_counter() - t0, 3)
        rows.append(row)
        del H
        torch.cuda.empty_cache()
    return rows


def bench_rules(args, stream):
    """Step rules on the 2000-bus LP (FP32 products, exact FP64 bound every
    100 iterations): iterations and wall time to an exact bound within 0.1 %
    of the HiGHS optimum, for each rule over a small grid of step sizes."""
    from paper_2406_13191_amd import _abi, synth
    net, p = synth.make_network("bus2000", 2000)
    opt = _lp_optimum(net, p)
    grid = [("gdm", dict(rho=0.99), [1e-4, 3e-4, 1e-3]),
            ("gdm+decay", dict(rho=0.99, decay=1e-3), [3e-4, 1e-3, 3e-3]),
            ("adam", dict(beta1=0.9, beta2=0.999, eps=1e-8), [0.1, 0.3, 1.0, 3.0, 10.0]),
            ("adagrad", dict(eps=1e-8), [3.0, 10.0, 30.0, 100.0, 300.0])]
    out = []
    for name, extra, alphas in grid:
        for a in alphas:
            kw = dict(rule=name.split("+")[0], alpha=a, precision="fp32", graph_iters=100, **extra)
            with _abi.DualSolver(p, stream=stream.cuda_stream, **kw) as s:
                t0 = time.perf_counter()
                res = s.solve(opt=opt, gap_tol=1e-3, max_iters=args.max_iters, check_every=100)
                dt = time.perf_counter() - t0
            hit = res["status"] == 1
            out.append(dict(rule=name, alpha=a, **{k: v for k, v in extra.items()},
                            reached=hit, iterations=int(res["iter_of_bound"]) if hit else None,
                            seconds=round(dt, 4), gap=res["gap"]))
            print(f"[bench] {name} alpha={a}: {'%d iterations' % res['iter_of_bound'] if hit else 'not reached'}"
                  f" ({dt*1e3:.1f} ms)", file=sys.stderr, flush=True)
    best = {}
    for r in out:
        if r["reached"] and (r["rule"] not in best or r["iterations"] < best[r["rule"]]["iterations"]):
            best[r["rule"]] = r
    return out, best


def bench_qpdual(args, stream):
    """The paper's QP dual with s iterated against the closed-form maximum
    over s, on the 10,000-bus QP (FP32 products): the best exact bound every
    100 iterations, against a certified upper bound (the repaired average of
    a closed-form run), so no external solver is needed."""
    from paper_2406_13191_amd import _abi, synth
    net, p = synth.make_network("bus10000", 10000)
    r = synth.STEP_RULES["bus10000"]
    n = args.max_iters
    kw = dict(rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp32", graph_iters=100)
    with _abi.DualSolver(p, stream=stream.cuda_stream, **kw) as s:
        s.step(n // 2)
        s.average(True)
        s.step(n - n // 2)
        rp = s.repair(None)
    if not rp["feasible"]:
        raise RuntimeError("repair of the closed-form average did not reach feasibility")
    ub = rp["cost"]
    out = dict(upper_bound=ub, repair_rounds=rp["rounds"], iterations=n)
    for mode in ("closed", "iterated"):
        best, pts, hit = -math.inf, [], {"1e-3": None, "1e-4": None}
        with _abi.DualSolver(p, stream=stream.cuda_stream, qp_dual=mode, **kw) as s:
            t0 = time.perf_counter()
            for k in range(100, n + 1, 100):
                s.step(100)
                best = max(best, s.bound())
                gap = (ub - best) / abs(ub)
                for t in hit:
                    if hit[t] is None and gap <= float(t):
                        hit[t] = k
                if k % 1000 == 0:
                    pts.append([k, gap])
            dt = time.perf_counter() - t0
            last_monitor = float(s.gammas(n - 1, 1)[0])
        out[mode] = dict(iterations_to_certified_gap=hit, gap_by_iteration=pts,
                         final_gap=gap, seconds=round(dt, 3),
                         monitor_gap=(ub - last_monitor) / abs(ub))
        print(f"[bench] qp dual {mode}: gap {gap:.2e} after {n}, to 1e-3 at {hit['1e-3']}, "
              f"1e-4 at {hit['1e-4']}", file=sys.stderr, flush=True)
    return out


def bench_single(args, stream, name, net, p, steps, warmup, log, with_cpu=True,
                 with_primal=True):
    """One instance on the single-instance path, FP32 products: iteration
    rate over `steps` iterations replayed as HIP graphs, the dominant
    kernel's roofline, time to a bound within 0.1 % (own iteration cap),
    setup time, and optionally primal recovery and the FP64 oracle."""
    import numpy as np
    import torch

    from paper_2406_13191_amd import _abi, synth
    r = synth.STEP_RULES[name]
    n_cols = len(np.unique(p.gen_bus))
    kw = dict(rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp32", panel=args.panel,
              graph_iters=100)
    if args.panel == "allbus":
        n_cols = p.n_bus
    # setup (reported apart from the iterations): copy of H to the device,
    # panel gather in both orientations, f_d = H d.  The first create of a
    # process also loads the library's kernels, so the second one is timed.
    setup = []
    for _ in range(2):
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        s = _abi.DualSolver(p, stream=stream.cuda_stream, **kw)
        torch.cuda.synchronize()
        setup.append(time.perf_counter() - t_s)
        if len(setup) == 1:
            s.close()
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    log(f"{name}: {steps} iterations in {ms:.2f} ms (wall {wall*1e3:.2f} ms)")
    # per-kernel durations for the roofline: events attached to each dispatch of
    # 200 real iterations (the iterate is restored afterwards), median of five
    # such samples
    ms_col, ms_line = (float(v) for v in
                       np.median(np.array([s.time_phases(200) for _ in range(5)]), axis=0))
    sch = s.scheme()
    s.close()
    scheme = sch["scheme"]
    b_col, b_line = panel_bytes(p.n_line, n_cols, p.n_gen, scheme)
    names = {"two_pass": ("colpass (w = P^T v, inner minimiser)",
                          "linepass (F = P x - f_d, mu step)"),
             "read_once": ("unit pass (w from the line pass's partials, inner minimiser)",
                           "line pass (F = P x - f_d, mu step, partials of the next P^T v)")}
    first = "colpass" if scheme == "two_pass" else "unitpass"
    if ms_line >= ms_col:
        kkey, kname, kms, kbytes = "linepass", names[scheme][1], ms_line, b_line
    else:
        kkey, kname, kms, kbytes = first, names[scheme][0], ms_col, b_col
    achieved = kbytes / (kms * 1e-3) / 1e9
    traffic = measured_traffic(f"{name}/{args.panel}/{scheme}:{kkey}", SINGLE_SRC)
    it_bytes = b_col + b_line
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=kname,
                    kernel_ms=round(kms, 5), bytes_per_launch=int(kbytes),
                    other_kernel_ms=round(min(ms_col, ms_line), 5), scheme=scheme,
                    iteration=dict(bytes=int(it_bytes), us=round(ms / steps * 1e3, 3),
                                   gbs=round(it_bytes / (ms / steps * 1e-3) / 1e9, 1),
                                   frac=round(it_bytes / (ms / steps * 1e-3) / 1e9
                                              / HBM_PEAK_GBS, 4)))
    if scheme == "read_once":
        # partials of P^T v: written by the line pass, read by the unit pass
        roofline["partial_bytes"] = int(2 * 4 * sch["line_groups"] * n_cols)

    # time to a bound within 0.1 % of the FP64 optimum (HiGHS reference for
    # an LP), with an iteration cap of its own
    ttb = primal = cpu = None
    if not p.is_qp:
        opt = _lp_optimum(net, p)
        target = "HiGHS optimum"
    else:
        # no QP solver here: the target is a certified upper bound, the cost
        # of the repaired primal average of a long run (every feasible cost
        # is >= OPT, so a bound within 0.1 % of it is within 0.1 % of OPT)
        with _abi.DualSolver(p, stream=stream.cuda_stream, **kw) as s3:
            s3.step(args.ttb_cap // 2)
            s3.average(True)
            s3.step(args.ttb_cap - args.ttb_cap // 2)
            lb_long = s3.bound()
            rp = s3.repair(None)
        opt = rp["cost"] if rp["feasible"] else None
        target = (f"certified upper bound: repaired primal average of {args.ttb_cap} "
                  f"iterations (cost {opt}, {(opt - lb_long) / abs(opt):.2e} above that run's "
                  f"last exact bound)" if opt is not None else None)
    if opt is not None:
        with _abi.DualSolver(p, stream=stream.cuda_stream, **kw) as s2:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = s2.solve(opt=opt, gap_tol=1e-3, max_iters=args.ttb_cap, check_every=100)
            dt = time.perf_counter() - t0
        ttb = dict(reached=res["status"] == 1, iterations=int(res["iter_of_bound"]),
                   iteration_cap=args.ttb_cap, seconds=round(dt, 5), gap=res["gap"],
                   check_every=100, target=target,
                   device_seconds=round(res["iter_of_bound"] * ms / steps / 1e3, 6))
    if with_primal:
        # primal recovery: the average of p* over iterations 2000..10000 (exact
        # bound checked every 100), then its repair into a feasible dispatch,
        # whose cost certifies the gap of the best bound without HiGHS
        with _abi.DualSolver(p, stream=stream.cuda_stream, **kw) as s3:
            s3.step(2000)
            s3.average(True)
            s3.solve(opt=float("nan"), gap_tol=0.0, max_iters=8000, check_every=100)
            lb, _ = s3.best()
            pr = s3.primal()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rp = s3.repair(None)
            t_rep = time.perf_counter() - t0
        opt = None if p.is_qp else _lp_optimum(net, p)
        primal = dict(window=[2000, 10000], cost=pr["cost"], best_lower_bound=lb,
                      gap_to_opt=None if p.is_qp else (pr["cost"] - opt) / abs(opt),
                      balance_mw=pr["balance"], max_overload_mw=pr["max_overload"],
                      overloaded_directions=pr["n_overloaded"],
                      repair=dict(feasible=rp["feasible"], cost=rp["cost"], rounds=rp["rounds"],
                                  lines_held=rp["n_active"], max_shift_mw=rp["max_shift"],
                                  seconds=round(t_rep, 5),
                                  certified_gap=(rp["cost"] - lb) / abs(rp["cost"])
                                  if rp["feasible"] else None,
                                  ub_minus_opt=None if p.is_qp else (rp["cost"] - opt) / abs(opt)))
    if with_cpu:
        cpu = cpu_baseline(p, r["alpha"], r["rho"])
    desc = (f"{name} single instance: {p.n_bus} buses, {p.n_line} lines, {p.n_gen} generators "
            f"on {n_cols} buses, {'quadratic' if p.is_qp else 'linear'} costs; "
            f"{'full-PTDF' if args.panel == 'allbus' else 'generator-bus'} panel; FP32 PTDF "
            f"products, FP64 multipliers and bound; gradient with momentum "
            f"alpha={r['alpha']}, rho={r['rho']}")
    return dict(value=steps / (ms / 1e3), ms=ms, steps=steps, warmup=warmup, workload=desc,
                time_to_bound=ttb, setup_seconds=round(setup[1], 5),
                setup_note="dcopf_dual_create on the host-resident problem: H "
                           f"({p.n_line} x {p.n_bus} FP64) copied to the device, panel "
                           f"gathered ({scheme.replace('_', '-')} scheme), f_d = H d; first "
                           "create "
                           f"(kernel loading included) {setup[0]:.4f} s",
                primal_recovery=primal, roofline=roofline, cpu_baseline=cpu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed iterations (default 2000 for the mixed batch, 20000 for a "
                         "single instance)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="mixed",
                    help="mixed (default) | bus2000 | bus4600 | bus10000 | warmstart | ptdf | "
                         "rules | qpdual | screening | copy")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--panel", default="genbus", choices=["genbus", "allbus"])
    ap.add_argument("--ttb-cap", type=int, default=20000,
                    help="iteration cap of the time-to-bound legs (independent of --steps)")
    ap.add_argument("--train", type=int, default=50000)
    ap.add_argument("--eval", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--target-iters", type=int, default=5000)
    ap.add_argument("--max-iters", type=int, default=5000)
    ap.add_argument("--tiles", default=None,
                    help="mixed batch: JSON list of per-network tiles (the 'tiles' of an "
                         "earlier run's config) to pin instead of autotuning")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on one device (batched "
              "instances would split across GPUs with no per-iteration exchange; one large "
              "instance would need an all-reduce of Pt v per iteration).", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 2000 if args.workload == "mixed" else 20000
    log = lambda m: print("[bench]", m, file=sys.stderr, flush=True)  # noqa: E731

    import numpy as np
    import torch

    # host-side inputs of the default workload first: nothing below this
    # point forks or spawns processes once the GPU is in use
    nets = prep_mixed(log) if args.workload == "mixed" else None
    wprep = prep_warmstart(args, log) if args.workload == "warmstart" else None
    sprep = prep_screening(log) if args.workload == "screening" else None

    from paper_2406_13191_amd import _abi, synth  # noqa: F401  (loads the library)

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload == "copy":
        copy_calibration()
        return
    if args.workload == "warmstart":
        r = bench_warmstart(args, stream, wprep)
        out = {
            "metric": "median iterations to a bound within 0.1% of the FP64 optimum, "
                      "learned warm start vs cold start",
            "value": r["median_iters_warm_fallback"], "unit": "iterations",
            "n_gpus": 1, "steps": args.max_iters, "warmup": 0, "ms_per_step": None,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16", "data": "synthetic",
            "config": {"workload": f"warm start on the 2000-bus network: MLP 2000-1024-1024-6401 "
                                   f"trained on {r['n_train']} cold-solve duals, evaluated on "
                                   f"{r['n_eval']} held-out scenarios", **r},
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(out), flush=True)
        return
    if args.workload == "qpdual":
        r = bench_qpdual(args, stream)
        it = r["iterated"]["iterations_to_certified_gap"]["1e-3"]
        out = {
            "metric": "iterations to an exact bound within 0.1% of a certified upper bound, "
                      "the paper's iterated-s QP dual (closed form beside it)",
            "value": it, "unit": "iterations", "n_gpus": 1, "steps": args.max_iters,
            "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "10,000-bus single instance with quadratic costs (12,700 "
                                   "lines, 2500 generators), FP32 products, exact FP64 bound "
                                   "every 100 iterations", **r},
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(out), flush=True)
        return
    if args.workload == "screening":
        res = bench_screening(args, stream, sprep, log)
        out = {
            "metric": "median iterations to an exact bound within 0.1% of the FP64 optimum, "
                      "default against unscreened line limits",
            "value": res["bus4600_raw"]["median_iterations"], "unit": "iterations",
            "n_gpus": 1, "steps": args.ttb_cap, "warmup": 0, "ms_per_step": None,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
            "data": "synthetic",
            "config": {"workload": "2000- and 4600-bus networks, 32 load and cost scenarios "
                                   "each, with the default limits and with the unscreened "
                                   "recipe; each network alone as a batch, GDM with its frozen "
                                   "rule, exact bound every 100 iterations",
                       "networks": res},
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(out), flush=True)
        return
    if args.workload == "rules":
        runs, best = bench_rules(args, stream)
        g = best.get("gdm")
        out = {
            "metric": "iterations to an exact bound within 0.1% of the FP64 optimum, by step rule",
            "value": min(r["iterations"] for r in best.values()) if best else None,
            "unit": "iterations", "n_gpus": 1, "steps": args.max_iters, "warmup": 0,
            "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "2000-bus single instance (3200 lines, 540 generators), "
                                   "FP32 products, exact FP64 bound every 100 iterations; "
                                   "each rule over a grid of step sizes on this instance",
                       "best": best, "runs": runs,
                       "gdm_frozen_rule": g},
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(out), flush=True)
        return
    if args.workload == "ptdf":
        rows = bench_ptdf(args, stream)
        big = rows[-1]
        cores = torch.get_num_threads()
        cpu = None
        if not args.no_cpu:
            # cpu_baseline leg: the FP64 oracle's dense build, timed once
            from oracle import ptdf as OP
            net = synth.make_topology("bus10000", 10000)
            t0 = time.perf_counter()
            OP.ptdf(net.n_bus, net.fbus, net.tbus, net.b, net.slack)
            cpu = {"value": round(time.perf_counter() - t0, 3), "unit": "s", "cores": cores,
                   "kind": "oracle", "sample": "one dense FP64 build of the 10,000-bus PTDF "
                                               "(numpy solve)"}
        out = {
            "metric": "seconds to build the PTDF of the 10,000-bus network",
            "value": big["seconds"], "unit": "s", "n_gpus": 1, "steps": 3, "warmup": 1,
            "ms_per_step": big["seconds"] * 1e3, "higher_is_better": False, "scaling": "strong",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "PTDF construction (dense FP64: blocked Cholesky, "
                                   "L^-1, W^T W, row gather) of the 2000-bus (3200 lines) and "
                                   "10,000-bus (12,700 lines) networks", "networks": rows},
            "roofline": {"bound": "mfma", "achieved": big["tflops"], "peak": 78.6,
                         "unit": "TFLOP/s", "frac": round(big["tflops"] / 78.6, 4),
                         "traffic": None, "kernel": "whole build (wall time, allocation "
                                                    "included)"},
            "cpu_baseline": cpu,
        }
        print(json.dumps(out), flush=True)
        return
    if args.workload == "mixed":
        r = bench_mixed(args, stream, nets, log)
        # the 2000-bus single instance (the batch's 2000-bus network, its
        # base loads and costs) on the single-instance path, for reference
        n2 = [n for n in nets if n["name"] == "bus2000"][0]
        single = bench_single(args, stream, "bus2000", n2["topo"], n2["base"], 2000, 200, log,
                              with_cpu=False, with_primal=False)
        cpu = None
        if not args.no_cpu:
            cpu = cpu_baseline_batch(nets)
            ttb = r["time_to_bound"]
            if ttb["reached"]:
                cpu["seconds_for_the_gpu_iterations_to_bound"] = round(
                    ttb["iterations"] * cpu["seconds_per_iteration"], 2)
            log(f"cpu baseline: {cpu['value']:.0f} instance-iterations/s ({cpu['cores']} threads)")
        out = {
            "metric": METRIC, "value": round(r["value"], 1), "unit": "instance-iterations/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms"] / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
            "config": {"workload": "mixed batch: " + ", ".join(
                f"{B} x {n} ({nl} lines, {nc} generator buses)" for n, nl, nc, ng, B in r["shapes"])
                + "; split-BF16 MFMA products (hi*hi + hi*lo + lo*hi, FP32 accumulation), FP32 "
                  "line state, FP64 lambda and exact bound; gradient with momentum",
                "instances": r["n_total"], "tiles": r["tiles"],
                "create_seconds": r["create_seconds"],
                "time_to_bound": r["time_to_bound"],
                "vs_single_instance_path": r["single_path"],
                "single_instance_bus2000": single,
                "certified": r["certified"]},
            "roofline": r["roofline"], "cpu_baseline": cpu,
        }
        print(json.dumps(out), flush=True)
        return
    t = time.perf_counter()
    net, p = synth.make_network(args.workload, {"bus2000": 2000, "bus4600": 4600,
                                                "bus10000": 10000}[args.workload])
    log(f"network {args.workload}: {time.perf_counter() - t:.1f} s")
    r = bench_single(args, stream, args.workload, net, p, args.steps, args.warmup, log,
                     with_cpu=not args.no_cpu, with_primal=not args.no_cpu)
    out = {
        "metric": METRIC, "value": round(r["value"], 1), "unit": "instance-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": r["workload"], "iterations": args.steps,
                   "time_to_bound": r["time_to_bound"], "setup_seconds": r["setup_seconds"],
                   "setup_note": r["setup_note"], "primal_recovery": r["primal_recovery"]},
        "roofline": r["roofline"],
        "cpu_baseline": r["cpu_baseline"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
