"""Seeded synthetic DCOPF instances (networks, PTDF, generators, loads, limits).

This module only *builds inputs*: topology, susceptances, the PTDF matrix of
the DCOPF statement (Section 2, eq. DCOPF: H = Omega E (E^T Omega E)^{-1},
H_a = H with a zero slack column), generator data, loads and line limits.
It holds none of the dual-ascent arithmetic.  Both the GPU path and the CPU
oracle take their inputs from here; nothing here imports either of them.

The paper evaluates on the PGLib 2000/4601/10000-bus cases, which are not
available; the recipes below generate stand-ins of the same sizes:

* ``tiny30``  - 30 buses, random recursive tree + 12 extra edges = 41 lines,
  6 generators with linear costs, 20 loaded buses at 60 % of capacity,
  5 limited lines (0.8 x merit-order flow), others 1e4 MW.
* ``geo``     - Euclidean MST over uniform points plus the shortest
  non-tree Delaunay edges up to the line count; lognormal susceptances;
  generators on uniformly drawn buses (repeats allowed), lognormal p_max,
  lognormal loads on 60 % of buses, a few per cent of lines targeted at
  0.8 x the economic-dispatch flow.

All randomness is ``numpy.random.Generator(PCG64(seed))`` with a fixed draw
order, so a (recipe, seed) pair always yields the same arrays.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import os
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import minimum_spanning_tree
from scipy.optimize import linprog
from scipy.spatial import Delaunay

__all__ = [
    "Network", "Problem", "NET_SPECS", "make_network", "make_problem",
    "make_scenarios", "make_topology", "ptdf", "config_problem", "STEP_RULES",
]


@dataclasses.dataclass
class Network:
    """Transmission topology.  Line l runs from ``fbus[l]`` to ``tbus[l]``."""
    n_bus: int
    fbus: np.ndarray   # int64 [n_line]
    tbus: np.ndarray   # int64 [n_line]
    b: np.ndarray      # float64 [n_line] series susceptance (p.u.)
    slack: int

    @property
    def n_line(self) -> int:
        return int(self.fbus.shape[0])


@dataclasses.dataclass
class Problem:
    """One DCOPF instance in the paper's statement (Section 2, eq. DCOPF).

    minimise sum_g c_g p_g + q_g p_g^2
    s.t. 1^T p = 1^T d,  -f_max <= H (C_g p - d) <= f_max,  p_min <= p <= p_max
    """
    H: np.ndarray          # float64 [n_line, n_bus] row-major, H[:, slack] == 0
    gen_bus: np.ndarray    # int32 [n_gen]
    c: np.ndarray          # float64 [n_gen]  $/MWh
    q: np.ndarray          # float64 [n_gen]  $/MW^2h (zeros for an LP)
    p_min: np.ndarray      # float64 [n_gen]  MW
    p_max: np.ndarray      # float64 [n_gen]  MW
    d: np.ndarray          # float64 [n_bus]  MW
    f_max: np.ndarray      # float64 [n_line] MW
    slack: int
    net: Optional[Network] = None

    @property
    def n_bus(self) -> int:
        return int(self.H.shape[1])

    @property
    def n_line(self) -> int:
        return int(self.H.shape[0])

    @property
    def n_gen(self) -> int:
        return int(self.gen_bus.shape[0])

    @property
    def is_qp(self) -> bool:
        return bool(np.any(self.q > 0))

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# PTDF (Section 2): H = Omega E (E^T Omega E)^{-1} over the non-slack buses,
# augmented with a zero column for the slack bus.
# --------------------------------------------------------------------------
def ptdf(net: Network) -> np.ndarray:
    """Dense PTDF H_a [n_line, n_bus] (float64) with a zero slack column.

    Solves the reduced susceptance system B_r Z = I with a sparse LU; row l of
    H_a is then b_l (Z[f_l, :] - Z[t_l, :]) where Z is padded with a zero row
    and column at the slack bus.
    """
    nb, nl = net.n_bus, net.n_line
    rows = np.arange(nl)
    E = sp.csr_matrix(
        (np.concatenate([np.ones(nl), -np.ones(nl)]),
         (np.concatenate([rows, rows]), np.concatenate([net.fbus, net.tbus]))),
        shape=(nl, nb))
    keep = np.array([i for i in range(nb) if i != net.slack])
    Er = E[:, keep].tocsc()
    Br = (Er.T @ sp.diags(net.b) @ Er).tocsc()
    lu = spla.splu(Br)
    Zr = lu.solve(np.eye(nb - 1))
    Z = np.zeros((nb, nb))
    Z[np.ix_(keep, keep)] = Zr
    H = net.b[:, None] * (Z[net.fbus, :] - Z[net.tbus, :])
    H[:, net.slack] = 0.0
    return np.ascontiguousarray(H)


# --------------------------------------------------------------------------
# Topologies
# --------------------------------------------------------------------------
def _tiny_tree_topology(rng, n_bus, n_extra):
    edges = []
    present = set()
    for i in range(1, n_bus):
        p = int(rng.integers(0, i))
        edges.append((p, i))
        present.add((min(p, i), max(p, i)))
    while len(edges) < n_bus - 1 + n_extra:
        i, j = (int(v) for v in rng.integers(0, n_bus, 2))
        key = (min(i, j), max(i, j))
        if i == j or key in present:
            continue
        present.add(key)
        edges.append(key)
    e = np.array(edges, dtype=np.int64)
    return e[:, 0], e[:, 1]


def _geometric_topology(rng, n_bus, n_line):
    pts = rng.random((n_bus, 2))
    tri = Delaunay(pts)
    s = tri.simplices
    e = np.vstack([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    length = np.hypot(*(pts[e[:, 0]] - pts[e[:, 1]]).T)
    G = sp.csr_matrix((length, (e[:, 0], e[:, 1])), shape=(n_bus, n_bus))
    T = minimum_spanning_tree(G).tocoo()
    tree = set(zip(np.minimum(T.row, T.col).tolist(), np.maximum(T.row, T.col).tolist()))
    if len(tree) != n_bus - 1:
        raise RuntimeError("Delaunay graph is not connected")
    in_tree = np.array([(int(a), int(b)) in tree for a, b in e])
    order = np.lexsort((e[:, 1], e[:, 0], length))
    extra = [k for k in order if not in_tree[k]][: n_line - (n_bus - 1)]
    if len(extra) < n_line - (n_bus - 1):
        raise RuntimeError("not enough candidate edges")
    chosen = np.concatenate([np.nonzero(in_tree)[0], np.array(extra, dtype=np.int64)])
    chosen.sort()
    return e[chosen, 0].astype(np.int64), e[chosen, 1].astype(np.int64)


# --------------------------------------------------------------------------
# Dispatch used only to place line limits (instance construction)
# --------------------------------------------------------------------------
def _unconstrained_dispatch(c, q, p_min, p_max, demand):
    """Cheapest dispatch ignoring lines: merit order (q == 0) or equal
    incremental cost by bisection (q > 0).  Used to target line limits."""
    if not np.any(q > 0):
        p = p_min.copy()
        rest = demand - p.sum()
        for g in np.lexsort((np.arange(c.size), c)):
            take = min(p_max[g] - p_min[g], rest)
            p[g] += take
            rest -= take
            if rest <= 0:
                break
        return p
    qq = np.where(q > 0, q, 1e-12)
    lo, hi = -1e4, 1e4
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        p = np.clip((mid - c) / (2 * qq), p_min, p_max)
        if p.sum() < demand:
            lo = mid
        else:
            hi = mid
    return np.clip((0.5 * (lo + hi) - c) / (2 * qq), p_min, p_max)


def _flows(H, gen_bus, p, d):
    inj = -d.copy()
    np.add.at(inj, gen_bus, p)
    return H @ inj


def _min_violation_dispatch(net, gen_bus, p_min, p_max, d, f_max):
    """Dispatch minimising the total line-limit violation (bus-angle form:
    C_g p - B theta = d, flows b (theta_f - theta_t), |flow| <= f_max + s,
    s >= 0, min sum s), solved by HiGHS.  Returns the flows at that dispatch
    and the violations s."""
    nb, nl, ng = net.n_bus, net.n_line, gen_bus.size
    rows = np.arange(nl)
    E = sp.csr_matrix((np.concatenate([np.ones(nl), -np.ones(nl)]),
                       (np.concatenate([rows, rows]),
                        np.concatenate([net.fbus, net.tbus]))), shape=(nl, nb))
    Fm = (sp.diags(net.b) @ E).tocsr()
    Bm = (E.T @ Fm).tocsr()
    Cg = sp.csr_matrix((np.ones(ng), (gen_bus, np.arange(ng))), shape=(nb, ng))
    z = sp.csr_matrix((nl, ng))
    I = sp.identity(nl, format="csr")
    res = linprog(np.concatenate([np.zeros(ng + nb), np.ones(nl)]),
                  A_ub=sp.vstack([sp.hstack([z, Fm, -I]),
                                  sp.hstack([z, -Fm, -I])]).tocsr(),
                  b_ub=np.concatenate([f_max, f_max]),
                  A_eq=sp.hstack([Cg, -Bm, sp.csr_matrix((nb, nl))]).tocsr(), b_eq=d,
                  bounds=list(zip(p_min, p_max)) +
                  [(0.0, 0.0) if i == net.slack else (None, None) for i in range(nb)] +
                  [(0.0, None)] * nl,
                  method="highs")
    if res.status != 0:
        raise RuntimeError("violation LP failed: " + str(res.message))
    theta = res.x[ng: ng + nb]
    return Fm @ theta, res.x[ng + nb:]


def _line_prices(net, gen_bus, c, p_min, p_max, d, f_max):
    """Linear-cost DCOPF in bus-angle form solved by HiGHS; returns the flows
    at the optimum and each line's limit price max(mu+, mu-)."""
    nb, nl, ng = net.n_bus, net.n_line, gen_bus.size
    rows = np.arange(nl)
    E = sp.csr_matrix((np.concatenate([np.ones(nl), -np.ones(nl)]),
                       (np.concatenate([rows, rows]),
                        np.concatenate([net.fbus, net.tbus]))), shape=(nl, nb))
    Fm = (sp.diags(net.b) @ E).tocsr()
    Bm = (E.T @ Fm).tocsr()
    Cg = sp.csr_matrix((np.ones(ng), (gen_bus, np.arange(ng))), shape=(nb, ng))
    z = sp.csr_matrix((nl, ng))
    res = linprog(np.concatenate([c, np.zeros(nb)]),
                  A_ub=sp.vstack([sp.hstack([z, Fm]), sp.hstack([z, -Fm])]).tocsr(),
                  b_ub=np.concatenate([f_max, f_max]),
                  A_eq=sp.hstack([Cg, -Bm]).tocsr(), b_eq=d,
                  bounds=list(zip(p_min, p_max)) +
                  [(0.0, 0.0) if i == net.slack else (None, None) for i in range(nb)],
                  method="highs")
    if res.status != 0:
        raise RuntimeError("pricing LP failed: " + str(res.message))
    mu = -res.ineqlin.marginals
    return Fm @ res.x[ng:], np.maximum(mu[:nl], mu[nl:])


def _cap_prices(net, gen_bus, c, p_min, p_max, d, f_max, cap, rounds=6):
    """Relax (to REPAIR_MARGIN x the optimal flow) every line whose limit price exceeds
    ``cap`` and re-solve, so that no congestion price is extreme.  A line the
    generators can barely influence needs an enormous multiplier to bind;
    such lines make the dual badly scaled and are not what the workload is
    meant to contain."""
    f = f_max.copy()
    for _ in range(rounds):
        flows, price = _line_prices(net, gen_bus, c, p_min, p_max, d, f)
        bad = price > cap
        if not np.any(bad):
            break
        f[bad] = np.abs(flows[bad]) * REPAIR_MARGIN
    return f


def _bridges(n_bus, fbus, tbus) -> np.ndarray:
    """Boolean mask of bridge lines (removal disconnects the graph), found by
    an iterative depth-first search with low-link values."""
    adj = [[] for _ in range(n_bus)]
    for l, (a, b) in enumerate(zip(fbus.tolist(), tbus.tolist())):
        adj[a].append((b, l))
        adj[b].append((a, l))
    disc = [-1] * n_bus
    low = [0] * n_bus
    is_bridge = np.zeros(fbus.size, bool)
    timer = 0
    for root in range(n_bus):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, iter(adj[root]))]
        while stack:
            u, pl, it = stack[-1]
            advanced = False
            for v, l in it:
                if l == pl:
                    continue
                if disc[v] < 0:
                    disc[v] = low[v] = timer
                    timer += 1
                    stack.append((v, l, iter(adj[v])))
                    advanced = True
                    break
                low[u] = min(low[u], disc[v])
            if not advanced:
                stack.pop()
                if stack:
                    p = stack[-1][0]
                    low[p] = min(low[p], low[u])
                    if low[u] > disc[p]:
                        is_bridge[pl] = True
    return is_bridge


def _relievable(net, gen_bus, p_min, p_max, d, F0, lines):
    """For each line, can some dispatch (box + balance, other lines ignored)
    bring its flow within 0.8 |F0|?  The flow is a linear function a.p - f_d
    of the dispatch; its range over {p in box, sum p = D} is found by filling
    generators in order of a (fractional knapsack), for every line at once."""
    H = ptdf(net) if getattr(net, "_H", None) is None else net._H
    A = H[np.ix_(lines, gen_bus)]                      # [L, n_g]
    fd = H[lines] @ d
    D = d.sum()
    span = p_max - p_min
    extra = D - p_min.sum()

    def extreme(sign):
        idx = np.argsort(sign * A, axis=1, kind="stable")
        a_s = np.take_along_axis(A, idx, 1)
        cap = span[idx]
        before = np.cumsum(cap, axis=1) - cap
        take = np.clip(extra - before, 0.0, cap)
        return (a_s * take).sum(1) + A @ p_min - fd

    lo, hi = extreme(1.0), extreme(-1.0)
    lim = 0.8 * F0[lines]
    return (lo <= lim) & (hi >= -lim)


def _widen_for_scenarios(net, gen_bus, p_min, p_max, d, f_max, rng, sigma=0.15,
                         samples=16, rounds=4):
    """Widen limits so that load scenarios around the base case (per-bus
    multipliers exp(N(0, sigma^2))) are feasible: for each sampled scenario
    the least-violation dispatch is computed and every limit it violates is
    raised to 1.1 x that flow."""
    f = f_max.copy()
    for _ in range(rounds):
        changed = False
        for _ in range(samples):
            dd = d * np.exp(rng.normal(0.0, sigma, d.size))
            if dd.sum() > p_max.sum() or dd.sum() < p_min.sum():
                continue
            flows, viol = _min_violation_dispatch(net, gen_bus, p_min, p_max, dd, f)
            bad = viol > 1e-9 * np.maximum(f, 1.0)
            if np.any(bad):
                f[bad] = np.abs(flows[bad]) * 1.1
                changed = True
        if not changed:
            break
    return f


def _place_targets(net, gen_bus, p_min, p_max, d, f_max, F0, order, n_target, screen=True):
    """Tighten the first ``n_target`` candidate lines of ``order`` to 0.8 |F0|
    and make the instance feasible with one LP.

    Bridge lines and lines that no dispatch can relieve on their own are not
    candidates (unless screen is False).  The dispatch of least total
    violation is then computed; every
    limit it still violates is raised to REPAIR_MARGIN x that dispatch's flow,
    so that dispatch is feasible and the instance is feasible by construction.
    """
    if screen:
        order = order[~_bridges(net.n_bus, net.fbus, net.tbus)[order]]
        order = order[_relievable(net, gen_bus, p_min, p_max, d, F0, order)]
    target = order[:n_target]
    f = f_max.copy()
    f[target] = 0.8 * F0[target]
    flows, viol = _min_violation_dispatch(net, gen_bus, p_min, p_max, d, f)
    raise_ = viol > 0
    f[raise_] = np.abs(flows[raise_]) * REPAIR_MARGIN
    return f


# --------------------------------------------------------------------------
# Recipes
# --------------------------------------------------------------------------
PRICE_CAP = 1000.0   # $/MWh, largest line-limit price allowed in a recipe
REPAIR_MARGIN = 1.25  # headroom of a repaired or relaxed limit over its flow, so
                      # that load scenarios around the base case stay feasible

NET_SPECS = {
    # name: (recipe, n_bus, n_line, n_gen, qp, c range, load fraction, bind fraction)
    "tiny30": dict(recipe="tiny", n_bus=30, n_line=41, n_gen=6, qp=False,
                   c=(10.0, 50.0), load_frac=0.60, n_target=5),
    "geo300": dict(recipe="geo", n_bus=300, n_line=420, n_gen=70, qp=False,
                   c=(10.0, 80.0), load_frac=0.70, bind_frac=0.03),
    "geo300q": dict(recipe="geo", n_bus=300, n_line=420, n_gen=70, qp=True,
                    c=(5.0, 60.0), q=(0.001, 0.05), load_frac=0.75, bind_frac=0.03),
    "bus2000": dict(recipe="geo", n_bus=2000, n_line=3200, n_gen=540, qp=False,
                    c=(10.0, 80.0), load_frac=0.70, bind_frac=0.03),
    "bus4600": dict(recipe="geo", n_bus=4600, n_line=5900, n_gen=1000, qp=False,
                    c=(10.0, 80.0), load_frac=0.70, bind_frac=0.03),
    "bus10000": dict(recipe="geo", n_bus=10000, n_line=12700, n_gen=2500, qp=True,
                     c=(5.0, 60.0), q=(0.001, 0.05), load_frac=0.75, bind_frac=0.02),
}
# The same networks and loads with limits that keep what the default recipe
# screens out: any of the upper half of lines by base flow may be tightened
# (bridges and lines no dispatch can relieve included) and no limit price is
# capped.  Feasibility is still made by construction, so each instance has
# an optimum; used to measure how much the screening eases the ascent.
for _n in ("bus2000", "bus4600"):
    NET_SPECS[_n + "_raw"] = dict(NET_SPECS[_n], raw=True)


def _cache_path(name: str, seed: int):
    """Directory for a generated network when DCOPF_SYNTH_CACHE names a
    cache directory (keyed by this module's source, so a changed recipe
    never reuses an old network); None otherwise."""
    root = os.environ.get("DCOPF_SYNTH_CACHE")
    if not root:
        return None
    with open(__file__, "rb") as f:
        tag = hashlib.sha256(f.read()).hexdigest()[:16]
    return os.path.join(root, f"{name}_{seed}_{tag}")


_CACHED = ("fbus", "tbus", "b", "H", "gen_bus", "c", "q", "p_min", "p_max", "d", "f_max")


def make_network(name: str, seed: int):
    """Return (Network, Problem) for the named recipe and seed."""
    path = _cache_path(name, seed)
    if path and os.path.exists(os.path.join(path, "done")):
        a = {k: np.load(os.path.join(path, k + ".npy"), allow_pickle=False) for k in _CACHED}
        net = Network(int(a["H"].shape[1]), a["fbus"], a["tbus"], a["b"], 0)
        net._H = None
        return net, Problem(H=a["H"], gen_bus=a["gen_bus"], c=a["c"], q=a["q"],
                            p_min=a["p_min"], p_max=a["p_max"], d=a["d"], f_max=a["f_max"],
                            slack=0, net=net)
    net, prob = _make_network(name, seed)
    if path:
        os.makedirs(path, exist_ok=True)
        vals = dict(fbus=net.fbus, tbus=net.tbus, b=net.b, H=prob.H, gen_bus=prob.gen_bus,
                    c=prob.c, q=prob.q, p_min=prob.p_min, p_max=prob.p_max, d=prob.d,
                    f_max=prob.f_max)
        for k in _CACHED:
            np.save(os.path.join(path, k + ".npy"), vals[k], allow_pickle=False)
        open(os.path.join(path, "done"), "w").close()
    return net, prob


def _topology(spec, rng) -> Network:
    """The network of a configuration: the first draws of its generator."""
    nb = spec["n_bus"]
    if spec["recipe"] == "tiny":
        fbus, tbus = _tiny_tree_topology(rng, nb, spec["n_line"] - (nb - 1))
        b = rng.uniform(5.0, 20.0, fbus.size)
    else:
        fbus, tbus = _geometric_topology(rng, nb, spec["n_line"])
        b = rng.lognormal(2.5, 0.5, fbus.size)
    return Network(nb, fbus, tbus, b, 0)


def make_topology(name: str, seed: int) -> Network:
    """Only the network (buses, lines, susceptances, slack) of
    ``make_network(name, seed)``, without its PTDF or dispatch data."""
    return _topology(NET_SPECS[name], np.random.Generator(np.random.PCG64(seed)))


def _make_network(name: str, seed: int):
    spec = NET_SPECS[name]
    rng = np.random.Generator(np.random.PCG64(seed))
    nb, ng = spec["n_bus"], spec["n_gen"]
    net = _topology(spec, rng)
    if spec["recipe"] == "tiny":
        gen_bus = rng.choice(nb, ng, replace=False).astype(np.int32)
        c = rng.uniform(*spec["c"], ng)
        q = np.zeros(ng)
        p_min = np.zeros(ng)
        p_max = rng.uniform(50.0, 200.0, ng)
        load_bus = rng.choice(nb, 20, replace=False)
        loads = rng.uniform(0.0, 60.0, 20)
    else:
        gen_bus = rng.integers(0, nb, ng).astype(np.int32)
        c = rng.uniform(*spec["c"], ng)
        q = rng.uniform(*spec["q"], ng) if spec["qp"] else np.zeros(ng)
        p_min = np.zeros(ng)
        p_max = rng.lognormal(math.log(100.0), 0.5, ng)
        load_bus = rng.choice(nb, int(round(0.6 * nb)), replace=False)
        loads = rng.lognormal(0.0, 1.0, load_bus.size)
    d = np.zeros(nb)
    d[load_bus] = loads
    d *= spec["load_frac"] * p_max.sum() / d.sum()
    H = ptdf(net)
    net._H = H
    p0 = _unconstrained_dispatch(c, q, p_min, p_max, d.sum())
    F0 = np.abs(_flows(H, gen_bus, p0, d))
    nl = net.n_line
    if spec["recipe"] == "tiny":
        cand = np.nonzero(F0 >= np.median(F0))[0]
        target = rng.choice(cand, spec["n_target"], replace=False)
        f_max = np.full(nl, 1e4)
        f_max[target] = 0.8 * F0[target]
    else:
        n_target = int(round(spec["bind_frac"] * nl))
        top = np.argsort(-F0, kind="stable")[: nl // 2]
        order = rng.permutation(top)
        f_max = np.maximum(2.0 * F0, 0.5 * np.median(F0))
        raw = spec.get("raw", False)
        f_max = _place_targets(net, gen_bus, p_min, p_max, d, f_max, F0, order,
                               n_target, screen=not raw)
        if not raw:
            f_max = _cap_prices(net, gen_bus, c, p_min, p_max, d, f_max,
                                cap=PRICE_CAP)
        f_max = _widen_for_scenarios(net, gen_bus, p_min, p_max, d, f_max, rng)
    net._H = None
    prob = Problem(H=H, gen_bus=gen_bus, c=c, q=q, p_min=p_min, p_max=p_max,
                   d=d, f_max=f_max, slack=0, net=net)
    return net, prob


def make_scenarios(base: Problem, seed0: int, count: int, load_sigma: float,
                   cost_pm: float = 0.0):
    """Per-instance load and cost scenarios on one network.

    Instance i uses PCG64(seed0 + i): a per-bus load multiplier
    exp(N(0, load_sigma^2)), then (if cost_pm > 0) a per-generator cost
    multiplier U[1 - cost_pm, 1 + cost_pm] applied to c and q.
    Returns (D [count, n_bus], Cc [count, n_gen], Q [count, n_gen]).
    """
    nb, ng = base.n_bus, base.n_gen
    D = np.empty((count, nb))
    Cc = np.empty((count, ng))
    Q = np.empty((count, ng))
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        m = np.exp(rng.normal(0.0, load_sigma, nb))
        D[i] = base.d * m
        if cost_pm > 0:
            u = rng.uniform(1.0 - cost_pm, 1.0 + cost_pm, ng)
        else:
            u = np.ones(ng)
        Cc[i] = base.c * u
        Q[i] = base.q * u
    return D, Cc, Q


def make_problem(name: str, seed: int) -> Problem:
    return make_network(name, seed)[1]


# Step rules frozen per workload (tuned on the oracle).  rule 0 = gradient
# with momentum (heavy-ball reading of Algorithm 1).
STEP_RULES = {
    "tiny30": dict(alpha=1e-4, rho=0.99),
    "geo300": dict(alpha=3e-4, rho=0.99),
    "geo300q": dict(alpha=1e-4, rho=0.99),
    "bus2000": dict(alpha=3e-4, rho=0.99),
    "bus4600": dict(alpha=3e-5, rho=0.99),
    "bus10000": dict(alpha=1e-4, rho=0.99),
}
STEP_RULES.update({n + "_raw": STEP_RULES[n] for n in ("bus2000", "bus4600")})


def config_problem(name: str) -> Problem:
    """Headline instance of each workload (fixed seeds)."""
    seeds = {"tiny30": 1, "bus2000": 2000, "bus4600": 4600, "bus10000": 10000}
    return make_problem(name, seeds[name])
