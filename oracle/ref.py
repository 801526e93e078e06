"""References that pin the FP64 oracle (TEST INFRASTRUCTURE ONLY).

* ``lp_vertex_enum``   - LP optimum of eq. general by enumerating basic
  solutions (textbook: a bounded feasible LP attains its optimum at a vertex).
* ``qp_kkt_enum``      - QP optimum by enumerating active sets and solving the
  KKT system (strictly convex QP: the KKT point is the unique optimum).
* ``econ_dispatch``    - DCOPF with no binding line is economic dispatch:
  merit order (LP) or equal incremental cost by bisection (QP).
* ``opt_ptdf``         - HiGHS on eq. DCOPF in PTDF form (dense), with its
  constraint duals converted to this oracle's (lambda, mu+, mu-).
* ``opt_btheta``       - HiGHS on the bus-angle form of DC power flow
  (B theta = C_g p - p_d, flows b (theta_f - theta_t)), which never forms the
  PTDF: an independent route to the same optimum.
* ``qp_certificate``   - QP: a dual lower bound from L-BFGS-B on the (smooth)
  dual function and a primal upper bound from the LP projection of p* onto
  the feasible set.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize as so
import scipy.sparse as sp

from . import dual as D


# ---------------------------------------------------------------------------
# constraint stacking shared by the brute-force references
# ---------------------------------------------------------------------------
def _ineq_rows(K: D.Canonical, drop_lines=None):
    """Inequalities G x <= h: line rows C x <= d plus the box."""
    n = K.c.size
    C, d = K.C, K.d
    if drop_lines is not None:
        nl = K.n_line
        keep = np.ones(2 * nl, bool)
        keep[np.asarray(drop_lines)] = False
        keep[nl + np.asarray(drop_lines)] = False
        C, d = C[keep], d[keep]
    G = np.vstack([C, np.eye(n), -np.eye(n)])
    h = np.concatenate([d, K.hi, -K.lo])
    return G, h


def lp_vertex_enum(K: D.Canonical, drop_lines=None, tol=1e-9):
    """min c^T x over {A x = b, G x <= h} by enumerating every choice of n - 1
    inequality rows made active together with the equality row."""
    n = K.c.size
    G, h = _ineq_rows(K, drop_lines)
    best, best_x = np.inf, None
    scale = 1.0 + np.abs(h).max()
    for S in itertools.combinations(range(G.shape[0]), n - 1):
        Mx = np.vstack([K.A, G[list(S)]])
        if abs(np.linalg.det(Mx)) < 1e-12:
            continue
        x = np.linalg.solve(Mx, np.concatenate([K.b, h[list(S)]]))
        if np.all(G @ x <= h + tol * scale):
            val = float(K.c @ x)
            if val < best:
                best, best_x = val, x
    return best, best_x


def qp_kkt_enum(K: D.Canonical, max_active=None, tol=1e-9):
    """min x^T M x + c^T x over {A x = b, G x <= h}, M > 0 diagonal, by
    solving the KKT system for every active set of size <= max_active and
    keeping primal-feasible points with nonnegative multipliers."""
    n = K.c.size
    G, h = _ineq_rows(K)
    m = G.shape[0]
    max_active = n if max_active is None else max_active
    best, best_x = np.inf, None
    scale = 1.0 + np.abs(h).max()
    Q2 = np.diag(2.0 * K.M)
    for k in range(0, max_active + 1):
        for S in itertools.combinations(range(m), k):
            GS = G[list(S)]
            top = np.hstack([Q2, K.A.T, GS.T])
            mid = np.hstack([K.A, np.zeros((1, 1 + k))])
            bot = np.hstack([GS, np.zeros((k, 1 + k))])
            KKT = np.vstack([top, mid, bot])
            rhs = np.concatenate([-K.c, K.b, h[list(S)]])
            try:
                sol = np.linalg.solve(KKT, rhs)
            except np.linalg.LinAlgError:
                continue
            if not np.all(np.isfinite(sol)):
                continue
            x, mu = sol[:n], sol[n + 1:]
            if k and np.any(mu < -tol * (1 + np.abs(mu).max())):
                continue
            if np.all(G @ x <= h + tol * scale) and abs((K.A @ x - K.b)[0]) <= tol * scale:
                val = float(x @ (K.M * x) + K.c @ x)
                if val < best:
                    best, best_x = val, x
    return best, best_x


def econ_dispatch(c, q, lo, hi, demand):
    """Economic dispatch (no network): returns (cost, p, marginal price).

    LP: fill units in increasing c; the price is the cost of the marginal
    (partly loaded) unit.  QP: bisection on the price lambda with
    p_g(lambda) = clip((lambda - c_g)/(2 q_g), lo, hi).
    """
    c, q, lo, hi = (np.asarray(v, float) for v in (c, q, lo, hi))
    if not np.any(q > 0):
        order = np.lexsort((np.arange(c.size), c))
        p = lo.copy()
        rest = demand - lo.sum()
        price = None
        for g in order:
            take = min(hi[g] - lo[g], rest)
            p[g] += take
            rest -= take
            if rest <= 1e-12 * max(1.0, demand):
                price = c[g]
                break
        return float(c @ p), p, float(price)
    a, bnd = -1e6, 1e6
    for _ in range(300):
        mid = 0.5 * (a + bnd)
        if np.clip((mid - c) / (2 * q), lo, hi).sum() < demand:
            a = mid
        else:
            bnd = mid
    lam = 0.5 * (a + bnd)
    p = np.clip((lam - c) / (2 * q), lo, hi)
    return float(c @ p + q @ (p * p)), p, float(lam)


def opt_ptdf(prob, want_duals=True):
    """HiGHS on eq. DCOPF (LP) in PTDF form.  Returns dict(opt, p, lam, mu)
    with mu stacked [mu_plus; mu_minus] in this oracle's sign convention."""
    K = D.canonical(prob)
    res = so.linprog(K.c, A_ub=K.C, b_ub=K.d, A_eq=-K.A, b_eq=-K.b,
                     bounds=list(zip(K.lo, K.hi)), method="highs")
    if res.status != 0:
        return dict(opt=None, status=res.status, message=res.message)
    out = dict(opt=float(res.fun), p=res.x, status=0)
    if want_duals:
        # HiGHS marginals are d(opt)/d(rhs).  For C x <= d the Lagrange
        # multiplier is -marginal >= 0.  The equality is passed as 1^T p = D,
        # so its marginal is d(opt)/dD, the price lambda of this oracle.
        out["mu"] = np.maximum(-res.ineqlin.marginals, 0.0)
        out["lam"] = float(res.eqlin.marginals[0])
    return out


def opt_btheta(net, prob):
    """HiGHS on the bus-angle form: variables (p, theta), theta_slack = 0,
    C_g p - B theta = p_d at every bus, |b_l (theta_f - theta_t)| <= f_max."""
    nb, nl, ng = prob.n_bus, prob.n_line, prob.n_gen
    rows = np.arange(nl)
    E = sp.csr_matrix((np.concatenate([np.ones(nl), -np.ones(nl)]),
                       (np.concatenate([rows, rows]),
                        np.concatenate([net.fbus, net.tbus]))), shape=(nl, nb))
    Fm = sp.diags(net.b) @ E                       # flows = Fm theta
    B = (E.T @ Fm).tocsr()                         # nodal susceptance
    Cg = sp.csr_matrix((np.ones(ng), (prob.gen_bus, np.arange(ng))), shape=(nb, ng))
    A_eq = sp.hstack([Cg, -B]).tocsr()
    A_ub = sp.vstack([sp.hstack([sp.csr_matrix((nl, ng)), Fm]),
                      sp.hstack([sp.csr_matrix((nl, ng)), -Fm])]).tocsr()
    b_ub = np.concatenate([prob.f_max, prob.f_max])
    bounds = [(lo, hi) for lo, hi in zip(prob.p_min, prob.p_max)]
    bounds += [(0.0, 0.0) if i == net.slack else (None, None) for i in range(nb)]
    cost = np.concatenate([prob.c, np.zeros(nb)])
    res = so.linprog(cost, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=prob.d,
                     bounds=bounds, method="highs")
    if res.status != 0:
        return dict(opt=None, status=res.status, message=res.message)
    return dict(opt=float(res.fun), p=res.x[:ng], theta=res.x[ng:], status=0)


def feasible_projection(K: D.Canonical, x0):
    """Nearest feasible point in l1: min ||x - x0||_1 s.t. A x = b, C x <= d,
    lo <= x <= hi (an LP in (x, t) with -t <= x - x0 <= t)."""
    n = x0.size
    I = sp.identity(n, format="csr")
    A_ub = sp.vstack([sp.hstack([sp.csr_matrix(K.C), sp.csr_matrix((K.C.shape[0], n))]),
                      sp.hstack([I, -I]), sp.hstack([-I, -I])]).tocsr()
    b_ub = np.concatenate([K.d, x0, -x0])
    A_eq = sp.hstack([sp.csr_matrix(K.A), sp.csr_matrix((1, n))]).tocsr()
    cost = np.concatenate([np.zeros(n), np.ones(n)])
    bounds = list(zip(K.lo, K.hi)) + [(0, None)] * n
    res = so.linprog(cost, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=K.b,
                     bounds=bounds, method="highs")
    if res.status != 0:
        return None
    return res.x[:n]


def qp_certificate(K: D.Canonical, maxiter=20000, x0=None, restarts=50):
    """Bracket the QP optimum (all M > 0): LB = dual value at the L-BFGS-B
    maximiser of the dual over mu >= 0 (a valid bound at any point), UB =
    primal cost of the feasible l1-projection of the inner minimiser.

    Returns dict(lb, ub, lam, mu)."""
    nl2 = K.C.shape[0]

    def f(z):
        ev = D.dual_value(K, z[0], z[1:])
        return -ev.g, -np.concatenate([[ev.grad_lam], ev.grad_mu])

    z = np.zeros(1 + nl2) if x0 is None else np.asarray(x0, float).copy()
    bounds = [(None, None)] + [(0.0, None)] * nl2
    prev = -np.inf
    # L-BFGS-B can stop early on the kinks of the piecewise-quadratic dual;
    # restarting from its own point until the value stops improving fixes it
    for _ in range(restarts):
        r = so.minimize(f, z, jac=True, method="L-BFGS-B", bounds=bounds,
                        options=dict(maxiter=maxiter, maxfun=2 * maxiter, ftol=1e-15,
                                     gtol=1e-10, maxcor=30))
        z = r.x
        if -r.fun - prev <= 1e-14 * abs(r.fun):
            break
        prev = -r.fun
    lam, mu = float(r.x[0]), r.x[1:]
    ev = D.dual_value(K, lam, mu)
    xf = feasible_projection(K, ev.x)
    ub = float(xf @ (K.M * xf) + K.c @ xf) if xf is not None else np.inf
    return dict(lb=ev.g, ub=ub, lam=lam, mu=mu, x=ev.x)
