"""FP64 oracle: repair of a primal candidate into a feasible dispatch.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not in the paper, whose lower bounds are compared with solver optima.  A
feasible dispatch p gives an upper bound c^T p + p^T M p >= OPT, so together
with the dual's exact lower bound it certifies the gap without an external
solver.  The candidate (for instance the ergodic average of the inner
minimisers) is nearly feasible; the repair moves it the least, in a norm
weighted by each generator's headroom, onto the constraints it violates.

Constraints of the canonical problem (Section 2.1, eq. general) with
A = -1^T and C = [H_a C_g; -H_a C_g]: the balance 1^T x = 1^T p_d, the line
rows C x <= d, and the box.  One round:

  1. residuals: r = C x - d per row, beta = 1^T p_d - 1^T x;
  2. every violated row (r > 0, at most one direction per line) joins the
     active set, in line order, keeping its direction; a line already held
     in the other direction switches to this one;
  3. stop when no row is violated and |beta| <= 1e-9 max(1, 1^T p_d);
  4. weights w_g = max(min(x_g - p_min_g, p_max_g - x_g), 1e-3 (p_max_g -
     p_min_g)): the headroom, floored so that a generator at a bound can
     still move inward (a move outward is undone by the clip of step 6);
  5. rows a_i = (H_a C_g)[l_i, :] of the active lines with targets
     t_i = -(delta + r_i) in flow units (the flow change that leaves the row
     delta inside its limit), and the balance row a = 1 with target beta;
  6. the active lines are inequalities (the flow may end anywhere inside
     limit - delta) and the balance an equality.  Working set S: start with
     every active line; y solves (A_S W A_S^T + eps I) y = t_S over S and the
     balance row (eps = 1e-12 of that matrix's largest diagonal).  Then, in
     this order: if a working line has a multiplier with sigma_i y_i > 0
     (holding it at its target pushes its flow out: as an inequality it is
     slack), the one with the largest sigma_i y_i leaves S; otherwise, if a
     line outside S would end more than delta / 2 past its target under the
     step (sigma_i ((G y)_i - t_i), G the Gram matrix of all active rows),
     the one ending furthest joins S again; otherwise S is final.  Ties go to
     the first in active-set order; at most 4 (m + 1) + 8 solves;
  7. x <- clip(x + W A^T y, p_min, p_max) with y zero outside S.

Before the clip, the step is the least sum_g dx_g^2 / w_g move that closes
the balance and brings every active line inside its limit less delta, the
binding lines being found by the primal-dual active-set rule of step 6.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle.dual import Canonical, primal_eval

MARGIN = 1e-6          # MW inside each held limit
BALANCE_TOL = 1e-9     # relative to max(1, total load)
MAX_ROWS = 256         # active lines + the balance row
WEIGHT_FLOOR = 1e-3    # of each generator's range


@dataclasses.dataclass
class RepairResult:
    x: np.ndarray
    feasible: bool
    rounds: int            # correction steps taken
    active: list           # [(line, direction)] in the order they joined
    cost: float
    balance: float
    max_overload: float
    max_shift: float


def repair(K: Canonical, x0: np.ndarray, max_rounds: int = 32) -> RepairResult:
    nl = K.n_line
    D = -float(K.b[0])
    tol = BALANCE_TOL * max(1.0, abs(D))
    lo, hi = K.lo, K.hi
    x = np.clip(np.asarray(x0, dtype=np.float64), lo, hi)
    HC = K.C[:nl]
    active: dict[int, int] = {}     # line -> direction (+1 / -1), insertion ordered
    rounds = 0
    feasible = False
    while True:
        r = K.C @ x - K.d
        beta = float(K.A[0] @ x - K.b[0])       # 1^T p_d - 1^T x
        viol = False
        for line in range(nl):
            if r[line] > 0.0:
                active[line] = 1
                viol = True
            elif r[nl + line] > 0.0:
                active[line] = -1
                viol = True
        if not viol and abs(beta) <= tol:
            feasible = True
            break
        if rounds >= max_rounds or len(active) + 1 > MAX_ROWS:
            break
        w = np.maximum(np.minimum(x - lo, hi - x), WEIGHT_FLOOR * (hi - lo))
        lines = list(active.keys())
        Am = np.vstack([HC[lines], np.ones((1, x.size))])
        t = np.empty(len(lines) + 1)
        for i, line in enumerate(lines):
            # flow change that leaves the row MARGIN inside: direction +1 wants
            # r+ = -MARGIN (dF = -MARGIN - r+); direction -1 wants r- = -MARGIN
            # (dF = MARGIN + r-)
            t[i] = (-MARGIN - r[line]) if active[line] > 0 else (MARGIN + r[nl + line])
        t[-1] = beta
        G = (Am * w) @ Am.T
        sig = np.array([active[line] for line in lines], dtype=float)
        nrow = len(lines)
        work = list(range(nrow))
        cap = 4 * (nrow + 1) + 8
        for _ in range(cap):
            S = work + [nrow]
            Gs = G[np.ix_(S, S)]
            dmax = float(np.max(np.diag(Gs)))
            if not dmax > 0.0:
                break
            Gs = Gs + 1e-12 * dmax * np.eye(len(S))
            L = np.linalg.cholesky(Gs)
            ys = np.linalg.solve(L.T, np.linalg.solve(L, t[S]))
            y = np.zeros(nrow + 1)
            y[S] = ys
            worst, kw = 0.0, -1
            for k, i in enumerate(work):
                if sig[i] * ys[k] > worst:
                    worst, kw = sig[i] * ys[k], i
            if kw >= 0:
                work.remove(kw)
                continue
            Gy = G @ y
            worst, ka = 0.5 * MARGIN, -1
            for i in range(nrow):
                if i not in work and sig[i] * (Gy[i] - t[i]) > worst:
                    worst, ka = sig[i] * (Gy[i] - t[i]), i
            if ka >= 0:
                work = sorted(work + [ka])
                continue
            break
        if not dmax > 0.0:
            break
        x = np.clip(x + w * (Am.T @ y), lo, hi)
        rounds += 1
    pe = primal_eval(K, x)
    return RepairResult(x=x, feasible=feasible, rounds=rounds,
                        active=[(k, v) for k, v in active.items()], cost=pe.cost,
                        balance=pe.balance, max_overload=pe.max_overload,
                        max_shift=float(np.max(np.abs(x - np.clip(x0, lo, hi)))) if x.size else 0.0)
