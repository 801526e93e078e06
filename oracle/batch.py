"""FP64 oracle for many instances on one network: the ascent of
``oracle.dual`` run for every instance at once, with the two products of
each iteration written as FP64 matrix products over the instances.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The instances share the network: the PTDF H_a, the generator buses (C_g),
the generator bounds and the line limits.  Instance i has its own loads d_i
and costs c_i, q_i (Section 2, eq. DCOPF for each instance).  The paper
solves one instance at a time and names many instances in parallel as
future work (Sections 1 and 5); nothing here changes the per-instance
method: column i of every matrix below is instance i's vector of
``oracle.dual``, and the updates are the functions of ``oracle.dual``
applied column-wise.

    C   = [H_a C_g ; -H_a C_g]                (2 n_l x n_g, shared)
    c   = [c_1 ... c_B],  M = [q_1 ... q_B]   (n_g x B)
    b_i = -1^T d_i,  d_i' = [f_max + H_a d_i ; f_max - H_a d_i]
    a   = c - 1 lambda^T + C^T mu             (reduced costs, n_g x B)
    g_i = sum_j (M x^2 + a x)_ji - lambda_i b_i - mu_i^T d_i'
"""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle import dual as D


@dataclasses.dataclass
class CanonicalBatch:
    C: np.ndarray      # [2 n_l, n_g] shared
    c: np.ndarray      # [n_g, B]
    M: np.ndarray      # [n_g, B]
    b: np.ndarray      # [B]
    d: np.ndarray      # [2 n_l, B]
    lo: np.ndarray     # [n_g]
    hi: np.ndarray     # [n_g]

    @property
    def n_line(self) -> int:
        return self.C.shape[0] // 2

    @property
    def n_inst(self) -> int:
        return self.c.shape[1]


def canonical_batch(base, loads, costs, quad=None) -> CanonicalBatch:
    """eq. general for every instance of one network (Section 2, 2.1).
    ``loads`` [B, n_bus], ``costs`` [B, n_gen], ``quad`` [B, n_gen] or None
    (linear costs).  C_g is an index map, so H_a C_g is the gather of H_a's
    generator-bus columns (column g of H_a C_g is column gen_bus[g] of H_a)."""
    H = np.asarray(base.H, dtype=np.float64)
    loads = np.asarray(loads, dtype=np.float64)
    HCg = H[:, np.asarray(base.gen_bus)]
    Hd = H @ loads.T                                   # [n_l, B]
    f = np.asarray(base.f_max, dtype=np.float64)[:, None]
    c = np.ascontiguousarray(np.asarray(costs, dtype=np.float64).T)
    M = np.zeros_like(c) if quad is None else np.ascontiguousarray(
        np.asarray(quad, dtype=np.float64).T)
    return CanonicalBatch(C=np.vstack([HCg, -HCg]), c=c, M=M, b=-loads.sum(axis=1),
                          d=np.vstack([f + Hd, f - Hd]),
                          lo=np.asarray(base.p_min, float).copy(),
                          hi=np.asarray(base.p_max, float).copy())


def instance(KB: CanonicalBatch, i: int) -> D.Canonical:
    """Instance i as the single-instance canonical data of ``oracle.dual``."""
    n_g = KB.C.shape[1]
    return D.Canonical(c=KB.c[:, i].copy(), M=KB.M[:, i].copy(), A=-np.ones((1, n_g)),
                       b=np.array([KB.b[i]]), C=KB.C, d=KB.d[:, i].copy(), lo=KB.lo,
                       hi=KB.hi)


def inner_argmin_batch(a, M, lo, hi):
    """``oracle.dual.inner_argmin`` for every column of a [n_g, B]: p_min
    where the reduced cost of a linear unit is positive, p_max where it is
    negative, the midpoint at zero; the clipped -a / 2M for quadratic units."""
    lo = lo[:, None]
    hi = hi[:, None]
    lin = M == 0
    x_lin = np.where(a > 0, lo, np.where(a < 0, hi, 0.5 * (lo + hi)))
    x_q = np.clip(-a / (2.0 * np.where(lin, 1.0, M)), lo, hi)
    return np.where(lin, x_lin, x_q)


def dual_value_batch(KB: CanonicalBatch, lam: np.ndarray, mu: np.ndarray) -> D.DualEval:
    """G of every instance (eqs. lagrangian, dual function).  ``lam`` [B],
    ``mu`` [2 n_l, B] stacked (mu_plus; mu_minus).  Returns a DualEval whose
    fields hold one column (or entry) per instance: g [B], x, a [n_g, B],
    grad_lam [B] (= 1^T d_i - 1^T p*_i), grad_mu [2 n_l, B]."""
    lam = np.asarray(lam, dtype=np.float64)
    a = KB.c - lam[None, :] + KB.C.T @ mu
    x = inner_argmin_batch(a, KB.M, KB.lo, KB.hi)
    g = np.sum(KB.M * x * x + a * x, axis=0) - lam * KB.b - np.sum(mu * KB.d, axis=0)
    grad_lam = -np.sum(x, axis=0) - KB.b
    grad_mu = KB.C @ x - KB.d
    return D.DualEval(g=g, x=x, a=a, grad_lam=grad_lam, grad_mu=grad_mu)


def cold_batch(KB: CanonicalBatch) -> D.AscentState:
    """Algorithm 1's cold start lambda = mu = 0 for every instance."""
    B, n2 = KB.n_inst, 2 * KB.n_line
    z = np.zeros((n2, B))
    return D.AscentState(lam=np.zeros(B), mu=z.copy(), v_lam=np.zeros(B), v_mu=z.copy(),
                         m_lam=np.zeros(B), m_mu=z.copy(), s_lam=np.zeros(B),
                         s_mu=z.copy(), t=0)


@dataclasses.dataclass
class BatchResult:
    state: D.AscentState   # fields hold one column (entry) per instance
    gammas: np.ndarray     # [n_iters, B]: G at the k-th iterate of each instance
    iters: int


def ascent_batch(KB: CanonicalBatch, n_iters: int, rule: str = "gdm", alpha=1e-3,
                 rho=0.9, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                 literal: bool = False, decay: float = 0.0,
                 state: D.AscentState | None = None) -> BatchResult:
    """``oracle.dual.ascent`` for every instance at once: iteration k records
    G at the current iterate, then applies the rule's update of
    ``oracle.dual`` (gdm_update, adam_update, adagrad_update) with the step
    ``oracle.dual.step_size(alpha, decay, t)``.  ``alpha`` and ``rho`` may
    be scalars or one value per instance."""
    st = cold_batch(KB) if state is None else state.copy()
    alpha = np.asarray(alpha, dtype=np.float64)
    gam = np.empty((n_iters, KB.n_inst))
    for k in range(n_iters):
        ev = dual_value_batch(KB, st.lam, st.mu)
        gam[k] = ev.g
        a_t = D.step_size(alpha, decay, st.t)
        if rule == "gdm":
            st = D.gdm_update(st, ev, a_t, rho, literal)
        elif rule == "adam":
            st = D.adam_update(st, ev, a_t, beta1, beta2, eps)
        elif rule == "adagrad":
            st = D.adagrad_update(st, ev, a_t, eps)
        else:
            raise ValueError(rule)
    return BatchResult(state=st, gammas=gam, iters=n_iters)
