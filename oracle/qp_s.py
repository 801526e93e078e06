"""FP64 oracle: the paper's QP dual with its auxiliary variables s iterated
(Section 3.2, eq. QP_finalgamma), the ablation of the closed-form maximum
over s that the main path uses.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

With m = (p_min + p_max) / 2 the centre of a unit's box, its quadratic cost
splits as q p^2 = q (p - m)^2 + 2 q m p - q m^2, and the paper bounds
q (p - m)^2 from below by -sqrt(q) s (p - m) - s^2 / 4 for every s (equality
at s = -2 sqrt(q) (p - m)).  For fixed s the Lagrangian is then linear in p,
so the inner minimiser is bang-bang (Algorithm 1's sign rule, midpoint at a
tie) on the shifted reduced cost

    a = r + 2 q m - sqrt(q) s,        r = c + A^T lambda + C^T mu,

and the dual value is

    G_s(lambda, mu, s) = sum_g [a p* - q m^2 + sqrt(q) s m - s^2 / 4]
                         - lambda^T b - mu^T d,

which is eq. QP_finalgamma written out of the normalised variables (the same
s), never above G(lambda, mu) and equal to it at s* = -2 sqrt(q) (x* - m)
with x* the closed-form minimiser.  Its supergradient in s is
-sqrt(q) (p* - m) - s / 2.  Units with q = 0 keep s = 0 (their gradient in
s is then 0).  The ascent applies Algorithm 1 (heavy ball) to
(lambda, mu, s) jointly with one step size.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle.dual import AscentState, Canonical, inner_argmin, gdm_update


@dataclasses.dataclass
class DualEvalS:
    g: float
    x: np.ndarray          # bang-bang minimiser for the given s
    a: np.ndarray          # shifted reduced cost
    grad_lam: float
    grad_mu: np.ndarray
    grad_s: np.ndarray


def dual_value_s(K: Canonical, lam: float, mu: np.ndarray, s: np.ndarray) -> DualEvalS:
    lam_v = np.array([lam], dtype=np.float64)
    m = 0.5 * (K.lo + K.hi)
    sq = np.sqrt(K.M)
    r = K.c + K.A.T @ lam_v + K.C.T @ mu
    a = r + 2.0 * K.M * m - sq * s
    x = inner_argmin(a, np.zeros_like(K.M), K.lo, K.hi)
    g = float(a @ x - np.sum(K.M * m * m) + np.sum(sq * s * m) - 0.25 * s @ s
              - lam_v @ K.b - mu @ K.d)
    return DualEvalS(g=g, x=x, a=a, grad_lam=float((K.A @ x - K.b)[0]),
                     grad_mu=K.C @ x - K.d, grad_s=-sq * (x - m) - 0.5 * s)


@dataclasses.dataclass
class AscentSResult:
    state: AscentState
    s: np.ndarray
    gammas: np.ndarray     # G_s at the k-th iterate
    best: float
    iters: int


def ascent_s(K: Canonical, n_iters: int, alpha: float, rho: float) -> AscentSResult:
    """Algorithm 1 (heavy ball) on (lambda, mu, s), s starting at 0."""
    st = AscentState.cold(K.n_line)
    s = np.zeros_like(K.c)
    v_s = np.zeros_like(K.c)
    gam = []
    for _ in range(n_iters):
        ev = dual_value_s(K, st.lam, st.mu, s)
        gam.append(ev.g)
        st = gdm_update(st, ev, alpha, rho)
        v_s = rho * v_s + alpha * ev.grad_s
        s = s + v_s
    gam = np.array(gam)
    return AscentSResult(state=st, s=s, gammas=gam, best=float(gam.max()), iters=n_iters)
