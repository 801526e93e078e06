"""FP64 oracle: the Lagrange dual of DCOPF and projected (sub)gradient ascent.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Notation follows the paper's canonical problem (Section 2.1, eq. general):

    min_x  x^T M x + c^T x   s.t.  A x - b = 0 : lambda,  C x - d <= 0 : mu,
    with x in the generator box [p_min, p_max].

For DCOPF (Section 2, eq. DCOPF) with n_g generators, n_l lines and the PTDF
H_a (zero slack column):

    A = -1^T (1 x n_g),  b = -1^T p_d        (power balance)
    C = [ H_a C_g ; -H_a C_g ]  (2 n_l x n_g)
    d = [ f_max + H_a p_d ; f_max - H_a p_d ]  (line limits, both directions)
    M = diag(q).

The sign of A is free in the canonical form; taking A = -1^T makes lambda the
marginal price (the reduced cost is c - lambda 1 + (H_a C_g)^T (mu+ - mu-)).
mu is stored as (mu_plus, mu_minus), the multipliers of the two halves of C.

The Lagrangian (eq. lagrangian) is minimised over the box generator by
generator.  For M = 0 this is the dual-norm step of Section 3.1 (eq. LP
dual); for M > 0 it is the closed-form maximum over s of the final QP dual
(Section 3.2, eq. QP_finalgamma), see ``g_q_paper``.  The paper's own
normalised formulas (Appendix A1, A2) are implemented separately in
``g_l_paper`` and ``g_q_paper`` and tested against ``dual_value``.
"""
from __future__ import annotations

import dataclasses

import numpy as np


# ---------------------------------------------------------------------------
# Canonical data (Section 2.1, eq. general)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Canonical:
    c: np.ndarray      # [n]     linear cost
    M: np.ndarray      # [n]     diagonal of M
    A: np.ndarray      # [1, n]
    b: np.ndarray      # [1]
    C: np.ndarray      # [2 n_l, n]
    d: np.ndarray      # [2 n_l]
    lo: np.ndarray     # [n]
    hi: np.ndarray     # [n]

    @property
    def n_line(self) -> int:
        return self.C.shape[0] // 2


def canonical(prob) -> Canonical:
    """Build eq. general from the DCOPF data (Section 2, 2.1)."""
    H = np.asarray(prob.H, dtype=np.float64)
    n_b = H.shape[1]
    n_g = len(prob.gen_bus)
    Cg = np.zeros((n_b, n_g))
    Cg[np.asarray(prob.gen_bus), np.arange(n_g)] = 1.0
    HCg = H @ Cg
    Hd = H @ prob.d
    C = np.vstack([HCg, -HCg])
    d = np.concatenate([prob.f_max + Hd, prob.f_max - Hd])
    A = -np.ones((1, n_g))
    b = np.array([-np.sum(prob.d)])
    return Canonical(c=np.asarray(prob.c, float).copy(), M=np.asarray(prob.q, float).copy(),
                     A=A, b=b, C=C, d=d,
                     lo=np.asarray(prob.p_min, float).copy(),
                     hi=np.asarray(prob.p_max, float).copy())


# ---------------------------------------------------------------------------
# Inner minimisation (Section 3.1 dual norm; Section 3.2 quadratic case)
# ---------------------------------------------------------------------------
def inner_argmin(a, M, lo, hi):
    """argmin over lo <= x <= hi of  M_j x_j^2 + a_j x_j, per coordinate.

    M_j = 0: a linear function on an interval is minimised at an endpoint:
    lo where a > 0, hi where a < 0 (the sign rule of Algorithm 1); at a = 0
    every point is a minimiser and the midpoint is returned.
    M_j > 0: the unconstrained minimiser -a/(2M) clipped to the interval.
    """
    a = np.asarray(a, dtype=np.float64)
    x = np.empty_like(a)
    lin = M == 0
    x[lin] = np.where(a[lin] > 0, lo[lin],
                      np.where(a[lin] < 0, hi[lin], 0.5 * (lo[lin] + hi[lin])))
    qd = ~lin
    x[qd] = np.clip(-a[qd] / (2.0 * M[qd]), lo[qd], hi[qd])
    return x


@dataclasses.dataclass
class DualEval:
    g: float               # dual value G(lambda, mu)
    x: np.ndarray          # inner minimiser (generator outputs p*)
    a: np.ndarray          # reduced cost c + A^T lambda + C^T mu
    grad_lam: float        # A x* - b   (= 1^T p_d - 1^T p*)
    grad_mu: np.ndarray    # C x* - d   (2 n_l: [F - f_max ; -F - f_max])


def dual_value(K: Canonical, lam: float, mu: np.ndarray) -> DualEval:
    """G(lambda, mu) = min_box L(x, lambda, mu) (eqs. lagrangian, dual function).

    ``mu`` is the stacked [mu_plus; mu_minus] (length 2 n_l), mu >= 0.
    The returned gradient is the constraint residual at the minimiser, a
    supergradient of the concave dual (Danskin).
    """
    lam_v = np.array([lam], dtype=np.float64)
    a = K.c + K.A.T @ lam_v + K.C.T @ mu
    x = inner_argmin(a, K.M, K.lo, K.hi)
    g = float(x @ (K.M * x) + a @ x - lam_v @ K.b - mu @ K.d)
    grad_lam = float((K.A @ x - K.b)[0])
    grad_mu = K.C @ x - K.d
    return DualEval(g=g, x=x, a=a, grad_lam=grad_lam, grad_mu=grad_mu)


def dual_value_at(K: Canonical, lam: float, mu: np.ndarray, x: np.ndarray) -> DualEval:
    """The Lagrangian (eq. lagrangian) and the constraint residuals at a given
    point x of the box, in the form of ``dual_value``.  At any minimiser x of
    the Lagrangian over the box this is G(lambda, mu) with a supergradient:
    where a linear unit's reduced cost is zero every point of its interval is
    a minimiser, and each choice gives another valid supergradient."""
    x = np.asarray(x, dtype=np.float64)
    lam_v = np.array([lam], dtype=np.float64)
    a = K.c + K.A.T @ lam_v + K.C.T @ mu
    g = float(x @ (K.M * x) + a @ x - lam_v @ K.b - mu @ K.d)
    return DualEval(g=g, x=x, a=a, grad_lam=float((K.A @ x - K.b)[0]), grad_mu=K.C @ x - K.d)


def split_mu(mu):
    n = mu.shape[0] // 2
    return mu[:n], mu[n:]


# ---------------------------------------------------------------------------
# The paper's normalised forms (Appendix A1 normalisation, A2 dual norm)
# ---------------------------------------------------------------------------
def normalise(K: Canonical):
    """x = M_sigma x~ + m_mu (Appendix A1).  Returns the data of the problem in
    x~ over the unit infinity ball plus the constant that the substitution
    moves out of the objective."""
    m = 0.5 * (K.hi + K.lo)
    s = 0.5 * (K.hi - K.lo)
    # x^T M x + c^T x = x~^T (S M S) x~ + (S c + 2 S M m)^T x~ + (c^T m + m^T M m)
    Mt = s * K.M * s
    ct = s * K.c + 2.0 * s * K.M * m
    const = float(K.c @ m + m @ (K.M * m))
    At = K.A * s[None, :]
    bt = K.b - K.A @ m
    Ct = K.C * s[None, :]
    dt = K.d - K.C @ m
    return dict(M=Mt, c=ct, A=At, b=bt, C=Ct, d=dt, const=const)


def g_l_paper(K: Canonical, lam: float, mu: np.ndarray) -> float:
    """Eq. (LP dual): -||c + lambda^T A + mu^T C||_1 - lambda^T b - mu^T d on the
    normalised data, plus the constant dropped by the normalisation."""
    N = normalise(K)
    lam_v = np.array([lam])
    y = N["c"] + N["A"].T @ lam_v + N["C"].T @ mu
    return float(-np.sum(np.abs(y)) - lam_v @ N["b"] - mu @ N["d"] + N["const"])


def g_q_paper(K: Canonical, lam: float, mu: np.ndarray, s: np.ndarray) -> float:
    """Eq. (QP_finalgamma) with free s on the normalised data:
    -||c + lambda^T A + mu^T C - s^T sqrt(M)||_1 - 0.25 s^T s - lambda^T b - mu^T d
    (+ the normalisation constant)."""
    N = normalise(K)
    lam_v = np.array([lam])
    y = N["c"] + N["A"].T @ lam_v + N["C"].T @ mu - np.sqrt(N["M"]) * s
    return float(-np.sum(np.abs(y)) - 0.25 * s @ s - lam_v @ N["b"] - mu @ N["d"]
                 + N["const"])


def s_star(K: Canonical, lam: float, mu: np.ndarray) -> np.ndarray:
    """Maximiser of g_q_paper over s: s* = -2 sqrt(M~) x~* (normalised units)."""
    N = normalise(K)
    lam_v = np.array([lam])
    a = N["c"] + N["A"].T @ lam_v + N["C"].T @ mu
    ones = np.ones_like(a)
    xt = inner_argmin(a, N["M"], -ones, ones)
    return -2.0 * np.sqrt(N["M"]) * xt


# ---------------------------------------------------------------------------
# Ascent (Section 3.3): Algorithm 1 (gradient with momentum), Adam, AdaGrad
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class AscentState:
    lam: float
    mu: np.ndarray         # [2 n_l] stacked (mu_plus, mu_minus)
    v_lam: float = 0.0
    v_mu: np.ndarray = None
    # Adam / AdaGrad moments (first and second), and the step counter
    m_lam: float = 0.0
    m_mu: np.ndarray = None
    s_lam: float = 0.0
    s_mu: np.ndarray = None
    t: int = 0

    @staticmethod
    def cold(n_line: int) -> "AscentState":
        z = np.zeros(2 * n_line)
        return AscentState(lam=0.0, mu=z.copy(), v_mu=z.copy(), m_mu=z.copy(),
                           s_mu=z.copy())

    def copy(self) -> "AscentState":
        return AscentState(self.lam, self.mu.copy(), self.v_lam, self.v_mu.copy(),
                           self.m_lam, self.m_mu.copy(), self.s_lam, self.s_mu.copy(),
                           self.t)


def gdm_update(st: AscentState, ev: DualEval, alpha: float, rho: float,
               literal: bool = False) -> AscentState:
    """One update of Algorithm 1 from the gradients in ``ev``.

    Heavy-ball reading: v <- rho v + alpha grad; theta <- theta + v.
    ``literal=True`` also applies the separately listed gradient update
    theta <- theta + alpha grad before the projection.  Finally mu <- max(mu, 0).
    """
    n = st.copy()
    n.v_lam = rho * st.v_lam + alpha * ev.grad_lam
    n.v_mu = rho * st.v_mu + alpha * ev.grad_mu
    n.lam = st.lam + n.v_lam
    n.mu = st.mu + n.v_mu
    if literal:
        n.lam = n.lam + alpha * ev.grad_lam
        n.mu = n.mu + alpha * ev.grad_mu
    n.mu = np.maximum(n.mu, 0.0)
    n.t = st.t + 1
    return n


def adam_update(st: AscentState, ev: DualEval, alpha: float, beta1: float,
                beta2: float, eps: float = 1e-8) -> AscentState:
    """Adam (Kingma and Ba) applied as ascent, with bias correction, then the
    projection mu <- max(mu, 0)."""
    n = st.copy()
    n.t = st.t + 1
    n.m_lam = beta1 * st.m_lam + (1 - beta1) * ev.grad_lam
    n.m_mu = beta1 * st.m_mu + (1 - beta1) * ev.grad_mu
    n.s_lam = beta2 * st.s_lam + (1 - beta2) * ev.grad_lam ** 2
    n.s_mu = beta2 * st.s_mu + (1 - beta2) * ev.grad_mu ** 2
    c1 = 1 - beta1 ** n.t
    c2 = 1 - beta2 ** n.t
    n.lam = st.lam + alpha * (n.m_lam / c1) / (np.sqrt(n.s_lam / c2) + eps)
    n.mu = st.mu + alpha * (n.m_mu / c1) / (np.sqrt(n.s_mu / c2) + eps)
    n.mu = np.maximum(n.mu, 0.0)
    return n


def adagrad_update(st: AscentState, ev: DualEval, alpha: float,
                   eps: float = 1e-8) -> AscentState:
    """AdaGrad (Duchi et al.) applied as ascent, then mu <- max(mu, 0)."""
    n = st.copy()
    n.t = st.t + 1
    n.s_lam = st.s_lam + ev.grad_lam ** 2
    n.s_mu = st.s_mu + ev.grad_mu ** 2
    n.lam = st.lam + alpha * ev.grad_lam / (np.sqrt(n.s_lam) + eps)
    n.mu = st.mu + alpha * ev.grad_mu / (np.sqrt(n.s_mu) + eps)
    n.mu = np.maximum(n.mu, 0.0)
    return n


@dataclasses.dataclass
class AscentResult:
    state: AscentState
    gammas: np.ndarray     # gamma_k = G at the k-th iterate (k = 0 is the start)
    best: float            # max_k gamma_k: the best valid lower bound
    best_iter: int
    iters: int             # updates performed
    stopped: bool          # True when |gamma_{k} - gamma_{k-1}| < tol fired
    x_sum: np.ndarray | None = None  # sum of the inner minimisers p*_k, k >= average_from
    n_avg: int = 0                   # number of terms in x_sum


def step_size(alpha: float, decay: float, t: int) -> float:
    """Step size of the update that follows t earlier updates.  The paper
    names step decay among the options of its ascent (Section 3.3) and uses
    it in its experiments (Section 4) without giving the schedule; the
    reading here is alpha_t = alpha / (1 + decay t), so decay = 0 is the
    constant step of Algorithm 1."""
    return alpha / (1.0 + decay * t)


def ascent(K: Canonical, n_iters: int, rule: str = "gdm", alpha: float = 1e-3,
           rho: float = 0.9, beta1: float = 0.9, beta2: float = 0.999,
           eps: float = 1e-8, literal: bool = False, tol: float = 0.0,
           state: AscentState | None = None,
           average_from: int | None = None, decay: float = 0.0) -> AscentResult:
    """Projected dual ascent (Section 3.3, Algorithm 1) for ``n_iters`` updates.

    Iteration k evaluates the dual and its supergradient at the current
    iterate (gamma_k), then updates with the step size
    ``step_size(alpha, decay, t)``, t being the number of updates the state
    has taken (its counter, which a given ``state`` carries).  With tol > 0
    the loop stops when |gamma_k - gamma_{k-1}| < tol (the stopping test of
    Algorithm 1).  With average_from = k0 the inner minimisers p*_k of the
    iterations k0 <= k < n_iters are summed (primal recovery,
    ``primal_eval``).
    """
    st = AscentState.cold(K.n_line) if state is None else state.copy()
    gam = []
    stopped = False
    it = 0
    x_sum = np.zeros_like(K.c) if average_from is not None else None
    n_avg = 0
    for k in range(n_iters):
        ev = dual_value(K, st.lam, st.mu)
        gam.append(ev.g)
        if average_from is not None and k >= average_from:
            x_sum += ev.x
            n_avg += 1
        if tol > 0 and k > 0 and abs(gam[-1] - gam[-2]) < tol:
            stopped = True
            break
        a_t = step_size(alpha, decay, st.t)
        if rule == "gdm":
            st = gdm_update(st, ev, a_t, rho, literal)
        elif rule == "adam":
            st = adam_update(st, ev, a_t, beta1, beta2, eps)
        elif rule == "adagrad":
            st = adagrad_update(st, ev, a_t, eps)
        else:
            raise ValueError(rule)
        it += 1
    gam = np.array(gam)
    kb = int(np.argmax(gam))
    return AscentResult(state=st, gammas=gam, best=float(gam[kb]), best_iter=kb,
                        iters=it, stopped=stopped, x_sum=x_sum, n_avg=n_avg)


# ---------------------------------------------------------------------------
# Primal recovery by ergodic averaging.  Not in the paper (which compares its
# lower bounds with solver optima): the average of the inner minimisers over
# a window of iterations is a primal candidate whose constraint residuals,
# the constraints being affine, are the averages of the supergradients; for
# (sub)gradient ascent they vanish as the window grows, and its cost then
# approaches the optimum from the other side of the lower bound.
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class PrimalEval:
    x: np.ndarray            # candidate generator outputs
    cost: float              # c^T x + x^T M x
    balance: float           # 1^T d - 1^T x  (= A x - b)
    overload: np.ndarray     # (C x - d)_+ per row: [F - f_max ; -F - f_max]_+
    max_overload: float
    sum_overload: float
    n_overloaded: int


def primal_eval(K: Canonical, x: np.ndarray) -> PrimalEval:
    """Cost and constraint residuals of a primal candidate x in the box."""
    x = np.asarray(x, dtype=np.float64)
    ov = np.maximum(K.C @ x - K.d, 0.0)
    return PrimalEval(x=x, cost=float(K.c @ x + x @ (K.M * x)),
                      balance=float((K.A @ x - K.b)[0]), overload=ov,
                      max_overload=float(ov.max()) if ov.size else 0.0,
                      sum_overload=float(ov.sum()), n_overloaded=int(np.count_nonzero(ov)))


def averaged_primal(res: AscentResult) -> np.ndarray:
    """The ergodic average of an ascent run with ``average_from`` set."""
    if res.x_sum is None or res.n_avg == 0:
        raise ValueError("no iterations averaged")
    return res.x_sum / res.n_avg
