"""Pins of the oracle's ascent rules (Section 3.3, Algorithm 1; Adam and
AdaGrad).  The paper prints no trajectory, so the ascent is pinned by step
identities, textbook properties of each rule, weak duality along the path and
convergence to the HiGHS optimum."""
import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from paper_2406_13191_amd import synth


def test_tiny30_converges_to_highs_optimum():
    net, p = synth.make_network("tiny30", 1)
    K = D.canonical(p)
    opt = ref.opt_btheta(net, p)["opt"]
    r = synth.STEP_RULES["tiny30"]
    res = D.ascent(K, 5000, alpha=r["alpha"], rho=r["rho"])
    # weak duality along the whole trajectory, and a 0.1 % bound at the end
    assert np.all(res.gammas <= opt + 1e-9 * opt)
    assert (opt - res.best) <= 1e-3 * opt
    # the cold start (lambda = mu = 0) value is the cost of every unit at p_min
    assert res.gammas[0] == pytest.approx(float(K.c @ K.lo))


def test_heavy_ball_literal_identity():
    # with rho = 0 the literal reading of Algorithm 1 (velocity update, then
    # gradient update) is the heavy-ball step with twice the step size
    p = synth.make_problem("tiny30", 1)
    K = D.canonical(p)
    a = D.ascent(K, 50, alpha=1e-4, rho=0.0, literal=True)
    b = D.ascent(K, 50, alpha=2e-4, rho=0.0, literal=False)
    np.testing.assert_allclose(a.gammas, b.gammas, rtol=1e-12)
    np.testing.assert_allclose(a.state.mu, b.state.mu, rtol=1e-12, atol=1e-12)


def test_qp_small_step_is_monotone():
    # the QP dual is smooth; a small enough plain step never decreases it
    net, p = synth.make_network("geo300q", 7)
    K = D.canonical(p)
    res = D.ascent(K, 200, alpha=1e-4, rho=0.0)
    assert np.all(np.diff(res.gammas) >= -1e-9 * np.abs(res.gammas[1:]))
    assert res.gammas[-1] > res.gammas[0]


@pytest.mark.parametrize("rule", ["adam", "adagrad"])
def test_adaptive_first_step_is_signed_alpha(rule):
    # with bias correction, Adam's first step moves every coordinate by alpha
    # times the sign of its gradient; so does AdaGrad's (g / sqrt(g^2))
    p = synth.make_problem("tiny30", 1)
    K = D.canonical(p)
    st0 = D.AscentState.cold(K.n_line)
    ev = D.dual_value(K, st0.lam, st0.mu)
    alpha = 0.5
    if rule == "adam":
        st1 = D.adam_update(st0, ev, alpha, 0.9, 0.999, eps=1e-12)
    else:
        st1 = D.adagrad_update(st0, ev, alpha, eps=1e-12)
    assert st1.lam == pytest.approx(alpha * np.sign(ev.grad_lam), rel=1e-9)
    expect = np.maximum(alpha * np.sign(ev.grad_mu), 0.0)
    np.testing.assert_allclose(st1.mu, expect, rtol=1e-9, atol=1e-12)


def test_stopping_rule():
    p = synth.make_problem("tiny30", 1)
    K = D.canonical(p)
    full = D.ascent(K, 3000, alpha=1e-4, rho=0.99)
    tol = 1e-3
    stop = D.ascent(K, 3000, alpha=1e-4, rho=0.99, tol=tol)
    dg = np.abs(np.diff(full.gammas))
    first = int(np.argmax(dg < tol)) + 1
    assert stop.stopped and len(stop.gammas) == first + 1


# ---------------------------------------------------------------------------
# Adaptive rules beyond the first step, and step decay.  Each value below is
# worked out by hand from the rule's definition (Kingma-Ba Adam with bias
# correction; AdaGrad with accumulated squares), so a wrong moment recursion,
# bias correction or step counter fails at t = 2 or 3 even where t = 1 agrees.
# ---------------------------------------------------------------------------
def _ev(g_lam, g_mu):
    """A DualEval carrying only the supergradient the updates read."""
    g_mu = np.asarray(g_mu, dtype=float)
    return D.DualEval(g=0.0, x=np.zeros(1), a=np.zeros(1), grad_lam=float(g_lam),
                      grad_mu=g_mu)


def _state(n_line, mu0=10.0):
    st = D.AscentState.cold(n_line)
    st.mu = np.full(2 * n_line, mu0)   # far from the projection
    return st


def test_adam_hand_worked_three_steps():
    # alpha = 1, beta1 = 1/2, beta2 = 3/4, eps = 0; gradients 2, -3, 1/2.
    # t=1: m = 1, s = 1; m^ = 2, s^ = 4 -> step 2/2 = 1
    # t=2: m = 1/2 - 3/2 = -1, s = 3/4 + 9/4 = 3; m^ = -1/(3/4) = -4/3,
    #      s^ = 3/(7/16) = 48/7 -> step (-4/3)/sqrt(48/7) = -sqrt(21)/9
    # t=3: m = -1/2 + 1/4 = -1/4, s = 9/4 + 1/16 = 37/16; m^ = (-1/4)/(7/8)
    #      = -2/7, s^ = (37/16)/(37/64) = 4 -> step (-2/7)/2 = -1/7
    expect = [1.0, 1.0 - np.sqrt(21) / 9, 1.0 - np.sqrt(21) / 9 - 1.0 / 7]
    st = _state(1)
    for t, g in enumerate([2.0, -3.0, 0.5]):
        st = D.adam_update(st, _ev(g, [g, -g]), 1.0, 0.5, 0.75, eps=0.0)
        assert st.t == t + 1
        assert st.lam == pytest.approx(expect[t], rel=1e-14, abs=1e-14)
        np.testing.assert_allclose(st.mu, [10.0 + expect[t], 10.0 - expect[t]], rtol=1e-14)


def test_adagrad_hand_worked_three_steps():
    # alpha = 1, eps = 0; gradients 2, -3, 1/2: accumulated squares 4, 13,
    # 53/4, steps 2/2 = 1, -3/sqrt(13), (1/2)/sqrt(53/4) = 1/sqrt(53)
    expect = np.cumsum([1.0, -3.0 / np.sqrt(13.0), 1.0 / np.sqrt(53.0)])
    st = _state(1)
    for t, g in enumerate([2.0, -3.0, 0.5]):
        st = D.adagrad_update(st, _ev(g, [g, -g]), 1.0, eps=0.0)
        assert st.lam == pytest.approx(expect[t], rel=1e-14)
        np.testing.assert_allclose(st.mu, [10.0 + expect[t], 10.0 - expect[t]], rtol=1e-14)


@pytest.mark.parametrize("rule", ["adam", "adagrad"])
def test_adaptive_constant_gradient_closed_form(rule):
    # a constant gradient g: Adam's bias-corrected moments are exactly g and
    # g^2, so every step is alpha g / (|g| + eps); AdaGrad's t-th step is
    # alpha g / (sqrt(t) |g| + eps)
    g, alpha, eps = -0.75, 0.3, 1e-3
    st = _state(2)
    pos = 0.0
    for t in range(1, 7):
        if rule == "adam":
            st = D.adam_update(st, _ev(g, np.full(4, g)), alpha, 0.9, 0.999, eps=eps)
            pos += alpha * g / (abs(g) + eps)
        else:
            st = D.adagrad_update(st, _ev(g, np.full(4, g)), alpha, eps=eps)
            pos += alpha * g / (np.sqrt(t) * abs(g) + eps)
        assert st.lam == pytest.approx(pos, rel=1e-12)
        np.testing.assert_allclose(st.mu, 10.0 + pos, rtol=1e-12)


def _one_unit_two_buses(c=40.0, p_max=10.0, load=4.0):
    """Two buses, one line with a limit no dispatch can reach (its multipliers
    stay at zero), one linear unit on bus 1 and the load on bus 0 (the slack).
    While lambda < c the unit sits at p_min = 0, so the balance residual, the
    lambda gradient, is the load itself."""
    from paper_2406_13191_amd.synth import Problem
    H = np.array([[0.0, 1.0]])   # flow of the line = injection at bus 1
    return Problem(H=H, gen_bus=np.array([1], np.int32), c=np.array([c]), q=np.zeros(1),
                   p_min=np.zeros(1), p_max=np.array([p_max]), d=np.array([load, 0.0]),
                   f_max=np.array([1e4]), slack=0)


def test_step_decay_schedule():
    # the schedule itself: alpha / (1 + decay t)
    assert D.step_size(2.0, 0.5, 0) == 2.0
    assert D.step_size(2.0, 0.5, 1) == pytest.approx(2.0 / 1.5)
    assert D.step_size(2.0, 0.5, 2) == 1.0
    assert D.step_size(2.0, 0.0, 7) == 2.0


def test_step_decay_through_the_ascent():
    # plain steps (rho = 0) with a constant lambda gradient of 4 MW:
    # lambda_k = 4 alpha sum_{t<k} 1 / (1 + decay t); the limit multipliers
    # stay at zero (their gradient is -F - f_max < 0 and F - f_max < 0)
    K = D.canonical(_one_unit_two_buses())
    alpha, decay = 0.5, 0.25
    res = D.ascent(K, 4, alpha=alpha, rho=0.0, decay=decay)
    lam3 = 4 * alpha * (1 + 1 / 1.25 + 1 / 1.5 + 1 / 1.75)
    assert res.state.lam == pytest.approx(lam3, rel=1e-14)
    assert np.all(res.state.mu == 0.0)
    # gamma_k = c p* + lambda (d - p*) - 0 = lambda_k * 4 at p* = 0
    lams = 4 * alpha * np.cumsum([0.0, 1.0, 1 / 1.25, 1 / 1.5])
    np.testing.assert_allclose(res.gammas, 4.0 * lams, rtol=1e-14)
    # heavy ball with decay: v_k = rho v_{k-1} + alpha_k 4
    rho = 0.5
    res = D.ascent(K, 3, alpha=alpha, rho=rho, decay=decay)
    v1 = alpha * 4
    v2 = rho * v1 + alpha / 1.25 * 4
    v3 = rho * v2 + alpha / 1.5 * 4
    assert res.state.lam == pytest.approx(v1 + v2 + v3, rel=1e-14)
    # a resumed state carries its counter: 2 + 2 updates equal 4
    a = D.ascent(K, 2, alpha=alpha, rho=0.0, decay=decay)
    b = D.ascent(K, 2, alpha=alpha, rho=0.0, decay=decay, state=a.state)
    assert b.state.lam == pytest.approx(lam3, rel=1e-14)
