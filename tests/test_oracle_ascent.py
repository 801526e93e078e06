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
