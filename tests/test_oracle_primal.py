"""Pins of the oracle's primal recovery (ergodic averaging of the inner
minimisers; not in the paper): the residuals of the averaged dispatch are the
averaged supergradients (the constraints are affine), a HiGHS optimum has
zero residuals at its own cost, and long averages approach the LP optimum
(HiGHS) and the unique QP optimum (certificate)."""
import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from paper_2406_13191_amd import synth


@pytest.fixture(scope="module")
def tiny():
    return synth.make_network("tiny30", 1)


def test_averaged_residuals_are_averaged_supergradients(tiny):
    _, p = tiny
    K = D.canonical(p)
    st = D.AscentState.cold(K.n_line)
    gl, gm = [], []
    for k in range(60):
        ev = D.dual_value(K, st.lam, st.mu)
        if k >= 20:
            gl.append(ev.grad_lam)
            gm.append(ev.grad_mu)
        st = D.gdm_update(st, ev, 1e-4, 0.99)
    res = D.ascent(K, 60, alpha=1e-4, rho=0.99, average_from=20)
    assert res.n_avg == 40
    pe = D.primal_eval(K, D.averaged_primal(res))
    assert pe.balance == pytest.approx(np.mean(gl), rel=1e-12, abs=1e-9)
    np.testing.assert_allclose(pe.overload, np.maximum(np.mean(gm, axis=0), 0.0),
                               rtol=1e-12, atol=1e-9)


def test_highs_optimum_is_feasible_at_its_cost(tiny):
    net, p = tiny
    o = ref.opt_btheta(net, p)
    K = D.canonical(p)
    pe = D.primal_eval(K, o["p"])
    assert pe.cost == pytest.approx(o["opt"], rel=1e-12)
    assert abs(pe.balance) <= 1e-6
    assert pe.max_overload <= 1e-6


def test_lp_average_approaches_the_highs_optimum(tiny):
    net, p = tiny
    opt = ref.opt_btheta(net, p)["opt"]
    K = D.canonical(p)
    r = synth.STEP_RULES["tiny30"]
    res = D.ascent(K, 20000, alpha=r["alpha"], rho=r["rho"], average_from=10000)
    pe = D.primal_eval(K, D.averaged_primal(res))
    assert abs(pe.cost - opt) <= 1e-4 * opt
    assert abs(pe.balance) <= 1e-2          # MW, against 60 % of 6 units' capacity
    assert pe.max_overload <= 1e-2          # MW
    assert res.best <= opt                   # weak duality of the bound itself


def test_qp_average_converges_to_the_unique_optimum(tiny):
    _, p = tiny
    rng = np.random.default_rng(5)
    K = D.canonical(p.replace(q=rng.uniform(0.001, 0.05, p.n_gen)))
    cert = ref.qp_certificate(K)
    assert cert["ub"] - cert["lb"] <= 1e-8 * abs(cert["lb"])
    res = D.ascent(K, 20000, alpha=1e-4, rho=0.99, average_from=10000)
    pe = D.primal_eval(K, D.averaged_primal(res))
    assert np.abs(pe.x - cert["x"]).max() <= 1e-4
    assert abs(pe.cost - cert["lb"]) <= 1e-8 * abs(cert["lb"])
    assert abs(pe.balance) <= 1e-6 and pe.max_overload <= 1e-6


def test_averaging_needs_a_window():
    K = D.Canonical(c=np.ones(1), M=np.zeros(1), A=-np.ones((1, 1)), b=-np.ones(1),
                    C=np.zeros((2, 1)), d=np.ones(2), lo=np.zeros(1), hi=np.ones(1) * 2)
    res = D.ascent(K, 5, alpha=0.1, rho=0.0)
    with pytest.raises(ValueError):
        D.averaged_primal(res)
