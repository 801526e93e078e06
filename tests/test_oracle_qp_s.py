"""Pins of the oracle's iterated-s QP dual (Section 3.2, eq. QP_finalgamma):
its value equals the paper's normalised formula (implemented separately in
``oracle.dual.g_q_paper``) at any s, never exceeds the closed-form dual and
meets it at s*, its supergradients match central differences away from
ties, and its ascent stays below the certified optimum while approaching
it."""
import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from oracle.qp_s import ascent_s, dual_value_s
from paper_2406_13191_amd import synth


@pytest.fixture(scope="module")
def qp():
    _, p = synth.make_network("tiny30", 1)
    rng = np.random.default_rng(5)
    return D.canonical(p.replace(q=rng.uniform(0.001, 0.05, p.n_gen)))


def rand_point(K, rng):
    lam = float(rng.uniform(20, 60))
    mu = rng.exponential(2.0, 2 * K.n_line) * (rng.random(2 * K.n_line) < 0.3)
    s = rng.normal(0.0, 5.0, K.c.size)
    return lam, mu, s


def test_value_is_the_paper_formula(qp):
    rng = np.random.default_rng(1)
    for _ in range(20):
        lam, mu, s = rand_point(qp, rng)
        assert dual_value_s(qp, lam, mu, s).g == pytest.approx(D.g_q_paper(qp, lam, mu, s),
                                                              rel=1e-12, abs=1e-8)


def test_below_closed_form_equal_at_s_star(qp):
    rng = np.random.default_rng(2)
    m = 0.5 * (qp.lo + qp.hi)
    for _ in range(20):
        lam, mu, s = rand_point(qp, rng)
        g = D.dual_value(qp, lam, mu)
        assert dual_value_s(qp, lam, mu, s).g <= g.g + 1e-9 * abs(g.g)
        s_star = -2.0 * np.sqrt(qp.M) * (g.x - m)
        assert dual_value_s(qp, lam, mu, s_star).g == pytest.approx(g.g, rel=1e-12)


def test_supergradients_by_central_differences(qp):
    rng = np.random.default_rng(3)
    lam, mu, s = rand_point(qp, rng)
    ev = dual_value_s(qp, lam, mu, s)
    assert np.min(np.abs(ev.a)) > 1e-3          # no tie within the steps below
    # G_s is quadratic in (lambda, mu, s) between ties, so a central
    # difference is exact up to rounding (|G| 1e-16 / h)
    h = 1e-4
    for j in range(qp.c.size):
        e = np.zeros_like(s)
        e[j] = h
        fd = (dual_value_s(qp, lam, mu, s + e).g - dual_value_s(qp, lam, mu, s - e).g) / (2 * h)
        assert fd == pytest.approx(ev.grad_s[j], rel=1e-6, abs=1e-6)
    fd = (dual_value_s(qp, lam + h, mu, s).g - dual_value_s(qp, lam - h, mu, s).g) / (2 * h)
    assert fd == pytest.approx(ev.grad_lam, rel=1e-6, abs=1e-6)
    for i in np.flatnonzero(mu > 0)[:10]:
        e = np.zeros_like(mu)
        e[i] = h
        fd = (dual_value_s(qp, lam, mu + e, s).g - dual_value_s(qp, lam, mu - e, s).g) / (2 * h)
        assert fd == pytest.approx(ev.grad_mu[i], rel=1e-6, abs=1e-6)


def test_ascent_bounds_the_certified_optimum(qp):
    cert = ref.qp_certificate(qp)
    res = ascent_s(qp, 20000, alpha=1e-4, rho=0.99)
    assert np.all(res.gammas <= cert["ub"] * (1 + 1e-12))
    closed = D.ascent(qp, 20000, alpha=1e-4, rho=0.99)
    gap_s = (cert["lb"] - res.best) / abs(cert["lb"])
    gap_c = (cert["lb"] - closed.best) / abs(cert["lb"])
    print(f"gap after 20000 iterations: iterated s {gap_s:.2e}, closed form {gap_c:.2e}")
    assert 0.0 <= gap_s < 2e-2   # below the optimum, and approaching it
