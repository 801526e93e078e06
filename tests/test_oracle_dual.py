"""Pins of the oracle's dual function (Section 3, Appendix A1/A2) against
closed forms, brute force, the paper's own normalised formulas and calculus."""
import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from paper_2406_13191_amd import synth


def _rand_multipliers(rng, K, scale=5.0, frac=0.3):
    lam = float(rng.uniform(0, 80))
    mu = rng.exponential(scale, 2 * K.n_line) * (rng.random(2 * K.n_line) < frac)
    return lam, mu


def test_inner_argmin_vs_grid():
    rng = np.random.default_rng(1)
    n = 400
    lo = rng.uniform(-5, 5, n)
    hi = lo + rng.uniform(0, 10, n)
    a = rng.normal(0, 3, n)
    a[:20] = 0.0
    M = np.where(rng.random(n) < 0.5, 0.0, rng.uniform(0.01, 2, n))
    x = D.inner_argmin(a, M, lo, hi)
    grid = lo[:, None] + (hi - lo)[:, None] * np.linspace(0, 1, 20001)[None, :]
    f = M[:, None] * grid ** 2 + a[:, None] * grid
    fbest = f.min(axis=1)
    fx = M * x * x + a * x
    assert np.all(fx <= fbest + 1e-9)
    assert np.all((x >= lo) & (x <= hi))
    # ties of the linear case return the midpoint
    lin0 = (M == 0) & (a == 0)
    np.testing.assert_allclose(x[lin0], 0.5 * (lo + hi)[lin0])


def test_dual_norm_identity():
    # Appendix A2: min over [l, u] of r p = r m - sigma |r| (m midpoint,
    # sigma half width), i.e. -||.||_1 on the unit infinity ball
    rng = np.random.default_rng(2)
    lo = rng.uniform(0, 50, 100)
    hi = lo + rng.uniform(0, 100, 100)
    r = rng.normal(0, 10, 100)
    x = D.inner_argmin(r, np.zeros(100), lo, hi)
    m, s = 0.5 * (lo + hi), 0.5 * (hi - lo)
    np.testing.assert_allclose(r * x, r * m - s * np.abs(r), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_lp_dual_equals_paper_normalised_form(seed):
    # Eq. (LP dual) on the data normalised per Appendix A1 (plus the constant
    # the substitution moves out) equals the box-form dual function
    p = synth.make_problem("tiny30", seed)
    K = D.canonical(p)
    rng = np.random.default_rng(seed)
    for _ in range(20):
        lam, mu = _rand_multipliers(rng, K)
        g = D.dual_value(K, lam, mu).g
        assert abs(g - D.g_l_paper(K, lam, mu)) <= 1e-9 * max(1.0, abs(g))


def test_qp_dual_s_form():
    # Eq. (QP_finalgamma): g_q(s*) equals the closed-form dual, and g_q(s) is
    # no larger for any other s ("exactly agree" claim of Section 3.2)
    net, p = synth.make_network("geo300q", 7)
    K = D.canonical(p)
    rng = np.random.default_rng(0)
    for _ in range(5):
        lam, mu = _rand_multipliers(rng, K)
        g = D.dual_value(K, lam, mu).g
        s = D.s_star(K, lam, mu)
        assert abs(D.g_q_paper(K, lam, mu, s) - g) <= 1e-9 * abs(g)
        for _ in range(5):
            s2 = s + rng.normal(0, 1.0, s.size)
            assert D.g_q_paper(K, lam, mu, s2) <= g + 1e-9 * abs(g)


def test_supergradient_matches_central_differences_qp():
    net, p = synth.make_network("geo300q", 7)
    K = D.canonical(p)
    rng = np.random.default_rng(4)
    lam, mu = _rand_multipliers(rng, K, scale=2.0)
    ev = D.dual_value(K, lam, mu)
    h = 1e-4
    gl = (D.dual_value(K, lam + h, mu).g - D.dual_value(K, lam - h, mu).g) / (2 * h)
    assert abs(gl - ev.grad_lam) <= 1e-5 * max(1.0, abs(ev.grad_lam))
    idx = rng.choice(mu.size, 40, replace=False)
    mu = mu.copy()
    mu[idx] = np.maximum(mu[idx], 1.0)  # interior points for a two-sided difference
    ev = D.dual_value(K, lam, mu)
    for i in idx:
        e = np.zeros_like(mu)
        e[i] = h
        fd = (D.dual_value(K, lam, mu + e).g - D.dual_value(K, lam, mu - e).g) / (2 * h)
        assert abs(fd - ev.grad_mu[i]) <= 1e-4 * max(1.0, abs(ev.grad_mu[i]))


def test_supergradient_lp_where_smooth():
    p = synth.make_problem("tiny30", 1)
    K = D.canonical(p)
    rng = np.random.default_rng(5)
    lam, mu = _rand_multipliers(rng, K)
    mu = mu + 1.0
    ev = D.dual_value(K, lam, mu)
    # |C| <= 1 entrywise, so a step h moves every reduced cost by at most h
    # per coordinate: no generator switches when min |a| > h
    h = 1e-4
    assert np.min(np.abs(ev.a)) > 1e-3
    gl = (D.dual_value(K, lam + h, mu).g - D.dual_value(K, lam - h, mu).g) / (2 * h)
    assert abs(gl - ev.grad_lam) <= 1e-5 * max(1.0, abs(ev.grad_lam))
    for i in range(mu.size):
        e = np.zeros_like(mu)
        e[i] = h
        fd = (D.dual_value(K, lam, mu + e).g - D.dual_value(K, lam, mu - e).g) / (2 * h)
        assert abs(fd - ev.grad_mu[i]) <= 1e-4 * max(1.0, abs(ev.grad_mu[i]))


def test_concavity():
    net, p = synth.make_network("geo300", 7)
    K = D.canonical(p)
    rng = np.random.default_rng(6)
    for _ in range(10):
        l1, m1 = _rand_multipliers(rng, K)
        l2, m2 = _rand_multipliers(rng, K)
        g1 = D.dual_value(K, l1, m1).g
        g2 = D.dual_value(K, l2, m2).g
        gm = D.dual_value(K, 0.5 * (l1 + l2), 0.5 * (m1 + m2)).g
        assert gm >= 0.5 * (g1 + g2) - 1e-9 * abs(gm)


@pytest.mark.parametrize("name,seed", [("tiny30", 1), ("geo300", 7)])
def test_weak_duality(name, seed):
    # Remarks 1-2: any mu >= 0, lambda gives a value <= every feasible cost
    net, p = synth.make_network(name, seed)
    K = D.canonical(p)
    opt = ref.opt_ptdf(p, want_duals=False)["opt"]
    rng = np.random.default_rng(seed)
    for _ in range(30):
        lam, mu = _rand_multipliers(rng, K, scale=float(rng.choice([0.1, 1, 10, 100])))
        assert D.dual_value(K, lam, mu).g <= opt + 1e-9 * abs(opt)
    # random feasible points: HiGHS optima of random objectives over the same set
    import scipy.optimize as so
    for _ in range(5):
        cr = rng.normal(size=K.c.size)
        r = so.linprog(cr, A_ub=K.C, b_ub=K.d, A_eq=-K.A, b_eq=-K.b,
                       bounds=list(zip(K.lo, K.hi)), method="highs")
        cost = float(K.c @ r.x + r.x @ (K.M * r.x))
        lam, mu = _rand_multipliers(rng, K)
        assert D.dual_value(K, lam, mu).g <= cost + 1e-9 * abs(cost)


@pytest.mark.parametrize("qp", [False, True])
def test_nu_form_complementary_split(qp):
    """The dual depends on (mu+, mu-) through nu = mu+ - mu- and the limit
    term -(mu+ + mu-)^T f_max only: moving to the complementary split
    (max(nu, 0), max(-nu, 0)) of the same nu raises it by exactly
    2 sum_l min(mu+_l, mu-_l) f_max_l, and leaves it unchanged when mu+ and
    mu- are already complementary."""
    _, p = synth.make_network("tiny30", 1)
    if qp:
        p = p.replace(q=np.random.default_rng(8).uniform(0.001, 0.05, p.n_gen))
    K = D.canonical(p)
    rng = np.random.default_rng(9)
    nl = p.n_line
    for _ in range(25):
        lam = float(rng.uniform(0.0, 80.0))
        mp = rng.exponential(3.0, nl) * (rng.random(nl) < 0.6)
        mm = rng.exponential(3.0, nl) * (rng.random(nl) < 0.6)
        nu = mp - mm
        g = D.dual_value(K, lam, np.r_[mp, mm]).g
        g_c = D.dual_value(K, lam, np.r_[np.maximum(nu, 0.0), np.maximum(-nu, 0.0)]).g
        gain = 2.0 * float(np.sum(np.minimum(mp, mm) * p.f_max))
        assert g <= g_c + 1e-9 * max(1.0, abs(g_c))
        assert g_c - g == pytest.approx(gain, rel=1e-9, abs=1e-6 * max(1.0, abs(g)))
        # already complementary: mu- zeroed wherever mu+ is positive
        mm0 = np.where(mp > 0, 0.0, mm)
        g0 = D.dual_value(K, lam, np.r_[mp, mm0]).g
        nu0 = mp - mm0
        g0_c = D.dual_value(K, lam, np.r_[np.maximum(nu0, 0.0), np.maximum(-nu0, 0.0)]).g
        assert g0_c == pytest.approx(g0, rel=1e-12, abs=1e-9)


def test_dual_value_at_minimiser_and_at_a_tie():
    """dual_value_at equals dual_value at the inner minimiser; at a linear
    unit whose reduced cost is exactly zero, every point of its interval
    gives the same value (the unit contributes 0 * p), while the residuals
    move by the unit's column of the constraints."""
    from oracle import dual as D
    from paper_2406_13191_amd import synth
    p = synth.make_problem("tiny30", 1)
    K = D.canonical(p)
    rng = np.random.default_rng(2)
    mu = rng.exponential(1.0, 2 * K.n_line) * (rng.random(2 * K.n_line) < 0.3)
    lam = 30.0
    ev = D.dual_value(K, lam, mu)
    at = D.dual_value_at(K, lam, mu, ev.x)
    assert at.g == ev.g and at.grad_lam == ev.grad_lam
    np.testing.assert_array_equal(at.grad_mu, ev.grad_mu)
    # put unit 0 exactly at its switching price (mu = 0, lambda = c_0)
    mu = np.zeros_like(mu)
    lam0 = float(K.c[0])
    ev0 = D.dual_value(K, lam0, mu)
    assert ev0.a[0] == 0.0
    for x0 in (K.lo[0], K.hi[0]):
        x = ev0.x.copy()
        x[0] = x0
        e = D.dual_value_at(K, lam0, mu, x)
        assert e.g == pytest.approx(ev0.g, rel=1e-14)
        assert e.grad_lam == pytest.approx(ev0.grad_lam - (x0 - ev0.x[0]), abs=1e-9)
        np.testing.assert_allclose(e.grad_mu, ev0.grad_mu + K.C[:, 0] * (x0 - ev0.x[0]),
                                   atol=1e-9)
