"""Pins of the oracle's primal repair (an extension; not in the paper).

Closed forms derived by hand on a one-line network (a generator at the slack
bus, one or two behind the line, the load behind the line), the stop rule on
a feasible input, the failure report, and on the synthetic networks: the
repaired average is feasible by an independent evaluation and its cost is an
upper bound no lower than the HiGHS optimum (weak duality), close to it."""
import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from oracle.repair import MARGIN, repair
from paper_2406_13191_amd import synth


def one_line(hi, fmax=50.0, load=100.0, load_bus=1):
    """Bus 0 (slack) - bus 1, one line 0 -> 1; generator 0 at bus 0, the
    others at bus 1.  The PTDF of the line is 0 for bus 0 and -1 for bus 1,
    so F = (load at bus 1) - (output at bus 1)."""
    n = len(hi)
    HC = np.array([[0.0] + [-1.0] * (n - 1)])
    Hd = np.array([-load if load_bus == 1 else 0.0])
    return D.Canonical(c=np.arange(1.0, n + 1.0), M=np.zeros(n), A=-np.ones((1, n)),
                       b=np.array([-load]), C=np.vstack([HC, -HC]),
                       d=np.concatenate([fmax + Hd, fmax - Hd]), lo=np.zeros(n),
                       hi=np.asarray(hi, float))


def test_two_generators_closed_form():
    # F = 100 - 35 = 65 > 50, balance 100 - 105 = -5: the line lands at
    # 50 - MARGIN (p1 = 50 + MARGIN), the balance fixes p0 = 50 - MARGIN
    K = one_line([200.0, 200.0])
    r = repair(K, np.array([70.0, 35.0]))
    assert r.feasible and r.rounds == 1 and r.active == [(0, 1)]
    np.testing.assert_allclose(r.x, [50.0 - MARGIN, 50.0 + MARGIN], rtol=0, atol=1e-9)


def test_headroom_weights_split_the_move():
    # generators 1 and 2 share the line row: together they must add
    # 15 + MARGIN, split 10 : 15 by their headroom min(p - lo, hi - p)
    K = one_line([200.0, 30.0, 100.0])
    r = repair(K, np.array([70.0, 20.0, 15.0]))
    assert r.feasible and r.rounds == 1
    np.testing.assert_allclose(
        r.x, [50.0 - MARGIN, 26.0 + 0.4 * MARGIN, 24.0 + 0.6 * MARGIN], rtol=0, atol=1e-9)


def test_bound_hit_takes_a_second_round():
    # F = 100 - 25 = 75, balance +5; headrooms 70, 4, 5.  The first step
    # moves generators 1 and 2 by (25 + MARGIN) 4/9 and 5/9: generator 1
    # would reach 31.1 and is clipped at 24 (F = 57.1 - 5/9 MARGIN, balance
    # 7.1 + 4/9 MARGIN).  Generator 1 now has only the floor weight 0.024
    # against 18.9 for generator 2: each later step pushes it out again
    # (undone by the clip), leaving 0.024 / 18.9 of the residual, until
    # generator 2 lands at 26 + MARGIN, generator 0 staying put
    K = one_line([200.0, 24.0, 100.0])
    r = repair(K, np.array([70.0, 20.0, 5.0]))
    assert r.feasible and 2 <= r.rounds <= 6
    # it stops once the balance is within 1e-9 of the load (1e-7 MW)
    np.testing.assert_allclose(r.x, [50.0 - MARGIN, 24.0, 26.0 + MARGIN], rtol=0, atol=1e-7)


def test_other_direction_and_balance_only():
    # load at the slack bus: F = -p1 = -60 < -50, balance 0; the line is
    # held at -(50 - MARGIN) and generator 0 takes what generator 1 sheds
    K = one_line([200.0, 200.0], load_bus=0)
    r = repair(K, np.array([40.0, 60.0]))
    assert r.feasible and r.rounds == 1 and r.active == [(0, -1)]
    np.testing.assert_allclose(r.x, [50.0 + MARGIN, 50.0 - MARGIN], rtol=0, atol=1e-9)
    # clipped into the box first: [-10, 60] -> [0, 60]; generator 0, at its
    # minimum, moves inward on its floor weight (0.2 against 60), where the
    # ridge leaves a residual inside the balance tolerance (1e-7 MW)
    r = repair(K, np.array([-10.0, 60.0]))
    assert r.feasible and r.active == [(0, -1)]
    np.testing.assert_allclose(r.x, [50.0 + MARGIN, 50.0 - MARGIN], rtol=0, atol=1e-7)
    # no line violated: one step spreads the balance by headroom (10 : 80)
    K = one_line([200.0, 200.0])
    r = repair(K, np.array([10.0, 80.0]))
    assert r.feasible and r.rounds == 1 and r.active == []
    np.testing.assert_allclose(r.x, [10.0 + 10.0 / 9.0, 80.0 + 80.0 / 9.0], rtol=0, atol=1e-9)


def test_slack_held_line_leaves_the_working_set():
    # radial: slack - line 1 - bus 1 (generator 2, load 90) - line 2 - bus 2
    # (generator 1, load 110); F1 = 200 - p1 - p2, F2 = 110 - p1, limits 50.
    # From (100, 40, 40) both lines are violated (F1 = 120, F2 = 70) and the
    # balance is +20.  Holding both at their limits gives line 2 the
    # multiplier sign of a slack inequality (sigma y = +0.75), so it leaves
    # the working set: the move is the least-norm one for line 1 and the
    # balance alone, headrooms 100 : 40 : 40, which takes line 2 to 35 too.
    HC = np.array([[0.0, -1.0, -1.0], [0.0, -1.0, 0.0]])
    Hd = np.array([-200.0, -110.0])
    fmax = np.array([50.0, 50.0])
    K = D.Canonical(c=np.array([1.0, 2.0, 3.0]), M=np.zeros(3), A=-np.ones((1, 3)),
                    b=np.array([-200.0]), C=np.vstack([HC, -HC]),
                    d=np.concatenate([fmax + Hd, fmax - Hd]), lo=np.zeros(3),
                    hi=np.full(3, 200.0))
    r = repair(K, np.array([100.0, 40.0, 40.0]))
    assert r.feasible and r.rounds == 1 and r.active == [(0, 1), (1, 1)]
    np.testing.assert_allclose(
        r.x, [50.0 - MARGIN, 75.0 + MARGIN / 2, 75.0 + MARGIN / 2], rtol=0, atol=1e-9)
    F = HC @ r.x - Hd
    assert F[1] == pytest.approx(35.0 - MARGIN / 2, abs=1e-9)


def test_feasible_input_is_returned_unchanged():
    K = one_line([200.0, 200.0])
    x = np.array([40.0, 60.0])
    r = repair(K, x)
    assert r.feasible and r.rounds == 0 and r.active == []
    np.testing.assert_array_equal(r.x, x)


def test_failure_is_reported():
    K = one_line([200.0, 200.0])
    r = repair(K, np.array([70.0, 35.0]), max_rounds=0)
    assert not r.feasible and r.rounds == 0
    np.testing.assert_array_equal(r.x, [70.0, 35.0])
    # the generator behind the line is at its maximum: the line cannot be
    # relieved, each step's move is undone by the clip
    K = one_line([200.0, 35.0])
    r = repair(K, np.array([65.0, 35.0]), max_rounds=5)
    assert not r.feasible and r.rounds == 5 and r.max_overload > 10.0


@pytest.mark.parametrize("name,seed,n", [("tiny30", 1, 20000), ("geo300", 7, 8000)])
def test_repaired_average_is_a_feasible_upper_bound(name, seed, n):
    net, p = synth.make_network(name, seed)
    K = D.canonical(p)
    r = synth.STEP_RULES[name]
    res = D.ascent(K, n, alpha=r["alpha"], rho=r["rho"], average_from=n // 2)
    rep = repair(K, D.averaged_primal(res))
    assert rep.feasible
    pe = D.primal_eval(K, rep.x)
    assert pe.max_overload == 0.0                   # MARGIN inside every limit
    assert abs(pe.balance) <= 1e-9 * np.sum(p.d)
    assert np.all(rep.x >= p.p_min) and np.all(rep.x <= p.p_max)
    opt = ref.opt_btheta(net, p)["opt"]
    assert res.best <= opt <= rep.cost * (1 + 1e-12)
    assert rep.cost - opt <= 1e-3 * abs(opt)
    print(f"{name}: UB - OPT = {(rep.cost - opt) / opt:.2e}, UB - LB = "
          f"{(rep.cost - res.best) / rep.cost:.2e} in {rep.rounds} rounds")


def test_perturbed_optima_repair_to_feasible_upper_bounds():
    # HiGHS optimum + N(0, 3 MW) noise per generator: many lines violated at
    # once; every candidate repairs to a feasible dispatch costing no less
    # than the optimum
    net, p = synth.make_network("geo300", 3)
    K = D.canonical(p)
    o = ref.opt_btheta(net, p)
    rng = np.random.default_rng(0)
    for _ in range(6):
        rep = repair(K, o["p"] + rng.normal(0.0, 3.0, o["p"].size), max_rounds=64)
        assert rep.feasible
        pe = D.primal_eval(K, rep.x)
        assert pe.max_overload == 0.0 and abs(pe.balance) <= 1e-9 * np.sum(p.d)
        assert rep.cost >= o["opt"] * (1 - 1e-12)


def test_qp_repair_bounds_the_certified_optimum():
    _, p = synth.make_network("tiny30", 1)
    rng = np.random.default_rng(5)
    K = D.canonical(p.replace(q=rng.uniform(0.001, 0.05, p.n_gen)))
    cert = ref.qp_certificate(K)
    res = D.ascent(K, 4000, alpha=1e-4, rho=0.99, average_from=2000)
    rep = repair(K, D.averaged_primal(res))
    assert rep.feasible
    assert rep.cost >= cert["lb"] * (1 - 1e-12)
    assert rep.cost - cert["lb"] <= 1e-4 * abs(cert["lb"])
