"""Repair on the batched HIP path (an extension, not in the paper) against the
FP64 oracle, instance by instance: the oracle's own averaged candidates of
an LP and a QP network in one batch take the same rounds and active sets
and land on the same dispatches; the device's cost and residuals are the
oracle's evaluation of its results; the repaired device averages are
feasible and bound each instance's best exact bound from above; instances
stop independently; argument errors."""
import numpy as np
import pytest

from oracle import dual as D
from oracle.repair import repair as oracle_repair
from paper_2406_13191_amd import synth

pytestmark = pytest.mark.gpu


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


_BASE = {}


def batch_net(name, seed, B, seed0):
    if (name, seed) not in _BASE:
        _BASE[(name, seed)] = synth.make_network(name, seed)[1]
    base = _BASE[(name, seed)]
    Dm, Cc, Q = synth.make_scenarios(base, seed0, B, 0.1, 0.1)
    r = synth.STEP_RULES[name]
    bn = _abi().BatchNetwork(base, Dm, Cc, Q if base.is_qp else None, alpha=r["alpha"],
                             rho=r["rho"])
    Ks = [D.canonical(base.replace(d=Dm[i], c=Cc[i], q=Q[i])) for i in range(B)]
    return bn, Ks


@pytest.fixture(scope="module")
def nets():
    return [batch_net("geo300", 7, 5, 9500), batch_net("geo300q", 7, 4, 9600)]


def oracle_candidates(Ks, name, n=1500):
    r = synth.STEP_RULES[name]
    return np.array([D.averaged_primal(D.ascent(K, n, alpha=r["alpha"], rho=r["rho"],
                                                 average_from=n // 2)) for K in Ks])


def test_oracle_candidates_match_oracle_repair(nets):
    A = _abi()
    (n1, K1), (n2, K2) = nets
    x1, x2 = oracle_candidates(K1, "geo300"), oracle_candidates(K2, "geo300q")
    with A.BatchSolver([n1, n2]) as b:
        g = [b.repair(0, x1), b.repair(1, x2)]
    for k, (Ks, xs) in enumerate(((K1, x1), (K2, x2))):
        for i, K in enumerate(Ks):
            o = oracle_repair(K, xs[i])
            err = np.abs(g[k]["p"][i] - o.x).max()
            print(f"net {k} instance {i}: rounds {g[k]['rounds'][i]}/{o.rounds}, active "
                  f"{g[k]['n_active'][i]}/{len(o.active)}, max |dp| {err:.2e}", flush=True)
            assert g[k]["feasible"][i] == o.feasible
            assert g[k]["rounds"][i] == o.rounds
            assert g[k]["n_active"][i] == len(o.active)
            assert err <= 1e-9 * max(np.abs(o.x).max(), 1.0)
            assert g[k]["cost"][i] == pytest.approx(o.cost, rel=1e-11)
            pe = D.primal_eval(K, g[k]["p"][i])
            assert g[k]["cost"][i] == pytest.approx(pe.cost, rel=1e-12)
            assert abs(g[k]["balance"][i] - pe.balance) <= 1e-12 * np.abs(g[k]["p"][i]).sum()
            assert g[k]["max_overload"][i] == pytest.approx(pe.max_overload, abs=1e-9)


def test_repaired_device_averages_bound_the_best_bounds(nets):
    A = _abi()
    (n1, K1), (n2, K2) = nets
    with A.BatchSolver([n1, n2], graph_iters=20) as b:
        b.step(1000)
        b.average(True)
        for _ in range(20):
            b.step(100)
            b.bound()                           # tracks each instance's best exact bound
        best, _ = b.best()
        g = [b.repair(0), b.repair(1)]
    lb = [best[:n1.B], best[n1.B:]]
    for k, Ks in enumerate((K1, K2)):
        assert np.all(g[k]["feasible"])
        for i, K in enumerate(Ks):
            pe = D.primal_eval(K, g[k]["p"][i])
            assert pe.max_overload <= 1e-9
            assert abs(pe.balance) <= 1e-9 * abs(K.b[0])
            assert lb[k][i] <= g[k]["cost"][i] * (1 + 1e-12)
        gap = (g[k]["cost"] - lb[k]) / np.abs(g[k]["cost"])
        print(f"net {k}: certified gaps {np.array2string(gap, precision=2)}", flush=True)


def test_instances_stop_independently_and_errors(nets):
    A = _abi()
    (n1, K1), _ = nets
    x1 = oracle_candidates(K1, "geo300", n=1000)
    feasible = np.array([oracle_repair(K, x).x for K, x in zip(K1, x1)])
    mixed = x1.copy()
    mixed[1] = feasible[1]                      # already feasible: no round
    with A.BatchSolver([n1]) as b:
        with pytest.raises(A.DcopfError):
            b.repair(0)                         # nothing averaged
        with pytest.raises(A.DcopfError):
            b.repair(0, np.full_like(x1, np.nan))
        with pytest.raises(A.DcopfError):
            b.repair(0, x1, max_rounds=-1)
        g0 = b.repair(0, x1, max_rounds=0)
        np.testing.assert_array_equal(g0["p"], np.clip(x1, K1[0].lo, K1[0].hi))
        assert np.all(g0["rounds"] == 0)
        g = b.repair(0, mixed)
    assert g["rounds"][1] == 0 and g["feasible"][1]
    np.testing.assert_array_equal(g["p"][1], feasible[1])
    for i in (0, 2, 3, 4):
        assert g["feasible"][i] and g["rounds"][i] == oracle_repair(K1[i], x1[i]).rounds
