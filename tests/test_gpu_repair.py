"""Primal repair on the HIP path (an extension, not in the paper) against the
FP64 oracle: the same candidate (the oracle's own averaged dispatch, or a
seeded perturbation of a HiGHS optimum) repaired on both sides takes the same
rounds and active set and lands on the same dispatch; the device's cost and
residuals are the oracle's evaluation of its result; on the 2000-bus
workload the repaired average of the FP32 path is feasible and bounds the
HiGHS optimum from above; argument errors and the stop rules."""
import numpy as np
import pytest

from oracle import dual as D
from oracle import ref
from oracle.repair import repair as oracle_repair
from paper_2406_13191_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("both_schemes")]


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


_NETS = {}


def net(name, seed):
    if (name, seed) not in _NETS:
        print(f"[gen] {name} seed={seed}", flush=True)
        _NETS[(name, seed)] = synth.make_network(name, seed)
    return _NETS[(name, seed)]


def solver(p):
    return _abi().DualSolver(p, rule="gdm", alpha=1e-4, rho=0.99, precision="fp64")


def compare(g, o, K):
    scale = max(float(np.abs(o.x).max()), 1.0)
    err = float(np.abs(g["p"] - o.x).max())
    print(f"rounds {g['rounds']}/{o.rounds}, active {g['n_active']}/{len(o.active)}, "
          f"max |p_gpu - p_oracle| = {err:.2e}", flush=True)
    assert g["feasible"] == o.feasible
    assert g["rounds"] == o.rounds
    assert g["n_active"] == len(o.active)
    assert err <= 1e-9 * scale
    assert g["cost"] == pytest.approx(o.cost, rel=1e-11)
    # the device's evaluation of its own result is the oracle's evaluation
    pe = D.primal_eval(K, g["p"])
    assert g["cost"] == pytest.approx(pe.cost, rel=1e-12)
    assert abs(g["balance"] - pe.balance) <= 1e-12 * float(np.abs(g["p"]).sum())
    assert g["max_overload"] == pytest.approx(pe.max_overload, abs=1e-9)


@pytest.mark.parametrize("name,seed,n", [("tiny30", 1, 4000), ("geo300", 7, 3000),
                                         ("geo300q", 7, 2000)])
def test_repair_of_oracle_average_matches_oracle(name, seed, n):
    _, p = net(name, seed)
    K = D.canonical(p)
    r = synth.STEP_RULES[name]
    res = D.ascent(K, n, alpha=r["alpha"], rho=r["rho"], average_from=n // 2)
    x0 = D.averaged_primal(res)
    o = oracle_repair(K, x0)
    assert o.feasible
    for precision in ("fp64", "fp32"):     # the repair is FP64 either way
        with _abi().DualSolver(p, rule="gdm", alpha=r["alpha"], rho=r["rho"],
                               precision=precision) as s:
            g = s.repair(x0)
        compare(g, o, K)


def test_repair_of_perturbed_optimum_matches_oracle():
    netw, p = net("geo300", 7)
    K = D.canonical(p)
    x_opt = ref.opt_btheta(netw, p)["p"]
    rng = np.random.default_rng(42)
    x0 = x_opt + rng.normal(0.0, 0.5, x_opt.size)
    o = oracle_repair(K, x0)
    with solver(p) as s:
        g = s.repair(x0)
    compare(g, o, K)
    assert g["max_shift"] == pytest.approx(o.max_shift, rel=1e-9, abs=1e-9)


def test_repair_of_the_device_average_matches_oracle():
    # FP64 loop on a QP network: the device average equals the oracle's to
    # ~1e-9, and so do the repairs of the two
    _, p = net("geo300q", 7)
    K = D.canonical(p)
    r = synth.STEP_RULES["geo300q"]
    with _abi().DualSolver(p, rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp64",
                           graph_iters=16) as s:
        s.step(300)
        s.average(True)
        s.step(900)
        g = s.repair(None)
    res = D.ascent(K, 1200, alpha=r["alpha"], rho=r["rho"], average_from=300)
    o = oracle_repair(K, D.averaged_primal(res))
    assert g["feasible"] and o.feasible
    assert g["rounds"] == o.rounds and g["n_active"] == len(o.active)
    assert np.abs(g["p"] - o.x).max() <= 1e-7 * max(np.abs(o.x).max(), 1.0)


def test_repaired_fp32_average_bounds_highs_optimum_2000_bus():
    netw, p = net("bus2000", 2000)
    K = D.canonical(p)
    r = synth.STEP_RULES["bus2000"]
    with _abi().DualSolver(p, rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp32",
                           graph_iters=100) as s:
        s.step(2000)
        s.average(True)
        s.step(8000)
        s.bound()                                # exact bound at the last iterate
        lb, _ = s.best()
        g = s.repair(None)
    opt = ref.opt_btheta(netw, p)["opt"]
    print(f"2000-bus: feasible {g['feasible']} in {g['rounds']} rounds, {g['n_active']} lines "
          f"held; UB - OPT = {(g['cost'] - opt) / opt:.2e}, UB - LB = "
          f"{(g['cost'] - lb) / g['cost']:.2e}", flush=True)
    assert g["feasible"]
    pe = D.primal_eval(K, g["p"])
    assert pe.max_overload <= 1e-9
    assert abs(pe.balance) <= 1e-9 * float(np.sum(p.d))
    assert np.all(g["p"] >= p.p_min) and np.all(g["p"] <= p.p_max)
    assert lb <= opt <= g["cost"] * (1 + 1e-12)
    assert g["cost"] - opt <= 1e-3 * opt


def test_feasible_input_unchanged_zero_rounds_and_errors():
    A = _abi()
    _, p = net("geo300", 7)
    K = D.canonical(p)
    r = synth.STEP_RULES["geo300"]
    res = D.ascent(K, 2000, alpha=r["alpha"], rho=r["rho"], average_from=1000)
    x0 = D.averaged_primal(res)
    with solver(p) as s:
        with pytest.raises(A.DcopfError):
            s.repair(None)                       # nothing averaged
        with pytest.raises(A.DcopfError):
            s.repair(np.full(p.n_gen, np.nan))
        with pytest.raises(A.DcopfError):
            s.repair(x0, max_rounds=-1)
        g0 = s.repair(x0, max_rounds=0)
        np.testing.assert_array_equal(g0["p"], np.clip(x0, p.p_min, p.p_max))
        assert g0["rounds"] == 0
        g = s.repair(x0)
        assert g["feasible"]
        again = s.repair(g["p"])
        assert again["feasible"] and again["rounds"] == 0 and again["n_active"] == 0
        np.testing.assert_array_equal(again["p"], g["p"])
        assert again["max_shift"] == 0.0
