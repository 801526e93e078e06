"""Primal recovery on the single-instance HIP path against the FP64 oracle:
the averaged dispatch, its cost and its residuals after the same iterations
(FP64 panel on an LP and a QP network, FP32 panel on the QP), isolation from
the timing iterations, and the error when nothing has been averaged."""
import numpy as np
import pytest

from oracle import dual as D
from paper_2406_13191_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("both_schemes")]


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


_PROBS = {}


def prob(name, seed):
    if (name, seed) not in _PROBS:
        _PROBS[(name, seed)] = synth.make_problem(name, seed)
    return _PROBS[(name, seed)]


def run_gpu(p, precision, k0, n, alpha, rho):
    A = _abi()
    with A.DualSolver(p, rule="gdm", alpha=alpha, rho=rho, precision=precision,
                      graph_iters=16) as s:
        s.step(k0)
        s.average(True)
        s.step(n)
        return s.primal()


def run_oracle(p, k0, n, alpha, rho):
    K = D.canonical(p)
    res = D.ascent(K, k0 + n, alpha=alpha, rho=rho, average_from=k0)
    return D.primal_eval(K, D.averaged_primal(res))


@pytest.mark.parametrize("name,seed,rtol", [("geo300q", 7, 1e-9), ("tiny30", 1, 1e-7),
                                            ("geo300", 7, 1e-7)])
def test_fp64_average_matches_oracle(name, seed, rtol):
    p = prob(name, seed)
    r = synth.STEP_RULES[name]
    k0, n = 150, 450
    g = run_gpu(p, "fp64", k0, n, r["alpha"], r["rho"])
    o = run_oracle(p, k0, n, r["alpha"], r["rho"])
    assert g["iterations"] == n
    scale = max(np.abs(o.x).max(), 1.0)
    err = np.abs(g["p"] - o.x).max()
    print(f"{name}: max |p_gpu - p_oracle| = {err:.3e}, cost {g['cost']:.6f} vs {o.cost:.6f}")
    assert err <= rtol * scale
    assert g["cost"] == pytest.approx(o.cost, rel=rtol, abs=1e-9)
    assert g["balance"] == pytest.approx(o.balance, rel=1e-6, abs=rtol * scale * p.n_gen)
    assert g["max_overload"] == pytest.approx(o.max_overload, rel=1e-6, abs=1e-6)
    assert g["sum_overload"] == pytest.approx(o.sum_overload, rel=1e-6, abs=1e-6)
    assert g["n_overloaded"] == o.n_overloaded


def test_fp32_average_tracks_oracle_on_qp():
    # the QP's inner minimiser is continuous, so FP32 products keep the
    # trajectory close to the FP64 oracle's
    p = prob("geo300q", 7)
    r = synth.STEP_RULES["geo300q"]
    g = run_gpu(p, "fp32", 100, 400, r["alpha"], r["rho"])
    o = run_oracle(p, 100, 400, r["alpha"], r["rho"])
    scale = max(np.abs(o.x).max(), 1.0)
    assert np.abs(g["p"] - o.x).max() <= 1e-4 * scale
    assert g["cost"] == pytest.approx(o.cost, rel=1e-6)


def test_timing_iterations_do_not_enter_the_average():
    A = _abi()
    p = prob("geo300q", 7)
    r = synth.STEP_RULES["geo300q"]
    kw = dict(rule="gdm", alpha=r["alpha"], rho=r["rho"], precision="fp64")
    with A.DualSolver(p, **kw) as a, A.DualSolver(p, **kw) as b:
        a.average(True)
        a.step(40)
        a.time_phases(10)
        a.step(60)
        b.average(True)
        b.step(100)
        pa, pb = a.primal(), b.primal()
    assert pa["iterations"] == pb["iterations"] == 100
    np.testing.assert_array_equal(pa["p"], pb["p"])


def test_average_stop_and_restart():
    A = _abi()
    p = prob("tiny30", 1)
    with A.DualSolver(p, rule="gdm", alpha=1e-4, rho=0.99, precision="fp64") as s:
        with pytest.raises(A.DcopfError):
            s.primal()                  # nothing averaged yet
        s.average(True)
        s.step(30)
        s.average(False)
        s.step(20)                      # not added
        assert s.primal()["iterations"] == 30
        s.average(True)                 # restart
        s.step(5)
        assert s.primal()["iterations"] == 5
