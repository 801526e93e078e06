"""Primal recovery on the batched HIP path (an extension: ergodic average of
the inner minimisers, not in the paper).

* The average equals the mean, over the averaged iterations, of the FP64
  oracle's inner minimiser at the multipliers the batch held before each
  iteration, to the split-BF16 error of the reduced cost (QP units) or up
  to the units whose reduced cost lay within that error of zero (LP units,
  where either bound of the box is a minimiser).
* The cost, balance and overloads the device reports for the averaged
  dispatch equal the oracle's evaluation of that same dispatch to FP64
  rounding.
* Counting, stop and restart, timed iterations, and the error when nothing
  has been averaged."""
import numpy as np
import pytest

from oracle import dual as D
from paper_2406_13191_amd import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U_SPLIT = 3 * 2.0 ** -18


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


_NETS = {}


def batch_net(name, seed, B, seed0):
    if (name, seed) not in _NETS:
        _NETS[(name, seed)] = synth.make_network(name, seed)[1]
    base = _NETS[(name, seed)]
    Dm, Cc, Q = synth.make_scenarios(base, seed0, B, 0.1, 0.1)
    r = synth.STEP_RULES[name]
    bn = _abi().BatchNetwork(base, Dm, Cc, Q if base.is_qp else None, alpha=r["alpha"],
                             rho=r["rho"])
    Ks = [D.canonical(base.replace(d=Dm[i], c=Cc[i], q=Q[i])) for i in range(B)]
    return bn, Ks


def w_error(K, v):
    """Error bound of the split-BF16 reduced-cost product P^T v."""
    nl = K.n_line
    s = np.abs(K.C[:nl]).T @ np.abs(v)
    return (U_SPLIT + 3 * (nl / 16 + 4) * U32) * s


@pytest.fixture(scope="module")
def mixed():
    """An LP network (geo300, 8 instances) and a QP network (geo300q, 6
    instances) in one batch; 40 iterations, then 50 averaged ones with the
    multipliers read before each."""
    A = _abi()
    n_lp, K_lp = batch_net("geo300", 7, 8, 9100)
    n_qp, K_qp = batch_net("geo300q", 7, 6, 9200)
    n_avg = 50
    seen = {0: [], 1: []}
    with A.BatchSolver([n_lp, n_qp]) as b:
        b.step(40)
        b.average(True)
        for _ in range(n_avg):
            for k in (0, 1):
                seen[k].append(b.get_multipliers(k))
            b.step(1)
        out = {k: b.primal(k) for k in (0, 1)}
    return dict(K={0: K_lp, 1: K_qp}, seen=seen, out=out, n_avg=n_avg)


@pytest.mark.parametrize("k", [0, 1])
def test_average_is_mean_of_inner_minimisers(mixed, k):
    Ks, seen, out, n = mixed["K"][k], mixed["seen"][k], mixed["out"][k], mixed["n_avg"]
    assert out["iterations"] == n
    worst = 0.0
    for i, K in enumerate(Ks):
        xs = np.zeros(K.c.size)
        slack = np.zeros(K.c.size)
        for lam, mp, mm in seen:
            mu = np.concatenate([mp[i], mm[i]])
            ev = D.dual_value(K, lam[i], mu)
            xs += ev.x
            dw = w_error(K, mp[i] - mm[i])
            width = K.hi - K.lo
            lin = K.M == 0
            # QP units: |dp| <= |dw| / (2 q); LP units: either end of the box
            # where the reduced cost is within the product's error of zero
            slack += np.where(lin, np.where(np.abs(ev.a) <= 2 * dw, width, 0.0),
                              np.minimum(2 * dw / (2 * np.where(lin, 1.0, K.M)), width))
        ref = xs / n
        tol = slack / n + 1e-9 * np.maximum(np.abs(ref), 1.0)
        err = np.abs(out["p"][i] - ref)
        worst = max(worst, float((err / np.maximum(tol, 1e-300)).max()))
        assert np.all(err <= tol), (i, int(np.argmax(err - tol)))
    print(f"network {k}: worst error / allowance = {worst:.3e}", flush=True)


@pytest.mark.parametrize("k", [0, 1])
def test_reported_residuals_are_the_oracle_evaluation(mixed, k):
    Ks, out = mixed["K"][k], mixed["out"][k]
    for i, K in enumerate(Ks):
        x = out["p"][i]
        pe = D.primal_eval(K, x)
        scale = float(np.abs(x).sum()) + 1.0
        nl = K.n_line
        fs = float((np.abs(K.C[:nl]) @ np.abs(x)).max() + np.abs(K.d[:nl]).max())
        assert out["cost"][i] == pytest.approx(pe.cost, rel=1e-12, abs=1e-9)
        assert abs(out["balance"][i] - pe.balance) <= 1e-12 * scale
        assert abs(out["max_overload"][i] - pe.max_overload) <= 1e-12 * fs
        assert abs(out["sum_overload"][i] - pe.sum_overload) <= 1e-12 * fs * nl
        r = K.C @ x - K.d
        assert np.count_nonzero(r > 1e-12 * fs) <= out["n_overloaded"][i] \
            <= np.count_nonzero(r > -1e-12 * fs)


def test_count_stop_restart_and_timed_iterations():
    A = _abi()
    n1, _ = batch_net("geo300q", 7, 4, 9300)
    with A.BatchSolver([n1]) as b:
        with pytest.raises(A.DcopfError):
            b.primal(0)                 # nothing averaged yet
        b.average(True)
        b.step(30)
        b.average(False)
        b.step(20)                      # not added
        assert b.primal(0)["iterations"] == 30
        b.average(True)                 # restart
        b.step(5)
        b.time_phases(7)                # timed iterations advance the batch
        r = b.primal(0)
        assert r["iterations"] == 12
        assert np.all(np.isfinite(r["p"])) and np.all(np.isfinite(r["cost"]))


def test_split_calls_average_like_one_call():
    A = _abi()
    n1, _ = batch_net("geo300", 7, 6, 9400)
    with A.BatchSolver([n1]) as a, A.BatchSolver([n1]) as b:
        a.average(True)
        b.average(True)
        a.step(60)
        for _ in range(3):
            b.step(20)
        pa, pb = a.primal(0), b.primal(0)
    np.testing.assert_array_equal(pa["p"], pb["p"])
    np.testing.assert_array_equal(pa["cost"], pb["cost"])
