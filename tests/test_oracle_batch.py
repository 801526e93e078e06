"""Pins of the batched FP64 oracle (oracle/batch.py): for every rule, the
batched ascent of instances that share a network equals the single-instance
oracle run on each instance alone (to the rounding of a different summation
order), on an LP and a QP network with load and cost scenarios."""
import numpy as np
import pytest

from oracle import batch as OB
from oracle import dual as D
from paper_2406_13191_amd import synth

RULES = [("gdm", dict(rho=0.99)), ("gdm", dict(rho=0.5, literal=True)),
         ("gdm", dict(rho=0.9, decay=0.05)), ("adam", dict(beta1=0.9, beta2=0.99)),
         ("adagrad", dict())]


@pytest.fixture(scope="module")
def nets():
    out = {}
    for name in ("geo300", "geo300q"):
        _, base = synth.make_network(name, 7)
        Dm, Cc, Q = synth.make_scenarios(base, 900, 5, 0.1, 0.1)
        out[name] = (base, Dm, Cc, Q)
    return out


@pytest.mark.parametrize("name", ["geo300", "geo300q"])
@pytest.mark.parametrize("rule,kw", RULES)
def test_batch_equals_single_instance_oracle(nets, name, rule, kw):
    base, Dm, Cc, Q = nets[name]
    KB = OB.canonical_batch(base, Dm, Cc, Q if base.is_qp else None)
    alpha = synth.STEP_RULES[name]["alpha"] * (3e3 if rule in ("adam", "adagrad") else 1.0)
    res = OB.ascent_batch(KB, 60, rule=rule, alpha=alpha, **kw)
    for i in range(Dm.shape[0]):
        K = D.canonical(base.replace(d=Dm[i], c=Cc[i], q=Q[i]))
        ref = D.ascent(K, 60, rule=rule, alpha=alpha, **kw)
        np.testing.assert_allclose(res.gammas[:, i], ref.gammas, rtol=1e-11)
        scale = max(np.abs(ref.state.mu).max(), 1.0)
        assert np.abs(res.state.mu[:, i] - ref.state.mu).max() <= 1e-10 * scale
        assert res.state.lam[i] == pytest.approx(ref.state.lam, rel=1e-11)
        assert res.state.t == ref.state.t == 60


def test_instance_view_and_dual_value(nets):
    # the canonical data of one column equal the single-instance canonical
    # data (the gather of generator-bus columns equals H C_g exactly), and the
    # batched dual value at random multipliers equals the single one
    base, Dm, Cc, Q = nets["geo300q"]
    KB = OB.canonical_batch(base, Dm, Cc, Q)
    rng = np.random.default_rng(4)
    lam = rng.uniform(10, 50, Dm.shape[0])
    mu = rng.exponential(1.0, (2 * KB.n_line, Dm.shape[0]))
    ev = OB.dual_value_batch(KB, lam, mu)
    for i in range(Dm.shape[0]):
        K = D.canonical(base.replace(d=Dm[i], c=Cc[i], q=Q[i]))
        Ki = OB.instance(KB, i)
        np.testing.assert_array_equal(Ki.C, K.C)
        np.testing.assert_allclose(Ki.d, K.d, rtol=1e-13, atol=1e-10)
        e1 = D.dual_value(K, lam[i], mu[:, i])
        assert ev.g[i] == pytest.approx(e1.g, rel=1e-12)
        np.testing.assert_allclose(ev.x[:, i], e1.x, rtol=1e-12, atol=1e-12)
        assert ev.grad_lam[i] == pytest.approx(e1.grad_lam, rel=1e-10, abs=1e-9)
