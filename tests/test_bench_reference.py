"""The benchmark's own reference pieces against the oracle: its bus-angle LP
optimum (the time-to-bound target) equals the oracle's HiGHS optimum on the
test networks and on perturbed scenarios, an infeasible instance gives NaN,
and the warm start's He initialisation draws the same weights as the
oracle's from the same generator."""
import numpy as np
import pytest

import bench
from oracle import mlp as R
from oracle import ref
from paper_2406_13191_amd import synth
from paper_2406_13191_amd import warmstart as W


@pytest.mark.parametrize("name,seed", [("tiny30", 1), ("geo300", 7)])
def test_lp_optimum_matches_oracle(name, seed):
    net, p = synth.make_network(name, seed)
    Dm, Cc, _ = synth.make_scenarios(p, 123, 3, 0.1, 0.1)
    cases = [p] + [p.replace(d=Dm[i], c=Cc[i]) for i in range(3)]
    for q in cases:
        o = ref.opt_btheta(net, q)["opt"]
        v = bench._lp_optimum(net, q)
        if o is None:
            assert np.isnan(v)
        else:
            assert v == pytest.approx(o, rel=1e-7)


def test_lp_optimum_infeasible_is_nan():
    net, p = synth.make_network("tiny30", 1)
    tight = p.replace(f_max=np.full(p.n_line, 1e-3))   # no dispatch meets these limits
    assert np.isnan(bench._lp_optimum(net, tight))


def test_he_init_matches_oracle_draws():
    dims = (30, 16, 8, 5)
    a = W.he_init(np.random.default_rng(0), dims)
    b = R.init_params(np.random.default_rng(0), dims)
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x.shape == y.shape
        np.testing.assert_array_equal(x, y)
    # N(0, 2 / fan_in): the sample variance of a wide layer is close to it
    w = W.he_init(np.random.default_rng(1), (4000, 500))[0]
    assert w.var() == pytest.approx(2.0 / 4000, rel=0.02)
