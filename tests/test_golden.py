"""The stored 30-bus FP64 configuration (tests/golden/c1_tiny30.json, written
by tests/golden/make_golden.py from the oracle only): the oracle still
reproduces it, and its best bound lies within 0.1 % below the HiGHS optimum
(weak duality, Section 3)."""
import json
import os

import numpy as np
import pytest

from oracle import dual as D
from paper_2406_13191_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c1_tiny30.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_oracle_reproduces_golden(golden):
    _, p = synth.make_network("tiny30", 1)
    res = D.ascent(D.canonical(p), golden["n_iters"], alpha=golden["alpha"], rho=golden["rho"])
    np.testing.assert_allclose(res.gammas[::100], golden["gammas_every_100"], rtol=1e-12)
    assert res.best == pytest.approx(golden["best"], rel=1e-12)
    assert res.best_iter == golden["best_iter"]
    assert res.state.lam == pytest.approx(golden["final_lambda"], rel=1e-12)
    nz = [[int(i), float(res.state.mu[i])] for i in np.flatnonzero(res.state.mu)]
    assert [i for i, _ in nz] == [i for i, _ in golden["final_mu_nonzero"]]
    np.testing.assert_allclose([v for _, v in nz], [v for _, v in golden["final_mu_nonzero"]],
                               rtol=1e-12)


def test_golden_bound_within_target(golden):
    assert golden["best"] <= golden["opt_highs"]
    assert 0.0 <= golden["gap"] <= 1e-3
