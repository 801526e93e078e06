"""The FP64 single-instance path on the stored 30-bus configuration
(tests/golden/c1_tiny30.json, oracle-written): 5000 iterations reproduce the
stored dual values every 100 iterations, the best bound (bound tolerance
1e-7 relative) and the final multipliers (1e-5 relative)."""
import json
import os

import numpy as np
import pytest

from paper_2406_13191_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("both_schemes")]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c1_tiny30.json")


def test_fp64_path_reproduces_golden():
    from paper_2406_13191_amd import _abi
    with open(GOLDEN) as f:
        g = json.load(f)
    _, p = synth.make_network("tiny30", 1)
    n = g["n_iters"]
    with _abi.DualSolver(p, rule="gdm", alpha=g["alpha"], rho=g["rho"], precision="fp64",
                         graph_iters=100) as s:
        s.step(n)
        gam = s.gammas(0, n)
        _, lam, mp, mm = s.bound(want_multipliers=True)
    ref_g = np.asarray(g["gammas_every_100"])
    rel = np.abs(gam[::100] - ref_g) / np.maximum(np.abs(ref_g), 1.0)   # gamma_0 = 0
    print(f"worst relative deviation of gamma every 100 iterations: {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-9
    assert gam.max() == pytest.approx(g["best"], rel=1e-7)
    assert lam == pytest.approx(g["final_lambda"], rel=1e-5)
    mu = np.concatenate([mp, mm])
    ref = np.zeros_like(mu)
    for i, v in g["final_mu_nonzero"]:
        ref[i] = v
    assert np.abs(mu - ref).max() <= 1e-5 * max(np.abs(ref).max(), 1e-3 * np.max(p.c))
