"""The paper's QP dual with s iterated (Section 3.2, eq. QP_finalgamma) on
the HIP path, an ablation of the closed-form maximum over s: FP64
trajectories against the oracle's, the exact bound at the same iterate never
below the iterated dual's value, identity with the closed form on an LP
network (where s stays 0), and the option checks."""
import numpy as np
import pytest

from oracle import dual as D
from oracle.qp_s import ascent_s
from paper_2406_13191_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("both_schemes")]


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


_P = {}


def prob(name, seed):
    if (name, seed) not in _P:
        _P[(name, seed)] = synth.make_problem(name, seed)
    return _P[(name, seed)]


@pytest.mark.parametrize("name,seed", [("geo300q", 7), ("tiny30", 1)])
def test_fp64_trajectory_matches_oracle(name, seed):
    p = prob(name, seed)
    if not p.is_qp:
        rng = np.random.default_rng(5)
        p = p.replace(q=rng.uniform(0.001, 0.05, p.n_gen))
    K = D.canonical(p)
    n, alpha, rho = 300, 1e-4, 0.99
    with _abi().DualSolver(p, rule="gdm", alpha=alpha, rho=rho, precision="fp64",
                           qp_dual="iterated") as s:
        s.step(n)
        g = s.gammas(0, n)
        bound, lam, mp, mm = s.bound(want_multipliers=True)
    o = ascent_s(K, n, alpha=alpha, rho=rho)
    rel = np.abs(g - o.gammas) / np.maximum(np.abs(o.gammas), 1.0)
    print(f"{name}: worst relative gamma deviation {rel.max():.2e}", flush=True)
    assert rel.max() <= 1e-9
    lam_o, mu_o = o.state.lam, o.state.mu
    assert lam == pytest.approx(lam_o, rel=1e-8, abs=1e-8)
    mu = np.concatenate([mp, mm])
    assert np.abs(mu - mu_o).max() <= 1e-8 * max(np.abs(mu_o).max(), 1.0)
    # the exact (closed-form) dual at the same lambda, mu is at least the
    # iterated dual's value there
    ev = D.dual_value(K, lam_o, mu_o)
    assert bound == pytest.approx(ev.g, rel=1e-11)


def test_exact_bound_not_below_monitor_fp32_qp():
    p = prob("geo300q", 7)
    with _abi().DualSolver(p, rule="gdm", alpha=1e-4, rho=0.99, precision="fp32",
                           qp_dual="iterated", graph_iters=20) as s:
        for _ in range(5):
            s.step(100)
            k = s.info()["iters"]
            b = s.bound()                          # exact dual at iterate k
            s.step(1)
            gk = s.gammas(k, 1)[0]                 # iterated dual at iterate k
            assert b >= gk - 1e-9 * abs(b)


def test_lp_network_identical_to_closed_form():
    p = prob("geo300", 7)
    kw = dict(rule="gdm", alpha=3e-4, rho=0.99, precision="fp32")
    with _abi().DualSolver(p, **kw) as a, _abi().DualSolver(p, qp_dual="iterated", **kw) as b:
        a.step(200)
        b.step(200)
        np.testing.assert_array_equal(a.gammas(0, 200), b.gammas(0, 200))
        assert a.bound() == b.bound()


def test_option_checks():
    A = _abi()
    p = prob("geo300q", 7)
    for kw in (dict(rule="adam"), dict(decay=1e-3), dict(literal=True)):
        with pytest.raises(A.DcopfError):
            A.DualSolver(p, alpha=1e-4, qp_dual="iterated", **kw)
    with A.DualSolver(p, rule="gdm", alpha=1e-4, rho=0.99, qp_dual="iterated") as s:
        s.step(5)
        with pytest.raises(A.DcopfError):
            s.get_state()
        with pytest.raises(A.DcopfError):
            s.time_phases(2)
