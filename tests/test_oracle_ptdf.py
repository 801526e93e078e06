"""PTDF invariants of the synthetic inputs (Section 2: H = Omega E (E^T Omega
E)^{-1} with a zero slack column).  These pin the data both paths consume."""
import numpy as np
import pytest

from paper_2406_13191_amd import synth


def _incidence(net):
    E = np.zeros((net.n_line, net.n_bus))
    E[np.arange(net.n_line), net.fbus] = 1.0
    E[np.arange(net.n_line), net.tbus] = -1.0
    return E


@pytest.mark.parametrize("name,seed", [("tiny30", 1), ("tiny30", 5), ("geo300", 7)])
def test_kcl_and_slack_column(name, seed):
    net, p = synth.make_network(name, seed)
    H = p.H
    assert np.all(H[:, net.slack] == 0.0)
    keep = [i for i in range(net.n_bus) if i != net.slack]
    E = _incidence(net)
    # flows of a unit injection at bus i (withdrawn at the slack) satisfy KCL:
    # E_r^T H_r = I on the non-slack buses
    np.testing.assert_allclose(E[:, keep].T @ H[:, keep], np.eye(len(keep)), atol=1e-10)
    assert np.abs(H).max() <= 1.0 + 1e-12


@pytest.mark.parametrize("name,seed", [("tiny30", 2), ("geo300", 3)])
def test_flows_match_reduced_B_solve(name, seed):
    net, p = synth.make_network(name, seed)
    rng = np.random.default_rng(seed)
    inj = rng.normal(size=net.n_bus)
    inj -= inj.mean()
    E = _incidence(net)
    B = E.T @ np.diag(net.b) @ E
    keep = [i for i in range(net.n_bus) if i != net.slack]
    theta = np.zeros(net.n_bus)
    theta[keep] = np.linalg.solve(B[np.ix_(keep, keep)], inj[keep])
    F_ref = net.b * (theta[net.fbus] - theta[net.tbus])
    np.testing.assert_allclose(p.H @ inj, F_ref, rtol=1e-10, atol=1e-10)


def test_tree_entries_and_scale_invariance():
    rng = np.random.default_rng(0)
    nb = 25
    fb = np.array([int(rng.integers(0, i)) for i in range(1, nb)])
    tb = np.arange(1, nb)
    net = synth.Network(nb, fb, tb, rng.uniform(5, 20, nb - 1), 0)
    H = synth.ptdf(net)
    # on a tree every unit transfer to the slack uses a unique path
    assert np.all(np.isclose(H, 0) | np.isclose(np.abs(H), 1))
    net2 = synth.Network(nb, fb, tb, 7.5 * net.b, 0)
    np.testing.assert_allclose(synth.ptdf(net2), H, atol=1e-12)


def test_generator_reproducible_and_sized():
    a = synth.make_problem("tiny30", 1)
    b = synth.make_problem("tiny30", 1)
    np.testing.assert_array_equal(a.H, b.H)
    np.testing.assert_array_equal(a.f_max, b.f_max)
    assert a.H.shape == (41, 30) and a.n_gen == 6
    assert abs(a.d.sum() - 0.6 * a.p_max.sum()) < 1e-9 * a.d.sum()
    assert np.sum(a.f_max < 1e4) == 5
    assert np.count_nonzero(a.d) == 20
