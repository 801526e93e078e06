"""Pins of the oracle's PTDF (Section 2): hand-derived current dividers on a
triangle, agreement with the input generator's independent sparse-LU
construction, KCL, the zero slack column, |H| <= 1, tree networks, scale
invariance, and the sampled-rows form against the dense one."""
import numpy as np
import pytest

from oracle import ptdf as OP
from paper_2406_13191_amd import synth


def test_triangle_equal_susceptances():
    # lines 0->1, 1->2, 0->2, slack 0.  A unit injection at bus 1 splits 2/3
    # on the direct line (flowing 1 -> 0) and 1/3 through bus 2; at bus 2,
    # 2/3 direct (2 -> 0) and 1/3 through bus 1.
    H = OP.ptdf(3, [0, 1, 0], [1, 2, 2], [5.0, 5.0, 5.0], 0)
    np.testing.assert_allclose(H[:, 0], 0.0, atol=0)
    np.testing.assert_allclose(H[:, 1], [-2 / 3, 1 / 3, -1 / 3], atol=1e-14)
    np.testing.assert_allclose(H[:, 2], [-1 / 3, -1 / 3, -2 / 3], atol=1e-14)


def test_triangle_current_divider():
    # b01 = 4 against the series path 1-2-0 of admittance 2*2/(2+2) = 1:
    # 4/5 of an injection at bus 1 takes the direct line
    H = OP.ptdf(3, [0, 1, 0], [1, 2, 2], [4.0, 2.0, 2.0], 0)
    np.testing.assert_allclose(H[:, 1], [-0.8, 0.2, -0.2], atol=1e-14)


@pytest.mark.parametrize("name,seed", [("tiny30", 1), ("geo300", 7)])
def test_matches_sparse_construction_and_kcl(name, seed):
    net, p = synth.make_network(name, seed)
    H = OP.ptdf(net.n_bus, net.fbus, net.tbus, net.b, net.slack)
    np.testing.assert_allclose(H, p.H, rtol=0, atol=1e-12)
    assert np.all(H[:, net.slack] == 0.0)
    keep = [i for i in range(net.n_bus) if i != net.slack]
    E = OP.incidence(net.n_bus, net.fbus, net.tbus)
    np.testing.assert_allclose(E[:, keep].T @ H[:, keep], np.eye(len(keep)), atol=1e-10)
    assert np.abs(H).max() <= 1.0 + 1e-12
    lines = np.array([0, 3, net.n_line // 2, net.n_line - 1])
    R = OP.ptdf_rows(net.n_bus, net.fbus, net.tbus, net.b, net.slack, lines)
    np.testing.assert_allclose(R, H[lines], rtol=0, atol=1e-12)


def test_tree_and_scale_invariance():
    rng = np.random.default_rng(3)
    nb = 40
    fb = np.array([int(rng.integers(0, i)) for i in range(1, nb)])
    tb = np.arange(1, nb)
    b = rng.uniform(5, 20, nb - 1)
    H = OP.ptdf(nb, fb, tb, b, 0)
    assert np.all(np.isclose(H, 0, atol=1e-12) | np.isclose(np.abs(H), 1, atol=1e-12))
    np.testing.assert_allclose(OP.ptdf(nb, fb, tb, 3.25 * b, 0), H, atol=1e-12)
