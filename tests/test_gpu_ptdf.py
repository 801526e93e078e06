"""PTDF construction on the HIP path (Section 2) against the FP64 oracle:
the hand-derived triangle, whole matrices on the 30- and 300-bus networks
(the latter spans five 64-blocks with a ragged tail), sampled rows of the
2000- and 10,000-bus networks against the oracle's sparse factorisation,
KCL on sampled buses of the 2000-bus network, a slack bus other than 0,
determinism, and the argument and connectivity errors."""
import numpy as np
import pytest

from oracle import ptdf as OP
from paper_2406_13191_amd import synth

pytestmark = pytest.mark.gpu


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


def gpu_ptdf(n_bus, fbus, tbus, b, slack):
    import torch
    H = torch.empty((len(fbus), n_bus), dtype=torch.float64, device="cuda")
    _abi().ptdf(n_bus, fbus, tbus, b, slack, H.data_ptr(),
                stream=torch.cuda.current_stream().cuda_stream)
    return H


def test_triangle_closed_form():
    H = gpu_ptdf(3, [0, 1, 0], [1, 2, 2], [4.0, 2.0, 2.0], 0).cpu().numpy()
    np.testing.assert_allclose(H[:, 0], 0.0, atol=0)
    np.testing.assert_allclose(H[:, 1], [-0.8, 0.2, -0.2], rtol=0, atol=1e-14)


@pytest.mark.parametrize("name,seed,slack", [("tiny30", 1, 0), ("geo300", 7, 0),
                                             ("geo300", 7, 123)])
def test_whole_matrix_matches_oracle(name, seed, slack):
    net = synth.make_topology(name, seed)
    H = gpu_ptdf(net.n_bus, net.fbus, net.tbus, net.b, slack).cpu().numpy()
    ref = OP.ptdf(net.n_bus, net.fbus, net.tbus, net.b, slack)
    err = np.abs(H - ref).max()
    print(f"{name} slack {slack}: max |H_gpu - H_oracle| = {err:.2e}", flush=True)
    assert np.all(H[:, slack] == 0.0)
    assert err <= 1e-11


@pytest.mark.parametrize("name,seed", [("bus2000", 2000), ("bus10000", 10000)])
def test_sampled_rows_full_size(name, seed):
    import torch
    net = synth.make_topology(name, seed)
    print(f"[ptdf] {name}: {net.n_bus} buses, {net.n_line} lines", flush=True)
    H = gpu_ptdf(net.n_bus, net.fbus, net.tbus, net.b, net.slack)
    rng = np.random.default_rng(seed)
    lines = np.sort(rng.choice(net.n_line, 40, replace=False))
    got = H[torch.as_tensor(lines, device="cuda")].cpu().numpy()
    ref = OP.ptdf_rows(net.n_bus, net.fbus, net.tbus, net.b, net.slack, lines)
    err = np.abs(got - ref).max()
    print(f"{name}: max |H_gpu - H_oracle| over {lines.size} sampled rows = {err:.2e}",
          flush=True)
    assert err <= 1e-10
    if name == "bus2000":
        # KCL: E_r^T H_r = I, checked on sampled buses over every line
        Hn = H.cpu().numpy()
        E = OP.incidence(net.n_bus, net.fbus, net.tbus)
        buses = np.sort(rng.choice(np.arange(1, net.n_bus), 30, replace=False))
        K = E[:, 1:].T @ Hn[:, buses]
        I = np.zeros((net.n_bus - 1, buses.size))
        I[buses - 1, np.arange(buses.size)] = 1.0
        np.testing.assert_allclose(K, I, atol=1e-9)
        assert np.abs(Hn).max() <= 1.0 + 1e-9


def test_deterministic():
    net = synth.make_topology("geo300", 7)
    a = gpu_ptdf(net.n_bus, net.fbus, net.tbus, net.b, 0).cpu().numpy()
    b = gpu_ptdf(net.n_bus, net.fbus, net.tbus, net.b, 0).cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_errors():
    A = _abi()
    with pytest.raises(A.DcopfError):          # bus index out of range
        gpu_ptdf(3, [0, 1], [1, 3], [1.0, 1.0], 0)
    with pytest.raises(A.DcopfError):          # line from a bus to itself
        gpu_ptdf(3, [0, 1], [1, 1], [1.0, 1.0], 0)
    with pytest.raises(A.DcopfError):          # non-positive susceptance
        gpu_ptdf(3, [0, 1], [1, 2], [1.0, 0.0], 0)
    with pytest.raises(A.DcopfError):          # bus 2 not connected
        gpu_ptdf(3, [0, 0], [1, 1], [1.0, 2.0], 0)
