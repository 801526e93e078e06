"""The PTDF entry point that allocates no device memory against the one that
does: two calls in a row on one device (the 2000-bus network, then a smaller
300-bus one with another slack bus, so the second call runs on a workspace
the first left dirty), each bitwise equal to dcopf_ptdf on the same input;
sizes beyond the fixed workspace are rejected before any device work."""
import numpy as np
import pytest

from paper_2406_13191_amd import synth

pytestmark = pytest.mark.gpu


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


def _both(net, slack):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    shape = (net.n_line, net.n_bus)
    ref = torch.full(shape, np.nan, dtype=torch.float64, device="cuda")
    got = torch.full(shape, np.nan, dtype=torch.float64, device="cuda")
    _abi().ptdf(net.n_bus, net.fbus, net.tbus, net.b, slack, ref.data_ptr(), stream=stream)
    _abi().ptdf_noalloc(net.n_bus, net.fbus, net.tbus, net.b, slack, got.data_ptr(),
                        stream=stream)
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_matches_allocating_entry_point():
    import torch
    big = synth.make_topology("bus2000", 2000)
    small = synth.make_topology("geo300", 300)
    for net, slack in [(big, big.slack), (small, 7)]:
        print(f"[noalloc] {net.n_bus} buses, {net.n_line} lines, slack {slack}", flush=True)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        ref, got = _both(net, slack)
        assert torch.cuda.memory_allocated() == before
        assert np.isfinite(got).all()
        assert np.array_equal(ref, got), np.abs(ref - got).max()
        assert np.all(got[:, slack] == 0.0)


def test_noalloc_rejects_sizes_beyond_its_workspace():
    import torch
    A = _abi()
    n = A.PTDF_NOALLOC_MAX_BUS + 1
    fbus = np.arange(n - 1)
    tbus = np.arange(1, n)
    H = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(A.DcopfError) as e:
        A.ptdf_noalloc(n, fbus, tbus, np.ones(n - 1), 0, H.data_ptr())
    assert e.value.status == -1 and "at most" in str(e.value)
