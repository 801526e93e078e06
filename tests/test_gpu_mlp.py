"""The warm-start network's GPU kernels against the FP64 reference: forward
values, every gradient tensor (per-tensor cosine >= 0.999 and relative l2
<= 2e-2, the BF16 operands being the only rounding beyond FP32), the Adam
update, and that training reduces the loss."""
import numpy as np
import pytest

from oracle import mlp as R

pytestmark = pytest.mark.gpu


def _abi():
    from paper_2406_13191_amd import _abi
    return _abi


def bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    import torch
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def setup(dims, batch, seed):
    rng = np.random.default_rng(seed)
    params = R.init_params(rng, dims)
    params = [p + (rng.normal(0, 0.05, p.shape) if p.ndim == 1 else 0) for p in params]
    X = rng.normal(size=(batch, dims[0]))
    T = rng.normal(size=(batch, dims[-1]))
    return [p.astype(np.float32).astype(np.float64) for p in params], X, T


def metrics(a, b):
    a, b = np.ravel(a), np.ravel(b)
    cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
    rel = float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))
    return cos, rel


@pytest.mark.parametrize("dims,batch", [((200, 128, 96, 150), 64),
                                        ((130, 70, 90, 33), 50),
                                        ((2000, 1024, 1024, 6401), 256)])
def test_forward_and_gradients_match_reference(dims, batch):
    import torch
    A = _abi()
    params, X, T = setup(dims, batch, 3)
    with A.MLP(*dims, max_batch=max(batch, 64)) as m:
        m.set_params(params)
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        Td = torch.tensor(T, dtype=torch.float32, device="cuda")
        Yd = torch.empty((batch, dims[-1]), dtype=torch.float32, device="cuda")
        m.forward(Xd.data_ptr(), batch, Yd.data_ptr())
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy().astype(np.float64)
        loss = m.train_step(Xd.data_ptr(), Td.data_ptr(), batch, 1e-9, want_loss=True)
        g = m.get_grads()
    # the reference uses the BF16 weights and inputs the matrix cores see
    pr = [bf16(p) if p.ndim == 2 else p for p in params]
    Yr, _ = R.forward(pr, bf16(X))
    c, r = metrics(Y, Yr)
    print(f"dims {dims}: forward cos {c:.6f} rel {r:.2e}", flush=True)
    assert c >= 0.9999 and r <= 1e-2
    lr_, gr = R.loss_and_grads(pr, bf16(X), T)
    assert loss == pytest.approx(lr_, rel=2e-2)
    for k, (a, b) in enumerate(zip(g, gr)):
        c, r = metrics(a, b)
        print(f"  grad {k}: cos {c:.6f} rel {r:.2e}", flush=True)
        assert c >= 0.999 and r <= 2e-2, (k, c, r)


def test_adam_update_matches_reference():
    import torch
    A = _abi()
    dims, batch = (64, 64, 64, 32), 64
    params, X, T = setup(dims, batch, 5)
    with A.MLP(*dims, max_batch=64, beta1=0.9, beta2=0.999, eps=1e-8) as m:
        m.set_params(params)
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        Td = torch.tensor(T, dtype=torch.float32, device="cuda")
        m.train_step(Xd.data_ptr(), Td.data_ptr(), batch, 1e-3)
        g = m.get_grads()
        new = m.get_params()
    zeros = [np.zeros_like(p) for p in params]
    ref, _, _ = R.adam_step(params, [x.astype(np.float64) for x in g], zeros, zeros, 1, 1e-3)
    for a, b in zip(new, ref):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss():
    import torch
    A = _abi()
    dims, batch = (100, 128, 128, 40), 128
    rng = np.random.default_rng(9)
    Wt = rng.normal(size=(40, 100)) / 10
    X = rng.normal(size=(batch, 100))
    T = np.tanh(X @ Wt.T)
    with A.MLP(*dims, max_batch=batch) as m:
        m.set_params([p.astype(np.float32) for p in R.init_params(rng, dims)])
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        Td = torch.tensor(T, dtype=torch.float32, device="cuda")
        first = m.train_step(Xd.data_ptr(), Td.data_ptr(), batch, 1e-3, want_loss=True)
        for _ in range(300):
            last = m.train_step(Xd.data_ptr(), Td.data_ptr(), batch, 1e-3, want_loss=False)
        last = m.train_step(Xd.data_ptr(), Td.data_ptr(), batch, 1e-3, want_loss=True)
    print(f"loss {first:.4e} -> {last:.4e}", flush=True)
    assert last < 0.1 * first
