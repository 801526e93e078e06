"""The warm-start network's GPU kernels against the FP64 reference: forward
values and every gradient tensor element by element, each within twice a
first-order bound derived from the kernels' arithmetic (BF16 operands,
FP32 accumulation), plus per-tensor cosine >= 0.999 and relative l2 <=
2e-2; the Adam update; and that training reduces the loss."""
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


U32 = 2.0 ** -24
UBF = 2.0 ** -8          # bfloat16 rounding to nearest: half an ulp, relative
GELU2 = 0.8              # max |gelu''(z)| = 2 phi(0) = 0.798


def gam(k):
    """Worst-case relative error of an FP32 sum of k terms (Higham's gamma_k)."""
    return k * U32 / (1.0 - k * U32)


def elementwise_bounds(pr, Xb, T):
    """First-order bounds on |GPU - FP64 reference| per element of Y and of
    every gradient, from the kernels' arithmetic: BF16 operands (the weights
    and X are rounded in the reference too; the hidden activations H1, H2,
    dY, dZ2, dZ1 are rounded to BF16 on the GPU only), FP32 accumulation of
    each product (gamma_K), FP32 GELU and GELU' (a few ulps), FP32 column
    sums for the biases.  Propagated layer by layer with absolute values."""
    W1, b1, W2, b2, W3, b3 = pr
    Y, (X, Z1, H1, Z2, H2) = R.forward(pr, Xb)
    n = Y.size
    gp1, gp2 = np.abs(R.gelu_grad(Z1)), np.abs(R.gelu_grad(Z2))
    aX, aW1, aW2, aW3 = np.abs(Xb), np.abs(W1), np.abs(W2), np.abs(W3)
    B, I = Xb.shape
    eZ1 = gam(I) * (aX @ aW1.T) + U32 * np.abs(Z1)
    eH1 = gp1 * eZ1 + 4 * U32 * np.abs(H1) + UBF * np.abs(H1)
    eZ2 = eH1 @ aW2.T + gam(W2.shape[1]) * (np.abs(H1) @ aW2.T) + U32 * np.abs(Z2)
    eH2 = gp2 * eZ2 + 4 * U32 * np.abs(H2) + UBF * np.abs(H2)
    eY = eH2 @ aW3.T + gam(W3.shape[1]) * (np.abs(H2) @ aW3.T) + U32 * np.abs(Y)
    dY = 2.0 * (Y - T) / n
    edY = 2.0 * eY / n + U32 * np.abs(dY)
    edYb = edY + UBF * np.abs(dY)
    aH1, aH2, adY = np.abs(H1), np.abs(H2), np.abs(dY)
    e_dW3 = edYb.T @ aH2 + adY.T @ eH2 + gam(B) * (adY.T @ aH2)
    e_db3 = edY.sum(0) + gam(B) * adY.sum(0)
    dH2 = dY @ W3
    e_dH2 = edYb @ aW3 + gam(W3.shape[0]) * (adY @ aW3)
    dZ2 = dH2 * R.gelu_grad(Z2)
    e_dZ2 = e_dH2 * gp2 + np.abs(dH2) * GELU2 * eZ2 + 4 * U32 * np.abs(dZ2)
    e_dZ2b = e_dZ2 + UBF * np.abs(dZ2)
    adZ2 = np.abs(dZ2)
    e_dW2 = e_dZ2b.T @ aH1 + adZ2.T @ eH1 + gam(B) * (adZ2.T @ aH1)
    e_db2 = e_dZ2.sum(0) + gam(B) * adZ2.sum(0)
    dH1 = dZ2 @ W2
    e_dH1 = e_dZ2b @ aW2 + gam(W2.shape[0]) * (adZ2 @ aW2)
    dZ1 = dH1 * R.gelu_grad(Z1)
    e_dZ1 = e_dH1 * gp1 + np.abs(dH1) * GELU2 * eZ1 + 4 * U32 * np.abs(dZ1)
    e_dZ1b = e_dZ1 + UBF * np.abs(dZ1)
    adZ1 = np.abs(dZ1)
    e_dW1 = e_dZ1b.T @ aX + gam(B) * (adZ1.T @ aX)
    e_db1 = e_dZ1.sum(0) + gam(B) * adZ1.sum(0)
    return eY, [e_dW1, e_db1, e_dW2, e_db2, e_dW3, e_db3]


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
    eY, eg = elementwise_bounds(pr, bf16(X), T)
    worst = float(np.max(np.abs(Y - Yr) / (2 * eY + 1e-30)))
    print(f"dims {dims}: forward cos {c:.6f} rel {r:.2e}, largest error / bound {worst:.2f}",
          flush=True)
    assert c >= 0.9999 and r <= 1e-2
    # every element within twice its first-order bound
    assert np.all(np.abs(Y - Yr) <= 2 * eY + 1e-30)
    lr_, gr = R.loss_and_grads(pr, bf16(X), T)
    assert loss == pytest.approx(lr_, rel=2e-2)
    for k, (a, b) in enumerate(zip(g, gr)):
        c, r = metrics(a, b)
        a = np.asarray(a, np.float64).reshape(b.shape)
        worst = float(np.max(np.abs(a - b) / (2 * eg[k] + 1e-30)))
        print(f"  grad {k}: cos {c:.6f} rel {r:.2e}, largest error / bound {worst:.2f}",
              flush=True)
        assert c >= 0.999 and r <= 2e-2, (k, c, r)
        assert np.all(np.abs(a - b) <= 2 * eg[k] + 1e-30), (k, worst)


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
        # a second step: the moments carried from the first, bias corrections at t = 2
        m.train_step(Xd.data_ptr(), Td.data_ptr(), batch, 1e-3)
        g2 = m.get_grads()
        new2 = m.get_params()
    zeros = [np.zeros_like(p) for p in params]
    ref, m1, v1 = R.adam_step(params, [x.astype(np.float64) for x in g], zeros, zeros, 1, 1e-3)
    for a, b in zip(new, ref):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-7)
    p1 = [np.asarray(a, np.float64) for a in new]
    ref2, _, _ = R.adam_step(p1, [x.astype(np.float64) for x in g2], m1, v1, 2, 1e-3)
    for a, b in zip(new2, ref2):
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


def test_standardize_and_fold_on_device():
    """Library-side standardisation: column means and deviations against
    numpy's (a constant column keeps deviation 1), the standardisation and
    its inverse, and the folded parameters against the same algebra written
    out in FP64 here, which make the network on raw inputs equal the
    original on standardised inputs mapped back (FP64 reference forward)."""
    import torch
    A = _abi()
    rng = np.random.default_rng(4)
    dims = (12, 16, 16, 9)
    params = [p.astype(np.float32).astype(np.float64) for p in R.init_params(rng, dims)]
    params[1] = rng.normal(0, 0.1, dims[1])
    params[5] = rng.normal(0, 0.1, dims[3])
    X = rng.lognormal(0.0, 1.0, (40, dims[0]))
    X[:, 3] = 2.5
    T = rng.normal(3.0, 2.0, (40, dims[-1]))
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Td = torch.tensor(T, dtype=torch.float32, device="cuda")
    X32, T32 = X.astype(np.float32).astype(np.float64), T.astype(np.float32).astype(np.float64)
    with A.MLP(*dims, max_batch=64) as m:
        from paper_2406_13191_amd import warmstart as W
        m.set_params(params)
        sx, st = W.Standardizer.fit(m, Xd), W.Standardizer.fit(m, Td)
        Xn = sx.apply(m, Xd)
        back = sx.apply(m, Xn, inverse=True)
        mx, sxd = sx.mean.cpu().numpy(), sx.std.cpu().numpy()
        my, syd = st.mean.cpu().numpy(), st.std.cpu().numpy()
        W.fold_standardizers(m, sx, st)
        folded = [np.asarray(p, np.float64) for p in m.get_params()]
        Xn, back = Xn.cpu().numpy(), back.cpu().numpy()
    ref_std = np.where(np.arange(dims[0]) == 3, 1.0, X32.std(0))
    np.testing.assert_allclose(mx, X32.mean(0), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(sxd, ref_std, rtol=1e-6)
    np.testing.assert_allclose(my, T32.mean(0), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(syd, T32.std(0), rtol=1e-6)
    np.testing.assert_allclose(Xn, (X32 - mx) / sxd, rtol=1e-6, atol=1e-6)
    assert np.all(Xn[:, 3] == 0.0)
    np.testing.assert_allclose(back, X32, rtol=1e-6, atol=1e-6)
    mx, sxd, my, syd = (np.asarray(a, np.float64) for a in (mx, sxd, my, syd))
    W1, b1, W2, b2, W3, b3 = params
    expect = [W1 / sxd[None, :], b1 - W1 @ (mx / sxd), W2, b2, syd[:, None] * W3, syd * b3 + my]
    for k, (a, b) in enumerate(zip(folded, expect)):
        np.testing.assert_allclose(a, b, rtol=1e-6, atol=1e-6 * np.abs(b).max(), err_msg=str(k))
    ref = R.forward(params, (X32 - mx) / sxd)[0] * syd + my
    got = R.forward(folded, X32)[0]
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())
