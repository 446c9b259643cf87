"""Pins of the surrogate's FP64 oracle: the convolution against an im2col matrix product and
against torch's CPU conv2d, its gradients against torch autograd and central finite
differences, Adam against torch.optim.Adam, and the restriction against its invariants."""
import numpy as np
import pytest
import torch

from oracle import cnn_ref


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(2024))


def _im2col(x):
    C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    cols = np.empty((H * W, C * 9))
    for c in range(C):
        for ky in range(3):
            for kx in range(3):
                cols[:, c * 9 + ky * 3 + kx] = xp[c, ky:ky + H, kx:kx + W].reshape(-1)
    return cols


def test_conv_equals_im2col_matmul(rng):
    x = rng.standard_normal((5, 13, 17))
    W = rng.standard_normal((7, 5, 3, 3))
    b = rng.standard_normal(7)
    y = cnn_ref.conv3x3(x, W, b)
    ref = (_im2col(x) @ W.reshape(7, -1).T + b).T.reshape(7, 13, 17)
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv_equals_torch_conv2d(rng):
    x = rng.standard_normal((32, 21, 19))
    W = rng.standard_normal((3, 32, 3, 3))
    b = rng.standard_normal(3)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x)[None], torch.from_numpy(W),
                                     torch.from_numpy(b), padding=1)[0].numpy()
    np.testing.assert_allclose(cnn_ref.conv3x3(x, W, b), ref, rtol=1e-12, atol=1e-12)


def test_identity_kernel_copies(rng):
    x = rng.standard_normal((4, 9, 11))
    W = np.zeros((4, 4, 3, 3))
    for c in range(4):
        W[c, c, 1, 1] = 1.0
    assert np.array_equal(cnn_ref.conv3x3(x, W, np.zeros(4)), x)


def test_conv_gradients_equal_torch_autograd(rng):
    x = rng.standard_normal((6, 10, 12))
    W = rng.standard_normal((5, 6, 3, 3))
    b = rng.standard_normal(5)
    dy = rng.standard_normal((5, 10, 12))
    tx = torch.from_numpy(x).requires_grad_()
    tW = torch.from_numpy(W).requires_grad_()
    tb = torch.from_numpy(b).requires_grad_()
    torch.nn.functional.conv2d(tx[None], tW, tb, padding=1)[0].backward(torch.from_numpy(dy))
    np.testing.assert_allclose(cnn_ref.conv3x3_dgrad(dy, W), tx.grad.numpy(), rtol=1e-12, atol=1e-12)
    dW, db = cnn_ref.conv3x3_wgrad(x, dy)
    np.testing.assert_allclose(dW, tW.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, tb.grad.numpy(), rtol=1e-12, atol=1e-12)


def _net(rng, cin=5, mid=6, cout=3):
    shapes = [(mid, cin), (mid, mid), (mid, mid), (cout, mid)]
    return [(rng.standard_normal((o, i, 3, 3)) * 0.4, rng.standard_normal(o) * 0.1) for o, i in shapes]


def test_network_gradients_against_finite_differences(rng):
    x = rng.standard_normal((5, 8, 9))
    params = _net(rng)
    target = rng.standard_normal((3, 8, 9))
    act = (rng.uniform(size=(3, 8, 9)) < 0.8).astype(float)

    def loss(ps, xx=x):
        out, _ = cnn_ref.forward(xx, ps)
        return cnn_ref.masked_mse(out, target, act)[0]

    out, cache = cnn_ref.forward(x, params)
    # stay away from ReLU kinks so central differences are smooth
    assert min(np.abs(z).min() for z in cache[1][:3]) > 1e-4
    _, dout = cnn_ref.masked_mse(out, target, act)
    grads, dx = cnn_ref.backward(dout, params, cache)
    h = 1e-6
    for layer in range(4):
        W, b = params[layer]
        for idx in [(0, 0, 0, 0), (1, 2, 1, 2), (W.shape[0] - 1, W.shape[1] - 1, 2, 1)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = [p if i != layer else (Wp, b) for i, p in enumerate(params)]
            pm = [p if i != layer else (Wm, b) for i, p in enumerate(params)]
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - grads[layer][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (layer, idx)
        bp, bm = b.copy(), b.copy()
        bp[0] += h
        bm[0] -= h
        fd = (loss([p if i != layer else (W, bp) for i, p in enumerate(params)]) -
              loss([p if i != layer else (W, bm) for i, p in enumerate(params)])) / (2 * h)
        assert abs(fd - grads[layer][1][0]) <= 1e-6 * max(1.0, abs(fd)), layer
    for idx in [(0, 0, 0), (3, 4, 5), (4, 7, 8)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (loss(params, xp) - loss(params, xm)) / (2 * h)
        assert abs(fd - dx[idx]) <= 1e-6 * max(1.0, abs(fd)), idx


def test_network_gradients_equal_torch_autograd(rng):
    x = rng.standard_normal((5, 12, 10))
    params = _net(rng, mid=8)
    target = rng.standard_normal((3, 12, 10))
    act = (rng.uniform(size=(3, 12, 10)) < 0.7).astype(float)
    out, cache = cnn_ref.forward(x, params)
    L, dout = cnn_ref.masked_mse(out, target, act)
    grads, _ = cnn_ref.backward(dout, params, cache)
    tp = [(torch.from_numpy(W).requires_grad_(), torch.from_numpy(b).requires_grad_()) for W, b in params]
    a = torch.from_numpy(x)[None]
    for i, (W, b) in enumerate(tp):
        a = torch.nn.functional.conv2d(a, W, b, padding=1)
        if i < 3:
            a = torch.relu(a)
    tact = torch.from_numpy(act)
    tl = ((a[0] - torch.from_numpy(target)) ** 2 * tact).sum() / tact.sum()
    tl.backward()
    assert abs(L - tl.item()) <= 1e-12 * abs(L)
    for (dW, db), (W, b) in zip(grads, tp):
        np.testing.assert_allclose(dW, W.grad.numpy(), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_adam_equals_torch_optim(rng):
    theta0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(6)]
    t = torch.from_numpy(theta0.copy()).requires_grad_()
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = theta0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, start=1):
        t.grad = torch.from_numpy(g.copy())
        opt.step()
        th, m, v = cnn_ref.adam_step(th, g, m, v, k)
        np.testing.assert_allclose(th, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_restriction_invariants(rng):
    NY, NX = 48, 64
    mask = (rng.uniform(size=(NY, NX)) < 0.75).astype(np.uint8)
    H = rng.uniform(5, 50, size=(NY, NX))
    const = np.full((NY, NX), 0.37)
    e_c, u_c, v_c, H_c, m_c = cnn_ref.restrict4(const, const, const, H, mask)
    wet_c = m_c != 0
    assert np.allclose(e_c[wet_c], 0.37) and not e_c[~wet_c].any()
    act = cnn_ref.activity(m_c)
    assert np.allclose(u_c[act[1] != 0], 0.37) and not u_c[act[1] == 0].any()
    assert np.allclose(v_c[act[2] != 0], 0.37) and not v_c[act[2] == 0].any()
    # water volume of the coarse water blocks is preserved
    eta = rng.standard_normal((NY, NX))
    e_c, *_ = cnn_ref.restrict4(eta, eta, eta, H, mask)
    n = (mask != 0).reshape(12, 4, 16, 4).sum(axis=(1, 3))
    fine = np.where(mask != 0, eta, 0.0).reshape(12, 4, 16, 4).sum(axis=(1, 3))
    np.testing.assert_allclose((e_c * n)[wet_c], fine[wet_c], rtol=1e-13)
    # a coarse cell is water iff at least 8 of its 16 fine cells are
    assert np.array_equal(wet_c, n >= 8)


def test_restriction_hand_example():
    mask = np.ones((8, 8), dtype=np.uint8)
    mask[0:4, 0:4] = 0
    mask[0, 0:4] = 1  # 4 of 16 wet: the block is land
    eta = np.arange(64, dtype=float).reshape(8, 8)
    u = np.zeros((8, 8))
    u[4:8, 3] = [1, 2, 3, 4]  # east face of coarse cell (1, 0): mean 2.5
    e_c, u_c, v_c, H_c, m_c = cnn_ref.restrict4(eta, u, np.zeros((8, 8)), np.ones((8, 8)), mask)
    assert m_c.tolist() == [[0, 1], [1, 1]]
    assert e_c[1, 1] == np.mean(eta[4:8, 4:8]) and e_c[0, 0] == 0.0
    assert u_c[1, 0] == 2.5 and u_c[0, 0] == 0.0


def test_rmse_and_correction():
    mask = np.zeros((5, 6), dtype=np.uint8)
    mask[1:4, 1:5] = 1
    a = np.zeros((5, 6))
    assert cnn_ref.rmse_wet(a + 0.25, a, mask) == 0.25
    out = np.ones((3, 5, 6))
    e, u, v = cnn_ref.apply_correction(a, a, a, out, np.array([1.0, 2.0, 3.0]), mask)
    assert e[2, 2] == 1.0 and e[0, 0] == 0.0
    assert u[2, 2] == 2.0 and u[2, 4] == 0.0  # east neighbour of (2, 4) is land
    assert v[2, 2] == 3.0 and v[3, 2] == 0.0


def test_splitmix64_published_outputs():
    # the first three outputs of SplitMix64 for seed 0, as published with the generator
    got = [int(x) for x in cnn_ref.splitmix64(0, np.arange(3))]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = cnn_ref.splitmix_uniform(12345, np.arange(200000))
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.01 and abs(u.var() - 1 / 3) < 0.01


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


def test_normalise_hand_example():
    """Channel order, (x - mean) / std and the 0/1 water flag on a hand-worked 2 x 3 grid."""
    g = _golden("normalise_2x3.json")
    f = lambda k: np.array(g[k], dtype=np.float64)
    y = cnn_ref.normalise(f("eta"), f("u"), f("v"), f("H"), np.array(g["mask"], dtype=np.uint8),
                          f("mean"), f("std"))
    assert y.shape == (5, 2, 3)
    assert np.array_equal(y, f("expected"))


def test_normalise_noise_counters():
    """Noise goes on eta, u, v only, at SplitMix64 counter 3 p + c; pixel 0 against the
    generator's published first outputs for seed 0, every other pixel against the pinned
    generator at its counter."""
    g = _golden("normalise_2x3.json")
    f = lambda k: np.array(g[k], dtype=np.float64)
    args = (f("eta"), f("u"), f("v"), f("H"), np.array(g["mask"], dtype=np.uint8), f("mean"), f("std"))
    amp, seed = g["noise_amp"], g["noise_seed"]
    clean = cnn_ref.normalise(*args)
    noisy = cnn_ref.normalise(*args, noise_amp=amp, noise_seed=seed)
    d = (noisy - clean) / amp
    assert not d[3:].any()
    published = [int(h, 16) for h in g["splitmix64_seed0_first_outputs"]]
    for c in range(3):
        want = (published[c] >> 40) / 2.0 ** 23 - 1.0
        assert abs(d[c, 0, 0] - want) <= 1e-15 * 4, (c, d[c, 0, 0], want)
    for j in range(2):
        for i in range(3):
            p = 3 * j + i
            for c in range(3):
                want = float(cnn_ref.splitmix_uniform(seed, 3 * p + c))
                assert abs(d[c, j, i] - want) <= 1e-14, (j, i, c)
    # another seed moves every noisy entry
    other = cnn_ref.normalise(*args, noise_amp=amp, noise_seed=12345)
    assert (other[:3] != noisy[:3]).all() and np.array_equal(other[3:], clean[3:])
