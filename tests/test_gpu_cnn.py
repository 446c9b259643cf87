"""GPU parity of the surrogate's building blocks against the FP64 oracle (oracle/cnn_ref.py).

Both sides see the same BF16-rounded inputs and weights; FP32 outputs are held to 1e-5
relative L2 (BF16 storage of outputs to 4e-3, the BF16 unit roundoff), weight gradients
(sums over thousands of pixels in FP32) to 1e-4.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import cnn_ref
from paper_1711_04471_amd import _lib
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")


def lib():
    return _lib.load()


def stream():
    return torch.cuda.current_stream().cuda_stream


def bf16(a):
    """Round to BF16 (nearest even) and return (torch bf16 tensor on GPU, float64 numpy)."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to(DEV), t.to(torch.float64).numpy()


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def to_nhwc(x_nchw, C):
    """[N][c][H][W] -> [N][H][W][C] zero-padded to C channels."""
    N, c, H, W = x_nchw.shape
    out = np.zeros((N, H, W, C), dtype=x_nchw.dtype)
    out[..., :c] = np.transpose(x_nchw, (0, 2, 3, 1))
    return out


def wk_layout(W, cin_pad):
    """oracle W[O][C][3][3] -> forward master layout [9][32][cin_pad] (zero padded)."""
    O, C = W.shape[:2]
    out = np.zeros((9, 32, cin_pad))
    out[:, :O, :C] = np.transpose(W, (2, 3, 0, 1)).reshape(9, O, C)
    return out


def check(rc):
    assert rc == 0, (rc, lib().sw2d_last_hip_error())


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(7))


def test_restrict4(rng):
    from paper_1711_04471_amd import inputs
    c = inputs.seeded_basin("r", 136, 104, 500.0, seed=12, n_bumps=4, steps=1, border=4)
    c.u = rng.uniform(-0.3, 0.3, c.u.shape).astype(np.float32)
    c.v = rng.uniform(-0.3, 0.3, c.v.shape).astype(np.float32)
    g = [torch.as_tensor(a).to(DEV) for a in (c.eta, c.u, c.v, c.H, c.mask)]
    ny, nx = c.ny // 4, c.nx // 4
    out = [torch.empty((ny, nx), dtype=torch.float32, device=DEV) for _ in range(4)]
    mc = torch.empty((ny, nx), dtype=torch.uint8, device=DEV)
    check(lib().sw2d_restrict4(*map(ptr, g), c.nx, c.ny, *map(ptr, out), ptr(mc), stream()))
    torch.cuda.synchronize()
    ref = cnn_ref.restrict4(c.eta, c.u, c.v, c.H, c.mask)
    assert np.array_equal(mc.cpu().numpy(), ref[4])
    for got, want in zip(out, ref[:4]):
        np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-6, atol=1e-7)
        assert np.array_equal(got.cpu().numpy() != 0, want != 0)


@pytest.mark.parametrize("noise", [0.0, 0.05])
def test_pack_input(rng, noise):
    H, W = 21, 37
    fields = [rng.standard_normal((H, W)).astype(np.float32) for _ in range(4)]
    mask = (rng.uniform(size=(H, W)) < 0.7).astype(np.uint8)
    mean = np.array([0.1, -0.2, 0.3, 20.0, 0.5], dtype=np.float32)
    std = np.array([0.5, 0.25, 2.0, 10.0, 0.5], dtype=np.float32)
    g = [torch.as_tensor(a).to(DEV) for a in fields] + [torch.as_tensor(mask).to(DEV)]
    out = torch.empty((H, W, 16), dtype=torch.bfloat16, device=DEV)
    mp = mean.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    sp = std.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    seed = 0x1234ABCD5678
    check(lib().sw2d_pack_input(*map(ptr, g), W, H, mp, sp, ctypes.c_float(noise), ctypes.c_uint64(seed),
                                ptr(out), stream()))
    ref = cnn_ref.normalise(*fields, mask, mean, std, noise_amp=noise, noise_seed=seed)
    got = out.float().cpu().numpy()
    want = np.transpose(ref, (1, 2, 0))[..., :5]
    # FP32 arithmetic then one BF16 rounding: within one BF16 unit of the FP64 value
    np.testing.assert_allclose(got[..., :5], want, rtol=2 ** -7, atol=1e-6)
    assert not got[..., 5:].any()


def _fwd(x_nchw, W, b, cin_pad, relu):
    N, _, H, Wd = x_nchw.shape
    xb, x64 = bf16(to_nhwc(x_nchw, cin_pad))
    master = torch.from_numpy(wk_layout(W, cin_pad).astype(np.float32)).to(DEV)
    wk = torch.empty((9, 32, cin_pad), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_cast_weights(ptr(master), cin_pad, ptr(wk), None, stream()))
    bias = torch.zeros(32, dtype=torch.float32, device=DEV)
    bias[:len(b)] = torch.from_numpy(b.astype(np.float32))
    if relu:
        out = torch.empty((N, H, Wd, 32), dtype=torch.bfloat16, device=DEV)
    else:
        out = torch.empty((N, 3, H, Wd), dtype=torch.float32, device=DEV)
    check(lib().sw2d_conv3x3_fwd(ptr(xb), cin_pad, ptr(wk), ptr(bias), int(relu), ptr(out), N, H, Wd, stream()))
    torch.cuda.synchronize()
    wq = wk.to(torch.float64).cpu().numpy()  # the BF16 weights the kernel used
    Wq = np.transpose(wq.reshape(3, 3, 32, cin_pad), (2, 3, 0, 1))[:W.shape[0], :W.shape[1]]
    return out, np.transpose(x64, (0, 3, 1, 2))[:, :W.shape[1]], Wq


@pytest.mark.parametrize("shape", [(1, 32, 32), (2, 37, 45), (1, 8, 96)])
def test_conv_forward_relu_first_layer(rng, shape):
    N, H, Wd = shape
    x = rng.standard_normal((N, 5, H, Wd))
    W = rng.standard_normal((32, 5, 3, 3)) * 0.3
    b = rng.standard_normal(32) * 0.1
    out, x64, Wq = _fwd(x, W, b, 16, True)
    got = out.float().cpu().numpy()
    for n in range(N):
        want = cnn_ref.relu(cnn_ref.conv3x3(x64[n], Wq, b.astype(np.float32)))
        g = np.transpose(got[n], (2, 0, 1))
        assert rel_l2(g, want) <= 4e-3, rel_l2(g, want)


@pytest.mark.parametrize("shape", [(1, 40, 64), (3, 17, 33)])
def test_conv_forward_hidden_and_last_layer(rng, shape):
    N, H, Wd = shape
    x = np.maximum(rng.standard_normal((N, 32, H, Wd)), 0)
    W = rng.standard_normal((32, 32, 3, 3)) * 0.1
    b = rng.standard_normal(32) * 0.1
    out, x64, Wq = _fwd(x, W, b, 32, True)
    got = out.float().cpu().numpy()
    for n in range(N):
        want = cnn_ref.relu(cnn_ref.conv3x3(x64[n], Wq, b.astype(np.float32)))
        assert rel_l2(np.transpose(got[n], (2, 0, 1)), want) <= 4e-3
    W3 = rng.standard_normal((3, 32, 3, 3)) * 0.1
    b3 = rng.standard_normal(3) * 0.1
    out, x64, Wq = _fwd(x, W3, b3, 32, False)
    got = out.cpu().numpy()
    for n in range(N):
        want = cnn_ref.conv3x3(x64[n], Wq, b3.astype(np.float32))
        assert rel_l2(got[n], want) <= 1e-5, rel_l2(got[n], want)


def test_conv_dgrad_with_relu_mask(rng):
    N, H, Wd = 2, 19, 40
    W = rng.standard_normal((32, 32, 3, 3)) * 0.1
    dy = rng.standard_normal((N, 32, H, Wd))
    act = np.maximum(rng.standard_normal((N, 32, H, Wd)), 0)
    master = torch.from_numpy(wk_layout(W, 32).astype(np.float32)).to(DEV)
    wk = torch.empty((9, 32, 32), dtype=torch.bfloat16, device=DEV)
    wd = torch.empty((9, 32, 32), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_cast_weights(ptr(master), 32, ptr(wk), ptr(wd), stream()))
    dyb, dy64 = bf16(to_nhwc(dy, 32))
    ab, a64 = bf16(to_nhwc(act, 32))
    dx = torch.empty((N, H, Wd, 32), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_conv3x3_dgrad(ptr(dyb), ptr(wd), ptr(ab), ptr(dx), N, H, Wd, stream()))
    torch.cuda.synchronize()
    Wq = np.transpose(wk.to(torch.float64).cpu().numpy().reshape(3, 3, 32, 32), (2, 3, 0, 1))
    got = dx.float().cpu().numpy()
    for n in range(N):
        want = cnn_ref.conv3x3_dgrad(np.transpose(dy64[n], (2, 0, 1)), Wq) * (np.transpose(a64[n], (2, 0, 1)) > 0)
        assert rel_l2(np.transpose(got[n], (2, 0, 1)), want) <= 4e-3


@pytest.mark.parametrize("cin,N,H,Wd", [(32, 2, 21, 70), (16, 1, 36, 64), (32, 1, 130, 200)])
def test_conv_wgrad(rng, cin, N, H, Wd):
    creal = 5 if cin == 16 else 32
    x = rng.standard_normal((N, creal, H, Wd))
    dy = rng.standard_normal((N, 32, H, Wd)) * 0.1
    xb, x64 = bf16(to_nhwc(x, cin))
    dyb, dy64 = bf16(to_nhwc(dy, 32))
    need = lib().sw2d_wgrad_workspace_bytes(cin, N, H, Wd)
    work = torch.empty(need, dtype=torch.uint8, device=DEV)
    dW = torch.empty((9, 32, cin), dtype=torch.float32, device=DEV)
    db = torch.empty(32, dtype=torch.float32, device=DEV)
    check(lib().sw2d_conv3x3_wgrad(ptr(xb), cin, ptr(dyb), N, H, Wd, ptr(dW), ptr(db), ptr(work), need, stream()))
    torch.cuda.synchronize()
    want_W = np.zeros((32, cin, 3, 3))
    want_b = np.zeros(32)
    for n in range(N):
        gw, gb = cnn_ref.conv3x3_wgrad(np.transpose(x64[n], (2, 0, 1)), np.transpose(dy64[n], (2, 0, 1)))
        want_W += gw
        want_b += gb
    got_W = np.transpose(dW.cpu().numpy().reshape(3, 3, 32, cin), (2, 3, 0, 1))
    assert rel_l2(got_W, want_W) <= 1e-4, rel_l2(got_W, want_W)
    assert rel_l2(db.cpu().numpy(), want_b) <= 1e-4


def test_mse_grad(rng):
    N, H, Wd = 2, 23, 31
    out = rng.standard_normal((N, 3, H, Wd)).astype(np.float32)
    tgt = rng.standard_normal((N, 3, H, Wd)).astype(np.float32)
    mask = (rng.uniform(size=(N, H, Wd)) < 0.8).astype(np.uint8)
    acts = [cnn_ref.activity(mask[n]) for n in range(N)]
    n_act = sum(a.sum() for a in acts)
    g_out, g_t, g_m = (torch.as_tensor(a).to(DEV) for a in (out, tgt, mask))
    d = torch.empty((N, H, Wd, 32), dtype=torch.bfloat16, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    wb = lib().sw2d_mse_workspace_bytes()
    work = torch.empty(wb, dtype=torch.uint8, device=DEV)
    scale = np.array([2.0, 0.5, 1.0], dtype=np.float32)
    check(lib().sw2d_mse_grad(ptr(g_out), ptr(g_t), scale.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ptr(g_m),
                              N, H, Wd, ctypes.c_float(1.0 / n_act), ptr(d), ptr(loss), ptr(work), wb, stream()))
    torch.cuda.synchronize()
    total = 0.0
    for n in range(N):
        L, dout = cnn_ref.masked_mse(out[n], tgt[n] * scale[:, None, None].astype(np.float64), acts[n])
        total += L * acts[n].sum()
        got = np.transpose(d[n].float().cpu().numpy(), (2, 0, 1))
        np.testing.assert_allclose(got[:3], dout * acts[n].sum() / n_act, rtol=8e-3, atol=1e-6)
        assert not got[3:].any()
    # r is formed in FP32 (target scaled in FP32), its squares summed in FP64
    assert abs(loss.item() - total) <= 1e-6 * total


def test_adam_and_casts(rng):
    n = 1000
    theta0 = rng.standard_normal(n).astype(np.float32)
    th = torch.from_numpy(theta0.copy()).to(DEV)
    m = torch.zeros(n, device=DEV)
    v = torch.zeros(n, device=DEV)
    ref_th, ref_m, ref_v = theta0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        gt = torch.from_numpy(g).to(DEV)
        check(lib().sw2d_adam(ptr(th), ptr(gt), ptr(m), ptr(v), n, t, ctypes.c_float(1e-3), ctypes.c_float(0.9),
                              ctypes.c_float(0.999), ctypes.c_float(1e-8), stream()))
        ref_th, ref_m, ref_v = cnn_ref.adam_step(ref_th, g, ref_m, ref_v, t)
    torch.cuda.synchronize()
    np.testing.assert_allclose(th.cpu().numpy(), ref_th, rtol=0, atol=2e-6)


def test_correction_and_rmse(rng):
    H, W = 33, 47
    mask = np.zeros((H, W), dtype=np.uint8)
    mask[2:-2, 3:-3] = (rng.uniform(size=(H - 4, W - 6)) < 0.85)
    e, u, v = (rng.standard_normal((H, W)).astype(np.float32) for _ in range(3))
    out = rng.standard_normal((3, H, W)).astype(np.float32)
    t_std = np.array([0.01, 0.02, 0.03], dtype=np.float32)
    ge, gu, gv, go, gm = (torch.as_tensor(a).to(DEV) for a in (e, u, v, out, mask))
    check(lib().sw2d_apply_correction(ptr(ge), ptr(gu), ptr(gv), ptr(go), ptr(gm), W, H,
                                      t_std.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), stream()))
    re, ru, rv = cnn_ref.apply_correction(e, u, v, out, t_std, mask)
    for g, r in ((ge, re), (gu, ru), (gv, rv)):
        np.testing.assert_allclose(g.cpu().numpy(), r, rtol=1e-6, atol=1e-7)
    ref = rng.standard_normal((H, W)).astype(np.float32)
    gr = torch.as_tensor(ref).to(DEV)
    s = torch.zeros(1, dtype=torch.float64, device=DEV)
    wb = lib().sw2d_rmse_workspace_bytes()
    work = torch.empty(wb, dtype=torch.uint8, device=DEV)
    check(lib().sw2d_rmse(ptr(ge), ptr(gr), ptr(gm), H * W, ptr(s), ptr(work), wb, stream()))
    torch.cuda.synchronize()
    want = cnn_ref.rmse_wet(ge.cpu().numpy(), ref, mask)
    assert abs(np.sqrt(s.item() / mask.sum()) - want) <= 1e-12 * want


def test_sub3_and_moments(rng):
    n = 5003
    a = [rng.standard_normal(n).astype(np.float32) for _ in range(3)]
    b = [rng.standard_normal(n).astype(np.float32) for _ in range(3)]
    ga, gb = [torch.as_tensor(x).to(DEV) for x in a], [torch.as_tensor(x).to(DEV) for x in b]
    out = torch.empty((3, n), dtype=torch.float32, device=DEV)
    check(lib().sw2d_sub3(*map(ptr, ga), *map(ptr, gb), n, ptr(out), stream()))
    np.testing.assert_array_equal(out.cpu().numpy(), np.stack(a) - np.stack(b))
    mask = (rng.uniform(size=n) < 0.6).astype(np.uint8)
    gm = torch.as_tensor(mask).to(DEV)
    res = torch.zeros(2, dtype=torch.float64, device=DEV)
    wb = lib().sw2d_moments_workspace_bytes()
    work = torch.empty(wb, dtype=torch.uint8, device=DEV)
    for m, sel in ((gm, mask != 0), (None, np.ones(n, bool))):
        check(lib().sw2d_moments(ptr(ga[0]), ptr(m) if m is not None else None, n, ptr(res), ptr(work), wb,
                                 stream()))
        x = a[0][sel].astype(np.float64)
        got = res.cpu().numpy()
        np.testing.assert_allclose(got, [x.sum(), (x * x).sum()], rtol=1e-12)


@pytest.mark.parametrize("shape", [(37, 45), (64, 96), (8, 33)])
def test_fused_first_and_last_layers_equal_the_unfused_path(rng, shape):
    """Layer 1 reading the raw state (packing fused in) equals pack_input + layer 1, and
    layer 4 adding its output to the state equals layer 4 + apply_correction, bit for bit;
    the unfused pieces are pinned to the oracle by the tests above."""
    H, W = shape
    fields = [rng.standard_normal((H, W)).astype(np.float32) for _ in range(4)]
    mask = np.zeros((H, W), dtype=np.uint8)
    mask[1:-1, 1:-1] = (rng.uniform(size=(H - 2, W - 2)) < 0.8)
    mean = np.array([0.1, -0.2, 0.3, 20.0, 0.5], dtype=np.float32)
    std = np.array([0.5, 0.25, 2.0, 10.0, 0.5], dtype=np.float32)
    mp = mean.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    sp = std.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    g = [torch.as_tensor(a).to(DEV) for a in fields] + [torch.as_tensor(mask).to(DEV)]
    W1 = torch.from_numpy(wk_layout(rng.standard_normal((32, 5, 3, 3)) * 0.3, 16).astype(np.float32)).to(DEV)
    wk1 = torch.empty((9, 32, 16), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_cast_weights(ptr(W1), 16, ptr(wk1), None, stream()))
    b1 = torch.from_numpy((rng.standard_normal(32) * 0.1).astype(np.float32)).to(DEV)
    # unfused: pack then layer 1
    x16 = torch.empty((H, W, 16), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_pack_input(*map(ptr, g), W, H, mp, sp, ctypes.c_float(0.0), ctypes.c_uint64(0), ptr(x16),
                                stream()))
    a1 = torch.empty((H, W, 32), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_conv3x3_fwd(ptr(x16), 16, ptr(wk1), ptr(b1), 1, ptr(a1), 1, H, W, stream()))
    f1 = torch.empty_like(a1)
    check(lib().sw2d_conv3x3_fwd_raw(*map(ptr, g), W, H, mp, sp, ptr(wk1), ptr(b1), ptr(f1), stream()))
    torch.cuda.synchronize()
    assert torch.equal(a1.view(torch.int16), f1.view(torch.int16))
    # layer 4 + correction
    W4 = torch.from_numpy(wk_layout(rng.standard_normal((3, 32, 3, 3)) * 0.1, 32).astype(np.float32)).to(DEV)
    wk4 = torch.empty((9, 32, 32), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_cast_weights(ptr(W4), 32, ptr(wk4), None, stream()))
    b4 = torch.zeros(32, dtype=torch.float32, device=DEV)
    b4[:3] = torch.from_numpy((rng.standard_normal(3) * 0.1).astype(np.float32))
    t_std = np.array([0.01, 0.02, 0.03], dtype=np.float32)
    tp = t_std.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    state = [torch.as_tensor(rng.standard_normal((H, W)).astype(np.float32)).to(DEV) for _ in range(3)]
    s2 = [t.clone() for t in state]
    out = torch.empty((1, 3, H, W), dtype=torch.float32, device=DEV)
    check(lib().sw2d_conv3x3_fwd(ptr(a1), 32, ptr(wk4), ptr(b4), 0, ptr(out), 1, H, W, stream()))
    check(lib().sw2d_apply_correction(*map(ptr, state), ptr(out), ptr(g[4]), W, H, tp, stream()))
    check(lib().sw2d_conv3x3_correct(ptr(a1), ptr(wk4), ptr(b4), tp, ptr(g[4]), *map(ptr, s2), W, H, stream()))
    torch.cuda.synchronize()
    for x, y in zip(state, s2):
        assert torch.equal(x, y)


@pytest.mark.parametrize("shape", [(1024, 1024), (37, 45), (16, 32), (17, 33), (3, 5), (130, 257)])
def test_fused_network_equals_the_layer_by_layer_chain(rng, shape):
    """The one-kernel forward (maps kept in LDS, tiles grown by the receptive field ahead of
    each layer) equals pack_input and the four layer kernels bit for bit, tile edges, image
    edges and ragged tails included; the layer kernels are pinned to the oracle above."""
    H, W = shape
    print(f"fused forward {H}x{W}", flush=True)
    fields = [rng.standard_normal((H, W)).astype(np.float32) for _ in range(4)]
    mask = (rng.uniform(size=(H, W)) < 0.8).astype(np.uint8)
    mean = np.array([0.1, -0.2, 0.3, 20.0, 0.5], dtype=np.float32)
    std = np.array([0.5, 0.25, 2.0, 10.0, 0.5], dtype=np.float32)
    mp = mean.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    sp = std.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    g = [torch.as_tensor(a).to(DEV) for a in fields] + [torch.as_tensor(mask).to(DEV)]
    wks, biases = [], []
    for cin, real_in, real_out, scale in ((16, 5, 32, 0.3), (32, 32, 32, 0.1), (32, 32, 32, 0.1), (32, 32, 3, 0.05)):
        Wm = torch.from_numpy(wk_layout(rng.standard_normal((real_out, real_in, 3, 3)) * scale, cin)
                              .astype(np.float32)).to(DEV)
        wk = torch.empty((9, 32, cin), dtype=torch.bfloat16, device=DEV)
        check(lib().sw2d_cast_weights(ptr(Wm), cin, ptr(wk), None, stream()))
        b = torch.zeros(32, dtype=torch.float32, device=DEV)
        b[:real_out] = torch.from_numpy((rng.standard_normal(real_out) * 0.1).astype(np.float32))
        wks.append(wk)
        biases.append(b)
    # layer by layer
    x = torch.empty((H, W, 16), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_pack_input(*map(ptr, g), W, H, mp, sp, ctypes.c_float(0.0), ctypes.c_uint64(0), ptr(x),
                                stream()))
    for layer in range(3):
        y = torch.empty((H, W, 32), dtype=torch.bfloat16, device=DEV)
        check(lib().sw2d_conv3x3_fwd(ptr(x), 16 if layer == 0 else 32, ptr(wks[layer]), ptr(biases[layer]), 1,
                                     ptr(y), 1, H, W, stream()))
        x = y
    ref = torch.empty((1, 3, H, W), dtype=torch.float32, device=DEV)
    check(lib().sw2d_conv3x3_fwd(ptr(x), 32, ptr(wks[3]), ptr(biases[3]), 0, ptr(ref), 1, H, W, stream()))
    # one kernel
    out = torch.full((1, 3, H, W), float("nan"), dtype=torch.float32, device=DEV)
    wk_arr = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in wks])
    b_arr = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in biases])
    check(lib().sw2d_cnn_forward(*map(ptr, g), W, H, mp, sp, wk_arr, b_arr, ptr(out), stream()))
    torch.cuda.synchronize()
    assert torch.isfinite(ref).all()
    assert torch.equal(ref.view(torch.int32), out.view(torch.int32))


# Images with more 8 x 32 output tiles than twice the workgroups the device can hold at once
# (at most 8 four-wave workgroups per CU x 256 CUs = 2048): every workgroup of the persistent
# conv grid walks two or more tiles, prefetching the next patch into registers while the
# current one is multiplied - the path every 1024^2 layer takes in training and inference.
MAX_RESIDENT = 2048
BIG = [(1, 1024, 1024), (2, 520, 1000)]


def _tiles(N, H, Wd):
    return N * ((H + 7) // 8) * ((Wd + 31) // 32)


@pytest.mark.parametrize("shape", BIG)
def test_conv_multi_tile_walk_matches_oracle(rng, shape):
    """First layer (16 padded inputs), a hidden layer (32 inputs, ReLU + BF16 store) and the
    last layer (FP32 planes) on images of 2+ tiles per workgroup, against the oracle."""
    N, H, Wd = shape
    assert _tiles(N, H, Wd) >= 2 * MAX_RESIDENT
    print(f"multi-tile conv {shape}", flush=True)
    for cin, creal, cout, relu in ((16, 5, 32, True), (32, 32, 32, True), (32, 32, 3, False)):
        x = rng.standard_normal((N, creal, H, Wd))
        if cin == 32:
            x = np.maximum(x, 0)
        W = rng.standard_normal((cout, creal, 3, 3)) * (0.3 if cin == 16 else 0.1)
        b = rng.standard_normal(cout) * 0.1
        out, x64, Wq = _fwd(x, W, b, cin, relu)
        got = out.float().cpu().numpy() if relu else out.cpu().numpy()
        for n in range(N):
            want = cnn_ref.conv3x3(x64[n], Wq, b.astype(np.float32))
            if relu:
                want = cnn_ref.relu(want)
                g = np.transpose(got[n], (2, 0, 1))
                err = rel_l2(g, want)
                assert err <= 4e-3, (cin, n, err)  # BF16 store of the output
            else:
                err = rel_l2(got[n], want)
                assert err <= 1e-5, (cin, n, err)
            print(f"  cin {cin} cout {cout} image {n}: rel-L2 {err:.3g}", flush=True)


@pytest.mark.parametrize("shape", BIG)
def test_conv_dgrad_multi_tile_walk_matches_oracle(rng, shape):
    N, H, Wd = shape
    assert _tiles(N, H, Wd) >= 2 * MAX_RESIDENT
    W = rng.standard_normal((32, 32, 3, 3)) * 0.1
    dy = rng.standard_normal((N, 32, H, Wd))
    act = np.maximum(rng.standard_normal((N, 32, H, Wd)), 0)
    master = torch.from_numpy(wk_layout(W, 32).astype(np.float32)).to(DEV)
    wk = torch.empty((9, 32, 32), dtype=torch.bfloat16, device=DEV)
    wd = torch.empty((9, 32, 32), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_cast_weights(ptr(master), 32, ptr(wk), ptr(wd), stream()))
    dyb, dy64 = bf16(to_nhwc(dy, 32))
    ab, a64 = bf16(to_nhwc(act, 32))
    dx = torch.empty((N, H, Wd, 32), dtype=torch.bfloat16, device=DEV)
    check(lib().sw2d_conv3x3_dgrad(ptr(dyb), ptr(wd), ptr(ab), ptr(dx), N, H, Wd, stream()))
    torch.cuda.synchronize()
    Wq = np.transpose(wk.to(torch.float64).cpu().numpy().reshape(3, 3, 32, 32), (2, 3, 0, 1))
    got = dx.float().cpu().numpy()
    for n in range(N):
        want = cnn_ref.conv3x3_dgrad(np.transpose(dy64[n], (2, 0, 1)), Wq) * (np.transpose(a64[n], (2, 0, 1)) > 0)
        err = rel_l2(np.transpose(got[n], (2, 0, 1)), want)
        print(f"dgrad {shape} image {n}: rel-L2 {err:.3g}", flush=True)
        assert err <= 4e-3, err


@pytest.mark.parametrize("cin", [32, 16])
def test_conv_wgrad_training_minibatch_matches_oracle(rng, cin):
    """The weight gradient at the training minibatch (4 images of 1024^2): 1024 chunks of
    16 tiles, so each of the reduction's 8 slices adds 128 partials in order."""
    N, H, Wd = 4, 1024, 1024
    creal = 5 if cin == 16 else 32
    print(f"wgrad {N}x{H}x{Wd} cin {cin}", flush=True)
    x = rng.standard_normal((N, creal, H, Wd)).astype(np.float32)
    if cin == 32:
        x = np.maximum(x, 0)
    dy = (rng.standard_normal((N, 32, H, Wd)) * 0.1).astype(np.float32)
    xb, x64 = bf16(to_nhwc(x, cin))
    dyb, dy64 = bf16(to_nhwc(dy, 32))
    del x, dy
    need = lib().sw2d_wgrad_workspace_bytes(cin, N, H, Wd)
    assert need >= 1024 * 9 * 32 * cin * 4
    work = torch.empty(need, dtype=torch.uint8, device=DEV)
    dW = torch.empty((9, 32, cin), dtype=torch.float32, device=DEV)
    db = torch.empty(32, dtype=torch.float32, device=DEV)
    check(lib().sw2d_conv3x3_wgrad(ptr(xb), cin, ptr(dyb), N, H, Wd, ptr(dW), ptr(db), ptr(work), need, stream()))
    torch.cuda.synchronize()
    want_W = np.zeros((32, cin, 3, 3))
    want_b = np.zeros(32)
    for n in range(N):
        gw, gb = cnn_ref.conv3x3_wgrad(np.transpose(x64[n], (2, 0, 1)), np.transpose(dy64[n], (2, 0, 1)))
        want_W += gw
        want_b += gb
    got_W = np.transpose(dW.cpu().numpy().reshape(3, 3, 32, cin), (2, 3, 0, 1))
    err_w, err_b = rel_l2(got_W, want_W), rel_l2(db.cpu().numpy(), want_b)
    print(f"  rel-L2 dW {err_w:.3g} db {err_b:.3g}", flush=True)
    assert err_w <= 1e-4 and err_b <= 1e-4, (err_w, err_b)
    if cin == 16:  # padded input channels carry exactly zero gradient
        assert not got_W[:, creal:].any()


def _bf16_round(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("shape", [(1024, 1024), (130, 257), (37, 45)])
def test_fused_network_matches_oracle_forward(rng, shape):
    """The one-kernel network (sw2d_cnn_forward, the kernel the rollout runs) against the
    oracle's forward pass from the raw coarse state, with the oracle storing the input and
    the hidden maps in BF16 where the kernel does. The residual comes from maps whose FP32
    and FP64 values round to neighbouring BF16 numbers (one BF16 unit, 2^-8 relative, on a
    small fraction of the entries), bounded here by 1e-3 relative L2."""
    H, W = shape
    print(f"fused forward vs oracle {H}x{W}", flush=True)
    eta = (rng.standard_normal((H, W)) * 0.3).astype(np.float32)
    u = (rng.standard_normal((H, W)) * 0.1).astype(np.float32)
    v = (rng.standard_normal((H, W)) * 0.1).astype(np.float32)
    Hd = rng.uniform(5, 50, (H, W)).astype(np.float32)
    mask = (rng.uniform(size=(H, W)) < 0.85).astype(np.uint8)
    mean = np.array([0.01, 0.0, 0.0, 25.0, 0.85], dtype=np.float32)
    std = np.array([0.3, 0.1, 0.1, 12.0, 0.36], dtype=np.float32)
    mp = mean.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    sp = std.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    g = [torch.as_tensor(a).to(DEV) for a in (eta, u, v, Hd, mask)]
    wks, biases, params = [], [], []
    for cin, real_in, real_out, scale in ((16, 5, 32, 0.3), (32, 32, 32, 0.1), (32, 32, 32, 0.1), (32, 32, 3, 0.05)):
        Wm = torch.from_numpy(wk_layout(rng.standard_normal((real_out, real_in, 3, 3)) * scale, cin)
                              .astype(np.float32)).to(DEV)
        wk = torch.empty((9, 32, cin), dtype=torch.bfloat16, device=DEV)
        check(lib().sw2d_cast_weights(ptr(Wm), cin, ptr(wk), None, stream()))
        b = torch.zeros(32, dtype=torch.float32, device=DEV)
        b[:real_out] = torch.from_numpy((rng.standard_normal(real_out) * 0.1).astype(np.float32))
        wks.append(wk)
        biases.append(b)
        torch.cuda.synchronize()
        wq = np.transpose(wk.to(torch.float64).cpu().numpy().reshape(3, 3, 32, cin), (2, 3, 0, 1))
        params.append((wq[:real_out, :real_in], b.cpu().numpy()[:real_out].astype(np.float64)))
    out = torch.full((3, H, W), float("nan"), dtype=torch.float32, device=DEV)
    wk_arr = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in wks])
    b_arr = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in biases])
    check(lib().sw2d_cnn_forward(*map(ptr, g), W, H, mp, sp, wk_arr, b_arr, ptr(out), stream()))
    torch.cuda.synchronize()
    x = _bf16_round(cnn_ref.normalise(eta, u, v, Hd, mask, mean, std))
    want, _ = cnn_ref.forward(x, params, store=_bf16_round)
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    err = rel_l2(got, want)
    print(f"  rel-L2 {err:.3g}", flush=True)
    assert err <= 1e-3, err
