"""The learned coarse-step surrogate end to end on the GPU: network gradients against the
FP64 oracle, training on snapshots the plain model generates, the judge/fallback policy,
and what the trained network gains over the coarse model without it."""
import ctypes
import json
import os

import numpy as np
import pytest
import torch

from oracle import cnn_ref
from paper_1711_04471_amd import _lib
from paper_1711_04471_amd import surrogate as S
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def _bf(a):
    """Round to BF16 (nearest even), returned as float64."""
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _oracle_params(net):
    th = net.theta.cpu().numpy()
    params = []
    for layer, cin in enumerate(S.CIN):
        wo, bo = net.offsets[layer]
        W = th[wo:bo].reshape(3, 3, 32, cin)
        W = np.transpose(W, (2, 3, 0, 1))[:S.REAL_OUT[layer], :S.REAL_IN[layer]]
        params.append((_bf(W), th[bo:bo + S.REAL_OUT[layer]].astype(np.float64)))
    return params


def test_network_gradients_match_oracle():
    """Forward + masked MSE + backward of the whole network against the oracle chain, with
    the oracle rounding to BF16 exactly where the network stores BF16 (input, weights,
    hidden activations, output gradient and hidden-layer gradients)."""
    rng = np.random.Generator(np.random.PCG64(3))
    N, H, W = 2, 24, 40
    net = S.ConvNet(seed=5)
    x = _bf(rng.standard_normal((N, 5, H, W)))
    tgt = rng.standard_normal((N, 3, H, W)).astype(np.float32)
    mask = (rng.uniform(size=(N, H, W)) < 0.8).astype(np.uint8)
    x16 = torch.zeros((N, H, W, 16), dtype=torch.bfloat16, device=DEV)
    x16[..., :5] = torch.from_numpy(np.transpose(x, (0, 2, 3, 1)).astype(np.float32)).to(DEV).to(torch.bfloat16)
    out = net.forward(x16, N, H, W)
    acts = sum(cnn_ref.activity(mask[n]).sum() for n in range(N))
    dout = torch.empty((N, H, W, 32), dtype=torch.bfloat16, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    lib = _lib.load()
    work = torch.empty(lib.sw2d_mse_workspace_bytes(), dtype=torch.uint8, device=DEV)
    one = np.ones(3, np.float32)
    gt, gm = torch.from_numpy(tgt).to(DEV), torch.from_numpy(mask).to(DEV)
    assert lib.sw2d_mse_grad(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(gt.data_ptr()),
                             one.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.c_void_p(gm.data_ptr()),
                             N, H, W, ctypes.c_float(1.0 / acts), ctypes.c_void_p(dout.data_ptr()),
                             ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(work.data_ptr()), work.numel(),
                             torch.cuda.current_stream().cuda_stream) == 0
    wk = torch.empty(max(lib.sw2d_wgrad_workspace_bytes(c, N, H, W) for c in (16, 32)), dtype=torch.uint8,
                     device=DEV)
    net.backward(x16, dout, N, H, W, wk)
    torch.cuda.synchronize()
    params = _oracle_params(net)
    grads_ref = [[np.zeros_like(p[0]), np.zeros_like(p[1])] for p in params]
    out_g = out.cpu().numpy()
    for n in range(N):
        # forward with BF16 storage of hidden activations
        a, acts_n, zs = x[n], [x[n]], []
        for i, (Wt, b) in enumerate(params):
            z = cnn_ref.conv3x3(a, Wt, b)
            zs.append(z)
            a = _bf(cnn_ref.relu(z)) if i < 3 else z
            acts_n.append(a)
        assert rel_l2(out_g[n], a) <= 1e-3
        act = cnn_ref.activity(mask[n])
        d = _bf(2.0 * act * (out_g[n] - tgt[n]) / acts)
        for i in range(3, -1, -1):
            gw, gb = cnn_ref.conv3x3_wgrad(acts_n[i], d)
            grads_ref[i][0] += gw
            grads_ref[i][1] += gb
            if i > 0:
                d = _bf(cnn_ref.conv3x3_dgrad(d, params[i][0]) * (acts_n[i] > 0))
    g = net.grad.cpu().numpy()
    for layer, cin in enumerate(S.CIN):
        wo, bo = net.offsets[layer]
        gw = np.transpose(g[wo:bo].reshape(3, 3, 32, cin), (2, 3, 0, 1))
        assert not gw[S.REAL_OUT[layer]:].any() and not gw[:, S.REAL_IN[layer]:].any()
        gw = gw[:S.REAL_OUT[layer], :S.REAL_IN[layer]]
        assert rel_l2(gw, grads_ref[layer][0]) <= 5e-3, (layer, rel_l2(gw, grads_ref[layer][0]))
        assert rel_l2(g[bo:bo + S.REAL_OUT[layer]], grads_ref[layer][1]) <= 5e-3, layer


FINE = 1024  # a quarter of the full configuration's side: 256^2 coarse
# the damping these reduced-size networks (input noise 0.05) were validated at; the full
# configuration's network takes the library default
SMALL_DAMPING = 0.5


@pytest.fixture(scope="module")
def small_dataset():
    return S.make_dataset([50000 + k for k in range(12)], n=FINE, pairs_per_run=100)


@pytest.fixture(scope="module")
def trained(small_dataset):
    net = S.ConvNet(seed=1)
    hist = S.Trainer(net, small_dataset, batch=4, noise=0.05).fit(epochs=24, lr=2e-3)
    return net, hist


def test_dataset_and_stats(small_dataset):
    ds = small_dataset
    assert tuple(ds.inputs.shape) == (3, 1200, 256, 256) and ds.targets.shape == ds.inputs.shape
    st = ds.stats
    assert np.all(st.in_std > 0) and np.all(st.t_std > 0)
    # the mask channel's mean is the water fraction of the coarse basins
    assert abs(st.in_mean[4] - float(ds.mask.float().mean())) < 1e-6


def test_training_reduces_the_loss(trained):
    _, hist = trained
    assert hist[-1] < 0.6 * hist[0], hist


def test_weights_round_trip(trained):
    net, _ = trained
    other = S.ConvNet(seed=9)
    other.load_state_dict(net.state_dict())
    x16 = torch.randn((1, 40, 72, 16), device=DEV).to(torch.bfloat16)
    a = net.forward(x16, 1, 40, 72).clone()
    b = other.forward(x16, 1, 40, 72)
    assert torch.equal(a, b)


def test_fallback_policy(trained):
    net, _ = trained
    case = S.fine_basin(50300, FINE)
    r = S.rollout(net, case, n_coarse=60, judge_every=20, threshold=0.0, damping=SMALL_DAMPING)
    assert r.fallbacks == 3 and len(r.rmse) == 3
    r = S.rollout(net, case, n_coarse=60, judge_every=20, threshold=1e9, damping=SMALL_DAMPING)
    assert r.fallbacks == 0
    # a corrupted network is caught by the judge and replaced by the fine model
    bad = S.ConvNet(seed=2)
    bad.load_state_dict(net.state_dict())
    bad.theta.mul_(25.0)
    bad.cast()
    r = S.rollout(bad, case, n_coarse=60, judge_every=20, threshold=1e-3, damping=SMALL_DAMPING)
    assert r.fallbacks >= 1 and not all(x <= 1e-3 for x in r.rmse)


def test_trained_network_gains_over_coarse_only(trained):
    """Held-out basins: eta RMSE after 20 coarse steps (80 fine) from the restricted fine
    state, with the learned (damped) correction against the coarse model alone: below it on
    every basin, and by 8 % on average. (The full configuration's gain at every checkpoint of
    a whole rollout is asserted for the default network, which runs every fifth step.)"""
    net, _ = trained
    ratios = []
    for seed in (50200, 50201, 50202, 50203):
        case = S.fine_basin(seed, FINE)
        base = S.rollout(None, case, n_coarse=20, judge_every=20, threshold=1e9).rmse[0]
        cnn = S.rollout(net, case, n_coarse=20, judge_every=20, threshold=1e9, damping=SMALL_DAMPING).rmse[0]
        ratios.append(cnn / base)
    print(json.dumps({"rmse_ratio_cnn_over_coarse": ratios}), flush=True)
    assert np.mean(ratios) < 0.92 and max(ratios) < 1.0, ratios


@pytest.fixture(scope="module")
def trained_every5():
    """A network trained on targets five coarse steps ahead (lead = 20 fine steps)."""
    ds = S.make_dataset([50000 + k for k in range(12)], n=FINE, pairs_per_run=100, lead=20)
    net = S.ConvNet(seed=1)
    S.Trainer(net, ds, batch=4, noise=0.05).fit(epochs=24, lr=2e-3)
    return net


def test_network_every_fifth_step_gains_over_coarse_only(trained_every5):
    """The network run before every fifth coarse step, its output correcting the state five
    steps later: eta RMSE after 20 coarse steps on held-out basins against the coarse model
    alone, as for the every-step network. Measured when this bar was set: ratios 0.62-0.86,
    mean 0.75."""
    ratios = []
    for seed in (50200, 50201, 50202, 50203):
        case = S.fine_basin(seed, FINE)
        base = S.rollout(None, case, n_coarse=20, judge_every=20, threshold=1e9).rmse[0]
        cnn = S.rollout(trained_every5, case, n_coarse=20, judge_every=20, threshold=1e9, correct_every=5,
                        damping=SMALL_DAMPING).rmse[0]
        ratios.append(cnn / base)
    print(json.dumps({"rmse_ratio_cnn_every5_over_coarse": ratios}), flush=True)
    assert np.mean(ratios) < 0.85 and max(ratios) < 0.95, ratios


def test_advance_equals_the_layer_by_layer_steps(trained):
    """The one-call corrected steps (one kernel for the network, the coarse step, the
    correction) give bitwise the state of the layer-by-layer path step by step."""
    net, _ = trained
    case = S.fine_basin(50301, FINE)
    fine = S.Sw2d.from_case(case)
    st = net.stats
    mean_a, mp = S._fptr(st.in_mean)
    std_a, sp = S._fptr(st.in_std)
    tstd_a, tp = S._fptr(st.t_std * 0.5)
    a, b = S.Coarse(fine, case), S.Coarse(fine, case)
    for _ in range(7):
        e, u, v = a.sim.state()
        hidden = net.forward_hidden_raw(e, u, v, a.H, a.mask, a.ny, a.nx, mp, sp)
        a.sim.step(1)
        e, u, v = a.sim.state()
        net.correct(hidden, e, u, v, a.mask, a.ny, a.nx, tp)
    net.advance(b.sim, 7, b.H, b.mask, mp, sp, tp)
    torch.cuda.synchronize()
    for x, y in zip(a.sim.state(), b.sim.state()):
        assert torch.equal(x, y)
    assert a.sim.steps_done == b.sim.steps_done == 7
    a.sim.close()
    b.sim.close()
    fine.close()


FULL = 4096  # the full configuration: 4096^2 fine, 1024^2 coarse


@pytest.fixture(scope="module")
def trained_full():
    """The benchmark's network: 2000 snapshot pairs from 20 plain 4096^2 runs (seeds
    50000-50019), targets five coarse steps ahead, input noise 0.3, 36 epochs."""
    ds = S.make_dataset([50000 + k for k in range(20)], n=FULL, pairs_per_run=100, every=20, lead=20)
    net = S.ConvNet(seed=1)
    S.Trainer(net, ds, batch=4, noise=0.3).fit(epochs=36, lr=2e-3)
    del ds
    torch.cuda.empty_cache()
    return net


def test_full_configuration_gains_at_every_checkpoint(trained_full):
    """4096^2 fine -> 1024^2 coarse, the network before every fifth coarse step, 500 coarse
    steps (2000 fine) judged every 50 with the threshold disabled, so that neither trajectory
    is ever reset: on each held-out basin the eta RMSE with the learned correction is below
    the coarse model's alone at every one of the 10 checkpoints."""
    ratios = {}
    for seed in (50200, 50201, 50202, 50203, 50204):
        case = S.fine_basin(seed, FULL)
        base = S.rollout(None, case, n_coarse=500, judge_every=50, threshold=1e9).rmse
        cnn = S.rollout(trained_full, case, n_coarse=500, judge_every=50, threshold=1e9, correct_every=5).rmse
        assert len(base) == len(cnn) == 10
        assert np.all(np.isfinite(cnn)), cnn
        ratios[seed] = [round(c / b, 3) for c, b in zip(cnn, base)]
    print(json.dumps({"rmse_ratio_cnn_over_coarse_per_checkpoint": ratios}), flush=True)
    allr = np.array(list(ratios.values()))
    assert np.all(allr < 1.0), ratios
    assert allr.mean() < 0.8, ratios
