"""Learned coarse-step surrogate of the 2DSW model, trained and run with the library's kernels.

The surrogate advances a 4x-coarsened state (restriction ``sw2d_restrict4``) with the same
fused step on the coarse grid (4 dx, 4 dt, so the Courant number is unchanged) and adds a
correction predicted by a small convolutional network (3x3 'same' convolutions 5 -> 32 ->
32 -> 32 -> 3, ReLU after the first three; BF16 weights and activations on the matrix
cores, FP32 accumulation and FP32 master weights). The network learns the difference
between the restricted fine state 4m fine steps later and m coarse steps from the
restricted fine state; in the rollout it runs before every m-th coarse step and its output
corrects the state m steps later (m = 1: every step). The plain fine model stays the judge: every ``judge_every`` coarse
steps it is advanced to the same time, restricted, and the RMSE of eta over coarse water
cells is measured; above the threshold the coarse state is reset from the fine one and a
fallback is counted.

PyTorch only allocates device memory and provides the stream; every arithmetic step is a
call into ``libsw2d.so``.
"""

from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib, inputs
from ._lib import check
from .judge import RolloutResult, judged_rollout  # noqa: F401  (RolloutResult: rollout's type)
from .sw2d import Sw2d

CIN = (16, 32, 32, 32)  # padded input channels per layer (5 real channels in the first)
REAL_IN = (5, 32, 32, 32)
REAL_OUT = (32, 32, 32, 3)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _fptr(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class ConvNet:
    """The correction network on one GPU: FP32 master weights in one flat buffer (with
    Adam's moments beside it), BF16 working copies in the forward and data-gradient
    layouts, and the activations of the last forward pass for the backward pass."""

    def __init__(self, seed=0, device="cuda"):
        self.dev = torch.device(device)
        self.lib = _lib.load()
        sizes, self.offsets = [], []
        off = 0
        for cin in CIN:
            w, b = 9 * 32 * cin, 32
            self.offsets.append((off, off + w))
            off += w + b
        self.n_params = off
        self.theta = torch.zeros(off, dtype=torch.float32, device=self.dev)
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.t = 0
        rng = np.random.Generator(np.random.PCG64(seed))
        host = np.zeros(off, dtype=np.float32)
        for layer, cin in enumerate(CIN):
            wo, bo = self.offsets[layer]
            w = np.zeros((9, 32, cin), dtype=np.float32)
            fan_in = 9 * REAL_IN[layer]
            scale = math.sqrt(2.0 / fan_in) * (0.1 if layer == 3 else 1.0)
            w[:, :REAL_OUT[layer], :REAL_IN[layer]] = rng.standard_normal(
                (9, REAL_OUT[layer], REAL_IN[layer])) * scale
            host[wo:bo] = w.reshape(-1)
        self.theta.copy_(torch.from_numpy(host))
        self.wk = [torch.empty((9, 32, cin), dtype=torch.bfloat16, device=self.dev) for cin in CIN]
        self.wd = [None] + [torch.empty((9, 32, 32), dtype=torch.bfloat16, device=self.dev) for _ in CIN[1:]]
        self.stats = None
        self._acts = None
        self.cast()

    @property
    def real_params(self) -> int:
        return sum(9 * i * o + o for i, o in zip(REAL_IN, REAL_OUT))

    def weight(self, layer, which="theta"):
        buf = getattr(self, which)
        wo, bo = self.offsets[layer]
        return buf[wo:bo], buf[bo:bo + 32]

    def stream(self):
        return torch.cuda.current_stream(self.dev).cuda_stream

    def cast(self):
        for layer, cin in enumerate(CIN):
            w, _ = self.weight(layer)
            check(self.lib.sw2d_cast_weights(_p(w), cin, _p(self.wk[layer]),
                                             _p(self.wd[layer]) if self.wd[layer] is not None else None,
                                             self.stream()), "sw2d_cast_weights")

    def _buffers(self, n, h, w):
        key = (n, h, w)
        if self._acts is None or self._acts[0] != key:
            mk = lambda c: torch.empty((n, h, w, c), dtype=torch.bfloat16, device=self.dev)
            self._acts = (key, [mk(32) for _ in range(3)], torch.empty((n, 3, h, w), dtype=torch.float32,
                                                                       device=self.dev),
                          [mk(32) for _ in range(2)])
        return self._acts

    def forward(self, x16, n, h, w):
        """x16: BF16 NHWC input with 16 channels. Returns the FP32 output planes [n][3][h][w]."""
        _, acts, out, _ = self._buffers(n, h, w)
        s = self.stream()
        src = x16
        for layer in range(3):
            check(self.lib.sw2d_conv3x3_fwd(_p(src), CIN[layer], _p(self.wk[layer]),
                                            _p(self.weight(layer)[1]), 1, _p(acts[layer]), n, h, w, s),
                  "sw2d_conv3x3_fwd")
            src = acts[layer]
        check(self.lib.sw2d_conv3x3_fwd(_p(src), 32, _p(self.wk[3]), _p(self.weight(3)[1]), 0, _p(out),
                                        n, h, w, s), "sw2d_conv3x3_fwd")
        return out

    def forward_hidden_raw(self, eta, u, v, H, mask, h, w, mean_ptr, std_ptr):
        """Layers 1-3 of one image straight from the raw coarse state (the input packing is
        fused into layer 1). Returns layer 3's activations for ``correct``."""
        _, acts, _, _ = self._buffers(1, h, w)
        s = self.stream()
        check(self.lib.sw2d_conv3x3_fwd_raw(_p(eta), _p(u), _p(v), _p(H), _p(mask), w, h, mean_ptr, std_ptr,
                                            _p(self.wk[0]), _p(self.weight(0)[1]), _p(acts[0]), s),
              "sw2d_conv3x3_fwd_raw")
        for layer in (1, 2):
            check(self.lib.sw2d_conv3x3_fwd(_p(acts[layer - 1]), 32, _p(self.wk[layer]),
                                            _p(self.weight(layer)[1]), 1, _p(acts[layer]), 1, h, w, s),
                  "sw2d_conv3x3_fwd")
        return acts[2]

    def forward_fused(self, eta, u, v, H, mask, h, w, mean_ptr, std_ptr):
        """All four layers of one image from the raw coarse state in one kernel (the maps stay
        on chip). Returns the FP32 output planes [1][3][h][w]."""
        _, _, out, _ = self._buffers(1, h, w)
        wk = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in self.wk])
        bias = (ctypes.c_void_p * 4)(*[self.weight(layer)[1].data_ptr() for layer in range(4)])
        check(self.lib.sw2d_cnn_forward(_p(eta), _p(u), _p(v), _p(H), _p(mask), w, h, mean_ptr, std_ptr, wk, bias,
                                        _p(out), self.stream()), "sw2d_cnn_forward")
        return out

    def advance(self, sim, nsteps, H, mask, mean_ptr, std_ptr, tstd_ptr):
        """nsteps corrected coarse steps on the coarse handle ``sim`` in one library call: the
        fused network on the state before each step, the step, then the correction."""
        _, _, out, _ = self._buffers(1, sim.ny, sim.nx)
        wk = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in self.wk])
        bias = (ctypes.c_void_p * 4)(*[self.weight(layer)[1].data_ptr() for layer in range(4)])
        check(self.lib.sw2d_surrogate_advance(sim._handle(), int(nsteps), _p(H), _p(mask), mean_ptr, std_ptr, wk, bias,
                                              tstd_ptr, _p(out)), "sw2d_surrogate_advance")

    def advance_noalloc(self, sim, nsteps, H, mask, mean_ptr, std_ptr, tstd_ptr):
        """``advance`` with the network output staged in the library's fixed device array
        instead of a buffer of this object (for callers that cannot allocate)."""
        wk = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in self.wk])
        bias = (ctypes.c_void_p * 4)(*[self.weight(layer)[1].data_ptr() for layer in range(4)])
        check(self.lib.sw2d_surrogate_advance_noalloc(sim._handle(), int(nsteps), _p(H), _p(mask), mean_ptr, std_ptr,
                                                      wk, bias, tstd_ptr), "sw2d_surrogate_advance_noalloc")

    def correct(self, hidden, eta, u, v, mask, h, w, tstd_ptr):
        """Layer 4 with its output added to the state as the correction (fused)."""
        check(self.lib.sw2d_conv3x3_correct(_p(hidden), _p(self.wk[3]), _p(self.weight(3)[1]), tstd_ptr, _p(mask),
                                            _p(eta), _p(u), _p(v), w, h, self.stream()), "sw2d_conv3x3_correct")

    def backward(self, x16, d_out, n, h, w, work):
        """Gradients of every layer into self.grad, for dL/dout = d_out (BF16 NHWC, 32 ch)."""
        _, acts, _, dz = self._buffers(n, h, w)
        s = self.stream()
        dy = d_out
        layer_in = [x16, acts[0], acts[1], acts[2]]
        for layer in range(3, -1, -1):
            gw, gb = self.weight(layer, "grad")
            cin = CIN[layer]
            need = self.lib.sw2d_wgrad_workspace_bytes(cin, n, h, w)
            assert need <= work.numel()
            check(self.lib.sw2d_conv3x3_wgrad(_p(layer_in[layer]), cin, _p(dy), n, h, w, _p(gw), _p(gb),
                                              _p(work), work.numel(), s), "sw2d_conv3x3_wgrad")
            if layer > 0:
                dx = dz[layer % 2]
                check(self.lib.sw2d_conv3x3_dgrad(_p(dy), _p(self.wd[layer]), _p(layer_in[layer]), _p(dx),
                                                  n, h, w, s), "sw2d_conv3x3_dgrad")
                dy = dx

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        check(self.lib.sw2d_adam(_p(self.theta), _p(self.grad), _p(self.m), _p(self.v), self.n_params, self.t,
                                 ctypes.c_float(lr), ctypes.c_float(beta1), ctypes.c_float(beta2),
                                 ctypes.c_float(eps), self.stream()), "sw2d_adam")
        self.cast()

    def state_dict(self):
        return {"theta": self.theta.detach().cpu(), "stats": self.stats, "t": self.t}

    def load_state_dict(self, d):
        self.theta.copy_(d["theta"].to(self.dev))
        self.stats = d["stats"]
        self.t = d["t"]
        self.cast()


@dataclass
class Stats:
    """Normalisation: per input channel (eta, u, v, H, mask) mean/std and per target
    channel std."""
    in_mean: np.ndarray
    in_std: np.ndarray
    t_std: np.ndarray


def fine_basin(seed, n=4096, dx=500.0, border=4, bumps=(2, 8)):
    """A seeded fine basin for the surrogate: n x n cells with a 4-cell land border."""
    return inputs.seeded_basin(f"fine_{n}_s{seed}", n, n, dx, seed=seed, n_bumps=bumps[0], steps=0,
                               border=border, bumps_range=bumps)


class Coarse:
    """Restriction of a fine Sw2d into coarse device buffers, and the coarse plain model."""

    def __init__(self, fine: Sw2d, case):
        self.lib = _lib.load()
        self.dev = fine.device
        self.nxf, self.nyf = case.nx, case.ny
        self.nx, self.ny = case.nx // 4, case.ny // 4
        mk = lambda dt=torch.float32: torch.empty((self.ny, self.nx), dtype=dt, device=self.dev)
        self.eta, self.u, self.v, self.H = mk(), mk(), mk(), mk()
        self.mask = mk(torch.uint8)
        self.fine_mask = fine.mask
        self.fine_H = fine.H
        self.restrict(fine)
        dx, dt = 4 * case.dx, 4 * case.dt
        self.sim = Sw2d(self.nx, self.ny, dx, dx, case.g, dt, case.eps, self.H, self.mask, self.eta, self.u,
                        self.v, device=self.dev)
        # three steps per pass on 8-row bands: on the 1024^2 coarse grid, advanced 5 steps per
        # call as the corrected rollout does, 7.6 us per step against 9.0 at two steps per pass
        # and 9.1 at four (50 steps per call: 7.2, 7.3, 7.4); the state is that of single steps
        if self.ny >= 8:
            self.sim.set_time_blocking(3, rows=8)
        self.rmse_work = torch.empty(self.lib.sw2d_rmse_workspace_bytes(), dtype=torch.uint8, device=self.dev)
        self.rmse_out = torch.zeros(1, dtype=torch.float64, device=self.dev)
        self.n_wet = int(np.count_nonzero(self.mask.cpu().numpy()))  # host-side count, once

    def restrict(self, fine: Sw2d, out=None):
        e, u, v = fine.state()
        eta, uu, vv, H, mask = out if out is not None else (self.eta, self.u, self.v, self.H, self.mask)
        check(self.lib.sw2d_restrict4(_p(e), _p(u), _p(v), _p(self.fine_H), _p(self.fine_mask), self.nxf,
                                      self.nyf, _p(eta), _p(uu), _p(vv), _p(H), _p(mask),
                                      torch.cuda.current_stream(self.dev).cuda_stream), "sw2d_restrict4")

    def rmse_eta(self, eta_ref):
        e, _, _ = self.sim.state()
        check(self.lib.sw2d_rmse(_p(e), _p(eta_ref), _p(self.mask), self.nx * self.ny, _p(self.rmse_out),
                                 _p(self.rmse_work), self.rmse_work.numel(),
                                 torch.cuda.current_stream(self.dev).cuda_stream), "sw2d_rmse")
        return math.sqrt(self.rmse_out.item() / max(self.n_wet, 1))


@dataclass
class Dataset:
    inputs: torch.Tensor   # FP32 [3][S][ny][nx]: restricted fine state (eta, u, v)
    targets: torch.Tensor  # FP32 [3][S][ny][nx]: restricted fine state lead = 4m fine steps later minus m coarse steps
    run_of: np.ndarray     # run index of each sample
    H: torch.Tensor        # FP32 [R][ny][nx]: coarse depth of each run
    mask: torch.Tensor     # uint8 [R][ny][nx]: coarse mask of each run
    stats: Stats | None = None
    gen_seconds: float = 0.0

    @property
    def samples(self) -> int:
        return int(self.inputs.shape[1])


def make_dataset(seeds, n=4096, pairs_per_run=100, every=20, lead=4, device="cuda", log=None) -> Dataset:
    """Snapshot pairs from plain fine runs: at fine steps 0, every, 2 every, ... the input is
    R(s_t) and the target R(s_{t+lead}) - C^m(R(s_t)), m = lead / 4 coarse steps of 4 dt (one
    by default)."""
    if lead <= 0 or lead % 4 or lead > every:
        raise ValueError("lead must be a positive multiple of 4 fine steps, at most every")
    dev = torch.device(device)
    lib = _lib.load()
    t0 = time.perf_counter()
    S, nc = len(seeds) * pairs_per_run, n // 4
    ins = torch.empty((3, S, nc, nc), dtype=torch.float32, device=dev)
    tgts = torch.empty_like(ins)
    Hs = torch.empty((len(seeds), nc, nc), dtype=torch.float32, device=dev)
    masks = torch.empty((len(seeds), nc, nc), dtype=torch.uint8, device=dev)
    runs = np.repeat(np.arange(len(seeds)), pairs_per_run)
    tgt = torch.empty((3, nc, nc), dtype=torch.float32, device=dev)
    k = 0
    for r, seed in enumerate(seeds):
        case = fine_basin(seed, n)
        with Sw2d.from_case(case, device=dev) as fine:
            fine.set_time_blocking(4, rows=56)  # bitwise the same states, one pass per coarse step
            co = Coarse(fine, case)
            Hs[r].copy_(co.H)
            masks[r].copy_(co.mask)
            ahead = [torch.empty_like(co.eta) for _ in range(3)] + [torch.empty_like(co.H),
                                                                  torch.empty_like(co.mask)]
            s = torch.cuda.current_stream(dev).cuda_stream
            for _ in range(pairs_per_run):
                co.restrict(fine)
                for c, f in enumerate((co.eta, co.u, co.v)):
                    ins[c, k].copy_(f)
                co.sim.set_state(co.eta, co.u, co.v, step=0)
                co.sim.step(lead // 4)
                ce, cu, cv = co.sim.state()
                fine.step(lead)
                co.restrict(fine, out=ahead)
                check(lib.sw2d_sub3(_p(ahead[0]), _p(ahead[1]), _p(ahead[2]), _p(ce), _p(cu), _p(cv), nc * nc,
                                    _p(tgt), s), "sw2d_sub3")
                for c in range(3):
                    tgts[c, k].copy_(tgt[c])
                fine.step(every - lead)
                k += 1
            co.sim.close()
        if log:
            log(f"dataset run {r} seed {seed}: {pairs_per_run} pairs")
    torch.cuda.synchronize(dev)
    ds = Dataset(ins, tgts, runs, Hs, masks)
    ds.gen_seconds = time.perf_counter() - t0
    ds.stats = compute_stats(ds)
    return ds


def _moments(x, mask=None):
    """(mean, std) of a device array through sw2d_moments (FP64 sums, fixed order)."""
    lib = _lib.load()
    dev = x.device
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    work = torch.empty(lib.sw2d_moments_workspace_bytes(), dtype=torch.uint8, device=dev)
    check(lib.sw2d_moments(_p(x), _p(mask) if mask is not None else None, x.numel(), _p(out), _p(work),
                           work.numel(), torch.cuda.current_stream(dev).cuda_stream), "sw2d_moments")
    s1, s2 = out.cpu().numpy()
    n = float(np.count_nonzero(mask.cpu().numpy())) if mask is not None else float(x.numel())
    mean = s1 / max(n, 1.0)
    return mean, math.sqrt(max(s2 / max(n, 1.0) - mean * mean, 0.0))


def compute_stats(ds: Dataset) -> Stats:
    mean, std = [], []
    for c in range(3):
        m, sd = _moments(ds.inputs[c])
        mean.append(m)
        std.append(sd)
    m, sd = _moments(ds.H)
    mean.append(m)
    std.append(sd)
    # the mask channel holds 0 / 1: its moments are the wet fraction (host-side, once)
    p = float(np.count_nonzero(ds.mask.cpu().numpy())) / ds.mask.numel()
    mean.append(p)
    std.append(math.sqrt(max(p * (1.0 - p), 0.0)))
    std = [max(x, 1e-6) for x in std]
    t_std = [max(_moments(ds.targets[c])[1], 1e-9) for c in range(3)]
    return Stats(np.array(mean, np.float32), np.array(std, np.float32), np.array(t_std, np.float32))


class Trainer:
    """Minibatch training of a ConvNet on a Dataset with the library's kernels. Inputs get
    uniform noise of amplitude ``noise`` (in normalised units) from the pack kernel, which
    makes the learned correction tolerate the drift of its own rollouts."""

    def __init__(self, net: ConvNet, ds: Dataset, batch=4, noise=0.3):
        self.net, self.ds, self.batch, self.noise = net, ds, batch, float(noise)
        self.lib = _lib.load()
        self.dev = net.dev
        _, S, ny, nx = ds.inputs.shape
        self.ny, self.nx = ny, nx
        self.x16 = torch.empty((batch, ny, nx, 16), dtype=torch.bfloat16, device=self.dev)
        self.tgt = torch.empty((batch, 3, ny, nx), dtype=torch.float32, device=self.dev)
        self.msk = torch.empty((batch, ny, nx), dtype=torch.uint8, device=self.dev)
        self.dout = torch.empty((batch, ny, nx, 32), dtype=torch.bfloat16, device=self.dev)
        need = max(self.lib.sw2d_wgrad_workspace_bytes(c, batch, ny, nx) for c in (16, 32))
        self.work = torch.empty(need, dtype=torch.uint8, device=self.dev)
        self.mse_work = torch.empty(self.lib.sw2d_mse_workspace_bytes(), dtype=torch.uint8, device=self.dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        net.stats = ds.stats
        self._tscale, self._tp = _fptr(1.0 / ds.stats.t_std)
        self._mean, self._mp = _fptr(ds.stats.in_mean)
        self._std, self._sp = _fptr(ds.stats.in_std)
        self.n_act = [self._active(ds.mask[r]) for r in range(ds.mask.shape[0])]
        self.calls = 0

    @staticmethod
    def _active(mask):
        """Active entries of the three output channels (host-side count, once per run)."""
        w = mask.cpu().numpy() != 0
        au = w[:, :-1] & w[:, 1:]
        av = w[:-1, :] & w[1:, :]
        return int(w.sum() + au.sum() + av.sum())

    def _pack(self, j, idx):
        s = self.net.stream()
        r = int(self.ds.run_of[idx])
        x = self.ds.inputs[:, idx]
        self.calls += 1
        seed = (0x5EED << 32) ^ self.calls
        check(self.lib.sw2d_pack_input(_p(x[0]), _p(x[1]), _p(x[2]), _p(self.ds.H[r]), _p(self.ds.mask[r]),
                                       self.nx, self.ny, self._mp, self._sp, ctypes.c_float(self.noise),
                                       ctypes.c_uint64(seed), _p(self.x16[j]), s), "sw2d_pack_input")
        self.msk[j].copy_(self.ds.mask[r])
        self.tgt[j].copy_(self.ds.targets[:, idx])
        return self.n_act[r]

    def step(self, idxs):
        n = len(idxs)
        n_act = sum(self._pack(j, int(i)) for j, i in enumerate(idxs))
        out = self.net.forward(self.x16, n, self.ny, self.nx)
        check(self.lib.sw2d_mse_grad(_p(out), _p(self.tgt), self._tp, _p(self.msk), n, self.ny, self.nx,
                                     ctypes.c_float(1.0 / n_act), _p(self.dout), _p(self.loss), _p(self.mse_work),
                                     self.mse_work.numel(), self.net.stream()), "sw2d_mse_grad")
        self.net.backward(self.x16, self.dout, n, self.ny, self.nx, self.work)
        return n_act

    def fit(self, epochs=1, lr=1e-3, seed=0, log=None, train_idx=None, decay=True):
        """Epochs of shuffled minibatches; returns the mean normalised loss of a sample of
        minibatches per epoch. With decay the learning rate halves after each third of the
        epochs."""
        rng = np.random.Generator(np.random.PCG64(seed))
        idx_all = np.arange(self.ds.samples) if train_idx is None else np.asarray(train_idx)
        history = []
        for ep in range(epochs):
            order = rng.permutation(idx_all)
            total, count = 0.0, 0
            lr_ep = lr * (0.5 ** (3 * ep // max(epochs, 1))) if decay else lr
            for bi, b0 in enumerate(range(0, len(order) - self.batch + 1, self.batch)):
                n_act = self.step(order[b0:b0 + self.batch])
                self.net.adam(lr=lr_ep)
                if bi % 25 == 0:
                    total += self.loss.item()
                    count += n_act
            history.append(total / max(count, 1))
            if log:
                log(f"epoch {ep}: sampled masked MSE (normalised) {history[-1]:.4g}")
        return history


def rollout(net: ConvNet | None, case, n_coarse=500, judge_every=50, threshold=1e-3, device="cuda",
            fine: Sw2d | None = None, damping=0.6, correct_every=1):
    """Advance the surrogate n_coarse coarse steps from the restricted initial state of
    `case`; the fine model judges every judge_every steps and takes over above threshold.
    With net None the coarse model runs alone (the method without the learned part).
    The correction is applied scaled by `damping` (a one-step-trained correction applied at
    full strength every step amplifies its own errors over long rollouts). correct_every = m:
    the network runs on the state before every m-th coarse step and its output corrects the
    state m steps later (a network trained with lead = 4 m fine steps)."""
    if correct_every < 1 or judge_every % correct_every:
        raise ValueError("correct_every must divide judge_every")
    dev = torch.device(device)
    lib = _lib.load()
    own_fine = fine is None
    if own_fine:
        fine = Sw2d.from_case(case, device=dev)
    co = Coarse(fine, case)
    s = torch.cuda.current_stream(dev).cuda_stream
    ref = [torch.empty_like(co.eta) for _ in range(3)] + [torch.empty_like(co.H), torch.empty_like(co.mask)]
    if net is not None:
        mean_a, mp = _fptr(net.stats.in_mean)
        std_a, sp = _fptr(net.stats.in_std)
        tstd_a, tp = _fptr(net.stats.t_std * damping)

    def advance(n):
        if net is None:
            co.sim.step(n)
        elif correct_every == 1:
            # the network sees the state before each coarse step, as in training; one kernel
            # runs all four layers and its output corrects the stepped state
            net.advance(co.sim, n, co.H, co.mask, mp, sp, tp)
        else:
            for _ in range(n // correct_every):
                e, u, v = co.sim.state()
                out = net.forward_fused(e, u, v, co.H, co.mask, co.sim.ny, co.sim.nx, mp, sp)
                co.sim.step(correct_every)
                e, u, v = co.sim.state()
                check(lib.sw2d_apply_correction(_p(e), _p(u), _p(v), _p(out), _p(co.mask), co.sim.nx, co.sim.ny,
                                                tp, s), "sw2d_apply_correction")

    def fine_advance(n):
        fine.step(n)
        co.restrict(fine, out=ref)

    def reset():
        co.sim.set_state(ref[0], ref[1], ref[2], step=co.sim.steps_done)

    res = judged_rollout(advance, fine_advance, lambda: co.rmse_eta(ref[0]), reset, n_coarse, judge_every,
                         threshold, sync=lambda: torch.cuda.synchronize(dev))
    co.sim.close()
    if own_fine:
        fine.close()
    return res
