"""FP64 numpy oracle for the learned coarse-step surrogate (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg may import
this module. It shares no code with the HIP path.

The surrogate advances a 4x-coarsened state of the 2DSW model (the model of Sect. 6.2)
with the same explicit step on the coarse grid and adds a correction predicted by a small
convolutional network. Every function below is the plain definition, written with
whole-array numpy operations and no blocking or fusion:

* ``restrict4``  - 4x4 block restriction of (eta, u, v, H, mask);
* ``conv3x3`` / ``conv3x3_dgrad`` / ``conv3x3_wgrad`` - 'same' 3x3 cross-correlation with
  zero padding and its two gradients, derived by hand from
  y[o, p] = b[o] + sum_c sum_(dy,dx) W[o, c, dy+1, dx+1] x[c, p + (dy, dx)]; for each tap the
  sum over channels (or, for the weight gradient, over pixels) is one library matrix
  product (numpy.tensordot);
* ``forward`` / ``backward`` - the 4-layer network (ReLU after layers 1-3);
* ``masked_mse`` - mean squared error over the active entries of each output channel;
* ``adam_step`` - Adam (Kingma & Ba, 2015) with bias correction;
* ``apply_correction`` and ``rmse_wet``.

Layouts: feature maps are [C][H][W] (row-major, H = ny rows, W = nx columns), weights are
[C_out][C_in][3][3].
"""

from __future__ import annotations

import numpy as np


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# --------------------------------------------------------------------------- restriction
def restrict4(eta, u, v, H, mask):
    """4x4 block restriction of a fine state to the coarse grid.

    eta_c: mean of eta over the water cells of the block; H_c likewise; a coarse cell is
    water when at least 8 of its 16 fine cells are; u_c: mean of the 4 fine u on the
    coarse cell's east face; v_c: mean of the 4 fine v on its north face; coarse land
    cells and inactive coarse faces are exactly zero.
    """
    eta, u, v, H = _f64(eta), _f64(u), _f64(v), _f64(H)
    wet = np.asarray(mask) != 0
    NY, NX = eta.shape
    assert NY % 4 == 0 and NX % 4 == 0
    ny, nx = NY // 4, NX // 4
    blk = lambda a: a.reshape(ny, 4, nx, 4)
    n = blk(wet.astype(np.float64)).sum(axis=(1, 3))
    s_eta = blk(np.where(wet, eta, 0.0)).sum(axis=(1, 3))
    s_H = blk(np.where(wet, H, 0.0)).sum(axis=(1, 3))
    mask_c = n >= 8
    safe = np.where(n > 0, n, 1.0)
    eta_c = np.where(mask_c, s_eta / safe, 0.0)
    H_c = np.where(n > 0, s_H / safe, 0.0)
    u_c = u[:, 3::4].reshape(ny, 4, nx).mean(axis=1)
    v_c = v[3::4, :].reshape(ny, nx, 4).mean(axis=2)
    au = np.zeros((ny, nx), dtype=bool)
    au[:, :-1] = mask_c[:, :-1] & mask_c[:, 1:]
    av = np.zeros((ny, nx), dtype=bool)
    av[:-1, :] = mask_c[:-1, :] & mask_c[1:, :]
    u_c = np.where(au, u_c, 0.0)
    v_c = np.where(av, v_c, 0.0)
    return eta_c, u_c, v_c, H_c, mask_c.astype(np.uint8)


def activity(mask):
    """Per-channel activity of a state: (wet cells, active u faces, active v faces)."""
    wet = np.asarray(mask) != 0
    au = np.zeros_like(wet)
    au[:, :-1] = wet[:, :-1] & wet[:, 1:]
    av = np.zeros_like(wet)
    av[:-1, :] = wet[:-1, :] & wet[1:, :]
    return np.stack([wet, au, av]).astype(np.float64)


# --------------------------------------------------------------------------- convolution
def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1)))


def conv3x3(x, W, b):
    """y[o] = b[o] + sum over taps (ky, kx) of W[:, :, ky, kx] applied to x shifted by (ky-1, kx-1)."""
    x, W, b = _f64(x), _f64(W), _f64(b)
    C, Hh, Ww = x.shape
    xp = _pad(x)
    y = np.broadcast_to(b[:, None, None], (W.shape[0], Hh, Ww)).copy()
    for ky in range(3):
        for kx in range(3):
            # the sum over input channels c of one tap: a matrix product
            y += np.tensordot(W[:, :, ky, kx], xp[:, ky:ky + Hh, kx:kx + Ww], axes=([1], [0]))
    return y


def conv3x3_dgrad(dy, W):
    """dL/dx for y = conv3x3(x, W, b): every output gradient flows back through each tap."""
    dy, W = _f64(dy), _f64(W)
    O, Hh, Ww = dy.shape
    dxp = np.zeros((W.shape[1], Hh + 2, Ww + 2))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + Hh, kx:kx + Ww] += np.tensordot(W[:, :, ky, kx], dy, axes=([0], [0]))
    return dxp[:, 1:-1, 1:-1]


def conv3x3_wgrad(x, dy):
    """(dL/dW, dL/db) for y = conv3x3(x, W, b)."""
    x, dy = _f64(x), _f64(dy)
    C, Hh, Ww = x.shape
    xp = _pad(x)
    dW = np.zeros((dy.shape[0], C, 3, 3))
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.tensordot(dy, xp[:, ky:ky + Hh, kx:kx + Ww], axes=([1, 2], [1, 2]))
    return dW, dy.sum(axis=(1, 2))


def relu(z):
    return np.maximum(_f64(z), 0.0)


# --------------------------------------------------------------------------- network
def forward(x, params, store=None):
    """params: list of (W, b) for the 4 layers. Returns (output, cache of pre-activations
    and layer inputs for backward). ``store``, if given, is applied to every hidden
    activation map after its ReLU: the precision in which an implementation keeps the maps
    between layers (e.g. rounding to BF16); None keeps FP64."""
    acts = [_f64(x)]
    zs = []
    a = acts[0]
    for i, (W, b) in enumerate(params):
        z = conv3x3(a, W, b)
        zs.append(z)
        if i < len(params) - 1:
            a = relu(z)
            if store is not None:
                a = _f64(store(a))
        else:
            a = z
        acts.append(a)
    return a, (acts, zs)


def backward(dout, params, cache):
    """Gradients [(dW, db), ...] of every layer, and dL/dx, for dL/dout = dout."""
    acts, zs = cache
    grads = [None] * len(params)
    d = _f64(dout)
    for i in range(len(params) - 1, -1, -1):
        if i < len(params) - 1:
            d = d * (zs[i] > 0)
        grads[i] = conv3x3_wgrad(acts[i], d)
        d = conv3x3_dgrad(d, params[i][0])
    return grads, d


def masked_mse(out, target, act):
    """L = sum(act (out - target)^2) / sum(act); returns (L, dL/dout)."""
    out, target, act = _f64(out), _f64(target), _f64(act)
    n = max(act.sum(), 1.0)
    r = act * (out - target)
    return float((r * r).sum() / n), 2.0 * r / n


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step). Returns (theta, m, v)."""
    theta, grad, m, v = _f64(theta), _f64(grad), _f64(m), _f64(v)
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --------------------------------------------------------------------------- surrogate glue
_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed, i):
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) output for counter i: the state
    seed + (i + 1) * golden gamma run through the variant-13 finaliser (mod 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(i, dtype=np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix_uniform(seed, i):
    """Top 24 bits of splitmix64 as a uniform number in [-1, 1)."""
    return (splitmix64(seed, i) >> np.uint64(40)).astype(np.float64) / 2.0 ** 23 - 1.0


def normalise(eta, u, v, H, mask, mean, std, noise_amp=0.0, noise_seed=0):
    """The 5 input channels (eta, u, v, H, water flag), each shifted and scaled:
    (x - mean) / std, the water flag being 1 where mask is nonzero and 0 elsewhere; plus
    (training only) noise_amp * U on channels 0..2, U = splitmix_uniform(seed, 3 p + c) for
    the row-major pixel index p."""
    flag = (np.asarray(mask) != 0).astype(np.float64)
    x = np.stack([_f64(eta), _f64(u), _f64(v), _f64(H), flag])
    y = (x - _f64(mean)[:, None, None]) / _f64(std)[:, None, None]
    if noise_amp > 0.0:
        H_, W_ = y.shape[1:]
        p = np.arange(H_ * W_, dtype=np.uint64).reshape(H_, W_)
        for c in range(3):
            y[c] += noise_amp * splitmix_uniform(noise_seed, p * np.uint64(3) + np.uint64(c))
    return y


def apply_correction(eta, u, v, out, t_std, mask):
    """state += activity * (out * t_std): the network predicts a scaled increment."""
    act = activity(mask)
    d = _f64(out) * _f64(t_std)[:, None, None] * act
    return _f64(eta) + d[0], _f64(u) + d[1], _f64(v) + d[2]


def rmse_wet(eta, eta_ref, mask):
    wet = np.asarray(mask) != 0
    if not wet.any():
        return 0.0
    d = _f64(eta)[wet] - _f64(eta_ref)[wet]
    return float(np.sqrt(np.mean(d * d)))
