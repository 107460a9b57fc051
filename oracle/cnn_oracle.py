"""FP64 reference of the K_eff surrogate network: forward, backward, Adam.

TEST INFRASTRUCTURE ONLY (imported by the tests; never by the product path).

The surrogate is not part of the paper; it learns the map that the paper's
local problems compute (Sec. 3, Eq. tensor-kappa): a periodic log-permeability
patch -> the diagonal of its effective permeability tensor. Network:

    x  = log K - mean(log K)            (one channel, H x W, periodic)
    a1 = relu(conv3x3(x;  W1, b1))      (1 -> C channels)
    a2 = relu(conv3x3(a1; W2, b2))      (C -> C)
    a3 = relu(conv3x3(a2; W3, b3))
    a4 = relu(conv3x3(a3; W4, b4))
    p  = mean over pixels of a4         (C)
    z  = [p, mean(log K)]               (C + 1)
    h  = relu(M1 z + c1)                (hidden)
    y  = M2 h + c2                      (2: log kxx - mean, log kyy - mean)

Convolutions wrap around the patch edges (circular padding), matching the
periodic local problems, so the network is exactly invariant to circular
shifts of the patch. Loss: mean over the batch and both outputs of the
squared error. Weight layout: W[tap, c_in, c_out] with tap = 3 (dy + 1) +
(dx + 1), and out[y, x] = sum_tap in[y + dy, x + dx] W[tap].
Written with plain array loops over the nine taps (np.roll does the wrap).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def init_params(C: int = 32, hidden: int = 32, seed: int = 0) -> dict:
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    p = {}
    cin = 1
    for l in range(1, 5):
        p[f"W{l}"] = rng.standard_normal((9, cin, C)) * np.sqrt(2.0 / (9 * cin))
        p[f"b{l}"] = np.zeros(C)
        cin = C
    p["M1"] = rng.standard_normal((hidden, C + 1)) * np.sqrt(2.0 / (C + 1))
    p["c1"] = np.zeros(hidden)
    p["M2"] = rng.standard_normal((2, hidden)) * np.sqrt(1.0 / hidden)
    p["c2"] = np.zeros(2)
    return p


def _shift(a, dy, dx):
    """a[..., y + dy, x + dx] with periodic wrap; a is [B, H, W, C]."""
    return np.roll(a, shift=(-dy, -dx), axis=(1, 2))


def conv3x3(a, W, b):
    """[B, H, W, Cin] -> [B, H, W, Cout], circular padding."""
    out = np.zeros(a.shape[:3] + (W.shape[2],))
    for t, (dy, dx) in enumerate(TAPS):
        out += _shift(a, dy, dx) @ W[t]
    return out + b


def conv3x3_backward(a, W, g):
    """Gradients of sum(g * conv3x3(a, W, b)) w.r.t. a, W and b."""
    da = np.zeros_like(a)
    dW = np.zeros_like(W)
    for t, (dy, dx) in enumerate(TAPS):
        sa = _shift(a, dy, dx)
        dW[t] = np.einsum("bhwi,bhwo->io", sa, g)
        # out[y, x] uses a[y + dy, x + dx]: send g back to that pixel
        da += _shift(g @ W[t].T, -dy, -dx)
    db = g.sum(axis=(0, 1, 2))
    return da, dW, db


def forward(p: dict, logk: np.ndarray):
    """logk: [B, H, W] FP64. Returns (y [B, 2], cache)."""
    logk = np.asarray(logk, dtype=np.float64)
    m = logk.mean(axis=(1, 2))
    x = (logk - m[:, None, None])[..., None]
    acts = [x]
    pre = []
    a = x
    for l in range(1, 5):
        z = conv3x3(a, p[f"W{l}"], p[f"b{l}"])
        pre.append(z)
        a = np.maximum(z, 0.0)
        acts.append(a)
    pool = a.mean(axis=(1, 2))
    zin = np.concatenate([pool, m[:, None]], axis=1)
    hpre = zin @ p["M1"].T + p["c1"]
    h = np.maximum(hpre, 0.0)
    y = h @ p["M2"].T + p["c2"]
    return y, dict(acts=acts, pre=pre, zin=zin, hpre=hpre, h=h, m=m)


def loss(y, target):
    return float(np.mean((y - target) ** 2))


def backward(p: dict, cache: dict, y, target) -> dict:
    """Gradients of loss(y, target) w.r.t. every parameter."""
    B = y.shape[0]
    g = {}
    dy = 2.0 * (y - target) / (B * y.shape[1])
    g["M2"] = dy.T @ cache["h"]
    g["c2"] = dy.sum(axis=0)
    dh = dy @ p["M2"]
    dhpre = dh * (cache["hpre"] > 0)
    g["M1"] = dhpre.T @ cache["zin"]
    g["c1"] = dhpre.sum(axis=0)
    dzin = dhpre @ p["M1"]
    C = p["W4"].shape[2]
    dpool = dzin[:, :C]
    a4 = cache["acts"][4]
    H, W = a4.shape[1], a4.shape[2]
    da = np.broadcast_to(dpool[:, None, None, :] / (H * W), a4.shape).copy()
    for l in range(4, 0, -1):
        dz = da * (cache["pre"][l - 1] > 0)
        da, g[f"W{l}"], g[f"b{l}"] = conv3x3_backward(cache["acts"][l - 1], p[f"W{l}"], dz)
    return g


def adam_step(p: dict, g: dict, state: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8) -> None:
    """One Adam update (Kingma and Ba) in place; state holds m, v and t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def flops_forward(H=32, W=32, C=32, hidden=32) -> int:
    """Multiply-adds x 2 of one forward pass."""
    n = H * W
    conv = 2 * n * 9 * (1 * C + 3 * C * C)
    mlp = 2 * (hidden * (C + 1) + 2 * hidden)
    return conv + mlp
