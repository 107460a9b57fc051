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
    s  = series/parallel features of k = exp(x) (4, below)
    z  = [p, mean(log K), s]            (C + 5)
    h  = relu(M1 z + c1)                (hidden)
    y  = M2 h + c2                      (2: log kxx - mean, log kyy - mean)

The four features are the logs of the classical series-parallel estimates of
an effective permeability of k = exp(x) (rows along x, columns along y):
    sx_lo = log mean_rows(harmonic mean along the row)
    sx_up = log harmonic mean over columns(arithmetic mean along the column)
    sy_lo = log mean_columns(harmonic mean along the column)
    sy_up = log harmonic mean over rows(arithmetic mean along the row)
(for Darcy flow they bound kxx and kyy; here they are only inputs).

Symmetry: K_eff is equivariant under the eight symmetries of the square
(pinned in the LBM oracle tests): with sym = t + 2 fx + 4 fy, output pixel
(y, x) of the transformed patch reads input pixel (v, u) where (u, v) = (x, y)
swapped if t, then u -> W-1-u if fx, v -> H-1-v if fy; a transposition
(t = 1) swaps kxx and kyy.

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


NFEAT = 5  # mean(log K) and the four series/parallel features


def transform(logk, sym):
    """Apply symmetry sym (0..7) to patches [B, H, W] (see the module text)."""
    t, fx, fy = sym & 1, (sym >> 1) & 1, (sym >> 2) & 1
    a = np.asarray(logk)
    # the mirrors act on the source indices (u, v), so they come first
    if fx:
        a = a[:, :, ::-1]
    if fy:
        a = a[:, ::-1, :]
    if t:
        a = np.swapaxes(a, 1, 2)
    return np.ascontiguousarray(a)


def series_parallel(x):
    """The four features of centred patches x [B, H, W]."""
    k = np.exp(x)
    row_h = 1.0 / np.mean(1.0 / k, axis=2)   # harmonic along x, per row
    col_a = np.mean(k, axis=1)                # arithmetic along y, per column
    col_h = 1.0 / np.mean(1.0 / k, axis=1)
    row_a = np.mean(k, axis=2)
    return np.stack([np.log(row_h.mean(axis=1)), -np.log(np.mean(1.0 / col_a, axis=1)),
                     np.log(col_h.mean(axis=1)), -np.log(np.mean(1.0 / row_a, axis=1))], axis=1)


def init_params(C: int = 32, hidden: int = 32, seed: int = 0) -> dict:
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    p = {}
    cin = 1
    for l in range(1, 5):
        p[f"W{l}"] = rng.standard_normal((9, cin, C)) * np.sqrt(2.0 / (9 * cin))
        p[f"b{l}"] = np.zeros(C)
        cin = C
    p["M1"] = rng.standard_normal((hidden, C + NFEAT)) * np.sqrt(2.0 / (C + NFEAT))
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
    """logk: [B, H, W] FP64 (already transformed, if a symmetry is used).
    Returns (y [B, 2], cache)."""
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
    zin = np.concatenate([pool, m[:, None], series_parallel(x[..., 0])], axis=1)
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


def predict_symmetric(p: dict, logk: np.ndarray, n_sym: int = 8) -> np.ndarray:
    """log K_eff prediction averaged over the first n_sym symmetries, each
    mapped back to the original axes: [B, 2]."""
    out = np.zeros((len(logk), 2))
    for sym in range(n_sym):
        y, c = forward(p, transform(logk, sym))
        pred = y + c["m"][:, None]
        out += pred[:, ::-1] if sym & 1 else pred
    return out / n_sym


def flops_forward(H=32, W=32, C=32, hidden=32) -> int:
    """Multiply-adds x 2 of one forward pass."""
    n = H * W
    conv = 2 * n * 9 * (1 * C + 3 * C * C)
    mlp = 2 * (hidden * (C + NFEAT) + 2 * hidden)
    return conv + mlp
