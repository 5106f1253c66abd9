"""FP64 reference of the pixel-pruning CNN -- test infrastructure only.

The network maps the Q-channel matched-filter image |A_q^H y_q| (Q x H x W,
each channel scaled by the largest value over all channels) to a per-pixel
probability that the pixel can be eliminated from every sensor's sub-problem
before the solve starts:

    a1 = conv(x, W1) + b1,  h1 = relu(a1)          Q  -> C channels
    a2 = conv(h1, W2) + b2, h2 = relu(a2)          C  -> C
    a3 = conv(h2, W3) + b3, h3 = relu(a3)          C  -> C
    a4 = conv(h3, W4) + b4, p = sigmoid(a4)        C  -> 1

conv is a 3x3 cross-correlation with zero 'same' padding:
    conv(x, W)[o, i, j] = sum_c sum_{dy,dx in -1..1} W[o, c, dy+1, dx+1] x[c, i+dy, j+dx].

Loss: weighted binary cross-entropy averaged over pixels,
    L = -(1/HW) sum_j w_j [t_j log p_j + (1 - t_j) log(1 - p_j)],
    w_j = pos_weight if t_j = 1 else 1,
whose gradient with respect to a4 is w_j (p_j - t_j) / HW.

Optimizer: Adam (Kingma & Ba 2015) with bias correction.
Everything below is the plain definition written with explicit loops over the
nine taps; it shares no code with the GPU kernels.
"""

from __future__ import annotations

import numpy as np


def init_params(Q: int, C: int = 32, seed: int = 0) -> dict:
    """Kaiming-normal weights (fan-in, ReLU gain), zero biases; FP64."""
    rng = np.random.default_rng(seed)
    shapes = [(C, Q), (C, C), (C, C), (1, C)]
    p = {}
    for l, (co, ci) in enumerate(shapes, start=1):
        std = np.sqrt(2.0 / (ci * 9))
        p[f"W{l}"] = rng.standard_normal((co, ci, 3, 3)) * std
        p[f"b{l}"] = np.zeros(co)
    return p


def normalize_input(mf: np.ndarray) -> np.ndarray:
    """Matched-filter images (Q, H, W) scaled by their largest value."""
    m = float(np.max(mf))
    return mf / m if m > 0 else mf.copy()


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    C_in, H, Wd = x.shape
    xp = np.zeros((C_in, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((W.shape[0], H, Wd))
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, dy:dy + H, dx:dx + Wd]                  # x[c, i+dy-1, j+dx-1]
            out += np.einsum("oc,chw->ohw", W[:, :, dy, dx], patch)
    return out + b[:, None, None]


def conv3x3_backward(x: np.ndarray, W: np.ndarray, g: np.ndarray):
    """Gradients of sum(g * conv3x3(x, W, b)) w.r.t. x, W, b."""
    C_in, H, Wd = x.shape
    xp = np.zeros((C_in, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, dy:dy + H, dx:dx + Wd]
            dW[:, :, dy, dx] = np.einsum("ohw,chw->oc", g, patch)
            dxp[:, dy:dy + H, dx:dx + Wd] += np.einsum("oc,ohw->chw", W[:, :, dy, dx], g)
    db = g.sum(axis=(1, 2))
    return dxp[:, 1:-1, 1:-1], dW, db


def sigmoid(a):
    return 1.0 / (1.0 + np.exp(-a))


def forward(p: dict, x: np.ndarray):
    """Returns (probability map (H, W), cache of activations)."""
    cache = {"x0": x}
    h = x
    for l in (1, 2, 3):
        a = conv3x3(h, p[f"W{l}"], p[f"b{l}"])
        cache[f"a{l}"] = a
        h = np.maximum(a, 0.0)
        cache[f"h{l}"] = h
    a4 = conv3x3(h, p["W4"], p["b4"])
    cache["a4"] = a4
    return sigmoid(a4[0]), cache


def bce_loss(prob: np.ndarray, target: np.ndarray, pos_weight: float) -> float:
    w = np.where(target > 0.5, pos_weight, 1.0)
    eps = 1e-300
    l = -(w * (target * np.log(np.maximum(prob, eps))
               + (1 - target) * np.log(np.maximum(1 - prob, eps))))
    return float(l.mean())


def backward(p: dict, cache: dict, target: np.ndarray, pos_weight: float) -> dict:
    """Gradients of bce_loss(forward(p, x)) with respect to every parameter."""
    prob = sigmoid(cache["a4"][0])
    w = np.where(target > 0.5, pos_weight, 1.0)
    g = (w * (prob - target) / prob.size)[None, :, :]             # dL/da4
    grads = {}
    h_in = {4: cache["h3"], 3: cache["h2"], 2: cache["h1"], 1: cache["x0"]}
    for l in (4, 3, 2, 1):
        dx, dW, db = conv3x3_backward(h_in[l], p[f"W{l}"], g)
        grads[f"W{l}"], grads[f"b{l}"] = dW, db
        if l > 1:
            g = dx * (cache[f"a{l - 1}"] > 0)                        # through relu
    return grads


class Adam:
    def __init__(self, params: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params: dict, grads: dict):
        self.t += 1
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * grads[k] ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)


def labels_from_solution(z: np.ndarray, active: np.ndarray) -> np.ndarray:
    """Training target per pixel: 1 when the optimum image is zero there and
    the pixel was eliminated in every sensor at the end of a pruned solve."""
    return ((np.abs(z) == 0) & (~np.asarray(active, bool)).all(axis=0)).astype(np.float64)
