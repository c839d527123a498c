"""FP64 reference of the scheduler network and its features -- TEST INFRASTRUCTURE.

Network: y = relu(relu(x W1 + b1) W2 + b2) W3 + b3 with x in R^98, hidden 128, y in R^2;
loss = mean over the m x 2 outputs of (y - t)^2; gradients by the chain rule written out
layer by layer (ReLU derivative 1 where the activation is > 0, else 0).  Parameters in one
flat array: W1[98][128], b1[128], W2[128][128], b2[128], W3[128][2], b3[2].
Features of a query: the 64 bits of its sketch 0 as +1/-1 (bit b -> feature b), then
log2(1 + size of its 13-bit prefix bucket) in tables 0..31 (0 for absent tables), then
the two inputs of adaptive-kNN(q, k, delta) (Algorithm 1) that set how far the walk
goes: log2 k and log2(1/delta), delta = 1 - recall (capped at 40 for delta < 2^-40).
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 98, 128, 2
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, OUT)),
          ("b3", (OUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(p: np.ndarray, x: np.ndarray):
    w = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ w["W1"] + w["b1"], 0.0)
    h2 = np.maximum(h1 @ w["W2"] + w["b2"], 0.0)
    y = h2 @ w["W3"] + w["b3"]
    return y, (x, h1, h2)


def loss_and_grad(p: np.ndarray, x: np.ndarray, t: np.ndarray):
    w = unpack(p)
    y, (x, h1, h2) = forward(p, x)
    e = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(e * e))
    dy = 2.0 * e / e.size
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dh2 = (dy @ w["W3"].T) * (h2 > 0)
    g["W2"], g["b2"] = h1.T @ dh2, dh2.sum(0)
    dh1 = (dh2 @ w["W2"].T) * (h1 > 0)
    g["W1"], g["b1"] = x.T @ dh1, dh1.sum(0)
    return loss, pack(g)


def features(sketch0: np.ndarray, bucket_sizes: np.ndarray, ks=10, recalls=0.9) -> np.ndarray:
    """sketch0: (m,) uint64; bucket_sizes: (m, tables) counts; ks, recalls: scalars or (m,);
    returns (m, 98) float64."""
    m = len(sketch0)
    f = np.zeros((m, IN))
    bits = (sketch0[:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)
    f[:, :64] = np.where(bits == 1, 1.0, -1.0)
    nt = min(32, bucket_sizes.shape[1])
    f[:, 64:64 + nt] = np.log2(1.0 + bucket_sizes[:, :nt].astype(np.float64))
    f[:, 96] = np.log2(np.broadcast_to(np.asarray(ks, dtype=np.float64), (m,)))
    delta = 1.0 - np.broadcast_to(np.asarray(recalls, dtype=np.float64), (m,))
    f[:, 97] = np.where(delta < 2.0 ** -40, 40.0, -np.log2(np.maximum(delta, 2.0 ** -40)))
    return f
