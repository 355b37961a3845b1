"""FP64 CPU oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

Plain numpy: every 3x3x3 convolution is a sum over the 27 taps of a shifted
input slice times a (Ci x Co) weight matrix (a library matmul per tap), with
zero padding of one cell; stride-2 convolutions sample every other output.
Tensors are channels-last [B, D, H, W, C].  Weights are [27, Ci, Co] with tap
t = (dz+1)*9 + (dy+1)*3 + (dx+1).

The network (a 3-level U-shaped conv net; each level is 4x coarser than the
one above it, reached by two stride-2 convolutions, so the coarsest level
sees the whole domain) is:
  a1 = relu(conv(x, 8->16))          a2 = relu(conv(a1, 16->16))       level 1
  h1 = relu(conv_s2(a2, 16->16))     d1 = relu(conv_s2(h1, 16->32))
  a3 = relu(conv(d1, 32->32))                                          level 2
  h2 = relu(conv_s2(a3, 32->32))     d2 = relu(conv_s2(h2, 32->48))
  a4 = relu(conv(d2, 48->32))                                          level 3
  c2 = [up4(a4), a3]                 a5 = relu(conv(c2, 64->32))       level 2
  c1 = [up4(a5), a2]                 a6 = relu(conv(c1, 48->16))       level 1
  y  = a6 . w_head + b_head          (1x1 head, 16 -> 1)
(input channels: log k and f, zero-padded to 8; up4 = nearest-neighbour
upsampling by 4, cropped to the finer grid.)
"""
from __future__ import annotations

import numpy as np

LAYERS = [  # name, Ci, Co, stride
    ("e1a", 8, 16, 1), ("e1b", 16, 16, 1), ("d1a", 16, 16, 2), ("d1b", 16, 32, 2),
    ("e2", 32, 32, 1), ("d2a", 32, 32, 2), ("d2b", 32, 48, 2), ("bott", 48, 32, 1),
    ("u2", 64, 32, 1), ("u1", 48, 16, 1),
]
HEAD_C = 16


def out_size(n, stride):
    return (n - 1) // stride + 1


def conv3d(x, w, b, stride=1):
    """y[p, co] = b[co] + sum_{t, ci} x[stride*p + o_t, ci] w[t, ci, co]."""
    B, D, H, W, Ci = x.shape
    Co = w.shape[2]
    Do, Ho, Wo = out_size(D, stride), out_size(H, stride), out_size(W, stride)
    xp = np.zeros((B, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    y = np.broadcast_to(b, (B, Do, Ho, Wo, Co)).astype(np.float64).copy()
    for t in range(27):
        dz, dy, dx = t // 9, (t // 3) % 3, t % 3
        sl = xp[:, dz:dz + stride * (Do - 1) + 1:stride, dy:dy + stride * (Ho - 1) + 1:stride,
                dx:dx + stride * (Wo - 1) + 1:stride]
        y += sl @ w[t]
    return y


def conv3d_backward(x, w, dy, stride=1):
    """Gradients (dx, dw, db) of conv3d for the upstream gradient dy."""
    B, D, H, W, Ci = x.shape
    _, Do, Ho, Wo, Co = dy.shape
    xp = np.zeros((B, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w, dtype=np.float64)
    for t in range(27):
        dz, ddy, dx_ = t // 9, (t // 3) % 3, t % 3
        idx = (slice(None), slice(dz, dz + stride * (Do - 1) + 1, stride),
               slice(ddy, ddy + stride * (Ho - 1) + 1, stride),
               slice(dx_, dx_ + stride * (Wo - 1) + 1, stride))
        sl = xp[idx]
        dw[t] = np.tensordot(sl, dy, axes=([0, 1, 2, 3], [0, 1, 2, 3]))
        dxp[idx] += dy @ w[t].T
    db = dy.sum(axis=(0, 1, 2, 3))
    return dxp[:, 1:-1, 1:-1, 1:-1], dw, db


def upsample(x, shape, f):
    """Nearest-neighbour upsampling by f, cropped to the spatial shape."""
    D, H, W = shape
    y = x.repeat(f, axis=1).repeat(f, axis=2).repeat(f, axis=3)
    return y[:, :D, :H, :W]


def upsample_backward(dy, coarse_shape, f):
    B, D, H, W, C = dy.shape
    d, h, w = coarse_shape
    out = np.zeros((B, d, h, w, C))
    for oz in range(f):
        for oy in range(f):
            for ox in range(f):
                part = dy[:, oz::f, oy::f, ox::f]
                out[:, :part.shape[1], :part.shape[2], :part.shape[3]] += part
    return out


def relu(x):
    return np.maximum(x, 0.0)


def init_params(seed):
    """He-normal weights, zero biases (same recipe as the library's)."""
    g = np.random.default_rng(seed)
    P = {}
    for name, ci, co, _ in LAYERS:
        P[name + ".w"] = g.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci))
        P[name + ".b"] = np.zeros(co)
    P["head.w"] = g.standard_normal(HEAD_C) * np.sqrt(1.0 / HEAD_C)
    P["head.b"] = np.zeros(1)
    return P


def forward(P, x):
    """Returns the output [B, D, H, W] and the cache for backward."""
    c = {"x": x}
    shape1 = x.shape[1:4]
    c["a1"] = relu(conv3d(x, P["e1a.w"], P["e1a.b"]))
    c["a2"] = relu(conv3d(c["a1"], P["e1b.w"], P["e1b.b"]))
    c["h1"] = relu(conv3d(c["a2"], P["d1a.w"], P["d1a.b"], 2))
    c["d1"] = relu(conv3d(c["h1"], P["d1b.w"], P["d1b.b"], 2))
    c["a3"] = relu(conv3d(c["d1"], P["e2.w"], P["e2.b"]))
    c["h2"] = relu(conv3d(c["a3"], P["d2a.w"], P["d2a.b"], 2))
    c["d2"] = relu(conv3d(c["h2"], P["d2b.w"], P["d2b.b"], 2))
    c["a4"] = relu(conv3d(c["d2"], P["bott.w"], P["bott.b"]))
    shape2 = c["a3"].shape[1:4]
    c["c2"] = np.concatenate([upsample(c["a4"], shape2, 4), c["a3"]], axis=-1)
    c["a5"] = relu(conv3d(c["c2"], P["u2.w"], P["u2.b"]))
    c["c1"] = np.concatenate([upsample(c["a5"], shape1, 4), c["a2"]], axis=-1)
    c["a6"] = relu(conv3d(c["c1"], P["u1.w"], P["u1.b"]))
    y = c["a6"] @ P["head.w"] + P["head.b"][0]
    return y, c


def backward(P, c, dy):
    """Gradients of all parameters for the upstream gradient dy [B, D, H, W]."""
    G = {}
    G["head.w"] = np.tensordot(c["a6"], dy, axes=([0, 1, 2, 3], [0, 1, 2, 3]))
    G["head.b"] = np.array([dy.sum()])
    da6 = dy[..., None] * P["head.w"]
    dz = da6 * (c["a6"] > 0)
    dc1, G["u1.w"], G["u1.b"] = conv3d_backward(c["c1"], P["u1.w"], dz)
    c_up = c["a5"].shape[-1]
    da5 = upsample_backward(dc1[..., :c_up], c["a5"].shape[1:4], 4)
    da2 = dc1[..., c_up:]
    dz = da5 * (c["a5"] > 0)
    dc2, G["u2.w"], G["u2.b"] = conv3d_backward(c["c2"], P["u2.w"], dz)
    c_up = c["a4"].shape[-1]
    da4 = upsample_backward(dc2[..., :c_up], c["a4"].shape[1:4], 4)
    da3 = dc2[..., c_up:]
    dz = da4 * (c["a4"] > 0)
    dd2, G["bott.w"], G["bott.b"] = conv3d_backward(c["d2"], P["bott.w"], dz)
    dz = dd2 * (c["d2"] > 0)
    dh2, G["d2b.w"], G["d2b.b"] = conv3d_backward(c["h2"], P["d2b.w"], dz, 2)
    dz = dh2 * (c["h2"] > 0)
    da3b, G["d2a.w"], G["d2a.b"] = conv3d_backward(c["a3"], P["d2a.w"], dz, 2)
    da3 = da3 + da3b
    dz = da3 * (c["a3"] > 0)
    dd1, G["e2.w"], G["e2.b"] = conv3d_backward(c["d1"], P["e2.w"], dz)
    dz = dd1 * (c["d1"] > 0)
    dh1, G["d1b.w"], G["d1b.b"] = conv3d_backward(c["h1"], P["d1b.w"], dz, 2)
    dz = dh1 * (c["h1"] > 0)
    da2b, G["d1a.w"], G["d1a.b"] = conv3d_backward(c["a2"], P["d1a.w"], dz, 2)
    da2 = da2 + da2b
    dz = da2 * (c["a2"] > 0)
    da1, G["e1b.w"], G["e1b.b"] = conv3d_backward(c["a1"], P["e1b.w"], dz)
    dz = da1 * (c["a1"] > 0)
    _, G["e1a.w"], G["e1a.b"] = conv3d_backward(c["x"], P["e1a.w"], dz)
    return G


def mse(y, t):
    """Mean squared error and its gradient."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def laplacian7(e):
    """(L e) for the 7-point Laplacian on each sample's grid, zero outside:
    6 e_p minus the in-grid neighbours."""
    out = 6.0 * e
    out[:, 1:] -= e[:, :-1]
    out[:, :-1] -= e[:, 1:]
    out[:, :, 1:] -= e[:, :, :-1]
    out[:, :, :-1] -= e[:, :, 1:]
    out[:, :, :, 1:] -= e[:, :, :, :-1]
    out[:, :, :, :-1] -= e[:, :, :, 1:]
    return out


def h1_loss(y, t, lam):
    """Energy-type loss e^T (L + lam I) e / N of e = y - t ([B, D, H, W]) and
    its gradient 2 (L e + lam e) / N."""
    e = y - t
    le = laplacian7(e) + lam * e
    return float(np.sum(e * le)) / e.size, 2.0 * le / e.size


def adam(P, G, M, V, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), in place."""
    for k in P:
        M[k] = b1 * M[k] + (1 - b1) * G[k]
        V[k] = b2 * V[k] + (1 - b2) * G[k] * G[k]
        mh = M[k] / (1 - b1 ** step)
        vh = V[k] / (1 - b2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
