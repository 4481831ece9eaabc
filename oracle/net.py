"""FP64 reference of the learned warm-start network (not part of the paper).

Part of the CPU oracle -- test infrastructure only.

The warm start predicts, for every lattice node, the displacement change of
the coming frame from 8 input channels (the previous two frames' node
displacements, the splatted point-to-plane residual at the plain
initialisation and its validity).  Architecture (a 3-level 3-D U-Net with
channels 16-32-64, 3x3x3 kernels, zero padding, ReLU, nearest up-sampling and
skip concatenation):

    e0a = relu(conv(x, 8->16))            e0  = relu(conv(e0a, 16->16))
    e1a = relu(conv_s2(e0, 16->32))       e1  = relu(conv(e1a, 32->32))
    e2a = relu(conv_s2(e1, 32->64))       e2  = relu(conv(e2a, 64->64))
    u1  = relu(conv(up(e2), 64->32))      d1  = relu(conv([u1, e1], 64->32))
    u0  = relu(conv(up(d1), 32->16))      d0  = relu(conv([u0, e0], 32->16))
    out = conv(d0, 16->3)

Loss: mean over nodes of ||out - target||^2 (sum over the 3 components).
Optimiser: Adam.  Tensors are (C, nz, ny, nx) with node index x + nx (y + ny z).
Convolution weights are (C_out, C_in, 3, 3, 3) indexed [co, ci, dz, dy, dx].
Stride-2 convolutions sample input position 2*out + tap - 1, so an axis of n
nodes becomes ceil(n / 2); up-sampling copies node j // 2 and is cropped to
the skip tensor's size.
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

# (name, c_in, c_out, stride, relu)
LAYERS: List[Tuple[str, int, int, int, bool]] = [
    ("e0a", 8, 16, 1, True),
    ("e0", 16, 16, 1, True),
    ("e1a", 16, 32, 2, True),
    ("e1", 32, 32, 1, True),
    ("e2a", 32, 64, 2, True),
    ("e2", 64, 64, 1, True),
    ("u1", 64, 32, 1, True),
    ("d1", 64, 32, 1, True),
    ("u0", 32, 16, 1, True),
    ("d0", 32, 16, 1, True),
    ("head", 16, 3, 1, False),
]


def out_size(n: int, stride: int) -> int:
    return n if stride == 1 else (n + 1) // 2


def _cols(x: np.ndarray, stride: int, shape_out) -> np.ndarray:
    """im2col: (C_in * 27, voxels_out) with rows ordered (ci, dz, dy, dx)."""
    C = x.shape[0]
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    D, H, W = shape_out
    cols = np.empty((C, 3, 3, 3, D, H, W))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                cols[:, dz, dy, dx] = xp[:, dz:dz + stride * D:stride,
                                         dy:dy + stride * H:stride, dx:dx + stride * W:stride]
    return cols.reshape(C * 27, D * H * W)


def conv3d(x: np.ndarray, W: np.ndarray, b: np.ndarray, stride: int = 1) -> np.ndarray:
    """y[co, v] = b[co] + sum_{ci, tap} W[co, ci, tap] x[ci, stride*v + tap - 1]."""
    shape_out = tuple(out_size(n, stride) for n in x.shape[1:])
    y = W.reshape(W.shape[0], -1) @ _cols(x, stride, shape_out) + b[:, None]
    return y.reshape((W.shape[0],) + shape_out)


def conv3d_backward(x, W, dy, stride=1):
    """Gradients (dx, dW, db) of conv3d for the upstream gradient dy."""
    shape_out = dy.shape[1:]
    cols = _cols(x, stride, shape_out)
    g = dy.reshape(dy.shape[0], -1)
    dW = (g @ cols.T).reshape(W.shape)
    db = g.sum(axis=1)
    dcols = (W.reshape(W.shape[0], -1).T @ g).reshape((x.shape[0], 3, 3, 3) + tuple(shape_out))
    D, H, Wd = shape_out
    dxp = np.zeros((x.shape[0],) + tuple(n + 2 for n in x.shape[1:]))
    for dz in range(3):
        for dy_ in range(3):
            for dx_ in range(3):
                dxp[:, dz:dz + stride * D:stride, dy_:dy_ + stride * H:stride,
                    dx_:dx_ + stride * Wd:stride] += dcols[:, dz, dy_, dx_]
    dx = dxp[:, 1:-1, 1:-1, 1:-1]
    return dx, dW, db


def upsample(x: np.ndarray, shape) -> np.ndarray:
    """Nearest x2: out[:, z, y, x] = in[:, z // 2, y // 2, x // 2], cropped."""
    D, H, W = shape
    return x[:, np.arange(D) // 2][:, :, np.arange(H) // 2][:, :, :, np.arange(W) // 2]


def upsample_backward(dy: np.ndarray, shape_in) -> np.ndarray:
    dx = np.zeros((dy.shape[0],) + tuple(shape_in))
    D, H, W = dy.shape[1:]
    zi, yi, xi = np.arange(D) // 2, np.arange(H) // 2, np.arange(W) // 2
    np.add.at(dx, (slice(None), zi[:, None, None], yi[None, :, None], xi[None, None, :]), dy)
    return dx


def init_params(rng: np.random.Generator, scale_head: float = 0.1) -> Dict[str, np.ndarray]:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the head is
    scaled down so an untrained net predicts nearly zero."""
    p = {}
    for name, ci, co, _, _ in LAYERS:
        std = np.sqrt(2.0 / (ci * 27))
        if name == "head":
            std *= scale_head
        p[name + ".W"] = rng.normal(scale=std, size=(co, ci, 3, 3, 3))
        p[name + ".b"] = np.zeros(co)
    return p


def _identity(a):
    return a


def forward(p: Dict[str, np.ndarray], x: np.ndarray, act_round=_identity):
    """Network output (3, nz, ny, nx) and the activations needed by backward.
    act_round is applied to every stored activation (e.g. bf16_round to model
    an implementation that keeps activations in bfloat16)."""
    a = {"x": x}
    relu = lambda v: act_round(np.maximum(v, 0.0))
    a["e0a"] = relu(conv3d(x, p["e0a.W"], p["e0a.b"]))
    a["e0"] = relu(conv3d(a["e0a"], p["e0.W"], p["e0.b"]))
    a["e1a"] = relu(conv3d(a["e0"], p["e1a.W"], p["e1a.b"], 2))
    a["e1"] = relu(conv3d(a["e1a"], p["e1.W"], p["e1.b"]))
    a["e2a"] = relu(conv3d(a["e1"], p["e2a.W"], p["e2a.b"], 2))
    a["e2"] = relu(conv3d(a["e2a"], p["e2.W"], p["e2.b"]))
    a["up1"] = upsample(a["e2"], a["e1"].shape[1:])
    a["u1"] = relu(conv3d(a["up1"], p["u1.W"], p["u1.b"]))
    a["c1"] = np.concatenate([a["u1"], a["e1"]], axis=0)
    a["d1"] = relu(conv3d(a["c1"], p["d1.W"], p["d1.b"]))
    a["up0"] = upsample(a["d1"], a["e0"].shape[1:])
    a["u0"] = relu(conv3d(a["up0"], p["u0.W"], p["u0.b"]))
    a["c0"] = np.concatenate([a["u0"], a["e0"]], axis=0)
    a["d0"] = relu(conv3d(a["c0"], p["d0.W"], p["d0.b"]))
    out = conv3d(a["d0"], p["head.W"], p["head.b"])
    return out, a


def backward(p: Dict[str, np.ndarray], a, dout: np.ndarray,
             grad_round=_identity) -> Dict[str, np.ndarray]:
    """Parameter gradients for the upstream gradient dout of the output.
    grad_round is applied to dout and to every stored gradient tensor: the
    gradients w.r.t. pre-activations, the skip parts of the concatenations
    and the gradients w.r.t. up-sampled tensors."""
    g = {}
    q = grad_round

    def conv_b(name, x_in, dy, stride=1):
        dx, g[name + ".W"], g[name + ".b"] = conv3d_backward(x_in, p[name + ".W"], dy, stride)
        return dx

    relu_b = lambda dy, y: q(dy * (y > 0))
    dout = q(dout)
    g_d0 = relu_b(conv_b("head", a["d0"], dout), a["d0"])
    dc0 = conv_b("d0", a["c0"], g_d0)
    g_u0, skip0 = relu_b(dc0[:16], a["u0"]), q(dc0[16:])
    dup0 = q(conv_b("u0", a["up0"], g_u0))
    g_d1 = relu_b(upsample_backward(dup0, a["d1"].shape[1:]), a["d1"])
    dc1 = conv_b("d1", a["c1"], g_d1)
    g_u1, skip1 = relu_b(dc1[:32], a["u1"]), q(dc1[32:])
    dup1 = q(conv_b("u1", a["up1"], g_u1))
    g_e2 = relu_b(upsample_backward(dup1, a["e2"].shape[1:]), a["e2"])
    g_e2a = relu_b(conv_b("e2", a["e2a"], g_e2), a["e2a"])
    g_e1 = relu_b(conv_b("e2a", a["e1"], g_e2a, 2) + skip1, a["e1"])
    g_e1a = relu_b(conv_b("e1", a["e1a"], g_e1), a["e1a"])
    g_e0 = relu_b(conv_b("e1a", a["e0"], g_e1a, 2) + skip0, a["e0"])
    g_e0a = relu_b(conv_b("e0", a["e0a"], g_e0), a["e0a"])
    g["x"] = conv_b("e0a", a["x"], g_e0a)
    return g


def flatten(p: Dict[str, np.ndarray]) -> np.ndarray:
    """Parameters (or gradients) as one vector: per layer W then b."""
    return np.concatenate([np.concatenate([p[n + ".W"].reshape(-1), p[n + ".b"]])
                           for n, *_ in LAYERS])


def unflatten(v: np.ndarray) -> Dict[str, np.ndarray]:
    p, o = {}, 0
    for name, ci, co, _, _ in LAYERS:
        nw = co * ci * 27
        p[name + ".W"] = np.asarray(v[o:o + nw], np.float64).reshape(co, ci, 3, 3, 3)
        p[name + ".b"] = np.asarray(v[o + nw:o + nw + co], np.float64)
        o += nw + co
    assert o == v.size
    return p


def mse_loss(out: np.ndarray, target: np.ndarray):
    """(loss, d loss / d out) with loss = mean over nodes of ||out - target||^2."""
    n = out[0].size
    diff = out - target
    return float(np.sum(diff * diff) / n), 2.0 * diff / n


def adam_step(p, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; t counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (round to nearest even) and back."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
