"""FP64 reference of the learned channel-estimate denoiser (forward, loss and gradients).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's checks.  The
product package never imports it and shares no code with it.

The network refines a least-squares channel estimate at the DMRS pilots (channel estimation
is the PHY block the paper names besides MIMO detection, abstract and Sec. III-B).  One image
is the estimate of one (receive antenna, layer) pair over the pilot grid: rows are DMRS
occasions, columns the port's pilot index j, two channels (real, imaginary).  Images of one
batch share the grid and are stored pixel-major, ``x[pixel][image][channel]`` with
``pixel = row * cols + col``.

    a0 = x
    z_l = conv3x3(a_{l-1}; W_l, b_l),  a_l = max(z_l, 0)        l = 1, 2, 3
    y  = conv3x3(a_3; W_4, b_4)
    out = x + y                                                  (residual)
    loss = sum((out - target)^2) / out.size

conv3x3 is a correlation with zero padding: for tap t = 3 (dy + 1) + (dx + 1),
``z[r][c] = b + sum_t x[r + dy][c + dx] @ W[t]`` with W[t] of shape [C_in][C_out] and
out-of-grid neighbours taken as zero.  Channels 2 -> 32 -> 32 -> 32 -> 2.

The gradients are the chain rule written out layer by layer; they are pinned against central
finite differences of ``forward`` in the tests.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

TAPS: List[Tuple[int, int]] = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = (2, 32, 32, 32, 2)
N_LAYERS = 4


def shift(x: np.ndarray, rows: int, cols: int, dy: int, dx: int) -> np.ndarray:
    """s[r][c] = x[r + dy][c + dx] (zero outside the grid); x is [P][B][C]."""
    g = x.reshape(rows, cols, *x.shape[1:])
    s = np.zeros_like(g)
    r0, r1 = max(0, -dy), min(rows, rows - dy)
    c0, c1 = max(0, -dx), min(cols, cols - dx)
    if r0 < r1 and c0 < c1:
        s[r0:r1, c0:c1] = g[r0 + dy:r1 + dy, c0 + dx:c1 + dx]
    return s.reshape(x.shape)


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray, rows: int, cols: int) -> np.ndarray:
    """3x3 correlation with zero padding: x [P][B][Ci], W [9][Ci][Co], b [Co] -> [P][B][Co]."""
    z = np.zeros(x.shape[:2] + (W.shape[2],)) + b
    for t, (dy, dx) in enumerate(TAPS):
        z += shift(x, rows, cols, dy, dx) @ W[t]
    return z


def init_params(rng: np.random.Generator) -> Dict[str, np.ndarray]:
    """He-normal weights (fan-in 9 C_in), zero biases; the last layer scaled by 0.1 so the
    untrained network starts near the identity map of its residual form."""
    p = {}
    for l in range(N_LAYERS):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if l == N_LAYERS - 1 else 1.0)
        p[f"W{l}"] = rng.standard_normal((9, ci, co)) * std
        p[f"b{l}"] = np.zeros(co)
    return p


def forward(x: np.ndarray, p: Dict[str, np.ndarray], rows: int, cols: int):
    """Returns the output and the list of activations a_0 .. a_3 (a_0 = x)."""
    acts = [x]
    a = x
    for l in range(N_LAYERS - 1):
        a = np.maximum(conv(a, p[f"W{l}"], p[f"b{l}"], rows, cols), 0.0)
        acts.append(a)
    y = conv(a, p[f"W{N_LAYERS - 1}"], p[f"b{N_LAYERS - 1}"], rows, cols)
    return x + y, acts


def loss(x: np.ndarray, target: np.ndarray, p, rows: int, cols: int) -> float:
    out, _ = forward(x, p, rows, cols)
    return float(np.sum((out - target) ** 2) / out.size)


def loss_and_grads(x: np.ndarray, target: np.ndarray, p, rows: int, cols: int):
    """Loss and its gradient with respect to every weight and bias."""
    out, acts = forward(x, p, rows, cols)
    g = {}
    dz = 2.0 * (out - target) / out.size  # d loss / d y  (out = x + y)
    for l in range(N_LAYERS - 1, -1, -1):
        a_in = acts[l]
        # z = b + sum_t shift_t(a_in) @ W[t]
        g[f"b{l}"] = dz.sum(axis=(0, 1))
        g[f"W{l}"] = np.stack([
            np.einsum("pbi,pbo->io", shift(a_in, rows, cols, dy, dx), dz) for (dy, dx) in TAPS])
        if l == 0:
            break
        # d a_in[q] = sum_t dz[q - t] @ W[t]^T  (the neighbour of q - t along t is q)
        da = np.zeros_like(a_in)
        for t, (dy, dx) in enumerate(TAPS):
            da += shift(dz, rows, cols, -dy, -dx) @ p[f"W{l}"][t].T
        dz = da * (a_in > 0)  # a_in = max(z_{l-1}, 0)
    return float(np.sum((out - target) ** 2) / out.size), g
