"""Pins of the FP64 denoiser oracle (oracle/cnn_ref.py) against facts other than itself:
tap orientation and zero padding, a library correlation, finite differences of the forward
pass, and the identity of the residual form."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn_ref as C


def test_shift_orientation_and_zero_fill():
    rows, cols = 2, 4
    x = np.arange(rows * cols, dtype=float).reshape(rows * cols, 1, 1) + 1
    s = C.shift(x, rows, cols, 0, 1).reshape(rows, cols)
    assert np.array_equal(s, [[2, 3, 4, 0], [6, 7, 8, 0]])  # s[r][c] = x[r][c + 1]
    s = C.shift(x, rows, cols, 1, -1).reshape(rows, cols)
    assert np.array_equal(s, [[0, 5, 6, 7], [0, 0, 0, 0]])  # s[r][c] = x[r + 1][c - 1]


def test_tap_index_layout():
    # tap t = 3 (dy + 1) + (dx + 1): the centre tap is t = 4, (dy, dx) = (0, +1) is t = 5.
    assert C.TAPS[4] == (0, 0) and C.TAPS[5] == (0, 1) and C.TAPS[1] == (-1, 0)


def test_centre_tap_identity_conv_is_identity():
    rng = np.random.default_rng(0)
    rows, cols, B, ch = 3, 7, 4, 5
    x = rng.standard_normal((rows * cols, B, ch))
    W = np.zeros((9, ch, ch))
    W[4] = np.eye(ch)
    assert np.allclose(C.conv(x, W, np.zeros(ch), rows, cols), x, atol=0)


def test_single_channel_matches_library_correlation():
    rng = np.random.default_rng(1)
    # one row: numpy.correlate over the zero-padded row with the centre row of the kernel
    cols = 11
    x = rng.standard_normal((cols, 1, 1))
    W = rng.standard_normal((9, 1, 1))
    z = C.conv(x, W, np.zeros(1), 1, cols)[:, 0, 0]
    want = np.correlate(np.pad(x[:, 0, 0], 1), W[3:6, 0, 0], mode="valid")
    assert np.allclose(z, want, rtol=1e-13, atol=1e-13)
    # a 2-D grid: scipy's correlate2d with zero fill
    rows, cols = 4, 9
    x = rng.standard_normal((rows * cols, 1, 1))
    W = rng.standard_normal((9, 1, 1))
    z = C.conv(x, W, np.zeros(1), rows, cols)[:, 0, 0].reshape(rows, cols)
    want = correlate2d(x[:, 0, 0].reshape(rows, cols), W[:, 0, 0].reshape(3, 3), mode="same",
                       boundary="fill", fillvalue=0)
    assert np.allclose(z, want, rtol=1e-13, atol=1e-13)


def test_multichannel_is_sum_of_single_channel_correlations():
    rng = np.random.default_rng(2)
    rows, cols, ci, co = 2, 6, 3, 2
    x = rng.standard_normal((rows * cols, 1, ci))
    W = rng.standard_normal((9, ci, co))
    b = rng.standard_normal(co)
    z = C.conv(x, W, b, rows, cols)[:, 0, :]
    for o in range(co):
        want = b[o] + sum(correlate2d(x[:, 0, i].reshape(rows, cols), W[:, i, o].reshape(3, 3),
                                      mode="same") for i in range(ci))
        assert np.allclose(z[:, o].reshape(rows, cols), want, rtol=1e-12, atol=1e-12)


def test_zero_last_layer_is_identity_and_blocks_gradients():
    rng = np.random.default_rng(3)
    rows, cols, B = 1, 8, 3
    p = C.init_params(rng)
    p["W3"][:] = 0
    p["b3"][:] = 0
    x = rng.standard_normal((rows * cols, B, 2))
    out, _ = C.forward(x, p, rows, cols)
    assert np.array_equal(out, x)
    target = x + rng.standard_normal(x.shape)
    _, g = C.loss_and_grads(x, target, p, rows, cols)
    for l in range(3):
        assert not np.any(g[f"W{l}"]) and not np.any(g[f"b{l}"])
    assert np.any(g["W3"]) and np.any(g["b3"])


@pytest.mark.parametrize("rows", [1, 2])
def test_gradients_match_central_differences(rows):
    rng = np.random.default_rng(10 + rows)
    cols, B = 5, 3
    p = C.init_params(rng)
    for l in range(4):
        p[f"b{l}"] = 0.1 * rng.standard_normal(p[f"b{l}"].shape)
    p["W3"] *= 10.0  # a last layer of ordinary size, so that every gradient is sizeable
    x = rng.standard_normal((rows * cols, B, 2))
    target = rng.standard_normal(x.shape)

    def pattern():  # the ReLU on/off pattern of every hidden unit
        a, masks = x, []
        for l in range(3):
            z = C.conv(a, p[f"W{l}"], p[f"b{l}"], rows, cols)
            masks.append(z > 0)
            a = np.maximum(z, 0)
        return np.concatenate([m.reshape(-1) for m in masks])

    base = pattern()
    L, g = C.loss_and_grads(x, target, p, rows, cols)
    assert np.isclose(L, C.loss(x, target, p, rows, cols), rtol=1e-14)
    eps = 1e-7
    for name in sorted(p):
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, 24), replace=False)
        gn = g[name].reshape(-1)
        for i in idx:
            keep = flat[i]
            flat[i] = keep + eps
            lp = C.loss(x, target, p, rows, cols)
            same = np.array_equal(pattern(), base)
            flat[i] = keep - eps
            lm = C.loss(x, target, p, rows, cols)
            same = same and np.array_equal(pattern(), base)
            flat[i] = keep
            # With the same ReLU pattern at both ends the loss is a polynomial along the
            # segment, so the central difference is exact up to O(eps^2) and rounding.
            assert same, (name, i)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - gn[i]) <= 1e-6 * max(1e-3, np.max(np.abs(gn))), (name, i, fd, gn[i])
