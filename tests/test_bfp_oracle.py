"""Pins of the BFP reference (oracle/bfp_ref.py) against facts other than itself: a
hand-packed block, exact round trips of representable values, the error bound of the shared
exponent, minimality of the exponent, and the storage size."""
import math

import numpy as np
import pytest

from oracle import bfp_ref as B


def test_hand_packed_block():
    # Nr = 2: one block of 4 values, exponent 0 (max |v| = 255), mantissas 255, -1, 3, -256
    # cannot occur (|m| <= 255), so use 255, -1, 3, -255.
    rx = np.array([[255 - 1j, 3 - 255j]], np.complex64)
    w = B.compress(rx, 2)
    assert w.size == B.words_per_block(2) == 3
    assert w[0] == 0
    bits = (255) | ((-1 & 0x1FF) << 9) | (3 << 18) | ((-255 & 0x1FF) << 27)
    assert int(w[1]) == bits & 0xFFFFFFFF and int(w[2]) == bits >> 32
    assert np.array_equal(B.decompress(w, 2, 2), rx.reshape(-1))


def test_representable_values_round_trip_exactly():
    rng = np.random.default_rng(0)
    for e in (-20, -3, 0, 5):
        m = rng.integers(-255, 256, size=(7, 32))
        m[:, 0] = 255  # the block maximum fixes the exponent at e
        v = (m * 2.0 ** e).astype(np.float32)
        rx = v.view(np.complex64).reshape(7, 16)
        assert np.array_equal(B.decompress(B.compress(rx, 16), 16, rx.size), rx.reshape(-1))


@pytest.mark.parametrize("n_rx", [2, 4, 8, 12, 16, 64])
def test_error_within_half_a_step_and_exponent_minimal(n_rx):
    rng = np.random.default_rng(n_rx)
    rx = (rng.standard_normal((50, n_rx)) + 1j * rng.standard_normal((50, n_rx))) \
        * rng.uniform(1e-3, 1e3, size=(50, 1))
    rx = rx.astype(np.complex64)
    words = B.compress(rx, n_rx)
    b = B.block_size(n_rx)
    assert words.size == 50 * (n_rx // b) * B.words_per_block(b)
    back = B.decompress(words, n_rx, rx.size).reshape(rx.shape)
    vals = rx.reshape(-1, n_rx // b, b).view(np.float32).reshape(-1, 2 * b).astype(np.float64)
    got = back.reshape(-1, n_rx // b, b).view(np.float32).reshape(-1, 2 * b).astype(np.float64)
    exps = words.reshape(-1, B.words_per_block(b))[:, 0].view(np.int32)
    for v, g, e in zip(vals, got, exps):
        step = 2.0 ** int(e)
        assert np.all(np.abs(g - v) <= step / 2)          # rounding error of one mantissa step
        a = np.max(np.abs(v))
        assert a <= 255 * step and a > 255 * step / 2       # e is the smallest that fits


def test_zero_block_and_unsupported_counts():
    assert B.block_exponent(np.zeros(8)) == 0
    w = B.compress(np.zeros((3, 4), np.complex64), 4)
    assert not np.any(w)
    with pytest.raises(ValueError):
        B.block_size(20)
