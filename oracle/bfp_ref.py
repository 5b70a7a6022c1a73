"""Reference of the block floating point (BFP) compression of received IQ samples.

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's checks.  The
product package never imports it and shares no code with it.

Sec. VI-A proposes block floating point compression of the IQ samples that distributed MIMO
carries over the fronthaul; the paper fixes no format, so the one below is a reading:

* the received grid rx[slot][symb][sc][rx] (complex64) is cut into blocks of B consecutive
  antennas of one resource element, B = 16 when Nr is a multiple of 16, else B = Nr (Nr < 16);
* a block's 2B real values v_i (I and Q interleaved, antenna order) share one exponent e, the
  smallest integer with max_i |v_i| <= 255 * 2^e (e = 0 for a block of zeros), and each value
  is stored as the 9-bit two's complement mantissa m_i = round_half_even(v_i / 2^e), so the
  decompressed value is m_i * 2^e (|m_i| <= 255);
* storage per block: one 32-bit word holding e, then W = ceil(18 B / 32) words holding the
  mantissas as a little-endian bit stream, m_i in bits 9 i .. 9 i + 8.

Every step is exact in FP64 (and in FP32: v / 2^e and m * 2^e scale by a power of two), so a
compressor that follows the definition is bit-exact with this one.
"""
from __future__ import annotations

import math

import numpy as np

MANT_BITS = 9
MANT_MAX = 255


def block_size(n_rx: int) -> int:
    if n_rx % 16 == 0:
        return 16
    if n_rx < 16:
        return n_rx
    raise ValueError("antenna count neither a multiple of 16 nor below 16")


def words_per_block(b: int) -> int:
    return 1 + (18 * b + 31) // 32


def block_exponent(vals: np.ndarray) -> int:
    """Smallest integer e with max|v| <= 255 * 2^e (0 for zeros)."""
    a = float(np.max(np.abs(vals)))
    if a == 0.0:
        return 0
    e = math.ceil(math.log2(a / MANT_MAX))
    while a > MANT_MAX * math.ldexp(1.0, e):
        e += 1
    while a <= MANT_MAX * math.ldexp(1.0, e - 1):
        e -= 1
    return e


def compress(rx: np.ndarray, n_rx: int) -> np.ndarray:
    """rx: complex64 array whose last axis is the antennas.  Returns uint32 words, blocks in
    the order of rx's resource elements, then antenna groups."""
    b = block_size(n_rx)
    w = words_per_block(b)
    flat = np.ascontiguousarray(rx, np.complex64).reshape(-1, n_rx // b, b)
    n_blocks = flat.shape[0] * flat.shape[1]
    vals = flat.view(np.float32).reshape(n_blocks, 2 * b).astype(np.float64)
    out = np.zeros((n_blocks, w), np.uint32)
    for i in range(n_blocks):
        v = vals[i]
        e = block_exponent(v)
        m = np.clip(np.rint(v / math.ldexp(1.0, e)), -256, MANT_MAX).astype(np.int64)
        out[i, 0] = np.uint32(e & 0xFFFFFFFF)
        bits = 0
        for k, mk in enumerate(m):
            bits |= (int(mk) & 0x1FF) << (MANT_BITS * k)
        for j in range(w - 1):
            out[i, 1 + j] = (bits >> (32 * j)) & 0xFFFFFFFF
    return out.reshape(-1)


def decompress(words: np.ndarray, n_rx: int, n_values: int) -> np.ndarray:
    """Inverse of compress for n_values complex samples (a multiple of n_rx)."""
    b = block_size(n_rx)
    w = words_per_block(b)
    blocks = np.asarray(words, np.uint32).reshape(-1, w)
    out = np.zeros((blocks.shape[0], 2 * b), np.float64)
    for i, blk in enumerate(blocks):
        e = int(np.int32(blk[0]))
        bits = 0
        for j in range(w - 1):
            bits |= int(blk[1 + j]) << (32 * j)
        for k in range(2 * b):
            mk = (bits >> (MANT_BITS * k)) & 0x1FF
            if mk >= 256:
                mk -= 512
            out[i, k] = math.ldexp(float(mk), e)
    return out.astype(np.float32).view(np.complex64).reshape(-1)[:n_values]
