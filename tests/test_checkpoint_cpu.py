"""The refinement network's checkpoint file on the host: format, exact round trip, BF16
rounding, integrity checks."""
import json
import os

import numpy as np
import pytest
import torch

import paper_2510_07843_amd as ranphy
from paper_2510_07843_amd import denoise


@pytest.fixture(scope="module")
def n():
    return ranphy.cnn_param_count()


def _vec(n, seed, scale=1.0):
    return torch.from_numpy((np.random.default_rng(seed).standard_normal(n) * scale)
                            .astype(np.float32))


def test_round_trip_is_exact(tmp_path, n):
    p, m, v = _vec(n, 1), _vec(n, 2, 1e-3), _vec(n, 3, 1e-6).abs()
    st = dict(steps=600, batch=2, lr=2e-3, seed=43, rng_state={"a": 1}, losses=[0.5, 0.25])
    f = str(tmp_path / "ck.bin")
    denoise.save_checkpoint(f, p, m, v, 123, st, dict(gate_min_noise_var=0.01))
    ck = denoise.load_checkpoint(f, "cpu")
    assert torch.equal(ck["params"], p) and torch.equal(ck["m"], m) and torch.equal(ck["v"], v)
    assert ck["step"] == 123 and ck["train_state"] == st
    assert ck["extra"] == dict(gate_min_noise_var=0.01)
    with open(f, "rb") as fh:
        header = json.loads(fh.readline())
    names = [s["name"] for s in header["sections"]]
    assert names == ["params_bf16", "params_f32", "adam_m", "adam_v"]
    assert header["sections"][0]["bytes"] == 2 * n and header["param_count"] == n
    assert os.path.getsize(f) == len(json.dumps(header)) + 1 + (2 + 4 * 3) * n


def test_bf16_blob_is_round_to_nearest_even(tmp_path, n):
    p = _vec(n, 4)
    special = torch.tensor([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 65504.0,
                            3.0e38, 1e-40, 0.0, -0.0], dtype=torch.float32)
    p[: special.numel()] = special
    f = str(tmp_path / "ck.bin")
    denoise.save_checkpoint(f, p)
    ck = denoise.load_checkpoint(f, "cpu")
    ref = p.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ck["params_bf16"], ref)
    # ties: 1 + 2^-8 rounds down to 1 (even), 1 + 3 2^-8 up to 1 + 2^-6
    assert ck["params_bf16"][0] == 0x3F80 and ck["params_bf16"][1] == 0x3F82
    assert ck["m"] is None and ck["v"] is None


def test_widened_bf16_when_f32_absent(tmp_path, n):
    # a file carrying only the BF16 blob loads as its widened values
    p = _vec(n, 5)
    f = str(tmp_path / "ck.bin")
    denoise.save_checkpoint(f, p)
    with open(f, "rb") as fh:
        header = json.loads(fh.readline())
        body = fh.read()
    bf = header["sections"][0]
    header["sections"] = [bf]
    blob = body[: bf["bytes"]]
    import hashlib
    header["sha256"] = hashlib.sha256(blob).hexdigest()
    with open(f, "wb") as fh:
        fh.write(json.dumps(header).encode() + b"\n" + blob)
    ck = denoise.load_checkpoint(f, "cpu")
    assert torch.equal(ck["params"], p.to(torch.bfloat16).float())


def test_corruption_and_wrong_files_are_refused(tmp_path, n):
    f = str(tmp_path / "ck.bin")
    denoise.save_checkpoint(f, _vec(n, 6))
    raw = bytearray(open(f, "rb").read())
    raw[-5] ^= 0x10
    open(f, "wb").write(bytes(raw))
    with pytest.raises(ValueError, match="checksum"):
        denoise.load_checkpoint(f, "cpu")
    g = str(tmp_path / "other.bin")
    open(g, "wb").write(json.dumps({"format": "something else"}).encode() + b"\n")
    with pytest.raises(ValueError, match="not a"):
        denoise.load_checkpoint(g, "cpu")
    with pytest.raises(ValueError):
        denoise.save_checkpoint(f, torch.zeros(n - 1))
