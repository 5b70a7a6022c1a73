"""ranphy_cnn_denoise_noalloc (the refinement on the library's own device workspace) against
ranphy_cnn_denoise (the same refinement on a caller's workspace), through the C ABI: the
results must be equal bit for bit, on two calls in a row, the second with a smaller input.
Both run the same kernels on the same inputs, and every slot is refined independently of the
others, so the number of slots per pass (set by the workspace size) cannot change a bit."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2510_07843_amd as ranphy
from paper_2510_07843_amd import denoise
from synth import SlotShape

pytestmark = pytest.mark.gpu

LIMIT = 32 << 20  # RANPHY_NOALLOC_SCRATCH_BYTES


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ranphy.lib()


def _estimate(shape, seed):
    """A pilot-resolution estimate of the shape's size: unit-variance complex Gaussian
    values (the refinement's arithmetic does not depend on where they came from)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0x0A11, seed])))
    n = ranphy.buffer_floats(shape, ranphy.BUF_H, ranphy.H_PILOT) // 2
    h = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    return torch.from_numpy(h).cuda()


def _both(shape, params, h, nvar, gate):
    """(reference with a caller workspace sized for every slot, no-allocation call)."""
    n_pilot = -(-shape.n_prb * 12 // shape.dmrs_comb)
    rows, nimg = len(shape.dmrs_sym0), shape.n_rx * shape.n_layers
    ws = torch.empty(ranphy.cnn_workspace_bytes(rows, n_pilot, nimg, shape.n_slots, False),
                     dtype=torch.uint8, device="cuda")
    ref = ranphy.cnn_denoise(shape, params, h, noise_var=nvar, min_noise_var=gate, workspace=ws)
    out = torch.full_like(h, complex(np.nan, np.nan))
    ranphy.cnn_denoise_noalloc(shape, params, h, noise_var=nvar, min_noise_var=gate, out=out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy(), ws.numel()


def test_noalloc_matches_workspace_call_twice_second_smaller():
    params = denoise.init_params(3)
    # 1st call: 64 x 16, 273 PRB, comb 8 x 2 symbols, 24 slots (one-row grid, one kernel per
    # pass); 24 slots need more than the array, so the call takes two passes.  Slots with a
    # noise variance below the gate keep the plain estimate.
    big = SlotShape(273, 14, 64, 16, 6, 8, 2, (2,), 24)
    assert ranphy.cnn_workspace_bytes(1, 410, 1024, 24, False) > LIMIT
    h = _estimate(big, 1)
    nvar = torch.linspace(1e-3, 1.0, big.n_slots, dtype=torch.float32, device="cuda")
    ref, got, wsb = _both(big, params, h, nvar, 0.05)
    assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))
    kept = (nvar.cpu().numpy() < 0.05).nonzero()[0]
    per = ref.size // big.n_slots
    hc = h.cpu().numpy()
    for s in kept:  # gated slots are the input itself
        assert np.array_equal(got[s * per:(s + 1) * per], hc[s * per:(s + 1) * per])
    assert not np.array_equal(got, hc)
    # 2nd call, smaller: 16 x 4 with two DMRS occasions (a two-row grid: the layered form,
    # every activation kept), 3 slots, more than the array holds: again several passes.
    small = SlotShape(273, 14, 16, 4, 8, 4, 1, (2, 11), 3)
    n_pilot = -(-small.n_prb * 12 // small.dmrs_comb)
    one = ranphy.cnn_workspace_bytes(2, n_pilot, 64, 1, False)
    assert one <= LIMIT < 3 * one
    h2 = _estimate(small, 2)
    ref2, got2, _ = _both(small, params, h2, None, 0.0)
    assert np.array_equal(ref2.view(np.uint32), got2.view(np.uint32))
    assert np.all(np.isfinite(got2))


def test_noalloc_rejects_a_slot_beyond_the_array():
    params = denoise.init_params(3)
    big = SlotShape(273, 14, 64, 16, 6, 8, 2, (2, 9), 1)  # two occasions: ~200 MB per slot
    h = _estimate(big, 3)
    out = torch.empty_like(h)
    with pytest.raises(ranphy.RanphyError) as e:
        ranphy.cnn_denoise_noalloc(big, params, h, out=out)
    assert e.value.status == ranphy.ERR_UNSUPPORTED
