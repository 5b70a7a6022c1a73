"""GPU parity of the block floating point compression of the received grid (ranphy_bfp_*)
against the oracle's definition (oracle/bfp_ref.py): packed words and decompressed samples
bit-exact on seeded grids of every block width class, with ties, zeros, powers of two and
extreme scales; the full-size 16- and 64-antenna grids sampled block by block, with the
error bound and exponent minimality checked on every block; and the one-launch chain run on
a decompressed grid against the oracle chain on the oracle's decompression of it."""
import sys

import numpy as np
import pytest
import torch

import oracle
import oracle.bfp_ref as bref
import paper_2510_07843_amd as ranphy
import synth
from synth import SlotShape

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ranphy.lib()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def shape_for(nr, n_prb=3, n_slots=2):
    nl = min(nr, 2)
    return SlotShape(n_prb=n_prb, n_symb=14, n_rx=nr, n_layers=nl, qm=2, dmrs_comb=2, dmrs_td=1,
                     dmrs_sym0=(2,), n_slots=n_slots)


def grid(shape, seed):
    """Gaussian samples with a per-resource-element scale spread over twelve decades, some
    all-zero resource elements and some exact zeros inside blocks."""
    rng = np.random.default_rng(seed)
    n_re = shape.n_slots * shape.n_symb * shape.n_sc
    z = rng.standard_normal((n_re, shape.n_rx, 2))
    z *= 10.0 ** rng.uniform(-6, 6, (n_re, 1, 1))
    z[rng.random(n_re) < 0.05] = 0.0
    z[rng.random(z.shape) < 0.02] = 0.0
    return z.astype(np.float32).view(np.complex64).reshape(-1)


def run(shape, rx):
    t = torch.from_numpy(rx).cuda()
    w = ranphy.bfp_compress(shape, t)
    back = ranphy.bfp_decompress(shape, w)
    torch.cuda.synchronize()
    return w.cpu().numpy().view(np.uint32), back.cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("nr", [1, 2, 3, 4, 7, 8, 12, 15, 16, 32, 64])
def test_bit_exact_against_oracle(nr):
    shape = shape_for(nr)
    say(f"bfp nr={nr}")
    rx = grid(shape, 100 + nr)
    w, back = run(shape, rx)
    wr = bref.compress(rx, nr)
    assert w.shape == wr.shape == (ranphy.bfp_words(shape),)
    assert np.array_equal(w, wr), np.flatnonzero(w != wr)[:8]
    br = bref.decompress(wr, nr, rx.size)
    assert np.array_equal(bits(back), bits(br))


def test_ties_powers_of_two_and_extreme_scales():
    """Blocks built on a chosen exponent: the peak exactly 255 * 2^e, the rest at half-odd
    and half-even multiples of 2^e (round half to even both ways), powers of two, values just
    past 255 * 2^e (the exponent steps up), and scales near the FP32 limits."""
    nr = 16
    shape = shape_for(nr, n_prb=1, n_slots=1)
    n_re = shape.n_symb * shape.n_sc
    rng = np.random.default_rng(7)
    v = np.zeros((n_re, 2 * nr), np.float64)
    for i in range(n_re):
        e = int(rng.integers(-140, 118))
        m = rng.integers(-255, 255, 2 * nr).astype(np.float64)
        kind = i % 4
        if kind == 0:
            m = m + 0.5                      # ties: half-even rounding decides
            m[0] = 255.0
        elif kind == 1:
            m = np.sign(m) * 2.0 ** rng.integers(0, 8, 2 * nr)
        elif kind == 2:
            m[0] = 255.0 + 2.0 ** -15        # just past the range of e (exact above 2^-126)
            e = max(e, -100)
        else:
            m[0] = -255.0
        v[i] = np.clip(m, -255.5, 255.0 + 2.0 ** -15) * 2.0 ** e
    rx = v.astype(np.float32)
    assert np.array_equal(rx.astype(np.float64), v)  # every test value exact in FP32
    rx = rx.view(np.complex64).reshape(-1)
    w, back = run(shape, rx)
    wr = bref.compress(rx, nr)
    assert np.array_equal(w, wr), np.flatnonzero(w != wr)[:8]
    assert np.array_equal(bits(back), bits(bref.decompress(wr, nr, rx.size)))


def block_checks(words, rx, nr):
    """Properties of every block: decompressed values within 2^(e-1) of the input, and e the
    smallest exponent whose range holds the block's peak."""
    b = bref.block_size(nr)
    wpb = bref.words_per_block(b)
    e = words.reshape(-1, wpb)[:, 0].view(np.int32).astype(np.float64)
    v = rx.view(np.float32).reshape(-1, 2 * b).astype(np.float64)
    return e, v


@pytest.mark.parametrize("name", ["c2", "m"])
def test_full_size_grid_sampled(name):
    c = synth.CONFIGS[name]
    shape = c["shape"].with_slots(1)
    say(f"bfp full size {name}: {shape}")
    d = synth.make_slot(shape, synth.rng_for(c["config_id"], 0, 0), c["scs_hz"], c["pdp"],
                        c["snr_db"][-1])
    rx = np.ascontiguousarray(d["rx"]).reshape(-1)
    w, back = run(shape, rx)
    nr = shape.n_rx
    b = bref.block_size(nr)
    wpb = bref.words_per_block(b)
    n_blocks = rx.size // b
    assert w.size == n_blocks * wpb
    # every block: the error bound and exponent minimality
    e, v = block_checks(w, rx, nr)
    vb = back.view(np.float32).reshape(-1, 2 * b).astype(np.float64)
    step = np.ldexp(1.0, e.astype(np.int64))
    assert np.all(np.abs(vb - v) <= 0.5 * step[:, None])
    peak = np.abs(v).max(axis=1)
    nz = peak > 0
    assert np.all(peak[nz] <= 255.0 * step[nz]) and np.all(peak[nz] > 127.5 * step[nz])
    sqnr = 10 * np.log10(np.sum(v ** 2) / np.sum((vb - v) ** 2))
    say(f"  {n_blocks} blocks, SQNR {sqnr:.1f} dB")
    # sampled blocks: words and samples bit-exact with the oracle
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(n_blocks, 3000, replace=False))
    sub = rx.reshape(n_blocks, b)[pick].reshape(-1)
    wr = bref.compress(sub, b)
    assert np.array_equal(w.reshape(n_blocks, wpb)[pick].reshape(-1), wr)
    assert np.array_equal(bits(back.reshape(n_blocks, b)[pick].reshape(-1)),
                          bits(bref.decompress(wr, b, sub.size)))


def test_receive_on_decompressed_grid():
    """The one-launch chain on a decompressed 4 x 2 QPSK slot at 20 dB: every hard decision
    is the transmitted bit, and the LLRs match the oracle chain run on the oracle's
    decompression of the same words."""
    c = synth.CONFIGS["c1"]
    shape = c["shape"].with_slots(1)
    d = synth.make_slot(shape, synth.rng_for(c["config_id"], 0, 0), c["scs_hz"], c["pdp"], 20.0)
    rx = np.ascontiguousarray(d["rx"]).reshape(-1)
    w = ranphy.bfp_compress(shape, torch.from_numpy(rx).cuda())
    rxd = ranphy.bfp_decompress(shape, w)
    pil = torch.from_numpy(np.ascontiguousarray(d["pilots"])).cuda().reshape(-1)
    nvar = torch.tensor([d["noise_var"]], dtype=torch.float32, device="cuda")
    llr = ranphy.receive(shape, rxd, pil, nvar)
    torch.cuda.synchronize()
    wr = bref.compress(rx, shape.n_rx)
    assert np.array_equal(w.cpu().numpy().view(np.uint32), wr)
    rxr = bref.decompress(wr, shape.n_rx, rx.size).reshape((1,) + d["rx"].shape)
    hr = oracle.chest_ls(shape, rxr, d["pilots"][None], oracle.H_PILOT).astype(np.complex64)
    xr, nvr = oracle.mmse_detect(shape, rxr, hr, oracle.H_PILOT,
                                 np.array([d["noise_var"]], np.float32))
    lr = oracle.llr_demap(shape, xr.astype(np.complex64), nvr.astype(np.float32))[0]
    lg = llr.cpu().numpy().reshape(lr.shape)
    assert np.array_equal((lg < 0).astype(np.uint8), d["bits"])
    dl = np.abs(lg - lr) / (np.abs(lr) + 1e-3)
    assert np.median(dl) < 1e-4 and np.quantile(dl, 0.999) < 1e-2, np.quantile(dl, 0.999)


# ---- decompression fused into the loads of the estimator and the detector ----------------

def _slot(shape, seed, snr=20.0):
    d = synth.make_slot(shape.with_slots(1), np.random.default_rng(seed), 30e3, ("exp", 1e-7), snr)
    return d


def _batch(shape, seed):
    """Slots of `shape` (n_slots of them) stacked, with words from the oracle's compressor."""
    ds = [_slot(shape, seed + i) for i in range(shape.n_slots)]
    rx = np.ascontiguousarray(np.stack([d["rx"] for d in ds])).reshape(-1)
    pil = np.ascontiguousarray(np.stack([d["pilots"] for d in ds])).reshape(-1)
    nv = np.array([d["noise_var"] for d in ds], np.float32)
    words = bref.compress(rx, shape.n_rx).view(np.int32)
    return (torch.from_numpy(words).cuda(), torch.from_numpy(pil).cuda(),
            torch.from_numpy(nv).cuda())


CHEST_SHAPES = {
    "64x16_comb8_td2": SlotShape(n_prb=3, n_symb=14, n_rx=64, n_layers=16, qm=6, dmrs_comb=8,
                                 dmrs_td=2, dmrs_sym0=(2,), n_slots=2),
    "16x4_2occ": SlotShape(n_prb=5, n_symb=14, n_rx=16, n_layers=4, qm=8, dmrs_comb=4, dmrs_td=1,
                           dmrs_sym0=(2, 11), n_slots=2),
    "12x3_odd": SlotShape(n_prb=7, n_symb=14, n_rx=12, n_layers=3, qm=4, dmrs_comb=2, dmrs_td=2,
                          dmrs_sym0=(3,), n_slots=1),
    "2x2": SlotShape(n_prb=4, n_symb=14, n_rx=2, n_layers=2, qm=2, dmrs_comb=2, dmrs_td=1,
                     dmrs_sym0=(2,), n_slots=3),
}


@pytest.mark.parametrize("name", sorted(CHEST_SHAPES))
@pytest.mark.parametrize("h_res", [0, 1])
def test_fused_estimate_equals_estimate_of_decompressed_grid(name, h_res):
    shape = CHEST_SHAPES[name]
    say(f"chest_ls_bfp {name} h_res={h_res}")
    words, pil, _ = _batch(shape, 300)
    rx = ranphy.bfp_decompress(shape, words)
    h_ref = ranphy.chest_ls(shape, rx, pil, h_res=h_res)
    h = ranphy.chest_ls_bfp(shape, words, pil, h_res=h_res)
    torch.cuda.synchronize()
    assert torch.equal(h.view(torch.int64), h_ref.view(torch.int64))


MFMA_SHAPES = {
    "64x16": SlotShape(n_prb=3, n_symb=14, n_rx=64, n_layers=16, qm=6, dmrs_comb=8, dmrs_td=2,
                       dmrs_sym0=(2,), n_slots=2),
    "32x7_256qam": SlotShape(n_prb=4, n_symb=14, n_rx=32, n_layers=7, qm=8, dmrs_comb=4,
                             dmrs_td=2, dmrs_sym0=(2,), n_slots=1),
    "16x5_short": SlotShape(n_prb=2, n_symb=7, n_rx=16, n_layers=5, qm=4, dmrs_comb=4, dmrs_td=2,
                            dmrs_sym0=(5,), n_slots=2),
}


@pytest.mark.parametrize("name", sorted(MFMA_SHAPES))
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_fused_detector_equals_detector_on_decompressed_grid(name, prec):
    """x, nv and LLRs bit for bit equal to ranphy_mmse_llr on the decompressed grid, every
    precision; the channel is made near-collinear on some subcarriers so that the FP64 route
    (which reads the samples again) runs too."""
    shape = MFMA_SHAPES[name]
    say(f"mmse_llr_bfp {name} prec={prec}")
    words, pil, nvar = _batch(shape, 400)
    rx = ranphy.bfp_decompress(shape, words)
    h = ranphy.chest_ls(shape, rx, pil)
    hv = h.view(shape.n_slots, shape.n_occ, -1, shape.n_rx, shape.n_layers)
    hv[:, :, ::5, :, 1] = hv[:, :, ::5, :, 0] * (1 + 1e-6)  # ill-conditioned pilot rows
    nvar = nvar * 1e-4
    out = {}
    for tag, fn, src in (("plain", ranphy.mmse_llr, rx), ("bfp", ranphy.mmse_llr_bfp, words)):
        x = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_X) // 2, dtype=torch.complex64,
                        device="cuda")
        nv = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_NV), device="cuda")
        llr = fn(shape, src, h, nvar, x=x, nv=nv, precision=prec)
        out[tag] = (x, nv, llr)
    torch.cuda.synchronize()
    for a, b in zip(out["plain"], out["bfp"]):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_fused_chain_full_size_64x16():
    """The compressed chain on the full 64 x 16 slot (273 PRB): estimate and LLRs from the
    words equal the FP32 chain on the decompressed grid bit for bit, and at 30 dB the 9-bit
    compression costs at most a few bit errors against the chain on the uncompressed grid."""
    c = synth.CONFIGS["m"]
    shape = c["shape"].with_slots(1)
    say(f"bfp full chain {shape}")
    d = synth.make_slot(shape, synth.rng_for(c["config_id"], 6, 0), c["scs_hz"], c["pdp"], 30.0)
    rxh = np.ascontiguousarray(d["rx"]).reshape(-1)
    words = ranphy.bfp_compress(shape, torch.from_numpy(rxh).cuda())
    pil = torch.from_numpy(np.ascontiguousarray(d["pilots"])).cuda().reshape(-1)
    nvar = torch.tensor([d["noise_var"]], dtype=torch.float32, device="cuda")
    rx = ranphy.bfp_decompress(shape, words)
    h_ref = ranphy.chest_ls(shape, rx, pil)
    l_ref = ranphy.mmse_llr(shape, rx, h_ref, nvar)
    h = ranphy.chest_ls_bfp(shape, words, pil)
    llr = ranphy.mmse_llr_bfp(shape, words, h, nvar)
    torch.cuda.synchronize()
    assert torch.equal(h.view(torch.int64), h_ref.view(torch.int64))
    assert torch.equal(llr.view(torch.int32), l_ref.view(torch.int32))
    l_fp = ranphy.mmse_llr(shape, torch.from_numpy(rxh).cuda(),
                           ranphy.chest_ls(shape, torch.from_numpy(rxh).cuda(), pil), nvar)
    bits = d["bits"].reshape(-1) > 0
    e_bfp = int(np.sum((llr.cpu().numpy() < 0) != bits))
    e_fp = int(np.sum((l_fp.cpu().numpy() < 0) != bits))
    say(f"  bit errors: BFP input {e_bfp}, FP32 input {e_fp} of {bits.size}")
    assert e_bfp <= 1.1 * e_fp + 20


RECEIVE_SHAPES = {
    "4x2_qpsk": SlotShape(n_prb=6, n_symb=14, n_rx=4, n_layers=2, qm=2, dmrs_comb=2, dmrs_td=1,
                          dmrs_sym0=(2,), n_slots=2),
    "16x4_2occ_256qam": SlotShape(n_prb=9, n_symb=14, n_rx=16, n_layers=4, qm=8, dmrs_comb=4,
                                  dmrs_td=1, dmrs_sym0=(2, 11), n_slots=2),
    "8x8_td2": SlotShape(n_prb=5, n_symb=14, n_rx=8, n_layers=8, qm=2, dmrs_comb=4, dmrs_td=2,
                         dmrs_sym0=(2,), n_slots=2),
    "12x3_3occ": SlotShape(n_prb=7, n_symb=14, n_rx=12, n_layers=3, qm=6, dmrs_comb=4,
                           dmrs_td=1, dmrs_sym0=(2, 6, 10), n_slots=1),
    "32x6_2occ": SlotShape(n_prb=4, n_symb=14, n_rx=32, n_layers=6, qm=4, dmrs_comb=4, dmrs_td=2,
                           dmrs_sym0=(2, 10), n_slots=1),
    "1x1": SlotShape(n_prb=3, n_symb=14, n_rx=1, n_layers=1, qm=4, dmrs_comb=2, dmrs_td=1,
                     dmrs_sym0=(3,), n_slots=2),
}


@pytest.mark.parametrize("name", sorted(RECEIVE_SHAPES))
def test_fused_one_launch_chain_equals_chain_on_decompressed_grid(name):
    """ranphy_receive_bfp: every path of the one-launch chain (per RE, channel pairs, factor,
    filter) reading the words gives ranphy_receive's LLRs on the decompressed grid bit for bit."""
    shape = RECEIVE_SHAPES[name]
    say(f"receive_bfp {name}")
    words, pil, nvar = _batch(shape, 500)
    rx = ranphy.bfp_decompress(shape, words)
    ref = ranphy.receive(shape, rx, pil, nvar)
    llr = ranphy.receive_bfp(shape, words, pil, nvar)
    torch.cuda.synchronize()
    assert torch.equal(llr.view(torch.int32), ref.view(torch.int32))


def test_fused_one_launch_chain_full_size_16x4():
    c = synth.CONFIGS["c2"]
    shape = c["shape"].with_slots(2)
    say(f"receive_bfp full size {shape}")
    ds = [synth.make_slot(shape.with_slots(1), synth.rng_for(c["config_id"], i, 0), c["scs_hz"],
                          c["pdp"], c["snr_db"][i]) for i in range(2)]
    rx = torch.from_numpy(np.ascontiguousarray(np.stack([d["rx"] for d in ds]))).cuda().reshape(-1)
    pil = torch.from_numpy(np.ascontiguousarray(np.stack([d["pilots"] for d in ds]))).cuda().reshape(-1)
    nvar = torch.tensor([d["noise_var"] for d in ds], dtype=torch.float32, device="cuda")
    words = ranphy.bfp_compress(shape, rx)
    ref = ranphy.receive(shape, ranphy.bfp_decompress(shape, words), pil, nvar)
    llr = ranphy.receive_bfp(shape, words, pil, nvar)
    torch.cuda.synchronize()
    assert torch.equal(llr.view(torch.int32), ref.view(torch.int32))


def test_launch_chunking_past_2_26_blocks():
    """A grid of more than 2^26 blocks (368 slots of the 64-antenna, 273-PRB shape: 67.4 M
    blocks, 8.6 GB of samples) takes two launches per direction: every block must satisfy
    the error bound and exponent minimality, and blocks on both sides of the chunk boundary
    must match the oracle bit for bit."""
    shape = synth.CONFIGS["m"]["shape"].with_slots(368)
    n = ranphy.buffer_floats(shape, ranphy.BUF_RX) // 2
    n_blocks = n // 16
    assert n_blocks > (1 << 26)
    say(f"bfp chunking: {n_blocks} blocks")
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    rx = torch.randn(n, dtype=torch.complex64, device="cuda", generator=g)
    words = ranphy.bfp_compress(shape, rx)
    back = ranphy.bfp_decompress(shape, words)
    torch.cuda.synchronize()
    v = torch.view_as_real(rx).reshape(n_blocks, 32)
    vb = torch.view_as_real(back).reshape(n_blocks, 32)
    e = words.view(n_blocks, 10)[:, 0].to(torch.float64)
    step = torch.pow(2.0, e).to(torch.float64)
    err = (vb.double() - v.double()).abs().amax(dim=1)
    assert bool((err <= 0.5 * step).all())
    peak = v.double().abs().amax(dim=1)
    assert bool((peak <= 255.0 * step).all()) and bool((peak > 127.5 * step).all())
    del v, vb, err, peak, step, e
    lo, hi = (1 << 26) - 64, (1 << 26) + 64
    sub = rx.view(n_blocks, 16)[lo:hi].cpu().numpy().reshape(-1)
    wr = bref.compress(sub, 16)
    assert np.array_equal(words.view(n_blocks, 10)[lo:hi].cpu().numpy().view(np.uint32).reshape(-1), wr)
    assert np.array_equal(bits(back.view(n_blocks, 16)[lo:hi].cpu().numpy().reshape(-1)),
                          bits(bref.decompress(wr, 16, sub.size)))


def _replay_check(step, outs, refs):
    """Capture `step` (writing `outs`) in a HIP graph after one eager warm-up on a side stream,
    then replay it three times with eager work (refilling the outputs) between replays;
    every replay must reproduce the eager results bit for bit."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for i in range(3):
        for o in outs:
            o.view(torch.int32).fill_(i - 7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, refs):
            assert torch.equal(o.view(torch.int32), r.view(torch.int32)), i


def test_graph_replay_of_the_word_reading_chains():
    """HIP-graph capture of the chains that read BFP words: the estimator and the
    matrix-core detector (64 x 16), and the one-launch chain (16 x 4, two occasions)."""
    shape = MFMA_SHAPES["64x16"]
    words, pil, nvar = _batch(shape, 700)
    h_ref = ranphy.chest_ls_bfp(shape, words, pil)
    l_ref = ranphy.mmse_llr_bfp(shape, words, h_ref, nvar)
    torch.cuda.synchronize()
    h = torch.empty_like(h_ref)
    llr = torch.empty_like(l_ref)

    def step():
        ranphy.chest_ls_bfp(shape, words, pil, h=h)
        ranphy.mmse_llr_bfp(shape, words, h, nvar, llr=llr)
    _replay_check(step, [h, llr], [h_ref, l_ref])

    shape2 = RECEIVE_SHAPES["16x4_2occ_256qam"]
    words2, pil2, nvar2 = _batch(shape2, 710)
    ref2 = ranphy.receive_bfp(shape2, words2, pil2, nvar2)
    torch.cuda.synchronize()
    out2 = torch.empty_like(ref2)
    _replay_check(lambda: ranphy.receive_bfp(shape2, words2, pil2, nvar2, llr=out2), [out2], [ref2])
