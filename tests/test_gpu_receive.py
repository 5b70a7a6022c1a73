"""GPU parity of the one-launch chain (ranphy_receive): LS estimate, interpolation, LMMSE
detection and max-log demapping in one kernel, against the FP64 oracle chain on identical
input bytes, hard decisions bit-exact away from decision boundaries and every LLR within 1e-3 |LLR| + 1e-4
of the oracle's or inside the range the FP32 forward-error bound of its Gram matrix allows;
graph replay and bitwise determinism; the full-size workload sampled per slot."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2510_07843_amd as ranphy
import synth
from synth import SlotShape
import parity
from parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ranphy.lib()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


def oracle_chain(shape, rx, pil, nvar):
    hr = oracle.chest_ls(shape, rx, pil, oracle.H_PILOT).astype(np.complex64)
    xr, nvr = oracle.mmse_detect(shape, rx, hr, oracle.H_PILOT, nvar)
    lr = oracle.llr_demap(shape, xr.astype(np.complex64), nvr.astype(np.float32))
    return dict(h=hr, x=xr, nv=nvr, llr=lr, noise_var=nvar)


def check(shape, lg, ref, label="receive"):
    """Hard decisions bit-exact away from boundaries; every LLR within 1e-3 |LLR| + 1e-4 of
    the oracle's, or else inside the range the FP32 forward-error bound of its Gram matrix
    allows (every such LLR audited; counts printed)."""
    grams = parity.gram_fn(shape, ref["h"], oracle.H_PILOT, ref["noise_var"])
    xr = ref["x"].reshape(-1, shape.n_layers)
    parity.audit_llrs(lg, ref["llr"], ref["x"], ref["nv"],
                      parity.kappa_radius(grams, xr, shape.n_layers), shape.qm, label)


def make(shape, seed, snr_db=20.0, pdp=("exp", 100e-9), doppler=None):
    rx = np.empty((shape.n_slots, shape.n_symb, shape.n_sc, shape.n_rx), np.complex64)
    pil = np.empty((shape.n_slots, shape.n_occ, shape.dmrs_td, shape.n_pilot, shape.n_layers),
                   np.complex64)
    nvar = np.empty(shape.n_slots, np.float32)
    for s in range(shape.n_slots):
        d = synth.make_slot(shape, synth.rng_for(91, seed, s), 30e3, pdp, snr_db)
        rx[s], pil[s], nvar[s] = d["rx"], d["pilots"], d["noise_var"]
    return rx, pil, nvar


SHAPES = {
    "c1": synth.CONFIGS["c1"]["shape"].with_slots(2),
    "c2": synth.CONFIGS["c2"]["shape"].with_slots(2),
    "prb1_l1": SlotShape(1, 14, 2, 1, 2, 2, 1, (2,), 3),
    "prb5_l3_c8": SlotShape(5, 14, 8, 3, 4, 8, 1, (2,), 2),
    "prb7_l5_c4t2": SlotShape(7, 14, 12, 5, 6, 4, 2, (2,), 2),
    "prb3_l7_3occ": SlotShape(3, 14, 16, 7, 8, 4, 2, (1, 6, 11), 2),
    "prb4_short": SlotShape(4, 7, 4, 2, 4, 2, 1, (0,), 2),
    "prb2_l8_r64": SlotShape(2, 14, 64, 8, 8, 4, 2, (2,), 2),
    "prb9_l6_2occ_r40": SlotShape(9, 14, 40, 6, 4, 8, 1, (2, 10), 1),
    "prb1_l4_dmrs_end": SlotShape(1, 14, 32, 4, 6, 2, 2, (12,), 2),
    # two occasions up to 4 layers: the per-subcarrier channel pairs and Gram pieces
    "prb7_l3_r12_2occ": SlotShape(7, 14, 12, 3, 6, 4, 1, (1, 10), 2),
    "prb3_l2_r64_2occ": SlotShape(3, 14, 64, 2, 4, 2, 1, (2, 11), 2),
    "prb4_l4_short_2occ": SlotShape(4, 7, 8, 4, 2, 4, 1, (0, 5), 2),
    "prb2_l1_r4_2occ_td2": SlotShape(2, 14, 4, 1, 8, 2, 2, (2, 10), 3),
    "p2": synth.CONFIGS["p2"]["shape"].with_slots(2),
    "p4": synth.CONFIGS["p4"]["shape"].with_slots(2),
    "p8": synth.CONFIGS["p8"]["shape"].with_slots(2),
}


@pytest.mark.parametrize("name", list(SHAPES))
def test_receive_matches_oracle_chain(name):
    shape = SHAPES[name]
    say(f"receive {name}: {shape.n_prb} PRB {shape.n_rx}x{shape.n_layers} qm {shape.qm} "
        f"occ {shape.dmrs_sym0} slots {shape.n_slots}")
    rx, pil, nvar = make(shape, 1)
    nvar = nvar * np.linspace(0.7, 1.4, shape.n_slots).astype(np.float32)
    lg = ranphy.receive(shape, dev(rx), dev(pil), dev(nvar))
    torch.cuda.synchronize()
    lg = lg.cpu().numpy().reshape(shape.n_slots, shape.n_dsym, shape.n_sc, shape.n_layers,
                                  shape.qm)
    check(shape, lg, oracle_chain(shape, rx, pil, nvar))


def test_receive_equals_three_call_chain_bits_where_arithmetic_matches():
    # Same slot through the one-launch chain and the three calls: hard decisions agree on every
    # bit away from boundaries (the two paths round differently, so only decisions compare).
    shape = SHAPES["c2"]
    rx, pil, nvar = make(shape, 2, snr_db=25.0)
    lg = ranphy.receive(shape, dev(rx), dev(pil), dev(nvar))
    h = ranphy.chest_ls(shape, dev(rx), dev(pil), h_res=ranphy.H_PILOT)
    x, nv = ranphy.mmse_detect(shape, dev(rx), h, dev(nvar), h_res=ranphy.H_PILOT)
    l3 = ranphy.llr_demap(shape, x, nv)
    torch.cuda.synchronize()
    a, b = lg.cpu().numpy(), l3.cpu().numpy()
    near = np.abs(b) <= 1e-3 * np.abs(b).max()
    assert np.array_equal((a < 0) | near, (b < 0) | near)
    assert np.allclose(a, b, rtol=1e-3, atol=1e-3 * np.abs(b).max())


def test_receive_empty_and_deterministic():
    shape = SHAPES["prb7_l5_c4t2"]
    e = torch.empty(0, dtype=torch.complex64, device="cuda")
    ranphy.receive(shape.with_slots(0), e, e, torch.empty(0, device="cuda"),
                   llr=torch.empty(0, device="cuda"))
    rx, pil, nvar = make(shape, 3)
    outs = [ranphy.receive(shape, dev(rx), dev(pil), dev(nvar)) for _ in range(3)]
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert torch.equal(o.view(torch.int32), outs[0].view(torch.int32))


def test_receive_graph_replay():
    shape = SHAPES["c2"]
    rx, pil, nvar = make(shape, 4)
    rx, pil, nvar = dev(rx), dev(pil), dev(nvar)
    ref = ranphy.receive(shape, rx, pil, nvar)
    torch.cuda.synchronize()
    out = torch.full_like(ref, 5.0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ranphy.receive(shape, rx, pil, nvar, llr=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ranphy.receive(shape, rx, pil, nvar, llr=out)
    for i in range(3):
        out.fill_(float(i) - 9.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), i


@pytest.mark.parametrize("name", ["c2", "prb3_l2_r64_2occ", "prb9_l6_2occ_r40"])
def test_receive_eight_byte_aligned_buffers(name):
    # The received grid and the LLR buffer 8-byte but not 16-byte aligned (the library's
    # minimum): the group line loads and record stores then move 8-byte pieces; the LLRs must
    # equal those of 16-byte aligned buffers bit for bit, and the word before the LLRs must
    # stay untouched.
    shape = SHAPES[name]
    rx, pil, nvar = make(shape, 5)
    rxd, pild, nvd = dev(rx), dev(pil), dev(nvar)
    ref = ranphy.receive(shape, rxd, pild, nvd)
    rx_big = torch.empty(rxd.numel() + 1, dtype=torch.complex64, device="cuda")
    rx_big[1:] = rxd
    llr_big = torch.full((ref.numel() + 2,), 7.0, dtype=torch.float32, device="cuda")
    assert (rx_big[1:].data_ptr() % 16, llr_big[2:].data_ptr() % 16) == (8, 8)
    ranphy.receive(shape, rx_big[1:], pild, nvd, llr=llr_big[2:])
    torch.cuda.synchronize()
    assert torch.equal(llr_big[2:].view(torch.int32), ref.view(torch.int32))
    assert llr_big[:2].tolist() == [7.0, 7.0]


@pytest.mark.parametrize("cfg", ["c2", "p8"])
def test_receive_full_size_sampled(cfg):
    # The configuration at the slot count the benchmark times; the oracle chain on a sample
    # of slots (first, last and a middle one).
    b = synth.make_batch(cfg, workers=8)
    shape = b["shape"]
    say(f"receive full size {cfg}: {shape.n_slots} slots")
    lg = ranphy.receive(shape, dev(b["rx"]), dev(b["pilots"]), dev(b["noise_var"]))
    torch.cuda.synchronize()
    lg = lg.cpu().numpy().reshape(shape.n_slots, shape.n_dsym, shape.n_sc, shape.n_layers,
                                  shape.qm)
    for s in sorted({0, shape.n_slots // 2, shape.n_slots - 1}):
        one = shape.with_slots(1)
        ref = oracle_chain(one, b["rx"][s:s + 1], b["pilots"][s:s + 1], b["noise_var"][s:s + 1])
        check(one, lg[s:s + 1], ref)


MFMA_RECEIVE = {
    "64x16_3prb": SlotShape(n_prb=3, n_symb=14, n_rx=64, n_layers=16, qm=6, dmrs_comb=8,
                            dmrs_td=2, dmrs_sym0=(2,), n_slots=2),
    "48x12_5prb": SlotShape(n_prb=5, n_symb=14, n_rx=48, n_layers=12, qm=4, dmrs_comb=8,
                            dmrs_td=2, dmrs_sym0=(3,), n_slots=1),
    "16x9_short": SlotShape(n_prb=4, n_symb=9, n_rx=16, n_layers=9, qm=8, dmrs_comb=8, dmrs_td=2,
                            dmrs_sym0=(0,), n_slots=2),
}


@pytest.mark.parametrize("name", sorted(MFMA_RECEIVE))
def test_one_launch_above_8_layers_equals_two_call_chain(name):
    """More than 8 layers: ranphy_receive runs the matrix-core detector with the pilot-resolution
    estimate formed inside it (same arithmetic as ranphy_chest_ls), so its LLRs equal
    ranphy_chest_ls -> ranphy_mmse_llr bit for bit (odd PRB counts put pilots past the band
    edge; 48 antennas leave part of the staging threads idle); from BFP words likewise."""
    shape = MFMA_RECEIVE[name]
    say(f"receive > 8 layers {name}")
    ds = [synth.make_slot(shape.with_slots(1), np.random.default_rng(600 + i), 30e3,
                          ("exp", 1e-7), 20.0) for i in range(shape.n_slots)]
    rx = dev(np.stack([d["rx"] for d in ds]))
    pil = dev(np.stack([d["pilots"] for d in ds]))
    nvar = torch.tensor([d["noise_var"] for d in ds], dtype=torch.float32, device="cuda")
    h = ranphy.chest_ls(shape, rx, pil)
    ref = ranphy.mmse_llr(shape, rx, h, nvar)
    llr = ranphy.receive(shape, rx, pil, nvar)
    words = ranphy.bfp_compress(shape, rx)
    rxd = ranphy.bfp_decompress(shape, words)
    ref_b = ranphy.mmse_llr(shape, rxd, ranphy.chest_ls(shape, rxd, pil), nvar)
    llr_b = ranphy.receive_bfp(shape, words, pil, nvar)
    torch.cuda.synchronize()
    assert torch.equal(llr.view(torch.int32), ref.view(torch.int32))
    assert torch.equal(llr_b.view(torch.int32), ref_b.view(torch.int32))
    bits = np.stack([d["bits"] for d in ds]).reshape(-1)  # a sanity floor (256QAM at 20 dB)
    assert np.mean((llr.cpu().numpy() < 0) == (bits > 0)) > 0.9


def test_one_launch_64x16_full_size_equals_two_call_chain():
    c = synth.CONFIGS["m"]
    shape = c["shape"].with_slots(2)
    say(f"receive full size {shape}")
    ds = [synth.make_slot(shape.with_slots(1), synth.rng_for(c["config_id"], 3 + i, 0),
                          c["scs_hz"], c["pdp"], c["snr_db"][3 + i]) for i in range(2)]
    rx = dev(np.stack([d["rx"] for d in ds]))
    pil = dev(np.stack([d["pilots"] for d in ds]))
    nvar = torch.tensor([d["noise_var"] for d in ds], dtype=torch.float32, device="cuda")
    ref = ranphy.mmse_llr(shape, rx, ranphy.chest_ls(shape, rx, pil), nvar)
    llr = ranphy.receive(shape, rx, pil, nvar)
    torch.cuda.synchronize()
    assert torch.equal(llr.view(torch.int32), ref.view(torch.int32))


def test_one_launch_above_8_layers_graph_replay():
    shape = MFMA_RECEIVE["48x12_5prb"]
    ds = [synth.make_slot(shape.with_slots(1), np.random.default_rng(650), 30e3, ("exp", 1e-7),
                          15.0)]
    rx, pil = dev(np.stack([d["rx"] for d in ds])), dev(np.stack([d["pilots"] for d in ds]))
    nvar = torch.tensor([d["noise_var"] for d in ds], dtype=torch.float32, device="cuda")
    ref = ranphy.receive(shape, rx, pil, nvar)
    torch.cuda.synchronize()
    out = torch.empty_like(ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ranphy.receive(shape, rx, pil, nvar, llr=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ranphy.receive(shape, rx, pil, nvar, llr=out)
    for i in range(3):
        out.fill_(float(i) - 9.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), i
