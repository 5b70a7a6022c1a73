"""GPU parity: every call of libranphy against the FP64 oracle on identical input bytes.

Bars (floating point throughout; integer only in the hard decisions):
  * chest_ls: |h_gpu - h_ref| <= 1e-6 |h_ref| + 1e-6 max|rx|  (a sum of T <= 2 products).
  * mmse_detect: per resource element ||x_gpu - x_ref|| / ||x_ref|| <= 1e-4 and the same
    relative bound on nv; an element over it must lie within the FP32 forward-error bound
    8 kappa(G) Nl 2^-24 of its Gram matrix (counted and printed, never loosened).
  * llr_demap (per call, identical x and nv): |llr_gpu - llr_ref| <= 1e-3 |llr_ref| + 1e-4.
  * end to end: hard decisions bit-exact and LLRs within the per-call bar for every bit whose
    oracle value is away from a decision boundary (axis distance > 1e-3 and |llr| > 1e-3);
    the excluded bits are counted and printed.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2510_07843_amd as ranphy
import synth
from synth import SlotShape

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ranphy.lib()  # raises if the library is not built


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().reshape(-1)


def host(t, shape):
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(shape)


def make_inputs(shape, seed, snr_db=20.0, scs=30e3, pdp=("exp", 100e-9), noiseless=False):
    rx = np.empty((shape.n_slots, shape.n_symb, shape.n_sc, shape.n_rx), np.complex64)
    pil = np.empty((shape.n_slots, shape.n_occ, shape.dmrs_td, shape.n_pilot, shape.n_layers), np.complex64)
    bits, xs = [], []
    nvar = np.full(shape.n_slots, 10 ** (-snr_db / 10), np.float32)
    for s in range(shape.n_slots):
        d = synth.make_slot(shape, synth.rng_for(77, seed, s), scs, pdp, snr_db, noiseless=noiseless)
        rx[s], pil[s] = d["rx"], d["pilots"]
        bits.append(d["bits"])
        xs.append(d["x"])
    return rx, pil, nvar, np.stack(bits), np.stack(xs)


def h_shape(shape, h_res):
    K = shape.n_pilot if h_res == ranphy.H_PILOT else shape.n_sc
    return (shape.n_slots, shape.n_occ, K, shape.n_rx, shape.n_layers)


def out_shape(shape):
    return (shape.n_slots, shape.n_dsym, shape.n_sc, shape.n_layers)


def gpu_chest(shape, rx, pil, h_res):
    h = ranphy.chest_ls(shape, dev(rx), dev(pil), h_res=h_res)
    return host(h, h_shape(shape, h_res))


def gpu_mmse(shape, rx, h, h_res, nvar):
    x, nv = ranphy.mmse_detect(shape, dev(rx), dev(h), dev(nvar), h_res=h_res)
    return host(x, out_shape(shape)), host(nv, out_shape(shape))


def gpu_llr(shape, x, nv):
    llr = ranphy.llr_demap(shape, dev(x.astype(np.complex64)), dev(nv.astype(np.float32)))
    return host(llr, out_shape(shape) + (shape.qm,))


def check_chest(hg, hr, rx):
    tol = 1e-6 * np.abs(hr) + 1e-6 * np.abs(rx).max()
    bad = np.abs(hg - hr) > tol
    assert not bad.any(), f"{bad.sum()} channel values over tolerance"


def check_mmse(shape, h, h_res, nvar, xg, nvg, xr, nvr):
    """Per-RE relative error on x and nv; elements over 1e-4 need the kappa bound."""
    err_x = np.linalg.norm(xg - xr, axis=-1) / np.linalg.norm(xr, axis=-1)
    err_v = np.max(np.abs(nvg - nvr) / np.abs(nvr), axis=-1) if np.all(nvr > 0) else \
        np.max(np.abs(nvg - nvr) / np.maximum(np.abs(nvr), 1e-30), axis=-1)
    over = np.argwhere((err_x > 1e-4) | (err_v > 1e-4))
    ds = shape.data_symbols()
    for (s, di, k) in over[:2000]:
        H = oracle.channel_at(shape, h, h_res, int(s), int(k), ds[di])
        G = H.conj().T @ H + float(nvar[s]) * np.eye(shape.n_layers)
        kappa = np.linalg.cond(G)
        bound = 8 * kappa * shape.n_layers * U32
        assert max(err_x[s, di, k], err_v[s, di, k]) <= bound, \
            (s, di, k, err_x[s, di, k], err_v[s, di, k], kappa)
    say(f"mmse parity: {err_x.size} REs, max rel err x {err_x.max():.2e} nv {err_v.max():.2e}, "
        f"{len(over)} over 1e-4 (all within the kappa bound)")
    return err_x


def llr_tol_ok(lg, lr):
    return np.abs(lg - lr) <= 1e-3 * np.abs(lr) + 1e-4


def axis_margin(x, qm):
    """Distance (normalised units) of each bit's axis value to that bit's nearest decision
    boundary, per bit in the [..][qm] order (b0, b2, .. in-phase; b1, b3, .. quadrature)."""
    m = qm // 2
    scale = synth.qam_scale(qm)
    out = np.zeros(x.shape + (qm,))
    for ax, v in ((0, x.real), (1, x.imag)):
        t = v * scale
        for i in range(m):
            if i > 0:
                t = 2.0 ** (m - i) - np.abs(t)
            out[..., 2 * i + ax] = np.abs(t) / scale
    return out


# ---------------------------------------------------------------------------------------
# Shapes: the three workloads (reduced slot counts) plus ragged and edge shapes.
# ---------------------------------------------------------------------------------------

C1 = synth.CONFIGS["c1"]["shape"]
C2 = synth.CONFIGS["c2"]["shape"]
M = synth.CONFIGS["m"]["shape"]

SHAPES = {
    "c1": C1.with_slots(2),
    "c2": C2.with_slots(2),
    "m": M.with_slots(1),
    # ragged: odd PRB count with comb 8 (n_sc/8 not an integer), odd layer counts
    "prb1_l1": SlotShape(1, 14, 2, 1, 2, 2, 1, (2,), 3),
    "prb5_l3_c8": SlotShape(5, 14, 8, 3, 4, 8, 1, (2,), 2),
    "prb7_l5_c4t2": SlotShape(7, 14, 12, 5, 6, 4, 2, (2,), 2),
    "prb3_l7_3occ": SlotShape(3, 14, 16, 7, 8, 4, 2, (1, 6, 11), 2),
    "prb11_l16_c8t2": SlotShape(11, 14, 64, 16, 6, 8, 2, (2,), 1),
    "prb9_l12_2occ": SlotShape(9, 14, 40, 12, 4, 8, 2, (2, 10), 1),
    "prb13_l16_r17": SlotShape(13, 14, 17, 16, 2, 8, 2, (3,), 1),
    "prb4_short": SlotShape(4, 7, 4, 2, 4, 2, 1, (0,), 2),
    # matrix-core detector shapes (one occasion, 5..16 layers, Nr a multiple of 16)
    "prb5_l9_r32": SlotShape(5, 14, 32, 9, 4, 8, 2, (2,), 2),
    "prb3_l12_r48": SlotShape(3, 14, 48, 12, 6, 8, 2, (3,), 2),
    "prb2_l5_r16": SlotShape(2, 14, 16, 5, 2, 4, 2, (2,), 3),
    "prb4_l8_short": SlotShape(4, 7, 16, 8, 4, 4, 2, (0,), 2),
    "prb1_l16_dmrs_end": SlotShape(1, 14, 64, 16, 8, 8, 2, (12,), 2),
    # the paper's square shapes at 60 RB
    "p2": synth.CONFIGS["p2"]["shape"].with_slots(2),
    "p4": synth.CONFIGS["p4"]["shape"].with_slots(2),
    "p8": synth.CONFIGS["p8"]["shape"].with_slots(2),
}


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("h_res", [ranphy.H_PILOT, ranphy.H_FULL])
def test_chest_ls_parity(name, h_res):
    shape = SHAPES[name]
    say(f"chest_ls {name} h_res={h_res}")
    rx, pil, *_ = make_inputs(shape, 1)
    hg = gpu_chest(shape, rx, pil, h_res)
    hr = oracle.chest_ls(shape, rx, pil, h_res)
    check_chest(hg, hr, rx)


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("h_res", [ranphy.H_PILOT, ranphy.H_FULL])
def test_mmse_detect_parity(name, h_res):
    shape = SHAPES[name]
    say(f"mmse_detect {name} h_res={h_res}")
    rx, pil, nvar, *_ = make_inputs(shape, 2, snr_db=15.0)
    nvar = nvar * np.linspace(0.5, 2.0, shape.n_slots).astype(np.float32)  # per-slot s2
    h = oracle.chest_ls(shape, rx, pil, h_res).astype(np.complex64)
    xg, nvg = gpu_mmse(shape, rx, h, h_res, nvar)
    xr, nvr = oracle.mmse_detect(shape, rx, h, h_res, nvar)
    check_mmse(shape, h, h_res, nvar, xg, nvg, xr, nvr)


@pytest.mark.parametrize("qm", [2, 4, 6, 8])
def test_llr_demap_parity(qm):
    say(f"llr_demap qm={qm}")
    shape = SlotShape(5, 14, 4, 3, qm, 4, 1, (2,), 2)
    rng = np.random.default_rng(qm)
    n = out_shape(shape)
    x = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 0.8).astype(np.complex64)
    nv = rng.uniform(1e-3, 2.0, n).astype(np.float32)
    lg = gpu_llr(shape, x, nv)
    lr = oracle.llr_demap(shape, x, nv)
    ok = llr_tol_ok(lg, lr)
    assert ok.all(), (np.argwhere(~ok)[:5], lg[~ok][:5], lr[~ok][:5])


def test_llr_demap_noiseless_constellation():
    for qm in (2, 4, 6, 8):
        M_ = 1 << qm
        shape = SlotShape(2, 14, 1, 1, qm, 2, 1, (2,), 1)  # 312 data REs >= 256 points
        bits = ((np.arange(M_)[:, None] >> np.arange(qm)[::-1]) & 1).astype(np.uint8)
        pts = synth.qam_map(bits, qm)
        x = np.zeros(out_shape(shape), np.complex64).reshape(-1)
        x[: M_] = pts
        lg = gpu_llr(shape, x.reshape(out_shape(shape)), np.full(out_shape(shape), 0.05, np.float32))
        assert np.array_equal((lg.reshape(-1, qm)[:M_] < 0).astype(np.uint8), bits)


def end_to_end(shape, rx, pil, nvar, h_res=ranphy.H_PILOT):
    """GPU chain and oracle chain on the same received grid."""
    hg = ranphy.chest_ls(shape, dev(rx), dev(pil), h_res=h_res)
    xg, nvg = ranphy.mmse_detect(shape, dev(rx), hg, dev(nvar), h_res=h_res)
    lg = ranphy.llr_demap(shape, xg, nvg)
    lg = host(lg, out_shape(shape) + (shape.qm,))
    xg = host(xg, out_shape(shape))
    hr = oracle.chest_ls(shape, rx, pil, h_res)
    xr, nvr = oracle.mmse_detect(shape, rx, hr.astype(np.complex64), h_res, nvar)
    lr = oracle.llr_demap(shape, xr.astype(np.complex64), nvr.astype(np.float32))
    return xg, lg, xr, nvr, lr


def check_end_to_end(shape, xg, lg, xr, lr):
    err = np.linalg.norm(xg - xr, axis=-1) / np.linalg.norm(xr, axis=-1)
    margin = axis_margin(xr, shape.qm)
    keep = (margin > 1e-3) & (np.abs(lr) > 1e-3)
    hard_g, hard_r = lg < 0, lr < 0
    mism = (hard_g != hard_r) & keep
    assert not mism.any(), f"{mism.sum()} hard decisions differ away from boundaries"
    ok = llr_tol_ok(lg, lr) | ~keep
    say(f"end to end: {err.size} REs, max rel x err {err.max():.2e}; bits excluded near "
        f"boundaries {int((~keep).sum())} of {keep.size}; LLR out of tolerance "
        f"{int((~ok).sum())}")
    return ok


def test_end_to_end_c1_slot():
    shape = C1.with_slots(1)
    c = synth.CONFIGS["c1"]
    d = synth.make_slot(shape, synth.rng_for(c["config_id"], 0, 0), c["scs_hz"], c["pdp"], 20.0)
    rx, pil = d["rx"][None], d["pilots"][None]
    nvar = np.array([d["noise_var"]], np.float32)
    xg, lg, xr, nvr, lr = end_to_end(shape, rx, pil, nvar)
    ok = check_end_to_end(shape, xg, lg, xr, lr)
    # LLRs: the per-call bar holds outside the exclusion band except where the x error
    # (bounded above) times 1/nv legitimately exceeds it; those are printed, and must be few.
    assert (~ok).mean() < 1e-3
    # Against the transmitted bits: 20 dB, 4x2 QPSK is error free on this slot.
    assert np.array_equal((lg[0] < 0).astype(np.uint8), d["bits"])


@pytest.mark.parametrize("h_res", [ranphy.H_PILOT, ranphy.H_FULL])
def test_end_to_end_c2_two_slots(h_res):
    b = synth.make_batch("c2", n_slots=2, snr_db=(15.0, 30.0))
    shape = b["shape"]
    xg, lg, xr, nvr, lr = end_to_end(shape, b["rx"], b["pilots"], b["noise_var"], h_res)
    ok = check_end_to_end(shape, xg, lg, xr, lr)
    assert (~ok).mean() < 1e-3


def test_deterministic_bitwise():
    b = synth.make_batch("c2", n_slots=1)
    shape = b["shape"]
    outs = []
    for _ in range(2):
        hg = ranphy.chest_ls(shape, dev(b["rx"]), dev(b["pilots"]))
        xg, nvg = ranphy.mmse_detect(shape, dev(b["rx"]), hg, dev(b["noise_var"]))
        lg = ranphy.llr_demap(shape, xg, nvg)
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy().copy() for t in (hg, xg, nvg, lg)])
    for a, c in zip(*outs):
        assert a.tobytes() == c.tobytes()


def test_zero_noise_variance_zf_and_singular_elements():
    shape = SlotShape(2, 14, 4, 2, 2, 2, 1, (2,), 1)
    rng = np.random.default_rng(5)
    H = ((rng.standard_normal((shape.n_sc, 4, 2)) + 1j * rng.standard_normal((shape.n_sc, 4, 2))) / 2)
    H[5, :, 1] = H[5, :, 0]  # rank-deficient channel on subcarrier 5
    d = synth.make_slot(shape, rng, 15e3, "taps8", 20.0, channel=H, noiseless=True)
    hfull = H[None, None].astype(np.complex64)
    nvar = np.zeros(1, np.float32)
    xg, nvg = gpu_mmse(shape, d["rx"][None], hfull, ranphy.H_FULL, nvar)
    xr, nvr = oracle.mmse_detect(shape, d["rx"][None], hfull, ranphy.H_FULL, nvar)
    bad = np.zeros(shape.n_sc, bool)
    bad[5] = True
    assert np.all(np.isnan(xg[0, :, bad])) and np.all(np.isinf(nvg[0, :, bad]))
    assert np.all(np.isnan(xr[0, :, bad])) and np.all(np.isinf(nvr[0, :, bad]))
    good = ~bad
    np.testing.assert_allclose(xg[0][:, good], d["x"][:, good], atol=1e-3)
    assert np.all(nvg[0][:, good] == 0)


def test_empty_batch_no_op():
    shape = C1.with_slots(0)
    e = torch.empty(0, dtype=torch.complex64, device="cuda")
    ef = torch.empty(0, dtype=torch.float32, device="cuda")
    ranphy.chest_ls(shape, e, e, h=e)
    ranphy.mmse_detect(shape, e, e, ef, x=e, nv=ef)
    ranphy.llr_demap(shape, e, ef, llr=ef)
    torch.cuda.synchronize()


def test_maximum_shape_sampled():
    # 275 PRB, 64 Rx, 16 layers, 256QAM, comb 8 with a time cover: the largest descriptor.
    shape = SlotShape(275, 14, 64, 16, 8, 8, 2, (2,), 1)
    say("maximum shape 275 PRB 64x16")
    rx, pil, nvar, bits, _ = make_inputs(shape, 9, snr_db=25.0, pdp=("exp", 300e-9))
    xg, lg, xr, nvr, lr = end_to_end(shape, rx, pil, nvar)
    check_end_to_end(shape, xg, lg, xr, lr)


def test_fp32_ber_matches_fp64_over_c2_sweep():
    # Paper Fig. 5(a): single precision keeps the detection accuracy of double precision.
    b = synth.make_batch("c2", n_slots=10, workers=8)  # 2 slots at each of 10..30 dB
    shape = b["shape"]
    xg, lg, xr, nvr, lr = end_to_end(shape, b["rx"], b["pilots"], b["noise_var"])
    for i in range(len(synth.CONFIGS["c2"]["snr_db"])):
        sel = b["snr_db"] == synth.CONFIGS["c2"]["snr_db"][i]
        eg = int(np.sum((lg[sel] < 0) != b["bits"][sel]))
        er = int(np.sum((lr[sel] < 0) != b["bits"][sel]))
        n = int(b["bits"][sel].size)
        say(f"SNR {synth.CONFIGS['c2']['snr_db'][i]} dB: BER fp32 {eg / n:.3e} fp64 {er / n:.3e}")
        assert abs(eg - er) <= 3 * math.sqrt(er + 1) + 5


def sinr_db(xhat, x):
    return 10 * np.log10(np.mean(np.abs(x) ** 2) / np.mean(np.abs(xhat - x) ** 2))


def test_reduced_precision_sinr_loss_64x16():
    # 64 Rx x 16 layers, one slot at each SNR of 0..30 dB.  The Gram and matched filter with
    # FP16 or BF16 inputs (FP32 accumulation) must stay within 0.1 dB of the FP64 oracle's
    # post-equalisation SINR; the EVM of each path against the oracle is printed.
    b = synth.make_batch("m", n_slots=7, workers=8)
    shape = b["shape"]
    h = oracle.chest_ls(shape, b["rx"], b["pilots"]).astype(np.complex64)
    xr, _ = oracle.mmse_detect(shape, b["rx"], h, ranphy.H_PILOT, b["noise_var"])
    out = {}
    for name, prec in (("fp32", ranphy.PREC_FP32), ("fp16", ranphy.PREC_FP16),
                       ("bf16", ranphy.PREC_BF16)):
        x, _ = ranphy.mmse_detect(shape, dev(b["rx"]), dev(h), dev(b["noise_var"]), precision=prec)
        out[name] = host(x, out_shape(shape))
    for i, snr in enumerate(b["snr_db"]):
        ref = sinr_db(xr[i], b["x"][i])
        line = [f"SNR {snr:4.1f} dB: SINR fp64 {ref:6.2f}"]
        for name in ("fp32", "fp16", "bf16"):
            s = sinr_db(out[name][i], b["x"][i])
            evm = 10 * np.log10(np.mean(np.abs(out[name][i] - xr[i]) ** 2) / np.mean(np.abs(xr[i]) ** 2))
            line.append(f"{name} {s:6.2f} (loss {ref - s:+.3f} dB, EVM vs fp64 {evm:6.1f} dB)")
            limit = 0.005 if name == "fp32" else 0.1
            assert ref - s <= limit, (name, snr, ref, s)
        say("; ".join(line))


def ill_conditioned_case():
    """Two slots at a matrix-core shape (16 Rx x 8 layers, full-resolution channel given):
    slot 0 (s2 = 1e-6) holds i.i.d. subcarriers, near-collinear layers 1/2 (delta 1e-6) and
    exactly collinear layers 1/2 (regularised by s2 alone); slot 1 (s2 = 0, zero forcing)
    holds i.i.d. subcarriers, identical layers 4/5 (singular) and near-collinear layers 4/5
    (delta 1e-4, kappa ~ 1e9)."""
    shape = SlotShape(2, 14, 16, 8, 4, 4, 2, (2,), 2)
    nsc, NR, NL, ND = shape.n_sc, shape.n_rx, shape.n_layers, shape.n_dsym
    rng = np.random.default_rng(21)
    cn = lambda *sz: ((rng.standard_normal(sz) + 1j * rng.standard_normal(sz)) / np.sqrt(2))
    H = cn(2, nsc, NR, NL).astype(np.complex64)
    w = cn(nsc, NR).astype(np.complex64)
    H[0, 8:16, :, 2] = H[0, 8:16, :, 1] + np.complex64(1e-6) * w[8:16]
    H[0, 16:, :, 2] = H[0, 16:, :, 1]
    H[1, 8:16, :, 5] = H[1, 8:16, :, 4]
    H[1, 16:, :, 5] = H[1, 16:, :, 4] + np.complex64(1e-4) * w[16:]
    bits = rng.integers(0, 2, (2, ND, nsc, NL, shape.qm)).astype(np.uint8)
    x = synth.qam_map(bits, shape.qm)
    nvar = np.array([1e-6, 0.0], np.float32)
    rx = np.zeros((2, shape.n_symb, nsc, NR), np.complex64)
    for di, s in enumerate(shape.data_symbols()):
        rx[:, s] = np.einsum("bkrl,bkl->bkr", H.astype(np.complex128), x[:, di])
    rx[0] += (1e-3 * cn(shape.n_symb, nsc, NR)).astype(np.complex64)
    Gc = np.einsum("bkrl,bkrm->bklm", H.conj().astype(np.complex128), H.astype(np.complex128))
    Gc = Gc + nvar[:, None, None, None] * np.eye(NL)
    kappa = np.linalg.cond(Gc)  # [slot][sc]
    return shape, H[:, None], rx, nvar, kappa


@pytest.mark.parametrize("prec", [ranphy.PREC_FP32, ranphy.PREC_FP16, ranphy.PREC_BF16])
def test_fp64_route_for_ill_conditioned_grams(prec):
    # Subcarriers whose Gram condition estimate exceeds 1e6 (or whose FP32 elimination
    # fails) are solved in FP64 from the FP32 channel and samples.  Where kappa > 1e6 an FP32
    # solve is off by O(1) (forward-error bound 8 kappa Nl 2^-24 >> 1), so agreement with the
    # FP64 oracle to 1e-4 shows the FP64 route ran; exactly singular systems (zero forcing
    # with identical layers) give NaN / +inf on both sides.
    shape, h, rx, nvar, kappa = ill_conditioned_case()
    say(f"ill-conditioned Grams prec={prec}: kappa per subcarrier "
        f"{np.array2string(np.log10(kappa), precision=1, max_line_width=200)}")
    x, nv = ranphy.mmse_detect(shape, dev(rx), dev(h), dev(nvar), h_res=ranphy.H_FULL,
                               precision=prec)
    xg, nvg = host(x, out_shape(shape)), host(nv, out_shape(shape))
    xr, nvr = oracle.mmse_detect(shape, rx, h, ranphy.H_FULL, nvar)
    singular = np.zeros(kappa.shape, bool)
    singular[1, 8:16] = True
    assert np.all(np.isnan(xr[1][:, 8:16])) and np.all(np.isinf(nvr[1][:, 8:16]))
    assert np.all(np.isnan(xg[1][:, 8:16])) and np.all(np.isinf(nvg[1][:, 8:16]))
    ill = (kappa > 1e6) & ~singular
    assert ill.sum() == 24  # slot 0 sc 8..23, slot 1 sc 16..23
    with np.errstate(invalid="ignore"):  # the singular REs (inf - inf), excluded below
        err_x = np.linalg.norm(xg - xr, axis=-1) / np.linalg.norm(xr, axis=-1)  # [slot][d][sc]
        err_v = np.max(np.abs(nvg - nvr) / np.maximum(np.abs(nvr), 1e-30), axis=-1)
    sel = np.broadcast_to(ill[:, None, :], err_x.shape)
    say(f"  kappa > 1e6: {int(sel.sum())} REs, max rel err x {err_x[sel].max():.2e} "
        f"nv {err_v[sel].max():.2e}")
    assert err_x[sel].max() <= 1e-4 and err_v[sel].max() <= 1e-4
    if prec == ranphy.PREC_FP32:
        well = np.broadcast_to((kappa < 1e4)[:, None, :], err_x.shape)
        assert err_x[well].max() <= 1e-4, err_x[well].max()


FUSED = ["m", "prb5_l9_r32", "prb3_l12_r48", "prb2_l5_r16", "prb4_l8_short",
         "prb1_l16_dmrs_end"]


@pytest.mark.parametrize("name", FUSED)
@pytest.mark.parametrize("h_res", [ranphy.H_PILOT, ranphy.H_FULL])
def test_fused_detect_demap(name, h_res):
    # Detection with the demapping in its epilogue: x and nv identical to the detector's,
    # LLRs within the per-call bar of llr_demap on those x and nv and of the oracle's
    # demapping of them, and the LLR-only mode identical to the mode that also writes x, nv.
    shape = SHAPES[name]
    say(f"mmse_llr {name} h_res={h_res}")
    rx, pil, nvar, *_ = make_inputs(shape, 4, snr_db=18.0)
    h = oracle.chest_ls(shape, rx, pil, h_res).astype(np.complex64)
    rxd, hd, nd = dev(rx), dev(h), dev(nvar)
    x1, v1 = ranphy.mmse_detect(shape, rxd, hd, nd, h_res=h_res)
    x2 = torch.empty_like(x1)
    v2 = torch.empty_like(v1)
    l2 = ranphy.mmse_llr(shape, rxd, hd, nd, h_res=h_res, x=x2, nv=v2)
    l3 = ranphy.mmse_llr(shape, rxd, hd, nd, h_res=h_res)
    ls = ranphy.llr_demap(shape, x1, v1)
    torch.cuda.synchronize()
    assert x1.cpu().numpy().tobytes() == x2.cpu().numpy().tobytes()
    assert v1.cpu().numpy().tobytes() == v2.cpu().numpy().tobytes()
    assert l2.cpu().numpy().tobytes() == l3.cpu().numpy().tobytes()
    lq = out_shape(shape) + (shape.qm,)
    lg, lsep = host(l2, lq), host(ls, lq)
    assert llr_tol_ok(lg, lsep).all()
    lr = oracle.llr_demap(shape, host(x2, out_shape(shape)), host(v2, out_shape(shape)))
    assert llr_tol_ok(lg, lr).all()
    # Against the FP64 chain on the same channel estimate.
    xr, nvr = oracle.mmse_detect(shape, rx, h, h_res, nvar)
    lr64 = oracle.llr_demap(shape, xr.astype(np.complex64), nvr.astype(np.float32))
    ok = check_end_to_end(shape, host(x2, out_shape(shape)), lg, xr, lr64)
    assert (~ok).mean() < 1e-3


@pytest.mark.parametrize("name", FUSED)
@pytest.mark.parametrize("h_res", [ranphy.H_PILOT, ranphy.H_FULL])
@pytest.mark.parametrize("prec", [ranphy.PREC_FP16, ranphy.PREC_BF16])
def test_fused_detect_demap_reduced_precision(name, h_res, prec):
    # The 16-bit modes stage the LLRs through LDS before storing them (16-byte pieces, or
    # 8-byte ones where Nl Qm is not a multiple of 4: prb2_l5_r16); 16 layers of 256QAM over
    # 12 data symbols fill a wave's staging area exactly (prb1_l16_dmrs_end).
    shape = SHAPES[name]
    say(f"mmse_llr {name} h_res={h_res} prec={prec}")
    rx, pil, nvar, *_ = make_inputs(shape, 6, snr_db=20.0)
    h = oracle.chest_ls(shape, rx, pil, h_res).astype(np.complex64)
    rxd, hd, nd = dev(rx), dev(h), dev(nvar)
    x1, v1 = ranphy.mmse_detect(shape, rxd, hd, nd, h_res=h_res, precision=prec)
    x2, v2 = torch.empty_like(x1), torch.empty_like(v1)
    lf = ranphy.mmse_llr(shape, rxd, hd, nd, h_res=h_res, x=x2, nv=v2, precision=prec)
    lo = ranphy.mmse_llr(shape, rxd, hd, nd, h_res=h_res, precision=prec)
    ls = ranphy.llr_demap(shape, x1, v1)
    torch.cuda.synchronize()
    assert x1.cpu().numpy().tobytes() == x2.cpu().numpy().tobytes()
    assert v1.cpu().numpy().tobytes() == v2.cpu().numpy().tobytes()
    assert lf.cpu().numpy().tobytes() == lo.cpu().numpy().tobytes()
    lq = out_shape(shape) + (shape.qm,)
    assert llr_tol_ok(host(lf, lq), host(ls, lq)).all()


def test_fused_detect_demap_empty_batch():
    shape = M.with_slots(0)
    e = torch.empty(0, dtype=torch.complex64, device="cuda")
    ef = torch.empty(0, dtype=torch.float32, device="cuda")
    ranphy.mmse_llr(shape, e, e, ef, llr=ef)
    torch.cuda.synchronize()


SMALL_BATCHED = {
    # >= 65536 subcarriers per call: the one-thread-per-subcarrier detector
    "p2": synth.CONFIGS["p2"]["shape"].with_slots(92),
    "p4": synth.CONFIGS["p4"]["shape"].with_slots(92),
    "p8": synth.CONFIGS["p8"]["shape"].with_slots(92),
    "r8_l3_c8": SlotShape(60, 14, 8, 3, 4, 8, 1, (3,), 92),
    "r4_l1_short": SlotShape(60, 7, 4, 1, 2, 2, 1, (0,), 184),
}


@pytest.mark.parametrize("name", list(SMALL_BATCHED))
@pytest.mark.parametrize("h_res", [ranphy.H_PILOT, ranphy.H_FULL])
def test_mmse_small_mimo_batched(name, h_res):
    shape = SMALL_BATCHED[name]
    say(f"mmse_detect batched {name} h_res={h_res}: {shape.n_slots * shape.n_sc} subcarriers")
    assert shape.n_slots * shape.n_sc >= 65536
    rx, pil, nvar, *_ = make_inputs(shape, 3, snr_db=12.0)
    nvar = nvar * np.linspace(0.5, 2.0, shape.n_slots).astype(np.float32)
    h = oracle.chest_ls(shape, rx, pil, h_res).astype(np.complex64)
    xg, nvg = gpu_mmse(shape, rx, h, h_res, nvar)
    xr, nvr = oracle.mmse_detect(shape, rx, h, h_res, nvar)
    check_mmse(shape, h, h_res, nvar, xg, nvg, xr, nvr)


@pytest.mark.parametrize("name", ["p2", "p4", "p8"])
def test_end_to_end_paper_shapes(name):
    # Square 2x2 / 4x4 / 8x8 at 60 RB, 15 kHz, QPSK: GPU chain vs FP64 oracle chain.
    b = synth.make_batch(name, n_slots=7, snr_db=synth.CONFIGS[name]["snr_db"])
    shape = b["shape"]
    say(f"end to end {name}: {shape.n_rx}x{shape.n_layers}")
    xg, lg, xr, nvr, lr = end_to_end(shape, b["rx"], b["pilots"], b["noise_var"])
    ok = check_end_to_end(shape, xg, lg, xr, lr)
    assert (~ok).mean() < 1e-3


def test_graph_replay_matches_eager():
    # One slot's chest_ls -> mmse_llr captured in a HIP graph: every replay, with eager work
    # and synchronisations in between, equals the eager result bit for bit.
    shape = SHAPES["prb5_l9_r32"].with_slots(1)
    rx, pil, nvar, *_ = make_inputs(shape, 12)
    rxd, pd, nd = dev(rx), dev(pil), dev(nvar)
    h = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_H) // 2, dtype=torch.complex64,
                    device="cuda")
    llr = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_LLR), dtype=torch.float32,
                      device="cuda")

    def chain():
        ranphy.chest_ls(shape, rxd, pd, h=h)
        ranphy.mmse_llr(shape, rxd, h, nd, llr=llr)

    chain()
    torch.cuda.synchronize()
    ref = llr.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        chain()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        chain()
    for i in range(4):
        llr.fill_(float(i))       # eager work between replays
        h.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(llr.view(torch.int32), ref.view(torch.int32)), i


def test_llr_demap_8_byte_aligned_buffers():
    # Buffers 8- but not 16-byte aligned take the one-element-per-thread kernel.
    qm = 6
    shape = SlotShape(3, 14, 4, 3, qm, 4, 1, (2,), 1)
    rng = np.random.default_rng(11)
    n = out_shape(shape)
    x = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 0.8).astype(np.complex64)
    nv = rng.uniform(1e-3, 2.0, n).astype(np.float32)
    xb = torch.zeros(x.size + 1, dtype=torch.complex64, device="cuda")
    vb = torch.zeros(nv.size + 2, dtype=torch.float32, device="cuda")
    lb = torch.zeros(nv.size * qm + 2, dtype=torch.float32, device="cuda")
    xb[1:] = dev(x)
    vb[2:] = dev(nv)
    xv, vv, lv = xb[1:], vb[2:], lb[2:]
    assert xv.data_ptr() % 16 == 8 and vv.data_ptr() % 16 == 8 and lv.data_ptr() % 16 == 8
    ranphy.llr_demap(shape, xv, vv, llr=lv)
    lg = host(lv, n + (qm,))
    lr = oracle.llr_demap(shape, x, nv)
    assert llr_tol_ok(lg, lr).all()
