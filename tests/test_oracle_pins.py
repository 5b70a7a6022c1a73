"""Pins of the FP64 oracle against facts fixed by the mathematics (no GPU).

Each test ties one part of the oracle to something other than itself: closed forms,
identities, special cases that reduce to a textbook result, brute force on tiny inputs,
or hand-computed fixtures under tests/golden/.  A dropped term, a wrong sign, a wrong
index or a transposed operand anywhere in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from synth import SlotShape

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def all_bits(qm):
    i = np.arange(1 << qm)
    return ((i[:, None] >> np.arange(qm)[::-1]) & 1).astype(np.uint8)


# ---------------------------------------------------------------------------------------
# Constellation (reading of the QAM mapping, 3GPP NR structure).
# ---------------------------------------------------------------------------------------

def test_qam16_golden_table():
    rows = np.loadtxt(os.path.join(GOLDEN, "qam16_points.txt"))
    pts = oracle.qam_points(4) * math.sqrt(10.0)
    for r in rows:
        b = r[:4].astype(int)
        idx = int("".join(map(str, b)), 2)
        assert pts[idx] == pytest.approx(r[4] + 1j * r[5], abs=1e-12)


@pytest.mark.parametrize("qm", [2, 4, 6, 8])
def test_constellation_independent_mappers_agree(qm):
    # Oracle (C) and generator (Python) implement the mapping separately.
    bits = all_bits(qm)
    np.testing.assert_allclose(oracle.qam_points(qm), synth.qam_map(bits, qm), atol=1e-14)


@pytest.mark.parametrize("qm", [2, 4, 6, 8])
def test_constellation_gray_unit_energy(qm):
    pts = oracle.qam_points(qm)
    assert np.mean(np.abs(pts) ** 2) == pytest.approx(1.0, abs=1e-12)
    assert len(np.unique(np.round(pts, 9))) == 1 << qm
    # Gray: nearest neighbours (horizontal or vertical) differ in exactly one bit.
    dmin = 2.0 / synth.qam_scale(qm)
    for i in range(1 << qm):
        for j in range(1 << qm):
            if abs(abs(pts[i] - pts[j]) - dmin) < 1e-9:
                assert bin(i ^ j).count("1") == 1
    # Square grid: per-axis levels are odd integers in unnormalised units.
    lv = np.unique(np.round(pts.real * synth.qam_scale(qm), 9))
    assert np.allclose(lv, np.arange(-(2 ** (qm // 2)) + 1, 2 ** (qm // 2), 2))


# ---------------------------------------------------------------------------------------
# P8: demapper closed forms and noiseless round trip.
# ---------------------------------------------------------------------------------------

def test_llr_qpsk_closed_form():
    rng = np.random.default_rng(1)
    x = crandn(rng, 2000) * 2
    nv = rng.uniform(0.01, 2.0, 2000)
    llr = oracle.llr_batch(x, nv, 2)
    np.testing.assert_allclose(llr[:, 0], 2 * math.sqrt(2) * x.real / nv, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(llr[:, 1], 2 * math.sqrt(2) * x.imag / nv, rtol=1e-12, atol=1e-12)


def test_llr_16qam_closed_form():
    rng = np.random.default_rng(2)
    x = crandn(rng, 4000) * 1.5
    nv = rng.uniform(0.01, 2.0, 4000)
    llr = oracle.llr_batch(x, nv, 4)
    for axis, (b_sign, b_mag) in ((x.real, (0, 2)), (x.imag, (1, 3))):
        u = math.sqrt(10.0) * axis
        d_sign = np.where(np.abs(u) <= 2, 4 * u, 8 * (u - np.sign(u)))
        d_mag = 4 * (2 - np.abs(u))
        np.testing.assert_allclose(llr[:, b_sign], d_sign / (10 * nv), rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(llr[:, b_mag], d_mag / (10 * nv), rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("qm", [2, 4, 6, 8])
def test_llr_bruteforce_equals_per_axis(qm):
    # For square Gray QAM the 2-D minimum splits per axis; evaluate it per axis here.
    rng = np.random.default_rng(3 + qm)
    x = crandn(rng, 1500) * 1.3
    nv = rng.uniform(0.05, 1.0, 1500)
    llr = oracle.llr_batch(x, nv, qm)
    m = qm // 2
    lv_bits = all_bits(m)
    levels = synth.pam_amplitude(lv_bits) / synth.qam_scale(qm) if m > 1 else \
        (1 - 2.0 * lv_bits[:, 0]) / synth.qam_scale(qm)
    for b in range(qm):
        axis = x.real if b % 2 == 0 else x.imag
        sel = lv_bits[:, b // 2]
        d = (axis[:, None] - levels[None, :]) ** 2
        d1 = d[:, sel == 1].min(axis=1)
        d0 = d[:, sel == 0].min(axis=1)
        np.testing.assert_allclose(llr[:, b], (d1 - d0) / nv, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("qm", [2, 4, 6, 8])
def test_llr_noiseless_round_trip(qm):
    bits = all_bits(qm)
    x = synth.qam_map(bits, qm)
    llr = oracle.llr_batch(x, 0.1, qm)
    assert np.array_equal((llr < 0).astype(np.uint8), bits)


# ---------------------------------------------------------------------------------------
# P1: least squares at the pilots.
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", ["c1", "c2", "m"])
def test_ls_noiseless_recovers_true_channel(cfg):
    c = synth.CONFIGS[cfg]
    shape = c["shape"].with_slots(1)
    if cfg == "m":
        shape = SlotShape(n_prb=5, n_symb=14, n_rx=8, n_layers=16, qm=6, dmrs_comb=8, dmrs_td=2,
                          dmrs_sym0=(2,), n_slots=1)
    rng = synth.rng_for(99, 0, 0)
    d = synth.make_slot(shape, rng, c["scs_hz"], c["pdp"], 20.0, noiseless=True)
    h = oracle.chest_ls(shape, d["rx"][None], d["pilots"][None])
    for p in range(shape.n_layers):
        cidx = p % shape.dmrs_comb
        for j in range(shape.port_pilot_count(p)):
            k = cidx + shape.dmrs_comb * j
            # Same pilot slot at every occasion under block fading.
            for o in range(shape.n_occ):
                np.testing.assert_allclose(h[0, o, j, :, p], d["h"][k, :, p], rtol=0, atol=2e-6)
        # Unused tail entries are zero.
        for j in range(shape.port_pilot_count(p), shape.n_pilot):
            assert np.all(h[0, :, j, :, p] == 0)


def test_ls_time_cover_separates_ports_sharing_a_comb():
    # Ports p and p + C share comb offset; only the cover code [1,1] vs [1,-1] separates them.
    shape = SlotShape(n_prb=2, n_symb=14, n_rx=3, n_layers=4, qm=2, dmrs_comb=2, dmrs_td=2,
                      dmrs_sym0=(2,), n_slots=1)
    rng = np.random.default_rng(7)
    H = crandn(rng, shape.n_sc, shape.n_rx, shape.n_layers)
    d = synth.make_slot(shape, rng, 15e3, "taps8", 30.0, channel=H, noiseless=True)
    h = oracle.chest_ls(shape, d["rx"][None], d["pilots"][None])
    for p in range(4):
        ks = np.arange(p % 2, shape.n_sc, 2)
        np.testing.assert_allclose(h[0, 0, : len(ks), :, p], H[ks, :, p], atol=2e-6)
    # Dropping the cover code would leave the sum of the two ports: check it is not that.
    ks = np.arange(0, shape.n_sc, 2)
    assert np.max(np.abs(h[0, 0, : len(ks), :, 0] - (H[ks, :, 0] + H[ks, :, 2]))) > 0.1


# ---------------------------------------------------------------------------------------
# P2: interpolation.
# ---------------------------------------------------------------------------------------

def _grid_from_samples(shape, samples):
    """rx grid with the given DMRS-symbol samples; pilots all 1."""
    rx = np.zeros((1, shape.n_symb, shape.n_sc, shape.n_rx), np.complex64)
    pil = np.ones((1, shape.n_occ, shape.dmrs_td, shape.n_pilot, shape.n_layers), np.complex64)
    for (s, k, r), v in samples.items():
        rx[0, s, k, r] = v
    return rx, pil


def test_interp_golden_one_prb_comb2():
    shape = SlotShape(n_prb=1, n_symb=14, n_rx=1, n_layers=2, qm=2, dmrs_comb=2, dmrs_td=1,
                      dmrs_sym0=(2,), n_slots=1)
    lines = open(os.path.join(GOLDEN, "interp_1prb_comb2.txt")).read().split("\n")
    lines = [l for l in lines if l and not l.startswith("#")]
    sec, pil, full = None, {}, {}
    for l in lines:
        if l in ("pilots", "full"):
            sec = l
            continue
        p, k, re, im = l.split()
        (pil if sec == "pilots" else full)[(int(p), int(k))] = float(re) + 1j * float(im)
    rx, pilots = _grid_from_samples(shape, {(2, k, 0): v for (p, k), v in pil.items()})
    h = oracle.chest_ls(shape, rx, pilots, oracle.H_FULL)
    for (p, k), v in full.items():
        assert h[0, 0, k, 0, p] == pytest.approx(v, abs=1e-12), (p, k)
    # The detector's channel at a data symbol (one occasion: held in time) is the same.
    hp = oracle.chest_ls(shape, rx, pilots, oracle.H_PILOT)
    for k in range(12):
        H = oracle.channel_at(shape, hp.astype(np.complex64), oracle.H_PILOT, 0, k, 7)
        for p in range(2):
            assert H[0, p] == pytest.approx(full[(p, k)], abs=1e-12)


def test_interp_exact_for_linear_and_flat_channels():
    shape = SlotShape(n_prb=3, n_symb=14, n_rx=2, n_layers=4, qm=2, dmrs_comb=4, dmrs_td=1,
                      dmrs_sym0=(2,), n_slots=1)
    rng = np.random.default_rng(11)
    a = crandn(rng, shape.n_rx, shape.n_layers)
    b = crandn(rng, shape.n_rx, shape.n_layers) * 0.05
    k = np.arange(shape.n_sc)
    for H in (a[None] + b[None] * k[:, None, None], np.broadcast_to(a, (shape.n_sc,) + a.shape)):
        d = synth.make_slot(shape, rng, 30e3, "taps8", 30.0, channel=np.array(H), noiseless=True)
        h = oracle.chest_ls(shape, d["rx"][None], d["pilots"][None], oracle.H_FULL)
        for p in range(shape.n_layers):
            c = p % shape.dmrs_comb
            last = c + shape.dmrs_comb * (shape.port_pilot_count(p) - 1)
            for kk in range(shape.n_sc):
                kref = min(max(kk, c), last)  # held outside the pilot span
                np.testing.assert_allclose(h[0, 0, kk, :, p], H[kref, :, p], atol=2e-6)


def test_time_interp_exact_for_channel_linear_in_time():
    shape = SlotShape(n_prb=1, n_symb=14, n_rx=2, n_layers=2, qm=2, dmrs_comb=2, dmrs_td=1,
                      dmrs_sym0=(2, 11), n_slots=1)
    rng = np.random.default_rng(12)
    a = crandn(rng, shape.n_rx, shape.n_layers)
    b = crandn(rng, shape.n_rx, shape.n_layers) * 0.1
    # Time-varying flat channel, a + b s; build the DMRS symbols with pilots = 1.
    samples = {}
    for s in (2, 11):
        for k in range(shape.n_sc):
            p = k % 2
            for r in range(shape.n_rx):
                samples[(s, k, r)] = a[r, p] + b[r, p] * s
    rx, pil = _grid_from_samples(shape, samples)
    h = oracle.chest_ls(shape, rx, pil).astype(np.complex64)
    for s in shape.data_symbols():
        sref = min(max(s, 2), 11)
        H = oracle.channel_at(shape, h, oracle.H_PILOT, 0, 5, s)
        np.testing.assert_allclose(H, a + b * sref, atol=2e-6)


def test_time_interp_double_symbol_occasion_centres():
    # Occasions {2,3} and {10,11}: centres 2.5 and 10.5.
    shape = SlotShape(n_prb=1, n_symb=14, n_rx=1, n_layers=1, qm=2, dmrs_comb=2, dmrs_td=2,
                      dmrs_sym0=(2, 10), n_slots=1)
    h = np.zeros((1, 2, shape.n_pilot, 1, 1), np.complex64)
    h[0, 0] = 1.0
    h[0, 1] = 9.0
    for s, want in ((0, 1.0), (1, 1.0), (4, 1.0 + 8 * 1.5 / 8), (6, 1.0 + 8 * 3.5 / 8),
                    (9, 1.0 + 8 * 6.5 / 8), (12, 9.0), (13, 9.0)):
        H = oracle.channel_at(shape, h, oracle.H_PILOT, 0, 3, s)
        assert H[0, 0] == pytest.approx(want, abs=1e-12), s


# ---------------------------------------------------------------------------------------
# P3: the MMSE solve.
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("nr,nl", [(4, 2), (16, 4), (64, 16), (3, 3), (8, 5)])
def test_lu_route_equals_covariance_route(nr, nl):
    rng = np.random.default_rng(nr * 100 + nl)
    n = 200
    H = crandn(rng, n, nr, nl)
    y = crandn(rng, n, nr) * 2
    s2 = rng.uniform(0.01, 1.0, n)
    a = oracle.mmse_batch(H, y, s2, oracle.ROUTE_LU)
    b = oracle.mmse_batch(H, y, s2, oracle.ROUTE_RCOV)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-10, atol=1e-12)


def test_gram_hermitian_pd_and_solution_residual():
    rng = np.random.default_rng(21)
    for nr, nl in ((4, 2), (16, 4), (64, 16)):
        H = crandn(rng, nr, nl)
        s2 = 0.05
        G = oracle.gram(H, s2)
        assert np.array_equal(G, G.conj().T)
        np.testing.assert_allclose(G, H.conj().T @ H + s2 * np.eye(nl), rtol=1e-13, atol=1e-13)
        lam = np.linalg.eigvalsh(G)
        assert lam.min() >= s2 * (1 - 1e-12)
        y = crandn(rng, nr)
        xt, nv, mu = oracle.mmse_batch(H[None], y[None], s2)
        xhat = mu[0] * xt[0]
        z = H.conj().T @ y
        res = np.linalg.norm(G @ xhat - z)
        assert res <= 100 * np.finfo(float).eps * np.linalg.norm(G, 2) * np.linalg.norm(xhat)
        # mu = diag(W H), W = G^-1 H^H;  nu2 = (1 - mu) / mu.
        W = np.linalg.solve(G, H.conj().T)
        np.testing.assert_allclose(mu[0], np.real(np.diag(W @ H)), rtol=1e-11)
        np.testing.assert_allclose(nv[0], (1 - mu[0]) / mu[0], rtol=1e-9)


def test_post_equalisation_variance_is_interference_plus_noise():
    # nu2 must equal E|x~ - x|^2 for unit-energy i.i.d. symbols (sum of residual
    # interference and noise after unbiasing), computed here from W directly.
    rng = np.random.default_rng(22)
    nr, nl, s2 = 8, 4, 0.2
    H = crandn(rng, nr, nl)
    G = H.conj().T @ H + s2 * np.eye(nl)
    W = np.linalg.solve(G, H.conj().T)
    A = W @ H
    mu = np.real(np.diag(A))
    var = (np.sum(np.abs(A) ** 2, axis=1) - mu ** 2 + s2 * np.sum(np.abs(W) ** 2, axis=1)) / mu ** 2
    _, nv, _ = oracle.mmse_batch(H[None], np.zeros((1, nr)), s2)
    np.testing.assert_allclose(nv[0], var, rtol=1e-10)


# ---------------------------------------------------------------------------------------
# P4 / P5: zero forcing and the MMSE -> ZF limit.
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("nr,nl,qm", [(4, 2, 2), (16, 4, 8), (64, 16, 6)])
def test_zf_noiseless_genie_recovers_symbols(nr, nl, qm):
    rng = np.random.default_rng(31 + nr)
    n = 300
    H = crandn(rng, n, nr, nl)
    bits = rng.integers(0, 2, size=(n, nl, qm), dtype=np.uint8)
    x = synth.qam_map(bits, qm)
    y = np.einsum("nrl,nl->nr", H, x)
    xt, nv, mu = oracle.mmse_batch(H, y, 0.0)
    np.testing.assert_allclose(xt, x, rtol=0, atol=1e-12)
    assert np.all(nv == 0) and np.all(mu == 1)
    llr = oracle.llr_batch(xt, nv.reshape(-1), qm).reshape(n, nl, qm)
    assert np.array_equal((llr < 0).astype(np.uint8), bits)


def test_zf_noiseless_slot_level_genie_full_h():
    # Slot-level path (interpolation + solve) with the true channel at full resolution.
    c = synth.CONFIGS["c1"]
    shape = c["shape"]
    rng = synth.rng_for(98, 0, 0)
    d = synth.make_slot(shape, rng, c["scs_hz"], c["pdp"], 20.0, noiseless=True)
    hfull = np.ascontiguousarray(d["h"][None, None].astype(np.complex64))
    x, nv = oracle.mmse_detect(shape, d["rx"][None], hfull, oracle.H_FULL, np.zeros(1, np.float32))
    np.testing.assert_allclose(x[0], d["x"], atol=2e-5)
    assert np.all(nv == 0)


def test_mmse_tends_to_zf_linearly_in_noise_variance():
    rng = np.random.default_rng(41)
    nr, nl = 8, 4
    H = crandn(rng, 1, nr, nl)
    y = crandn(rng, 1, nr)
    xt0, _, mu0 = oracle.mmse_batch(H, y, 0.0)
    zf = xt0[0] * mu0[0]
    s2s = np.logspace(-8, -2, 7)
    errs = []
    for s2 in s2s:
        xt, _, mu = oracle.mmse_batch(H, y, s2)
        errs.append(np.linalg.norm(xt[0] * mu[0] - zf))
    slope = np.polyfit(np.log10(s2s), np.log10(errs), 1)[0]
    assert slope == pytest.approx(1.0, abs=0.02)


# ---------------------------------------------------------------------------------------
# P6 / P7: single layer and orthogonal columns reduce to ML exactly.
# ---------------------------------------------------------------------------------------

def _ml_maxlog(H, y, s2, qm):
    """Joint ML max-log LLRs by enumerating every transmit vector (tiny cases only)."""
    nl = H.shape[1]
    pts_bits = all_bits(qm)
    pts = synth.qam_map(pts_bits, qm)
    M = len(pts)
    idx = np.array(np.meshgrid(*[np.arange(M)] * nl, indexing="ij")).reshape(nl, -1).T
    S = pts[idx]  # [hyp][nl]
    metric = np.sum(np.abs(y[None, :] - S @ H.T) ** 2, axis=1) / s2
    out = np.zeros((nl, qm))
    for l in range(nl):
        for b in range(qm):
            bit = pts_bits[idx[:, l], b]
            out[l, b] = metric[bit == 1].min() - metric[bit == 0].min()
    return out


@pytest.mark.parametrize("qm", [2, 4, 6])
def test_single_layer_mmse_llr_equals_ml(qm):
    rng = np.random.default_rng(51 + qm)
    for _ in range(50):
        nr = int(rng.integers(1, 6))
        H = crandn(rng, nr, 1)
        s2 = float(rng.uniform(0.05, 1.0))
        y = H[:, 0] * synth.qam_map(rng.integers(0, 2, (qm,)), qm) + crandn(rng, nr) * math.sqrt(s2)
        xt, nv, _ = oracle.mmse_batch(H[None], y[None], s2)
        llr = oracle.llr_batch(xt[0], nv[0], qm)
        np.testing.assert_allclose(llr[0], _ml_maxlog(H, y, s2, qm)[0], rtol=1e-9, atol=1e-9)


def test_orthogonal_columns_mmse_llr_equals_joint_ml_2x2_qpsk():
    rng = np.random.default_rng(61)
    for _ in range(50):
        Q, _ = np.linalg.qr(crandn(rng, 2, 2))
        H = Q @ np.diag(rng.uniform(0.3, 2.0, 2))
        s2 = float(rng.uniform(0.05, 1.0))
        x = synth.qam_map(rng.integers(0, 2, (2, 2)), 2)
        y = H @ x + crandn(rng, 2) * math.sqrt(s2)
        xt, nv, _ = oracle.mmse_batch(H[None], y[None], s2)
        llr = oracle.llr_batch(xt[0], nv[0], 2).reshape(2, 2)
        np.testing.assert_allclose(llr, _ml_maxlog(H, y, s2, 2), rtol=1e-9, atol=1e-9)


def test_ml_no_worse_than_mmse_2x2_qpsk():
    # Joint ML hard decisions are the best possible; MMSE may not beat them beyond noise.
    rng = np.random.default_rng(62)
    n, s2 = 4000, 10 ** (-10 / 10)
    H = crandn(rng, n, 2, 2)
    bits = rng.integers(0, 2, (n, 2, 2), dtype=np.uint8)
    x = synth.qam_map(bits, 2)
    y = np.einsum("nrl,nl->nr", H, x) + crandn(rng, n, 2) * math.sqrt(s2)
    xt, nv, _ = oracle.mmse_batch(H, y, s2)
    mm = (oracle.llr_batch(xt, nv.reshape(-1), 2).reshape(n, 2, 2) < 0)
    ml = np.stack([_ml_maxlog(H[i], y[i], s2, 2) < 0 for i in range(n)])
    e_mm, e_ml = np.sum(mm != bits), np.sum(ml != bits)
    assert e_ml <= e_mm + 3 * math.sqrt(e_mm + 1)
    assert np.mean(mm == ml) > 0.9


# ---------------------------------------------------------------------------------------
# P9: whole detector statistics against the closed-form ZF BER.
# ---------------------------------------------------------------------------------------

def zf_ber_formula(nr, nl, snr_db):
    L = nr - nl + 1
    g = 1.0 / (2 * 10 ** (-snr_db / 10))
    mu = math.sqrt(g / (1 + g))
    return ((1 - mu) / 2) ** L * sum(math.comb(L - 1 + k, k) * ((1 + mu) / 2) ** k for k in range(L))


def test_zf_ber_golden_values_match_formula():
    for nr, nl, snr, ber in np.loadtxt(os.path.join(GOLDEN, "zf_ber_closed_form.txt")):
        assert zf_ber_formula(int(nr), int(nl), snr) == pytest.approx(ber, rel=5e-3)


@pytest.mark.parametrize("nr,nl,snr_db", [(4, 2, 0.0), (4, 2, 10.0), (2, 2, 0.0), (2, 2, 10.0),
                                          (2, 2, 20.0)])
def test_zf_ber_matches_closed_form(nr, nl, snr_db):
    rng = np.random.default_rng(int(1000 + nr * 10 + nl + snr_db))
    n_bits = 2_000_000
    n = n_bits // (nl * 2)
    s2 = 10 ** (-snr_db / 10)
    H = crandn(rng, n, nr, nl)
    bits = rng.integers(0, 2, (n, nl, 2), dtype=np.uint8)
    y = np.einsum("nrl,nl->nr", H, synth.qam_map(bits, 2)) + crandn(rng, n, nr) * math.sqrt(s2)
    xt, nv, _ = oracle.mmse_batch(H, y, 0.0)  # genie channel, zero forcing
    llr = oracle.llr_batch(xt, nv.reshape(-1), 2).reshape(n, nl, 2)
    errs = int(np.sum((llr < 0) != bits))
    p = zf_ber_formula(nr, nl, snr_db)
    lo, hi = stats.binom.ppf([0.005, 0.995], n * nl * 2, p)
    assert lo <= errs <= hi, (errs / (n * nl * 2), p)


# ---------------------------------------------------------------------------------------
# Slot-level detector = per-element detector on the interpolated channel.
# ---------------------------------------------------------------------------------------

def test_slot_level_detector_consistent_with_per_element():
    b = synth.make_batch("c2", n_slots=1)
    shape = b["shape"]
    h = oracle.chest_ls(shape, b["rx"], b["pilots"]).astype(np.complex64)
    x, nv = oracle.mmse_detect(shape, b["rx"], h, oracle.H_PILOT, b["noise_var"])
    ds = shape.data_symbols()
    rng = np.random.default_rng(5)
    for _ in range(20):
        di, k = int(rng.integers(len(ds))), int(rng.integers(shape.n_sc))
        H = oracle.channel_at(shape, h, oracle.H_PILOT, 0, k, ds[di])
        y = b["rx"][0, ds[di], k].astype(np.complex128)
        xt, nv1, _ = oracle.mmse_batch(H[None], y[None], float(b["noise_var"][0]))
        np.testing.assert_allclose(x[0, di, k], xt[0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(nv[0, di, k], nv1[0], rtol=1e-12)


def test_singular_system_gives_nan_and_inf():
    rng = np.random.default_rng(71)
    h = crandn(rng, 4, 1)
    H = np.concatenate([h, h], axis=1)  # identical columns, zero noise variance
    xt, nv, mu = oracle.mmse_batch(H[None], crandn(rng, 1, 4), 0.0)
    assert np.all(np.isnan(xt)) and np.all(np.isinf(nv))
