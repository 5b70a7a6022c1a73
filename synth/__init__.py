"""Seeded synthetic uplink slots: the inputs that both the GPU path and the oracle read.

This module holds no step of the receiver's arithmetic (no channel estimation, no
interpolation, no detection, no demapping).  It only draws what a transmitter and a
channel would produce:

* uniform bits mapped to Gray square QAM (the 3GPP NR structure: bits b0, b2, ... on
  the in-phase axis, b1, b3, ... on the quadrature axis, amplitude built by nested
  sign flips, unit average energy);
* DMRS pilots: comb-C frequency multiplexing with an optional length-2 time-domain
  orthogonal cover code; ports that share a comb offset share a unit-modulus QPSK
  base sequence;
* a tapped-delay-line Rayleigh channel with an exponential power delay profile,
  block fading over a slot, i.i.d. across receive antennas and layers;
* circularly symmetric complex Gaussian noise of variance ``10**(-snr_db/10)`` on every
  resource element (unit-energy symbols per layer, unit-power channel entries).

The paper (Sec. IV) evaluates its detector inside a 3GPP NR link simulator with a
TDL-C channel; the TDL-C tap table is not available here, so an exponential power
delay profile of the stated rms delay spread stands in for it.

Streams are seeded from ``SeedSequence([0x5EED, config_id, snr_index, slot])`` so that
no two (configuration, SNR point, slot) triples share random numbers.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

SEED_ROOT = 0x5EED


@dataclasses.dataclass(frozen=True)
class SlotShape:
    """Shape of one batch of uplink slots (mirrors the C descriptor field by field)."""

    n_prb: int
    n_symb: int
    n_rx: int
    n_layers: int
    qm: int
    dmrs_comb: int
    dmrs_td: int
    dmrs_sym0: tuple
    n_slots: int = 1

    @property
    def n_occ(self) -> int:
        return len(self.dmrs_sym0)

    @property
    def n_sc(self) -> int:
        return 12 * self.n_prb

    @property
    def n_pilot(self) -> int:
        """Pilot slots reserved per port and occasion: ceil(n_sc / comb)."""
        return -(-self.n_sc // self.dmrs_comb)

    def dmrs_symbols(self) -> List[int]:
        out = []
        for s0 in self.dmrs_sym0:
            out.extend(range(s0, s0 + self.dmrs_td))
        return out

    def data_symbols(self) -> List[int]:
        d = set(self.dmrs_symbols())
        return [s for s in range(self.n_symb) if s not in d]

    @property
    def n_dsym(self) -> int:
        return len(self.data_symbols())

    @property
    def n_data_re(self) -> int:
        """Data resource elements per batch (all slots)."""
        return self.n_slots * self.n_dsym * self.n_sc

    def with_slots(self, n: int) -> "SlotShape":
        return dataclasses.replace(self, n_slots=n)

    def port_comb_offset(self, p: int) -> int:
        return p % self.dmrs_comb

    def port_pilot_count(self, p: int) -> int:
        c = self.port_comb_offset(p)
        return -(-(self.n_sc - c) // self.dmrs_comb)


# ---------------------------------------------------------------------------------------
# Workload definitions (shapes, channel and SNR grid).
# ---------------------------------------------------------------------------------------

CONFIGS: Dict[str, dict] = {
    # 4 Rx x 2 layers, 52 PRB, DMRS on symbol 2 (comb 2), QPSK, 8-tap exponential PDP,
    # block fading, 20 dB; one slot.
    "c1": dict(
        config_id=1,
        shape=SlotShape(n_prb=52, n_symb=14, n_rx=4, n_layers=2, qm=2, dmrs_comb=2,
                        dmrs_td=1, dmrs_sym0=(2,), n_slots=1),
        scs_hz=15e3, pdp="taps8", snr_db=(20.0,), slots_per_snr=1),
    # 16 Rx x 4 layers, 273 PRB at 30 kHz, 256QAM, two single-symbol DMRS occasions,
    # exponential PDP with 100 ns rms delay spread, 10..30 dB, 20 slots per point.
    "c2": dict(
        config_id=2,
        shape=SlotShape(n_prb=273, n_symb=14, n_rx=16, n_layers=4, qm=8, dmrs_comb=4,
                        dmrs_td=1, dmrs_sym0=(2, 11), n_slots=1),
        scs_hz=30e3, pdp=("exp", 100e-9), snr_db=(10.0, 15.0, 20.0, 25.0, 30.0),
        slots_per_snr=20),
    # 64 Rx x 16 layers, 273 PRB at 30 kHz, 64QAM, one double-symbol DMRS occasion with
    # comb 8 and a length-2 time cover (16 ports), 300 ns rms delay spread, 0..30 dB.
    "m": dict(
        config_id=3,
        shape=SlotShape(n_prb=273, n_symb=14, n_rx=64, n_layers=16, qm=6, dmrs_comb=8,
                        dmrs_td=2, dmrs_sym0=(2,), n_slots=1),
        scs_hz=30e3, pdp=("exp", 300e-9),
        snr_db=(0.0, 5.0, 10.0, 15.0, 20.0, 25.0, 30.0), slots_per_snr=20),
}

# The paper's own evaluation shapes (Sec. IV): square 2x2, 4x4 and 8x8 MIMO over 60 RB at
# 15 kHz, MCS 9 (QPSK), 14-symbol slots.  DMRS: comb C and time cover T with C T >= layers
# (2x2: comb 2 on symbol 2; 4x4: comb 2, double symbol; 8x8: comb 4, double symbol).  The
# paper's TDL-C table is not available; an exponential PDP with 300 ns rms delay spread
# stands in for it, as for the other workloads.
for _n, (_cid, _nl, _c, _t) in {"p2": (4, 2, 2, 1), "p4": (5, 4, 2, 2), "p8": (6, 8, 4, 2)}.items():
    CONFIGS[_n] = dict(
        config_id=_cid,
        shape=SlotShape(n_prb=60, n_symb=14, n_rx=_nl, n_layers=_nl, qm=2, dmrs_comb=_c,
                        dmrs_td=_t, dmrs_sym0=(2,), n_slots=1),
        scs_hz=15e3, pdp=("exp", 300e-9),
        snr_db=(0.0, 5.0, 10.0, 15.0, 20.0, 25.0, 30.0), slots_per_snr=100)


def rng_for(config_id: int, snr_index: int, slot: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([SEED_ROOT, int(config_id), int(snr_index), int(slot)])))


# ---------------------------------------------------------------------------------------
# Transmitter side.
# ---------------------------------------------------------------------------------------

def pam_amplitude(bits_axis: np.ndarray) -> np.ndarray:
    """Gray PAM amplitude (unnormalised) from the bits of one axis, most significant first.

    amplitude = (1-2c0) * (2^(m-1) - (1-2c1) * (2^(m-2) - (1-2c2) * (...)))
    """
    m = bits_axis.shape[-1]
    sgn = 1.0 - 2.0 * bits_axis.astype(np.float64)
    amp = np.ones(bits_axis.shape[:-1])
    # Innermost level first: start from 1 for the last bit, then wrap outwards.
    for i in range(m - 1, 0, -1):
        amp = float(2 ** (m - i)) - sgn[..., i] * amp
    return sgn[..., 0] * amp


def qam_scale(qm: int) -> float:
    """Normalisation making the average symbol energy 1: sqrt(2 (M-1) / 3)."""
    return math.sqrt(2.0 * ((1 << qm) - 1) / 3.0)


def qam_map(bits: np.ndarray, qm: int) -> np.ndarray:
    """Map bits (..., qm) of {0,1} to unit-energy Gray square QAM symbols (complex128)."""
    if qm == 2:
        re = 1.0 - 2.0 * bits[..., 0]
        im = 1.0 - 2.0 * bits[..., 1]
    else:
        re = pam_amplitude(bits[..., 0::2])
        im = pam_amplitude(bits[..., 1::2])
    return (re + 1j * im) / qam_scale(qm)


def make_pilots(rng: np.random.Generator, shape: SlotShape) -> np.ndarray:
    """Pilots [occ][t][j][layer] (complex64), time cover code included.

    Base sequence: unit-modulus QPSK per (comb offset, occasion, t, j); port p takes
    comb offset p mod C and cover code p div C, with codes [+1,+1] and [+1,-1].
    """
    C, T = shape.dmrs_comb, shape.dmrs_td
    J = shape.n_pilot
    q = rng.integers(0, 2, size=(C, shape.n_occ, T, J, 2))
    base = ((1 - 2 * q[..., 0]) + 1j * (1 - 2 * q[..., 1])) / math.sqrt(2.0)
    occ_code = np.array([[1.0, 1.0], [1.0, -1.0]])
    out = np.zeros((shape.n_occ, T, J, shape.n_layers), dtype=np.complex128)
    for p in range(shape.n_layers):
        c, w = p % C, p // C
        for t in range(T):
            out[:, t, :, p] = base[c, :, t, :] * occ_code[w, t]
    return out.astype(np.complex64)


# ---------------------------------------------------------------------------------------
# Channel.
# ---------------------------------------------------------------------------------------

def power_delay_profile(pdp, scs_hz: float):
    """Return (delays in s, powers summing to 1) for a named profile.

    * "taps8": 8 taps spaced 1/(1024 * scs), power ~ exp(-n/2).
    * ("exp", tau_rms): taps spaced 1/(1024 * scs), power ~ exp(-n dt / tau_rms),
      truncated at 5 tau_rms.
    """
    dt = 1.0 / (1024.0 * scs_hz)
    if pdp == "taps8":
        n = np.arange(8)
        p = np.exp(-n / 2.0)
    else:
        kind, tau = pdp
        assert kind == "exp"
        n = np.arange(max(1, int(math.ceil(5.0 * tau / dt)) + 1))
        p = np.exp(-n * dt / tau)
    p = p / p.sum()
    return n * dt, p


def rms_delay_spread(delays: np.ndarray, powers: np.ndarray) -> float:
    m = float(np.sum(powers * delays))
    return math.sqrt(float(np.sum(powers * delays ** 2)) - m * m)


def tdl_frequency_response(rng: np.random.Generator, n_rx: int, n_layers: int, n_sc: int,
                           scs_hz: float, delays: np.ndarray, powers: np.ndarray) -> np.ndarray:
    """H[sc][rx][layer] (complex128) of one block-fading TDL realisation.

    H(k) = sum_n g_n sqrt(P_n) exp(-j 2 pi k scs tau_n), g_n ~ CN(0, 1) i.i.d. per
    (tap, rx, layer); unit average power per entry.
    """
    nt = len(delays)
    g = (rng.standard_normal((nt, n_rx * n_layers)) + 1j * rng.standard_normal((nt, n_rx * n_layers)))
    g *= np.sqrt(powers / 2.0)[:, None]
    k = np.arange(n_sc)
    steer = np.exp(-2j * np.pi * np.outer(k * scs_hz, delays))  # [sc][tap]
    return (steer @ g).reshape(n_sc, n_rx, n_layers)


def rayleigh_flat(rng: np.random.Generator, shape_prefix: Sequence[int]) -> np.ndarray:
    """i.i.d. CN(0, 1) entries."""
    return (rng.standard_normal(tuple(shape_prefix)) + 1j * rng.standard_normal(tuple(shape_prefix))) / math.sqrt(2.0)


def awgn(rng: np.random.Generator, shape_prefix: Sequence[int], noise_var: float) -> np.ndarray:
    """CN(0, noise_var) samples as complex64 (drawn in float32 pairs)."""
    w = rng.standard_normal(tuple(shape_prefix) + (2,), dtype=np.float32)
    w *= np.float32(math.sqrt(noise_var / 2.0))
    return w.view(np.complex64)[..., 0]


# ---------------------------------------------------------------------------------------
# Slot assembly.
# ---------------------------------------------------------------------------------------

def transmit_grid(shape: SlotShape, pilots: np.ndarray, x_data: np.ndarray) -> np.ndarray:
    """Per-port transmitted grid X[symb][sc][layer] (complex128).

    Data symbols carry x_data[dsym][sc][layer]; DMRS symbol s0+t carries, for port p,
    the pilot on subcarriers k = (p mod C) + C j and nothing elsewhere.
    """
    X = np.zeros((shape.n_symb, shape.n_sc, shape.n_layers), dtype=np.complex128)
    for di, s in enumerate(shape.data_symbols()):
        X[s] = x_data[di]
    for o, s0 in enumerate(shape.dmrs_sym0):
        for t in range(shape.dmrs_td):
            for p in range(shape.n_layers):
                c = p % shape.dmrs_comb
                ks = np.arange(c, shape.n_sc, shape.dmrs_comb)
                X[s0 + t, ks, p] = pilots[o, t, : len(ks), p]
    return X


def make_slot(shape: SlotShape, rng: np.random.Generator, scs_hz: float, pdp, snr_db: float,
              channel: Optional[np.ndarray] = None, noiseless: bool = False):
    """Draw one slot; returns a dict of host arrays.

    rx [symb][sc][rx] complex64, pilots [occ][t][j][layer] complex64,
    bits [dsym][sc][layer][qm] uint8, x [dsym][sc][layer] complex128,
    h [sc][rx][layer] complex128 (the true channel), noise_var float.
    """
    n_sc, nd = shape.n_sc, shape.n_dsym
    bits = rng.integers(0, 2, size=(nd, n_sc, shape.n_layers, shape.qm), dtype=np.uint8)
    x = qam_map(bits, shape.qm)
    pilots = make_pilots(rng, shape)
    if channel is None:
        delays, powers = power_delay_profile(pdp, scs_hz)
        h = tdl_frequency_response(rng, shape.n_rx, shape.n_layers, n_sc, scs_hz, delays, powers)
    else:
        h = channel
    X = transmit_grid(shape, pilots, x)
    y = np.matmul(h, X.transpose(1, 2, 0)).transpose(2, 0, 1).astype(np.complex64)  # [symb][sc][rx]
    noise_var = 10.0 ** (-snr_db / 10.0)
    if not noiseless:
        y += awgn(rng, y.shape, noise_var)
    return dict(rx=np.ascontiguousarray(y), pilots=pilots, bits=bits, x=x, h=h,
                noise_var=float(noise_var))


def make_batch(name: str, n_slots: Optional[int] = None, snr_db: Optional[Sequence[float]] = None,
               keep_truth: bool = True, first_slot: int = 0, workers: int = 1):
    """Draw a batch of slots for a named workload.

    Slot i is drawn at SNR point i mod len(snr_grid), realisation first_slot + i div
    len(snr_grid), each from its own seeded stream, so the result does not depend on
    ``workers`` (threads drawing slots concurrently).  Returns stacked arrays with a
    leading slot axis.
    """
    cfg = CONFIGS[name]
    grid = tuple(snr_db) if snr_db is not None else cfg["snr_db"]
    n = n_slots if n_slots is not None else len(grid) * cfg["slots_per_snr"]
    shape = cfg["shape"].with_slots(n)
    rx = np.empty((n, shape.n_symb, shape.n_sc, shape.n_rx), np.complex64)
    pil = np.empty((n, shape.n_occ, shape.dmrs_td, shape.n_pilot, shape.n_layers), np.complex64)
    nv = np.empty(n, np.float32)
    snrs = np.array([grid[i % len(grid)] for i in range(n)])
    truth = [None] * n

    def one(i):
        si = i % len(grid)
        sl = first_slot + i // len(grid)
        snr_index = cfg["snr_db"].index(grid[si]) if grid[si] in cfg["snr_db"] else 100 + si
        rng = rng_for(cfg["config_id"], snr_index, sl)
        d = make_slot(shape, rng, cfg["scs_hz"], cfg["pdp"], grid[si])
        rx[i], pil[i], nv[i] = d["rx"], d["pilots"], d["noise_var"]
        if keep_truth:
            truth[i] = (d["bits"], d["x"], d["h"])

    if workers > 1:
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(n)))
    else:
        for i in range(n):
            one(i)
    out = dict(shape=shape, rx=rx, pilots=pil, noise_var=nv, snr_db=snrs)
    if keep_truth:
        out.update(bits=np.stack([t[0] for t in truth]), x=np.stack([t[1] for t in truth]),
                   h=np.stack([t[2] for t in truth]))
    return out


def batch_slot(name: str, i: int) -> dict:
    """Slot i of ``make_batch(name)`` (default SNR grid, first_slot 0) drawn on its own: the
    same seeded stream, so the same bytes as that slot of the whole batch."""
    cfg = CONFIGS[name]
    grid = cfg["snr_db"]
    si, sl = i % len(grid), i // len(grid)
    rng = rng_for(cfg["config_id"], si, sl)
    return make_slot(cfg["shape"].with_slots(1), rng, cfg["scs_hz"], cfg["pdp"], grid[si])


# ---------------------------------------------------------------------------------------
# DMRS-only slots with a time-varying channel (training and test data of the learned
# refinement of the pilot-resolution estimate).
# ---------------------------------------------------------------------------------------

def dmrs_shape(shape: SlotShape, n_slots: int) -> SlotShape:
    """The DMRS occasion of `shape` alone: its T DMRS symbols at symbol 0 and one empty data
    symbol (the smallest slot the library accepts)."""
    return SlotShape(n_prb=shape.n_prb, n_symb=shape.dmrs_td + 1, n_rx=shape.n_rx,
                     n_layers=shape.n_layers, qm=shape.qm, dmrs_comb=shape.dmrs_comb,
                     dmrs_td=shape.dmrs_td, dmrs_sym0=(0,), n_slots=n_slots)


def make_dmrs_slot(shape: SlotShape, rng: np.random.Generator, scs_hz: float, tau_rms: float,
                   doppler_hz: float, snr_db: float, n_sinusoids: int = 16):
    """One DMRS occasion (shape = dmrs_shape(..)) through a TDL channel with an exponential
    PDP of rms delay spread tau_rms whose taps change over the occasion's T symbols with
    maximum Doppler shift doppler_hz (each tap of each (rx, port) link a sum of n_sinusoids
    complex sinusoids of frequency doppler_hz cos(alpha) with random alpha and phase: a
    Jakes-type spectrum, unit power).

    Returns rx [symb][sc][rx] complex64 (data symbol empty), pilots [1][T][J][layer]
    complex64, h [1][J][rx][layer] complex64: the true channel at port layer's pilot
    subcarrier (layer mod C) + C j averaged over the T DMRS symbols (zero where that
    subcarrier is past the band), noise_var.
    """
    C, T, J = shape.dmrs_comb, shape.dmrs_td, shape.n_pilot
    NR, NL, nsc = shape.n_rx, shape.n_layers, shape.n_sc
    pilots = make_pilots(rng, shape)
    delays, powers = power_delay_profile(("exp", tau_rms), scs_hz)
    nt = len(delays)
    t_sym = 1.0 / scs_hz * (1.0 + 144.0 / 2048.0)  # OFDM symbol with its normal cyclic prefix
    alpha = rng.uniform(0, 2 * np.pi, (nt, NR, NL, n_sinusoids))
    phi = rng.uniform(0, 2 * np.pi, (nt, NR, NL, n_sinusoids))
    t = np.arange(T) * t_sym
    g = np.exp(1j * (2 * np.pi * doppler_hz * np.cos(alpha)[..., None] * t + phi[..., None]))
    g = g.sum(axis=3) * np.sqrt(powers / n_sinusoids)[:, None, None, None]  # [tap][rx][port][t]
    k = (np.arange(NL)[None, :] % C) + C * np.arange(J)[:, None]  # [j][port]
    steer = np.exp(-2j * np.pi * scs_hz * k[..., None] * delays)   # [j][port][tap]
    # [t][j][rx][port]: per port, [j][tap] @ [tap][rx t] (a BLAS product per port)
    Ht = np.matmul(steer.transpose(1, 0, 2), g.transpose(2, 0, 1, 3).reshape(NL, nt, NR * T))
    Ht = Ht.reshape(NL, J, NR, T).transpose(3, 1, 2, 0)
    inband = (k < nsc)[None, :, None, :]
    Ht = np.where(inband, Ht, 0)
    y = np.zeros((shape.n_symb, nsc, NR), np.complex128)
    for p in range(NL):
        ks = k[:, p]
        ok = ks < nsc
        for tt in range(T):
            y[tt, ks[ok], :] += Ht[tt, ok, :, p] * pilots[0, tt, ok, p][:, None]
    noise_var = 10.0 ** (-snr_db / 10.0)
    y = y.astype(np.complex64)
    y[:T] += awgn(rng, (T, nsc, NR), noise_var)
    h = Ht.mean(axis=0).astype(np.complex64)[None]
    return dict(rx=y, pilots=pilots, h=h, noise_var=float(noise_var))


# Training / test draws of the refinement: per slot a delay spread in 30..300 ns, a maximum
# Doppler shift in 0..500 Hz and an SNR in 0..30 dB, uniformly.
DMRS_RANGES = dict(tau_rms=(30e-9, 300e-9), doppler_hz=(0.0, 500.0), snr_db=(0.0, 30.0))


def make_dmrs_batch(shape: SlotShape, n_slots: int, seed: int, scs_hz: float = 30e3,
                    snr_db: Optional[Sequence[float]] = None, tau_rms: Optional[float] = None,
                    doppler_hz: Optional[float] = None, workers: int = 1):
    """n_slots DMRS occasions, slot i from its own stream SeedSequence([root, 7, seed, i]);
    fixed snr_db (cycled), tau_rms or doppler_hz replace the uniform draws."""
    sh = dmrs_shape(shape, n_slots)
    rx = np.empty((n_slots, sh.n_symb, sh.n_sc, sh.n_rx), np.complex64)
    pil = np.empty((n_slots, 1, sh.dmrs_td, sh.n_pilot, sh.n_layers), np.complex64)
    h = np.empty((n_slots, 1, sh.n_pilot, sh.n_rx, sh.n_layers), np.complex64)
    nv = np.empty(n_slots, np.float32)
    draws = np.empty((n_slots, 3))

    def one(i):
        rng = rng_for(7, seed, i)
        u = rng.uniform(size=3)
        lo = DMRS_RANGES
        ds = tau_rms if tau_rms is not None else lo["tau_rms"][0] + u[0] * (lo["tau_rms"][1] - lo["tau_rms"][0])
        fd = doppler_hz if doppler_hz is not None else lo["doppler_hz"][0] + u[1] * (lo["doppler_hz"][1] - lo["doppler_hz"][0])
        snr = (snr_db[i % len(snr_db)] if snr_db is not None
               else lo["snr_db"][0] + u[2] * (lo["snr_db"][1] - lo["snr_db"][0]))
        d = make_dmrs_slot(sh, rng, scs_hz, ds, fd, snr)
        rx[i], pil[i], h[i], nv[i] = d["rx"], d["pilots"], d["h"], d["noise_var"]
        draws[i] = (ds, fd, snr)

    if workers > 1:
        import concurrent.futures as cf
        from threadpoolctl import threadpool_limits
        # one BLAS thread per worker: the per-port products are small, and BLAS's own
        # threads on top of the workers' oversubscribe the cores
        with threadpool_limits(limits=1, user_api="blas"), \
                cf.ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(n_slots)))
    else:
        for i in range(n_slots):
            one(i)
    return dict(shape=sh, rx=rx, pilots=pil, h=h, noise_var=nv, tau_rms=draws[:, 0],
                doppler_hz=draws[:, 1], snr_db=draws[:, 2])
