"""Shared parity checks of the GPU tests against the FP64 oracle (not a test module).

Bars, per resource element (RE) and per bit, with no fractional allowance anywhere:

* equalised symbols: ||x_gpu - x_ref|| / ||x_ref|| <= 1e-4 per RE; an RE over it must lie
  within the forward-error bound of its arithmetic, 8 kappa(G + s2 I) Nl u ||x_ref|| with u
  the unit roundoff of the FP32 inversion (2^-24);
* LLRs: |llr_gpu - llr_ref| <= 1e-3 |llr_ref| + 1e-4, or else inside the range the oracle's
  max-log LLR takes over the forward-error ball of its RE (each axis value moved by up to
  the bound above, the post-detection variance by the same relative amount), widened by
  the same per-call bar.  Max-log LLRs are piecewise linear in each axis value with kinks
  on the integer lattice of the unnormalised constellation (the bits of one axis depend on
  that axis alone), so the range is attained at the ends of the interval or at a lattice
  point inside it;
* hard decisions: bit-exact wherever the oracle's axis value lies more than 1e-3 from the
  bit's decision boundary and |llr_ref| > 1e-3 (reading R10); every bit, excluded or not,
  still meets the LLR bar above.

Every over-tolerance element is audited (none is skipped); counts are printed.
"""
from __future__ import annotations

import sys

import numpy as np

import oracle
import synth

U32 = 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def llr_tol(lr):
    return 1e-3 * np.abs(lr) + 1e-4


def llr_tol_ok(lg, lr):
    return np.abs(lg - lr) <= llr_tol(lr)


def kappa_delta(G, nl, u=U32):
    """Relative forward-error bound 8 kappa(G) Nl u of a solve with the Gram G (batched)."""
    return 8.0 * np.linalg.cond(G) * nl * u


def llr_interval(x, nv, r, rho, qm):
    """Range [lo, hi] (each [n][qm]) of the oracle's max-log LLRs over every x' whose real
    and imaginary parts are within r of those of x and every variance within nv (1 +- rho).
    x complex [n]; nv, r, rho real [n]."""
    x = np.asarray(x, np.complex128).reshape(-1)
    n = x.size
    nv = np.broadcast_to(np.asarray(nv, np.float64), (n,))
    r = np.broadcast_to(np.asarray(r, np.float64), (n,))
    rho = np.broadcast_to(np.asarray(rho, np.float64), (n,))
    if n == 0:
        return np.zeros((0, qm)), np.zeros((0, qm))
    sc = synth.qam_scale(qm)
    lim = 2 ** (qm // 2)  # kinks lie on integers within the constellation's span

    def axis(v):
        lo_u, hi_u = (v - r) * sc, (v + r) * sc
        a = np.maximum(np.ceil(lo_u), -lim)
        b = np.minimum(np.floor(hi_u), lim)
        k = int(np.clip(np.max(b - a + 1), 0, 2 * lim + 1)) if n else 0
        cols = [v - r, v, v + r]
        for i in range(k):
            cols.append(np.clip((a + i) / sc, v - r, v + r))  # past b: clipped to an end
        return np.stack(cols, axis=1)

    re_, im_ = axis(x.real), axis(x.imag)
    w = max(re_.shape[1], im_.shape[1])
    re_ = np.pad(re_, ((0, 0), (0, w - re_.shape[1])), mode="edge")
    im_ = np.pad(im_, ((0, 0), (0, w - im_.shape[1])), mode="edge")
    pts = (re_ + 1j * im_).reshape(-1)  # candidate j pairs the j-th value of each axis
    v = oracle.llr_batch(pts, np.repeat(nv, w), qm).reshape(n, w, qm)
    with np.errstate(divide="ignore", invalid="ignore"):
        s_lo, s_hi = 1.0 / (1.0 + rho), 1.0 / np.maximum(1.0 - rho, 1e-300)
    cand = np.concatenate([v * s_lo[:, None, None], v * s_hi[:, None, None]], axis=1)
    return cand.min(axis=1), cand.max(axis=1)


def audit_llrs(lg, lr, xr, nvr, radius, qm, label="", cap=None):
    """Hard decisions and LLRs of one set of REs against the oracle (see module docstring).

    lg, lr: [..][qm] GPU and oracle LLRs; xr, nvr: [..] oracle x~ and nu2 of each (RE, layer);
    radius(idx) -> (r, rho): absolute per-axis radius and relative variance bound of the
    (RE, layer) elements at flat indices idx (arrays).  cap: fail if more elements need the
    audit than this (a loud limit on the audit's cost, never a silent one)."""
    lg = np.asarray(lg).reshape(-1, qm)
    lr = np.asarray(lr).reshape(-1, qm)
    xr = np.asarray(xr).reshape(-1)
    nvr = np.asarray(nvr).reshape(-1)
    keep = (axis_margin(xr, qm) > 1e-3) & (np.abs(lr) > 1e-3)
    mism = ((lg < 0) != (lr < 0)) & keep
    assert not mism.any(), (f"{label}: {int(mism.sum())} hard decisions differ away from "
                            f"boundaries, e.g. at {np.argwhere(mism)[:5].tolist()}")
    tol = llr_tol(lr)
    over = ~(np.abs(lg - lr) <= tol)
    rows = np.unique(np.nonzero(over)[0])
    if cap is not None:
        assert rows.size <= cap, f"{label}: {rows.size} elements need the audit (cap {cap})"
    worst_r = 0.0
    if rows.size:
        r, rho = radius(rows)
        lo, hi = llr_interval(xr[rows], nvr[rows], r, rho, qm)
        g, t = lg[rows], tol[rows]
        bad = over[rows] & ~((g >= lo - t) & (g <= hi + t))
        assert not bad.any(), (f"{label}: {int(bad.sum())} LLRs outside the forward-error "
                               f"range; first: element {rows[np.nonzero(bad)[0][0]]} gpu "
                               f"{g[bad][:4]} ref {lr[rows][bad][:4]} range "
                               f"{lo[bad][:4]}..{hi[bad][:4]}")
        worst_r = float(np.max(r / np.maximum(np.abs(xr[rows]), 1e-30)))
    say(f"  {label}: {lg.size} LLRs, over the per-call bar {int(over.sum())} (all inside "
        f"their forward-error range, largest relative radius {worst_r:.1e}), near "
        f"boundaries {int((~keep).sum())}")
    return int(over.sum())


def kappa_radius(grams, xr_re, nl, u=U32):
    """radius() for audit_llrs from per-RE Grams: grams(idx_re) -> G [k][nl][nl] of the REs
    at flat RE indices idx_re; xr_re: oracle x~ [n_re][nl].  The radius of element
    (RE, layer) is kappa_delta(G) ||x~_RE||, the variance bound kappa_delta(G)."""
    def radius(idx):
        re_idx = idx // nl
        uniq, inv = np.unique(re_idx, return_inverse=True)
        d = kappa_delta(grams(uniq), nl, u)
        norm = np.linalg.norm(xr_re[uniq], axis=-1)
        return (d * norm)[inv], d[inv]
    return radius


def check_x(xg, xr, nvg, nvr, grams, nl, label="", u=U32, cap=200000):
    """Per-RE relative error of x~ and nu2 (arrays [..][nl]); REs over 1e-4 must satisfy the
    forward-error bound of their Gram (grams(flat RE indices) -> G)."""
    xg = np.asarray(xg).reshape(-1, nl)
    xr = np.asarray(xr).reshape(-1, nl)
    nvg = np.asarray(nvg).reshape(-1, nl)
    nvr = np.asarray(nvr).reshape(-1, nl)
    err_x = np.linalg.norm(xg - xr, axis=-1) / np.linalg.norm(xr, axis=-1)
    err_v = np.max(np.abs(nvg - nvr) / np.maximum(np.abs(nvr), 1e-30), axis=-1)
    over = np.nonzero((err_x > 1e-4) | (err_v > 1e-4))[0]
    assert over.size <= cap, f"{label}: {over.size} REs over 1e-4 (audit cap {cap})"
    kmax = 0.0
    if over.size:
        d = kappa_delta(grams(over), nl, u)
        e = np.maximum(err_x[over], err_v[over])
        bad = e > d
        assert not bad.any(), (f"{label}: REs over the forward-error bound: "
                               f"{over[bad][:5].tolist()} err {e[bad][:5]} bound {d[bad][:5]}")
        kmax = float(np.max(d))
    say(f"  {label}: {err_x.size} REs, max rel err x {err_x.max():.2e} nv {err_v.max():.2e}, "
        f"{over.size} over 1e-4 (all within their bound, largest {kmax:.1e})")
    return err_x


def gram_fn(shape, h, h_res, nvar):
    """grams(idx) for flat RE indices over [slot][dsym][sc]: the oracle's Gram
    H^H H + s2 I of each RE's interpolated channel (h is what both sides read)."""
    h = np.ascontiguousarray(h, np.complex64)
    ds = shape.data_symbols()
    nd, nsc = shape.n_dsym, shape.n_sc
    cache = {}

    def grams(idx):
        out = np.empty((len(idx), shape.n_layers, shape.n_layers), np.complex128)
        for i, f in enumerate(np.asarray(idx)):
            s, rem = divmod(int(f), nd * nsc)
            d, k = divmod(rem, nsc)
            key = (s, k, ds[d] if shape.n_occ > 1 else -1)
            G = cache.get(key)
            if G is None:
                H = oracle.channel_at(shape, h, h_res, s, k, ds[d])
                G = cache[key] = oracle.gram(H, float(nvar[s]))
            out[i] = G
        return out
    return grams


# ---- the 16-bit product modes --------------------------------------------------------------
# The kernels round the channel (interpolated in FP32) and the received samples to the 16-bit
# type before the Gram and matched-filter products, and form those products exactly (a product
# of two 16-bit values is exact in FP32) with FP32 accumulation; inversion and everything after
# it run in FP32.  So the result is the FP32 detection of the rounded inputs, and the oracle
# run on the same rounded inputs must meet the FP32 bars above.

SIG_BITS = {"fp16": 11, "bf16": 8}


def round_sig(v, p):
    """float32 values rounded to p significant bits, ties to even, exponent unbounded (the
    16-bit rounding of values inside the type's normal range)."""
    m, e = np.frexp(np.asarray(v, np.float64))
    return np.ldexp(np.rint(np.ldexp(m, p)), e - p).astype(np.float32)


def round_complex(z, p):
    z = np.asarray(z, np.complex64)
    return (round_sig(z.real, p) + 1j * round_sig(z.imag, p)).astype(np.complex64)


def freq_rule(shape, p, k):
    """Pilot indices (j0, j1) and weight a of port p at subcarriers k (arrays), reading R2:
    linear between the port's consecutive pilots, nearest pilot held outside."""
    C = shape.dmrs_comb
    c = p % C
    jp = -(-(shape.n_sc - c) // C)
    last = c + C * (jp - 1)
    inner = (k > c) & (k < last)
    j0 = np.where(k <= c, 0, np.where(k >= last, jp - 1, (k - c) // C))
    j1 = np.where(inner, j0 + 1, j0)
    a = np.where(inner, (k - c - C * j0) / C, 0.0)
    return j0, j1, a


def fp32_interpolated_channel(shape, h):
    """[slot][sc][rx][layer] complex64: a one-occasion pilot-resolution estimate h
    [slot][1][j][rx][layer] interpolated in FP32 as v0 + a (v1 - v0) with a single rounding
    (a fused multiply-add; a = m / C is exact), as the detector forms it before rounding."""
    assert shape.n_occ == 1
    h = np.asarray(h, np.complex64)
    S, nsc, NR, NL = shape.n_slots, shape.n_sc, shape.n_rx, shape.n_layers
    k = np.arange(nsc)
    out = np.empty((S, nsc, NR, NL), np.complex64)
    for p in range(NL):
        j0, j1, a = freq_rule(shape, p, k)
        al = np.asarray(a, np.longdouble)[None, :, None]
        parts = []
        for comp in (np.real, np.imag):
            v0 = comp(h[:, 0][:, j0][..., p]).astype(np.float32)  # [slot][sc][rx]
            v1 = comp(h[:, 0][:, j1][..., p]).astype(np.float32)
            d = (v1 - v0).astype(np.float32)
            parts.append((al * d.astype(np.longdouble) + v0.astype(np.longdouble)).astype(np.float32))
        out[:, :, :, p] = parts[0] + 1j * parts[1]
    return out


def rounding_bound(Hsc, y, xt, nv, s2, u):
    """Per (RE, layer) bound on |x~(rounded inputs) - x~(exact inputs)| and on the variance,
    from perturbation theory with every channel value and sample moved by at most u of its
    magnitude: ||dG|| <= u ||H||_F (2 ||H||_2 + u ||H||_F), ||dz|| <= u (||H||_F + ||H||_2
    + u ||H||_F) ||y||, ||dx^|| <= (||dz|| + ||dG|| ||x^||) / (lmin - ||dG||),
    |d diag(A^-1)| <= ||dG|| / (lmin (lmin - ||dG||)), then through mu = 1 - s2 d.
    Hsc [n][nr][nl] (per RE), y [n][nr], xt/nv [n][nl] (oracle on exact inputs), s2 [n].
    Returns (bx [n][nl], bv [n][nl], valid [n]); invalid REs have no finite bound."""
    nF = np.linalg.norm(Hsc, axis=(1, 2))
    n2 = np.linalg.norm(Hsc, ord=2, axis=(1, 2))
    ny = np.linalg.norm(y, axis=1)
    G = np.einsum("nrl,nrm->nlm", Hsc.conj(), Hsc) + s2[:, None, None] * np.eye(Hsc.shape[2])
    lam = np.linalg.eigvalsh(G)[:, 0]
    eG = u * nF * (2 * n2 + u * nF)
    ez = u * (nF + n2 + u * nF) * ny
    mu = 1.0 / (1.0 + nv)
    ex = (ez + eG * np.linalg.norm(xt * mu, axis=1)) / (lam - eG)
    dmu = s2[:, None] * (eG / (lam * (lam - eG)))[:, None]
    valid = (lam > eG) & np.all(mu > dmu, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        bx = (ex[:, None] + np.abs(xt) * dmu) / (mu - dmu)
        bv = dmu / (mu * (mu - dmu))
    return bx, bv, valid


def refined_bound(Hsc, y, xt, nv, s2, p):
    """Per (RE, layer) bound on |x~(refined 16-bit mode) - x~(exact inputs)| and on the
    variance, for the one-step refinement of the 16-bit detector (without FP32 rounding,
    which the caller adds).  Each value is split into a p-bit part (error u1 = 2^-p of its
    magnitude) and a p-bit remainder (what is left, u2 = 2^-2p).  With A = G~ + s2 I the
    inverted 16-bit system, dG the first-order Gram correction, dZ (resp. dG2) what the
    split leaves out of the matched filter (resp. the Gram), E = A^-1 (dG + dG2) and x* the
    exact solution, the refined x^ differs from x* by
        -A^-1 dZ + A^-1 dG A^-1 dZ + A^-1 dG2 (I + E) x* - E^2 x*
    and diag(A^-1 - A^-1 dG A^-1) from diag(G^-1) by at most ||dG2|| / lA^2 + ||E||^2 / l,
    so with ||dG|| <= u1 nF (2 n2 + u1 nF), ||dG2|| <= u1^2 nF^2 + u2 nF (2 n2 + 2 u1 nF +
    u2 nF), ||dZ|| <= (u1^2 nF + u2 (2 nF + n2 + u1 nF)) ||y|| (nF, n2: Frobenius and
    spectral norms of H; l = lmin(G + s2 I), lA >= l - ||dG|| - ||dG2||).  Returns
    (bx [n][nl], bv [n][nl], valid [n]) as rounding_bound does."""
    u1, u2 = 2.0 ** -p, 2.0 ** (-2 * p)
    nF = np.linalg.norm(Hsc, axis=(1, 2))
    n2 = np.linalg.norm(Hsc, ord=2, axis=(1, 2))
    ny = np.linalg.norm(y, axis=1)
    G = np.einsum("nrl,nrm->nlm", Hsc.conj(), Hsc) + s2[:, None, None] * np.eye(Hsc.shape[2])
    lam = np.linalg.eigvalsh(G)[:, 0]
    eD = u1 * nF * (2 * n2 + u1 * nF)
    eD2 = u1 ** 2 * nF ** 2 + u2 * nF * (2 * n2 + 2 * u1 * nF + u2 * nF)
    ez = (u1 ** 2 * nF + u2 * (2 * nF + n2 + u1 * nF)) * ny
    lA = lam - eD - eD2
    E = (eD + eD2) / lA
    mu = 1.0 / (1.0 + nv)
    xs = np.linalg.norm(xt * mu, axis=1)  # ||x^*|| (biased solution)
    ex = ez * (1.0 + eD / lA) / lA + eD2 * (1.0 + E) * xs / lA + E ** 2 * xs
    dd = eD2 / lA ** 2 + E ** 2 / lam
    dmu = s2[:, None] * dd[:, None]
    valid = (lA > 0) & (E < 1) & np.all(mu > dmu, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        bx = (ex[:, None] + np.abs(xt) * dmu) / (mu - dmu)
        bv = dmu / (mu * (mu - dmu))
    return bx, bv, valid
