"""CPU checks of the audit that the GPU parity tests rely on (tests/parity.py): the LLR range
over a forward-error ball brackets the oracle's LLR at every point of the ball, and the audit
passes results inside their bound and fails a planted error outside it."""
import numpy as np
import pytest

import oracle
import parity
import synth


@pytest.mark.parametrize("qm", [2, 4, 6, 8])
def test_llr_interval_brackets_every_point_of_the_ball(qm):
    rng = np.random.default_rng(qm)
    n = 400
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 0.9
    nv = rng.uniform(1e-3, 1.0, n)
    r = rng.uniform(0.0, 0.3, n) * rng.choice([1e-4, 1e-2, 1.0], n)
    rho = rng.uniform(0.0, 0.2, n)
    lo, hi = parity.llr_interval(x, nv, r, rho, qm)
    for _ in range(20):
        dx = (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)) * r
        f = 1.0 + rng.uniform(-1, 1, n) * rho
        v = oracle.llr_batch(x + dx, nv * f, qm)
        slack = 1e-9 * (1 + np.abs(v))
        assert np.all(v >= lo - slack) and np.all(v <= hi + slack)
    # the range is attained: its ends are LLRs of points of the ball
    v0 = oracle.llr_batch(x, nv, qm)
    assert np.all(lo <= v0 + 1e-12) and np.all(v0 <= hi + 1e-12)


def test_llr_interval_of_a_point_is_the_point():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    lo, hi = parity.llr_interval(x, 0.1, 0.0, 0.0, 6)
    v = oracle.llr_batch(x, 0.1, 6)
    np.testing.assert_array_equal(lo, v)
    np.testing.assert_array_equal(hi, v)


def _detector_case(seed=3, nr=4, nl=2, n=3000, s2=1e-3):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((n, nr, nl)) + 1j * rng.standard_normal((n, nr, nl))) / np.sqrt(2)
    bits = rng.integers(0, 2, (n, nl, 4)).astype(np.uint8)
    xs = synth.qam_map(bits, 4)
    y = np.einsum("nrl,nl->nr", H, xs) + np.sqrt(s2 / 2) * (
        rng.standard_normal((n, nr)) + 1j * rng.standard_normal((n, nr)))
    xt, nv, _ = oracle.mmse_batch(H, y, s2)
    G = np.einsum("nrl,nrm->nlm", H.conj(), H) + s2 * np.eye(nl)
    return H, y, xt, nv, G


def test_audit_passes_results_inside_the_bound_and_fails_a_planted_error():
    H, y, xt, nv, G = _detector_case()
    nl, qm = 2, 4
    lr = oracle.llr_batch(xt.reshape(-1), nv.reshape(-1), qm).reshape(-1, nl, qm)
    delta = parity.kappa_delta(G, nl)
    radius = parity.kappa_radius(lambda idx: G[idx], xt, nl)
    # a result perturbed within its bound (half of it) passes
    rng = np.random.default_rng(4)
    d = 0.5 * delta[:, None] * np.linalg.norm(xt, axis=-1)[:, None]
    xg = xt + d * (rng.uniform(-1, 1, xt.shape) + 1j * rng.uniform(-1, 1, xt.shape)) / np.sqrt(2)
    nvg = nv * (1 + 0.5 * delta[:, None] * rng.uniform(-1, 1, nv.shape))
    lg = oracle.llr_batch(xg.reshape(-1), nvg.reshape(-1), qm).reshape(-1, nl, qm)
    parity.audit_llrs(lg, lr, xt, nv, radius, qm, "inside the bound")
    parity.check_x(xg, xt, nvg, nv, lambda idx: G[idx], nl, "inside the bound")
    # one LLR moved well outside its range fails, even with its hard decision unchanged
    bad = lg.copy()
    k = int(np.argmax(np.abs(lr[:, 0, 1])))
    bad[k, 0, 1] = lr[k, 0, 1] * (1.5 + 100 * delta[k])
    with pytest.raises(AssertionError):
        parity.audit_llrs(bad, lr, xt, nv, radius, qm, "planted LLR error")
    # one symbol moved past its bound fails the per-RE check
    xb = xg.copy()
    xb[k] = xt[k] * (1 + 10 * max(delta[k], 1e-4))
    with pytest.raises(AssertionError):
        parity.check_x(xb, xt, nvg, nv, lambda idx: G[idx], nl, "planted symbol error")
    # a flipped hard decision away from a boundary fails
    fl = lg.copy()
    m = parity.axis_margin(xt.reshape(-1), qm).reshape(-1, nl, qm)
    j = int(np.argmax(m[:, 1, 0]))
    fl[j, 1, 0] = -lg[j, 1, 0]
    with pytest.raises(AssertionError):
        parity.audit_llrs(fl, lr, xt, nv, radius, qm, "planted flip")


def test_audit_cap_is_loud():
    H, y, xt, nv, G = _detector_case(n=200)
    lr = oracle.llr_batch(xt.reshape(-1), nv.reshape(-1), 4).reshape(-1, 2, 4)
    with pytest.raises(AssertionError, match="cap"):
        parity.audit_llrs(lr * 1.1, lr, xt, nv, parity.kappa_radius(lambda i: G[i], xt, 2), 4,
                          "capped", cap=3)


def test_batch_slot_is_the_batch_slot():
    b = synth.make_batch("p4", n_slots=10)
    for i in (0, 6, 9):
        d = synth.batch_slot("p4", i)
        assert np.array_equal(b["rx"][i], d["rx"])
        assert np.array_equal(b["pilots"][i], d["pilots"])
        assert b["noise_var"][i] == np.float32(d["noise_var"])


def test_round_sig_is_the_16_bit_rounding():
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-8, 8, 200000))).astype(np.float32)
    x = np.concatenate([x, np.float32([1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, -(1.0 + 2 ** -8),
                                       1.0 + 3 * 2 ** -8])])  # ties of both types
    normal16 = (np.abs(x) >= 2.0 ** -14) & (np.abs(x) <= 65504)
    np.testing.assert_array_equal(parity.round_sig(x, 11)[normal16],
                                  x[normal16].astype(np.float16).astype(np.float32))
    # bfloat16: the top 16 bits of the float32 pattern after round-to-nearest-even
    b = x.view(np.uint32).astype(np.uint64)
    rb = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    np.testing.assert_array_equal(parity.round_sig(x, 8), rb)


def test_fp32_interpolation_model_is_the_interpolation():
    # The FP32 single-rounding interpolation the 16-bit test feeds the oracle stays within one
    # FP32 rounding of the oracle's own FP64 interpolation of the same estimate.
    from synth import SlotShape
    shape = SlotShape(5, 14, 16, 9, 4, 8, 2, (2,), 2)
    rng = np.random.default_rng(8)
    h = (rng.standard_normal((2, 1, shape.n_pilot, 16, 9)) +
         1j * rng.standard_normal((2, 1, shape.n_pilot, 16, 9))).astype(np.complex64)
    hk = parity.fp32_interpolated_channel(shape, h)
    for s in range(2):
        for k in (0, 3, 7, 8, 31, shape.n_sc - 1):
            H = oracle.channel_at(shape, h, oracle.H_PILOT, s, k, 0)
            ref = H.astype(np.complex128)
            err = np.abs(hk[s, k] - ref)  # two FP32 roundings (v1 - v0, then the fma)
            assert np.all(err <= 2.0 ** -22 * np.abs(h[s]).max()), err.max()


def _round_c(z, p):
    """Complex values rounded to p significant bits per part, in float64 (no range limit)."""
    def r(v):
        m, e = np.frexp(v)
        return np.ldexp(np.rint(np.ldexp(m, p)), e - p)
    return r(z.real) + 1j * r(z.imag)


@pytest.mark.parametrize("p", [11, 8])
def test_refined_bound_holds_for_the_refinement_step(p):
    # The refinement of the 16-bit detector written out in float64 (each value split into a
    # p-bit part and a p-bit remainder; inverse of the split Gram; one correction of the
    # solution and of diag(G^-1) with dG = H_hi^H H_lo + H_lo^H H_hi), against the exact
    # unbiased MMSE solution: every element within parity.refined_bound, which must also be
    # far below the unrefined rounding bound; and a planted slip (the correction's sign
    # flipped) must break it.
    rng = np.random.default_rng(7 + p)
    nr, nl, n = 32, 8, 60
    H = (rng.standard_normal((n, nr, nl)) + 1j * rng.standard_normal((n, nr, nl))) / np.sqrt(2)
    x = (rng.choice([-1, 1], (n, nl)) + 1j * rng.choice([-1, 1], (n, nl))) / np.sqrt(2)
    s2 = np.full(n, 10 ** -2.0)
    y = np.einsum("nrl,nl->nr", H, x) + np.sqrt(s2[:, None] / 2) * (
        rng.standard_normal((n, nr)) + 1j * rng.standard_normal((n, nr)))
    eye = np.eye(nl)

    def unbiased(xh, d):
        mu = 1 - s2[:, None] * d
        return xh / mu, (1 - mu) / mu

    G = np.einsum("nrl,nrm->nlm", H.conj(), H) + s2[:, None, None] * eye
    Gi = np.linalg.inv(G)
    xt, nvt = unbiased(np.einsum("nlm,nm->nl", Gi, np.einsum("nrl,nr->nl", H.conj(), y)),
                       np.real(np.einsum("nll->nl", Gi)))

    def refined(sign, dsign):
        Hh, yh = _round_c(H, p), _round_c(y, p)
        Hl, yl = _round_c(H - Hh, p), _round_c(y - yh, p)
        A = np.einsum("nrl,nrm->nlm", Hh.conj(), Hh) + s2[:, None, None] * eye
        dG = np.einsum("nrl,nrm->nlm", Hh.conj(), Hl) + np.einsum("nrl,nrm->nlm", Hl.conj(), Hh)
        z = sum(np.einsum("nrl,nr->nl", a.conj(), b) for a, b in ((Hh, yh), (Hh, yl), (Hl, yh)))
        Ai = np.linalg.inv(A)
        x0 = np.einsum("nlm,nm->nl", Ai, z)
        M = Ai @ dG
        x1 = x0 - sign * np.einsum("nlm,nm->nl", M, x0)
        d1 = np.real(np.einsum("nll->nl", Ai - dsign * (M @ Ai)))
        return unbiased(x1, d1), unbiased(x0, np.real(np.einsum("nll->nl", Ai)))

    def rms(a, b):
        return np.sqrt(np.mean(np.abs(a - b) ** 2))

    (xg, nvg), (x0, nv0) = refined(+1, +1)
    bx, bv, valid = parity.refined_bound(H, y, xt, nvt, s2, p)
    bx1, bv1, valid1 = parity.rounding_bound(H, y, xt, nvt, s2, 2.0 ** -p)
    assert valid.all() and valid1.all()
    assert np.all(np.abs(xg - xt) <= bx) and np.all(np.abs(nvg - nvt) <= bv)
    assert np.median(bx / bx1) < 0.1  # an order of magnitude below the unrefined bound
    # the step's effect: the refined errors far below the unrefined ones
    assert rms(xg, xt) < 0.1 * rms(x0, xt) and rms(nvg, nvt) < 0.1 * rms(nv0, nvt)
    # planted slips: the correction's sign flipped, or diag(G^-1) left uncorrected
    (xb, _), _ = refined(-1, +1)
    assert not rms(xb, xt) < 0.1 * rms(x0, xt)
    (_, nvb), _ = refined(+1, 0)
    assert not rms(nvb, nvt) < 0.1 * rms(nv0, nvt)
