"""The C ABI on the host (no GPU): the library loads, exports what the header declares,
and its validation rejects bad input before any launch."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2510_07843_amd as ranphy
import synth
from synth import SlotShape

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ranphy.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ranphy.LIB_PATH):
        from paper_2510_07843_amd import build
        build.build_library()
    return ranphy.lib()


def header_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"RANPHY_API\s+[\w\s\*]+?\b(ranphy_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    assert header_functions() == sorted(ranphy.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", ranphy.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(\w+)$", out, re.M))
    for f in header_functions():
        assert f in exported
        assert hasattr(L, f)
    # Only the C ABI is visible.
    assert exported == set(header_functions())


def test_abi_version_matches_header(L):
    v = int(re.search(r"#define RANPHY_ABI_VERSION (\d+)", open(HEADER).read()).group(1))
    assert ranphy.abi_version() == v


def test_status_strings(L):
    for s in (0, -1, -2, -3, 7):
        assert isinstance(ranphy.status_str(s), str) and ranphy.status_str(s)
    assert ranphy.status_str(-2) != ranphy.status_str(-1)


@pytest.mark.parametrize("name", ["c1", "c2", "m"])
def test_buffer_sizes_match_layouts(L, name):
    sh = synth.CONFIGS[name]["shape"].with_slots(3)
    S, J = 3, sh.n_pilot
    assert ranphy.buffer_floats(sh, ranphy.BUF_RX) == 2 * S * 14 * sh.n_sc * sh.n_rx
    assert ranphy.buffer_floats(sh, ranphy.BUF_PILOTS) == 2 * S * sh.n_occ * sh.dmrs_td * J * sh.n_layers
    assert ranphy.buffer_floats(sh, ranphy.BUF_H, ranphy.H_PILOT) == 2 * S * sh.n_occ * J * sh.n_rx * sh.n_layers
    assert ranphy.buffer_floats(sh, ranphy.BUF_H, ranphy.H_FULL) == 2 * S * sh.n_occ * sh.n_sc * sh.n_rx * sh.n_layers
    assert ranphy.buffer_floats(sh, ranphy.BUF_NOISE_VAR) == S
    assert ranphy.buffer_floats(sh, ranphy.BUF_X) == 2 * S * sh.n_dsym * sh.n_sc * sh.n_layers
    assert ranphy.buffer_floats(sh, ranphy.BUF_NV) == S * sh.n_dsym * sh.n_sc * sh.n_layers
    assert ranphy.buffer_floats(sh, ranphy.BUF_LLR) == S * sh.n_dsym * sh.n_sc * sh.n_layers * sh.qm


GOOD = dict(n_prb=4, n_symb=14, n_rx=8, n_layers=4, qm=4, dmrs_comb=4, dmrs_td=1, dmrs_sym0=(2,),
            n_slots=2)

BAD = [
    (dict(n_prb=0), -1), (dict(n_prb=276), -1), (dict(n_symb=15), -1), (dict(n_symb=0), -1),
    (dict(n_rx=0), -1), (dict(n_rx=65, n_layers=4), -2), (dict(n_layers=0), -1),
    (dict(n_layers=17, n_rx=32, dmrs_comb=8, dmrs_td=2), -2), (dict(n_layers=9, n_rx=8), -2),
    (dict(qm=3), -1), (dict(qm=10), -1), (dict(dmrs_comb=3), -1), (dict(dmrs_comb=1), -1),
    (dict(dmrs_td=3), -1), (dict(n_layers=5), -2),  # 5 > C T = 4
    (dict(dmrs_sym0=(13,), dmrs_td=2), -1), (dict(dmrs_sym0=(-1,)), -1),
    (dict(dmrs_sym0=(5, 3)), -1), (dict(dmrs_sym0=(2, 2)), -1), (dict(dmrs_sym0=(2, 3), dmrs_td=2), -1),
    (dict(n_slots=-1), -1), (dict(dmrs_sym0=(0,), n_symb=1), -1),  # no data symbol left
]


def _desc(**kw):
    a = dict(GOOD)
    a.update(kw)
    return ranphy.SlotDesc.make(**a)


def _calls(L, d, p):
    P = ctypes.c_void_p
    return [
        L.ranphy_chest_ls(ctypes.byref(d), P(p), P(p), P(p), 0, None),
        L.ranphy_mmse_detect(ctypes.byref(d), P(p), P(p), 0, P(p), P(p), P(p), None),
        L.ranphy_llr_demap(ctypes.byref(d), P(p), P(p), P(p), None),
        L.ranphy_mmse_llr(ctypes.byref(d), P(p), P(p), 0, P(p), P(p), P(p), P(p), 0, None),
        L.ranphy_receive(ctypes.byref(d), P(p), P(p), P(p), P(p), None),
    ]


@pytest.mark.parametrize("kw,code", BAD)
def test_invalid_descriptors_rejected_before_launch(L, kw, code):
    d = _desc(**kw)
    # Pointers that would fault if touched; validation must stop first.
    assert _calls(L, d, 0x1000) == [code] * 5
    assert L.ranphy_buffer_floats(ctypes.byref(d), ranphy.BUF_RX, 0) == code


def test_null_descriptor(L):
    P = ctypes.c_void_p
    assert L.ranphy_chest_ls(None, P(0x1000), P(0x1000), P(0x1000), 0, None) == -1
    assert L.ranphy_mmse_detect(None, P(8), P(8), 0, P(8), P(8), P(8), None) == -1
    assert L.ranphy_llr_demap(None, P(8), P(8), P(8), None) == -1
    assert L.ranphy_receive(None, P(8), P(8), P(8), P(8), None) == -1


def test_one_launch_chain_above_8_layers_needs_the_matrix_core_shapes(L):
    P = ctypes.c_void_p
    d = _desc(n_layers=9, n_rx=12, dmrs_comb=8, dmrs_td=2)  # 12 antennas: no matrix-core form
    assert L.ranphy_receive(ctypes.byref(d), P(16), P(16), P(16), P(16), None) == -2
    d = _desc(n_layers=9, n_rx=16, dmrs_comb=8, dmrs_td=2, dmrs_sym0=(2, 10))  # two occasions
    assert L.ranphy_receive(ctypes.byref(d), P(16), P(16), P(16), P(16), None) == -2
    d = _desc(n_layers=9, n_rx=16, dmrs_comb=8, dmrs_td=2)
    assert L.ranphy_receive(ctypes.byref(d), P(8), P(16), P(16), P(16), None) == -2  # rx 8-aligned
    assert L.ranphy_receive(ctypes.byref(d), P(16), P(16), P(16), P(0x1008), None) == -2
    assert L.ranphy_receive(ctypes.byref(d), P(16), P(16), P(0x1002), P(16), None) == -1


def test_null_and_misaligned_pointers_rejected(L):
    d = _desc()
    assert _calls(L, d, 0) == [-1] * 5
    assert _calls(L, d, 0x1004) == [-1] * 5
    P = ctypes.c_void_p
    assert L.ranphy_chest_ls(ctypes.byref(d), P(8), P(8), P(8), 2, None) == -1  # bad h_res
    assert L.ranphy_mmse_detect(ctypes.byref(d), P(8), P(8), 5, P(8), P(8), P(8), None) == -1


def test_empty_batch_is_a_no_op(L):
    d = _desc(n_slots=0)
    assert _calls(L, d, 0) == [0] * 5


def test_binding_refuses_host_tensors(L):
    import torch
    sh = SlotShape(**{k: v for k, v in GOOD.items()})
    rx = torch.zeros(ranphy.buffer_floats(sh, ranphy.BUF_RX) // 2, dtype=torch.complex64)
    pil = torch.zeros(ranphy.buffer_floats(sh, ranphy.BUF_PILOTS) // 2, dtype=torch.complex64)
    with pytest.raises(ValueError, match="GPU tensor"):
        ranphy.chest_ls(sh, rx, pil, h=torch.zeros(1, dtype=torch.complex64))


def test_reduced_precision_rejected_off_the_matrix_core_shapes(L):
    P = ctypes.c_void_p
    # Two DMRS occasions (time-varying channel): only the FP32 path takes it.
    d = _desc(n_rx=16, n_layers=8, dmrs_comb=4, dmrs_td=2, dmrs_sym0=(2, 10))
    for prec in (1, 2):
        assert L.ranphy_mmse_detect_prec(ctypes.byref(d), P(0x1000), P(0x1000), 0, P(0x1000),
                                         P(0x1000), P(0x1000), prec, None) == -2
    # Four layers: below the matrix-core range.
    d = _desc(n_rx=16, n_layers=4)
    assert L.ranphy_mmse_detect_prec(ctypes.byref(d), P(0x1000), P(0x1000), 0, P(0x1000),
                                     P(0x1000), P(0x1000), 1, None) == -2
    # Unknown precision code.
    assert L.ranphy_mmse_detect_prec(ctypes.byref(d), P(0x1000), P(0x1000), 0, P(0x1000),
                                     P(0x1000), P(0x1000), 7, None) == -1


def test_fused_detect_demap_validation(L):
    P = ctypes.c_void_p
    # Matrix-core shape: 16 Rx, 8 layers, one occasion.
    d = _desc(n_rx=16, n_layers=8, dmrs_comb=4, dmrs_td=2)
    a = P(0x1000)
    # x and nv come together or not at all.
    assert L.ranphy_mmse_llr(ctypes.byref(d), a, a, 0, a, a, None, a, 0, None) == -1
    assert L.ranphy_mmse_llr(ctypes.byref(d), a, a, 0, a, None, a, a, 0, None) == -1
    # The LLR buffer is required; the noise variances are required.
    assert L.ranphy_mmse_llr(ctypes.byref(d), a, a, 0, a, None, None, None, 0, None) == -1
    assert L.ranphy_mmse_llr(ctypes.byref(d), a, a, 0, None, None, None, a, 0, None) == -1
    # Unknown precision or channel resolution.
    assert L.ranphy_mmse_llr(ctypes.byref(d), a, a, 0, a, None, None, a, 5, None) == -1
    assert L.ranphy_mmse_llr(ctypes.byref(d), a, a, 3, a, None, None, a, 0, None) == -1
    # 8-byte but not 16-byte aligned LLR buffer: the fused path needs 16-byte stores.
    assert L.ranphy_mmse_llr(ctypes.byref(d), a, a, 0, a, None, None, P(0x1008), 0, None) == -2
    # Off the matrix-core shapes: two DMRS occasions, or four layers.
    d2 = _desc(n_rx=16, n_layers=8, dmrs_comb=4, dmrs_td=2, dmrs_sym0=(2, 10))
    assert L.ranphy_mmse_llr(ctypes.byref(d2), a, a, 0, a, None, None, a, 0, None) == -2
    d3 = _desc(n_rx=16, n_layers=4)
    assert L.ranphy_mmse_llr(ctypes.byref(d3), a, a, 0, a, a, a, a, 1, None) == -2
    # the refined 16-bit modes (3, 4) are matrix-core modes too
    for prec in (3, 4):
        assert L.ranphy_mmse_llr(ctypes.byref(d3), a, a, 0, a, a, a, a, prec, None) == -2
        assert L.ranphy_mmse_detect_prec(ctypes.byref(d3), a, a, 0, a, a, a, prec, None) == -2


def test_batch_plan_validation(L):
    P = ctypes.c_void_p

    def ue(**kw):
        u = ranphy.UeRec()
        a = dict(GOOD, n_slots=1)
        a.update(kw)
        u.desc = ranphy.SlotDesc.make(**a)
        u.rx = u.pilots = u.noise_var = u.llr = 0x1000
        return u

    arr = (ranphy.UeRec * 2)(ue(), ue(qm=6))
    n = L.ranphy_batch_plan_bytes(arr, 2, 256)
    assert n > 256
    # a plan smaller than needed, or misaligned, is refused before any copy
    assert L.ranphy_batch_plan(arr, 2, 256, P(0x10000), n - 1) == -1
    assert L.ranphy_batch_plan(arr, 2, 256, P(0x10010), n) == -1
    assert L.ranphy_batch_plan_bytes(arr, 0, 256) == -1
    assert L.ranphy_batch_plan_bytes(arr, 2, 0) == -1
    bad = (ranphy.UeRec * 1)(ue(n_slots=2))
    assert L.ranphy_batch_plan_bytes(bad, 1, 256) == -1
    bad = (ranphy.UeRec * 1)(ue(n_rx=16, n_layers=9, dmrs_comb=8, dmrs_td=2))
    assert L.ranphy_batch_plan_bytes(bad, 1, 256) == -2  # more than 8 layers
    u = ue()
    u.rx = 0x1004
    bad = (ranphy.UeRec * 1)(u)
    assert L.ranphy_batch_plan_bytes(bad, 1, 256) == -1
    assert L.ranphy_batch_run(None, 4, None) == -1
    assert L.ranphy_batch_run(P(0x10000), 0, None) == -1


def test_bfp_sizes_and_validation(L):
    P = ctypes.c_void_p
    import oracle.bfp_ref as bref
    for nr, nl in ((1, 1), (2, 2), (4, 4), (8, 4), (12, 4), (16, 8), (32, 8), (64, 16)):
        kw = dict(n_rx=nr, n_layers=min(nl, nr), dmrs_comb=8 if nl > 8 else 4,
                  dmrs_td=2 if nl > 4 else 1)
        d = _desc(**kw)
        b = bref.block_size(nr)
        n_re = GOOD["n_slots"] * 14 * 12 * GOOD["n_prb"]
        assert L.ranphy_bfp_words(ctypes.byref(d)) == n_re * (nr // b) * bref.words_per_block(b)
    for nr in (17, 20, 40):  # neither below 16 nor a multiple of 16
        d = _desc(n_rx=nr)
        assert L.ranphy_bfp_words(ctypes.byref(d)) == -2
        assert L.ranphy_bfp_compress(ctypes.byref(d), P(8), P(8), None) == -2
        assert L.ranphy_bfp_decompress(ctypes.byref(d), P(8), P(8), None) == -2
    d = _desc()
    assert L.ranphy_bfp_words(None) == -1
    assert L.ranphy_bfp_compress(None, P(8), P(8), None) == -1
    assert L.ranphy_bfp_compress(ctypes.byref(d), P(0x1004), P(8), None) == -1  # rx
    assert L.ranphy_bfp_compress(ctypes.byref(d), P(8), P(0x1002), None) == -1  # packed
    assert L.ranphy_bfp_decompress(ctypes.byref(d), P(0), P(8), None) == -1
    assert L.ranphy_bfp_decompress(ctypes.byref(d), P(8), P(0x1004), None) == -1
    d0 = _desc(n_slots=0)
    assert L.ranphy_bfp_words(ctypes.byref(d0)) == 0
    assert L.ranphy_bfp_compress(ctypes.byref(d0), P(0), P(0), None) == 0
    assert L.ranphy_bfp_decompress(ctypes.byref(d0), P(0), P(0), None) == 0


def test_cnn_validation(L):
    P = ctypes.c_void_p
    L.ranphy_cnn_workspace_bytes.restype = ctypes.c_int64
    fwd = L.ranphy_cnn_forward
    fwd.argtypes = [P, P, P, ctypes.c_float, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                    ctypes.c_int, P, ctypes.c_int64, P]
    ok = dict(rows=1, cols=410, n_img=1024, n_groups=2)

    def call(ws=0x10000, wsb=1 << 40, nv=None, gate=0.0, **kw):
        a = dict(ok, **kw)
        return fwd(P(0x1000), P(0x1000), P(nv), gate, P(0x1000), a["rows"], a["cols"],
                   a["n_img"], a["n_groups"], P(ws), wsb, None)

    # sizes: one-row inference needs far less than the layered form (two activation tensors)
    one = L.ranphy_cnn_workspace_bytes(1, 410, 1024, 2, 0)
    two = L.ranphy_cnn_workspace_bytes(2, 205, 1024, 2, 0)
    train = L.ranphy_cnn_workspace_bytes(1, 410, 1024, 2, 1)
    assert 0 < one < two < train
    assert one >= 2 * 410 * 1024 * 4  # the BF16 input copy
    assert L.ranphy_cnn_workspace_bytes(0, 410, 1024, 2, 0) == -1
    # limits and validation happen before any launch
    assert call(cols=1 << 15, n_img=1 << 16) == -2   # 2^31 pixel-images per group
    assert call(cols=(1 << 20) + 1, n_img=1) == -2
    assert call(n_img=0) == -1
    assert call(ws=0) == -1
    assert call(ws=0x10010) == -1                      # workspace not 256-byte aligned
    assert call(wsb=one - 1) == -1                     # workspace too small
    wz = L.ranphy_cnn_workspace_bytes(1, 410, 1024, 0, 0)  # the packed weights alone
    assert call(n_groups=0, wsb=wz - 1) == -1
    assert call(n_groups=0, wsb=wz) == 0                # no groups: a no-op
    assert call(gate=-1.0) == -1


def test_fused_bfp_validation(L):
    P = ctypes.c_void_p
    d = _desc(n_rx=20, n_layers=4)  # no block width for 20 antennas
    assert L.ranphy_chest_ls_bfp(ctypes.byref(d), P(8), P(8), P(8), 0, None) == -2
    d = _desc()  # 8 x 4: estimator yes, matrix-core detector no
    assert L.ranphy_chest_ls_bfp(ctypes.byref(d), P(0), P(8), P(8), 0, None) == -1
    assert L.ranphy_chest_ls_bfp(ctypes.byref(d), P(0x1002), P(8), P(8), 0, None) == -1
    assert L.ranphy_chest_ls_bfp(ctypes.byref(d), P(8), P(8), P(8), 2, None) == -1
    assert L.ranphy_mmse_llr_bfp(ctypes.byref(d), P(16), P(16), 0, P(16), None, None, P(16), 0,
                                 None) == -2
    m = _desc(n_rx=64, n_layers=16, dmrs_comb=8, dmrs_td=2, qm=6)
    assert L.ranphy_mmse_llr_bfp(ctypes.byref(m), P(0x1004), P(16), 0, P(16), None, None, P(16),
                                 0, None) == -1  # words not 8-byte aligned
    assert L.ranphy_mmse_llr_bfp(ctypes.byref(m), P(16), P(16), 0, P(16), P(16), None, P(16), 0,
                                 None) == -1  # x without nv
    assert L.ranphy_mmse_llr_bfp(ctypes.byref(m), P(16), P(16), 0, P(16), None, None, P(16), 5,
                                 None) == -1  # precision
    assert L.ranphy_mmse_llr_bfp(ctypes.byref(m), P(16), P(0x1008), 0, P(16), None, None, P(16),
                                 0, None) == -2  # channel not 16-byte aligned: not the MFMA form
    m0 = _desc(n_rx=64, n_layers=16, dmrs_comb=8, dmrs_td=2, qm=6, n_slots=0)
    assert L.ranphy_mmse_llr_bfp(ctypes.byref(m0), P(0), P(0), 0, P(0), None, None, P(0), 0,
                                 None) == 0
    assert L.ranphy_chest_ls_bfp(ctypes.byref(m0), P(0), P(0), P(0), 0, None) == 0
    # the one-launch chain: up to 8 layers, antenna counts with a block width
    assert L.ranphy_receive_bfp(ctypes.byref(d), P(0x1002), P(8), P(8), P(8), None) == -1
    assert L.ranphy_receive_bfp(ctypes.byref(d), P(8), P(8), P(8), P(0x1004), None) == -1
    assert L.ranphy_receive_bfp(ctypes.byref(_desc(n_rx=20, n_layers=4)), P(8), P(8), P(8), P(8),
                                None) == -2
    assert L.ranphy_receive_bfp(ctypes.byref(m), P(8), P(8), P(8), P(8), None) == -2  # 16 layers
    assert L.ranphy_receive_bfp(ctypes.byref(_desc(n_slots=0)), P(0), P(0), P(0), P(0), None) == 0


def test_cnn_denoise_noalloc_validation(L):
    # The no-allocation refinement validates everything, and rejects slots whose workspace
    # exceeds the library's own array, before it looks up that array or touches the GPU.
    P = ctypes.c_void_p
    f = L.ranphy_cnn_denoise_noalloc
    f.argtypes = [ctypes.POINTER(ranphy.SlotDesc), P, P, ctypes.c_float, P, P, P]
    f.restype = ctypes.c_int
    L.ranphy_cnn_workspace_bytes.restype = ctypes.c_int64
    limit = 32 << 20  # RANPHY_NOALLOC_SCRATCH_BYTES
    # 64 x 16 at 273 PRB, comb 8 x 2 symbols: one slot is a one-row grid of 410 x 1024 images
    m = _desc(n_prb=273, n_rx=64, n_layers=16, qm=6, dmrs_comb=8, dmrs_td=2, dmrs_sym0=(2,),
              n_slots=140)
    assert L.ranphy_cnn_workspace_bytes(1, 410, 1024, 1, 0) <= limit
    # the same with two occasions keeps every layer's activations: far beyond the array
    big = _desc(n_prb=273, n_rx=64, n_layers=16, qm=6, dmrs_comb=8, dmrs_td=2,
                dmrs_sym0=(2, 9), n_slots=1)
    assert L.ranphy_cnn_workspace_bytes(2, 410, 1024, 1, 0) > limit
    assert f(ctypes.byref(big), P(0x1000), None, 0.0, P(0x1000), P(0x1000), None) == -2
    assert f(ctypes.byref(m), None, None, 0.0, P(0x1000), P(0x1000), None) == -1
    assert f(ctypes.byref(m), P(0x1000), None, 0.0, P(0x1004), P(0x1000), None) == -1
    assert f(ctypes.byref(m), P(0x1000), P(0x1002), 0.0, P(0x1000), P(0x1000), None) == -1
    assert f(ctypes.byref(m), P(0x1000), None, -1.0, P(0x1000), P(0x1000), None) == -1
    assert f(None, P(0x1000), None, 0.0, P(0x1000), P(0x1000), None) == -1
    empty = _desc(n_prb=273, n_rx=64, n_layers=16, qm=6, dmrs_comb=8, dmrs_td=2,
                  dmrs_sym0=(2,), n_slots=0)
    assert f(ctypes.byref(empty), P(0x1000), None, 0.0, P(0x1000), P(0x1000), None) == 0
