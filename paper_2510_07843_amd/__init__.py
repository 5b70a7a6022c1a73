"""Python binding of libranphy (MI355X uplink receive hot path).

Argument marshalling only: tensors are checked for device, dtype, contiguity and size, their
device pointers and the current HIP stream are handed to the C ABI (include/ranphy.h), and
every step of the computation runs in the library's HIP kernels.  PyTorch provides device
memory and streams.  There is no fallback: if ``libranphy.so`` has not been built, or the
tensors are not on a GPU, the calls raise.

    import paper_2510_07843_amd as ranphy
    h  = ranphy.chest_ls(shape, rx, pilots)                 # pilot resolution
    x, nv = ranphy.mmse_detect(shape, rx, h, noise_var)
    llr = ranphy.llr_demap(shape, x, nv)

``shape`` is any object with the descriptor fields (n_prb, n_symb, n_rx, n_layers, qm,
dmrs_comb, dmrs_td, dmrs_sym0, n_slots), or a :class:`SlotDesc`.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libranphy.so")

H_PILOT, H_FULL = 0, 1
PREC_FP32, PREC_FP16, PREC_BF16, PREC_FP16_REFINED, PREC_BF16_REFINED = 0, 1, 2, 3, 4
OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_LAUNCH = 0, -1, -2, -3
BUF_RX, BUF_PILOTS, BUF_H, BUF_NOISE_VAR, BUF_X, BUF_NV, BUF_LLR = range(7)

EXPORTED_SYMBOLS = (
    "ranphy_abi_version", "ranphy_status_str", "ranphy_buffer_floats",
    "ranphy_chest_ls", "ranphy_mmse_detect", "ranphy_mmse_detect_prec", "ranphy_mmse_llr",
    "ranphy_llr_demap", "ranphy_cnn_param_count", "ranphy_cnn_workspace_bytes",
    "ranphy_cnn_forward", "ranphy_cnn_grad", "ranphy_cnn_adam", "ranphy_cnn_denoise",
    "ranphy_cnn_denoise_noalloc",
    "ranphy_batch_plan_bytes", "ranphy_batch_plan", "ranphy_batch_run", "ranphy_receive",
    "ranphy_bfp_words", "ranphy_bfp_compress", "ranphy_bfp_decompress", "ranphy_chest_ls_bfp",
    "ranphy_mmse_llr_bfp", "ranphy_receive_bfp",
)


class SlotDesc(ctypes.Structure):
    """Mirror of ``ranphy_slot_desc``."""

    _fields_ = [
        ("n_prb", ctypes.c_int32), ("n_symb", ctypes.c_int32), ("n_rx", ctypes.c_int32),
        ("n_layers", ctypes.c_int32), ("qm", ctypes.c_int32), ("dmrs_comb", ctypes.c_int32),
        ("dmrs_td", ctypes.c_int32), ("n_occ", ctypes.c_int32),
        ("dmrs_sym0", ctypes.c_int32 * 4), ("n_slots", ctypes.c_int32),
    ]

    @classmethod
    def make(cls, n_prb: int, n_symb: int, n_rx: int, n_layers: int, qm: int, dmrs_comb: int,
             dmrs_td: int, dmrs_sym0: Sequence[int], n_slots: int) -> "SlotDesc":
        d = cls()
        d.n_prb, d.n_symb, d.n_rx, d.n_layers, d.qm = n_prb, n_symb, n_rx, n_layers, qm
        d.dmrs_comb, d.dmrs_td, d.n_occ = dmrs_comb, dmrs_td, len(dmrs_sym0)
        for i, s in enumerate(list(dmrs_sym0)[:4]):
            d.dmrs_sym0[i] = s
        d.n_slots = n_slots
        return d


class UeRec(ctypes.Structure):
    """Mirror of ``ranphy_ue``."""

    _fields_ = [("desc", SlotDesc), ("rx", ctypes.c_void_p), ("pilots", ctypes.c_void_p),
                ("noise_var", ctypes.c_void_p), ("llr", ctypes.c_void_p)]


def desc_of(shape) -> SlotDesc:
    if isinstance(shape, SlotDesc):
        return shape
    return SlotDesc.make(shape.n_prb, shape.n_symb, shape.n_rx, shape.n_layers, shape.qm,
                         shape.dmrs_comb, shape.dmrs_td, tuple(shape.dmrs_sym0), shape.n_slots)


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python paper_2510_07843_amd/build.py` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        D = ctypes.POINTER(SlotDesc)
        P = ctypes.c_void_p
        L.ranphy_abi_version.restype = ctypes.c_int
        L.ranphy_status_str.argtypes = [ctypes.c_int]
        L.ranphy_status_str.restype = ctypes.c_char_p
        L.ranphy_buffer_floats.argtypes = [D, ctypes.c_int, ctypes.c_int]
        L.ranphy_buffer_floats.restype = ctypes.c_int64
        L.ranphy_chest_ls.argtypes = [D, P, P, P, ctypes.c_int, P]
        L.ranphy_mmse_detect.argtypes = [D, P, P, ctypes.c_int, P, P, P, P]
        L.ranphy_mmse_detect_prec.argtypes = [D, P, P, ctypes.c_int, P, P, P, ctypes.c_int, P]
        L.ranphy_mmse_llr.argtypes = [D, P, P, ctypes.c_int, P, P, P, P, ctypes.c_int, P]
        L.ranphy_llr_demap.argtypes = [D, P, P, P, P]
        I, I64 = ctypes.c_int, ctypes.c_int64
        L.ranphy_cnn_param_count.restype = I64
        L.ranphy_cnn_workspace_bytes.argtypes = [I, I, I, I, I]
        L.ranphy_cnn_workspace_bytes.restype = I64
        L.ranphy_cnn_forward.argtypes = [P, P, P, ctypes.c_float, P, I, I, I, I, P, I64, P]
        L.ranphy_cnn_grad.argtypes = [P, P, P, P, P, P, I, I, I, I, P, I64, P]
        L.ranphy_cnn_adam.argtypes = [P, P, P, P, I, ctypes.c_float, P]
        L.ranphy_cnn_denoise.argtypes = [D, P, P, ctypes.c_float, P, P, P, I64, P]
        L.ranphy_cnn_denoise_noalloc.argtypes = [D, P, P, ctypes.c_float, P, P, P]
        UE = ctypes.POINTER(UeRec)
        L.ranphy_batch_plan_bytes.argtypes = [UE, I, I]
        L.ranphy_batch_plan_bytes.restype = I64
        L.ranphy_batch_plan.argtypes = [UE, I, I, P, I64]
        L.ranphy_batch_run.argtypes = [P, I, P]
        L.ranphy_receive.argtypes = [D, P, P, P, P, P]
        L.ranphy_bfp_words.argtypes = [D]
        L.ranphy_bfp_words.restype = I64
        L.ranphy_bfp_compress.argtypes = [D, P, P, P]
        L.ranphy_bfp_decompress.argtypes = [D, P, P, P]
        L.ranphy_chest_ls_bfp.argtypes = [D, P, P, P, ctypes.c_int, P]
        L.ranphy_mmse_llr_bfp.argtypes = [D, P, P, ctypes.c_int, P, P, P, P, ctypes.c_int, P]
        L.ranphy_receive_bfp.argtypes = [D, P, P, P, P, P]
        for f in ("ranphy_chest_ls", "ranphy_mmse_detect", "ranphy_mmse_detect_prec",
                  "ranphy_mmse_llr", "ranphy_llr_demap", "ranphy_cnn_forward", "ranphy_cnn_grad",
                  "ranphy_cnn_adam", "ranphy_cnn_denoise", "ranphy_cnn_denoise_noalloc",
                  "ranphy_batch_plan",
                  "ranphy_batch_run", "ranphy_receive", "ranphy_bfp_compress",
                  "ranphy_bfp_decompress", "ranphy_chest_ls_bfp", "ranphy_mmse_llr_bfp",
                  "ranphy_receive_bfp"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def abi_version() -> int:
    return lib().ranphy_abi_version()


def status_str(status: int) -> str:
    return lib().ranphy_status_str(status).decode()


def buffer_floats(shape, buf: int, h_res: int = H_PILOT) -> int:
    d = desc_of(shape)
    n = lib().ranphy_buffer_floats(ctypes.byref(d), buf, h_res)
    if n < 0:
        raise ValueError(f"invalid descriptor: {status_str(int(n))}")
    return int(n)


class RanphyError(RuntimeError):
    def __init__(self, where: str, status: int):
        super().__init__(f"{where}: {status_str(status)} ({status})")
        self.status = status


def _check(where: str, status: int):
    if status != OK:
        raise RanphyError(where, status)


def _as_dev(t: torch.Tensor, name: str, want: torch.dtype, n_floats: int) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be a GPU tensor (got {t.device})")
    if t.dtype != want:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    per = 2 if want == torch.complex64 else 1
    if t.numel() * per != n_floats:
        raise ValueError(f"{name}: {t.numel() * per} floats, expected {n_floats}")
    return t.data_ptr()


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def chest_ls(shape, rx: torch.Tensor, pilots: torch.Tensor, h: Optional[torch.Tensor] = None,
             h_res: int = H_PILOT, stream=None) -> torch.Tensor:
    """LS channel estimate at the pilots (``H_PILOT``) or interpolated (``H_FULL``)."""
    d = desc_of(shape)
    nh = buffer_floats(d, BUF_H, h_res)
    if h is None:
        h = torch.empty(nh // 2, dtype=torch.complex64, device=rx.device)
    args = (_as_dev(rx, "rx", torch.complex64, buffer_floats(d, BUF_RX)),
            _as_dev(pilots, "pilots", torch.complex64, buffer_floats(d, BUF_PILOTS)),
            _as_dev(h, "h", torch.complex64, nh))
    _check("ranphy_chest_ls", lib().ranphy_chest_ls(ctypes.byref(d), *args, h_res, _stream(stream)))
    return h


def mmse_detect(shape, rx: torch.Tensor, h: torch.Tensor, noise_var: torch.Tensor,
                h_res: int = H_PILOT, x: Optional[torch.Tensor] = None,
                nv: Optional[torch.Tensor] = None, stream=None,
                precision: int = PREC_FP32) -> Tuple[torch.Tensor, torch.Tensor]:
    """Unbiased LMMSE symbols and post-equalisation variances, [slot][dsym][sc][layer].

    ``precision`` selects the input precision of the Gram and matched-filter products
    (PREC_FP32, PREC_FP16, PREC_BF16, and the refined PREC_FP16_REFINED, PREC_BF16_REFINED);
    the 16-bit modes need the matrix-core shapes."""
    d = desc_of(shape)
    nx = buffer_floats(d, BUF_X)
    if x is None:
        x = torch.empty(nx // 2, dtype=torch.complex64, device=rx.device)
    if nv is None:
        nv = torch.empty(buffer_floats(d, BUF_NV), dtype=torch.float32, device=rx.device)
    args = (_as_dev(rx, "rx", torch.complex64, buffer_floats(d, BUF_RX)),
            _as_dev(h, "h", torch.complex64, buffer_floats(d, BUF_H, h_res)))
    pn = _as_dev(noise_var, "noise_var", torch.float32, buffer_floats(d, BUF_NOISE_VAR))
    px = _as_dev(x, "x", torch.complex64, nx)
    pv = _as_dev(nv, "nv", torch.float32, buffer_floats(d, BUF_NV))
    if precision == PREC_FP32:
        st = lib().ranphy_mmse_detect(ctypes.byref(d), *args, h_res, pn, px, pv, _stream(stream))
    else:
        st = lib().ranphy_mmse_detect_prec(ctypes.byref(d), *args, h_res, pn, px, pv, precision,
                                           _stream(stream))
    _check("ranphy_mmse_detect", st)
    return x, nv


def mmse_llr(shape, rx: torch.Tensor, h: torch.Tensor, noise_var: torch.Tensor,
             h_res: int = H_PILOT, llr: Optional[torch.Tensor] = None,
             x: Optional[torch.Tensor] = None, nv: Optional[torch.Tensor] = None,
             precision: int = PREC_FP32, stream=None) -> torch.Tensor:
    """Detection and max-log demapping in one pass; returns the LLRs.  ``x`` and ``nv``
    (both or neither) also receive the equalised symbols and variances."""
    d = desc_of(shape)
    nl = buffer_floats(d, BUF_LLR)
    if llr is None:
        llr = torch.empty(nl, dtype=torch.float32, device=rx.device)
    if (x is None) != (nv is None):
        raise ValueError("x and nv are given together or not at all")
    args = (_as_dev(rx, "rx", torch.complex64, buffer_floats(d, BUF_RX)),
            _as_dev(h, "h", torch.complex64, buffer_floats(d, BUF_H, h_res)))
    pn = _as_dev(noise_var, "noise_var", torch.float32, buffer_floats(d, BUF_NOISE_VAR))
    px = None if x is None else _as_dev(x, "x", torch.complex64, buffer_floats(d, BUF_X))
    pv = None if nv is None else _as_dev(nv, "nv", torch.float32, buffer_floats(d, BUF_NV))
    pl = _as_dev(llr, "llr", torch.float32, nl)
    _check("ranphy_mmse_llr", lib().ranphy_mmse_llr(ctypes.byref(d), *args, h_res, pn, px, pv, pl,
                                                    precision, _stream(stream)))
    return llr


def receive(shape, rx: torch.Tensor, pilots: torch.Tensor, noise_var: torch.Tensor,
            llr: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The whole chain (LS estimate, interpolation, detection, demapping) in one launch, up to
    8 layers; returns the LLRs [slot][dsym][sc][layer][qm]."""
    d = desc_of(shape)
    nl = buffer_floats(d, BUF_LLR)
    if llr is None:
        llr = torch.empty(nl, dtype=torch.float32, device=rx.device)
    _check("ranphy_receive", lib().ranphy_receive(
        ctypes.byref(d), _as_dev(rx, "rx", torch.complex64, buffer_floats(d, BUF_RX)),
        _as_dev(pilots, "pilots", torch.complex64, buffer_floats(d, BUF_PILOTS)),
        _as_dev(noise_var, "noise_var", torch.float32, buffer_floats(d, BUF_NOISE_VAR)),
        _as_dev(llr, "llr", torch.float32, nl), _stream(stream)))
    return llr


def bfp_words(shape) -> int:
    """32-bit words of the block floating point form of the received grid of `shape`."""
    n = int(lib().ranphy_bfp_words(ctypes.byref(desc_of(shape))))
    if n < 0:
        raise RanphyError("ranphy_bfp_words", n)
    return n


def bfp_compress(shape, rx: torch.Tensor, packed: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
    """Block floating point form (int32 words holding the unsigned bit patterns) of the
    received grid rx [slot][symb][sc][rx] complex64."""
    d = desc_of(shape)
    nw = bfp_words(shape)
    if packed is None:
        packed = torch.empty(nw, dtype=torch.int32, device=rx.device)
    _check("ranphy_bfp_compress", lib().ranphy_bfp_compress(
        ctypes.byref(d), _as_dev(rx, "rx", torch.complex64, buffer_floats(d, BUF_RX)),
        _as_dev(packed, "packed", torch.int32, nw), _stream(stream)))
    return packed


def bfp_decompress(shape, packed: torch.Tensor, rx: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """The received grid [slot][symb][sc][rx] complex64 from its block floating point form."""
    d = desc_of(shape)
    nr = buffer_floats(d, BUF_RX)
    if rx is None:
        rx = torch.empty(nr // 2, dtype=torch.complex64, device=packed.device)
    _check("ranphy_bfp_decompress", lib().ranphy_bfp_decompress(
        ctypes.byref(d), _as_dev(packed, "packed", torch.int32, bfp_words(shape)),
        _as_dev(rx, "rx", torch.complex64, nr), _stream(stream)))
    return rx


def chest_ls_bfp(shape, packed: torch.Tensor, pilots: torch.Tensor,
                 h: Optional[torch.Tensor] = None, h_res: int = H_PILOT,
                 stream=None) -> torch.Tensor:
    """chest_ls reading the received grid in block floating point form (bfp_compress)."""
    d = desc_of(shape)
    nh = buffer_floats(d, BUF_H, h_res)
    if h is None:
        h = torch.empty(nh // 2, dtype=torch.complex64, device=packed.device)
    args = (_as_dev(packed, "packed", torch.int32, bfp_words(shape)),
            _as_dev(pilots, "pilots", torch.complex64, buffer_floats(d, BUF_PILOTS)),
            _as_dev(h, "h", torch.complex64, nh))
    _check("ranphy_chest_ls_bfp",
           lib().ranphy_chest_ls_bfp(ctypes.byref(d), *args, h_res, _stream(stream)))
    return h


def mmse_llr_bfp(shape, packed: torch.Tensor, h: torch.Tensor, noise_var: torch.Tensor,
                 h_res: int = H_PILOT, llr: Optional[torch.Tensor] = None,
                 x: Optional[torch.Tensor] = None, nv: Optional[torch.Tensor] = None,
                 precision: int = PREC_FP32, stream=None) -> torch.Tensor:
    """mmse_llr reading the received grid in block floating point form, decoded in the
    detector's load; returns the LLRs."""
    d = desc_of(shape)
    nl = buffer_floats(d, BUF_LLR)
    if llr is None:
        llr = torch.empty(nl, dtype=torch.float32, device=packed.device)
    if (x is None) != (nv is None):
        raise ValueError("x and nv are given together or not at all")
    args = (_as_dev(packed, "packed", torch.int32, bfp_words(shape)),
            _as_dev(h, "h", torch.complex64, buffer_floats(d, BUF_H, h_res)))
    pn = _as_dev(noise_var, "noise_var", torch.float32, buffer_floats(d, BUF_NOISE_VAR))
    px = None if x is None else _as_dev(x, "x", torch.complex64, buffer_floats(d, BUF_X))
    pv = None if nv is None else _as_dev(nv, "nv", torch.float32, buffer_floats(d, BUF_NV))
    pl = _as_dev(llr, "llr", torch.float32, nl)
    _check("ranphy_mmse_llr_bfp", lib().ranphy_mmse_llr_bfp(
        ctypes.byref(d), *args, h_res, pn, px, pv, pl, precision, _stream(stream)))
    return llr


def receive_bfp(shape, packed: torch.Tensor, pilots: torch.Tensor, noise_var: torch.Tensor,
                llr: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """receive with the received grid in block floating point form, decoded in the loads."""
    d = desc_of(shape)
    nl = buffer_floats(d, BUF_LLR)
    if llr is None:
        llr = torch.empty(nl, dtype=torch.float32, device=packed.device)
    _check("ranphy_receive_bfp", lib().ranphy_receive_bfp(
        ctypes.byref(d), _as_dev(packed, "packed", torch.int32, bfp_words(shape)),
        _as_dev(pilots, "pilots", torch.complex64, buffer_floats(d, BUF_PILOTS)),
        _as_dev(noise_var, "noise_var", torch.float32, buffer_floats(d, BUF_NOISE_VAR)),
        _as_dev(llr, "llr", torch.float32, nl), _stream(stream)))
    return llr


def llr_demap(shape, x: torch.Tensor, nv: torch.Tensor, llr: Optional[torch.Tensor] = None,
              stream=None) -> torch.Tensor:
    """Max-log LLRs [slot][dsym][sc][layer][qm] (positive favours bit 0)."""
    d = desc_of(shape)
    nl = buffer_floats(d, BUF_LLR)
    if llr is None:
        llr = torch.empty(nl, dtype=torch.float32, device=x.device)
    args = (_as_dev(x, "x", torch.complex64, buffer_floats(d, BUF_X)),
            _as_dev(nv, "nv", torch.float32, buffer_floats(d, BUF_NV)),
            _as_dev(llr, "llr", torch.float32, nl))
    _check("ranphy_llr_demap", lib().ranphy_llr_demap(ctypes.byref(d), *args, _stream(stream)))
    return llr


# ---------------------------------------------------------------------------------------
# Learned refinement of the pilot-resolution channel estimate (include/ranphy.h).
# ---------------------------------------------------------------------------------------

def cnn_param_count() -> int:
    return int(lib().ranphy_cnn_param_count())


def cnn_workspace_bytes(rows: int, cols: int, n_img: int, n_groups: int, train: bool) -> int:
    n = int(lib().ranphy_cnn_workspace_bytes(rows, cols, n_img, n_groups, int(train)))
    if n < 0:
        raise ValueError(f"invalid denoiser dimensions: {status_str(n)}")
    return n


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _f32(t: torch.Tensor, name: str, n: int) -> int:
    return _as_dev(t, name, torch.float32, n)


def cnn_forward(params: torch.Tensor, x: torch.Tensor, rows: int, cols: int, n_img: int,
                n_groups: int, out: Optional[torch.Tensor] = None,
                workspace: Optional[torch.Tensor] = None, noise_var: Optional[torch.Tensor] = None,
                min_noise_var: float = 0.0, stream=None) -> torch.Tensor:
    """The network on x [group][rows * cols][image][2] float32 (flat); with per-group noise
    variances it refines noise-normalised estimates (out = x + sigma y) and groups below
    min_noise_var keep x."""
    n = n_groups * rows * cols * n_img * 2
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=x.device)
    nb = cnn_workspace_bytes(rows, cols, n_img, n_groups, False)
    ws = workspace if workspace is not None else _workspace(nb, x.device)
    pn = None if noise_var is None else _f32(noise_var, "noise_var", n_groups)
    _check("ranphy_cnn_forward", lib().ranphy_cnn_forward(
        _f32(params, "params", cnn_param_count()), _f32(x, "x", n), pn, float(min_noise_var),
        _f32(out, "out", n), rows, cols, n_img, n_groups, ws.data_ptr(), ws.numel(),
        _stream(stream)))
    return out


def cnn_grad(params: torch.Tensor, x: torch.Tensor, target: torch.Tensor, rows: int, cols: int,
             n_img: int, n_groups: int, grad: Optional[torch.Tensor] = None,
             loss: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
             noise_var: Optional[torch.Tensor] = None, stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """(loss, grad): the MSE loss of the network on x against target (in noise-normalised
    units when noise variances are given) and its parameter gradient."""
    n = n_groups * rows * cols * n_img * 2
    if grad is None:
        grad = torch.empty(cnn_param_count(), dtype=torch.float32, device=x.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    nb = cnn_workspace_bytes(rows, cols, n_img, n_groups, True)
    ws = workspace if workspace is not None else _workspace(nb, x.device)
    pn = None if noise_var is None else _f32(noise_var, "noise_var", n_groups)
    _check("ranphy_cnn_grad", lib().ranphy_cnn_grad(
        _f32(params, "params", cnn_param_count()), _f32(x, "x", n), _f32(target, "target", n),
        pn, _f32(grad, "grad", cnn_param_count()), _f32(loss, "loss", 1), rows, cols, n_img,
        n_groups, ws.data_ptr(), ws.numel(), _stream(stream)))
    return loss, grad


def cnn_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
             step: int, lr: float, stream=None) -> None:
    n = cnn_param_count()
    _check("ranphy_cnn_adam", lib().ranphy_cnn_adam(
        _f32(params, "params", n), _f32(grad, "grad", n), _f32(m, "m", n), _f32(v, "v", n),
        step, lr, _stream(stream)))


def cnn_denoise(shape, params: torch.Tensor, h: torch.Tensor,
                noise_var: Optional[torch.Tensor] = None, min_noise_var: float = 0.0,
                out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """The trained network applied to a pilot-resolution estimate (returns the refined one).
    Slots with noise_var below min_noise_var keep the plain estimate."""
    d = desc_of(shape)
    nh = buffer_floats(d, BUF_H, H_PILOT)
    if out is None:
        out = torch.empty(nh // 2, dtype=torch.complex64, device=h.device)
    if workspace is None:
        n_pilot = -(-shape.n_prb * 12 // shape.dmrs_comb)
        nb = cnn_workspace_bytes(len(shape.dmrs_sym0), n_pilot, shape.n_rx * shape.n_layers,
                                 max(1, min(shape.n_slots, 8)), False)
        workspace = _workspace(nb, h.device)
    pn = None if noise_var is None else _as_dev(noise_var, "noise_var", torch.float32,
                                                buffer_floats(d, BUF_NOISE_VAR))
    _check("ranphy_cnn_denoise", lib().ranphy_cnn_denoise(
        ctypes.byref(d), _f32(params, "params", cnn_param_count()), pn, float(min_noise_var),
        _as_dev(h, "h", torch.complex64, nh), _as_dev(out, "out", torch.complex64, nh),
        workspace.data_ptr(), workspace.numel(), _stream(stream)))
    return out


def cnn_denoise_noalloc(shape, params: torch.Tensor, h: torch.Tensor,
                        noise_var: Optional[torch.Tensor] = None, min_noise_var: float = 0.0,
                        out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """cnn_denoise on the library's own device workspace: the call allocates nothing (``out``
    must be given).  Calls that overlap on one GPU share that workspace and race."""
    d = desc_of(shape)
    nh = buffer_floats(d, BUF_H, H_PILOT)
    if out is None:
        raise ValueError("out is required: this call allocates nothing")
    pn = None if noise_var is None else _as_dev(noise_var, "noise_var", torch.float32,
                                                buffer_floats(d, BUF_NOISE_VAR))
    _check("ranphy_cnn_denoise_noalloc", lib().ranphy_cnn_denoise_noalloc(
        ctypes.byref(d), _f32(params, "params", cnn_param_count()), pn, float(min_noise_var),
        _as_dev(h, "h", torch.complex64, nh), _as_dev(out, "out", torch.complex64, nh),
        _stream(stream)))
    return out


# ---------------------------------------------------------------------------------------
# Many UEs in one persistent launch (include/ranphy.h).
# ---------------------------------------------------------------------------------------

class Batch:
    """A plan over UEs, each a dict with ``shape`` (one slot) and GPU tensors ``rx``,
    ``pilots``, ``noise_var`` (one value) and ``llr`` (allocated when missing).  The tensors
    are kept alive with the plan; their contents may change between runs."""

    def __init__(self, ues, tile_re: int = 512):
        self.ues = ues
        recs = (UeRec * len(ues))()
        for i, u in enumerate(ues):
            sh = u["shape"]
            d = desc_of(sh)
            if "llr" not in u or u["llr"] is None:
                u["llr"] = torch.empty(buffer_floats(d, BUF_LLR), dtype=torch.float32,
                                       device=u["rx"].device)
            recs[i].desc = d
            recs[i].rx = _as_dev(u["rx"], "rx", torch.complex64, buffer_floats(d, BUF_RX))
            recs[i].pilots = _as_dev(u["pilots"], "pilots", torch.complex64,
                                     buffer_floats(d, BUF_PILOTS))
            recs[i].noise_var = _as_dev(u["noise_var"], "noise_var", torch.float32, 1)
            recs[i].llr = _as_dev(u["llr"], "llr", torch.float32, buffer_floats(d, BUF_LLR))
        self._recs = recs
        self.tile_re = tile_re
        n = int(lib().ranphy_batch_plan_bytes(recs, len(ues), tile_re))
        if n < 0:
            raise RanphyError("ranphy_batch_plan_bytes", n)
        self.plan = torch.empty(n, dtype=torch.uint8, device=ues[0]["rx"].device)
        _check("ranphy_batch_plan", lib().ranphy_batch_plan(recs, len(ues), tile_re,
                                                            self.plan.data_ptr(), n))
        self.n_items = int(self.plan[4:8].cpu().view(torch.int32).item())

    def run(self, n_blocks: int, stream=None) -> None:
        _check("ranphy_batch_run", lib().ranphy_batch_run(self.plan.data_ptr(), n_blocks,
                                                          _stream(stream)))
