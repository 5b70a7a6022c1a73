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
PREC_FP32, PREC_FP16, PREC_BF16 = 0, 1, 2
OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_LAUNCH = 0, -1, -2, -3
BUF_RX, BUF_PILOTS, BUF_H, BUF_NOISE_VAR, BUF_X, BUF_NV, BUF_LLR = range(7)

EXPORTED_SYMBOLS = (
    "ranphy_abi_version", "ranphy_status_str", "ranphy_buffer_floats",
    "ranphy_chest_ls", "ranphy_mmse_detect", "ranphy_mmse_detect_prec", "ranphy_mmse_llr",
    "ranphy_llr_demap",
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
                "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
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
        for f in ("ranphy_chest_ls", "ranphy_mmse_detect", "ranphy_mmse_detect_prec",
                  "ranphy_mmse_llr", "ranphy_llr_demap"):
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
    (PREC_FP32, PREC_FP16, PREC_BF16); the 16-bit modes need the matrix-core shapes."""
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
