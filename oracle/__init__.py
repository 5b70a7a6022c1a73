"""ctypes wrapper of the FP64 CPU oracle (``libranphy_ref.so``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline
leg of the benchmark.  The product package never imports it and shares no code with it.

Inputs are numpy arrays on the host in the same layouts and dtypes the GPU library takes
(complex64 / float32); outputs are double precision.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libranphy_ref.so")
SRC_PATH = os.path.join(_HERE, "ranphy_ref.c")

H_PILOT, H_FULL = 0, 1
ROUTE_LU, ROUTE_RCOV = 0, 1


class RefDesc(ctypes.Structure):
    _fields_ = [
        ("n_prb", ctypes.c_int32), ("n_symb", ctypes.c_int32), ("n_rx", ctypes.c_int32),
        ("n_layers", ctypes.c_int32), ("qm", ctypes.c_int32), ("dmrs_comb", ctypes.c_int32),
        ("dmrs_td", ctypes.c_int32), ("n_occ", ctypes.c_int32),
        ("dmrs_sym0", ctypes.c_int32 * 4), ("n_slots", ctypes.c_int32),
    ]


SAN_LIB_PATH = os.path.join(_HERE, "libranphy_ref_san.so")
# Set to the sanitized library's path (with the sanitizer runtimes preloaded) to run the
# oracle's checks under AddressSanitizer and UndefinedBehaviorSanitizer.
LIB_ENV = "RANPHY_REF_LIB"


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall",
               "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def build_sanitized() -> str:
    """The same oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (every
    undefined-behaviour finding fatal), without OpenMP (one thread: the sanitizers then see
    one deterministic order of the loops).  Load it by setting RANPHY_REF_LIB to its path,
    with libasan and libubsan preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-o", SAN_LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(SAN_LIB_PATH + ".tmp", SAN_LIB_PATH)
    return SAN_LIB_PATH


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        path = os.environ.get(LIB_ENV) or LIB_PATH
        if path == LIB_PATH and (not os.path.exists(LIB_PATH) or
                                 os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        D = ctypes.POINTER(RefDesc)
        L.ranphy_ref_chest_ls.argtypes = [D, P, P, P, ctypes.c_int]
        L.ranphy_ref_mmse_detect.argtypes = [D, P, P, ctypes.c_int, P, P, P, ctypes.c_int]
        L.ranphy_ref_llr_demap.argtypes = [D, P, P, P]
        L.ranphy_ref_channel_at.argtypes = [D, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, P]
        L.ranphy_ref_gram.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_double, P]
        L.ranphy_ref_mmse_batch.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P, P,
                                            ctypes.c_int, P, P, P]
        L.ranphy_ref_llr_batch.argtypes = [ctypes.c_int64, ctypes.c_int, P, P, P]
        L.ranphy_ref_qam_points.argtypes = [ctypes.c_int, P]
        L.ranphy_ref_set_threads.argtypes = [ctypes.c_int]
        L.ranphy_ref_set_threads.restype = None
        _lib = L
    return _lib


def desc(shape) -> RefDesc:
    """Build the oracle's descriptor from an object with the slot-shape fields."""
    d = RefDesc()
    d.n_prb, d.n_symb, d.n_rx = shape.n_prb, shape.n_symb, shape.n_rx
    d.n_layers, d.qm = shape.n_layers, shape.qm
    d.dmrs_comb, d.dmrs_td = shape.dmrs_comb, shape.dmrs_td
    d.n_occ = len(shape.dmrs_sym0)
    for i, s in enumerate(shape.dmrs_sym0):
        d.dmrs_sym0[i] = s
    d.n_slots = shape.n_slots
    return d


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} returned {rc}")


def chest_ls(shape, rx: np.ndarray, pilots: np.ndarray, h_res: int = H_PILOT) -> np.ndarray:
    """LS channel estimate; complex128 [slot][occ][j or sc][rx][layer]."""
    rx = np.ascontiguousarray(rx, np.complex64)
    pilots = np.ascontiguousarray(pilots, np.complex64)
    K = shape.n_pilot if h_res == H_PILOT else shape.n_sc
    h = np.zeros((shape.n_slots, len(shape.dmrs_sym0), K, shape.n_rx, shape.n_layers), np.complex128)
    d = desc(shape)
    _check(lib().ranphy_ref_chest_ls(ctypes.byref(d), _ptr(rx), _ptr(pilots), _ptr(h), h_res), "chest_ls")
    return h


def mmse_detect(shape, rx: np.ndarray, h: np.ndarray, h_res: int, noise_var: np.ndarray,
                route: int = ROUTE_LU):
    """Unbiased MMSE; returns (x~ complex128, nu2 float64), each [slot][dsym][sc][layer]."""
    rx = np.ascontiguousarray(rx, np.complex64)
    h = np.ascontiguousarray(h, np.complex64)
    nvar = np.ascontiguousarray(noise_var, np.float32)
    out_shape = (shape.n_slots, shape.n_dsym, shape.n_sc, shape.n_layers)
    x = np.zeros(out_shape, np.complex128)
    nv = np.zeros(out_shape, np.float64)
    d = desc(shape)
    _check(lib().ranphy_ref_mmse_detect(ctypes.byref(d), _ptr(rx), _ptr(h), h_res, _ptr(nvar),
                                        _ptr(x), _ptr(nv), route), "mmse_detect")
    return x, nv


def llr_demap(shape, x: np.ndarray, nv: np.ndarray) -> np.ndarray:
    """Brute-force max-log LLRs (float64) [slot][dsym][sc][layer][qm]."""
    x = np.ascontiguousarray(x, np.complex64)
    nv = np.ascontiguousarray(nv, np.float32)
    llr = np.zeros(x.shape + (shape.qm,), np.float64)
    d = desc(shape)
    _check(lib().ranphy_ref_llr_demap(ctypes.byref(d), _ptr(x), _ptr(nv), _ptr(llr)), "llr_demap")
    return llr


def channel_at(shape, h: np.ndarray, h_res: int, slot: int, sc: int, symb: int) -> np.ndarray:
    h = np.ascontiguousarray(h, np.complex64)
    H = np.zeros((shape.n_rx, shape.n_layers), np.complex128)
    d = desc(shape)
    _check(lib().ranphy_ref_channel_at(ctypes.byref(d), _ptr(h), h_res, slot, sc, symb, _ptr(H)),
           "channel_at")
    return H


def gram(H: np.ndarray, s2: float) -> np.ndarray:
    H = np.ascontiguousarray(H, np.complex128)
    nr, nl = H.shape
    G = np.zeros((nl, nl), np.complex128)
    _check(lib().ranphy_ref_gram(nr, nl, _ptr(H), float(s2), _ptr(G)), "gram")
    return G


def mmse_batch(H: np.ndarray, y: np.ndarray, s2, route: int = ROUTE_LU):
    """H [n][nr][nl], y [n][nr] complex128; s2 scalar or [n].  Returns (x~, nu2, mu)."""
    H = np.ascontiguousarray(H, np.complex128)
    y = np.ascontiguousarray(y, np.complex128)
    n, nr, nl = H.shape
    s2a = np.ascontiguousarray(np.broadcast_to(np.asarray(s2, np.float64), (n,)))
    xt = np.zeros((n, nl), np.complex128)
    nv = np.zeros((n, nl), np.float64)
    mu = np.zeros((n, nl), np.float64)
    _check(lib().ranphy_ref_mmse_batch(n, nr, nl, _ptr(H), _ptr(y), _ptr(s2a), route, _ptr(xt),
                                       _ptr(nv), _ptr(mu)), "mmse_batch")
    return xt, nv, mu


def llr_batch(x: np.ndarray, nv, qm: int) -> np.ndarray:
    x = np.ascontiguousarray(x, np.complex128).reshape(-1)
    nva = np.ascontiguousarray(np.broadcast_to(np.asarray(nv, np.float64), x.shape))
    llr = np.zeros((x.size, qm), np.float64)
    _check(lib().ranphy_ref_llr_batch(x.size, qm, _ptr(x), _ptr(nva), _ptr(llr)), "llr_batch")
    return llr


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().ranphy_ref_threads())


def set_threads(n: int) -> None:
    """Run the oracle's later loops on n threads (timing only; results do not change)."""
    lib().ranphy_ref_set_threads(int(n))


def qam_points(qm: int) -> np.ndarray:
    pts = np.zeros(1 << qm, np.complex128)
    _check(lib().ranphy_ref_qam_points(qm, _ptr(pts)), "qam_points")
    return pts
