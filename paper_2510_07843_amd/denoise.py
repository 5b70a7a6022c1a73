"""Training and gating of the learned refinement of the pilot-resolution channel estimate.

Orchestration only: every forward, backward and update step runs in the library's kernels
(``ranphy_cnn_grad``, ``ranphy_cnn_adam``, ``ranphy_cnn_forward``, ``ranphy_cnn_denoise``).
Data are pilot-resolution estimates and their targets as [slot][occ][j][rx][layer] complex64
tensors on the GPU (one slot = one group of rx * layer images over an occasion x pilot grid).
"""
from __future__ import annotations

import math
import time
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import (chest_ls, cnn_adam, cnn_denoise, cnn_forward, cnn_grad, cnn_param_count,
               cnn_workspace_bytes, mmse_detect)

CHANNELS = (2, 32, 32, 32, 2)
LAYER_PARAMS = 9 * 32 * 32 + 32


def init_params(seed: int, device="cuda") -> torch.Tensor:
    """He-normal weights (fan-in 9 C_in) on the real channels, zero biases and zero padding;
    the last layer scaled by 0.1 so that training starts near the plain estimate."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0xC22, seed])))
    v = np.zeros(cnn_param_count(), np.float32)
    for l in range(4):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if l == 3 else 1.0)
        W = np.zeros((9, 32, 32), np.float32)
        W[:, :ci, :co] = rng.standard_normal((9, ci, co)) * std
        v[l * LAYER_PARAMS:l * LAYER_PARAMS + 9 * 1024] = W.reshape(-1)
    return torch.from_numpy(v).to(device)


def _as_groups(h: torch.Tensor, n_slots: int) -> torch.Tensor:
    return torch.view_as_real(h.reshape(-1)).reshape(n_slots, -1)


def train(h_est: torch.Tensor, h_true: torch.Tensor, noise_var: torch.Tensor, n_slots: int,
          rows: int, cols: int, n_img: int, steps: int = 300, batch: int = 4, lr: float = 2e-3,
          seed: int = 0, params: Optional[torch.Tensor] = None) -> Dict:
    """Adam on the noise-normalised MSE between the refined and the true channel at the
    pilots; mini-batches of `batch` slots drawn without replacement per step from a seeded
    stream, cosine-decayed learning rate.  Returns the parameters, the loss of every 10th step
    and the time."""
    dev = h_est.device
    x_all, t_all = _as_groups(h_est, n_slots), _as_groups(h_true, n_slots)
    p = init_params(seed, dev) if params is None else params
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    ws = torch.empty(cnn_workspace_bytes(rows, cols, n_img, batch, True), dtype=torch.uint8,
                     device=dev)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0xC23, seed])))
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        idx = torch.from_numpy(rng.choice(n_slots, batch, replace=False)).to(dev)
        xb = x_all.index_select(0, idx).reshape(-1).contiguous()
        tb = t_all.index_select(0, idx).reshape(-1).contiguous()
        nb = noise_var.index_select(0, idx).contiguous()
        loss, grad = cnn_grad(p, xb, tb, rows, cols, n_img, batch, workspace=ws, noise_var=nb)
        rate = lr * max(0.5 * (1.0 + math.cos(math.pi * step / steps)), 0.01)
        cnn_adam(p, grad, m, v, step, rate)
        if step % 10 == 0:
            losses.append(loss)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(params=p, losses=[float(l.item()) for l in losses], seconds=dt, steps=steps,
                batch=batch, images_per_step=batch * n_img)


def nmse_db(est: torch.Tensor, true: torch.Tensor) -> float:
    e = torch.sum(torch.abs(est - true) ** 2).item()
    return 10.0 * math.log10(e / torch.sum(torch.abs(true) ** 2).item())


def choose_gate(params: torch.Tensor, h_est: torch.Tensor, h_true: torch.Tensor,
                noise_var: torch.Tensor, snr_db: Sequence[float], rows: int, cols: int,
                n_img: int) -> Dict:
    """Per-SNR NMSE of the plain and the refined estimate on validation slots, and the
    noise-variance gate: refine slots up to the highest SNR point of the validation grid at
    which every point at or below it gains, keep the plain estimate above it."""
    n = len(snr_db)
    out = cnn_forward(params, torch.view_as_real(h_est.reshape(-1)).reshape(-1).contiguous(),
                      rows, cols, n_img, n, noise_var=noise_var)
    ref = torch.view_as_complex(out.reshape(-1, 2)).reshape(n, -1)
    est, true = h_est.reshape(n, -1), h_true.reshape(n, -1)
    snr = np.asarray(snr_db, dtype=float)
    table = []
    for s in sorted(set(snr.tolist())):
        sel = torch.from_numpy(np.flatnonzero(snr == s)).to(h_est.device)
        a = nmse_db(est.index_select(0, sel), true.index_select(0, sel))
        b = nmse_db(ref.index_select(0, sel), true.index_select(0, sel))
        table.append((s, a, b))
    top = None
    for s, a, b in table:
        if a - b > 0.0:
            top = s
        else:
            break
    min_nv = math.inf if top is None else 10.0 ** (-top / 10.0)
    return dict(min_noise_var=min_nv, max_snr_db=top,
                nmse=[dict(snr_db=s, plain_db=round(a, 3), refined_db=round(b, 3),
                           gain_db=round(a - b, 3)) for s, a, b in table])


def sinr_db(x_hat: np.ndarray, x: np.ndarray) -> float:
    """Post-equalisation SINR E|x|^2 / E|x_hat - x|^2 in dB."""
    return 10.0 * math.log10(float(np.mean(np.abs(x) ** 2)) /
                             float(np.mean(np.abs(x_hat - x) ** 2)))


def choose_gate_sinr(params: torch.Tensor, shape, rx: torch.Tensor, pilots: torch.Tensor,
                     noise_var: torch.Tensor, x_true: np.ndarray, snr_db: Sequence[float]) -> Dict:
    """The noise-variance gate chosen by what detection sees: per SNR point of full validation
    slots, the post-equalisation SINR of the FP32 detector with the plain and with the refined
    (ungated) estimate against the transmitted symbols; refine up to the highest SNR point at
    or below which every point gains, keep the plain estimate above it."""
    h = chest_ls(shape, rx, pilots)
    hr = cnn_denoise(shape, params, h, noise_var=noise_var)
    xs = {}
    for name, est in (("plain", h), ("refined", hr)):
        x, _ = mmse_detect(shape, rx, est, noise_var)
        torch.cuda.synchronize()
        xs[name] = x.cpu().numpy().reshape(x_true.shape)
    snr = np.asarray(snr_db, dtype=float)
    table = []
    for s in sorted(set(snr.tolist())):
        sel = np.flatnonzero(snr == s)
        a = sinr_db(xs["plain"][sel], x_true[sel])
        b = sinr_db(xs["refined"][sel], x_true[sel])
        table.append((s, a, b))
    top = None
    for s, a, b in table:
        if b - a > 0.0:
            top = s
        else:
            break
    min_nv = math.inf if top is None else 10.0 ** (-top / 10.0)
    return dict(min_noise_var=min_nv, max_snr_db=top,
                sinr=[dict(snr_db=s, plain_db=round(a, 3), refined_db=round(b, 3),
                           gain_db=round(b - a, 3)) for s, a, b in table])
