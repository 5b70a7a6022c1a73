"""Training and gating of the learned refinement of the pilot-resolution channel estimate.

Orchestration only: every forward, backward and update step runs in the library's kernels
(``ranphy_cnn_grad``, ``ranphy_cnn_adam``, ``ranphy_cnn_forward``, ``ranphy_cnn_denoise``).
Data are pilot-resolution estimates and their targets as [slot][occ][j][rx][layer] complex64
tensors on the GPU (one slot = one group of rx * layer images over an occasion x pilot grid).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time
from typing import Dict, Iterable, Optional, Sequence

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


# ---- checkpoints ---------------------------------------------------------------------------
# One file: a JSON header on the first line, then the binary sections it lists, each a flat
# little-endian array at the byte offset given (relative to the end of the header line):
#   params_bf16  the parameters rounded to BF16 (round to nearest even): the compact form the
#                network's convolutions use (weights are packed to BF16 for the matrix cores;
#                biases are FP32 in the kernels, so inference from this blob alone differs
#                from params_f32 by the biases' rounding);
#   params_f32   the FP32 parameters;  adam_m, adam_v  the Adam moments (FP32).
# The header carries the format name and version, the parameter count and layout, the step,
# the training state needed to resume (learning rate, total steps, batch, seed, the state of
# the minibatch stream, the losses so far), optional extra fields, and the SHA-256 of the
# binary part, checked on load.
CKPT_FORMAT = "ranphy-cnn-checkpoint"
CKPT_VERSION = 1


def bf16_bits(v: np.ndarray) -> np.ndarray:
    """FP32 values rounded to BF16 (nearest, ties to even), as uint16 bit patterns; NaN stays
    a quiet NaN."""
    u = np.ascontiguousarray(v, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    nan = np.isnan(np.asarray(v, np.float32))
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def save_checkpoint(path: str, params: torch.Tensor, m: Optional[torch.Tensor] = None,
                    v: Optional[torch.Tensor] = None, step: int = 0,
                    train_state: Optional[Dict] = None, extra: Optional[Dict] = None) -> None:
    """Write the parameters (BF16 and FP32), the Adam moments if given and the training state
    to `path` (written to a temporary file, then renamed)."""
    p32 = params.detach().float().cpu().numpy().ravel()
    n = p32.size
    if n != cnn_param_count():
        raise ValueError(f"{n} parameters, expected {cnn_param_count()}")
    blobs = [("params_bf16", "bf16", bf16_bits(p32).tobytes()), ("params_f32", "f32", p32.tobytes())]
    for name, t in (("adam_m", m), ("adam_v", v)):
        if t is not None:
            blobs.append((name, "f32", t.detach().float().cpu().numpy().ravel().tobytes()))
    sections, off, h = [], 0, hashlib.sha256()
    for name, dt, b in blobs:
        sections.append(dict(name=name, dtype=dt, count=n, offset=off, bytes=len(b)))
        off += len(b)
        h.update(b)
    header = dict(format=CKPT_FORMAT, version=CKPT_VERSION, param_count=n,
                  layout="per layer l = 0..3: W_l[9][32 in][32 out] then b_l[32]",
                  channels=list(CHANNELS), step=int(step), sections=sections,
                  sha256=h.hexdigest(), train_state=train_state or {}, extra=extra or {})
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        f.write(json.dumps(header).encode() + b"\n")
        for _, _, b in blobs:
            f.write(b)
    os.replace(tmp, path)


def load_checkpoint(path: str, device="cuda") -> Dict:
    """Read a checkpoint: params (FP32, from params_f32, else the BF16 blob widened), m and v
    (None when absent), params_bf16 (uint16 array), step, train_state and extra.  Raises on a
    wrong format, version, size or checksum."""
    with open(path, "rb") as f:
        header = json.loads(f.readline().decode())
        body = f.read()
    if header.get("format") != CKPT_FORMAT or header.get("version") != CKPT_VERSION:
        raise ValueError(f"{path}: not a {CKPT_FORMAT} v{CKPT_VERSION} file")
    if hashlib.sha256(body).hexdigest() != header["sha256"]:
        raise ValueError(f"{path}: checksum mismatch")
    n = header["param_count"]
    if n != cnn_param_count():
        raise ValueError(f"{path}: {n} parameters, the library has {cnn_param_count()}")
    sec = {d["name"]: d for d in header["sections"]}

    def arr(name):
        d = sec.get(name)
        if d is None:
            return None
        raw = body[d["offset"]:d["offset"] + d["bytes"]]
        if d["dtype"] == "bf16":
            return np.frombuffer(raw, np.uint16).copy()
        return np.frombuffer(raw, np.float32).copy()

    bf = arr("params_bf16")
    p32 = arr("params_f32")
    if p32 is None:
        p32 = (bf.astype(np.uint32) << 16).view(np.float32)
    dev = lambda a: None if a is None else torch.from_numpy(a).to(device)  # noqa: E731
    return dict(params=dev(p32), m=dev(arr("adam_m")), v=dev(arr("adam_v")), params_bf16=bf,
                step=header["step"], train_state=header["train_state"], extra=header["extra"])


def _as_groups(h: torch.Tensor, n_slots: int) -> torch.Tensor:
    return torch.view_as_real(h.reshape(-1)).reshape(n_slots, -1)


def _update(p, m, v, x_all, t_all, noise_var, idx, rows, cols, n_img, ws, step, steps, lr):
    """One Adam step on the slots idx of the grouped data; the cosine-decayed learning rate
    (floored at 1 % of lr) at step of steps.  Returns the minibatch loss (a device tensor)."""
    xb = x_all.index_select(0, idx).reshape(-1).contiguous()
    tb = t_all.index_select(0, idx).reshape(-1).contiguous()
    nb = noise_var.index_select(0, idx).contiguous()
    loss, grad = cnn_grad(p, xb, tb, rows, cols, n_img, idx.numel(), workspace=ws, noise_var=nb)
    rate = lr * max(0.5 * (1.0 + math.cos(math.pi * step / steps)), 0.01)
    cnn_adam(p, grad, m, v, step, rate)
    return loss


def train(h_est: torch.Tensor, h_true: torch.Tensor, noise_var: torch.Tensor, n_slots: int,
          rows: int, cols: int, n_img: int, steps: int = 300, batch: int = 4, lr: float = 2e-3,
          seed: int = 0, params: Optional[torch.Tensor] = None, resume: Optional[str] = None,
          checkpoint: Optional[str] = None, checkpoint_every: int = 0,
          stop_after: Optional[int] = None, on_step=None) -> Dict:
    """Adam on the noise-normalised MSE between the refined and the true channel at the
    pilots; mini-batches of `batch` slots drawn without replacement per step from a seeded
    stream, cosine-decayed learning rate over `steps`.  Returns the parameters, the loss of
    every 10th step and the time.

    resume: a checkpoint written by this function: parameters, Adam moments, the minibatch
    stream and the losses continue from its step, so that the resumed run's parameters equal
    an uninterrupted run's bit for bit (the library's training kernels are deterministic).
    checkpoint / checkpoint_every: write one every that many steps (and after the last step).
    stop_after: end after that step (a run interrupted there, for checkpoint tests).
    on_step(step, params): called after every update (validation curves)."""
    dev = h_est.device
    x_all, t_all = _as_groups(h_est, n_slots), _as_groups(h_true, n_slots)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0xC23, seed])))
    losses, first = [], 1
    if resume is not None:
        ck = load_checkpoint(resume, dev)
        st = ck["train_state"]
        if (st.get("steps"), st.get("batch"), st.get("lr"), st.get("seed")) != (steps, batch, lr, seed):
            raise ValueError("resume: steps, batch, lr and seed must match the checkpoint's")
        p, m, v = ck["params"], ck["m"], ck["v"]
        rng.bit_generator.state = st["rng_state"]
        losses = [torch.tensor(l) for l in st["losses"]]
        first = ck["step"] + 1
    else:
        p = init_params(seed, dev) if params is None else params
        m, v = torch.zeros_like(p), torch.zeros_like(p)
    ws = torch.empty(cnn_workspace_bytes(rows, cols, n_img, batch, True), dtype=torch.uint8,
                     device=dev)

    def save(step):
        save_checkpoint(checkpoint, p, m, v, step, dict(
            steps=steps, batch=batch, lr=lr, seed=seed, rng_state=rng.bit_generator.state,
            losses=[float(l.item()) for l in losses]))

    last = steps if stop_after is None else min(steps, stop_after)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(first, last + 1):
        idx = torch.from_numpy(rng.choice(n_slots, batch, replace=False)).to(dev)
        loss = _update(p, m, v, x_all, t_all, noise_var, idx, rows, cols, n_img, ws, step,
                       steps, lr)
        if step % 10 == 0:
            losses.append(loss)
        if on_step is not None:
            on_step(step, p)
        if checkpoint and ((checkpoint_every and step % checkpoint_every == 0) or step == last):
            save(step)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(params=p, losses=[float(l.item()) for l in losses], seconds=dt, steps=steps,
                batch=batch, images_per_step=batch * n_img, last_step=last)


def train_stream(chunks: Iterable, n_chunks: int, rows: int, cols: int, n_img: int,
                 steps: int = 300, batch: int = 4, lr: float = 2e-3, seed: int = 0,
                 params: Optional[torch.Tensor] = None, on_step=None) -> Dict:
    """Adam as in train() over a training set held a chunk at a time (for sets larger than
    memory).  chunks yields n_chunks tuples (h_est, h_true, noise_var, n_slots); the steps
    are split evenly over the chunks (the first ones take the remainder) and, within a
    chunk, the minibatches walk seeded permutations of its slots, so that a chunk given
    n_slots / batch steps is passed over exactly once.  The learning rate decays over all
    steps as in train().  Returns what train() returns, plus the slots seen."""
    if n_chunks < 1 or steps < n_chunks:
        raise ValueError("train_stream: need at least one chunk and one step per chunk")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0xC24, seed])))
    it = iter(chunks)
    p = m = v = ws = None
    losses, step, seen, dt = [], 0, 0, 0.0
    for c in range(n_chunks):
        h_est, h_true, noise_var, n_slots = next(it)
        if n_slots < batch:
            raise ValueError("train_stream: a chunk holds fewer slots than a minibatch")
        dev = h_est.device
        if p is None:
            p = init_params(seed, dev) if params is None else params
            m, v = torch.zeros_like(p), torch.zeros_like(p)
            ws = torch.empty(cnn_workspace_bytes(rows, cols, n_img, batch, True),
                             dtype=torch.uint8, device=dev)
        x_all, t_all = _as_groups(h_est, n_slots), _as_groups(h_true, n_slots)
        k = steps // n_chunks + (1 if c < steps % n_chunks else 0)
        order = np.concatenate([rng.permutation(n_slots)
                                for _ in range(-(-k * batch // n_slots))])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            step += 1
            idx = torch.from_numpy(order[i * batch:(i + 1) * batch]).to(dev)
            loss = _update(p, m, v, x_all, t_all, noise_var, idx, rows, cols, n_img, ws, step,
                           steps, lr)
            if step % 10 == 0:
                losses.append(loss)
            if on_step is not None:
                on_step(step, p)
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        seen += min(n_slots, k * batch)
        del x_all, t_all, h_est, h_true, noise_var
    return dict(params=p, losses=[float(l.item()) for l in losses], seconds=dt, steps=steps,
                batch=batch, images_per_step=batch * n_img, last_step=step, slots_seen=seen)


def validation_loss(params: Optional[torch.Tensor], h_est: torch.Tensor, h_true: torch.Tensor,
                    noise_var: torch.Tensor, n_slots: int, rows: int, cols: int,
                    n_img: int) -> torch.Tensor:
    """The training objective on held-out slots: the mean squared error per real component
    between the refined estimate and the truth, each slot's divided by its noise variance
    (the loss of ranphy_cnn_grad); with params None that of the plain estimate.  A device
    scalar, so that a curve of it costs no synchronisation."""
    x, t = _as_groups(h_est, n_slots), _as_groups(h_true, n_slots)
    if params is None:
        out = x
    else:
        out = cnn_forward(params, x.reshape(-1).contiguous(), rows, cols, n_img, n_slots,
                          noise_var=noise_var).reshape(n_slots, -1)
    per_slot = ((out - t) ** 2).sum(dim=1) / noise_var
    return per_slot.sum() / t.numel()


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
