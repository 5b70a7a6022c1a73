"""Benchmark of the uplink receive hot path on one MI355X.

A step is one pass of the whole path -- channel estimation, detection, demapping -- over one
batch of synthetic slots already resident in HBM: chest_ls -> mmse_llr (detection with the
demapping in its epilogue) where the shape takes the matrix-core detector; for up to 8 layers
otherwise the whole chain as one launch (receive), with the three-call chain chest_ls ->
mmse_detect -> llr_demap timed beside it.  The default workload is 64 Rx x 16
layers, 273 PRB (3276 subcarriers) x 14 symbols, 64QAM, one double-symbol DMRS occasion
(comb 8, time cover 2), exponential-PDP TDL channel with 300 ns rms delay spread, SNR 0..30
dB in 5 dB steps, 20 slots per SNR point: 140 slots, 39312 data REs each.

Prints one JSON line: data REs detected per second (whole job), the dominant kernel's
roofline figures (HIP-event timing on the launch stream) and the FP64 oracle timed on the
host cores for a bounded sample of the same batch.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_MFMA_PEAK_TFLOPS = 157.3    # dense FP32 matrix
FP32_VALU_PEAK_TFLOPS = 78.6     # FP32 vector FMA without packed-FP32 instructions

CMAC = 8  # real flops per complex multiply-accumulate

PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = {
    "mmse_detect": ("paper_2510_07843_amd/csrc/mmse_mfma.hip", "paper_2510_07843_amd/csrc/geom.h",
                    "paper_2510_07843_amd/csrc/llr_math.h"),
    "mmse_llr": ("paper_2510_07843_amd/csrc/mmse_mfma.hip", "paper_2510_07843_amd/csrc/geom.h",
                 "paper_2510_07843_amd/csrc/llr_math.h"),
    "receive": ("paper_2510_07843_amd/csrc/batch.hip", "paper_2510_07843_amd/csrc/batch.h",
                "paper_2510_07843_amd/csrc/geom.h", "paper_2510_07843_amd/csrc/llr_math.h"),
    "batch_kernel": ("paper_2510_07843_amd/csrc/batch.hip", "paper_2510_07843_amd/csrc/batch.h",
                     "paper_2510_07843_amd/csrc/geom.h", "paper_2510_07843_amd/csrc/llr_math.h"),
}


def source_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel: str, tag: str):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary for this workload, or None when there is none or the kernel's source has changed
    since the counters were taken."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_{tag}.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    fields = dict(l.split(": ", 1) for l in open(path).read().splitlines()
                  if l.startswith(kernel + "_"))
    if fields.get(f"{kernel}_source_sha256") != source_digest(kernel):
        return None
    return float(fields[f"{kernel}_traffic_bytes_per_launch"])


def measured_counters(kernel: str, prec: str, tag: str):
    """Per-wave instruction counts and busy fractions of ``kernel`` from the committed
    rocprofv3 SQ-counter summary for this workload and precision (VALU instructions other
    than MFMA per wave, MFMA per wave, the fractions of the SIMD cycles the MFMA and the
    other VALU instructions occupy), or None when there is none or the kernel's source has
    changed since the counters were taken."""
    path = os.path.join(PROFILES, f"counters_{kernel}_{prec}_{tag}.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    key = f"{kernel}_{prec}_"
    fields = dict(l.split(": ", 1) for l in open(path).read().splitlines() if l.startswith(key))
    if fields.get(key + "source_sha256") != source_digest(kernel):
        return None
    return {n: float(fields[key + n]) for n in ("valu_per_wave", "mfma_per_wave",
                                                 "mfma_busy_frac", "valu_busy_frac")}


def algorithmic_costs(shape, h_res=0):
    """Per-launch algorithmic HBM bytes and flops of each call (each input read once, each
    output written once; flops of the method's own arithmetic in the z-form: Hermitian half
    Gram per subcarrier, Cholesky and triangular inverse, matched filter, two triangular
    solves per RE)."""
    S, nsc, nd, NR, NL, Q = shape.n_slots, shape.n_sc, shape.n_dsym, shape.n_rx, shape.n_layers, shape.qm
    occ, T, J = shape.n_occ, shape.dmrs_td, shape.n_pilot
    n_dmrs_sym = occ * T
    K = J if h_res == 0 else nsc
    h_bytes = S * occ * K * NR * NL * 8
    chest = dict(
        bytes=S * n_dmrs_sym * nsc * NR * 8 + S * occ * T * J * NL * 8 + h_bytes,
        flops=S * occ * J * NR * NL * T * CMAC)
    re = S * nd * nsc
    gram_per_sc = NL * (NL + 1) // 2 * NR            # CMAC, once per sc per occasion
    chol_per_sc = 2 * NL ** 3 // 6                    # Cholesky + L^-1, CMAC
    per_re = NL * NR + NL * NL                        # matched filter + two triangular solves
    n_gram = occ if occ == 1 else nd                  # time-varying channel: per data symbol
    mmse = dict(
        bytes=re * NR * 8 + h_bytes + S * 4 + re * NL * 8 + re * NL * 4,
        flops=CMAC * (S * nsc * n_gram * (gram_per_sc + chol_per_sc) + re * per_re))
    llr = dict(bytes=re * NL * (8 + 4) + re * NL * Q * 4, flops=re * NL * Q * 6)
    fused = dict(bytes=mmse["bytes"] - re * NL * (8 + 4) + re * NL * Q * 4,
                 flops=mmse["flops"] + llr["flops"])
    # one launch: the whole received grid, the pilots and the noise variances in, LLRs out
    receive = dict(bytes=S * shape.n_symb * nsc * NR * 8 + S * occ * T * J * NL * 8 + S * 4
                   + re * NL * Q * 4,
                   flops=chest["flops"] + mmse["flops"] + llr["flops"])
    return dict(chest_ls=chest, mmse_detect=mmse, llr_demap=llr, mmse_llr=fused,
                receive=receive, data_re=re)


def fused_eligible(shape) -> bool:
    """Shapes the matrix-core detector (and so the fused detection + demapping) takes."""
    return (shape.n_occ == 1 and 5 <= shape.n_layers <= 16 and shape.n_rx % 16 == 0
            and shape.n_rx <= 64 and shape.n_dsym <= 16)


def host_cpu() -> dict:
    """The host the oracle runs on: logical CPUs, the CPUs this process may use, the model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "model": model}


def cpu_baseline(b, budget_s: float, reps: int = 5):
    """The FP64 oracle on the host for a fixed sample of the batch (its first slot):
    chest_ls + mmse_detect (LU route) + llr_demap, timed `reps` times on all the threads the
    oracle uses and `reps` times on one thread, the median of each reported.  A leg stops
    repeating once its runs have used `budget_s / 2` (at least one run each)."""
    import oracle
    shape = b["shape"]
    one = shape.with_slots(1)
    rx, pil, nvar = b["rx"][:1], b["pilots"][:1], b["noise_var"][:1]
    per_slot = shape.n_dsym * shape.n_sc

    def once():
        t0 = time.perf_counter()
        h = oracle.chest_ls(one, rx, pil).astype(np.complex64)
        x, nv = oracle.mmse_detect(one, rx, h, oracle.H_PILOT, nvar)
        oracle.llr_demap(one, x.astype(np.complex64), nv.astype(np.float32))
        return time.perf_counter() - t0

    all_threads = oracle.threads()
    legs = {}
    try:
        for n in (all_threads, 1):
            oracle.set_threads(n)
            ts, spent = [], 0.0
            while len(ts) < reps and (not ts or spent < budget_s / 2):
                ts.append(once())
                spent += ts[-1]
            legs[n] = {"value": per_slot / float(np.median(ts)), "runs": len(ts),
                       "seconds": [round(t, 3) for t in ts]}
    finally:
        oracle.set_threads(all_threads)
    cpu = host_cpu()
    out = dict(value=legs[all_threads]["value"], unit="RE/s", cores=all_threads, kind="oracle",
               sample=f"slot 0 of the batch ({per_slot} data REs), chest_ls + mmse_detect (LU "
                      f"route) + llr_demap in FP64; median of {legs[all_threads]['runs']} runs "
                      f"on {all_threads} threads",
               runs_seconds=legs[all_threads]["seconds"], host=cpu)
    out["single_thread"] = {"value": legs[1]["value"], "unit": "RE/s", "cores": 1,
                            "runs_seconds": legs[1]["seconds"],
                            "sample": f"the same slot, median of {legs[1]['runs']} runs"}
    return out


def PRECISIONS(ranphy):
    """The detector's precision modes: name, library code."""
    return (("fp32", ranphy.PREC_FP32), ("fp16", ranphy.PREC_FP16), ("bf16", ranphy.PREC_BF16),
            ("fp16_refined", ranphy.PREC_FP16_REFINED), ("bf16_refined", ranphy.PREC_BF16_REFINED))


def detection_quality(torch, ranphy, synth):
    """Post-equalisation SINR of each detector precision and of the FP64 oracle on one slot
    per SNR point of the 64 x 16 workload (the same seeded slots as the batch's first 7)."""
    import oracle
    t = synth.make_batch("m", n_slots=len(synth.CONFIGS["m"]["snr_db"]), workers=8)
    sh = t["shape"]
    hq = oracle.chest_ls(sh, t["rx"], t["pilots"]).astype(np.complex64)
    xr, _ = oracle.mmse_detect(sh, t["rx"], hq, oracle.H_PILOT, t["noise_var"])
    dev = torch.device("cuda:0")
    rx = torch.from_numpy(t["rx"]).to(dev).reshape(-1)
    pil = torch.from_numpy(t["pilots"]).to(dev).reshape(-1)
    nvar = torch.from_numpy(t["noise_var"]).to(dev)

    def sinr(xh, x):
        return 10 * np.log10(np.mean(np.abs(x) ** 2) / np.mean(np.abs(xh - x) ** 2))

    ref = [sinr(xr[i], t["x"][i]) for i in range(sh.n_slots)]
    out = {}
    for name, p in PRECISIONS(ranphy):
        hg = ranphy.chest_ls(sh, rx, pil)
        xg, _ = ranphy.mmse_detect(sh, rx, hg, nvar, precision=p)
        torch.cuda.synchronize()
        xg = xg.cpu().numpy().reshape(xr.shape)
        s = [sinr(xg[i], t["x"][i]) for i in range(sh.n_slots)]
        evm = [10 * np.log10(np.mean(np.abs(xg[i] - xr[i]) ** 2) / np.mean(np.abs(xr[i]) ** 2))
               for i in range(sh.n_slots)]
        out[name] = {"sinr_db": [round(v, 3) for v in s],
                     "sinr_loss_db_max": round(float(max(r - v for r, v in zip(ref, s))), 4),
                     "evm_vs_fp64_db_max": round(float(max(evm)), 1)}
    out["fp32"]["sinr_fp64_db"] = [round(v, 3) for v in ref]
    out["fp32"]["snr_db"] = [float(v) for v in t["snr_db"]]
    return out


def slot_latency(torch, ranphy, shape, rx, pil, nvar, h_res, prec, path, scs_hz, reps=200):
    """One slot through the whole chain: mean time per slot launched eagerly (one call per
    step, synchronised at the end) and replayed from a HIP graph holding the slot's launches;
    the replayed LLRs must equal the eager ones bit for bit."""
    one = shape.with_slots(1)
    dev = rx.device
    n_rx = ranphy.buffer_floats(one, ranphy.BUF_RX) // 2
    n_pil = ranphy.buffer_floats(one, ranphy.BUF_PILOTS) // 2
    rx1, pil1, nv1 = rx[:n_rx], pil[:n_pil], nvar[:1]
    h1 = torch.empty(ranphy.buffer_floats(one, ranphy.BUF_H, h_res) // 2, dtype=torch.complex64, device=dev)
    x1 = torch.empty(ranphy.buffer_floats(one, ranphy.BUF_X) // 2, dtype=torch.complex64, device=dev)
    v1 = torch.empty(ranphy.buffer_floats(one, ranphy.BUF_NV), dtype=torch.float32, device=dev)
    l1 = torch.empty(ranphy.buffer_floats(one, ranphy.BUF_LLR), dtype=torch.float32, device=dev)

    def chain():
        if path == "receive":
            ranphy.receive(one, rx1, pil1, nv1, llr=l1)
            return
        ranphy.chest_ls(one, rx1, pil1, h=h1, h_res=h_res)
        if path == "fused":
            ranphy.mmse_llr(one, rx1, h1, nv1, h_res=h_res, llr=l1, precision=prec)
        else:
            ranphy.mmse_detect(one, rx1, h1, nv1, h_res=h_res, x=x1, nv=v1, precision=prec)
            ranphy.llr_demap(one, x1, v1, llr=l1)

    def timed(fn):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e3

    eager_us = timed(chain)
    ref = l1.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capturing stream
        chain()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        chain()
    graph_us = timed(graph.replay)
    l1.zero_()
    graph.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(l1.view(torch.int32), ref.view(torch.int32)))
    # the fixed cost of the two launch modes: two one-element kernels, eager and replayed
    tiny = torch.zeros(1, device=dev)

    def two_tiny():
        tiny.add_(1.0)
        tiny.mul_(0.5)

    floor_eager = timed(two_tiny)
    with torch.cuda.stream(side):
        two_tiny()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        two_tiny()
    floor_graph = timed(g2.replay)
    slot_us = 1000.0 * 15e3 / scs_hz  # 14-symbol slot: 1 ms at 15 kHz, 0.5 ms at 30 kHz
    return {"eager_us": round(eager_us, 2), "graph_us": round(graph_us, 2),
            "graph_matches_eager": same, "slot_duration_us": slot_us,
            "data_re_per_slot": one.n_dsym * one.n_sc,
            "two_empty_kernels_us": {"eager": round(floor_eager, 2), "graph": round(floor_graph, 2)}}


def h2d_rate(torch, rx_host, ms_step, re, ranphy=None, shape=None, fused_step=None):
    """The received grids' upload over PCIe from pinned host memory, measured on a copy of
    the batch's rx (not part of `value`: the library takes device buffers); with it the chain
    rate if every step first uploaded its grids without overlap."""
    src = torch.from_numpy(rx_host).reshape(-1).pin_memory()
    dst = torch.empty(src.shape, dtype=src.dtype, device="cuda")
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    a.record()
    for _ in range(reps):
        dst.copy_(src, non_blocking=True)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    nbytes = src.numel() * src.element_size()
    out = {"bytes": nbytes, "ms": round(ms, 4), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1),
           "chain_with_upload_re_per_s": re / ((ms_step + ms) * 1e-3)}
    if shape is not None:
        out["bfp"] = bfp_upload(torch, ranphy, shape, dst, ms_step, re, fused_step)
    return out


def bfp_upload(torch, ranphy, shape, rx_dev, ms_step, re, fused_step=None):
    """The same grids sent as block floating point words (16-antenna blocks, 9-bit mantissas,
    shared exponent): upload of the words from pinned host memory, decompression on the GPU,
    and the chain rate with both before every step (no overlap).  With `fused_step(words)`
    (the estimator and detector reading the words themselves) also that chain's own time and
    its rate with the upload."""
    words = ranphy.bfp_compress(shape, rx_dev)
    host = torch.empty(words.shape, dtype=words.dtype, pin_memory=True)
    host.copy_(words)
    back = torch.empty_like(rx_dev)
    ranphy.bfp_decompress(shape, words, back)
    torch.cuda.synchronize()
    err = (back - rx_dev).abs().pow(2).sum().item()
    sqnr = 10.0 * math.log10(rx_dev.abs().pow(2).sum().item() / err) if err > 0 else None
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = 3
    ev[0].record()
    for _ in range(reps):
        words.copy_(host, non_blocking=True)
    ev[1].record()
    for _ in range(reps):
        ranphy.bfp_decompress(shape, words, back)
    ev[2].record()
    torch.cuda.synchronize()
    up = ev[0].elapsed_time(ev[1]) / reps
    dec = ev[1].elapsed_time(ev[2]) / reps
    nb = words.numel() * 4
    out = {"bytes": nb, "ratio": round(rx_dev.numel() * 8 / nb, 3), "upload_ms": round(up, 4),
           "decompress_ms": round(dec, 4),
           "decompress_GB/s": round((nb + rx_dev.numel() * 8) / (dec * 1e-3) / 1e9, 1),
           "sqnr_db": None if sqnr is None else round(sqnr, 1),
           "chain_with_upload_re_per_s": re / ((ms_step + up + dec) * 1e-3)}
    if fused_step is not None:
        fused_step(words)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            fused_step(words)
        e1.record()
        torch.cuda.synchronize()
        fm = e0.elapsed_time(e1) / reps
        out["fused_chain_ms"] = round(fm, 4)
        out["fused_chain_re_per_s"] = re / (fm * 1e-3)
        out["fused_chain_with_upload_re_per_s"] = re / ((up + fm) * 1e-3)
    return out


def held_out_curve(torch, synth, denoise, shape, ls, steps, cols, nimg, seed, points=12):
    """The training objective on 14 held-out DMRS slots (two per SNR point 0, 5, .., 30 dB;
    delay spread and Doppler drawn as for training, realisations of their own) at the
    initial parameters and every steps / points steps, kept on the device until the end.
    Returns the on_step hook for the trainer and a function that reads out the report."""
    dev = torch.device("cuda:0")
    grid = (0.0, 5.0, 10.0, 15.0, 20.0, 25.0, 30.0)
    ho = synth.make_dmrs_batch(shape, 2 * len(grid), seed=44, snr_db=grid,
                               workers=min(16, os.cpu_count() or 1))
    n = 2 * len(grid)
    he, ht = ls(ho), torch.from_numpy(ho["h"]).to(dev)
    hv = torch.from_numpy(ho["noise_var"]).to(dev)
    every = max(1, steps // points)
    pts = [(0, denoise.validation_loss(denoise.init_params(seed, dev), he, ht, hv, n, 1, cols,
                                       nimg))]
    plain = denoise.validation_loss(None, he, ht, hv, n, 1, cols, nimg)

    def on_step(step, p):
        if step % every == 0 or step == steps:
            pts.append((step, denoise.validation_loss(p, he, ht, hv, n, 1, cols, nimg)))

    def report():
        return {"slots": n, "snr_db": list(grid), "per_snr_point": 2,
                "plain_estimate": round(float(plain.item()), 5),
                "steps": [k for k, _ in pts], "loss": [round(float(l.item()), 5) for _, l in pts]}
    return {"on_step": on_step, "report": report}


def train_refinement(torch, ranphy, synth, shape, steps=600, batch=2, n_train=96):
    """Train the pilot-estimate refinement on the GPU for the workload's DMRS grid (delay
    spread 30..300 ns, Doppler 0..500 Hz, SNR 0..30 dB) and choose its noise-variance gate by
    the detector's post-equalisation SINR on full validation slots of the 64 x 16 workload
    (realisations other than those the quality figures use); the NMSE at the pilots on DMRS
    slots at the largest delay spread is reported beside it.  Returns the parameters, the gate
    and a report."""
    from paper_2510_07843_amd import denoise
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    tr = synth.make_dmrs_batch(shape, n_train, seed=41, workers=min(16, os.cpu_count() or 1))
    grid = (0.0, 5.0, 10.0, 15.0, 20.0, 25.0, 30.0)
    va = synth.make_dmrs_batch(shape, 2 * len(grid), seed=42, snr_db=grid,
                               tau_rms=synth.DMRS_RANGES["tau_rms"][1],
                               workers=min(16, os.cpu_count() or 1))
    t_gen = time.perf_counter() - t0
    ts = tr["shape"]
    cols, nimg = ts.n_pilot, ts.n_rx * ts.n_layers

    def ls(b):
        return ranphy.chest_ls(b["shape"], torch.from_numpy(b["rx"]).to(dev).reshape(-1),
                               torch.from_numpy(b["pilots"]).to(dev).reshape(-1))

    curve = held_out_curve(torch, synth, denoise, shape, ls, steps, cols, nimg, seed=43)
    res = denoise.train(ls(tr), torch.from_numpy(tr["h"]).to(dev),
                        torch.from_numpy(tr["noise_var"]).to(dev), n_train, 1, cols, nimg,
                        steps=steps, batch=batch, seed=43, on_step=curve["on_step"])
    nmse = denoise.choose_gate(res["params"], ls(va), torch.from_numpy(va["h"]).to(dev),
                               torch.from_numpy(va["noise_var"]).to(dev), va["snr_db"], 1, cols,
                               nimg)
    vs = synth.make_batch("m", n_slots=2 * len(synth.CONFIGS["m"]["snr_db"]), first_slot=1,
                          workers=min(16, os.cpu_count() or 1))
    gate = denoise.choose_gate_sinr(res["params"], vs["shape"],
                                    torch.from_numpy(vs["rx"]).to(dev).reshape(-1),
                                    torch.from_numpy(vs["pilots"]).to(dev).reshape(-1),
                                    torch.from_numpy(vs["noise_var"]).to(dev), vs["x"],
                                    vs["snr_db"])
    report = {"train_slots": n_train, "images_per_slot": nimg, "steps": steps,
              "images_per_step": res["images_per_step"], "train_seconds": round(res["seconds"], 2),
              "data_seconds": round(t_gen, 1), "validation_loss": curve["report"](),
              "refine_up_to_snr_db": gate["max_snr_db"], "validation_sinr": gate["sinr"],
              "validation_nmse_at_pilots": nmse["nmse"]}
    return res["params"], gate["min_noise_var"], report


def train_study(args, torch, ranphy, synth):
    """The learned refinement trained with one optimisation budget (steps x batch slots) on
    training sets of several sizes, nested (each set is a prefix of the next, slots drawn
    as for the benchmark's training: delay spread 30..300 ns, Doppler 0..500 Hz, SNR
    0..30 dB).  Per size: the held-out loss curve, the post-equalisation SINR of the FP32
    detector with the plain and the (ungated) refined estimate per SNR point on full
    validation slots of the 64 x 16 workload, the gate that SINR selects, and the NMSE at
    the pilots at the largest delay spread.  Prints one JSON line."""
    from paper_2510_07843_amd import denoise
    dev = torch.device("cuda:0")
    shape = synth.CONFIGS["m"]["shape"]
    workers = min(16, os.cpu_count() or 1)
    budgets = sorted(int(b) for b in args.train_study.split(","))
    steps, batch, piece = args.study_steps, 2, 1024
    ts = synth.dmrs_shape(shape, 1)
    cols, nimg = ts.n_pilot, ts.n_rx * ts.n_layers
    per = cols * nimg  # complex entries per slot

    def ls(b):
        return ranphy.chest_ls(b["shape"], torch.from_numpy(b["rx"]).to(dev).reshape(-1),
                               torch.from_numpy(b["pilots"]).to(dev).reshape(-1))

    def log(msg):
        print(f"[train-study] {msg}", file=sys.stderr, flush=True)

    top = budgets[-1]
    he = torch.empty((top, per), dtype=torch.complex64, device=dev)
    ht = torch.empty_like(he)
    hv = torch.empty(top, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for c in range(0, top, piece):
        k = min(piece, top - c)
        b = synth.make_dmrs_batch(shape, k, seed=41 if c == 0 else 41000 + c // piece,
                                  workers=workers)
        he[c:c + k] = ls(b).reshape(k, per)
        ht[c:c + k] = torch.from_numpy(b["h"].reshape(k, per)).to(dev)
        hv[c:c + k] = torch.from_numpy(b["noise_var"]).to(dev)
        del b
        log(f"training slots {c + k}/{top} generated ({time.perf_counter() - t0:.0f} s)")
    t_gen = time.perf_counter() - t0
    grid = (0.0, 5.0, 10.0, 15.0, 20.0, 25.0, 30.0)
    va = synth.make_dmrs_batch(shape, 2 * len(grid), seed=42, snr_db=grid,
                               tau_rms=synth.DMRS_RANGES["tau_rms"][1], workers=workers)
    vs = synth.make_batch("m", n_slots=2 * len(synth.CONFIGS["m"]["snr_db"]), first_slot=1,
                          workers=workers)
    va_h, va_t = ls(va), torch.from_numpy(va["h"]).to(dev)
    va_v = torch.from_numpy(va["noise_var"]).to(dev)
    vs_rx = torch.from_numpy(vs["rx"]).to(dev).reshape(-1)
    vs_p = torch.from_numpy(vs["pilots"]).to(dev).reshape(-1)
    vs_v = torch.from_numpy(vs["noise_var"]).to(dev)
    rows = []
    for n in budgets:
        curve = held_out_curve(torch, synth, denoise, shape, ls, steps, cols, nimg, seed=43,
                               points=16)
        res = denoise.train_stream([(he[:n], ht[:n], hv[:n], n)], 1, 1, cols, nimg,
                                   steps=steps, batch=batch, seed=43, on_step=curve["on_step"])
        gate = denoise.choose_gate_sinr(res["params"], vs["shape"], vs_rx, vs_p, vs_v, vs["x"],
                                        vs["snr_db"])
        nmse = denoise.choose_gate(res["params"], va_h, va_t, va_v, va["snr_db"], 1, cols, nimg)
        rows.append({"train_slots": n, "passes": round(steps * batch / n, 2),
                     "train_seconds": round(res["seconds"], 2),
                     "validation_loss": curve["report"](),
                     "train_loss_last100_steps": round(float(np.mean(res["losses"][-10:])), 5),
                     "refine_up_to_snr_db": gate["max_snr_db"], "sinr": gate["sinr"],
                     "nmse_at_pilots_tau300ns": nmse["nmse"]})
        g = {r["snr_db"]: r["gain_db"] for r in gate["sinr"]}
        log(f"{n} slots: SINR gain {g.get(0.0)} dB at 0 dB, {g.get(10.0)} dB at 10 dB, "
            f"held-out loss {rows[-1]['validation_loss']['loss'][-1]}")
    print(json.dumps({"study": "learned estimate refinement vs training-set size",
                      "steps": steps, "batch_slots": batch, "lr": 2e-3,
                      "images_per_slot": nimg, "data_seconds": round(t_gen, 1),
                      "validation_slots": {"held_out_loss": 14, "sinr_full_slots": len(vs["snr_db"]),
                                           "nmse": len(va["snr_db"])},
                      "budgets": rows}), flush=True)


def learned_quality(torch, ranphy, synth, params, min_nv):
    """Post-equalisation SINR with the refined estimate and with the plain one (FP32
    detector) on one slot per SNR point of the 64 x 16 workload."""
    t = synth.make_batch("m", n_slots=len(synth.CONFIGS["m"]["snr_db"]), workers=8)
    sh = t["shape"]
    dev = torch.device("cuda:0")
    rx = torch.from_numpy(t["rx"]).to(dev).reshape(-1)
    pil = torch.from_numpy(t["pilots"]).to(dev).reshape(-1)
    nvar = torch.from_numpy(t["noise_var"]).to(dev)

    def sinr(xh, x):
        return 10 * np.log10(np.mean(np.abs(x) ** 2) / np.mean(np.abs(xh - x) ** 2))

    hg = ranphy.chest_ls(sh, rx, pil)
    hr = ranphy.cnn_denoise(sh, params, hg, noise_var=nvar, min_noise_var=min_nv)
    out = {}
    for name, h in (("plain", hg), ("refined", hr)):
        xg, _ = ranphy.mmse_detect(sh, rx, h, nvar)
        torch.cuda.synchronize()
        xg = xg.cpu().numpy().reshape(t["x"].shape)
        out[name] = [sinr(xg[i], t["x"][i]) for i in range(sh.n_slots)]
    return {"snr_db": [float(v) for v in t["snr_db"]],
            "sinr_plain_db": [round(v, 3) for v in out["plain"]],
            "sinr_refined_db": [round(v, 3) for v in out["refined"]],
            "sinr_gain_db": [round(b - a, 3) for a, b in zip(out["plain"], out["refined"])]}


def make_batch_ues(torch, synth, n_ue=200, seed=5):
    """The batching workload: n_ue UEs over 10 cells (cell = UE index mod 10), each one slot
    with PRB uniform in 4..273, 1..8 layers, Rx from {4, 8, 16, 32, 64} (>= layers),
    QPSK..256QAM, SNR uniform in 0..30 dB, 30 kHz, exponential-PDP TDL at 100 ns; DMRS on
    symbol 2 with comb and cover by the layer count (comb 2 up to 2 layers, comb 2 x 2 symbols
    up to 4, comb 4 x 2 symbols up to 8)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0xBA7, seed])))
    specs = []
    for i in range(n_ue):
        nl = int(rng.integers(1, 9))
        nr = int(rng.choice([r for r in (4, 8, 16, 32, 64) if r >= nl]))
        comb, td = (2, 1) if nl <= 2 else ((2, 2) if nl <= 4 else (4, 2))
        shape = synth.SlotShape(int(rng.integers(4, 274)), 14, nr, nl, int(rng.choice([2, 4, 6, 8])),
                                comb, td, (2,), 1)
        specs.append((shape, float(rng.uniform(0, 30))))
    out = [None] * n_ue

    def one(i):
        shape, snr = specs[i]
        out[i] = synth.make_slot(shape, synth.rng_for(8, seed, i), 30e3, ("exp", 100e-9), snr)

    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(one, range(n_ue)))
    dev = torch.device("cuda:0")
    ues = []
    for i, d in enumerate(out):
        ues.append(dict(shape=specs[i][0], cell=i % 10, snr_db=specs[i][1],
                        rx=torch.from_numpy(d["rx"]).to(dev).reshape(-1),
                        pilots=torch.from_numpy(d["pilots"]).to(dev).reshape(-1),
                        noise_var=torch.tensor([d["noise_var"]], dtype=torch.float32, device=dev),
                        rx_h=d["rx"][None], pil_h=d["pilots"][None],
                        nv_h=np.array([d["noise_var"]], np.float32)))
    return ues


def bench_batch(args, torch, ranphy, synth):
    """The multi-UE persistent launch: autotuned plan, captured in a HIP graph and replayed;
    the same UEs launched one call per UE and step beside it."""
    from paper_2510_07843_amd import tune
    t0 = time.perf_counter()
    ues = make_batch_ues(torch, synth, n_ue=args.slots or 200)
    t_gen = time.perf_counter() - t0
    re = sum(u["shape"].n_dsym * u["shape"].n_sc for u in ues)
    if args.batch_config:  # a fixed configuration (profiled runs): no autotuning launches
        tile, bpc = (int(v) for v in args.batch_config.split(","))
        tuned = tune.autotune(ues, tiles=(tile,), blocks_per_cu=(bpc,), reps=1)
    else:
        tuned = tune.autotune(ues, reps=3, cache=args.tune_cache)
    b, nb = tuned["batch"], tuned["n_blocks"]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run(nb)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.run(nb)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # one call per UE: chest_ls, mmse_detect, llr_demap (the library's single-UE path)
    bufs = []
    for u in ues:
        sh = u["shape"]
        bufs.append(dict(
            h=torch.empty(ranphy.buffer_floats(sh, ranphy.BUF_H) // 2, dtype=torch.complex64, device="cuda"),
            x=torch.empty(ranphy.buffer_floats(sh, ranphy.BUF_X) // 2, dtype=torch.complex64, device="cuda"),
            nv=torch.empty(ranphy.buffer_floats(sh, ranphy.BUF_NV), dtype=torch.float32, device="cuda"),
            llr=torch.empty(ranphy.buffer_floats(sh, ranphy.BUF_LLR), dtype=torch.float32, device="cuda")))

    def per_ue():
        for u, q in zip(ues, bufs):
            sh = u["shape"]
            ranphy.chest_ls(sh, u["rx"], u["pilots"], h=q["h"])
            ranphy.mmse_detect(sh, u["rx"], q["h"], u["noise_var"], x=q["x"], nv=q["nv"])
            ranphy.llr_demap(sh, q["x"], q["nv"], llr=q["llr"])

    for _ in range(2):
        per_ue()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(max(1, args.steps // 4)):
        per_ue()
    e1.record()
    torch.cuda.synchronize()
    ms_per_ue = e0.elapsed_time(e1) / max(1, args.steps // 4)

    def per_ue_receive():  # the one-launch chain, one launch per UE
        for u in ues:
            ranphy.receive(u["shape"], u["rx"], u["pilots"], u["noise_var"], llr=u["llr"])

    for _ in range(2):
        per_ue_receive()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(max(1, args.steps // 4)):
        per_ue_receive()
    e1.record()
    torch.cuda.synchronize()
    ms_per_ue_rx = e0.elapsed_time(e1) / max(1, args.steps // 4)
    # algorithmic bytes and flops of the fused chain: every input read once, LLRs written once
    nbytes = flops = 0
    for u in ues:
        sh = u["shape"]
        c = algorithmic_costs(sh)
        nbytes += (sh.n_symb * sh.n_sc * sh.n_rx * 8 + sh.n_occ * sh.dmrs_td * sh.n_pilot * sh.n_layers * 8
                   + 4 + sh.n_dsym * sh.n_sc * sh.n_layers * sh.qm * 4)
        flops += c["chest_ls"]["flops"] + c["mmse_llr"]["flops"]
    sec = ms * 1e-3
    t_bytes = nbytes / (HBM_PEAK_GBS * 1e9)
    t_flops = flops / (FP32_VALU_PEAK_TFLOPS * 1e12)
    if t_bytes >= t_flops:
        roof = dict(bound="hbm", achieved=nbytes / sec / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    else:
        roof = dict(bound="alu", achieved=flops / sec / 1e12, peak=FP32_VALU_PEAK_TFLOPS,
                    unit="TFLOP/s")
    roof.update(frac=roof["achieved"] / roof["peak"], kernel="batch_kernel",
                traffic=measured_traffic("batch_kernel", f"batch_{len(ues)}ues"),
                algorithmic_bytes=nbytes, algorithmic_flops=flops,
                counters=measured_counters("batch_kernel", "fp32", f"batch_{len(ues)}ues"))
    shapes = [u["shape"] for u in ues]
    out = {
        "metric": "REs/s detected, 64Rx×16L MMSE: FP32 plain vs mixed/learned at ≤0.1 dB loss",
        "value": re / sec, "unit": "RE/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded TDL exponential-PDP channel, Gray QAM, AWGN)",
        "config": {"workload": f"{len(ues)} UEs over 10 cells, one slot each, PRB 4..273 "
                               f"(total {sum(s.n_prb for s in shapes)}), 1..8 layers, Rx 4..64, "
                               f"QPSK..256QAM, SNR 0..30 dB; one persistent launch, HIP graph",
                   "ues": len(ues), "data_re_per_step": re, "path": "batch_persistent_fp32",
                   "work_items": b.n_items, "tile_re": tuned["tile_re"],
                   "autotune_cached": tuned.get("cached", False),
                   "blocks": nb, "data_seconds": round(t_gen, 1)},
        "kernels_ms": {"batch_kernel": ms},
        "roofline": roof,
        "autotune": tuned["table"],
        "variants": {"per_ue_launches": {"value": re / (ms_per_ue * 1e-3), "ms_per_step": ms_per_ue,
                                         "launches_per_step": 3 * len(ues)},
                     "per_ue_receive": {"value": re / (ms_per_ue_rx * 1e-3),
                                        "ms_per_step": ms_per_ue_rx,
                                        "launches_per_step": len(ues)}},
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        n = done = 0
        for u in ues:
            sh = u["shape"]
            hr = oracle.chest_ls(sh, u["rx_h"], u["pil_h"])
            xr, nvr = oracle.mmse_detect(sh, u["rx_h"], hr.astype(np.complex64), oracle.H_PILOT, u["nv_h"])
            oracle.llr_demap(sh, xr.astype(np.complex64), nvr.astype(np.float32))
            n += sh.n_dsym * sh.n_sc
            done += 1
            if time.perf_counter() - t0 >= args.cpu_budget:
                break
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=n / dt, unit="RE/s", cores=oracle.threads(), kind="oracle",
                                   sample=f"{done} of the {len(ues)} UEs ({n} data REs), chest_ls + "
                                          f"mmse_detect (LU route) + llr_demap in FP64, {dt:.1f} s",
                                   host=host_cpu())
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="m", choices=["m", "c2", "c1", "p2", "p4", "p8", "batch"],
                    help="m: 64x16 (default); c1/c2: 4x2 and 16x4; p2/p4/p8: the paper's "
                         "square 2x2/4x4/8x8 at 60 RB, 15 kHz; batch: 200 UEs of uneven "
                         "allocations in one persistent launch (--slots sets the UE count)")
    ap.add_argument("--slots", type=int, default=None, help="override the batch size")
    ap.add_argument("--batch-config", default=None, metavar="TILE_RE,BLOCKS_PER_CU",
                    help="batch workload: use this plan configuration instead of autotuning")
    ap.add_argument("--tune-cache", default=None, metavar="JSON",
                    help="batch workload: autotune cache file (a batch class in it is not "
                         "timed again)")
    ap.add_argument("--h-res", default="pilot", choices=["pilot", "full"])
    ap.add_argument("--prec", default="fp32",
                    choices=["fp32", "fp16", "bf16", "fp16_refined", "bf16_refined"],
                    help="input precision of the detector's Gram and matched filter (the "
                         "refined modes add one iterative-refinement step)")
    ap.add_argument("--path", default="auto", choices=["auto", "fused", "receive", "separate"],
                    help="fused detection + demapping (matrix-core shapes), the whole chain "
                         "in one launch (up to 8 layers) or three calls")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the one-slot latency runs (profiled runs: they launch the same "
                         "kernels at one-slot size)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training and timing the learned estimate refinement")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP16/BF16 detector runs and the SINR comparison")
    ap.add_argument("--train-study", default=None, metavar="SLOTS,SLOTS,..",
                    help="only train the learned refinement on training sets of these sizes "
                         "(one optimisation budget) and report held-out loss and SINR gain")
    ap.add_argument("--study-steps", type=int, default=4096,
                    help="--train-study: Adam steps of two slots each per training set")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter reference)")
    args = ap.parse_args()
    if args.copy_ref:
        import torch
        n = args.copy_ref * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes_each_way": n * 4, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (slots, "
                                   "cells and UEs are independent, so the work shards by slot)"}))
        sys.exit(2)

    import torch
    import paper_2510_07843_amd as ranphy
    import synth

    if args.train_study:
        train_study(args, torch, ranphy, synth)
        return
    if args.workload == "batch":
        bench_batch(args, torch, ranphy, synth)
        return
    t_gen = time.perf_counter()
    b = synth.make_batch(args.workload, n_slots=args.slots, keep_truth=False,
                         workers=min(16, os.cpu_count() or 1))
    t_gen = time.perf_counter() - t_gen
    shape = b["shape"]
    h_res = ranphy.H_PILOT if args.h_res == "pilot" else ranphy.H_FULL
    prec = dict(PRECISIONS(ranphy))[args.prec]
    print(f"# workload {args.workload}: {shape.n_slots} slots {shape.n_rx}x{shape.n_layers} "
          f"{shape.n_prb} PRB qm={shape.qm}; generated in {t_gen:.1f} s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    rx = torch.from_numpy(b["rx"]).to(dev).reshape(-1)
    pil = torch.from_numpy(b["pilots"]).to(dev).reshape(-1)
    nvar = torch.from_numpy(b["noise_var"]).to(dev)
    h = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_H, h_res) // 2, dtype=torch.complex64, device=dev)
    x = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_X) // 2, dtype=torch.complex64, device=dev)
    nv = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_NV), dtype=torch.float32, device=dev)
    llr = torch.empty(ranphy.buffer_floats(shape, ranphy.BUF_LLR), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    if args.path != "auto":
        path = args.path
    elif fused_eligible(shape):
        path = "fused"
    elif ((shape.n_layers <= 4 or (shape.n_occ > 1 and shape.n_layers <= 8))
          and h_res == ranphy.H_PILOT and prec == ranphy.PREC_FP32):
        path = "receive"  # measured faster than the three calls for these shapes
    else:
        path = "separate"
    fused = path == "fused"

    def run_timed(precision, fused, refine=None, one_launch=False):
        """Warm up, then time exactly args.steps steps; returns (ms per step, per-kernel ms).
        refine = (params, min_noise_var, workspace) inserts the learned estimate refinement;
        one_launch times the whole chain as one kernel."""
        names = ("chest_ls", "mmse_llr") if fused else ("chest_ls", "mmse_detect", "llr_demap")
        if one_launch:
            names = ("receive",)
        if refine is not None:
            names = names[:1] + ("cnn_denoise",) + names[1:]
        ev = {n: [] for n in names}

        def step(record):
            marks = ([torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
                     if record else None)
            base = 2 if refine is not None else 1  # mark index after the steps before detection
            if record:
                marks[0].record()
            if one_launch:
                ranphy.receive(shape, rx, pil, nvar, llr=llr)
                if record:
                    marks[1].record()
                    ev["receive"].append((marks[0], marks[1]))
                return
            ranphy.chest_ls(shape, rx, pil, h=h, h_res=h_res)
            if record:
                marks[1].record()
            if refine is not None:
                ranphy.cnn_denoise(shape, refine[0], h, noise_var=nvar, min_noise_var=refine[1],
                                   out=h, workspace=refine[2])
                if record:
                    marks[2].record()
            if fused:
                ranphy.mmse_llr(shape, rx, h, nvar, h_res=h_res, llr=llr, precision=precision)
            else:
                ranphy.mmse_detect(shape, rx, h, nvar, h_res=h_res, x=x, nv=nv,
                                   precision=precision)
                if record:
                    marks[base + 1].record()
                ranphy.llr_demap(shape, x, nv, llr=llr)
            if record:
                marks[-1].record()
                for i, n in enumerate(names):
                    ev[n].append((marks[i], marks[i + 1]))

        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        t_start.record()
        for _ in range(args.steps):
            step(True)
        t_end.record()
        torch.cuda.synchronize()
        return (t_start.elapsed_time(t_end) / args.steps,
                {n: float(np.mean([a.elapsed_time(c) for a, c in ev[n]])) for n in names})

    ms_step, kern_ms = run_timed(prec, fused, one_launch=path == "receive")
    names = tuple(kern_ms)

    costs = algorithmic_costs(shape, h_res)
    re = costs["data_re"]
    value = re / (ms_step * 1e-3)

    # Dominant kernel and its bound: time at the HBM roof vs at the compute roof.
    dom = max(names, key=lambda n: kern_ms[n])
    c = costs[dom]
    on_mfma = dom in ("mmse_detect", "mmse_llr") and fused_eligible(shape)
    compute_peak = FP32_MFMA_PEAK_TFLOPS if on_mfma else FP32_VALU_PEAK_TFLOPS
    t_bytes = c["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_flops = c["flops"] / (compute_peak * 1e12)
    sec = kern_ms[dom] * 1e-3
    if t_bytes >= t_flops:
        roof = dict(bound="hbm", achieved=c["bytes"] / sec / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    else:
        roof = dict(bound="mfma" if on_mfma else "alu",
                    achieved=c["flops"] / sec / 1e12, peak=compute_peak, unit="TFLOP/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    tag = f"{shape.n_rx}x{shape.n_layers}_{shape.n_slots}slots"
    roof["traffic"] = (measured_traffic(dom, tag) if (h_res == ranphy.H_PILOT and prec == ranphy.PREC_FP32)
                       else None)
    roof["algorithmic_bytes"] = c["bytes"]
    roof["algorithmic_flops"] = c["flops"]
    # SQ counters of the same kernel (committed summary): per-wave VALU / MFMA instructions
    # and the shares of the SIMD cycles they occupy (FP32 MFMA and VALU issue do not overlap)
    roof["counters"] = (measured_counters(dom, args.prec, tag) if h_res == ranphy.H_PILOT
                        else None)

    out = {
        "metric": "REs/s detected, 64Rx×16L MMSE: FP32 plain vs mixed/learned at ≤0.1 dB loss",
        "value": value, "unit": "RE/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16 products, f32 accumulate",
                  "bf16": "bf16 products, f32 accumulate",
                  "fp16_refined": "f16 products, f32 accumulate, one f32-residual refinement",
                  "bf16_refined": "bf16 products, f32 accumulate, one f32-residual refinement"
                  }[args.prec], "data": "synthetic (seeded TDL exponential-PDP channel, Gray QAM, AWGN)",
        "config": {"workload": f"{shape.n_rx}Rx x {shape.n_layers}L, {shape.n_prb} PRB x {shape.n_symb} "
                               f"symbols, qm={shape.qm}, DMRS comb {shape.dmrs_comb} x TD {shape.dmrs_td}, "
                               f"{shape.n_slots} slots, h_res={args.h_res}, detector {args.prec}",
                   "slots": shape.n_slots, "data_re_per_step": re,
                   "path": ("plain_fp32" if args.prec == "fp32" else f"mixed_{args.prec}")
                           + "_" + path},
        "kernels_ms": kern_ms,
        "roofline": roof,
    }
    for n in names:
        cc = costs[n]
        out.setdefault("kernel_rates", {})[n] = {
            "GB/s": cc["bytes"] / (kern_ms[n] * 1e-3) / 1e9,
            "TFLOP/s": cc["flops"] / (kern_ms[n] * 1e-3) / 1e12,
            "bytes_per_launch": cc["bytes"], "flops_per_launch": cc["flops"]}
    # the paper's own figures, for context (its hardware, its baseline; not this metric)
    out["paper_context"] = {
        "hardware": "Intel Core i9-14900KF, AVX2 (256-bit SIMD), one CPU",
        "throughput_gain_vs_cpu_only": "about 1.5x (SIMD vs the same vRAN without SIMD)",
        "energy_efficiency_gain_vs_cpu_only": "more than 2x (argued from cited studies)",
        "detection_2x2_us": {"scalar": 3.3, "simd": "< 1.5"},
        "detection_4x4_ms_per_tti": 0.03,
    }
    out["layer_re_per_s"] = value * shape.n_layers
    out["llr_bits_per_s"] = value * shape.n_layers * shape.qm
    if not args.no_latency:
        fused_step = None
        if path == "fused" and h_res == ranphy.H_PILOT:
            def fused_step(words):  # the decompression inside the estimator's and detector's loads
                ranphy.chest_ls_bfp(shape, words, pil, h=h)
                ranphy.mmse_llr_bfp(shape, words, h, nvar, llr=llr, precision=prec)
        elif path == "receive":
            def fused_step(words):  # the one-launch chain decoding the words where it loads them
                ranphy.receive_bfp(shape, words, pil, nvar, llr=llr)
        out["pcie_h2d"] = h2d_rate(torch, b["rx"], ms_step, re, ranphy, shape, fused_step)
        out["slot_latency"] = slot_latency(torch, ranphy, shape, rx, pil, nvar, h_res, prec,
                                           path, scs_hz=synth.CONFIGS[args.workload]["scs_hz"])
    if path == "receive":  # the three-call chain on the same batch, for comparison
        v_ms, v_k = run_timed(prec, False)
        out["variants"] = {"separate": {"value": re / (v_ms * 1e-3), "ms_per_step": v_ms,
                                        "kernels_ms": v_k}}
    if args.workload == "m" and h_res == ranphy.H_PILOT and not args.no_variants:
        variants = {}
        quality = detection_quality(torch, ranphy, synth)
        for name, p in PRECISIONS(ranphy):
            for fz in (True, False):
                key = name + ("" if fz else "_separate")
                if p == prec and fz == fused:
                    v_ms, v_k = ms_step, kern_ms
                else:
                    v_ms, v_k = run_timed(p, fz)
                variants[key] = {"value": re / (v_ms * 1e-3), "ms_per_step": v_ms,
                                 "kernels_ms": v_k}
                variants[key].update(quality[name])
        if path != "receive":  # the whole chain as one launch (pilot rows estimated per block)
            v_ms, v_k = run_timed(ranphy.PREC_FP32, True, one_launch=True)
            variants["fp32_one_launch"] = {"value": re / (v_ms * 1e-3), "ms_per_step": v_ms,
                                           "kernels_ms": v_k}
        if not args.no_learned:
            params, min_nv, report = train_refinement(torch, ranphy, synth, shape)
            nimg = shape.n_rx * shape.n_layers
            # one pass over the batch where the grid has one row (small workspace), else 35 slots
            wsb = ranphy.cnn_workspace_bytes(shape.n_occ, shape.n_pilot, nimg,
                                             shape.n_slots if shape.n_occ == 1
                                             else min(shape.n_slots, 35), False)
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
            v_ms, v_k = run_timed(ranphy.PREC_FP32, fused, refine=(params, min_nv, ws))
            variants["learned_fp32"] = {"value": re / (v_ms * 1e-3), "ms_per_step": v_ms,
                                        "kernels_ms": v_k, "training": report}
            variants["learned_fp32"].update(learned_quality(torch, ranphy, synth, params, min_nv))
        out["variants"] = variants
        out["variants_note"] = ("Gram and matched filter with FP32 / FP16 / BF16 inputs (FP32 "
                                "accumulation, FP32 inversion; _refined: plus one refinement "
                                "step with the FP32 residual), demapping fused into the "
                                "detector or (_separate) as its own pass; SINR = E|x|^2 / "
                                "E|x~ - x|^2 against the transmitted symbols on one slot per "
                                "SNR point (0..30 dB), loss relative to the FP64 oracle on the "
                                "same slots")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
