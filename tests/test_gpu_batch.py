"""GPU parity of the multi-UE persistent launch (ranphy_batch_*): every UE's LLRs against the
FP64 oracle chain on that UE's slot, to the end-to-end bar of the single-UE tests (hard
decisions bit-exact away from decision boundaries, every LLR within 1e-3 |LLR| + 1e-4 of the
oracle's or inside the range the FP32 forward-error bound of its Gram allows, tests/parity.py);
allocations up to the full 273 PRB; graph replay; independence of the result from the tile
size and the grid."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2510_07843_amd as ranphy
import synth
from synth import SlotShape
import parity
from parity import say
from paper_2510_07843_amd import tune

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu_ready():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ranphy.lib()


def make_ues(n, seed, max_prb=273):
    """UEs of random allocations: 4..max_prb PRB, 1..8 layers, 4..64 antennas, QPSK..256QAM,
    SNR 0..30 dB; one DMRS occasion (comb and cover by the layer count) or, for up to two
    layers, two single-symbol occasions (a time-varying channel estimate)."""
    rng = np.random.default_rng(seed)
    ues = []
    for i in range(n):
        nl = int(rng.integers(1, 9))
        nr = int(rng.choice([r for r in (4, 8, 16, 32, 64) if r >= nl]))
        qm = int(rng.choice([2, 4, 6, 8]))
        prb = int(rng.integers(4, max_prb + 1))
        comb, td = (2, 1) if nl <= 2 else ((2, 2) if nl <= 4 else (4, 2))
        occ = (2, 11) if (nl <= 2 and rng.uniform() < 0.5) else (2,)
        shape = SlotShape(prb, 14, nr, nl, qm, comb, td, occ, 1)
        snr = float(rng.uniform(0, 30))
        d = synth.make_slot(shape, synth.rng_for(9, seed, i), 30e3, ("exp", 100e-9), snr)
        ues.append(dict(shape=shape, rx_h=d["rx"][None], pil_h=d["pilots"][None],
                        nv_h=np.array([d["noise_var"]], np.float32),
                        rx=torch.from_numpy(d["rx"]).cuda().reshape(-1),
                        pilots=torch.from_numpy(d["pilots"]).cuda().reshape(-1),
                        noise_var=torch.tensor([d["noise_var"]], dtype=torch.float32,
                                               device="cuda")))
    return ues


def oracle_ref(u):
    sh = u["shape"]
    hr = oracle.chest_ls(sh, u["rx_h"], u["pil_h"]).astype(np.complex64)
    xr, nvr = oracle.mmse_detect(sh, u["rx_h"], hr, oracle.H_PILOT, u["nv_h"])
    lr = oracle.llr_demap(sh, xr.astype(np.complex64), nvr.astype(np.float32))
    return hr, xr, nvr, lr


def test_batch_matches_oracle_per_ue():
    # 24 UEs of 4..273 PRB (the workload's allocation range), 1..8 layers, 4..64 antennas.
    ues = make_ues(24, seed=1)
    b = ranphy.Batch(ues, tile_re=512)
    say(f"batch of {len(ues)} UEs ({sum(u['shape'].n_prb for u in ues)} PRB), "
        f"{b.n_items} work items")
    b.run(256 * 2)
    torch.cuda.synchronize()
    assert max(u["shape"].n_prb for u in ues) > 200
    for i, u in enumerate(ues):
        sh = u["shape"]
        lg = u["llr"].cpu().numpy().reshape(1, sh.n_dsym, sh.n_sc, sh.n_layers, sh.qm)
        hr, xr, nvr, lr = oracle_ref(u)
        grams = parity.gram_fn(sh, hr, oracle.H_PILOT, u["nv_h"])
        parity.audit_llrs(lg, lr, xr, nvr,
                          parity.kappa_radius(grams, xr.reshape(-1, sh.n_layers), sh.n_layers),
                          sh.qm, f"UE {i}: {sh.n_prb} PRB {sh.n_rx}x{sh.n_layers} qm {sh.qm} "
                                 f"occ {sh.dmrs_sym0}")


def test_batch_bench_workload_sampled():
    # The 200-UE workload the benchmark times, at the plan its profiles use (tile of 2048
    # REs, 3 blocks per compute unit; other tiles give the same bits, test below) and replayed
    # from a HIP graph as the benchmark does; a sample of UEs against the oracle chain: the
    # first, middle and last, the largest allocation, and the first UE of one layer and of
    # eight.
    import bench
    ues = bench.make_batch_ues(torch, synth, n_ue=200)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    b = ranphy.Batch(ues, tile_re=2048)
    say(f"bench batch: {len(ues)} UEs, {b.n_items} work items, {3 * cus} blocks")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run(3 * cus)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = [u["llr"].clone() for u in ues]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(3 * cus)
    for u in ues:
        u["llr"].fill_(-3.0)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for u, r in zip(ues, ref):
        assert torch.equal(u["llr"].view(torch.int32), r.view(torch.int32))
    pick = {0, len(ues) // 2, len(ues) - 1,
            max(range(len(ues)), key=lambda i: ues[i]["shape"].n_prb * ues[i]["shape"].n_rx)}
    for nl in (1, 8):
        pick.add(next(i for i, u in enumerate(ues) if u["shape"].n_layers == nl))
    for i in sorted(pick):
        u = ues[i]
        sh = u["shape"]
        lg = u["llr"].cpu().numpy().reshape(1, sh.n_dsym, sh.n_sc, sh.n_layers, sh.qm)
        hr, xr, nvr, lr = oracle_ref(u)
        grams = parity.gram_fn(sh, hr, oracle.H_PILOT, u["nv_h"])
        parity.audit_llrs(lg, lr, xr, nvr,
                          parity.kappa_radius(grams, xr.reshape(-1, sh.n_layers), sh.n_layers),
                          sh.qm, f"bench UE {i}: {sh.n_prb} PRB {sh.n_rx}x{sh.n_layers} qm {sh.qm}")


def test_batch_graph_replay_and_grid_independence():
    ues = make_ues(10, seed=2, max_prb=24)
    b = ranphy.Batch(ues, tile_re=256)
    b.run(256)
    torch.cuda.synchronize()
    ref = [u["llr"].clone() for u in ues]
    # another tile size and grid: the same arithmetic per RE, so the same bits
    b2 = ranphy.Batch(ues, tile_re=2048)
    for u in ues:
        u["llr"].fill_(7.0)
    b2.run(37)
    torch.cuda.synchronize()
    for u, r in zip(ues, ref):
        assert torch.equal(u["llr"].view(torch.int32), r.view(torch.int32))
    # HIP graph of the reset and the persistent kernel, replayed with eager work in between
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run(256)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(256)
    for rep in range(3):
        for u in ues:
            u["llr"].fill_(float(rep) - 5.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for u, r in zip(ues, ref):
            assert torch.equal(u["llr"].view(torch.int32), r.view(torch.int32)), rep


def test_batch_eight_byte_aligned_grids():
    # UEs whose received grid sits 8 bytes past a 16-byte boundary (the library's minimum
    # alignment) take the 8-byte pieces of the group line loads; their LLRs must equal those
    # of the same UEs with aligned grids bit for bit.
    ues = make_ues(8, seed=4, max_prb=16)
    b = ranphy.Batch(ues, tile_re=512)
    b.run(256)
    torch.cuda.synchronize()
    ref = [u["llr"].clone() for u in ues]
    keep = []
    for u in ues:
        big = torch.empty(u["rx"].numel() + 1, dtype=torch.complex64, device="cuda")
        big[1:] = u["rx"]
        keep.append(big)
        u["rx"] = big[1:]
        assert u["rx"].data_ptr() % 16 == 8
        u["llr"] = None
    b2 = ranphy.Batch(ues, tile_re=512)
    b2.run(256)
    torch.cuda.synchronize()
    assert any(u["shape"].n_rx % 16 == 0 for u in ues)
    for u, r in zip(ues, ref):
        assert torch.equal(u["llr"].view(torch.int32), r.view(torch.int32))


def test_autotune_returns_a_valid_configuration():
    ues = make_ues(12, seed=3, max_prb=32)
    res = tune.autotune(ues, tiles=(256, 1024), blocks_per_cu=(1, 3), reps=2)
    say(f"autotune: {res['table']} -> tile {res['tile_re']} x {res['blocks_per_cu']} blocks/CU")
    assert len(res["table"]) == 4 and res["ms"] > 0
    ref = [u["llr"].clone() for u in ues]
    res["batch"].run(res["n_blocks"])
    torch.cuda.synchronize()
    for u, r in zip(ues, ref):
        assert torch.equal(u["llr"].view(torch.int32), r.view(torch.int32))


def test_autotune_cache_times_a_class_once(tmp_path):
    # The first batch of a class is timed and stored; a second batch of the same class (the
    # same UE kinds, another order and PRB split) is planned from the cache untimed, and its
    # LLRs equal those of the same plan built directly.
    f = str(tmp_path / "tune.json")
    ues = make_ues(8, seed=4, max_prb=32)
    first = tune.autotune(ues, tiles=(256, 512), blocks_per_cu=(1, 2), reps=2, cache=f)
    assert not first["cached"]
    again = [dict(u) for u in reversed(ues)]
    for u in again:
        u.pop("llr", None)
    second = tune.autotune(again, tiles=(256, 512), blocks_per_cu=(1, 2), reps=2, cache=f)
    assert second["cached"]
    assert (second["tile_re"], second["blocks_per_cu"]) == (first["tile_re"], first["blocks_per_cu"])
    second["batch"].run(second["n_blocks"])
    got = [u["llr"].clone() for u in again]
    for u in again:
        u["llr"] = None
    direct = ranphy.Batch(again, tile_re=second["tile_re"])
    direct.run(second["n_blocks"])
    torch.cuda.synchronize()
    for a, u in zip(got, again):
        assert torch.equal(a, u["llr"])
