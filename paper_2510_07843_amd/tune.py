"""Tile autotuner of the multi-UE persistent launch.

For a given batch of UEs it builds a plan for each candidate tile size (resource elements per
work item), times every (tile size, blocks per compute unit) pair with HIP events on the
current stream, and returns the fastest.  The timing runs the library's own kernels; the
candidates are the tile sizes the planner accepts and the block counts the kernel's LDS and
registers allow per compute unit (3 of 256 threads).

With a cache file the choice is kept per batch class (the GPU, and the batch's mix of UE
shapes and size), so that a class is timed once: a later batch of the same class is planned
with the cached tile size and block count without timing anything.
"""
from __future__ import annotations

import json
import math
import os
from collections import Counter
from typing import Dict, Optional, Sequence

import torch

from . import Batch, abi_version

TILES = (128, 256, 512, 1024, 2048)
BLOCKS_PER_CU = (1, 2, 3)
CACHE_VERSION = 1


def batch_class(shapes, device_name: str, cus: int) -> str:
    """Key of a batch's class: the GPU (name, compute units), the library ABI, the multiset of
    UE kinds (receive antennas, layers, DMRS occasions, comb x cover, modulation order) and the
    total data REs rounded to two significant bits (the plan's work items scale with it)."""
    kinds = Counter((s.n_rx, s.n_layers, len(s.dmrs_sym0), s.dmrs_comb * s.dmrs_td, s.qm)
                    for s in shapes)
    re = sum(s.n_dsym * s.n_sc for s in shapes)
    e = max(0, int(math.floor(math.log2(max(re, 1)))) - 1)
    re_class = (re >> e) << e
    return json.dumps(dict(device=device_name, cus=cus, abi=abi_version(),
                           kinds=sorted([list(k) + [n] for k, n in kinds.items()]),
                           data_re=re_class), sort_keys=True)


def load_cache(path: str) -> Dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    return d.get("entries", {}) if d.get("version") == CACHE_VERSION else {}


def store_cache(path: str, key: str, entry: Dict) -> None:
    entries = load_cache(path)
    entries[key] = entry
    tmp = path + ".tmp"
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(tmp, "w") as f:
        json.dump(dict(version=CACHE_VERSION, entries=entries), f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_run(batch: Batch, n_blocks: int, reps: int = 5) -> float:
    for _ in range(2):
        batch.run(n_blocks)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        batch.run(n_blocks)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def autotune(ues, tiles: Sequence[int] = TILES, blocks_per_cu: Sequence[int] = BLOCKS_PER_CU,
             reps: int = 5, cache: Optional[str] = None) -> Dict:
    """Returns the fastest configuration, its plan and the table of every candidate (ms).
    With `cache` (a JSON file), a batch whose class is in it is planned with the cached
    configuration untimed (``cached`` True), and a timed result is added to it."""
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    key = batch_class([u["shape"] for u in ues], props.name, cus) if cache else None
    if cache:
        hit = load_cache(cache).get(key)
        if hit is not None:
            b = Batch(ues, tile_re=hit["tile_re"])
            return dict(tile_re=hit["tile_re"], blocks_per_cu=hit["blocks_per_cu"],
                        n_blocks=cus * hit["blocks_per_cu"], ms=hit["ms"], batch=b,
                        table=hit["table"], cached=True)
    table = []
    best = None
    for t in tiles:
        b = Batch(ues, tile_re=t)
        for bpc in blocks_per_cu:
            ms = time_run(b, cus * bpc, reps)
            table.append(dict(tile_re=t, blocks_per_cu=bpc, items=b.n_items, ms=round(ms, 4)))
            if best is None or ms < best[0]:
                best = (ms, t, bpc, b)
    ms, t, bpc, b = best
    if cache:
        store_cache(cache, key, dict(tile_re=t, blocks_per_cu=bpc, ms=ms, table=table))
    return dict(tile_re=t, blocks_per_cu=bpc, n_blocks=cus * bpc, ms=ms, batch=b, table=table,
                cached=False)
