"""Tile autotuner of the multi-UE persistent launch.

For a given batch of UEs it builds a plan for each candidate tile size (resource elements per
work item), times every (tile size, blocks per compute unit) pair with HIP events on the
current stream, and returns the fastest.  The timing runs the library's own kernels; the
candidates are the tile sizes the planner accepts and the block counts the kernel's LDS and
registers allow per compute unit (3 of 256 threads).
"""
from __future__ import annotations

from typing import Dict, Sequence

import torch

from . import Batch

TILES = (128, 256, 512, 1024, 2048)
BLOCKS_PER_CU = (1, 2, 3)


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
             reps: int = 5) -> Dict:
    """Returns the fastest configuration, its plan and the table of every candidate (ms)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
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
    return dict(tile_re=t, blocks_per_cu=bpc, n_blocks=cus * bpc, ms=ms, batch=b, table=table)
