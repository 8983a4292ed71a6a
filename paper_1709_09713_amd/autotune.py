"""Launch-shape autotuner for the fused stage kernel.

For one grid size and storage precision, times every candidate launch shape
(tile of ns_set_fused_config's table x z-chunk length) on a scratch
Taylor-Green solve running the real RK3 launches (one member of a
one-stream batch), and keeps the fastest.  Results are cached per
(grid, precision) in memory and optionally in a JSON file, so a serving
process tunes each grid size once.  Every candidate computes the same
result (the tiling only changes which block computes which point), so the
choice affects speed only.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import _native as nat
from .batch import Batch

DEFAULT_ZCHUNKS = (0, 6, 11)   # 0 = the library's default for the grid


def _key(n, precision):
    n = (n, n, n) if isinstance(n, int) else tuple(n)
    return n, f"{n[0]}x{n[1]}x{n[2]}:{precision}"


class Autotuner:
    def __init__(self, cache_path: str | None = None, tiles=None, zchunks=DEFAULT_ZCHUNKS,
                 steps: int = 3, reps: int = 3):
        self.cache_path = cache_path
        self.tiles = tuple(nat.TILES) if tiles is None else tuple(tiles)
        self.zchunks = tuple(zchunks)
        self.steps = steps
        self.reps = reps
        self.table = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.table = json.load(f)

    def lookup(self, n, precision):
        """(tile, zchunk) for this grid, tuning it on first use."""
        n, key = _key(n, precision)
        if key not in self.table:
            self.table[key] = self.tune(n, precision)
            self.save()
        e = self.table[key]
        return e["tile"], e["zchunk"]

    def save(self):
        if self.cache_path:
            tmp = self.cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, self.cache_path)

    def tune(self, n, precision):
        n, _ = _key(n, precision)
        stream = torch.cuda.current_stream()
        state = torch.empty((5, n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
        p = nat.make_params(n)
        work = torch.empty(nat.ns_workspace_bytes(p, nat.NS_ALGO_FUSED, nat.PRECS[precision]),
                           dtype=torch.uint8, device="cuda")
        dt = 1e-4
        timings = []
        t_wall = time.perf_counter()
        for tile in self.tiles:
            for zc in self.zchunks:
                if zc and zc > n[2]:
                    continue
                b = Batch(1, precision, nstreams=1)
                try:
                    nat.tgv_init(p, state, stream)
                    big = self.steps * (self.reps + 1)
                    slot = nat.ns_batch_add(b.handle, p, dt, big, state, work, tile=tile,
                                            zchunk=zc)
                    b.step(self.steps, stream)          # warm-up
                    best = float("inf")
                    for _ in range(self.reps):
                        e0 = torch.cuda.Event(enable_timing=True)
                        e1 = torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        b.step(self.steps, stream)
                        e1.record(stream)
                        e1.synchronize()
                        best = min(best, e0.elapsed_time(e1) / self.steps)
                    nat.ns_batch_remove(b.handle, slot)
                finally:
                    b.close()
                timings.append((best, tile, zc))
        timings.sort()
        best, tile, zc = timings[0]
        dtile = nat.ns_get_fused_config(p, nat.PRECS[precision])[0]
        dflt = [t for t, tl, z in timings if z == 0 and tl == dtile]
        return {"tile": tile, "zchunk": zc, "ms_per_step": best,
                "default_ms_per_step": dflt[0] if dflt else None,
                "candidates": len(timings), "tune_seconds": time.perf_counter() - t_wall,
                "ranking": [[round(t, 5), tl, z] for t, tl, z in timings[:6]]}
