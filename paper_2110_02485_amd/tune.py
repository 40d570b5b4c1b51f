"""Autotuner of the R-tSVD restoration's work split on the device at hand.

Two options of the factorization change only how the work is divided, never a result (bit for
bit, which tune() checks):
  * face_groups, the schedule: the per-face work issued as 1, 2 or 3 concurrent groups of faces on
    the library's streams, staggered so that one group's passes over A-hat overlap another group's
    latency-bound kernels (Gram, Cholesky, eigensolver);
  * sketch_tile, the tile shape: 1, 2, 4 or 8 sixteen-column MFMA tiles per workgroup in the
    products with A-hat (sketch, power step, projection, Q = Y R^-1, W = A-hat V).  Fewer columns
    per workgroup give more workgroups but read A-hat once per column tile.
tune() times every candidate pair the way the benchmark times a step (restorations, factor and
solve, issued back to back on the current stream between two events), keeps the best of `rounds`
runs per candidate and returns the fastest pair with the whole table.
"""
from __future__ import annotations

import torch

from . import rtsvd as rt


def candidates(r: int, faces: int):
    """(face_groups, sketch_tile) pairs worth timing for sketch width r and `faces` Fourier faces:
    group counts that leave at least four faces per group, tile counts up to the first that covers
    r columns (wider ones only add zero padding)."""
    groups = [g for g in (1, 2, 3) if g == 1 or faces >= 4 * g]
    tiles = [t for t in (1, 2, 4, 8) if t == 1 or 16 * (t // 2) < r]
    return [(g, t) for g in groups for t in tiles]


def _restorations(A, B, omega, k_max, oversample, power_iters, precision, delta, eta, groups, tile, count):
    last, res = None, None
    for _ in range(count):
        f = rt.factor(A, k_max, oversample, power_iters, precision, omega, face_groups=groups, sketch_tile=tile)
        res = f.solve(B, delta, eta, 1)
        if last is not None:
            last.close()
        last = f
    return last, res


def tune(A, B, omega, k_max: int, oversample: int, power_iters: int, precision: str, delta: float, eta: float,
         steps: int = 4, rounds: int = 2) -> dict:
    """Time every candidate (candidates()) on the device tensors A, B, omega (storage order, as
    rtsvd.factor takes them) and return {"face_groups", "sketch_tile", "ms_per_step", "identical",
    "table"}: the fastest pair, its time per restoration, whether every candidate's X equalled the
    first candidate's bit for bit, and the best time of every candidate (ms)."""
    r = min(k_max + oversample, A.shape[1])
    faces = A.shape[0] // 2 + 1
    table: dict = {}
    ref = None
    identical = True
    args = (A, B, omega, k_max, oversample, power_iters, precision, delta, eta)
    for _ in range(rounds):
        for g, t in candidates(r, faces):
            f, _ = _restorations(*args, g, t, 1)           # warm-up (scratch buffers, code objects)
            f.close()
            torch.cuda.synchronize()
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record()
            f, res = _restorations(*args, g, t, steps)
            end.record()
            torch.cuda.synchronize()
            ms = start.elapsed_time(end) / steps
            if ref is None:
                ref = res.X.clone()
            elif not torch.equal(res.X, ref):
                identical = False
            f.close()
            table[(g, t)] = min(ms, table.get((g, t), float("inf")))
    best = min(table, key=table.get)
    return {"face_groups": best[0], "sketch_tile": best[1], "ms_per_step": table[best], "identical": identical,
            "table": {f"groups{g}_tile{t}": round(ms, 4) for (g, t), ms in table.items()}}
