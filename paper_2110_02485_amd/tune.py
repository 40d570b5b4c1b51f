"""Autotuner of the R-tSVD restoration's work split and schedule on the device at hand.

Three options change only how the work is divided and issued, never a result (bit for bit, which
tune() checks):
  * face_groups, the schedule inside one restoration: the per-face work issued as 1, 2 or 3
    concurrent groups of faces on the library's streams, staggered so that one group's passes
    over A-hat overlap another group's latency-bound kernels (Gram, Cholesky, eigensolver);
  * sketch_tile, the tile shape: 1, 2, 4 or 8 sixteen-column MFMA tiles per workgroup in the
    products with A-hat (sketch, power step, projection, Q = Y R^-1, W = A-hat V).  Fewer columns
    per workgroup give more workgroups but read A-hat once per column tile;
  * in_flight, the schedule across restorations: consecutive independent restorations issued
    round robin on 1, 2 or 3 caller streams, so that one restoration's latency-bound eigensolver
    and Cholesky kernels (one workgroup per face, a quarter of the CUs) overlap the next one's
    bandwidth-bound passes.  Only with one face group: a call with one group keeps all of its work
    on its caller's stream, while the face-group streams are shared by every call on the device
    (and a process gets four hardware queues by default: more streams than that serialize).
tune() times every candidate the way the benchmark times its steps (restorations, factor and
solve, issued back to back between two events on the current stream, which every caller stream
waits for and joins back into), keeps the best of `rounds` runs per candidate and returns the
fastest with the whole table.
"""
from __future__ import annotations

import torch

from . import rtsvd as rt

MAX_IN_FLIGHT = 3
_streams: dict = {}


def caller_streams(n: int, device=None) -> list:
    """n caller streams (default priority) of the current device, created once and kept."""
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    pool = _streams.setdefault(dev, [])
    while len(pool) < n:
        pool.append(torch.cuda.Stream(device=dev))
    return pool[:n]


def candidates(r: int, faces: int):
    """(face_groups, sketch_tile, in_flight) triples worth timing for sketch width r and `faces`
    Fourier faces: group counts that leave at least four faces per group, tile counts up to the
    first that covers r columns (wider ones only add zero padding), and 2 or 3 restorations in
    flight for one face group."""
    groups = [g for g in (1, 2, 3) if g == 1 or faces >= 4 * g]
    tiles = [t for t in (1, 2, 4, 8) if t == 1 or 16 * (t // 2) < r]
    out = [(g, t, 1) for g in groups for t in tiles]
    out += [(1, t, s) for t in tiles for s in range(2, MAX_IN_FLIGHT + 1)]
    return out


def restorations(A, B, omega, k_max, oversample, power_iters, precision, delta, eta, groups, tile, in_flight,
                 count, start=None):
    """`count` restorations (factor + solve) issued round robin on `in_flight` caller streams
    (the current stream when in_flight is 1).  Every caller stream first waits for `start` (an
    event recorded on the current stream) and the current stream finally waits for every caller
    stream, so events on the current stream bracket all of the work.  Returns the last factor
    (the others are closed) and the list of results."""
    cur = torch.cuda.current_stream()
    streams = [cur] if in_flight <= 1 else caller_streams(in_flight)
    if start is not None:
        for s in streams:
            if s != cur:
                s.wait_event(start)
    last, results = None, []
    for i in range(count):
        with torch.cuda.stream(streams[i % len(streams)]):
            f = rt.factor(A, k_max, oversample, power_iters, precision, omega, face_groups=groups, sketch_tile=tile)
            results.append(f.solve(B, delta, eta, 1))
        if last is not None:
            last.close()
        last = f
    for s in streams:
        if s != cur:
            cur.wait_stream(s)
    return last, results


def tune(A, B, omega, k_max: int, oversample: int, power_iters: int, precision: str, delta: float, eta: float,
         steps: int = 6, rounds: int = 2) -> dict:
    """Time every candidate (candidates()) on the device tensors A, B, omega (storage order, as
    rtsvd.factor takes them) and return {"face_groups", "sketch_tile", "in_flight", "ms_per_step",
    "identical", "table"}: the fastest triple, its time per restoration, whether every
    restoration's X equalled the first candidate's bit for bit, and the best time of every
    candidate (ms)."""
    r = min(k_max + oversample, A.shape[1])
    faces = A.shape[0] // 2 + 1
    table: dict = {}
    ref = None
    identical = True
    args = (A, B, omega, k_max, oversample, power_iters, precision, delta, eta)
    for _ in range(rounds):
        for g, t, s in candidates(r, faces):
            f, _ = restorations(*args, g, t, s, s)         # warm-up (scratch buffers of every stream)
            f.close()
            torch.cuda.synchronize()
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record()
            f, res = restorations(*args, g, t, s, steps, start)
            end.record()
            torch.cuda.synchronize()
            ms = start.elapsed_time(end) / steps
            for out in res:
                if ref is None:
                    ref = out.X.clone()
                elif not torch.equal(out.X, ref):
                    identical = False
            f.close()
            table[(g, t, s)] = min(ms, table.get((g, t, s), float("inf")))
    best = min(table, key=table.get)
    return {"face_groups": best[0], "sketch_tile": best[1], "in_flight": best[2], "ms_per_step": table[best],
            "identical": identical,
            "table": {f"groups{g}_tile{t}_inflight{s}": round(ms, 4) for (g, t, s), ms in table.items()}}
