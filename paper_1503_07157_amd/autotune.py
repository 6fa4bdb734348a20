"""Tile-class tuner for the batched QB (qb_factor_batched).

Each product role of a block iteration (sample, Gram, T^{-1} application,
the two re-projection products, B_i, downdate) takes one output tile class
per panel-width class (w <= 16, <= 32, <= 64); see qb_batched_set_tile in
include/qb.h.  The tuner measures the caller's own batch: coordinate descent
over the (role, width class) entries that the batch uses, timing the whole
batched factorisation for every allowed class of one entry while the others
stay at their current best, and keeping the fastest.  Every allowed class
computes the same products, so tuning changes speed, and results only in the
last bits.
"""
from __future__ import annotations

import time

import torch

from . import _lib
from .qb import batched_tiles, qb_factor_batched, set_batched_tiles


def _time_batch(As, eps, bs, seeds, repeats):
    best = float("inf")
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        qb_factor_batched(As, eps, bs, seeds)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_batched(As, eps, bs, seeds, repeats: int = 2, rounds: int = 1, log=None):
    """Tune the tile table on this batch; leaves the best table set and
    returns (table, seconds_before, seconds_after, measurements)."""
    widths = sorted({0 if b <= 16 else 1 if b <= 32 else 2 for b in bs})
    qb_factor_batched(As, eps, bs, seeds)  # warm-up
    best_t = _time_batch(As, eps, bs, seeds, repeats)
    start_t = best_t
    trials = 0
    for _ in range(rounds):
        changed = False
        for role in _lib.BATCH_ROLES:
            for wc in widths:
                current = batched_tiles()[role][wc]
                for name in _lib.BATCH_TILES:
                    if name == current:
                        continue
                    entry = [None, None, None]
                    entry[wc] = name
                    try:
                        set_batched_tiles({role: entry})
                    except _lib.QBError:
                        continue  # not allowed for this role
                    t = _time_batch(As, eps, bs, seeds, repeats)
                    trials += 1
                    if log:
                        log(f"[tune] {role} w-class {wc}: {name} {t * 1e3:.1f} ms "
                            f"(best {current} {best_t * 1e3:.1f} ms)")
                    if t < best_t:
                        best_t, current, changed = t, name, True
                    else:
                        entry[wc] = current
                        set_batched_tiles({role: entry})
        if not changed:
            break
    return batched_tiles(), start_t, best_t, trials
