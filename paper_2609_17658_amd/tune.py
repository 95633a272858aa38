"""Autotuner of the walk's launch shape for a batch of boxes.

It searches the targets per wavefront group (``group_max``), the leaf size
(``leaf_max``) and the mixed walk's per-target list depth
(``walk_list_cap``) by timing replays of the batch's captured graph (build +
walk of every box) with HIP events, and keeps the fastest.  ``group_max``
and ``walk_list_cap`` do not change any result; ``leaf_max`` does (the tree
is a different one), so a tuned leaf size must be checked against the oracle
at that leaf size.
"""
from __future__ import annotations

import itertools
import time

DEFAULT_SPACE = {"group_max": [32, 64], "walk_list_cap": [4, 8], "leaf_max": [8, 16]}


def time_batch(items, group_max=64, walk_list_cap=4, leaf_max=None, precision="mixed", reps=3,
               stream=None):
    """Mean ms per graph replay (build + walk of every box) for one setting.
    items: list of (pos, mass, box, params-dict) with device tensors."""
    import torch

    from . import og

    stream = stream or torch.cuda.Stream()
    prepared = []
    for pos, mass, box, prm in items:
        p = dict(prm)
        if leaf_max is not None:
            p["leaf_max"] = leaf_max
        prepared.append((pos, mass, box, p))
    with torch.cuda.stream(stream):
        bt = og.Batch(prepared, stream=stream, precision=precision, group_max=group_max,
                      walk_list_cap=walk_list_cap)
        bt.replay()  # capture + first replay
        stream.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            bt.replay()
        ev[1].record(stream)
        stream.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        status = bt.status()
        bt.close()
    if status != 0:
        raise RuntimeError("batch status %d" % status)
    return ms


def tune_batch(items, space=None, precision="mixed", reps=3, log=None):
    """Try every combination of `space`; returns {"best": {...}, "trials": [...]}."""
    space = space or DEFAULT_SPACE
    keys = list(space)
    trials = []
    t0 = time.time()
    for vals in itertools.product(*(space[k] for k in keys)):
        cfg = dict(zip(keys, vals))
        ms = time_batch(items, precision=precision, reps=reps, **cfg)
        trials.append(dict(cfg, ms=ms))
        if log:
            log("tune %s: %.3f ms" % (cfg, ms))
    best = min(trials, key=lambda t: t["ms"])
    return {"best": best, "trials": trials, "seconds": time.time() - t0}
