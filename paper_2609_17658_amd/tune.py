"""Autotuner of the walk's launch shape, for a batch of boxes and for a
single tree.

It searches the targets per wavefront group (``group_max``), the leaf size
(``leaf_max``) and the mixed walk's per-target list depth
(``walk_list_cap``) by timing, with HIP events, replays of a batch's
captured graph (build + walk of every box) or the build and walk of one
tree, and keeps the fastest.  ``group_max`` and ``walk_list_cap`` do not
change any result; ``leaf_max`` does (the tree is a different one), so a
tuned leaf size must be checked against the oracle at that leaf size, and
``tune_tree(fixed_leaf=...)`` keeps a prescribed one.

Choices are cached in a JSON file keyed by the device (name, architecture,
compute units) and the problem (N rounded to a power of two, precision,
periodicity, theta, r_cut / r_s, curve): ``OG_TUNE_CACHE`` names the file,
by default ``~/.cache/paper_2609_17658_amd/tune.json``.
"""
from __future__ import annotations

import itertools
import json
import math
import os
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


TREE_SPACE = {"group_max": [32, 64], "walk_list_cap": [4, 8], "leaf_max": [4, 8, 16]}


def time_tree(pos, mass, box, params, group_max=64, walk_list_cap=4, leaf_max=None, precision="mixed",
              reps=3, workspace=None):
    """Mean ms of og_tree_build + og_tree_force on every particle for one
    setting (HIP events on torch's current stream)."""
    import torch

    from . import og

    p = dict(params)
    if leaf_max is not None:
        p["leaf_max"] = leaf_max
    p.update(group_max=group_max, walk_list_cap=walk_list_cap, precision=precision)
    stream = torch.cuda.current_stream()
    n = int(pos.shape[0])
    ws = workspace
    need = og.og_tree_workspace_bound(n, og.make_params(p))
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=pos.device)
    acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    pot = torch.empty(n, dtype=torch.float64, device=pos.device)

    def step():
        t = og.Tree(pos, mass, box, p, stream=stream, workspace=ws)
        t.force(acc=acc, pot=pot)
        return t

    step().close()  # warm-up
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    trees = []
    ev[0].record(stream)
    for _ in range(reps):
        trees.append(step())
    ev[1].record(stream)
    torch.cuda.synchronize()
    status = trees[-1].status()
    for t in trees:
        t.close()
    if status != 0:
        raise RuntimeError("tree status %d" % status)
    return ev[0].elapsed_time(ev[1]) / reps


def tune_tree(pos, mass, box, params, space=None, precision="mixed", reps=3, fixed_leaf=None, log=None):
    """Time every combination of `space` (leaf_max held at `fixed_leaf` when
    given); returns {"best": {...}, "trials": [...], "seconds": s}."""
    space = dict(space or TREE_SPACE)
    if fixed_leaf is not None:
        space["leaf_max"] = [fixed_leaf]
    keys = list(space)
    trials = []
    t0 = time.time()
    for vals in itertools.product(*(space[k] for k in keys)):
        cfg = dict(zip(keys, vals))
        ms = time_tree(pos, mass, box, params, precision=precision, reps=reps, **cfg)
        trials.append(dict(cfg, ms=ms))
        if log:
            log("tune tree %s: %.3f ms" % (cfg, ms))
    best = min(trials, key=lambda t: t["ms"])
    return {"best": best, "trials": trials, "seconds": time.time() - t0}


def device_key():
    import torch

    pr = torch.cuda.get_device_properties(0)
    arch = getattr(pr, "gcnArchName", "") or ""
    return "%s|%s|%d" % (pr.name, arch.split(":")[0], pr.multi_processor_count)


def problem_key(n, params, precision, kind="tree"):
    p = dict(params)
    r_s = p.get("r_s", 0.0)
    rc = p.get("r_cut", 0.0) or 4.5 * r_s
    return "%s|N2^%d|%s|per%d|theta%.2f|rc/rs%.2f|curve%s" % (
        kind, int(round(math.log2(max(int(n), 1)))), precision, int(p.get("periodic", 1)),
        float(p.get("theta", 0.5)), rc / r_s if r_s > 0 else 0.0, p.get("curve", 0))


def cache_path():
    return os.environ.get("OG_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                            "paper_2609_17658_amd", "tune.json")


def cache_get(key, path=None):
    try:
        with open(path or cache_path()) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def cache_put(key, value, path=None):
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data[key] = value
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_tree_settings(pos, mass, box, params, precision="mixed", fixed_leaf=None, reps=3, log=None,
                        path=None):
    """The cached choice for this device and problem, or a fresh search
    stored in the cache."""
    key = device_key() + "||" + problem_key(pos.shape[0], params, precision) + (
        "|leaf%d" % fixed_leaf if fixed_leaf is not None else "")
    hit = cache_get(key, path)
    if hit is not None:
        return dict(hit, cached=True)
    res = tune_tree(pos, mass, box, params, precision=precision, reps=reps, fixed_leaf=fixed_leaf, log=log)
    val = {"best": res["best"], "trials": res["trials"]}
    cache_put(key, val, path)
    return dict(val, cached=False)
