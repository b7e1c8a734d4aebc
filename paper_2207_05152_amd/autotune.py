"""Autotuner of the batched launch: picks the coder layout per image size and
the density grid by timing captured graphs, and caches the choice as JSON.

Knobs (read by the library through dlic_batch_create and dlic_batch_tune):
  * rows per group: an image of height h is split into ceil(h / rows) row
    groups (more groups = more workgroups per image and a shorter decode
    span; each group adds 32 or 64 flushed states to the stream);
  * lanes per group: 2, 4, 32 or 64 interleaved rANS states (a group's
    sub-round covers that many rows of one wavefront step);
  * density grid: workgroups of the persistent density kernel;
  * search fan-out: coder lanes per pixel in the decoder's symbol search, 16
    (one level of a 16-level bucket per lane; layouts of at most 4 lanes) or
    2 (binary halvings split over two half-waves), 0 for the library default;
  * decode grid: workgroups of the persistent decode kernel, 0 for as many
    as stay resident.

The search is coordinate-wise: every (rows, lanes) layout with default
grids and fan-out first, then the other knobs on the best layout.  The score
is the time of one encode graph plus one decode graph replay, measured with
HIP events (torch.cuda.Event on the replay stream).  Cache key: device
architecture, model dtype and width, and the multiset of image sizes.  The
cache file is $DLIC_AUTOTUNE_CACHE, else ~/.cache/dlic/autotune.json.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

DEFAULT = {"rows_per_group": 192, "lanes": 32, "density_grid": 0, "search_lanes": 0,
           "decode_grid": 0}
# (rows per group, lanes) pairs, the likeliest first in case the budget ends
LAYOUTS = ((96, 32), (12, 4), (16, 4), (24, 4), (96, 64), (64, 64), (64, 32), (192, 32),
           (12, 2))
GRIDS = (0, 2048)
DECODE_GRIDS = (0, 256, 128)


def search_options(lanes: int):
    """Search fan-outs a layout of this many lanes per group allows (0 = default)."""
    if lanes <= 4:
        return (0, 2)
    if lanes <= 32:
        return (0, 1)
    return (0,)


def knob_trials(layout_best: dict):
    """Second stage: the other knobs around the best layout, one at a time."""
    out = []
    for g in GRIDS:
        if g != layout_best["density_grid"]:
            out.append(dict(layout_best, density_grid=g))
    for sl in search_options(layout_best["lanes"]):
        if sl != layout_best["search_lanes"]:
            out.append(dict(layout_best, search_lanes=sl))
    for dg in DECODE_GRIDS:
        if dg != layout_best["decode_grid"]:
            out.append(dict(layout_best, decode_grid=dg))
    return out


def cache_path() -> str:
    return os.environ.get("DLIC_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "dlic", "autotune.json")


def key(model, sizes) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    ms = sorted((int(h), int(w)) for h, w in sizes)
    digest = hashlib.sha1(json.dumps(ms).encode()).hexdigest()[:16]
    return f"{arch}/{model.dtype}/{model.c.h1}/{len(ms)}:{digest}"


def coders_for(sizes, rows_per_group: int, lanes: int):
    """(G, L) per image: ceil(h / rows) groups, kept within the format's limits."""
    out = []
    for h, _ in sizes:
        g = min(1024, max(1, math.ceil(h / rows_per_group)))
        if g > 1 and h < 2 * g:
            g = max(1, h // 2)
        while math.ceil(h / g) > 256:
            g += 1
        if g > 1024:
            raise ValueError(f"no layout of at most 1024 groups of 256 rows fits height {h}")
        out.append((g, lanes))
    return out


def _time_config(dl, torch, model, sizes, images, knobs, reps):
    b = dl.Batch(model, sizes, coders=coders_for(sizes, knobs["rows_per_group"], knobs["lanes"]),
                 density_grid=knobs["density_grid"], search_lanes=knobs.get("search_lanes", 0),
                 decode_grid=knobs.get("decode_grid", 0))
    try:
        b.load(images)
        b.capture()
        s = torch.cuda.current_stream()
        for _ in range(1):  # warm-up
            b.replay(False, s)
            b.replay(True, s)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        enc = dec = 0.0
        for _ in range(reps):
            e0.record(s)
            b.replay(False, s)
            e1.record(s)
            b.replay(True, s)
            e2.record(s)
            torch.cuda.synchronize()
            enc += e0.elapsed_time(e1)
            dec += e1.elapsed_time(e2)
        ok = bool((b.status == 0).all().item())
        nbytes = int(b.lens.sum().item())
        return {"encode_ms": enc / reps, "decode_ms": dec / reps, "ok": ok, "bytes": nbytes}
    finally:
        b.close()


def tune(model, sizes, images, reps: int = 2, budget_s: float = 60.0, use_cache: bool = True,
         log=None) -> dict:
    """Best knobs for this workload (cached).  Returns {'knobs', 'trials', 'key', 'cached'}."""
    import torch

    import paper_2207_05152_amd as dl
    k = key(model, sizes)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if use_cache and k in cache:
        return {"knobs": cache[k]["knobs"], "trials": cache[k].get("trials", []), "key": k,
                "cached": True}
    trials = []
    best = None
    t_start = time.perf_counter()

    def trial(knobs):
        nonlocal best
        r = _time_config(dl, torch, model, sizes, images, knobs, reps)
        r.update(knobs)
        trials.append(r)
        if log:
            log(r)
        score = r["encode_ms"] + r["decode_ms"]
        if r["ok"] and (best is None or score < best[0]):
            best = (score, knobs)

    for rows, lanes in LAYOUTS:
        if time.perf_counter() - t_start > budget_s:
            break
        trial(dict(DEFAULT, rows_per_group=rows, lanes=lanes))
    if best is not None:
        for knobs in knob_trials(best[1]):
            if time.perf_counter() - t_start > budget_s:
                break
            trial(knobs)
    knobs = best[1] if best else dict(DEFAULT)
    if use_cache:
        cache[k] = {"knobs": knobs, "trials": trials}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return {"knobs": knobs, "trials": trials, "key": k, "cached": False}
