"""Autotuner front: chooses launch shapes per launch group and caches them in
JSON, keyed by device, launch kind, shape class and a size bucket.

The measurement is the library's (lbp_autotune: HIP-event timing of every
candidate shape); this module only reuses earlier choices.  Shapes never
change results, only speed.  Cache file: $LBP_TUNE_CACHE, else
~/.cache/lbp_tune.json; entries missing there are looked up in the table
shipped with the package (tuned_shapes.json, measured on MI355X), which is
never written.
"""
from __future__ import annotations

import json
import math
import os


PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_shapes.json")


def cache_path():
    return os.environ.get("LBP_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "lbp_tune.json")


def _key(device, d, T, ln):
    bucket = int(math.log2(max(1, ln["items"])))
    mode = "maxprod" if T == 0 else "lse"
    return "%s|%s|p%d|k%d|a%d|b%d|n2^%d" % (device, mode, ln["phase"], ln["kind"], ln["a"], ln["b"], bucket)


def device_key(index: int = 0) -> str:
    """Architecture name and compute-unit count of a device (the marketing
    name can be empty, for instance under a profiler)."""
    import torch

    p = torch.cuda.get_device_properties(index)
    arch = getattr(p, "gcnArchName", "") or torch.cuda.get_device_name(index) or "unknown"
    return "%s|cu%d" % (arch.split(":")[0], p.multi_processor_count)


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def apply_or_tune(graph, damping: float, temperature: float, reps: int = 20, path=None, device=None,
                  packaged: bool = True):
    """Applies cached shapes to every launch group of ``graph``; runs the
    autotuner (and records its choices in the user cache) when any group is
    missing.  packaged: also consult the shipped table."""
    path = path or cache_path()
    device = device or device_key(graph.ctx.device)
    user = _load(path)
    cache = dict(_load(PACKAGED)) if packaged else {}
    cache.update(user)
    lns = graph.launches()
    keys = [_key(device, damping, temperature, ln) for ln in lns]
    fkey = None
    if graph.fused:
        es = max(1, graph.ES)
        fkey = "%s|%s|fused|es2^%d" % (device, "maxprod" if temperature == 0 else "lse", int(math.log2(es)))
    if all(k in cache for k in keys) and (fkey is None or fkey in cache):
        for i, k in enumerate(keys):
            graph.set_launch(i, cache[k]["wpb"], cache[k]["swizzle"])
            if fkey is not None and lns[i]["phase"] == 1:
                graph.set_fused_launch(i, cache[k]["fused_wpb"], cache[k].get("fused_variant", 0))
        if fkey is not None:
            graph.use_fused(cache[fkey]["use"])
        return {"source": "cache", "shapes": [cache[k] for k in keys],
                "fused": graph.fused_in_use}
    ms = graph.autotune(damping, temperature, reps)
    lns = graph.launches()
    cache = user
    for k, ln, t in zip(keys, lns, ms):
        cache[k] = {"wpb": ln["wpb"], "swizzle": ln["swizzle"], "ms": float(t),
                    "fused_wpb": ln["fused_wpb"], "fused_variant": ln["fused_variant"]}
    if fkey is not None:
        cache[fkey] = {"use": graph.fused_in_use}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass
    return {"source": "tuned", "shapes": [cache[k] for k in keys], "fused": graph.fused_in_use}
