"""Band-width autotuner for batched solves.

For each size class (a range of orders) the tuner times hgv_zhegvx on a synthetic
GUE-like pencil of the class's middle order for every candidate band width and keeps
the fastest.  Results are cached as JSON keyed by (device name, class bounds, fraction
of eigenpairs), so a tuned table is reused across runs.
"""
import json
import math
import os

import torch

from .tensors import Context

DEFAULT_CLASSES = ((500, 1000), (1000, 2000), (2000, 3001))
DEFAULT_CANDIDATES = (32, 48, 64)


def _cache_path(path):
    if path:
        return path
    return os.environ.get("HGV_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hgv_autotune.json"))


def _time_solve(ctx, A, B, iu, nb, reps=2):
    ctx.zhegvx(A, B, 1, iu, "fp64", nb)          # warm up
    torch.cuda.synchronize(ctx.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.zhegvx(A, B, 1, iu, "fp64", nb)
    e1.record()
    torch.cuda.synchronize(ctx.device)
    return e0.elapsed_time(e1) / reps


def tune(device="cuda:0", classes=DEFAULT_CLASSES, candidates=DEFAULT_CANDIDATES, frac=0.2, path=None,
         use_cache=True):
    """Return {(lo, hi): nb} and update the JSON cache."""
    from inputs import gue_pair
    path = _cache_path(path)
    name = torch.cuda.get_device_name(torch.device(device))
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    ctx = Context.get(device)
    table = {}
    for lo, hi in classes:
        key = "%s|%d-%d|%.3f" % (name, lo, hi, frac)
        if key in cache:
            table[(lo, hi)] = int(cache[key]["nb"])
            continue
        n = (lo + hi) // 2
        A, B = gue_pair(n, [7, n], cond_b=1e2, device=device)
        iu = max(1, int(math.ceil(frac * n)))
        times = {nb: _time_solve(ctx, A, B, iu, nb) for nb in candidates}
        best = min(times, key=times.get)
        table[(lo, hi)] = best
        cache[key] = {"nb": best, "ms": times}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return table


def nb_for(table, n):
    for (lo, hi), nb in table.items():
        if lo <= n < hi:
            return nb
    return 0
