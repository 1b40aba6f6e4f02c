"""Autotuner for the batched labeling kernel.

For one batch layout (instance offsets) and its device buffers, time a grid of
``ccl_tuning`` candidates -- workgroup size, resident workgroups per CU, work
item sizes, the LDS small-instance path and the fused / phased / tiled
schedule --
keep only candidates whose labels equal a reference labeling (by default the
one-launch-per-instance schedule) and whose plan reports no error, and
return the fastest.  Results are cached in a JSON file keyed by the device
name, a coarse description of the layout (instance count and size
quantiles) and the search space, so later runs on the same kind of batch
skip the search.

Cache file: $CCL_AUTOTUNE_CACHE, else ~/.cache/ccl_mi355x/autotune.json.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import numpy as np
import torch

import paper_1603_08357_amd as ccl

DEFAULT_SPACE = {
    "schedule": (3, 2, 1),
    "block_threads": (256, 512, 1024),
    "blocks_per_cu": (2, 4, 8),
    "bonds_per_chunk": (16384, 65536, 262144),
    "sites_per_chunk": (16384, 65536),
    "small_sites": (0, -1),
}


def cache_path() -> str:
    p = os.environ.get("CCL_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "ccl_mi355x", "autotune.json")


def layout_key(site_off) -> str:
    so = np.asarray(site_off, dtype=np.int64)
    sizes = np.diff(so)
    if len(sizes) == 0:
        return "empty"
    q = np.percentile(sizes, [0, 50, 90, 100]).astype(np.int64)
    # sizes rounded to powers of two so that batches of the same kind share an entry
    r = [int(2 ** round(np.log2(max(x, 1)))) for x in q]
    return f"K{len(sizes)}-q{r[0]}-{r[1]}-{r[2]}-{r[3]}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(d: dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def space_key(space=None) -> str:
    full = dict(DEFAULT_SPACE, **(space or {}))
    text = json.dumps({k: list(v) for k, v in sorted(full.items())})
    return hashlib.sha1(text.encode()).hexdigest()[:12]


def candidates(space=None, limit=None):
    space = dict(DEFAULT_SPACE, **(space or {}))
    keys = sorted(space)
    out = []
    for vals in itertools.product(*(space[k] for k in keys)):
        t = dict(zip(keys, vals))
        lds = (max(t["small_sites"], 0) + 1) // 2 * 4  # 16-bit parents; 0 = library default
        if lds * t["blocks_per_cu"] > 160 * 1024:
            continue
        # the tiled schedule has no merge items: one bonds_per_chunk suffices
        if t["schedule"] == 3 and t["bonds_per_chunk"] != min(space["bonds_per_chunk"]):
            continue
        out.append(t)
    return out[:limit] if limit else out


def _time_plan(plan, src, dst, occ, out, reps: int) -> float:
    stream = torch.cuda.current_stream()
    plan.label(src, dst, occ, out=out, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.label(src, dst, occ, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(site_off, bond_off, src, dst, occ, space=None, reps: int = 3, use_cache: bool = True,
         limit: int | None = None, verbose: bool = False, reference=None) -> dict:
    """Best tuning (a dict of ccl_tuning fields) for this batch layout.

    Every candidate's labels are compared with `reference` (device int32
    labels of the whole batch); when None, the reference is the one-launch-
    per-instance schedule (ccl_label per instance: a different kernel path
    from the batched kernel).  A candidate whose plan reports an error, or
    whose labels differ, is never chosen."""
    dev_name = torch.cuda.get_device_name()
    key = f"{dev_name}|{layout_key(site_off)}|{space_key(space)}"
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key]["tuning"])
    n = int(np.asarray(site_off)[-1])
    out = torch.empty(n, dtype=torch.int32, device=src.device)
    if reference is None:
        reference = ccl.label_batched_per_instance(site_off, bond_off, src, dst, occ)
        torch.cuda.synchronize()
    results = []
    for t in candidates(space, limit):
        try:
            plan = ccl.Plan(site_off, bond_off, t)
        except ccl.CclError:
            continue
        ms = _time_plan(plan, src, dst, occ, out, reps)
        ok = plan.check() == 0 and bool(torch.equal(out, reference))
        plan.close()
        results.append((ms, ok, t))
        if verbose:
            print(f"  {ms:9.4f} ms {'ok ' if ok else 'BAD'} {t}", flush=True)
    good = [r for r in results if r[1]]
    if not good:
        raise RuntimeError("autotune: no candidate produced the reference labels")
    best_ms, _, best = min(good, key=lambda r: r[0])
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tuning": best, "ms": best_ms, "when": time.strftime("%Y-%m-%d %H:%M:%S"),
                      "candidates": len(results)}
        _store_cache(cache)
    return dict(best)
