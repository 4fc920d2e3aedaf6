"""Autotuner for libtacsl launch shapes and work-list order.

Searches block size, tile size, schedule (one workgroup per tile, persistent
static stride, persistent dynamic queue), persistent grid size and tile order
(instance-major, XCD-aware object grouping, longest first, object-major,
object-major with per-XCD runs, and the same over pads in a spatial order
rebuilt every call) by timing the
forward call on the device with HIP events, and caches the winner per
(GPU architecture, CU count, scene shape signature) in a JSON file
(``TACSL_TUNE_CACHE`` or ``~/.cache/tacsl/tune.json``).
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional

import numpy as np
import torch


def cache_path() -> str:
    return os.environ.get("TACSL_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tacsl", "tune.json"))


def shape_signature(scene) -> str:
    """Hash of what the best launch shape depends on: pad sizes and grid sizes."""
    counts = np.diff(np.asarray(scene.tmpl_offset))[np.asarray(scene.inst_tmpl)]
    dims = np.asarray(scene.sdf_dims).reshape(-1, 3)[np.asarray(scene.env_sdf)[np.asarray(scene.inst_env)]]
    key = np.concatenate([counts[:, None], dims], axis=1)
    uniq, num = np.unique(key, axis=0, return_counts=True)
    h = hashlib.sha1()
    h.update(np.int64(scene.n_inst).tobytes())
    h.update(np.ascontiguousarray(uniq, np.int64).tobytes())
    h.update(np.ascontiguousarray(num, np.int64).tobytes())
    return h.hexdigest()[:16]


def device_key(device=None) -> str:
    p = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", p.name)
    return f"{arch}|{p.multi_processor_count}"


def _load_cache() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: Dict[str, dict]):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_forward(plan, state, out, reps: int = 6, warmup: int = 2) -> float:
    """Median milliseconds of one forward call (prologue + kernels) on the current stream."""
    for _ in range(warmup):
        plan.forward(state, out)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        plan.forward(state, out)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def candidates(plan, stage: int, base: Optional[dict] = None, schedules=(0, 1, 2)) -> List[dict]:
    info = plan.info()
    cu = int(info.cu_count)
    counts = np.diff(plan.offsets())
    cmax = int(counts.max()) if counts.size else 0
    out = []
    if stage == 0:
        tiles = [0] + [t for t in (512, 1024, 2048, 4096) if t < cmax]
        for tile in tiles:
            for order in (0, 1, 2, 3, 4, 5):
                if 0 in schedules:
                    out.append(dict(block=256, tile_taxels=tile, schedule=0, grid=0, order=order))
                for sch in (s for s in schedules if s in (1, 2)):
                    for k in (2, 4, 8, 16):
                        out.append(dict(block=256, tile_taxels=tile, schedule=sch, grid=cu * k, order=order))
    else:
        for block in (64, 128, 256, 512):
            c = dict(base)
            c["block"] = block
            out.append(c)
    return out


def autotune(plan, scene, state, out, reps: int = 6, use_cache: bool = True, schedules=(0, 1, 2),
             verbose: bool = False, tag: str = "") -> dict:
    """Pick and install the fastest tuning for ``plan``; returns it with its timing table."""
    key = f"{device_key(plan.device)}|{shape_signature(scene)}|{tag}|{','.join(map(str, schedules))}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        best = cache[key]["tuning"]
        plan.set_tuning(best)
        return dict(tuning=best, cached=True, ms=cache[key]["ms"], table=[])
    table = []
    t0 = time.time()
    best, best_ms = None, float("inf")
    for stage in (0, 1):
        for cand in candidates(plan, stage, best, schedules):
            plan.set_tuning(cand)
            ms = time_forward(plan, state, out, reps=reps)
            table.append((dict(cand), ms))
            if verbose:
                print(f"[autotune] {cand} {ms:.4f} ms", flush=True)
            if ms < best_ms:
                best, best_ms = dict(cand), ms
    plan.set_tuning(best)
    if use_cache:
        cache = _load_cache()
        cache[key] = dict(tuning=best, ms=best_ms, searched=len(table), seconds=round(time.time() - t0, 2))
        _store_cache(cache)
    return dict(tuning=best, cached=False, ms=best_ms, table=table)
