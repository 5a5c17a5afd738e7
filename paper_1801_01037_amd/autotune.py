"""Autotuner of the batched launch configuration.

For a batch of planned circuits it times each candidate (work-groups per CU,
tiles per task) on the device with HIP events, keeps the fastest, and caches
the choice in a JSON file keyed by GPU architecture, dtype and a workload tag
(the SV_TUNE_CACHE environment variable overrides the file's location).
"""
from __future__ import annotations

import json
import os

import paper_1801_01037_amd as sv

CANDIDATES = ((1, 1), (1, 8), (2, 1), (2, 4), (2, 8), (2, 32), (3, 4), (3, 8), (3, 16), (4, 8), (4, 64))


def cache_path() -> str:
    return os.environ.get("SV_TUNE_CACHE", os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1801_01037_amd", "tune.json"))


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass   # a read-only home: tune again next time


def tune_batch(dtype: int, plans, tag: str, stream=None, repeats: int = 2,
               candidates=CANDIDATES, use_cache: bool = True):
    """Best (blocks_per_cu, tiles_per_task) for running `plans` as one batch,
    and the per-candidate times (ms). The plans' states are overwritten."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    key = f"{arch}/batch/{'c64' if dtype == sv.SV_C64 else 'c128'}/{tag}"
    cache = _load()
    if use_cache and key in cache:
        return tuple(cache[key]["best"]), cache[key]["times_ms"]
    s = stream if stream is not None else torch.cuda.current_stream()
    b = sv.sv_batch_create(dtype, s.cuda_stream)
    times = {}
    try:
        for bpc, tpt in candidates:
            sv.sv_batch_config(b, bpc, tpt)
            sv.sv_batch_run(b, plans)                      # warm-up
            best = float("inf")
            for _ in range(repeats):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                sv.sv_batch_run(b, plans)
                e1.record(s)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1))
            times[f"{bpc}x{tpt}"] = best
    finally:
        sv.sv_batch_destroy(b)
    choice = min(times, key=times.get)
    best = tuple(int(x) for x in choice.split("x"))
    cache[key] = {"best": list(best), "times_ms": times}
    _save(cache)
    return best, times
