"""Autotuners of the batched launch configuration and of the tile geometry.

For a batch of planned circuits `tune_batch` times each candidate
(work-groups per CU, tiles per task) on the device with HIP events; for one
circuit on one state `tune_tile_geometry` times each candidate tile geometry
(tile qubits, register qubits, fixed low qubits; sv_set_tile_geometry) on the
tile passes. Each keeps the fastest and caches the choice in a JSON file keyed
by GPU architecture, dtype and a workload tag (the SV_TUNE_CACHE environment
variable overrides the file's location).
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


# (tile qubits, register qubits, fixed low qubits); 0 / -1: the default
TILE_CANDIDATES = ((0, 0, -1), (0, 3, -1), (11, 0, -1), (10, 0, -1), (0, 0, 3), (0, 0, 4), (0, 0, 6))


def tune_tile_geometry(st, gates, tag: str, flags: int = sv.SV_FUSE | sv.SV_JIT,
                       basis_index: int = 0, repeats: int = 2, candidates=TILE_CANDIDATES,
                       use_cache: bool = True):
    """Best tile geometry for running `gates` on the StateVector `st` with
    `flags`, and the per-candidate tile time (ms, the best of `repeats` runs
    after one warm-up run, which plans and compiles). Candidates the planner
    cannot place the gates in are skipped. Leaves the best geometry set on
    `st`; the state is overwritten (reset to `basis_index` before each run)."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName
    key = f"{arch}/tile/{'c64' if st.dtype == sv.SV_C64 else 'c128'}/{st.n}/{tag}"
    cache = _load()
    if use_cache and key in cache:
        best = tuple(cache[key]["best"])
        st.set_tile_geometry(*best)
        return best, cache[key]["times_ms"]
    times = {}
    for cand in candidates:
        st.set_tile_geometry(*cand)
        st.reset(basis_index)
        try:
            st.run(gates, flags)                      # warm-up: plan, compile
        except sv.SVError as e:
            # a geometry the planner cannot place every gate in (a gate with
            # more qubits than the tile holds) is skipped
            if e.status != sv.SV_EUNSUPPORTED:
                raise
            continue
        best = float("inf")
        for _ in range(repeats):
            st.reset(basis_index)
            torch.cuda.synchronize()
            sv.sv_profile(st.handle, True)
            st.run(gates, flags)
            torch.cuda.synchronize()
            sv.sv_profile(st.handle, False)
            prof = sv.sv_profile_read(st.handle)
            best = min(best, sum(v["total_ms"] for k, v in prof.items() if k in ("tile", "graph")))
        times["%d,%d,%d" % cand] = round(best, 3)
    if not times:
        st.set_tile_geometry(0, 0, -1)
        raise sv.SVError(sv.SV_EUNSUPPORTED, "no candidate geometry can run these gates")
    best_key = min(times, key=times.get)
    best = tuple(int(x) for x in best_key.split(","))
    st.set_tile_geometry(*best)
    if use_cache:
        cache[key] = {"best": list(best), "times_ms": times}
        _save(cache)
    return best, times
