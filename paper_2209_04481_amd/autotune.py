"""Work-item shape and schedule autotuner for the ensemble launch.

A work item is one column tile of one instance over a chunk of radial layers;
the chunk length is the tile's depth, a runtime setting of the library
(cfv_tuning.chunk_layers; the outputs do not depend on it).  The tuner times,
on the ensemble's bound buffers with HIP events on the launch stream, every
schedule (static or queued item list, workgroups per compute unit, item order)
at the default depth, then every depth in CHUNKS with the fastest schedule,
keeps the fastest pair, and caches the choice in a JSON file keyed by the
device name, the operation, the instance shapes in their order and a hash of
the loaded libcfv.so (a rebuilt library or a reordered ensemble is tuned
afresh).
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from .binding import LIB_PATH, Ensemble, Tuning

SCHEDULES = [Tuning(q, b, o) for q in (0, 1) for b in (1, 2, 4) for o in (0, 1)]
CHUNKS = (4, 8, 12, 16, 24, 32, 64)


def cache_path() -> str:
    p = os.environ.get("CFV_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2209_04481_amd", "ensemble_tuning.json")


_LIB_HASH = None


def library_hash() -> str:
    global _LIB_HASH
    if _LIB_HASH is None:
        h = hashlib.sha1()
        with open(LIB_PATH, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _LIB_HASH = h.hexdigest()[:16]
    return _LIB_HASH


def cache_key(ens: Ensemble, dual: bool) -> str:
    shapes = [(c.grid.N, c.grid.Nr) for c in ens.contexts]
    h = hashlib.sha1(json.dumps(shapes).encode()).hexdigest()[:16]
    return f"{torch.cuda.get_device_name()}|{'jvp' if dual else 'res'}|{len(shapes)}|{h}|{library_hash()}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_schedule(ens: Ensemble, tuning: Tuning, reps: int = 5, stream=None) -> float:
    """Mean milliseconds of one eager run of the bound ensemble."""
    s = stream or torch.cuda.current_stream()
    ens.set_tuning(tuning)
    ens.run(s)  # warm-up
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        ens.run(s)
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / reps


def autotune(ens: Ensemble, dual: bool = True, reps: int = 5, stream=None, use_cache: bool = True):
    """Pick and set the fastest schedule and chunk length; returns
    (tuning, {repr: ms}) with every timed candidate."""
    path, key = cache_path(), cache_key(ens, dual)
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            t = Tuning(**hit["tuning"])
            ens.set_tuning(t)
            return t, hit.get("ms", {})
    ms = {}
    stage1 = [Tuning(t.queue, t.blocks_per_cu, t.order, 0) for t in SCHEDULES]
    for t in stage1:
        ms[repr(t)] = time_schedule(ens, t, reps, stream)
    best = min(stage1, key=lambda t: ms[repr(t)])
    for kc in CHUNKS:
        t = Tuning(best.queue, best.blocks_per_cu, best.order, kc)
        ms[repr(t)] = time_schedule(ens, t, reps, stream)
        if ms[repr(t)] < ms[repr(best)]:
            best = t
    ens.set_tuning(best)
    if use_cache:
        data = _load(path)
        data[key] = {"tuning": best.as_dict(), "ms": ms}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best, ms
