"""Schedule autotuner for the ensemble launch.

Times every candidate schedule (static or queued item list, workgroups per
compute unit, item order) on the ensemble's bound buffers with HIP events on
the launch stream, keeps the fastest, and caches the choice in a JSON file
keyed by the device name and the instance shapes.  The tile shape itself is
fixed at compile time (16 x 16 columns, 16 layers per chunk).
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from .binding import Ensemble, Tuning

CANDIDATES = [Tuning(q, b, o) for q in (0, 1) for b in (1, 2, 4) for o in (0, 1)]


def cache_path() -> str:
    p = os.environ.get("CFV_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2209_04481_amd", "ensemble_tuning.json")


def cache_key(ens: Ensemble, dual: bool) -> str:
    shapes = sorted((c.grid.N, c.grid.Nr) for c in ens.contexts)
    h = hashlib.sha1(json.dumps(shapes).encode()).hexdigest()[:16]
    return f"{torch.cuda.get_device_name()}|{'jvp' if dual else 'res'}|{len(shapes)}|{h}"


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
    """Pick and set the fastest schedule; returns (tuning, {repr: ms})."""
    path, key = cache_path(), cache_key(ens, dual)
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            t = Tuning(**hit["tuning"])
            ens.set_tuning(t)
            return t, hit.get("ms", {})
    ms = {repr(t): time_schedule(ens, t, reps, stream) for t in CANDIDATES}
    best = min(CANDIDATES, key=lambda t: ms[repr(t)])
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
