"""Autotuning of the short-DFT path per plan shape, with an on-disk cache.

For a plan shape (N, s, parameters) and a batch size, every short-DFT path
the library accepts for it (1: VALU in LDS, 2: split, 3: matrix cores in LDS,
4: split with matrix-core columns; see sft_params.dft_path) is timed on a synthetic input with HIP events on the
launch stream, and the fastest is kept.  All paths compute the same
transform; paths 1 and 2 give bitwise equal results, as do paths 3 and 4,
which sum the p-point step in another order.  Results are cached per device architecture, plan
shape and batch-size class in a JSON file (``$SFT_TUNE_CACHE``, default
``~/.cache/paper_1706_02740_amd/tune.json``), so a shape is measured once.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, Optional

PATHS = (3, 1, 4, 2)   # tried in this order; ties keep the earlier one


def cache_path() -> str:
    return os.environ.get("SFT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1706_02740_amd", "tune.json"))


def batch_class(batch: int) -> str:
    """Batch sizes that lead to the same choice: one transform, a few, many."""
    return "1" if batch <= 1 else ("2-16" if batch <= 16 else "17+")


def shape_key(arch: str, N: int, s: int, batch: int, params: dict) -> str:
    p = {k: v for k, v in sorted(params.items()) if k != "dft_path"}
    return f"{arch}|N={int(N)}|s={int(s)}|{json.dumps(p, sort_keys=True)}|batch={batch_class(batch)}"


class Cache:
    def __init__(self, path: Optional[str] = None):
        self.path = path or cache_path()
        self.data: Dict[str, dict] = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as fh:
                    self.data = json.load(fh)
            except (OSError, ValueError):
                self.data = {}   # unreadable cache: measure again

    def get(self, key: str) -> Optional[dict]:
        return self.data.get(key)

    def put(self, key: str, entry: dict) -> None:
        self.data[key] = entry
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.data, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def choose(key: str, measure: Callable[[int], Optional[float]], cache: Cache) -> dict:
    """The cached entry for key, else measure(path) -> ms per transform (None:
    the library refuses the path for this shape) for every path, keep the
    fastest and cache it."""
    hit = cache.get(key)
    if hit is not None:
        return hit
    times = {}
    for path in PATHS:
        ms = measure(path)
        if ms is not None:
            times[str(path)] = float(ms)
    if not times:
        raise RuntimeError(f"no short-DFT path accepts {key}")
    best = min(times, key=lambda k: (times[k], PATHS.index(int(k))))
    entry = {"dft_path": int(best), "ms_per_transform": times}
    cache.put(key, entry)
    return entry


def _measure_on_device(N: int, s: int, batch: int, params: dict, reps: int = 3):
    import torch

    from . import SFT_EUNSUPPORTED, Plan, SftError, execute_many

    g = torch.Generator(device="cuda").manual_seed(12345)
    f = torch.complex(torch.randn(N, device="cuda", generator=g),
                      torch.randn(N, device="cuda", generator=g)).to(torch.complex64)

    def measure(path: int) -> Optional[float]:
        try:
            plan = Plan(N, s, dft_path=path, **params)
        except SftError as e:
            if e.code == SFT_EUNSUPPORTED:
                return None
            raise
        plans, fs = [plan] * batch, [f] * batch
        outs, counts = execute_many(plans, fs)   # warm-up (and the batch workspace)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            execute_many(plans, fs, outs, counts)
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / (reps * batch)

    return measure


def best_dft_path(N: int, s: int, batch: int = 1, cache: Optional[Cache] = None, **params) -> int:
    """The fastest short-DFT path for transforms of this shape launched
    `batch` at a time on the current device (measured once, then cached)."""
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    key = shape_key(arch, N, s, batch, params)
    cache = cache or Cache()
    hit = cache.get(key)
    if hit is not None:   # no device work at all
        return hit["dft_path"]
    return choose(key, _measure_on_device(N, s, batch, params), cache)["dft_path"]


def tuned_plan(N: int, s: int, batch: int = 1, cache: Optional[Cache] = None, **params):
    """A Plan with the tuned short-DFT path."""
    from . import Plan
    return Plan(N, s, dft_path=best_dft_path(N, s, batch, cache, **params), **params)
