"""Autotuning of the kernel configuration per plan shape, with an on-disk cache.

A configuration is what the library lets a plan choose without changing the
transform (sft_params): the short-DFT path (1: VALU in LDS, 2: split, 3:
matrix cores in LDS, 4: split with matrix-core columns), the filtered-sample
kernel (gather_path 1: one node per lane, band sums on the vector ALUs; 2:
the band sums as matrix-core products) and, for path 3, the moduli split
threshold (dft_split: -1 one launch, j the moduli [0, j) in a launch of their
own with a smaller LDS allocation, 0 the library's LDS rule).  For a plan
shape (N, s, parameters) and a batch size the tuner times, on a synthetic
input with HIP events on the launch stream, every (dft_path, gather_path)
pair the library accepts with the automatic split, then every split of the
fastest pair when that pair runs path 3, and keeps the fastest.  All
configurations compute the same transform (paths 1 and 2 bitwise equal up
to s1 = 256, as are 3 and 4 and every split; the gathers, the two path
families and paths 1 and 2 at s1 >= 512 differ by rounding order).  Results are cached per device architecture, plan shape
and batch-size class in a JSON file (``$SFT_TUNE_CACHE``, default
``~/.cache/paper_1706_02740_amd/tune.json``), so a shape is measured once.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, Iterable, Optional

PATHS = (3, 1, 4, 2)     # tried in this order; ties keep the earlier configuration
GATHERS = (1, 2)
TUNED = ("dft_path", "gather_path", "dft_split")


def cache_path() -> str:
    return os.environ.get("SFT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1706_02740_amd", "tune.json"))


def batch_class(batch: int) -> str:
    """Batch sizes that lead to the same choice: one transform, a few, many."""
    return "1" if batch <= 1 else ("2-16" if batch <= 16 else "17+")


def shape_key(arch: str, N: int, s: int, batch: int, params: dict) -> str:
    p = {k: v for k, v in sorted(params.items()) if k not in TUNED}
    return f"{arch}|N={int(N)}|s={int(s)}|{json.dumps(p, sort_keys=True)}|batch={batch_class(batch)}"


def config_name(cfg: dict) -> str:
    return f"dft{cfg['dft_path']}-gather{cfg['gather_path']}-split{cfg['dft_split']}"


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
        hit = self.data.get(key)
        return hit if hit is not None and all(k in hit for k in TUNED) else None   # older entries: measure again

    def put(self, key: str, entry: dict) -> None:
        self.data[key] = entry
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.data, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def choose(key: str, measure: Callable[[dict], Optional[float]], cache: Cache,
           splits: Callable[[dict], Iterable[int]] = lambda cfg: ()) -> dict:
    """The cached entry for key, else: measure(config) -> ms per transform
    (None: the library refuses the configuration) for every (dft_path,
    gather_path) with the automatic split, then for the fastest, if it runs
    path 3, every split in splits(config); keep the fastest and cache it."""
    hit = cache.get(key)
    if hit is not None:
        return hit
    times: Dict[str, float] = {}
    order = []
    for path in PATHS:
        for g in GATHERS:
            cfg = {"dft_path": path, "gather_path": g, "dft_split": 0}
            ms = measure(cfg)
            if ms is not None:
                times[config_name(cfg)] = float(ms)
                order.append(cfg)
    if not times:
        raise RuntimeError(f"no kernel configuration accepts {key}")
    best = min(order, key=lambda c: (times[config_name(c)], order.index(c)))
    if best["dft_path"] == 3:
        for j in splits(best):
            cfg = dict(best, dft_split=int(j))
            if config_name(cfg) in times:
                continue
            ms = measure(cfg)
            if ms is not None:
                times[config_name(cfg)] = float(ms)
                order.append(cfg)
        best = min(order, key=lambda c: (times[config_name(c)], order.index(c)))
    entry = dict(best, ms_per_transform=times)
    cache.put(key, entry)
    return entry


def _measure_on_device(N: int, s: int, batch: int, params: dict, reps: int = 3):
    import torch

    from . import SFT_EUNSUPPORTED, Plan, SftError, execute_many

    g = torch.Generator(device="cuda").manual_seed(12345)
    f = torch.complex(torch.randn(N, device="cuda", generator=g),
                      torch.randn(N, device="cuda", generator=g)).to(torch.complex64)

    def measure(cfg: dict) -> Optional[float]:
        try:
            plan = Plan(N, s, **cfg, **params)
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

    def splits(cfg: dict):
        K = Plan(N, s, **cfg, **params).info["K"]
        return [-1] + list(range(1, K))

    return measure, splits


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName


def best_config(N: int, s: int, batch: int = 1, cache: Optional[Cache] = None, **params) -> dict:
    """The fastest kernel configuration ({dft_path, gather_path, dft_split})
    for transforms of this shape launched `batch` at a time on the current
    device (measured once, then cached)."""
    key = shape_key(_arch(), N, s, batch, params)
    cache = cache or Cache()
    hit = cache.get(key)
    if hit is None:
        measure, splits = _measure_on_device(N, s, batch, params)
        hit = choose(key, measure, cache, splits)
    return {k: hit[k] for k in TUNED}


def best_dft_path(N: int, s: int, batch: int = 1, cache: Optional[Cache] = None, **params) -> int:
    """The short-DFT path of best_config."""
    return best_config(N, s, batch, cache, **params)["dft_path"]


def tuned_plan(N: int, s: int, batch: int = 1, cache: Optional[Cache] = None, **params):
    """A Plan with the tuned kernel configuration."""
    from . import Plan
    return Plan(N, s, **best_config(N, s, batch, cache, **params), **params)
