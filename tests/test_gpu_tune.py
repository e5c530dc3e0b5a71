"""The kernel-configuration tuner on the device: the chosen configuration is
one the library accepts, a plan built with it gives the same results as an
explicit plan with that configuration, and the cache answers the second
request without measuring."""
import numpy as np
import pytest

import siggen
from tests.test_gpu_parity import dev, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_tuned_plan_and_cache(gpu, tmp_path):
    from paper_1706_02740_amd import tune
    cache = tune.Cache(str(tmp_path / "tune.json"))
    N, s = 2 ** 16, 40
    say("tune", N, s)
    cfg = tune.best_config(N, s, batch=8, cache=cache)
    path = cfg["dft_path"]
    assert path in (1, 2, 3, 4) and cfg["gather_path"] in (1, 2)
    entry = next(iter(cache.data.values()))
    measured = set(entry["ms_per_transform"])
    # every path and both gathers fit this shape; splits of path 3 when it won
    assert {f"dft{p}-gather{g}-split0" for p in (1, 2, 3, 4) for g in (1, 2)} <= measured
    if path == 3:
        K = gpu.Plan(N, s).info["K"]
        assert {f"dft3-gather{cfg['gather_path']}-split{j}" for j in [-1] + list(range(1, K))} <= measured
    tuned = tune.tuned_plan(N, s, batch=8, cache=cache)
    explicit = gpu.Plan(N, s, **cfg)
    f = dev(siggen.sparse_signal(N, s, seed=4, snr_db=20.0).f32)
    a = [t.cpu().numpy() for t in tuned.execute(f)]
    b = [t.cpu().numpy() for t in explicit.execute(f)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)

    def no_measure(*args, **kw):
        raise AssertionError("measured again")

    orig = tune._measure_on_device
    tune._measure_on_device = no_measure
    try:
        assert tune.best_config(N, s, batch=12, cache=tune.Cache(cache.path)) == cfg
    finally:
        tune._measure_on_device = orig
