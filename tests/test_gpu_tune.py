"""The short-DFT path tuner on the device: the chosen path is one the library
accepts, a plan built with it gives the same results as an explicit plan with
that path, and the cache answers the second request without measuring."""
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
    path = tune.best_dft_path(N, s, batch=8, cache=cache)
    assert path in (1, 2, 3, 4)
    entry = next(iter(cache.data.values()))
    assert set(entry["ms_per_transform"]) == {"1", "2", "3", "4"}   # every path fits this shape
    tuned = tune.tuned_plan(N, s, batch=8, cache=cache)
    explicit = gpu.Plan(N, s, dft_path=path)
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
        assert tune.best_dft_path(N, s, batch=12, cache=tune.Cache(cache.path)) == path
    finally:
        tune._measure_on_device = orig
