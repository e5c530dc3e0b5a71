"""Host logic of the short-DFT path tuner: the choice, the refused paths, the
on-disk cache (no device needed: the measurement is injected)."""
import json

import pytest

from paper_1706_02740_amd import tune


def test_choose_takes_the_fastest_and_skips_refused_paths(tmp_path):
    cache = tune.Cache(str(tmp_path / "t.json"))
    times = {1: 2.0, 2: 1.5, 3: None, 4: None}
    entry = tune.choose("k", lambda p: times[p], cache)
    assert entry["dft_path"] == 2
    assert entry["ms_per_transform"] == {"1": 2.0, "2": 1.5}


def test_ties_keep_the_earlier_path(tmp_path):
    cache = tune.Cache(str(tmp_path / "t.json"))
    assert tune.choose("k", lambda p: 1.0, cache)["dft_path"] == tune.PATHS[0]


def test_cache_is_reused_and_persisted(tmp_path):
    path = str(tmp_path / "sub" / "t.json")
    calls = []

    def measure(p):
        calls.append(p)
        return {1: 3.0, 2: 4.0, 3: 2.5, 4: 3.5}[p]

    assert tune.choose("k", measure, tune.Cache(path))["dft_path"] == 3
    n = len(calls)
    again = tune.Cache(path)                       # a new process reads the file
    assert tune.choose("k", measure, again)["dft_path"] == 3
    assert len(calls) == n                         # not measured again
    assert json.load(open(path))["k"]["dft_path"] == 3


def test_unreadable_cache_is_measured_again(tmp_path):
    path = tmp_path / "t.json"
    path.write_text("{not json")
    assert tune.choose("k", lambda p: float(p), tune.Cache(str(path)))["dft_path"] == 1


def test_no_accepted_path_raises(tmp_path):
    with pytest.raises(RuntimeError):
        tune.choose("k", lambda p: None, tune.Cache(str(tmp_path / "t.json")))


def test_keys():
    a = tune.shape_key("gfx950", 2 ** 22, 64, 256, {"preset": 0, "dft_path": 3})
    b = tune.shape_key("gfx950", 2 ** 22, 64, 100, {"preset": 0})
    assert a == b                                  # dft_path is what is tuned; 100 and 256 share a class
    assert a != tune.shape_key("gfx950", 2 ** 22, 64, 1, {"preset": 0})
    assert a != tune.shape_key("gfx942", 2 ** 22, 64, 256, {"preset": 0})
    assert [tune.batch_class(b) for b in (1, 2, 16, 17)] == ["1", "2-16", "2-16", "17+"]
