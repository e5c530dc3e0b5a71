"""Host logic of the kernel-configuration tuner: the choice, the refused
configurations, the split search of the matrix-core short DFT, the on-disk
cache (no device needed: the measurement is injected)."""
import json

import pytest

from paper_1706_02740_amd import tune


def _cfg_time(table):
    """measure(config) from a table keyed by (dft_path, gather_path, dft_split)."""
    return lambda c: table.get((c["dft_path"], c["gather_path"], c["dft_split"]))


def test_choose_takes_the_fastest_and_skips_refused_configurations(tmp_path):
    cache = tune.Cache(str(tmp_path / "t.json"))
    table = {(1, 1, 0): 2.0, (1, 2, 0): 2.5, (2, 1, 0): 1.5, (2, 2, 0): 1.7}   # paths 3 and 4 refused
    entry = tune.choose("k", _cfg_time(table), cache)
    assert (entry["dft_path"], entry["gather_path"], entry["dft_split"]) == (2, 1, 0)
    assert entry["ms_per_transform"] == {"dft1-gather1-split0": 2.0, "dft1-gather2-split0": 2.5,
                                         "dft2-gather1-split0": 1.5, "dft2-gather2-split0": 1.7}


def test_split_search_only_for_the_matrix_core_path(tmp_path):
    table = {(3, 1, 0): 1.0, (3, 2, 0): 1.2, (1, 1, 0): 1.1, (3, 1, -1): 1.05, (3, 1, 3): 0.9, (3, 1, 5): 0.95}
    asked = []

    def splits(cfg):
        asked.append(dict(cfg))
        return [-1, 3, 5, 6]      # 6 refused (no entry)

    entry = tune.choose("k", _cfg_time(table), tune.Cache(str(tmp_path / "t.json")), splits)
    assert (entry["dft_path"], entry["gather_path"], entry["dft_split"]) == (3, 1, 3)
    assert asked == [{"dft_path": 3, "gather_path": 1, "dft_split": 0}]
    # a fastest configuration on another path measures no split
    asked.clear()
    table2 = {(1, 1, 0): 0.5, (3, 1, 0): 1.0}
    entry = tune.choose("k2", _cfg_time(table2), tune.Cache(str(tmp_path / "t2.json")), splits)
    assert entry["dft_path"] == 1 and entry["dft_split"] == 0 and asked == []


def test_ties_keep_the_earlier_configuration(tmp_path):
    cache = tune.Cache(str(tmp_path / "t.json"))
    entry = tune.choose("k", lambda c: 1.0, cache)
    assert (entry["dft_path"], entry["gather_path"], entry["dft_split"]) == (tune.PATHS[0], tune.GATHERS[0], 0)


def test_cache_is_reused_and_persisted(tmp_path):
    path = str(tmp_path / "sub" / "t.json")
    calls = []

    def measure(c):
        calls.append(c)
        return {1: 3.0, 2: 4.0, 3: 2.5, 4: 3.5}[c["dft_path"]] + (0.1 if c["gather_path"] == 2 else 0.0)

    assert tune.choose("k", measure, tune.Cache(path))["dft_path"] == 3
    n = len(calls)
    again = tune.Cache(path)                       # a new process reads the file
    assert tune.choose("k", measure, again)["dft_path"] == 3
    assert len(calls) == n                         # not measured again
    saved = json.load(open(path))["k"]
    assert saved["dft_path"] == 3 and saved["gather_path"] == 1 and saved["dft_split"] == 0


def test_unreadable_or_older_cache_is_measured_again(tmp_path):
    path = tmp_path / "t.json"
    path.write_text("{not json")
    assert tune.choose("k", lambda c: float(c["dft_path"]), tune.Cache(str(path)))["dft_path"] == 1
    old = tmp_path / "old.json"
    old.write_text(json.dumps({"k": {"dft_path": 4, "ms_per_transform": {"4": 1.0}}}))   # without gather/split
    assert tune.choose("k", lambda c: float(c["dft_path"]), tune.Cache(str(old)))["dft_path"] == 1


def test_no_accepted_configuration_raises(tmp_path):
    with pytest.raises(RuntimeError):
        tune.choose("k", lambda c: None, tune.Cache(str(tmp_path / "t.json")))


def test_keys():
    a = tune.shape_key("gfx950", 2 ** 22, 64, 256, {"preset": 0, "dft_path": 3, "gather_path": 2, "dft_split": -1})
    b = tune.shape_key("gfx950", 2 ** 22, 64, 100, {"preset": 0})
    assert a == b                                  # the tuned fields are not part of the key
    assert a != tune.shape_key("gfx950", 2 ** 22, 64, 1, {"preset": 0})
    assert a != tune.shape_key("gfx942", 2 ** 22, 64, 256, {"preset": 0})
    assert [tune.batch_class(b) for b in (1, 2, 16, 17)] == ["1", "2-16", "2-16", "17+"]
