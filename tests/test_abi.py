"""The C-ABI library on the CPU: it loads, exports every symbol include/sft.h
declares, and its host-side plan rules (written separately from the oracle's)
give the same plan as the oracle, field by field.  No compute call needs a GPU."""
import os
import re
import subprocess

import pytest

import oracle
import paper_1706_02740_amd as sftlib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sft.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sft_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = sftlib.load_library()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", sftlib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sft_\w+)", out))
    assert set(names) <= exported
    assert set(sftlib.EXPORTED) == set(names)


def test_binding_fetch_kinds_match_the_header():
    """Every SFT_FETCH_* kind the header defines has the same value in the
    binding (the class lists' kind included)."""
    text = open(os.path.join(ROOT, "include", "sft.h")).read()
    kinds = dict(re.findall(r"#define SFT_FETCH_([A-Z_]+)\s+(\d+)", text))
    assert "CLASSES" in kinds and len(kinds) >= 7
    for name, value in kinds.items():
        assert getattr(sftlib, "FETCH_" + name) == int(value), name


def test_symbols_have_c_linkage():
    out = subprocess.run(["nm", "-D", "--defined-only", sftlib.LIB_PATH], capture_output=True, text=True).stdout
    assert not re.search(r"\bT _Z\w*sft_(execute|plan)", out)


CASES = [
    (2 ** 14, 8, {}), (2 ** 22, 64, {}), (10_000_019, 128, {}), (5 * 2 ** 19 + 1, 200, {}),
    (3 * 2 ** 20, 16, {}), (2 ** 26, 1024, {}), (2 ** 24, 256, {}), (2 ** 18, 16, {}),
    (31, 1, {}), (31, 31, {}), (1000, 5, {}), (97, 3, {}), (4096, 3, {"preset": 2}),
    (2 ** 22, 64, {"preset": 2}), (2 ** 20, 50, {"preset": 1}), (2 ** 20, 50, {"preset": 2, "r": 2.0}),
    (2 ** 16, 40, {"s1_mult": 2}), (2 ** 16, 40, {"group": 3}), (2 ** 16, 40, {"heavy_T": 17}),
    (2 ** 16, 40, {"tau": 0.2}), (2 ** 16, 40, {"kappa": 8}), (2 ** 16, 40, {"sigma_t": 1.7}),
    (65537, 7, {"preset": 1}), (2 ** 30, 64, {}), (2 ** 22, 64, {"ident": 1}),
    (3001, 5, {"ident": 1, "kappa": 12}),
]


@pytest.mark.parametrize("N,s,kw", CASES)
def test_library_plan_equals_oracle_plan(N, s, kw):
    lib = sftlib.describe(N, s, **kw)
    orc = oracle.make_plan(N, s, oracle.Params(**kw))
    for name in ("N", "s", "kappa", "Q", "L", "s1", "G", "K", "T", "preset", "ident"):
        assert lib[name] == getattr(orc, name), name
    assert lib["primes"] == orc.primes
    assert lib["P"] == orc.P
    assert lib["q"] == orc.q
    assert lib["M"] == orc.M
    assert lib["depth"] == oracle.class_depth(orc.G)
    # device choices: set by sft_plan_create only
    assert lib["dft_path"] == 0 and lib["dft_split"] == 0 and lib["gather_path"] == 0
    for name in ("sigma_t", "beta", "c1", "tau", "alpha", "c2", "r"):
        assert lib[name] == getattr(orc, name), name     # same FP64 formula, same order


@pytest.mark.parametrize("N,s,kw", [(12, 2, {}), (100, 0, {}), (100, 101, {}), (100, 5, {"tau": 0.5}),
                                    (30, 2, {"preset": 2, "r": 1.0}), (30, 1, {}), (100, 5, {"ident": 2})])
def test_invalid_plans_rejected_alike(N, s, kw):
    with pytest.raises(ValueError):
        oracle.make_plan(N, s, oracle.Params(**kw))
    with pytest.raises(sftlib.SftError) as ei:
        sftlib.describe(N, s, **kw)
    assert ei.value.code == sftlib.SFT_EINVAL
    assert str(ei.value)


def test_unsupported_sizes():
    with pytest.raises(sftlib.SftError) as ei:
        sftlib.describe(2 ** 31, 4)
    assert ei.value.code == sftlib.SFT_EUNSUPPORTED
    with pytest.raises(sftlib.SftError):
        sftlib.make_params(preset=7)
