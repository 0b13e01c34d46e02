"""Host-side tests of plan selection (fracsolve_plan, the plan cache read by
fracsolve_create for leaf = 0 / crossover = 0) and of the tuner's file
format.  No GPU is needed: the plan is resolved on the host."""
import json
import os

import pytest

from paper_1710_11593_amd import binding, tune

PROB = dict(gamma=0.5, M=300, N=1000)


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "plan.json"
    monkeypatch.setenv("FRACSOLVE_TUNE_CACHE", str(path))
    monkeypatch.delenv("FRACSOLVE_TUNE", raising=False)
    return path


def builtin(problems=(PROB,), **kw):
    old = os.environ.get("FRACSOLVE_TUNE")
    os.environ["FRACSOLVE_TUNE"] = "0"
    try:
        return binding.plan(list(problems), **kw)
    finally:
        if old is None:
            del os.environ["FRACSOLVE_TUNE"]
        else:
            os.environ["FRACSOLVE_TUNE"] = old


def entries(*rows):
    return {"fracsolve_plan": 1, "entries": [dict(zip(("precision", "equation", "m_max", "leaf", "crossover"), r))
                                             for r in rows]}


def test_without_a_cache_file_the_builtin_table_is_used(cache):
    lf, cr, src = binding.plan([PROB])
    assert src == "builtin"
    assert (lf, cr) == builtin()[:2]
    assert lf in (4, 8, 16) and (cr == -1 or 16 <= cr <= 1024)


def test_explicit_options_win(cache):
    cache.write_text(json.dumps(entries((0, 0, 4096, 4, 256))))
    assert binding.plan([PROB], leaf=16, crossover=128) == (16, 128, "options")
    assert binding.plan([PROB], leaf=4, crossover=-5) == (4, -1, "options")
    lf, cr, src = binding.plan([PROB], leaf=16)          # crossover from the cache
    assert (lf, cr, src) == (16, 256, "cache")


def test_cache_entry_of_the_smallest_matching_bucket(cache):
    cache.write_text(json.dumps(entries((0, 0, 128, 4, 32), (0, 0, 512, 8, 256), (0, 0, 4096, 8, 512),
                                        (1, 0, 512, 4, 1024))))
    assert binding.plan([dict(PROB, M=100)]) == (4, 32, "cache")
    assert binding.plan([dict(PROB, M=128)]) == (4, 32, "cache")
    assert binding.plan([dict(PROB, M=129)]) == (8, 256, "cache")
    assert binding.plan([dict(PROB, M=3000)]) == (8, 512, "cache")
    assert binding.plan([dict(PROB, M=300)], precision="fp32") == (4, 1024, "cache")
    # a batch is planned for its widest instance, its float64 crossover
    # capped at 128
    assert binding.plan([dict(PROB, M=100), dict(PROB, M=3000)]) == (8, 128, "cache")
    assert binding.plan([dict(PROB, M=100), dict(PROB, M=300)], precision="fp32") == (4, 1024, "cache")
    # no entry for this equation: built-in
    assert binding.plan([dict(PROB, gamma=1.5)], equation="diffusion_cn")[2] == "builtin"


def test_batches_cap_the_float64_crossover_at_128():
    one = builtin([dict(PROB, M=4000)])
    two = builtin([dict(PROB, M=4000), dict(PROB, M=64)])
    assert two[0] == one[0] and two[1] == min(one[1], 128)
    small = builtin([dict(PROB, M=500)] * 3)
    assert small[1] <= 128 and builtin([dict(PROB, M=500)])[1] > 128
    # an explicit crossover is taken as given
    assert builtin([PROB, PROB], crossover=512)[1] == 512


def test_no_matching_entry_falls_back(cache):
    cache.write_text(json.dumps(entries((0, 0, 128, 4, 32))))
    assert binding.plan([dict(PROB, M=129)]) == builtin([dict(PROB, M=129)])
    assert binding.plan([PROB], precision="fp32")[2] == "builtin"


@pytest.mark.parametrize("text", [
    "",
    "not json",
    '{"fracsolve_plan": 1, "entries": [',                                  # truncated
    '{"fracsolve_plan": 2, "entries": []}',                                 # unknown version
    '{"entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": 4, "crossover": 32}]}',
    '{"fracsolve_plan": 1, "entries": {"precision": 0}}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": 5, "crossover": 32}]}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": 4, "crossover": 0}]}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": 4, "crossover": 2048}]}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": -3, "leaf": 4, "crossover": 32}]}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": 4.5, "crossover": 32}]}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": "4", "crossover": 32}]}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": 4}]}',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 4096, "leaf": 4, "crossover": 32}]} x',
    '{"fracsolve_plan": 1, "entries": [{"precision": 0, "equation": 0, "m_max": 1e999, "leaf": 4, "crossover": 32}]}',
    '[' * 64 + ']' * 64,                                                    # deep nesting
    '\x00\x01\x02',
])
def test_corrupt_cache_falls_back_to_the_builtin_table(cache, text):
    cache.write_text(text)
    assert binding.plan([PROB]) == builtin()


def test_a_malformed_entry_discards_the_whole_file(cache):
    good = {"precision": 0, "equation": 0, "m_max": 4096, "leaf": 4, "crossover": 32}
    bad = dict(good, leaf=7)
    cache.write_text(json.dumps({"fracsolve_plan": 1, "entries": [good, bad]}))
    assert binding.plan([PROB]) == builtin()


def test_tune_off_ignores_the_cache(cache, monkeypatch):
    cache.write_text(json.dumps(entries((0, 0, 4096, 4, 32))))
    assert binding.plan([PROB]) == (4, 32, "cache")
    monkeypatch.setenv("FRACSOLVE_TUNE", "0")
    assert binding.plan([PROB])[2] == "builtin"


def test_unknown_keys_are_ignored(cache):
    plan = entries((0, 0, 4096, 4, 32))
    plan["device"] = "gfx950"
    plan["timings_ms"] = {"x": 1.0}
    plan["entries"][0]["ms"] = 12.5
    cache.write_text(json.dumps(plan))
    assert binding.plan([PROB]) == (4, 32, "cache")


def test_leaf_16_from_the_cache_needs_narrow_leaf_threads(cache):
    cache.write_text(json.dumps(entries((0, 0, 64, 16, 64), (0, 0, 4096, 16, 64), (0, 1, 4096, 16, 64))))
    assert binding.plan([dict(PROB, M=64)])[0] == 16
    assert binding.plan([dict(PROB, M=4096)])[0] == 8         # the scan leaf at M = 4096 holds 8 rows per thread
    assert binding.plan([dict(PROB, M=64)], equation="advection") == (8, 64, "cache")   # advection leaf: L <= 8


def test_plan_rejects_bad_problems(cache):
    with pytest.raises(binding.FracsolveError, match="gamma"):
        binding.plan([dict(PROB, gamma=1.0)])
    with pytest.raises(binding.FracsolveError, match="leaf"):
        binding.plan([PROB], leaf=5)


def test_tuner_output_is_read_back(cache):
    """The tuner's file format (written by tune.write) is what the library reads."""
    plan = {"fracsolve_plan": 1, "device": "x", "N": 16384, "reps": 3,
            "entries": [{"precision": 0, "equation": 0, "m_max": 256, "leaf": 4, "crossover": 128, "ms": 1.0},
                        {"precision": 0, "equation": 0, "m_max": 1 << 20, "leaf": 8, "crossover": 256, "ms": 2.0}],
            "timings_ms": {"fp64 M=256 L=4 s*=128": 1.0, "fp64 M=256 L=16 s*=64": None}}
    tune.write(plan, str(cache))
    assert binding.plan([dict(PROB, M=200)]) == (4, 128, "cache")
    assert binding.plan([dict(PROB, M=3000)]) == (8, 256, "cache")


def test_default_path_follows_the_library(monkeypatch, tmp_path):
    monkeypatch.setenv("FRACSOLVE_TUNE_CACHE", str(tmp_path / "a.json"))
    assert tune.default_path() == str(tmp_path / "a.json")
    monkeypatch.delenv("FRACSOLVE_TUNE_CACHE")
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    assert tune.default_path() == str(tmp_path / "fracsolve" / "plan.json")
