"""The autotuner's result cache (host logic, no GPU): a miss runs the
timing and stores its result, a hit returns it without timing, and a
damaged or foreign file is treated as empty."""
import json

from paper_2308_12698_amd.sim import autotune_cached


def test_miss_runs_then_hit_returns_the_stored_shape(tmp_path):
    path = str(tmp_path / "tune.json")
    calls = []

    def run():
        calls.append(1)
        return {"block": 128, "steps_per_launch": 1000, "grid_blocks": 0}

    assert autotune_cached(path, "k1", run) == run()
    assert len(calls) == 2                       # the miss and the direct call above
    assert autotune_cached(path, "k1", lambda: 1 / 0) == {"block": 128, "steps_per_launch": 1000,
                                                          "grid_blocks": 0}
    other = autotune_cached(path, "k2", lambda: {"block": 256, "steps_per_launch": 500, "grid_blocks": 2048})
    assert other["block"] == 256
    table = json.load(open(path))
    assert set(table) == {"k1", "k2"}


def test_damaged_or_foreign_files_are_treated_as_empty(tmp_path):
    path = tmp_path / "tune.json"
    shape = {"block": 64, "steps_per_launch": 25, "grid_blocks": 0}
    for content in ("{not json", "[1, 2, 3]", json.dumps({"k": {"block": 64}})):
        path.write_text(content)
        assert autotune_cached(str(path), "k", lambda: dict(shape)) == shape
        assert json.load(open(path))["k"] == shape
