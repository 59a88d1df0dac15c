"""Host logic of the autotuner: selection rule and cache."""
import os

from paper_2606_11529_amd import autotune as A
from paper_2606_11529_amd import renderer as R


def test_pick_best_median_and_tie_order():
    t = {(64, 1): [5.0, 5.1, 9.0], (128, 2): [3.95, 3.96, 3.95], (256, 4): [3.9, 3.9, 3.95]}
    # (128, 2) is within 2% of the fastest and listed first
    assert A.pick_best(t) == (128, 2)
    assert A.pick_best(t, tie=0.0) == (256, 4)
    assert A.pick_best({"a": [1.0]}) == "a"


def test_cache_roundtrip(tmp_path):
    path = os.path.join(tmp_path, "tune.json")
    key = A.cache_key("MI355X", 3_000_000, 3, [(1600, 1064)], (16,))
    assert "n=3000000" in key and "1600x1064" in key
    r = A.TuneResult(16, "presort", 256, 2, 128, 4, {"x": 1.0})
    c = A.load_cache(path)
    assert c == {}
    c[key] = r.__dict__
    A.save_cache(path, c)
    back = A.TuneResult(**A.load_cache(path)[key])
    assert back == r
    cfg = back.apply(R.Config())
    assert (cfg.lds_batch, cfg.fwd_ppt, cfg.bwd_lds_batch, cfg.bwd_ppt) == (256, 2, 128, 4)
    assert cfg.to_c().bwd_lds_batch == 128


def test_schedule_applies_order_and_persistence():
    base = A.TuneResult(16, "presort", 256, 1, 64, 4, {})
    assert base.schedule == "index"
    c = base.apply(R.Config(persistent=True, tile_order=True))
    assert not c.tile_order and not c.persistent and c.to_c().persistent == 0
    lf = A.TuneResult(16, "presort", 256, 1, 64, 4, {}, schedule="longest_first").apply(R.Config())
    assert lf.tile_order and not lf.persistent
    ps = A.TuneResult(16, "presort", 256, 1, 64, 4, {}, schedule="persistent").apply(R.Config())
    assert ps.tile_order and ps.persistent and ps.to_c().persistent == 1
    # cache entries written before the schedule phase still load
    old = {k: v for k, v in base.__dict__.items() if k != "schedule"}
    assert A.TuneResult(**old).schedule == "index"
