"""Host logic of the autotune cache (no device)."""
from paper_2012_04838_amd import tune


class FakePlan:
    n, n_scalars, precision, batch = 64, 2, 32, 4
    n_schedules = 3

    def __init__(self, widths=(16, 16, 8)):
        self.widths = widths
        self.chosen = None
        self.timed = 0

    def schedule_info(self, i):
        return {"index": i, "col_width": self.widths[i]}

    def set_schedule(self, i):
        self.chosen = i

    def tune(self, state, ws, reps):
        self.timed += 1
        self.chosen = 2
        return 2, [3.0, 2.5, 1.0]


def test_cache_roundtrip_and_hit(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    p = FakePlan()
    assert tune.autotune(p, None, None, cache=tune.TuneCache(path), device="dev") == 2
    assert p.timed == 1
    q = FakePlan()
    assert tune.autotune(q, None, None, cache=tune.TuneCache(path), device="dev") == 2
    assert q.timed == 0 and q.chosen == 2


def test_key_separates_devices_shapes_and_schedule_tables(tmp_path):
    p = FakePlan()
    k = tune.cache_key("dev", p)
    assert k != tune.cache_key("other", p)
    q = FakePlan(widths=(16, 8, 8))
    assert tune.cache_key("dev", q) != k
    r = FakePlan()
    r.batch = 8
    assert tune.cache_key("dev", r) != k


def test_corrupt_or_out_of_range_entries_are_ignored(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    c = tune.TuneCache(str(path))
    assert c.get("x") is None
    p = FakePlan()
    c.put(tune.cache_key("dev", p), 7, [1.0])  # index beyond the compiled schedules
    assert tune.autotune(p, None, None, cache=tune.TuneCache(str(path)), device="dev") == 2
    assert p.timed == 1
