"""Host logic of the autotuner: size buckets, the choice among timed
candidates (fastest admissible, earlier on ties), the table round trip and
what apply_table sets on a context."""
import json

from paper_2606_03140_amd import autotune


def test_buckets():
    assert autotune.bucket(1) == "n<=256"
    assert autotune.bucket(256) == "n<=256"
    assert autotune.bucket(257) == "n<=512"
    assert autotune.bucket(628) == "n<=1024"
    assert autotune.bucket(1673) == "n<=2048"


def test_pick_fastest_admissible():
    res = [{"opts": {"a": 1}, "ms": 5.0, "ok": True}, {"opts": {"a": 2}, "ms": 3.0, "ok": False},
           {"opts": {"a": 3}, "ms": 4.0, "ok": True}, {"opts": {"a": 4}, "ms": 4.0, "ok": True}]
    assert autotune.pick(res)["opts"] == {"a": 3}
    assert autotune.pick([{"opts": {}, "ms": 1.0, "ok": False}]) is None
    assert autotune.pick([{"opts": {"leaf_rows": 32}, "ms": 2.0}])["opts"] == {"leaf_rows": 32}


class FakeCtx:
    def __init__(self):
        self.calls = []

    def set_fp64_options(self, leaf_rows):
        self.calls.append(("fp64", leaf_rows))

    def set_mixed_storage(self, upper):
        self.calls.append(("storage", upper))

    def set_mixed_inverse_start(self, degree):
        self.calls.append(("inv_start", degree))

    def set_mixed_options(self, ns_inv=0):
        self.calls.append(("ns_inv", ns_inv))


def test_table_round_trip_and_apply(tmp_path):
    table = {"n<=1024": {"fp64": {"choice": {"leaf_rows": 32}, "ms": 1.0},
                         "mixed": {"choice": {"upper_tiles": 0, "ns_inv": 3}, "ms": 2.0}}}
    f = tmp_path / "t.json"
    autotune.save_table(table, str(f))
    assert autotune.load_table(str(f)) == json.loads(f.read_text())
    assert autotune.load_table(str(tmp_path / "missing.json")) == {}
    c = FakeCtx()
    used = autotune.apply_table(c, table, 628, paths=("fp64", "mixed"))
    assert used == {"fp64": {"leaf_rows": 32}, "mixed": {"upper_tiles": 0, "ns_inv": 3}}
    # an entry without "inv_start" predates the quartic start: quadratic
    assert c.calls == [("fp64", 32), ("storage", False), ("inv_start", 2), ("ns_inv", 3)]
    # a bucket without an entry falls back to the library defaults
    c = FakeCtx()
    used = autotune.apply_table(c, table, 1673, paths=("fp64", "mixed"))
    assert used == {"fp64": {"leaf_rows": 64}, "mixed": {"upper_tiles": 1, "inv_start": 4, "ns_inv": 1}}
    assert c.calls == [("fp64", 64), ("storage", True), ("inv_start", 4), ("ns_inv", 1)]
