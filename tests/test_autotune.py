"""Host logic of the launch-shape autotuner: the shipped MI355X tuning
table covers the workloads' grid classes with valid shapes, lookups prefer
the user cache, and apply() hands every field to the context."""
import json

import pytest

import synth
from paper_2008_11778_amd import autotune


def _table():
    with open(autotune.SHIPPED) as f:
        return {k: v for k, v in json.load(f).items() if not k.startswith("_")}


def _valid(shape):
    for k in range(4):
        assert shape[str(k)] in (autotune.CANDIDATES + autotune.CANDIDATES_TWO)
        assert shape[f"order{k}"] in (0, 1)
    for k in range(3):
        assert isinstance(shape[f"two{k}"], bool)
        if not shape[f"two{k}"]:
            assert shape[str(k)] in autotune.CANDIDATES and shape[str(k)] <= 64  # one-step strips
        else:
            assert shape[str(k)] in autotune.CANDIDATES_TWO


@pytest.mark.parametrize("make", [lambda: synth.config2(nt=8), lambda: synth.config3(nt=8),
                                  lambda: synth.config5(nt=8), lambda: synth.learned_instance(0, nt=8),
                                  synth.config1], ids=["fwi", "lsrtm", "large", "learned", "small"])
def test_shipped_table_covers_workload_grids(make):
    g = make()[0]
    table = _table()
    key = autotune.grid_key(g)
    assert key in table, key
    _valid(table[key])


def test_lookup_prefers_user_cache(tmp_path, monkeypatch):
    g = synth.config2(nt=8)[0]
    key = autotune.grid_key(g)
    monkeypatch.setenv("AAFWI_TUNE_CACHE", str(tmp_path))
    shipped = autotune.tune(g, None)  # empty user cache: the shipped entry, no device work
    assert shipped == {(int(k) if k.isdigit() else k): v for k, v in _table()[key].items()}
    mine = {"0": 16, "order0": 0, "two0": True, "1": 24, "order1": 1, "two1": False,
            "2": 32, "order2": 0, "two2": False, "3": 12, "order3": 1}
    with open(tmp_path / "tiles.json", "w") as f:
        json.dump({key: mine}, f)
    got = autotune.tune(g, None)
    assert got[0] == 16 and got["two0"] is True and got[3] == 12 and got["order1"] == 1


def test_apply_sets_every_field():
    calls = []

    class Ctx:
        def set_time_blocking(self, on, k):
            calls.append(("two", k, on))

        def set_tile(self, rows, k):
            calls.append(("rows", k, rows))

        def set_tile_order(self, order, k):
            calls.append(("order", k, order))

    shape = {0: 8, "order0": 1, "two0": False, 1: 48, "order1": 0, "two1": True,
             2: 96, "order2": 1, "two2": True, 3: 64, "order3": 0}
    autotune.apply(Ctx(), shape)
    assert sorted(calls) == sorted([("two", 0, False), ("two", 1, True), ("two", 2, True),
                                    ("rows", 0, 8), ("rows", 1, 48), ("rows", 2, 96), ("rows", 3, 64),
                                    ("order", 0, 1), ("order", 1, 0), ("order", 2, 1), ("order", 3, 0)])
