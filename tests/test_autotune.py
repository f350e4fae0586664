"""Host logic of the launch-shape autotuner: the shipped MI355X tuning
table covers the workloads' grid classes with valid shapes, lookups prefer
the user cache, and apply() hands every field to the context."""
import json

import numpy as np
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


def test_class_rows_per_mode():
    entry = {0: 48, "two0": True, "rows_one0": 8, "rows_two0": 48, 1: 64, "two1": False, 2: 20, "two2": True,
             3: 28}
    assert autotune.class_rows(entry, 0, True) == 48
    assert autotune.class_rows(entry, 0, False) == 8
    # no per-mode entry: the winner's height when the modes agree, else the default
    assert autotune.class_rows(entry, 1, False) == 64
    assert autotune.class_rows(entry, 1, True) == 0
    assert autotune.class_rows(entry, 2, True) == 20
    assert autotune.class_rows(entry, 3, False) == 28


def test_tune_batch_sets_heights_per_grid_class(tmp_path, monkeypatch):
    """Two grid classes (three instances, one class twice): each class is
    looked up once (with at most 8 shots) and every instance gets its class's
    heights for the batch's launch modes."""
    monkeypatch.setenv("AAFWI_TUNE_CACHE", str(tmp_path))
    ga = synth.make_geometry(64, 96, 10.0, 8, 1e-3, 12, rec_stride=2)
    gb = synth.make_geometry(32, 200, 10.0, 8, 1e-3, 5, rec_stride=2)
    entries = {
        autotune.grid_key(ga.subset_shots(list(range(8)))): {"0": 16, "two0": True, "rows_one0": 12, "rows_two0": 16,
                                                            "1": 24, "two1": False, "2": 32, "two2": True, "3": 40,
                                                            "order0": 0, "order1": 0, "order2": 0, "order3": 0},
        autotune.grid_key(gb): {"0": 8, "two0": False, "rows_one0": 8, "rows_two0": 64, "1": 20, "two1": True,
                                "2": 24, "two2": True, "3": 12, "order0": 0, "order1": 0, "order2": 0, "order3": 0},
    }
    with open(tmp_path / "tiles.json", "w") as f:
        json.dump(entries, f)
    calls = []

    class FakeBatch:
        def time_blocking(self):
            return 0b101  # forward and adjoint two steps per launch, recompute one

        def set_instance_tile(self, i, rows, k):
            calls.append((i, k, rows))

    out = autotune.tune_batch(FakeBatch(), [ga, gb, ga], [None, None, None])
    got = {(i, k): rows for i, k, rows in calls}
    # class a: forward two-step 16, recompute one-step 24, adjoint two-step 32, Born 40
    assert [got[(0, k)] for k in range(4)] == [16, 24, 32, 40] == [got[(2, k)] for k in range(4)]
    # class b: forward two-step 64 (its one-step winner is not the batch's mode),
    # recompute: its winner is two-step, no one-step height stored -> default 0
    assert [got[(1, k)] for k in range(4)] == [64, 0, 24, 12]
    assert len(out) == 2


def test_shipped_network_weights():
    """The network weights that ship with the package load without pickles,
    have the network's parameter count, are finite and carry their training
    provenance (the learned workload's recipe and cost)."""
    import numpy as np
    from paper_2008_11778_amd.learned import SHIPPED_WEIGHTS, shipped_weights
    from paper_2008_11778_amd._lib import CNN_PARAMS
    w, meta = shipped_weights()
    assert w.dtype == np.float32 and w.shape == (CNN_PARAMS,)
    assert np.isfinite(w).all() and np.abs(w).max() > 0
    assert meta["training_cost_s"] > 0 and "bench.py --workload learned" in meta["_about"]
    assert np.array_equal(np.load(SHIPPED_WEIGHTS, allow_pickle=False), w)


def test_family_instances_continue_the_batched_family():
    """Instances drawn from a later index are new members of the same family
    (the grids, spacings and shot counts of the batched workload's table),
    and the batched workload's own 32 are unchanged by the offset."""
    base = synth.config4_instances(32)
    again = synth.config4_instances(4, first=0)
    later = synth.config4_instances(8, first=100)
    for (g0, mt0, m00), (g1, mt1, m01) in zip(base[:4], again):
        assert (g0.nx, g0.nz, g0.h, g0.nt, g0.dt, g0.nshots) == (g1.nx, g1.nz, g1.h, g1.nt, g1.dt, g1.nshots)
        assert np.array_equal(mt0, mt1) and np.array_equal(m00, m01)
    grids = {(128, 128), (256, 128), (384, 128), (512, 256), (768, 256), (1024, 384), (1024, 512)}
    for g, mt, m0 in later:
        assert (g.nx, g.nz) in grids and g.h in (10.0, 12.5, 15.0, 20.0) and 4 <= g.nshots <= 96
        assert not any(mt.shape == b[1].shape and np.array_equal(mt, b[1]) for b in base)
