"""The tracer schedule table on the CPU: forcing, lookup by class, JSON
persistence keyed by device architecture.  No kernel runs here; the GPU tests
check that every schedule gives the same bits and exercise the autotuner."""
import json

import pytest

from paper_1811_02357_amd import irtps


@pytest.fixture(autouse=True)
def clean_table():
    irtps.set_schedule(0, 0)
    irtps.tuning_clear()
    yield
    irtps.set_schedule(0, 0)
    irtps.tuning_clear()
    irtps.load_shipped_tuning()


def _arch(tmp_path):
    p = tmp_path / "empty.json"
    irtps.tuning_save(p)
    doc = json.loads(p.read_text())
    assert doc["entries"] == []
    return doc["arch"]


def test_default_and_forced_schedule():
    assert irtps.get_schedule(2048, 2048, 3, 16, 3) == {"tile_w": 16, "ready_batch": 32}
    irtps.set_schedule(64, 0)
    assert irtps.get_schedule(2048, 2048, 3, 16, 3) == {"tile_w": 64, "ready_batch": 32}
    irtps.set_ready_batch(8)
    assert irtps.get_ready_batch() == 8
    assert irtps.get_schedule(100, 100, 1, 8, 1) == {"tile_w": 64, "ready_batch": 8}
    irtps.set_schedule(0, 0)
    assert irtps.get_schedule(100, 100, 1, 8, 1) == {"tile_w": 16, "ready_batch": 32}


@pytest.mark.parametrize("tw,rb", [(12, 0), (4, 0), (128, 0), (0, 65), (0, -1)])
def test_invalid_schedules_refused(tw, rb):
    with pytest.raises(RuntimeError):
        irtps.set_schedule(tw, rb)


def test_table_lookup_save_load(tmp_path):
    arch = _arch(tmp_path)
    # side class round(log2 sqrt(W H)): 2048^2 -> 11; K 16 -> 4; 1000 x 1100 -> 10; K 9 -> 4
    doc = {"arch": arch, "entries": [
        {"side": 11, "kcls": 4, "C": 3, "B": 3, "tile_w": 32, "ready_batch": 24, "ms": 150.0},
        {"side": 10, "kcls": 4, "C": 1, "B": 2, "tile_w": 8, "ready_batch": 48, "ms": 20.0},
        {"side": 9, "kcls": 3, "C": 1, "B": 2, "tile_w": 12, "ready_batch": 48, "ms": 1.0},  # invalid width
    ]}
    src = tmp_path / "t.json"
    src.write_text(json.dumps(doc))
    assert irtps.tuning_load(src) == 2
    assert irtps.tuning_entries() == 2
    assert irtps.get_schedule(2048, 2048, 3, 16, 3) == {"tile_w": 32, "ready_batch": 24}
    assert irtps.get_schedule(1000, 1100, 1, 9, 2) == {"tile_w": 8, "ready_batch": 48}
    assert irtps.get_schedule(2048, 2048, 1, 16, 3) == {"tile_w": 16, "ready_batch": 32}  # other class
    irtps.set_schedule(0, 16)  # a forced field wins over the table
    assert irtps.get_schedule(2048, 2048, 3, 16, 3) == {"tile_w": 32, "ready_batch": 16}
    irtps.set_schedule(0, 0)
    out = tmp_path / "out.json"
    irtps.tuning_save(out)
    irtps.tuning_clear()
    assert irtps.tuning_entries() == 0
    assert irtps.tuning_load(out) == 2
    assert irtps.get_schedule(2048, 2048, 3, 16, 3) == {"tile_w": 32, "ready_batch": 24}


def test_other_architecture_loads_nothing(tmp_path):
    arch = _arch(tmp_path)
    doc = {"arch": arch + "x", "entries": [
        {"side": 11, "kcls": 4, "C": 3, "B": 3, "tile_w": 32, "ready_batch": 24, "ms": 150.0}]}
    src = tmp_path / "t.json"
    src.write_text(json.dumps(doc))
    assert irtps.tuning_load(src) == 0
    assert irtps.get_schedule(2048, 2048, 3, 16, 3) == {"tile_w": 16, "ready_batch": 32}
    with pytest.raises(RuntimeError):
        irtps.tuning_load(tmp_path / "missing.json")
