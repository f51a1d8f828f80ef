"""Host-side checks of the tuning table (no GPU needed): JSON round trip, merge order,
and the errors for unreadable, malformed or out-of-range files.  The package's shipped
table must parse and hold only valid choices."""
import json
import os

import pytest

from paper_1906_11029_amd import mtp


@pytest.fixture(autouse=True)
def empty_table():
    mtp.mtp_tune_clear()
    yield
    mtp.mtp_tune_clear()


def _entry(key, **kw):
    e = {"key": key, "schedule": 0, "tile_order": 0, "grid_frac": 1.0, "ms_best": 1.0, "ms_default": 1.0,
         "candidates": 1}
    e.update(kw)
    return e


def _write(path, entries, fmt="mtp-tuning-1"):
    with open(path, "w") as f:
        json.dump({"format": fmt, "entries": entries}, f)


def test_round_trip_and_merge(tmp_path):
    a = tmp_path / "a.json"
    _write(a, [_entry("solver|x|d3|p4", schedule=1, tile_order=2, grid_frac=0.75, ms_best=2.5, ms_default=3.0,
                      candidates=7),
               _entry("batch|x|d2|p2345", tile_order=3)])
    mtp.mtp_tune_load(str(a))
    assert mtp.mtp_tune_size() == 2
    b = tmp_path / "b.json"
    mtp.mtp_tune_save(str(b))
    got = json.load(open(b))
    assert got["format"] == "mtp-tuning-1"
    by_key = {e["key"]: e for e in got["entries"]}
    assert by_key["solver|x|d3|p4"] == _entry("solver|x|d3|p4", schedule=1, tile_order=2, grid_frac=0.75,
                                             ms_best=2.5, ms_default=3.0, candidates=7)
    assert by_key["batch|x|d2|p2345"]["tile_order"] == 3
    # a later file replaces entries of the same key and keeps the others
    c = tmp_path / "c.json"
    _write(c, [_entry("solver|x|d3|p4", schedule=0, tile_order=1), _entry("solver|y", grid_frac=0.5)])
    mtp.mtp_tune_load(str(c))
    assert mtp.mtp_tune_size() == 3
    mtp.mtp_tune_save(str(b))
    by_key = {e["key"]: e for e in json.load(open(b))["entries"]}
    assert by_key["solver|x|d3|p4"]["schedule"] == 0 and by_key["solver|x|d3|p4"]["tile_order"] == 1
    assert by_key["solver|y"]["grid_frac"] == 0.5
    mtp.mtp_tune_clear()
    assert mtp.mtp_tune_size() == 0


def test_missing_members_take_defaults(tmp_path):
    a = tmp_path / "a.json"
    _write(a, [{"key": "k", "extra": [1, {"x": None}], "ok": True}])
    mtp.mtp_tune_load(str(a))
    mtp.mtp_tune_save(str(a))
    e = json.load(open(a))["entries"][0]
    assert (e["schedule"], e["tile_order"], e["grid_frac"]) == (0, 0, 1.0)


@pytest.mark.parametrize("bad", [
    _entry("k", schedule=2), _entry("k", tile_order=4), _entry("k", tile_order=-1), _entry("k", grid_frac=0.0),
    _entry("k", grid_frac=1.5), {"schedule": 1}, _entry("k", schedule="dag")])
def test_out_of_range_entries_are_rejected_whole(tmp_path, bad):
    a = tmp_path / "a.json"
    _write(a, [_entry("good"), bad])
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_tune_load(str(a))
    assert e.value.code == -1
    assert mtp.mtp_tune_size() == 0   # nothing of a rejected file is merged


@pytest.mark.parametrize("text", ["", "{", '{"format": "mtp-tuning-1", "entries": [}', "[1, 2]",
                                  '{"format": "other", "entries": []}', '{"format": "mtp-tuning-1"}',
                                  '{"format": "mtp-tuning-1", "entries": []} trailing'])
def test_malformed_files(tmp_path, text):
    a = tmp_path / "a.json"
    a.write_text(text)
    with pytest.raises(mtp.MTPError) as e:
        mtp.mtp_tune_load(str(a))
    assert e.value.code == -1


def test_unreadable_and_unwritable_paths(tmp_path):
    with pytest.raises(mtp.MTPError):
        mtp.mtp_tune_load(str(tmp_path / "missing.json"))
    with pytest.raises(mtp.MTPError):
        mtp.mtp_tune_save(str(tmp_path / "no" / "such" / "dir.json"))


def test_shipped_table_is_valid():
    if not os.path.exists(mtp.TUNE_FILE):
        pytest.skip("no tuning table shipped")
    mtp.mtp_tune_load(mtp.TUNE_FILE)
    entries = json.load(open(mtp.TUNE_FILE))["entries"]
    assert mtp.mtp_tune_size() == len({e["key"] for e in entries}) > 0
    for e in entries:
        assert e["key"].split("|")[0] in ("solver", "batch")
        assert e["ms_best"] <= e["ms_default"]
