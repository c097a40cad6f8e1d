"""CPU checks of bench.py's host logic: the traffic record lookup and the
fixed FLOP units of the roofline."""
import hashlib
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def test_recorded_traffic_follows_the_source_hash(tmp_path):
    files = ["paper_2512_16896_amd/csrc/place.hip", "paper_2512_16896_amd/csrc/device.h"]
    rec = {"k_place demo 0xf04": {"sources": files, "source_sha256": _hash(files),
                                  "bytes_per_launch": 1234}}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(rec))
    assert bench.recorded_traffic("k_place demo 0xf04", str(p)) == 1234
    assert bench.recorded_traffic("k_place other 0xf04", str(p)) is None
    rec["k_place demo 0xf04"]["source_sha256"] = "0" * 64      # sources changed since
    p.write_text(json.dumps(rec))
    assert bench.recorded_traffic("k_place demo 0xf04", str(p)) is None


def test_committed_traffic_records_name_existing_sources():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    for key, rec in json.load(open(path)).items():
        for f in rec["sources"]:
            assert os.path.exists(os.path.join(ROOT, f)), (key, f)
        assert rec["bytes_per_launch"] > 0


def test_flop_units_are_the_fixed_reporting_units():
    assert (bench.FLOP_PAIR, bench.FLOP_BOX, bench.FLOP_GRID, bench.FLOP_XFORM) == (11, 26, 45, 10)


def test_multi_gpu_request_exits_with_a_message(capsys, monkeypatch):
    import pytest
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err
