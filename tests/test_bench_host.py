"""bench.py's host-side helpers: the committed counter summaries are read only while the
kernel sources they were taken with are unchanged, and the weights' description comes
from their record."""
import json

import bench


def test_conv_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    hbm, alg = bench.measured_traffic()
    assert hbm is not None and alg is not None and 1.0 <= hbm / alg < 1.5
    changed = tmp_path / "mgnet.hip"
    changed.write_bytes(open(bench.CONV_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "CONV_SOURCE", str(changed))
    assert bench.measured_traffic() == (None, None)


def test_apply_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    got = bench.measured_apply_traffic()
    assert set(got) == {"512x512_64dir", "64x64x64_96dir"}
    # at least the algorithmic bytes: 4 B in + 4 B out per unknown + 8 B per cell
    assert got["512x512_64dir"] >= 8 * 512 * 512 * 64 + 8 * 512 * 512
    changed = tmp_path / "apply.hip"
    changed.write_bytes(open(bench.APPLY_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "APPLY_SOURCE", str(changed))
    assert bench.measured_apply_traffic() == {}


def test_trained_description_is_the_record():
    rec = json.load(open(bench.TRAINED[:-len(".mgn1")] + ".json"))["record"]
    d = bench.trained_description()
    assert "%d steps" % rec["steps"] in d and "c2_mgnet.json" in d
