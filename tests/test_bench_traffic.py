"""bench.py reports a stored HBM-traffic figure only when the record was
taken with the kernel source and the tile of the run (host logic, no GPU)."""
import json
import os

import bench


def test_stored_traffic_matches_source_and_tile(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "yy_kernels.hip"
    src.write_text("kernel source v1\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    tiles = json.dumps({"res.u_p": "lds64x4k", "res.T": "lds64x8k"})
    rec = {"tile": "lds64x4k", "source_sha256": bench.kernel_source_sha(), "bytes_per_launch": 123.0}
    (prof / "traffic_residual_up_fp64_lds64x4k.json").write_text(json.dumps(rec))
    assert bench.stored_traffic("residual_up", "fp64", tiles) == 123.0
    # another tile in the run: no record for it
    other = json.dumps({"res.u_p": "lds64x8k"})
    assert bench.stored_traffic("residual_up", "fp64", other) is None
    # no tiles, or a class without records
    assert bench.stored_traffic("residual_up", "fp64", None) is None
    assert bench.stored_traffic("sweep_p", "fp64", tiles) is None
    # the kernel source changed since the counters were taken
    src.write_text("kernel source v2\n")
    assert bench.stored_traffic("residual_up", "fp64", tiles) is None


def test_committed_records_name_their_tile_and_source():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prof = os.path.join(root, "profiles")
    names = [n for n in os.listdir(prof) if n.startswith("traffic_residual_")]
    assert names
    for n in names:
        with open(os.path.join(prof, n)) as fh:
            rec = json.load(fh)
        assert n.endswith("_%s.json" % rec["tile"])
        assert len(rec["source_sha256"]) == 64 and rec["bytes_per_launch"] > 0
