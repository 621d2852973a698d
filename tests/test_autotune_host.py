"""Host logic of the per-(T, m) bucket tuner: bucket keys, the per-shape table
derived from a stored bucket table, and what store_buckets keeps."""
import json

from paper_2109_10392_amd import autotune as A


def test_bucket_of_groups_horizon_and_sixteen_obstacle_counts():
    assert A.bucket_of((100, 10.0, 0)) == "T100/m0-15"
    assert A.bucket_of((100, 10.0, 15)) == "T100/m0-15"
    assert A.bucket_of((100, 10.0, 16)) == "T100/m16-31"
    assert A.bucket_of((50, 5.0, 64)) == "T50/m64-79"
    assert A.bucket_of((150, 15.0, 47)) == "T150/m32-47"


def test_shape_groups_from_a_bucket_table():
    shapes = [(100, 10.0, 3), (100, 10.0, 20), (50, 5.0, 20), (150, 15.0, 64)]
    assert A.shape_groups(shapes, None) == [0, 0, 0, 0]
    assert A.shape_groups(shapes, {}) == [0, 0, 0, 0]
    assert A.shape_groups(shapes, {"T100/m16-31": 12, "T150/m64-79": 8}) == [0, 12, 0, 8]


def test_store_buckets_keeps_only_sizes_other_than_the_tile(tmp_path):
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps({"uneven/fp32": {"kernel": "group", "group": 16, "persistent": True, "waves": 1,
                                                "ms": 15.0}}))
    A.store_buckets("uneven", "fp32", {"T50/m0-15": 16, "T100/m16-31": 12}, 14.8, 15.0,
                    {"T100/m16-31": {12: 14.812, 8: 15.5}}, path=str(path))
    entry = json.loads(path.read_text())["uneven/fp32"]
    assert entry["buckets"] == {"T100/m16-31": 12}
    assert entry["buckets_ms"] == 14.8 and entry["single_tile_ms"] == 15.0
    assert entry["bucket_sweep"] == {"T100/m16-31": {"12": 14.812, "8": 15.5}}
    assert entry["group"] == 16 and entry["kernel"] == "group"


def test_the_stored_uneven_table_runs_the_single_tile():
    tile = A.lookup("uneven", "fp32")
    assert tile is not None and tile[0] == "group"
    assert A.lookup_buckets("uneven", "fp32") == {}
