"""Host logic of bench.py (no GPU): the traffic records the bench line's roofline reads and
the names of the kernels it reports."""
import json
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _write(tmp_path, records):
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({"records": records}))
    return str(p)


def _rec(kernel, xcd, nbytes, source_hash=None, workload="soil512"):
    return {"kernel": kernel, "workload": workload, "xcd_map": xcd, "hbm_bytes_per_launch": nbytes,
            "source_hash": source_hash if source_hash is not None else bench.source_hash()}


def test_traffic_record_keyed_by_kernel_and_block_order(tmp_path):
    k_cmp, k_blk = "k_step8z<float,2,true,true,true>", "k_step8z<float,2,true,false,true>"
    path = _write(tmp_path, [_rec(k_blk, 1, 1.0e9), _rec(k_cmp, 0, 1.3e9), _rec(k_cmp, 1, 0.9e9)])
    assert bench.load_traffic(path, k_cmp, "soil512", 0) == 1.3e9
    assert bench.load_traffic(path, k_cmp, "soil512", 1) == 0.9e9
    assert bench.load_traffic(path, k_blk, "soil512", True) == 1.0e9
    assert bench.load_traffic(path, k_blk, "soil512", 0) is None  # not measured
    assert bench.load_traffic(path, k_cmp, "soil256", 0) is None  # other workload


def test_traffic_record_of_other_sources_ignored(tmp_path):
    k = "k_step8z<float,2,true,true,true>"
    path = _write(tmp_path, [_rec(k, 0, 1.3e9, source_hash="0000000000000000")])
    assert bench.load_traffic(path, k, "soil512", 0) is None
    assert bench.load_traffic(str(tmp_path / "missing.json"), k, "soil512", 0) is None


def test_committed_traffic_records_well_formed():
    recs = json.load(open(bench.TRAFFIC_FILE))["records"]
    assert recs, "no traffic records"
    for r in recs:
        assert r["workload"] == "soil512" and r["xcd_map"] in (0, 1)
        assert r["hbm_bytes_per_launch"] > 6.4e8  # at least the algorithmic bytes of soil512


@pytest.mark.parametrize("launch,name", [
    ({"kernel": "column_xch", "layout": "compact"}, "k_step8z<float,2,true,true,true>"),
    ({"kernel": "column_xch", "layout": "blocks"}, "k_step8z<float,2,true,false,true>"),
    ({"kernel": "column", "layout": "compact"}, "k_step8z<float,2,false,true,true>"),
    ({"kernel": "column_lanes", "layout": "compact"}, "k_step8l<float,2,true>"),
    ({"kernel": "block", "layout": "blocks"}, "k_step8<float,2,true>"),
])
def test_step_kernel_names(launch, name):
    assert bench.step_kernel_name(8, launch, 2) == name
