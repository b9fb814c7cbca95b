"""bench.py's contract pieces that need no GPU: one GPU only, and the stored
HBM-traffic record it reads is complete and names the sources it covers."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_records_are_complete():
    sys.path.insert(0, ROOT)
    import bench
    records = list(bench.TRAFFIC_HEADLINE.values()) + [bench.TRAFFIC_BATCH]
    assert any(os.path.exists(path) for path, _ in bench.TRAFFIC_HEADLINE.values())
    for path, srcs in records:
        if not os.path.exists(path):
            continue
        with open(path) as f:
            t = json.load(f)
        for key in ("kernel", "counters", "hbm_bytes_per_launch", "algorithmic_bytes_per_launch",
                    "src", "src_sha256", "command"):
            assert key in t, key
        assert set(t["counters"]) == {"FETCH_SIZE", "WRITE_SIZE"}
        for c in t["counters"].values():
            assert c["dispatches"] > 0 and c["scale"] > 0 and c["bytes_per_dispatch"] > 0
        assert abs(t["hbm_bytes_per_launch"] - sum(c["bytes_per_dispatch"]
                                                   for c in t["counters"].values())) < 1.0
        # the record covers exactly the sources bench hashes, and its command runs
        # committed files only
        names = [os.path.basename(p) for p in srcs]
        assert [os.path.basename(s) for s in t["src"].split(",")] == names
        assert "_work" not in t["command"] and "bench.py" in t["command"]
