"""bench.py's host-side contract: more than one GPU is refused with a
message before anything touches a GPU, and the per-form byte accounting and
counter bookkeeping are consistent."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""


def test_counter_files_match_their_forms():
    import bench

    for st, name in bench.STORAGE_NAME.items():
        path = bench.counter_file(st)
        if not os.path.exists(path):
            continue
        c = json.load(open(path))
        assert f"St{ {0: 64, 1: 32, 2: 16}[st] }" in c["kernel"].replace(" ", "")
        assert c["algorithmic_bytes_per_launch"] == 512 ** 3 * bench.BYTES_PER_CELL[st]
        assert abs(c["hbm_bytes_per_launch"] - c["hbm_read_bytes_per_launch"] - c["hbm_write_bytes_per_launch"]) < 1.0
        # a fresh counter file is the one bench.py reports as traffic
        if c["kernel_src_sha"] == bench.kernel_source_hash():
            assert bench.measured_traffic(st)[0] == c["hbm_bytes_per_launch"]
