"""Host logic of bench.py (no GPU): the one-GPU refusal and the rule that a committed
counter summary is used only for the kernel source and launch shape it was taken on."""

import json
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def _profiled_tile():
    with open(bench.PMC_FILE) as fh:
        text = fh.read()
    m = re.search(r"^kernel k_step(_lds|_sf)?<(\d+),(\d+),", text, re.M)
    return int(m.group(2)), int(m.group(3)), {None: 0, "_lds": 1, "_sf": 2}[m.group(1)]


def test_committed_traffic_is_read_only_for_its_own_source_and_launch():
    tile = _profiled_tile()
    t = bench.measured_traffic(tile)
    if t is None:
        # the summary predates the current kernel source: then no tile may read it
        assert bench.measured_traffic() is None
        return
    assert t > bench.BYTES_PER_CELL * 2048 * 2048          # HBM bytes per launch, above algorithmic
    other = (256, 1, 0) if tile != (256, 1, 0) else (64, 4, 0)
    assert bench.measured_traffic(other) is None
    assert bench.measured_traffic() == t


def test_traffic_is_ignored_when_the_kernel_source_changes(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None
    assert bench.measured_traffic(_profiled_tile()) is None
