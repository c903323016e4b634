"""Host logic of bench.py (no GPU): the one-GPU refusal and the rule that a committed
counter summary is used only for the kernel source, launch shape and tile order it was
taken on."""

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


def _profiled_tiles():
    """(tile_x, tile_y, mode) -> HBM bytes per launch of every launch shape in the summary."""
    out = {}
    with open(bench.PMC_FILE) as fh:
        for line in fh:
            m = re.match(r"kernel k_step(_lds|_sf|_sh)?<(\d+),(\d+),\S* .*hbm_bytes_per_launch (\S+)", line)
            if m:
                out[(int(m.group(2)), int(m.group(3)), {None: 0, "_lds": 1, "_sf": 2, "_sh": 3}[m.group(1)])] = float(m.group(4))
    return out


def test_committed_traffic_is_read_only_for_its_own_source_and_launch():
    tiles = _profiled_tiles()
    assert tiles, "the counter summary lists no launch shape"
    current = any(bench.measured_traffic(t) is not None for t in tiles)
    for tile, b in tiles.items():
        t = bench.measured_traffic(tile)
        if not current:
            # the summary predates the current kernel source: then no shape may read it
            assert t is None
            continue
        assert t == b
        assert t > 0.9 * bench.BYTES_PER_CELL * 2048 * 2048   # HBM bytes per launch, about algorithmic or above
    for other in ((512, 1, 0), (16, 16, 2), (64, 4, 1)):
        if other not in tiles:
            assert bench.measured_traffic(other) is None


def test_committed_traffic_is_read_only_for_its_own_tile_order():
    orders = {}
    with open(bench.PMC_FILE) as fh:
        for line in fh:
            m = re.match(r"kernel k_step(_lds|_sf|_sh)?<(\d+),(\d+),.* launch \S+:(\d)", line)
            if m:
                mode = {None: 0, "_lds": 1, "_sf": 2, "_sh": 3}[m.group(1)]
                orders[(int(m.group(2)), int(m.group(3)), mode)] = int(m.group(4))
    assert orders, "the counter summary names no tile order"
    tiles = _profiled_tiles()
    for tile, order in orders.items():
        if bench.measured_traffic(tile) is None:
            continue                       # the summary predates the current kernel source
        assert bench.measured_traffic(tile + (order,)) == tiles[tile]
        assert bench.measured_traffic(tile + (1 - order,)) is None


def test_traffic_is_ignored_when_the_kernel_source_changes(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    for tile in _profiled_tiles():
        assert bench.measured_traffic(tile) is None
