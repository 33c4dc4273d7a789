"""Host logic of bench.py (no GPU): the kernel-code hash that keys the measured
HBM traffic, and the refusal of more than one GPU."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.fixture()
def src_copy(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2206_00366_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2206_00366_amd", "csrc", f), csrc / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return csrc


def test_hash_ignores_comments_and_blank_lines(src_copy):
    h0 = bench.kernel_source_hash()
    assert len(h0) == 16 and int(h0, 16) >= 0
    p = src_copy / bench.KERNEL_SOURCES[1]
    text = p.read_text()
    p.write_text("// a new comment line\n\n" + text.replace("\n", "  // trailing note\n", 3))
    assert bench.kernel_source_hash() == h0


def test_hash_changes_with_the_code(src_copy):
    h0 = bench.kernel_source_hash()
    p = src_copy / bench.KERNEL_SOURCES[0]
    p.write_text(p.read_text() + "\nstatic const int kUnused = 1;\n")
    assert bench.kernel_source_hash() != h0


def test_measured_traffic_is_close_to_the_algorithmic_bytes():
    # each stored figure is HBM bytes per launch of the headline step (2 x 19 x 4 B
    # per node of 256 x 256 x 128); a kernel that re-read populations would show more
    algorithmic = 2 * 19 * 4 * 256 * 256 * 128
    for key, traffic in bench.MEASURED_TRAFFIC.items():
        assert len(key) == 16
        assert 0.99 < traffic / algorithmic < 1.01


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    msg = json.loads(res.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
