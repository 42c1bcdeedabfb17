"""Host-side logic of the benchmark (no GPU): the one-GPU guard and the rule
that the HBM traffic figure is used only while the residual kernel's sources
are the ones its byte counters were taken from."""
import hashlib
import os
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _tree(tmp_path, profile_text):
    csrc = tmp_path / "paper_2510_02156_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("k_resid.hip", "rorbk_device.h", "xgram.h"):
        shutil.copy(os.path.join(ROOT, "paper_2510_02156_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_resid_dense_f32_tall_100000x2000.md").write_text(profile_text)
    return tmp_path


def _sha():
    h = hashlib.sha256()
    for f in ("k_resid.hip", "rorbk_device.h", "xgram.h"):
        with open(os.path.join(ROOT, "paper_2510_02156_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def test_traffic_used_when_sources_match(tmp_path, monkeypatch):
    text = f"- kernel_source_sha256: {_sha()}\n  traffic_bytes_per_launch: 801000000 (x)\n"
    monkeypatch.setattr(bench, "ROOT", str(_tree(tmp_path, text)))
    assert bench.measured_traffic("tall_100000x2000", "f32") == 801000000


def test_traffic_dropped_when_sources_changed(tmp_path, monkeypatch):
    text = f"- kernel_source_sha256: {'0' * 64}\n  traffic_bytes_per_launch: 801000000 (x)\n"
    monkeypatch.setattr(bench, "ROOT", str(_tree(tmp_path, text)))
    assert bench.measured_traffic("tall_100000x2000", "f32") is None


def test_traffic_absent_without_a_profile():
    assert bench.measured_traffic("csr_200000", "f32") is None

