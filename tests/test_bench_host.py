"""Host-side logic of bench.py (no GPU): algorithmic flop counts, the source
hash that ties a committed HBM-traffic record to the kernels it measured, and
the refusal of multi-GPU runs."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("K,f0,f2", [(16, 6.3e3, 3.5e4), (24, 1.69e4, 1.02e5), (32, 3.52e4, 2.25e5),
                                     (48, 1.03e5, 7.0e5)])
def test_flop_counts(K, f0, f2):
    # LAPACK convention: Cholesky n^3/3 FMAs, 2 n^2 per right-hand side solve,
    # 20 flops per scalar covariance entry, 60 per spin-2 block
    assert bench.flops_spin0(K) == pytest.approx(f0, rel=0.01)
    assert bench.flops_spin2(K) == pytest.approx(f2, rel=0.01)


def _tree(tmp_path):
    dst = tmp_path / "paper_1003_4984_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_1003_4984_amd", "csrc"), dst,
                    ignore=shutil.ignore_patterns("_obj_*"))
    return dst


def test_source_hash_ignores_comments_and_unmeasured_sources(tmp_path, monkeypatch):
    csrc = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    dev = csrc / "device.h"
    text = dev.read_text()
    dev.write_text("// a comment\n/* a block\n comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash() == h0
    for name in bench.NOT_MEASURED:
        f = csrc / name
        f.write_text(f.read_text() + "\nint unmeasured_change;\n")
    assert bench.kernel_source_hash() == h0
    dev.write_text(text + "\nint measured_change;\n")
    assert bench.kernel_source_hash() != h0


def test_traffic_record_requires_matching_sources(tmp_path, monkeypatch):
    _tree(tmp_path)
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = prof / "traffic_interp_tqu_nside4096_K32.md"
    monkeypatch.setitem(bench.TRAFFIC_FILES, "shared", str(rec))
    rec.write_text(f"traffic_bytes_per_launch: 1.5e11\nsource_sha256: {bench.kernel_source_hash()}\n")
    assert bench.measured_traffic("nside4096", "shared") == 1.5e11
    assert bench.measured_traffic("nside512", "shared") is None
    rec.write_text("traffic_bytes_per_launch: 1.5e11\nsource_sha256: 0000\n")
    assert bench.measured_traffic("nside4096", "shared") is None


def test_multi_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
