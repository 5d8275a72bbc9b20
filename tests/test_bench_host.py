"""Host logic of bench.py that needs no GPU: the kernel-source fingerprint that
decides whether the recorded HBM counter measurements still describe the
kernels, and the refusal of more than one GPU."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SOURCES = ("nem_passes.hip", "nem_pair.h", "nem_dev.h")


def _copy_sources(tmp_path):
    d = tmp_path / "paper_2108_08919_amd" / "csrc"
    d.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2108_08919_amd", "csrc", f), d / f)
    return d


def test_recorded_fingerprint_matches_sources():
    assert bench.kernel_fingerprint() == bench.MEASURED_TRAFFIC["fingerprint"]


def test_fingerprint_ignores_comments_not_code(tmp_path, monkeypatch):
    d = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_fingerprint()
    p = d / "nem_pair.h"
    src = p.read_text()
    p.write_text("// a new comment line\n\n" + src.replace("\n", "   // trailing note\n", 1) + "/* block\ncomment */\n")
    assert bench.kernel_fingerprint() == base
    p.write_text(src.replace("0xFFFu", "0x7FFu", 1) if "0xFFFu" in src else src + "int changed_code;\n")
    assert bench.kernel_fingerprint() != base


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
