"""Command-line and loading behaviour that needs no GPU.

- bench.py with more than one GPU exits with status 2 and a message instead of
  measuring.
- The binding refuses to run without the HIP library: with the library path
  pointed at a missing file, library() raises ImportError naming the build
  step (no host fallback exists).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_0711_0999_amd import fkdmft
    monkeypatch.setattr(fkdmft, "_lib", None)
    monkeypatch.setattr(fkdmft, "LIB_PATH", str(tmp_path / "libfkdmft.so"))
    with pytest.raises(ImportError, match="build"):
        fkdmft.library()
