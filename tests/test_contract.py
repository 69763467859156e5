"""CPU checks of the entry points' contracts: the benchmark refuses more than
one GPU with a message, and the binding fails loudly (no fallback) when the
HIP library is missing."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_binding_raises_without_library(monkeypatch):
    from paper_1705_01263_amd import qpt
    monkeypatch.setattr(qpt, "_lib", None)
    monkeypatch.setattr(qpt, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libqpt.so"))
    with pytest.raises(ImportError):
        qpt.lib()
    with pytest.raises(ImportError):
        qpt.Context(-1)
