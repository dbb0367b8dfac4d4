"""The product path has no CPU fallback: without libfd.so the binding
raises instead of computing anything."""
import importlib
import os

import pytest


def test_missing_library_raises(monkeypatch, tmp_path):
    from paper_2311_05038_amd import _abi
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "absent" / "libfd.so"))
    with pytest.raises(ImportError):
        _abi.lib()


def test_package_does_not_import_the_oracle():
    import sys
    import paper_2311_05038_amd  # noqa: F401
    import paper_2311_05038_amd.serve  # noqa: F401
    import paper_2311_05038_amd.autograd  # noqa: F401
    for name in ("paper_2311_05038_amd", "paper_2311_05038_amd.serve",
                 "paper_2311_05038_amd.autograd", "paper_2311_05038_amd._abi"):
        src = open(importlib.import_module(name).__file__).read()
        assert "oracle" not in src.replace("oracle-", ""), name


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus N > 1 exits with status 2 and says
    why, before any device work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
