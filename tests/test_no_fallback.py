"""The product path has no CPU fallback: without libfd.so the binding
raises instead of computing anything."""
import importlib

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
