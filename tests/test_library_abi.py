"""The C-ABI library loads and exports every symbol include/twk.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(twk_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = _declared("twk.h")
    for must in ("twk_create", "twk_point_mag", "twk_finite_mag", "twk_lightcurves"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2501_03322_amd import twk
    if not os.path.exists(twk.LIB_PATH):
        pytest.skip("libtwk.so not built")
    lib = ctypes.CDLL(twk.LIB_PATH)
    for name in _declared("twk.h"):
        assert hasattr(lib, name), name
    assert set(twk.EXPORTS) <= set(_declared("twk.h"))


def test_cpu_backend_exports_every_declared_symbol():
    from paper_2501_03322_amd import build, cpu
    if not os.path.exists(cpu.LIB_PATH):
        build.build_cpu()
    lib = ctypes.CDLL(cpu.LIB_PATH)
    names = _declared("twk_cpu.h")
    assert names == ["twk_cpu_finite_mag", "twk_cpu_lightcurves"]
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_without_gpu():
    from paper_2501_03322_amd import twk
    if not os.path.exists(twk.LIB_PATH):
        pytest.skip("libtwk.so not built")
    assert twk.strerror(0) == "ok"
    assert "invalid" in twk.strerror(-1)


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    from paper_2501_03322_amd import twk
    monkeypatch.setattr(twk, "_lib", None)
    monkeypatch.setattr(twk, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        twk.load()


def test_device_code_digest_covers_device_code_only():
    """The committed HBM-traffic record is keyed on the device code: the
    digest reads the .hip_fatbin section, which is present, non-trivial and
    differs from the digest of the whole file."""
    import bench
    from paper_2501_03322_amd import twk
    if not os.path.exists(twk.LIB_PATH):
        pytest.skip("library not built")
    d = bench.device_code_digest(twk.LIB_PATH)
    assert re.fullmatch(r"[0-9a-f]{64}", d)
    assert d != bench.lib_digest(twk.LIB_PATH)
    assert d == bench.device_code_digest(twk.LIB_PATH)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and a
    message, before any GPU work."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus must be 1" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
