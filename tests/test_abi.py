"""The C ABI boundary on the CPU: the library loads, exports every function that
include/cc.h declares, the binding covers exactly those, and the product path has
no route to the oracle and no CPU fallback."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cc.h")
PKG = os.path.join(ROOT, "paper_2507_03695_amd")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(cc_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def _lib_path():
    import paper_2507_03695_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_2507_03695_amd import _build
        _build.build()
    return pkg.LIB_PATH


def test_header_parses():
    names = header_functions()
    for must in ["cc_solve", "cc_solve_async", "cc_batch", "cc_serve_open", "cc_serve_submit",
                 "cc_serve_wait", "cc_serve_close", "cc_init", "cc_hook", "cc_compress",
                 "cc_canon", "cc_zroot", "cc_push"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_race_testing_build_exports_the_same_symbols():
    """libccmi_stress.so (the sources built with CCM_STRESS_DELAYS, loaded by the
    delay-injection GPU test through CCMI_LIBRARY) is the same ABI."""
    from paper_2507_03695_amd import _build
    if not os.path.exists(_build.STRESS_LIB):
        _build.build(stress=True)
    lib = ctypes.CDLL(_build.STRESS_LIB)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_the_header():
    import paper_2507_03695_amd as pkg
    assert sorted(pkg.SIGNATURES) == header_functions()


def test_status_strings_without_gpu():
    import paper_2507_03695_amd as pkg
    lib = pkg.load()
    assert lib.cc_strerror(-2).startswith(b"CC_ERANGE")
    assert lib.cc_version() >= 100


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2507_03695_amd as pkg
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(pkg, "_lib", None)
    with pytest.raises(ImportError):
        pkg.load()


def test_product_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", text), f"{f} mentions the oracle"
                assert "import graphgen" not in text


def test_oracle_never_touches_the_product():
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2507_03695_amd" not in text and "cc.h" not in text


def test_id_bytes_without_gpu():
    """cc_id_bytes is host arithmetic: it agrees with the oracle's width rule."""
    import oracle
    import paper_2507_03695_amd as pkg
    lib = pkg.load()
    for n in [0, 1, 2, 255, 256, 257, 65535, 65536, 65537, (1 << 24) - 1, 1 << 24, (1 << 24) + 1,
              68109812, 1 << 30, (1 << 32) - 1, 1 << 32]:
        assert lib.cc_id_bytes(n) == oracle.id_bytes(n), n


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why, before
    touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_traffic_is_keyed_to_the_hook_sources():
    """The HBM traffic figure is reported only for the sources it was measured on."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    t = bench.TRAFFIC[("rmat26", "zroot")]
    assert bench.measured_traffic("rmat26", "zroot") in (None, t["bytes"])
    assert bench.measured_traffic("rmat22", "zroot") is None
