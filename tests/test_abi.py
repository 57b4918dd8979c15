"""CPU-side checks of the boundary: the HIP library builds/loads and exports
every symbol the public header declares; the binding lists exactly those."""
import os
import re
import subprocess

import pytest

from paper_1709_06793_amd import hhg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "hhg.h")).read()
    return sorted(set(re.findall(r"^\S.*?\b(hhg_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def _header2d_symbols():
    src = open(os.path.join(ROOT, "include", "hhg2d.h")).read()
    return sorted(set(re.findall(r"^\S.*?\b(hhg2d_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_and_binding_agree():
    assert _header_symbols() == sorted(hhg.EXPORTS)
    from paper_1709_06793_amd import hhg2d
    assert _header2d_symbols() == sorted(hhg2d.EXPORTS2D)


def test_library_exports_every_2d_symbol_and_checks_arguments():
    if not os.path.exists(hhg.LIB_PATH):
        pytest.skip("libhhg.so not built")
    import ctypes
    import numpy as np
    from paper_1709_06793_amd import hhg2d
    out = subprocess.run(["nm", "-D", "--defined-only", hhg.LIB_PATH], capture_output=True, text=True).stdout
    names = {l.split()[-1] for l in out.splitlines() if l.strip()}
    assert not [s for s in _header2d_symbols() if s not in names]
    L = hhg2d.load()
    h = ctypes.c_void_p()
    X = np.zeros((3, 2))
    T = np.array([[0, 1, 5]], dtype=np.int32)
    # bad vertex id and bad level: rejected before any device call
    assert L.hhg2d_create(X.ctypes.data_as(ctypes.c_void_p), 3, T.ctypes.data_as(ctypes.c_void_p), 1, 2, 0,
                          ctypes.byref(h)) == hhg.EMESH and not h.value
    T = np.array([[0, 1, 2]], dtype=np.int32)
    assert L.hhg2d_create(X.ctypes.data_as(ctypes.c_void_p), 3, T.ctypes.data_as(ctypes.c_void_p), 1, 14, 0,
                          ctypes.byref(h)) == hhg.EINVAL and not h.value


def test_library_exports_every_declared_symbol():
    if not os.path.exists(hhg.LIB_PATH):
        pytest.skip("libhhg.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", hhg.LIB_PATH], capture_output=True, text=True).stdout
    names = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [s for s in _header_symbols() if s not in names]
    assert not missing, missing
    L = hhg.load()
    for s in _header_symbols():
        assert hasattr(L, s)


def test_create_rejects_bad_arguments_without_gpu_work():
    """Argument checks run before any device call."""
    if not os.path.exists(hhg.LIB_PATH):
        pytest.skip("libhhg.so not built")
    import numpy as np
    X = np.zeros((4, 3))
    T = np.array([[0, 1, 2, 7]], dtype=np.int32)   # vertex id out of range
    with pytest.raises(hhg.HHGError) as e:
        hhg.Context(X, T, 2)
    assert e.value.code == -1
    with pytest.raises(hhg.HHGError):
        hhg.Context(X, np.array([[0, 1, 2, 3]], dtype=np.int32), 11)   # level out of range


def test_product_and_oracle_are_separate():
    """The product package never imports or names the oracle, the oracle never
    imports the product, and the input generators hold no method code from
    either side."""
    import glob
    prod = glob.glob(os.path.join(ROOT, "paper_1709_06793_amd", "*.py")) + \
        glob.glob(os.path.join(ROOT, "paper_1709_06793_amd", "csrc", "*"))
    for p in prod:
        src = open(p, errors="replace").read()
        assert not re.search(r"\boracle\b", src), p
    for p in glob.glob(os.path.join(ROOT, "oracle", "*.py")) + glob.glob(os.path.join(ROOT, "oracle", "*.c")):
        src = open(p).read()
        assert "paper_1709_06793_amd" not in src and "libhhg" not in src, p
    for p in glob.glob(os.path.join(ROOT, "hhg_inputs", "*.py")):
        src = open(p).read()
        assert "paper_1709_06793_amd" not in src and "from oracle" not in src and "import oracle" not in src, p


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stdout
