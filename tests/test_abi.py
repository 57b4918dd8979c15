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


def _create_error(X, T, level=2):
    """The status hhg_create_macro returns for (X, T) on a host without a GPU:
    the mesh checks run before any device call, so a conforming mesh gets as
    far as the first device allocation and fails there."""
    import numpy as np
    try:
        hhg.Context(np.asarray(X, dtype=np.float64), np.asarray(T, dtype=np.int32), level)
    except hhg.HHGError as e:
        return e.code, str(e)
    return 0, ""


def test_create_rejects_non_conforming_macro_meshes():
    if not os.path.exists(hhg.LIB_PATH):
        pytest.skip("libhhg.so not built")
    if _gpu_present():
        pytest.skip("a GPU is present: conforming meshes would be created")
    from hhg_inputs import kuhn_cube, kuhn_cube_2x2x2, cube12, unit_tet, flat_tet, regular_tet
    for fn in (kuhn_cube, kuhn_cube_2x2x2, cube12, unit_tet, flat_tet, regular_tet):
        code, msg = _create_error(*fn())
        assert code != hhg.EMESH, (fn.__name__, msg)
    # a face whose two sides use different ids for one vertex (coincident vertices)
    X = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 0, 0], [0, 0, -1]]
    code, msg = _create_error(X, [[0, 1, 2, 3], [0, 2, 4, 5]])
    assert code == hhg.EMESH and "coincide" in msg, msg
    # a hanging vertex: the midpoint of one tet's edge is a vertex of the tets below
    X = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.5, 0.5, 0], [0, 0, -1]]
    code, msg = _create_error(X, [[0, 1, 2, 3], [0, 4, 1, 5], [0, 2, 4, 5]])
    assert code == hhg.EMESH and "lies on macro edge" in msg, msg
    # a vertex inside another tet's face
    X = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.25, 0.25, 0], [0, 0, -1]]
    code, msg = _create_error(X, [[0, 1, 2, 3], [0, 4, 1, 5], [1, 4, 2, 5], [2, 4, 0, 5]])
    assert code == hhg.EMESH and "lies on macro face" in msg, msg
    # a square split along one diagonal above and along the other below
    X = [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0.5, 0.5, 1], [0.5, 0.5, -1]]
    code, msg = _create_error(X, [[0, 1, 2, 4], [0, 2, 3, 4], [0, 3, 1, 5], [1, 3, 2, 5]])
    assert code == hhg.EMESH and "overlap" in msg, msg


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_binding_rejects_wrong_vectors_before_the_library():
    """Vector arguments are validated in the binding: a wrong size, dtype,
    layout or device never reaches a kernel."""
    import numpy as np
    torch = pytest.importorskip("torch")
    sizes = dict(n_slots=10, n_unknowns=3, n_nodes=8)
    ok64 = torch.zeros(10, dtype=torch.float64)
    assert hhg.check_vectors(sizes, 2, (ok64, ok64), require_cuda=False) == hhg.F64
    assert hhg.check_vectors(sizes, 2, (ok64.float(),), require_cuda=False) == hhg.F32
    bad = [
        ((ok64,), dict()),                                                    # host tensor
        ((torch.zeros(9, dtype=torch.float64),), dict(require_cuda=False)),   # short
        ((ok64, torch.zeros(10, dtype=torch.float32)), dict(require_cuda=False)),   # mixed dtypes
        ((torch.zeros(20, dtype=torch.float64)[::2],), dict(require_cuda=False)),   # strided
        ((torch.zeros(10, dtype=torch.int64),), dict(require_cuda=False)),    # integer
        ((np.zeros(10),), dict(require_cuda=False)),                          # not a tensor
        ((ok64,), dict(require_cuda=False, dtype=torch.float32)),             # wrong dtype for the call
        ((ok64,), dict(require_cuda=False, n="n_nodes")),                     # slots where nodes are expected
    ]
    for vecs, kw in bad:
        with pytest.raises(hhg.HHGError) as e:
            hhg.check_vectors(sizes, 2, vecs, **kw)
        assert e.value.code == hhg.EINVAL
    # the methods validate before calling the library: a context whose
    # library handle is NULL would fail loudly in the library otherwise
    ctx = hhg.Context.__new__(hhg.Context)
    ctx._sizes = {3: dict(sizes)}
    ctx.max_level = 3
    for call in (lambda: ctx.apply_scaled(3, ok64, ok64), lambda: ctx.apply_nodal(3, ok64, ok64[:9]),
                 lambda: ctx.residual(3, ok64, ok64, ok64), lambda: ctx.smooth(3, ok64, ok64, 1),
                 lambda: ctx.learned_forward(3, ok64, ok64), lambda: ctx.set_coefficient(np.ones(7)),
                 lambda: ctx.set_coefficient(torch.ones(8, dtype=torch.float32))):
        with pytest.raises(hhg.HHGError) as e:
            call()
        assert e.value.code == hhg.EINVAL
