"""Thin binding of the 2D C ABI (include/hhg2d.h) in libhhg.so: argument
marshalling only; every step runs in the library's HIP kernels."""
import ctypes

import numpy as np

from .hhg import load as _load_lib, HHGError, F64, F32, _ptr, _dtype_code, _stream

EXPORTS2D = ["hhg2d_create", "hhg2d_destroy", "hhg2d_last_error", "hhg2d_sizes", "hhg2d_node_coords",
             "hhg2d_set_coefficient", "hhg2d_from_canonical", "hhg2d_to_canonical", "hhg2d_apply_scaled",
             "hhg2d_apply_nodal"]
FLAG_NO_MODIFICATION = 1

_ready = False


def load():
    global _ready
    L = _load_lib()
    if not _ready:
        P, I32, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        sig = {
            "hhg2d_create": [P, I32, P, I32, I32, U32, ctypes.POINTER(P)],
            "hhg2d_destroy": [P],
            "hhg2d_sizes": [P, P, P, P, P],
            "hhg2d_node_coords": [P, P, P],
            "hhg2d_set_coefficient": [P, P],
            "hhg2d_from_canonical": [P, I32, P, P, P],
            "hhg2d_to_canonical": [P, I32, P, P, P],
            "hhg2d_apply_scaled": [P, I32, P, P, P],
            "hhg2d_apply_nodal": [P, I32, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = I32
        L.hhg2d_last_error.argtypes = [P]
        L.hhg2d_last_error.restype = ctypes.c_char_p
        _ready = True
    return L


class Context2D:
    """A triangular macro mesh refined `level` times on the current GPU."""

    def __init__(self, X, T, level, flags=0):
        L = load()
        X = np.ascontiguousarray(X, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.int32)
        self._h = ctypes.c_void_p()
        s = L.hhg2d_create(_ptr(X), X.shape[0], _ptr(T), T.shape[0], int(level), int(flags), ctypes.byref(self._h))
        if s < 0:
            raise HHGError(s, "hhg2d_create failed")
        self.level = int(level)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().hhg2d_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s):
        if s < 0:
            raise HHGError(s, load().hhg2d_last_error(self._h).decode())
        return s

    def sizes(self):
        v = [ctypes.c_int64() for _ in range(4)]
        self._check(load().hhg2d_sizes(self._h, *[ctypes.byref(x) for x in v]))
        return dict(n_slots=v[0].value, n_nodes=v[1].value, n_unknowns=v[2].value, n_modified=v[3].value)

    def node_coords(self):
        n = self.sizes()["n_nodes"]
        xy = np.empty((n, 2), dtype=np.float64)
        d = np.empty(n, dtype=np.uint8)
        self._check(load().hhg2d_node_coords(self._h, _ptr(xy), _ptr(d)))
        return xy, d.astype(bool)

    def set_coefficient(self, k):
        k = np.ascontiguousarray(k, dtype=np.float64)
        nn = self.sizes()["n_nodes"]
        if k.size != nn:
            raise HHGError(-1, f"coefficient has {k.size} values, expected {nn}")
        self._check(load().hhg2d_set_coefficient(self._h, _ptr(k)))

    def vector(self, dtype=None):
        import torch
        return torch.zeros(self.sizes()["n_slots"], dtype=dtype or torch.float64, device="cuda")

    def _vecs(self, *vecs, n="n_slots"):
        from .hhg import check_vectors
        return check_vectors(self.sizes(), self.level, vecs, n=n)

    def from_canonical(self, v):
        dt = self._vecs(v, n="n_nodes")
        out = self.vector(v.dtype)
        self._check(load().hhg2d_from_canonical(self._h, dt, _ptr(v), _ptr(out), _stream()))
        return out

    def to_canonical(self, v):
        import torch
        dt = self._vecs(v)
        out = torch.empty(self.sizes()["n_nodes"], dtype=v.dtype, device="cuda")
        self._check(load().hhg2d_to_canonical(self._h, dt, _ptr(v), _ptr(out), _stream()))
        return out

    def apply_scaled(self, u, y):
        dt = self._vecs(u, y)
        self._check(load().hhg2d_apply_scaled(self._h, dt, _ptr(u), _ptr(y), _stream()))
        return y

    def apply_nodal(self, u, y):
        dt = self._vecs(u, y)
        self._check(load().hhg2d_apply_nodal(self._h, dt, _ptr(u), _ptr(y), _stream()))
        return y
