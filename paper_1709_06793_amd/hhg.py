"""Python binding of libhhg (include/hhg.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy /
torch arguments to pointers and sizes, passes the current torch stream, and
turns error codes into exceptions.  PyTorch provides device memory and streams.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhhg.so")

F64, F32 = 0, 1
JACOBI, CHEBYSHEV, LEARNED = 0, 1, 2
SOLVE_F64, SOLVE_MIXED, SOLVE_LEARNED = 0, 1, 2
FLAG_NO_MODIFICATION = 1
FLAG_COARSE_K_GEOMETRIC = 2
# macro primitives whose rows use nodal integration in apply_mixed (Sec. 5)
PRIM_VERTICES, PRIM_EDGES, PRIM_FACES = 1, 2, 4
LEARNED_NPARAM = 817
WFALLBACK = 1
# error codes of include/hhg.h
EINVAL, EMESH, ECOEF, EHIP, ESTATE, ENOMEM = -1, -2, -3, -4, -5, -6

# every symbol include/hhg.h declares
EXPORTS = [
    "hhg_create_macro", "hhg_destroy", "hhg_last_error", "hhg_vector_size", "hhg_node_coords",
    "hhg_to_canonical", "hhg_from_canonical", "hhg_set_coefficient", "hhg_set_coarse_level",
    "hhg_level_info", "hhg_apply_scaled", "hhg_residual_noalloc", "hhg_set_graphs", "hhg_set_timing", "hhg_read_timing", "hhg_set_kernel_variant", "hhg_apply_nodal", "hhg_apply_mixed", "hhg_store_stencils", "hhg_apply_stored", "hhg_set_tensor_coefficient", "hhg_apply_tensor", "hhg_apply_tensor_nodal", "hhg_residual", "hhg_smooth",
    "hhg_vcycle", "hhg_solve", "hhg_solve_tensor", "hhg_solve_form", "hhg_learned_set_weights", "hhg_learned_set_fallback",
    "hhg_learned_forward", "hhg_learned_backward", "hhg_learned_loss_grad", "hhg_training_pair",
    "hhg_adam_update",
]


class HHGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hhg error {code}: {msg}")
        self.code = code


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("rho", ctypes.c_double),
                ("seconds", ctypes.c_double)]


_lib = None


def load():
    """Load the in-tree libhhg.so; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1709_06793_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    sig = {
        "hhg_create_macro": [P, I32, P, I32, I32, U32, P, ctypes.POINTER(P)],
        "hhg_destroy": [P],
        "hhg_vector_size": [P, I32, P, P, P],
        "hhg_node_coords": [P, I32, P, P],
        "hhg_to_canonical": [P, I32, I32, P, P, P],
        "hhg_from_canonical": [P, I32, I32, P, P, P],
        "hhg_set_coefficient": [P, P, ctypes.c_int, P],
        "hhg_set_coarse_level": [P, I32],
        "hhg_level_info": [P, I32, P, P, P],
        "hhg_apply_scaled": [P, I32, I32, P, P, P],
        "hhg_set_timing": [P, I32],
        "hhg_set_graphs": [P, I32],
        "hhg_set_kernel_variant": [I32],
        "hhg_read_timing": [P, P, P],
        "hhg_apply_nodal": [P, I32, I32, P, P, P],
        "hhg_apply_mixed": [P, I32, I32, I32, P, P, P],
        "hhg_store_stencils": [P, I32],
        "hhg_set_tensor_coefficient": [P, P, ctypes.c_int, P],
        "hhg_apply_tensor": [P, I32, I32, P, P, P],
        "hhg_apply_tensor_nodal": [P, I32, I32, P, P, P],
        "hhg_apply_stored": [P, I32, I32, P, P, P],
        "hhg_residual": [P, I32, I32, P, P, P, P, P],
        "hhg_residual_noalloc": [P, I32, I32, P, P, P, P, P],
        "hhg_smooth": [P, I32, I32, I32, I32, D, P, P, P],
        "hhg_vcycle": [P, I32, I32, I32, I32, I32, P, P, P, P],
        "hhg_solve": [P, I32, I32, I32, I32, D, I32, P, P, P, P],
        "hhg_solve_tensor": [P, I32, I32, I32, I32, I32, D, I32, P, P, P, P],
        "hhg_solve_form": [P, I32, I32, I32, I32, I32, I32, D, I32, P, P, P, P],
        "hhg_learned_set_weights": [P, P, I64],
        "hhg_learned_set_fallback": [P, D, D],
        "hhg_learned_forward": [P, I32, P, P, P],
        "hhg_learned_backward": [P, I32, P, P, P, P],
        "hhg_learned_loss_grad": [P, I32, P, P, P, P, P],
        "hhg_training_pair": [P, I32, P, P, P, P, P, P],
        "hhg_adam_update": [P, P, P, P, I64, I32, D, D, D, D],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = I32
    L.hhg_last_error.argtypes = [P]
    L.hhg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(x):
    """Device/host pointer of a torch tensor or numpy array (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(x.data_ptr())


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("vectors must be float64 or float32 torch tensors")


def check_vectors(sizes, level, vecs, n="n_slots", dtype=None, require_cuda=True):
    """Validate vector arguments before any pointer reaches the library: torch
    tensors, on the GPU, contiguous, one dtype (float64 or float32, or the one
    given), and exactly sizes(level)[n] elements each.  Returns the dtype
    code.  Raises HHGError(EINVAL) otherwise: a wrong-sized or wrong-typed
    buffer would make the kernels read or write out of bounds."""
    import torch
    want = sizes[n]
    dt = None
    for v in vecs:
        if not isinstance(v, torch.Tensor):
            raise HHGError(EINVAL, f"level {level}: vectors must be torch tensors, got {type(v).__name__}")
        if require_cuda and not v.is_cuda:
            raise HHGError(EINVAL, f"level {level}: vectors must live on the GPU")
        if not v.is_contiguous():
            raise HHGError(EINVAL, f"level {level}: vectors must be contiguous")
        if v.numel() != want:
            raise HHGError(EINVAL, f"level {level}: vector has {v.numel()} elements, expected {want} ({n})")
        if v.dtype not in (torch.float64, torch.float32):
            raise HHGError(EINVAL, f"level {level}: vectors must be float64 or float32, got {v.dtype}")
        if dt is None:
            dt = v.dtype
        elif v.dtype != dt:
            raise HHGError(EINVAL, f"level {level}: mixed dtypes {dt} and {v.dtype}")
    if dtype is not None and dt != dtype:
        raise HHGError(EINVAL, f"level {level}: vectors must be {dtype}, got {dt}")
    return F64 if dt == torch.float64 else F32


def _stream():
    """Handle of torch's current stream on the current device (the raw
    accessors avoid building a Stream object on every call)."""
    import torch
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    dev = getattr(torch._C, "_cuda_getDevice", None)
    if raw is not None and dev is not None:
        return ctypes.c_void_p(raw(dev()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One macro mesh with its refinement hierarchy on the current GPU."""

    def __init__(self, X, T, max_level, flags=0):
        L = load()
        X = np.ascontiguousarray(X, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.int32)
        self._h = ctypes.c_void_p()
        s = L.hhg_create_macro(_ptr(X), X.shape[0], _ptr(T), T.shape[0], int(max_level), int(flags),
                               None, ctypes.byref(self._h))
        if s < 0:
            raise HHGError(s, L.hhg_last_error(None).decode())
        self.max_level = int(max_level)
        self.X, self.T = X, T

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().hhg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s):
        if s < 0:
            raise HHGError(s, load().hhg_last_error(self._h).decode())
        return s

    # ---- sizes and layout
    def _size_table(self, level):
        cache = self.__dict__.setdefault("_sizes", {})
        if level not in cache:
            a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            self._check(load().hhg_vector_size(self._h, level, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
            cache[level] = dict(n_slots=a.value, n_unknowns=b.value, n_nodes=c.value)
        return cache[level]

    def sizes(self, level):
        return dict(self._size_table(level))

    def _vecs(self, level, *vecs, n="n_slots", dtype=None):
        return check_vectors(self._size_table(level), level, vecs, n=n, dtype=dtype)

    def _f32(self):
        import torch
        return torch.float32

    def _f64(self):
        import torch
        return torch.float64

    def node_coords(self, level):
        n = self.sizes(level)["n_nodes"]
        xyz = np.empty((n, 3))
        d = np.empty(n, dtype=np.uint8)
        self._check(load().hhg_node_coords(self._h, level, _ptr(xyz), _ptr(d)))
        return xyz, d.astype(bool)

    def vector(self, level, dtype=None, fill=0.0):
        import torch
        dtype = dtype or torch.float64
        return torch.full((self.sizes(level)["n_slots"],), fill, dtype=dtype, device="cuda")

    def to_canonical(self, level, v):
        import torch
        dt = self._vecs(level, v)
        out = torch.empty(self.sizes(level)["n_nodes"], dtype=v.dtype, device=v.device)
        self._check(load().hhg_to_canonical(self._h, level, dt, _ptr(v), _ptr(out), _stream()))
        return out

    def from_canonical(self, level, v):
        import torch
        dt = self._vecs(level, v, n="n_nodes")
        out = torch.zeros(self.sizes(level)["n_slots"], dtype=v.dtype, device=v.device)
        self._check(load().hhg_from_canonical(self._h, level, dt, _ptr(v), _ptr(out), _stream()))
        return out

    # ---- coefficient and solver data
    def set_coefficient(self, k):
        """Finest-level nodal k, canonical order (numpy float64 or a torch tensor)."""
        nn = self.sizes(self.max_level)["n_nodes"]
        if isinstance(k, np.ndarray):
            k = np.ascontiguousarray(k, dtype=np.float64)
            if k.size != nn:
                raise HHGError(EINVAL, f"coefficient has {k.size} values, expected {nn}")
            self._check(load().hhg_set_coefficient(self._h, _ptr(k), 0, _stream()))
        else:
            check_vectors(self.sizes(self.max_level), self.max_level, (k,), n="n_nodes",
                          dtype=self._f64(), require_cuda=False)
            self._check(load().hhg_set_coefficient(self._h, _ptr(k), 1 if k.is_cuda else 0, _stream()))

    def set_coarse_level(self, level):
        self._check(load().hhg_set_coarse_level(self._h, level))

    def level_info(self, level):
        lam, nm, cl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int32()
        self._check(load().hhg_level_info(self._h, level, ctypes.byref(lam), ctypes.byref(nm), ctypes.byref(cl)))
        return dict(lambda_max=lam.value, n_modified=nm.value, coarse_level=cl.value)

    # ---- operators
    def apply_scaled(self, level, u, y):
        dt = self._vecs(level, u, y)
        self._check(load().hhg_apply_scaled(self._h, level, dt, _ptr(u), _ptr(y), _stream()))
        return y

    def set_timing(self, enable):
        self._check(load().hhg_set_timing(self._h, 1 if enable else 0))

    def read_timing(self):
        """(summed ms of the timed applies' stencil kernels, number of applies)"""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(load().hhg_read_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def apply_mixed(self, level, u, y, nodal_primitives=PRIM_VERTICES | PRIM_EDGES):
        dt = self._vecs(level, u, y)
        self._check(load().hhg_apply_mixed(self._h, level, dt, int(nodal_primitives), _ptr(u), _ptr(y),
                                           _stream()))
        return y

    def set_tensor_coefficient(self, k6):
        """k6: (6, n_nodes) component fields at the finest level (numpy or a
        contiguous float64 device tensor), canonical node order."""
        nn = self.sizes(self.max_level)["n_nodes"]
        if tuple(k6.shape) != (6, nn):
            raise HHGError(EINVAL, f"tensor coefficient has shape {tuple(k6.shape)}, expected (6, {nn})")
        if isinstance(k6, np.ndarray):
            a = np.ascontiguousarray(k6, dtype=np.float64)
            self._check(load().hhg_set_tensor_coefficient(self._h, _ptr(a), 0, _stream()))
        else:
            t = k6.contiguous()
            if t.dtype != self._f64():
                raise HHGError(EINVAL, f"tensor coefficient must be float64, got {t.dtype}")
            self._check(load().hhg_set_tensor_coefficient(self._h, _ptr(t), 1 if t.is_cuda else 0, _stream()))

    def apply_tensor(self, level, u, y):
        dt = self._vecs(level, u, y)
        self._check(load().hhg_apply_tensor(self._h, level, dt, _ptr(u), _ptr(y), _stream()))
        return y

    def apply_tensor_nodal(self, level, u, y):
        dt = self._vecs(level, u, y)
        self._check(load().hhg_apply_tensor_nodal(self._h, level, dt, _ptr(u), _ptr(y), _stream()))
        return y

    def store_stencils(self, level):
        self._check(load().hhg_store_stencils(self._h, level))

    def apply_stored(self, level, u, y):
        dt = self._vecs(level, u, y)
        self._check(load().hhg_apply_stored(self._h, level, dt, _ptr(u), _ptr(y), _stream()))
        return y

    def apply_nodal(self, level, u, y):
        dt = self._vecs(level, u, y)
        self._check(load().hhg_apply_nodal(self._h, level, dt, _ptr(u), _ptr(y), _stream()))
        return y

    def residual(self, level, f, u, r, norm=False):
        nv = ctypes.c_double()
        dt = self._vecs(level, f, u, r)
        self._check(load().hhg_residual(self._h, level, dt, _ptr(f), _ptr(u), _ptr(r),
                                        ctypes.byref(nv) if norm else None, _stream()))
        return nv.value if norm else r

    def residual_noalloc(self, level, f, u, r, norm=False):
        """hhg_residual_noalloc: hhg_residual without any device allocation
        (the norm's scratch is the library's static per-GPU array)."""
        nv = ctypes.c_double()
        dt = self._vecs(level, f, u, r)
        self._check(load().hhg_residual_noalloc(self._h, level, dt, _ptr(f), _ptr(u), _ptr(r),
                                                ctypes.byref(nv) if norm else None, _stream()))
        return nv.value if norm else r

    def smooth(self, level, f, u, sweeps, smoother=JACOBI, omega=2.0 / 3.0):
        dt = self._vecs(level, f, u)
        self._check(load().hhg_smooth(self._h, level, dt, smoother, sweeps, omega,
                                      _ptr(f), _ptr(u), _stream()))
        return u

    def vcycle(self, level, f, u, pre=2, post=2, smoother=CHEBYSHEV, rel_res=False):
        rr = ctypes.c_double()
        dt = self._vecs(level, f, u)
        self._check(load().hhg_vcycle(self._h, level, dt, pre, post, smoother, _ptr(f),
                                      _ptr(u), ctypes.byref(rr) if rel_res else None, _stream()))
        return rr.value if rel_res else u

    def set_graphs(self, enable):
        """hhg_set_graphs: solve-loop V-cycles as captured HIP graphs, or eager (default)."""
        self._check(load().hhg_set_graphs(self._h, int(bool(enable))))

    def solve(self, level, f, u, mode=SOLVE_F64, tol=1e-8, max_iter=100, pre=2, post=2):
        self._vecs(level, f, u, dtype=self._f64())
        st = SolveStats()
        s = self._check(load().hhg_solve(self._h, level, mode, pre, post, tol, max_iter, _ptr(f), _ptr(u),
                                         ctypes.byref(st), _stream()))
        return dict(iterations=st.iterations, fallback=st.fallback, rel_residual=st.rel_residual,
                    rho=st.rho, seconds=st.seconds, status=s)

    def solve_tensor(self, level, f, u, form="scaled", mode=SOLVE_F64, tol=1e-8, max_iter=100, pre=2, post=2):
        """hhg_solve_tensor: the tensor operator with every component scaled
        (form "scaled") or nodally integrated (form "nodal")."""
        fc = {"scaled": 0, "nodal": 1}[form]
        self._vecs(level, f, u, dtype=self._f64())
        st = SolveStats()
        s = self._check(load().hhg_solve_tensor(self._h, level, fc, mode, pre, post, tol, max_iter, _ptr(f), _ptr(u),
                                                ctypes.byref(st), _stream()))
        return dict(iterations=st.iterations, fallback=st.fallback, rel_residual=st.rel_residual,
                    rho=st.rho, seconds=st.seconds, status=s)

    def solve_form(self, level, f, u, form="nodal", nodal_primitives=0, mode=SOLVE_F64, tol=1e-8, max_iter=100,
                   pre=2, post=2):
        """hhg_solve_form: the scalar problem on the scaled ("scaled"), nodal
        ("nodal") or primitive-mixed ("mixed", nodal rows on
        nodal_primitives) operator."""
        fc = {"scaled": 0, "nodal": 1, "mixed": 2}[form]
        self._vecs(level, f, u, dtype=self._f64())
        st = SolveStats()
        s = self._check(load().hhg_solve_form(self._h, level, fc, nodal_primitives, mode, pre, post, tol, max_iter,
                                              _ptr(f), _ptr(u), ctypes.byref(st), _stream()))
        return dict(iterations=st.iterations, fallback=st.fallback, rel_residual=st.rel_residual,
                    rho=st.rho, seconds=st.seconds, status=s)

    # ---- learned correction
    def learned_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != LEARNED_NPARAM:
            raise HHGError(EINVAL, f"{w.size} parameters, expected {LEARNED_NPARAM}")
        self._check(load().hhg_learned_set_weights(self._h, _ptr(w), w.size))

    def learned_forward(self, level, r, c_out):
        self._vecs(level, r, c_out, dtype=self._f32())
        self._check(load().hhg_learned_forward(self._h, level, _ptr(r), _ptr(c_out), _stream()))
        return c_out

    def learned_backward(self, level, r, g):
        self._vecs(level, r, g, dtype=self._f32())
        dw = np.zeros(LEARNED_NPARAM, dtype=np.float32)
        self._check(load().hhg_learned_backward(self._h, level, _ptr(r), _ptr(g), _ptr(dw), _stream()))
        return dw

    def learned_set_fallback(self, max_rate=1.0, plain_margin=1.05):
        """Reject a learned cycle whose residual ratio exceeds max_rate or
        plain_margin x the plain cycle's ratio (0 turns that test off)."""
        self._check(load().hhg_learned_set_fallback(self._h, float(max_rate), float(plain_margin)))

    def learned_loss_grad(self, level, r, e):
        self._vecs(level, r, e, dtype=self._f32())
        dw = np.zeros(LEARNED_NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(load().hhg_learned_loss_grad(self._h, level, _ptr(r), _ptr(e), ctypes.byref(loss),
                                                 _ptr(dw), _stream()))
        return loss.value, dw

    def training_pair(self, level, f, u, u_star, r_out, e_out):
        self._vecs(level, f, u, u_star, dtype=self._f64())
        self._vecs(level, r_out, e_out, dtype=self._f32())
        self._check(load().hhg_training_pair(self._h, level, _ptr(f), _ptr(u), _ptr(u_star), _ptr(r_out),
                                             _ptr(e_out), _stream()))


def set_kernel_variant(variant):
    """Interior-kernel variant for the whole process (0 = default policy)."""
    s = load().hhg_set_kernel_variant(int(variant))
    if s < 0:
        raise HHGError(s, "kernel variant out of range")


def adam_update(w, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam step in the library (host) on numpy float32 arrays, in place."""
    s = load().hhg_adam_update(_ptr(w), _ptr(m), _ptr(v), _ptr(g), w.size, int(t), lr, beta1, beta2, eps)
    if s < 0:
        raise HHGError(s, "adam update failed")
