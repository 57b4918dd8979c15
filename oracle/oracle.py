"""CPU oracle for the stencil-scaling P1 Darcy operator on hierarchical hybrid grids.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of bench.py may import this module; the product library never does, and
the two share no code, header, table or helper.  Everything is float64.

Route: the refined mesh comes from oracle_topo.c (recursive Bey refinement,
exact integer node numbering).  Here, plain numpy/scipy assembles GLOBAL CSR
matrices by loops over the refined elements and then does SpMV, Jacobi,
Chebyshev and multigrid on them.  Nothing here uses lattice directions,
reference stencils or any structure of the GPU path.

Paper passages followed (arXiv 1709.06793):
* element matrices  A_t[a,b] = int_t grad phi_a . grad phi_b            (Sec. 3.2)
* scaled form       eq. (discrete), assembled through Lemma 3.2 eq. (equal):
                    off-diagonal factor (k_a+k_b)/2, diagonal by eq. (zerosum)
* brute-force form  eq. (discrete) summed directly over node pairs       (Sec. 2.1)
* nodal form        eq. (standardfe): mean vertex k times A_t            (Sec. 3.2)
* modification      Sec. 4.1 (MA2 and k_mod), read for 3D as listed in
                    modification_factors()
* primitive mix     Sec. 5 eq. (modst): nodal-integration rows on the nodes
                    of the chosen macro primitives, scaled rows elsewhere
* tensor K          Sec. 2.1 eq. (integral): a = sum_m a_m, a_m with its own
                    coefficient k_m and D_m = c_m.grad; each a_m scaled as the
                    scalar form (or nodal integration)
* rates             Lemma 3.1 (O(h^2) in L2, O(h) in H1)
"""
import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_topo.c")
_LIB = os.path.join(_HERE, "liboracle_topo.so")
_CSR_SRC = os.path.join(_HERE, "oracle_csr.c")
_CSR_LIB = os.path.join(_HERE, "liboracle_csr.so")


def build(force=False):
    """Compile oracle_topo.c and oracle_csr.c (OpenMP) with gcc into in-tree
    shared libraries."""
    for src, lib, extra in ((_SRC, _LIB, []), (_CSR_SRC, _CSR_LIB, ["-fopenmp"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            tmp = lib + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared"] + extra + [src, "-o", tmp])
            os.replace(tmp, lib)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.om_create.restype = P
        L.om_create.argtypes = [P, I32, P, I32, I32]
        L.om_destroy.argtypes = [P]
        L.om_n_nodes.restype = I64
        L.om_n_nodes.argtypes = [P]
        L.om_node_info.argtypes = [P, P, P]
        L.om_n_elements.restype = I64
        L.om_n_elements.argtypes = [P]
        L.om_elements.restype = I64
        L.om_elements.argtypes = [P, P, P]
        L.om_elements_bary.restype = I64
        L.om_elements_bary.argtypes = [P, P, P, P]
        L.om_incident.restype = I64
        L.om_incident.argtypes = [P, I64, P, P, I64]
        L.om_coarse_to_fine.argtypes = [P, P, P]
        L.om_prolongation.restype = I64
        L.om_prolongation.argtypes = [P, P, P, P, P]
        L.om_valence.restype = I32
        L.om_valence.argtypes = [P, P, I32]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Mesh:
    """Uniformly refined macro mesh at one level, with canonical node numbering."""

    def __init__(self, X, T, level):
        L = _load()
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.T = np.ascontiguousarray(T, dtype=np.int32)
        self.level = int(level)
        self.h = 2.0 ** (-self.level)
        self._h = L.om_create(_p(self.X), self.X.shape[0], _p(self.T), self.T.shape[0], self.level)
        if not self._h:
            raise ValueError("oracle: invalid macro mesh")
        self.n_nodes = int(L.om_n_nodes(self._h))
        self.xyz = np.empty((self.n_nodes, 3))
        dir_u8 = np.empty(self.n_nodes, dtype=np.uint8)
        L.om_node_info(self._h, _p(self.xyz), _p(dir_u8))
        self.dirichlet = dir_u8.astype(bool)
        self.unknowns = np.flatnonzero(~self.dirichlet)
        self._elements = None

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.om_destroy(self._h)
            self._h = None

    @property
    def n_elements(self):
        return int(_load().om_n_elements(self._h))

    def elements(self):
        """(conn int64 (ne,4) canonical vertex ids, macro int64 (ne,))."""
        if self._elements is None:
            ne = self.n_elements
            conn = np.empty((ne, 4), dtype=np.int32)
            macro = np.empty(ne, dtype=np.int32)
            _load().om_elements(self._h, _p(conn), _p(macro))
            self._elements = (conn.astype(np.int64), macro.astype(np.int64))
        return self._elements

    def incident(self, node, cap=512):
        """Elements whose closure holds `node` (restricted refinement)."""
        conn = np.empty((cap, 4), dtype=np.int32)
        macro = np.empty(cap, dtype=np.int32)
        n = int(_load().om_incident(self._h, int(node), _p(conn), _p(macro), cap))
        if n < 0 or n > cap:
            raise RuntimeError("oracle: incident search failed")
        return conn[:n].astype(np.int64), macro[:n].astype(np.int64)

    def valence(self, vids):
        v = np.ascontiguousarray(vids, dtype=np.int32)
        return int(_load().om_valence(self._h, _p(v), len(v)))


def coarse_to_fine(coarse, fine):
    """Canonical index on `fine` (level l+1) of every node of `coarse` (level l)."""
    m = np.empty(coarse.n_nodes, dtype=np.int64)
    _load().om_coarse_to_fine(coarse._h, fine._h, _p(m))
    return m


def prolongation(coarse, fine):
    """P1 interpolation matrix (fine.n_nodes x coarse.n_nodes), all nodes."""
    ne = coarse.n_elements
    rows = np.empty(16 * ne, dtype=np.int64)
    cols = np.empty(16 * ne, dtype=np.int64)
    vals = np.empty(16 * ne)
    n = int(_load().om_prolongation(coarse._h, fine._h, _p(rows), _p(cols), _p(vals)))
    key = rows[:n] * coarse.n_nodes + cols[:n]
    _, first = np.unique(key, return_index=True)
    return sp.csr_matrix((vals[first], (rows[first], cols[first])),
                         shape=(fine.n_nodes, coarse.n_nodes))


# ---------------------------------------------------------------- elements
def element_matrices(xyz, conn):
    """A_t[a,b] = |t| grad(lambda_a) . grad(lambda_b) for every element (ne,4,4),
    lambda the barycentric (P1 nodal) functions of t, and the volumes |t|."""
    P = xyz[conn]                                   # (ne,4,3)
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                         # rows = grad lambda_1..3
    G = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)  # (ne,4,3)
    vol = np.abs(det) / 6.0
    A = vol[:, None, None] * np.einsum("eai,ebi->eab", G, G)
    return A, vol


# directions c_m of the six components D_m = c_m . grad of the tensor form
_TDIRS = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [0, 1, 1]], dtype=np.float64)


def tensor_element_matrices(xyz, conn):
    """A^m_t[a,b] = |t| (c_m . grad lambda_a)(c_m . grad lambda_b), (6,ne,4,4),
    and the element gradients (ne,4,3) and volumes."""
    P = xyz[conn]
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    Jinv = np.linalg.inv(J)
    G = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)
    vol = np.abs(np.linalg.det(J)) / 6.0
    D = np.einsum("eai,mi->mea", G, _TDIRS)
    return vol[None, :, None, None] * D[:, :, :, None] * D[:, :, None, :], G, vol


def _tensor_element_blocks(xyz, conn, K6, kind):
    """Per-element 4x4 blocks of sum_m a_m for the elements conn (see
    assemble_tensor for the two forms)."""
    Am, _, _ = tensor_element_matrices(xyz, conn)
    KA = np.zeros(Am.shape[1:])
    idx = np.arange(4)
    for m in range(6):
        kv = K6[m][conn]
        if kind == "nodal":
            KA += kv.mean(axis=1)[:, None, None] * Am[m]
        else:
            T = (kv[:, :, None] + kv[:, None, :]) / 2.0 * Am[m]
            T[:, idx, idx] = 0.0
            T[:, idx, idx] = -T.sum(axis=2)
            KA += T
    return KA


def apply_tensor_rows(mesh, K6_at, u, nodes, kind="scaled"):
    """(A_K u)_p of the tensor operator for the given nodes, each row summed
    from the elements holding that node only (for sizes the full assembly
    cannot reach).  K6_at maps points (n, 3) to the six fields (6, n) there;
    u's Dirichlet entries read as 0, Dirichlet rows 0."""
    uu = np.where(mesh.dirichlet, 0.0, u)
    res = np.zeros(len(nodes))
    for i, p in enumerate(nodes):
        if mesh.dirichlet[p]:
            continue
        conn, _ = mesh.incident(p)
        loc = np.unique(conn)
        xl = mesh.xyz[loc]
        cl = np.searchsorted(loc, conn)
        KA = _tensor_element_blocks(xl, cl, K6_at(xl), kind)
        a = np.argmax(conn == p, axis=1)
        res[i] = float(np.einsum("eb,eb->", KA[np.arange(conn.shape[0]), a], uu[conn]))
    return res


def assemble_tensor(mesh, K6, kind="scaled"):
    """Global matrix over all nodes of sum_m a_m (Sec. 2.1 eq. (integral)) with
    the six coefficient fields K6 (6, n_nodes): per component, scaled =
    off-diagonal factor (k_m,a + k_m,b)/2 and zero element row sums (the scalar
    form of Lemma 3.2 applied to a_m), nodal = mean vertex k_m times A^m_t."""
    conn, _ = mesh.elements()
    KA = _tensor_element_blocks(mesh.xyz, conn, K6, kind)
    rows = np.repeat(conn, 4, axis=1).ravel()
    cols = np.tile(conn, (1, 4)).ravel()
    M = sp.coo_matrix((KA.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    M.sum_duplicates()
    return M


def make_tensor_operator(mesh, K6, kind="scaled"):
    return Operator(mesh, assemble_tensor(mesh, K6, kind))


def assemble_galerkin_constant_tensor(mesh, K):
    """Exact Galerkin matrix of int grad(v) . K grad(w) for a constant K:
    |t| G K G^T per element."""
    conn, _ = mesh.elements()
    _, G, vol = tensor_element_matrices(mesh.xyz, conn)
    KA = vol[:, None, None] * np.einsum("eai,ij,ebj->eab", G, np.asarray(K, dtype=np.float64), G)
    rows = np.repeat(conn, 4, axis=1).ravel()
    cols = np.tile(conn, (1, 4)).ravel()
    M = sp.coo_matrix((KA.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    M.sum_duplicates()
    return M


def _lambda_min(A):
    """Smallest non-zero generalised eigenvalue of A x = lambda (4I - 11^T) x per
    element: the 3D analogue of the matrix [[2,-1,-1],..] of Sec. 4.1 (both
    forms vanish exactly on constants).  With an orthonormal basis B of the
    complement of the constants, (4I-11^T) restricted is 4I."""
    B = np.array([[1, -1, 0, 0], [1, 1, -2, 0], [1, 1, 1, -3]], dtype=np.float64).T
    B /= np.linalg.norm(B, axis=0)
    R = np.einsum("ai,eab,bj->eij", B, A, B)
    return np.linalg.eigvalsh(R)[:, 0] / 4.0


_PAIRS = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def modification_factors(mesh, k, A=None, lam_level=None):
    """3D reading of the pre-asymptotic modification (Sec. 4.1, MA2 / k_mod).

    Per macro tet T and per edge e = (a,b) of T's refined mesh:
      a_plus  = max over elements t of T holding e of A_t[a,b];
                e is a candidate iff a_plus > 0 (a positive element entry);
      k_e     = (k_a + k_b)/2;
      k_emin  = min of (k_c + k_d)/2 over all edges (c,d) of the elements of T
                holding e (the edges of the closed patch omega_{e;T});
      lam_T   = min over the elements of T of the smallest non-zero eigenvalue
                of A_t x = lambda (4I - 11^T) x.
    Triggered iff (k_e - k_emin) a_plus > k_emin lam_T, and then T's scaling
    factor for e becomes k_mod = k_emin (1 + lam_T / a_plus).

    Returns a dict mapping (T, min(a,b), max(a,b)) -> k_mod for triggered
    edges, plus the candidate count, as (mods, n_candidates)."""
    conn, macro = mesh.elements()
    if A is None:
        A, _ = element_matrices(mesh.xyz, conn)
    lam_el = _lambda_min(A)
    lam_T = np.full(mesh.T.shape[0], np.inf)
    np.minimum.at(lam_T, macro, lam_el)
    kmin_el = np.min(np.stack([(k[conn[:, a]] + k[conn[:, b]]) / 2 for a, b in _PAIRS], axis=1), axis=1)
    n = mesh.n_nodes
    keys, aval, kmin = [], [], []
    for a, b in _PAIRS:
        lo = np.minimum(conn[:, a], conn[:, b])
        hi = np.maximum(conn[:, a], conn[:, b])
        keys.append((macro * n + lo) * n + hi)
        aval.append(A[:, a, b])
        kmin.append(kmin_el)
    keys = np.concatenate(keys)
    aval = np.concatenate(aval)
    kmin = np.concatenate(kmin)
    uk, inv = np.unique(keys, return_inverse=True)
    a_plus = np.full(uk.shape[0], -np.inf)
    np.maximum.at(a_plus, inv, aval)
    k_emin = np.full(uk.shape[0], np.inf)
    np.minimum.at(k_emin, inv, kmin)
    T = uk // (n * n)
    lo = (uk // n) % n
    hi = uk % n
    cand = a_plus > 0
    k_e = (k[lo] + k[hi]) / 2
    lamT = lam_T[T]
    trig = cand & ((k_e - k_emin) * a_plus > k_emin * lamT)
    kmod = k_emin * (1.0 + lamT / np.where(cand, a_plus, 1.0))
    mods = {(int(t), int(a), int(b)): float(v)
            for t, a, b, v in zip(T[trig], lo[trig], hi[trig], kmod[trig])}
    info = dict(n_candidates=int(cand.sum()), n_triggered=int(trig.sum()),
                k_e=k_e[trig], k_emin=k_emin[trig], k_mod=kmod[trig],
                lam_T=lam_T, a_plus=a_plus[cand])
    return mods, info


def _pair_factors(conn, macro, k, kind, mods, n):
    """(ne,4,4) factor matrix per element: scaled -> (k_a+k_b)/2 off-diagonal
    (or k_mod on triggered edges), nodal -> mean vertex k everywhere."""
    ne = conn.shape[0]
    if kind == "nodal":
        kbar = k[conn].mean(axis=1)
        return np.broadcast_to(kbar[:, None, None], (ne, 4, 4)).copy()
    kv = k[conn]
    F = (kv[:, :, None] + kv[:, None, :]) / 2.0
    if mods:
        keys = np.array([(t * n + a) * n + b for (t, a, b) in mods], dtype=np.int64)
        vals = np.array(list(mods.values()))
        order = np.argsort(keys)
        keys, vals = keys[order], vals[order]
        for a, b in _PAIRS:
            lo = np.minimum(conn[:, a], conn[:, b])
            hi = np.maximum(conn[:, a], conn[:, b])
            q = (macro * n + lo) * n + hi
            pos = np.searchsorted(keys, q)
            pos = np.minimum(pos, len(keys) - 1)
            hit = keys[pos] == q
            F[hit, a, b] = vals[pos[hit]]
            F[hit, b, a] = vals[pos[hit]]
    return F


def assemble(mesh, k, kind="scaled", modification=False, mods=None):
    """Global matrix over ALL nodes (Dirichlet rows included) by an element loop.

    scaled: sum_t K_t o A_t with (K_t)_ab = (k_a+k_b)/2 for a != b and the
            diagonal of K_t from eq. (zerosum), i.e. each element row of
            K_t o A_t sums to zero (Lemma 3.2, eq. (equal)).
    nodal:  sum_t kbar_t A_t, kbar_t the mean of k at t's vertices (eq. (standardfe)).
    """
    conn, macro = mesh.elements()
    A, _ = element_matrices(mesh.xyz, conn)
    if kind == "scaled" and modification and mods is None:
        mods, _ = modification_factors(mesh, k, A)
    F = _pair_factors(conn, macro, k, kind, mods if kind == "scaled" else None, mesh.n_nodes)
    KA = F * A
    if kind == "scaled":
        idx = np.arange(4)
        KA[:, idx, idx] = 0.0
        KA[:, idx, idx] = -KA.sum(axis=2)
    rows = np.repeat(conn, 4, axis=1).ravel()
    cols = np.tile(conn, (1, 4)).ravel()
    M = sp.coo_matrix((KA.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    M.sum_duplicates()
    return M


def assemble_mass(mesh):
    """Consistent P1 mass matrix: M_t = |t|/20 (1 + delta_ab)."""
    conn, _ = mesh.elements()
    _, vol = element_matrices(mesh.xyz, conn)
    loc = (np.ones((4, 4)) + np.eye(4)) / 20.0
    vals = (vol[:, None, None] * loc[None]).ravel()
    rows = np.repeat(conn, 4, axis=1).ravel()
    cols = np.tile(conn, (1, 4)).ravel()
    return sp.coo_matrix((vals, (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()


def brute_force_scaled(mesh, k):
    """eq. (discrete) evaluated literally: A[p,q] = a_h(phi_q, phi_p) =
    1/4 sum_T sum_{i,j} (k_i+k_j)(nu_i-nu_j)(chi_j-chi_i) int_T grad phi_i.grad phi_j,
    with nu = e_q, chi = e_p, and the T-integrals G_T[i,j] taken as sums of
    element integrals over the elements of T.  Dense; small levels only."""
    conn, macro = mesh.elements()
    A, _ = element_matrices(mesh.xyz, conn)
    n = mesh.n_nodes
    out = np.zeros((n, n))
    for T in range(mesh.T.shape[0]):
        sel = macro == T
        G = np.zeros((n, n))
        c = conn[sel]
        for a in range(4):
            for b in range(4):
                np.add.at(G, (c[:, a], c[:, b]), A[sel, a, b])
        nodes = np.unique(c)
        # (nu_i - nu_j)(chi_j - chi_i) with nu = e_q, chi = e_p:
        #   p != q: only (i,j) = (q,p) and (p,q) contribute, each -1  -> -(k_p+k_q)/2 * G[p,q]
        #   p == q: every j != p contributes (i,j)=(p,j),(j,p)        -> sum_j (k_p+k_j)/2 G[p,j]
        for p in nodes:
            for q in nodes:
                if p == q:
                    s = 0.0
                    for j in nodes:
                        if j != p:
                            s += 0.25 * (k[p] + k[j]) * G[p, j] * (-1.0) * 2.0
                    out[p, p] += s
                elif G[p, q] != 0.0:
                    out[p, q] += 0.25 * (k[p] + k[q]) * G[q, p] * 2.0
    return out


def brute_force_nodal(mesh, k):
    """eq. (standardfe) evaluated literally with the nodal quadrature rule:
    sum_t |t|/(d+1) sum_i k(x_i^t) grad phi_q . grad phi_p (gradients constant on t)."""
    conn, _ = mesh.elements()
    P = mesh.xyz[conn]
    n = mesh.n_nodes
    out = np.zeros((n, n))
    for e in range(conn.shape[0]):
        J = np.stack([P[e, 1] - P[e, 0], P[e, 2] - P[e, 0], P[e, 3] - P[e, 0]], axis=1)
        vol = abs(np.linalg.det(J)) / 6.0
        Ji = np.linalg.inv(J)
        G = np.vstack([-Ji.sum(axis=0), Ji])
        quad = vol / 4.0 * sum(k[conn[e, i]] for i in range(4))
        for a in range(4):
            for b in range(4):
                out[conn[e, a], conn[e, b]] += quad * G[a] @ G[b]
    return out


# ---------------------------------------------------------------- rows one by one
def rows(mesh, k, nodes, kind="scaled"):
    """Rows of the (unmodified) operator at the given canonical nodes, each from
    the elements holding that node only (for sizes the full assembly cannot
    reach).  Returns a list of (cols, vals)."""
    out = []
    for p in nodes:
        conn, macro = mesh.incident(p)
        A, _ = element_matrices(mesh.xyz, conn)
        F = _pair_factors(conn, macro, k, kind, None, mesh.n_nodes)
        KA = F * A
        if kind == "scaled":
            idx = np.arange(4)
            KA[:, idx, idx] = 0.0
            KA[:, idx, idx] = -KA.sum(axis=2)
        cols, vals = [], []
        for e in range(conn.shape[0]):
            a = int(np.flatnonzero(conn[e] == p)[0])
            for b in range(4):
                cols.append(conn[e, b])
                vals.append(KA[e, a, b])
        cols = np.array(cols)
        vals = np.array(vals)
        uc, inv = np.unique(cols, return_inverse=True)
        acc = np.zeros(len(uc))
        np.add.at(acc, inv, vals)
        out.append((uc, acc))
    return out


def apply_rows(mesh, k, u, nodes, kind="scaled"):
    """(A u)_p for the given nodes, with u's Dirichlet entries read as 0 and
    Dirichlet rows returning 0."""
    uu = np.where(mesh.dirichlet, 0.0, u)
    res = np.empty(len(nodes))
    for i, (p, (c, v)) in enumerate(zip(nodes, rows(mesh, k, nodes, kind))):
        res[i] = 0.0 if mesh.dirichlet[p] else float(v @ uu[c])
    return res


# ---------------------------------------------------------------- operator on vectors
class Operator:
    """A level's matrix restricted to the unknowns; vectors live on all nodes
    with Dirichlet entries 0."""

    def __init__(self, mesh, M):
        self.mesh = mesh
        self.full = M
        u = mesh.unknowns
        self.A = M[u][:, u].tocsr()
        self.diag = self.A.diagonal()

    def apply(self, x):
        y = np.zeros(self.mesh.n_nodes)
        y[self.mesh.unknowns] = self.A @ x[self.mesh.unknowns]
        return y

    def residual(self, f, x):
        r = f - self.apply(x)
        r[self.mesh.dirichlet] = 0.0
        return r


def make_operator(mesh, k, kind="scaled", modification=False):
    return Operator(mesh, assemble(mesh, k, kind, modification))


def primitive_dims(mesh):
    """Dimension of the macro primitive that holds each node (Sec. 5: the
    node sets W_V, W_E, W_F of the vertex, edge and face primitives; 3 = the
    interior of a macro tet): the number of nonzero barycentric weights of the
    node in a macro tet containing it, minus one."""
    conn, macro = mesh.elements()
    owner = np.full(mesh.n_nodes, -1, dtype=np.int64)
    owner[conn.ravel()] = np.repeat(macro, 4)
    dims = np.empty(mesh.n_nodes, dtype=np.int64)
    for t in range(mesh.T.shape[0]):
        idx = np.flatnonzero(owner == t)
        if len(idx) == 0:
            continue
        B = np.vstack([mesh.X[mesh.T[t]].T, np.ones(4)])
        lam = np.linalg.solve(B, np.vstack([mesh.xyz[idx].T, np.ones(len(idx))]))
        dims[idx] = (np.abs(lam) > 1e-9).sum(axis=0) - 1
    return dims


def assemble_mixed(mesh, k, nodal_dims, modification=False):
    """Sec. 5 eq. (modst): the row of node i is its nodal-integration row
    (eq. standardfe) when i lies on a macro primitive whose dimension is in
    `nodal_dims` (0 vertices, 1 edges, 2 faces), its stencil-scaling row
    (eq. discrete, with the Sec. 4.1 modification if asked) otherwise."""
    S = assemble(mesh, k, "scaled", modification)
    N = assemble(mesh, k, "nodal")
    sel = np.isin(primitive_dims(mesh), list(nodal_dims)).astype(np.float64)
    return (sp.diags(sel) @ N + sp.diags(1.0 - sel) @ S).tocsr()


def make_mixed_operator(mesh, k, nodal_dims, modification=False):
    return Operator(mesh, assemble_mixed(mesh, k, nodal_dims, modification))


def jacobi(op, f, u, sweeps, omega=2.0 / 3.0, history=False):
    """u <- u + omega D^{-1} (f - A u), all iterates if history."""
    u = u.copy()
    u[op.mesh.dirichlet] = 0.0
    idx = op.mesh.unknowns
    its = []
    for _ in range(sweeps):
        r = op.residual(f, u)
        u[idx] += omega * r[idx] / op.diag
        if history:
            its.append(u.copy())
    return (u, its) if history else u


def gershgorin_lambda(op):
    """Upper bound of the spectrum of D^{-1} A (Gershgorin discs of the rows of
    the reduced matrix): max_i sum_j |A_ij| / A_ii."""
    return float(np.max(abs(op.A).sum(axis=1).A1 / op.diag))


def chebyshev(op, f, u, steps, lam_max, lo=0.1, hi=1.0):
    """Chebyshev iteration on D^{-1} A over [lo lam_max, hi lam_max]
    (three-term recurrence; `steps` residual evaluations)."""
    a, b = lo * lam_max, hi * lam_max
    theta, delta = (b + a) / 2, (b - a) / 2
    sigma = theta / delta
    idx = op.mesh.unknowns
    u = u.copy()
    u[op.mesh.dirichlet] = 0.0
    r = op.residual(f, u)
    d = np.zeros_like(u)
    d[idx] = r[idx] / op.diag / theta
    rho = 1.0 / sigma
    for s in range(steps):
        u += d
        if s == steps - 1:
            break
        r = op.residual(f, u)
        rho_new = 1.0 / (2 * sigma - rho)
        d_new = np.zeros_like(u)
        d_new[idx] = rho_new * rho * d[idx] + (2 * rho_new / delta) * r[idx] / op.diag
        d, rho = d_new, rho_new
    return u


def geometric_coarse_k(P, kf):
    """Coarse coefficients as geometric full-weighting averages of the fine
    ones: k_c = exp(sum_f P_fc log k_f / sum_f P_fc), P the P1 interpolation
    matrix (fine x coarse, all nodes)."""
    R = P.T.tocsr()
    return np.exp((R @ np.log(kf)) / (R @ np.ones(P.shape[0])))


class Multigrid:
    """Geometric multigrid on the nested uniformly refined meshes: P1
    interpolation P, restriction P^T, rediscretised operators with k sampled at
    each level's nodes (coarse_k="sample"; with kfine given, the coarse values
    at the nested nodes) or averaged geometrically from the next finer level
    (coarse_k="geometric", geometric_coarse_k), exact dense solve on the
    coarsest level."""

    def __init__(self, X, T, level, coarse_level, kfun=None, kfine=None, kind="scaled",
                 modification=False, coarse_k="sample"):
        self.levels = list(range(coarse_level, level + 1))
        self.meshes = {l: Mesh(X, T, l) for l in self.levels}
        self.ops, self.P, self.lam = {}, {}, {}
        for l in self.levels[1:]:
            self.P[l] = prolongation(self.meshes[l - 1], self.meshes[l])
        kl = {}
        if coarse_k == "geometric":
            kl[level] = kfine if kfine is not None else kfun(self.meshes[level].xyz)
            for l in reversed(self.levels[:-1]):
                kl[l] = geometric_coarse_k(self.P[l + 1], kl[l + 1])
        elif kfine is not None:
            kl[level] = kfine
            for l in reversed(self.levels[:-1]):
                kl[l] = kl[l + 1][coarse_to_fine(self.meshes[l], self.meshes[l + 1])]
        else:
            for l in self.levels:
                kl[l] = kfun(self.meshes[l].xyz)
        self.k = kl
        for l in self.levels:
            self.ops[l] = make_operator(self.meshes[l], kl[l], kind, modification)
            if l > coarse_level:
                self.lam[l] = gershgorin_lambda(self.ops[l])
        cop = self.ops[coarse_level]
        self.coarse_dense = cop.A.toarray()

    def coarse_solve(self, f):
        m = self.meshes[self.levels[0]]
        u = np.zeros(m.n_nodes)
        u[m.unknowns] = np.linalg.solve(self.coarse_dense, f[m.unknowns])
        return u

    def vcycle(self, l, f, u, pre=2, post=2, smoother="chebyshev", omega=2.0 / 3.0):
        if l == self.levels[0]:
            return self.coarse_solve(f)
        op = self.ops[l]
        u = self._smooth(op, f, u, pre, smoother, omega, self.lam[l])
        r = op.residual(f, u)
        P = self.P[l]
        mc = self.meshes[l - 1]
        fc = P.T @ r
        fc[mc.dirichlet] = 0.0
        uc = self.vcycle(l - 1, fc, np.zeros(mc.n_nodes), pre, post, smoother, omega)
        u = u + P @ uc
        u[op.mesh.dirichlet] = 0.0
        u = self._smooth(op, f, u, post, smoother, omega, self.lam[l])
        return u

    @staticmethod
    def _smooth(op, f, u, n, smoother, omega, lam):
        if n == 0:
            return u
        if smoother == "jacobi":
            return jacobi(op, f, u, n, omega)
        return chebyshev(op, f, u, n, lam)

    def solve(self, f, tol=1e-8, maxit=100, **kw):
        L = self.levels[-1]
        op = self.ops[L]
        u = np.zeros(op.mesh.n_nodes)
        nf = np.linalg.norm(f[op.mesh.unknowns])
        hist = [np.linalg.norm(op.residual(f, u)) / nf]
        while hist[-1] > tol and len(hist) <= maxit:
            u = self.vcycle(L, f, u, **kw)
            hist.append(np.linalg.norm(op.residual(f, u)) / nf)
        return u, hist


# ---------------------------------------------------------------- errors
def _conical_rule(order=4):
    """Stroud's conical product rule on the unit tetrahedron from Gauss-Legendre
    points (Duffy map x=a, y=b(1-a), z=c(1-a)(1-b), Jacobian (1-a)^2 (1-b));
    `order` points per direction integrate polynomials of degree 2*order-3 exactly."""
    g, w = np.polynomial.legendre.leggauss(order)
    g = (g + 1) / 2
    w = w / 2
    A, B, C = np.meshgrid(g, g, g, indexing="ij")
    WA, WB, WC = np.meshgrid(w, w, w, indexing="ij")
    x = A
    y = B * (1 - A)
    z = C * (1 - A) * (1 - B)
    wt = WA * WB * WC * (1 - A) ** 2 * (1 - B)
    bary = np.stack([1 - x - y - z, x, y, z], axis=-1).reshape(-1, 4)
    return bary, wt.ravel()


def errors(mesh, uh, uexact, grad_exact, chunk=200000):
    """Exact L2 and H1-seminorm errors of the P1 function uh against uexact by
    per-element quadrature (degree 5), plus the discrete nodal L2 error
    (h^3 sum_i e_i^2)^(1/2) over the unknowns."""
    conn, _ = mesh.elements()
    bary, wq = _conical_rule(4)
    e2, g2 = 0.0, 0.0
    for a in range(0, conn.shape[0], chunk):
        c = conn[a:a + chunk]
        P = mesh.xyz[c]
        J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
        det = np.abs(np.linalg.det(J))
        Ji = np.linalg.inv(J)
        G = np.concatenate([-Ji.sum(axis=1, keepdims=True), Ji], axis=1)
        ue = uh[c]                                   # (ne,4)
        grad_h = np.einsum("ea,eai->ei", ue, G)      # (ne,3)
        pts = np.einsum("qa,eai->eqi", bary, P)      # (ne,nq,3)
        flat = pts.reshape(-1, 3)
        uex = uexact(flat).reshape(c.shape[0], -1)
        gex = grad_exact(flat).reshape(c.shape[0], -1, 3)
        uq = ue @ bary.T                             # (ne,nq)
        e2 += np.sum(det[:, None] * wq[None] * (uq - uex) ** 2)
        g2 += np.sum(det[:, None] * wq[None] * np.sum((grad_h[:, None, :] - gex) ** 2, axis=2))
    dof = mesh.unknowns
    nodal = np.sqrt(mesh.h ** 3 * np.sum((uh[dof] - uexact(mesh.xyz[dof])) ** 2))
    return dict(L2=np.sqrt(e2), H1=np.sqrt(g2), nodal_L2=nodal)


# ---------------------------------------------------------------- CSR SpMV (C)
def spmv_timing_matrix(op):
    """Plain CSR arrays (int64 row pointers, int32 column indices) of the
    reduced operator for timing."""
    A = op.A
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), np.ascontiguousarray(A.data)


_csr = None


def _csr_lib():
    global _csr
    if _csr is None:
        build()
        L = ctypes.CDLL(_CSR_LIB)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.csr_spmv.argtypes = [I64, P, P, P, P, P, I32]
        L.csr_spmv.restype = None
        L.csr_spmv_bench.argtypes = [I64, P, P, P, P, P, I32, I32, I32, P]
        L.csr_spmv_bench.restype = None
        L.csr_max_threads.restype = I32
        _csr = L
    return _csr


def spmv_threaded(op, x, threads):
    """A x over the unknowns (vector on all nodes, Dirichlet entries 0) by the
    threaded C CSR product; equals op.apply(x) (same summation order)."""
    ip, ix, dv = spmv_timing_matrix(op)
    xu = np.ascontiguousarray(x[op.mesh.unknowns], dtype=np.float64)
    yu = np.empty_like(xu)
    _csr_lib().csr_spmv(len(xu), _p(ip), _p(ix), _p(dv), _p(xu), _p(yu), int(threads))
    y = np.zeros(op.mesh.n_nodes)
    y[op.mesh.unknowns] = yu
    return y


def spmv_bench(op, threads, warm=20, reps=200, seed=0):
    """Seconds of each of `reps` threaded CSR products with the reduced
    operator (after `warm` untimed ones), on a uniform random vector."""
    ip, ix, dv = spmv_timing_matrix(op)
    n = len(ip) - 1
    x = np.random.default_rng(seed).uniform(-1, 1, n)
    y = np.empty(n)
    times = np.empty(reps)
    _csr_lib().csr_spmv_bench(n, _p(ip), _p(ix), _p(dv), _p(x), _p(y), int(threads), int(warm), int(reps),
                              _p(times))
    return times
