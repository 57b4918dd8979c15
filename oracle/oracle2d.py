"""CPU oracle for the 2D variant: P1 on uniformly refined triangular macro
meshes, stencil scaling with the exact pre-asymptotic modification of
Sec. 4.1 (MA2), and nodal integration.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of bench.py may import this module; the product library never does, and
the two share no code.  Everything is float64; plain numpy/scipy assembly of
GLOBAL CSR matrices by loops over the refined elements.

Paper passages followed (arXiv 1709.06793):
* element matrices  A_t[a,b] = int_t grad phi_a . grad phi_b              (Sec. 3.2)
* scaled form       eq. (meshdep) with M = 1: off-diagonal factor
                    k_e = (k_a + k_b)/2 per element edge, diagonal by zero row
                    sums (Lemma 3.2)
* modification      Sec. 4.1, 2D: gray edges = element edges with a positive
                    reference entry a_12^T > 0 (only in macro triangles with an
                    obtuse angle); patch omega_{e;T} = elements of T holding e;
                    k_{e;min} = min over the edges of the closed patch of their
                    k_e; lambda_min^T = smallest non-degenerate eigenvalue of
                    A_T x = lambda [[2,-1,-1],[-1,2,-1],[-1,-1,2]] x; if (MA2)
                    (k_e - k_{e;min}) a_12^T > k_{e;min} lambda_min^T, the
                    factor of e in T becomes k_{e;min} (1 + lambda_min^T / a_12^T)
* nodal form        eq. (standardfe): mean vertex k times A_t             (Sec. 3.2)
* Lemma 4.1         non-obtuse macro meshes give an M-matrix Laplacian
* Lemma 3.1         O(h^2) L2 error of the scaled form (rates pin)
"""
import numpy as np
import scipy.sparse as sp


class Mesh2D:
    """Uniform refinement of a triangular macro mesh: every macro triangle T
    with vertices (v0, v1, v2) carries the lattice points
    x = (w0 X[v0] + w1 X[v1] + w2 X[v2]) / n, w = (n-i-j, i, j), n = 2^level;
    points are identified across triangles by their macro vertices and
    integer weights.  Each lattice cell gives the elements
    (i,j),(i+1,j),(i,j+1) and (i+1,j),(i+1,j+1),(i,j+1).  Dirichlet nodes: those
    on macro edges held by one triangle."""

    def __init__(self, X, T, level):
        self.X, self.T, self.level = np.asarray(X, np.float64), np.asarray(T, np.int64), level
        n = 2 ** level
        self.n = n
        ids, xy = {}, []

        def node(t, i, j):
            w = (n - i - j, i, j)
            key = tuple(sorted((int(self.T[t, a]), w[a]) for a in range(3) if w[a] > 0))
            if key not in ids:
                ids[key] = len(xy)
                xy.append(sum(w[a] * self.X[self.T[t, a]] for a in range(3)) / n)
            return ids[key]

        conn, macro = [], []
        for t in range(self.T.shape[0]):
            for j in range(n):
                for i in range(n - j):
                    conn.append((node(t, i, j), node(t, i + 1, j), node(t, i, j + 1)))
                    macro.append(t)
                    if i + j <= n - 2:
                        conn.append((node(t, i + 1, j), node(t, i + 1, j + 1), node(t, i, j + 1)))
                        macro.append(t)
        self.xy = np.array(xy)
        self.conn = np.array(conn, dtype=np.int64)
        self.macro = np.array(macro, dtype=np.int64)
        self.n_nodes = self.xy.shape[0]
        # boundary macro edges: held by exactly one triangle
        cnt = {}
        for t in self.T:
            for a in range(3):
                e = tuple(sorted((int(t[a]), int(t[(a + 1) % 3]))))
                cnt[e] = cnt.get(e, 0) + 1
        bnd = {e for e, c in cnt.items() if c == 1}
        self.dirichlet = np.zeros(self.n_nodes, dtype=bool)
        # macro primitive of each node: 0 vertex, 1 edge, 2 triangle interior
        self.prim_dim = np.zeros(self.n_nodes, dtype=np.int64)
        for key, q in ids.items():
            self.prim_dim[q] = len(key) - 1
            vs = tuple(sorted(v for v, _ in key))
            if len(vs) == 1:
                self.dirichlet[q] = any(vs[0] in e for e in bnd)
            elif len(vs) == 2:
                self.dirichlet[q] = vs in bnd
        self.unknowns = np.flatnonzero(~self.dirichlet)


def element_matrices(xy, conn):
    """A_t = |t| G G^T with G the (3, 2) gradients of the barycentric
    functions; returns (ne, 3, 3) and the areas."""
    P = xy[conn]
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=2)  # columns: edges
    Jinv = np.linalg.inv(J)
    G = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)
    area = np.abs(np.linalg.det(J)) / 2.0
    return area[:, None, None] * np.einsum("eai,ebi->eab", G, G), area


_B = np.array([[2.0, -1.0, -1.0], [-1.0, 2.0, -1.0], [-1.0, -1.0, 2.0]])


def lambda_min(A):
    """Smallest non-degenerate eigenvalue of A x = lambda B x (B above): both
    vanish exactly on constants; on the complement B = 3 I."""
    Q = np.array([[1.0, -1.0, 0.0], [1.0, 1.0, -2.0]]).T
    Q /= np.linalg.norm(Q, axis=0)
    R = np.einsum("ai,...ab,bj->...ij", Q, A, Q)
    return np.linalg.eigvalsh(R)[..., 0] / 3.0


_PAIRS = [(0, 1), (0, 2), (1, 2)]


def modification(mesh, k, A=None):
    """MA2 (Sec. 4.1) per macro triangle T and gray edge e of T's refined
    mesh.  Returns ({(T, lo, hi): k_mod} for the triggered edges, number of
    gray edges)."""
    conn, macro = mesh.conn, mesh.macro
    if A is None:
        A, _ = element_matrices(mesh.xy, conn)
    lam = lambda_min(A)
    lam_T = np.full(mesh.T.shape[0], np.inf)
    np.minimum.at(lam_T, macro, lam)
    kmin_el = np.min(np.stack([(k[conn[:, a]] + k[conn[:, b]]) / 2 for a, b in _PAIRS], axis=1), axis=1)
    info = {}  # (T, lo, hi) -> [a_plus, k_emin]
    for e in range(conn.shape[0]):
        T = int(macro[e])
        for a, b in _PAIRS:
            lo, hi = sorted((int(conn[e, a]), int(conn[e, b])))
            cur = info.setdefault((T, lo, hi), [-np.inf, np.inf])
            cur[0] = max(cur[0], A[e, a, b])
            cur[1] = min(cur[1], kmin_el[e])
    mods, n_gray = {}, 0
    for (T, lo, hi), (a_plus, k_emin) in info.items():
        if a_plus <= 0:
            continue
        n_gray += 1
        k_e = (k[lo] + k[hi]) / 2
        if (k_e - k_emin) * a_plus > k_emin * lam_T[T]:
            mods[(T, lo, hi)] = k_emin * (1.0 + lam_T[T] / a_plus)
    return mods, n_gray


def assemble(mesh, k, kind="scaled", modification_on=False):
    """Global matrix over all nodes (Dirichlet rows and columns included)."""
    conn, macro = mesh.conn, mesh.macro
    A, _ = element_matrices(mesh.xy, conn)
    if kind == "nodal":
        KA = k[conn].mean(axis=1)[:, None, None] * A
    else:
        F = np.zeros_like(A)
        for a, b in _PAIRS:
            f = (k[conn[:, a]] + k[conn[:, b]]) / 2
            F[:, a, b] = F[:, b, a] = f
        if modification_on:
            mods, _ = modification(mesh, k, A)
            for e in range(conn.shape[0]):
                for a, b in _PAIRS:
                    lo, hi = sorted((int(conn[e, a]), int(conn[e, b])))
                    km = mods.get((int(macro[e]), lo, hi))
                    if km is not None:
                        F[e, a, b] = F[e, b, a] = km
        KA = F * A
        idx = np.arange(3)
        KA[:, idx, idx] = 0.0
        KA[:, idx, idx] = -KA.sum(axis=2)
    rows = np.repeat(conn, 3, axis=1).ravel()
    cols = np.tile(conn, (1, 3)).ravel()
    M = sp.coo_matrix((KA.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    M.sum_duplicates()
    return M


def reduced(mesh, M):
    u = mesh.unknowns
    return M[u][:, u]


def apply(mesh, M, x):
    """y = A x on the unknowns (x's Dirichlet entries read as 0; Dirichlet rows 0)."""
    xx = np.where(mesh.dirichlet, 0.0, x)
    y = M @ xx
    y[mesh.dirichlet] = 0.0
    return y


def assemble_mass(mesh):
    """P1 mass matrix: |t|/12 [[2,1,1],[1,2,1],[1,1,2]] per element."""
    _, area = element_matrices(mesh.xy, mesh.conn)
    Mt = (np.ones((3, 3)) + np.eye(3)) / 12.0
    KA = area[:, None, None] * Mt[None]
    conn = mesh.conn
    rows = np.repeat(conn, 3, axis=1).ravel()
    cols = np.tile(conn, (1, 3)).ravel()
    M = sp.coo_matrix((KA.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    M.sum_duplicates()
    return M


def solve(mesh, M, b):
    """Direct solve on the unknowns (Dirichlet values 0)."""
    import scipy.sparse.linalg as spla
    u = np.zeros(mesh.n_nodes)
    idx = mesh.unknowns
    u[idx] = spla.spsolve(reduced(mesh, M).tocsc(), b[idx])
    return u
